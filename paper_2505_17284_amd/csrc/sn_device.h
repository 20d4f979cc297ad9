// sn_device.h -- data shared between the host plan and the gfx950 kernels.
//
// Internal to libsnrt; not part of the C ABI.
//
// Device layout of every per-cell plane (psi per ordinate, phi, its
// per-group partials, the region map): [ny_alloc][pitch] elements, rows of a
// whole number of 128-byte lines of psi. Interior cell (i, j) sits at
//     origin + j * pitch + i,    origin = 2 * pitch + ox,
// ox = 128 / sizeof(psi element) (32 for FP32, 64 for BF16), so that every
// 128-column tile of a row starts on a 128-byte line and the stage kernels
// write whole lines. Around the interior is a frame of two ghost cells on
// every side (columns ox - 2, ox - 1, ox + nx, ox + nx + 1; rows 0, 1,
// ny + 2, ny + 3). The ghost cells of psi carry, per ordinate and side, the
// value that makes the interior reconstruction formula produce the boundary
// traces of the method (see sn_stage_impl.h); the stage kernels write them for
// the state they produce.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace snk {

constexpr int kWave = 64;                      // CDNA wavefront width
constexpr int kCellsPerLane = 2;               // consecutive x-cells held by one lane
constexpr int kTileX = kCellsPerLane * kWave;  // 128 output columns per wave (two per lane)
constexpr int kGhost = 2;                      // ghost-frame width
constexpr int kMaxTallies = 8;
constexpr int kMaxRects = 4;
constexpr int kMaxProbes = 8;
// QoI slots: mass and absorption per tally (summed by the compute waves),
// outflow and inflow per rectangle, then phi, J_x, J_y per space-time probe
// (both summed by the loader wave)
constexpr int kMaxQWave = 1 + kMaxTallies;
constexpr int kMaxQ = kMaxQWave + 2 * kMaxRects + 3 * kMaxProbes;
constexpr int kMaxFluenceBlocks = 1024;
constexpr int kProbePerLane = 8;  // probe cells one loader lane accumulates
// Per-workgroup QoI partials one finalize workgroup sums (256 threads x 8):
// a QoI slot with more partials is summed in ceil(n_wg / kQoiChunk) chunks
// whose sums the last of them adds up in chunk order.
constexpr int kQoiChunk = 2048;

enum StageMode : int {
    kUpdate = 0,   // psi_out = psi_in + dt F(psi_in)                   (Euler, Heun stage 1)
    kAverage = 1,  // psi_out = (psi_old + psi_in + dt F(psi_in)) / 2   (Heun stage 2)
    kQoiOnly = 2,  // QoIs of psi_in, nothing written
};

enum Bc : int { kVacuum = 0, kInflow = 1, kReflect = 2 };
enum Side : int { kW = 0, kE = 1, kS = 2, kN = 3 };

// Per-ordinate constants, computed in FP64 on the host and rounded once.
struct alignas(16) OrdConst {
    float cx;       // dt * xi / h
    float cy;       // dt * eta / h
    float w;        // quadrature weight
    int32_t flags;  // bit 0: xi > 0, bit 1: eta > 0
    int32_t mx;     // ordinate with xi negated
    int32_t my;     // ordinate with eta negated
    int32_t pad0, pad1;
    double fx;      // w |xi|  (face QoI weight along x-faces, times h in finalize)
    double fy;      // w |eta|
};

// Per-region constants.
struct alignas(16) RegConst {
    float st;       // dt * (sigma_a + sigma_s)
    float cs;       // dt * sigma_s / (2 pi)
    float cq;       // dt * Q
    int32_t tally;  // absorption tally id
    double sa;      // sigma_a (absorption QoI, FP64)
    double pad;
};

struct StageArgs {
    const void* psi_in;   // stage input: stencils
    const void* psi_old;  // kAverage: psi^n at the cell (may equal psi_out)
    void* psi_out;
    const float* phi;     // scalar flux of psi_in (plane)
    float* phi_part;      // [G] planes: per-group partial scalar fluxes of psi_out
    const OrdConst* ord;
    const RegConst* reg;
    const uint8_t* region;  // plane of region ids
    double* qpart;          // [nq][n_wg] per-workgroup QoI partial sums
    const int32_t* counter; // stages finalised so far (seeds BF16 stochastic rounding)
    int64_t plane;          // ny_alloc * pitch (elements)
    int32_t nx, ny, pitch, M;
    int32_t ox;             // column of interior cell 0 in a row
    int32_t G, Mg;          // ordinate groups and ordinates per group
    int32_t ntx, nty;       // tiles along x (128 columns) and y (waves * rows_per_wave rows)
    int32_t n_wg;
    int32_t n_tallies, n_rects, nq;
    int32_t bc[4];
    float eps2;             // order 3: the limiter's epsilon^2, (h^2)^6
    // rectangle-boundary faces (outflow and inflow QoIs): the loader wave of
    // tile t sums every face's flux over the ordinates, its entries held in
    // registers, or, for tiles with more than kFaceRegs per lane, copied into
    // dynamic LDS (face_lds bytes: the largest such tile's table; 0 if none)
    const struct FaceEntry* fent;   // faces, grouped by tile, then by lane
    const int32_t* ftile;           // [ntiles][3]: first entry, entries per lane, lanes
    int32_t face_lds;
    // space-time probes: the loader wave of tile t accumulates phi, J_x, J_y
    // of the stage input over the tile's probe cells into QoI slots
    // qprobe + 3 p + m (qprobe = 1 + n_tallies + 2 n_rects)
    const struct ProbeEntry* pent;  // probe cells, grouped by tile, then by lane
    const int32_t* ptile;           // [ntiles][3]: first entry, entries per lane, lanes
    const double* pmom;             // [M][3] w, w xi, w eta in FP64
    int32_t n_probes, qprobe;
};

// One rectangle-boundary face as a loader lane reads it (16 bytes): element
// offsets, in a ring slot, of the four cells on the face's normal line, c0
// c1 | c2 c3 (the face lies between c1 and c2; increasing x for a face
// normal to x, increasing y otherwise), then, for order 3, of the neighbours
// of c1 and of c2 across that line (lower, then upper). Offsets take 14 bits;
// the two high bits of off[0] hold the rectangle, of off[1] the axis (bit
// 14: y) and the side the rectangle holds (bit 15: c2, i.e. a west or south
// face), of off[2] first order (bit 14: a face on the grid's boundary) and
// validity (bit 15; padding entries have it clear).
struct alignas(16) FaceEntry {
    uint16_t off[8];
};
constexpr uint32_t kFaceOffMask = 0x3fffu;
constexpr int kFacePerLaneMax = 64;  // entries per loader lane (at most 64 x 64 faces per tile)
// Entries a loader lane keeps in registers (orders 1 and 2; at order 3 the
// limiter's operands would raise the kernel's register count); a tile with
// more per lane reads them from a copy of its table in dynamic LDS. Three
// cover a tile crossed by one rectangle edge along x plus a few along y (the
// benchmark problems need at most three) and keep the batched kernel at
// 4 workgroups per compute unit (91 VGPRs; four entries: 97, 3 workgroups).
constexpr int kFaceRegs = 3;
constexpr int face_regs(int order) { return order == 3 ? 0 : kFaceRegs; }

// Ring slot layout (the stage kernels' LDS staging, also needed by the
// host's face tables): the stencil rows of the stage input, 128 cells each,
// rounded up to whole copies of kWave x 16 bytes; then the x-halo, 4 cells
// (-2, -1, 128, 129 of the tile) per output row, plus one row above and one
// below at order 3; then what the stage kind adds. Offsets in elements.
constexpr int ring_rows_per_copy(int elem_bytes) { return kWave * 16 / (kTileX * elem_bytes); }
constexpr int ring_halo_elem(int stencil_rows, int elem_bytes) {
    return (stencil_rows + ring_rows_per_copy(elem_bytes) - 1) / ring_rows_per_copy(elem_bytes) *
           ring_rows_per_copy(elem_bytes) * kTileX;
}

// One probe cell as a loader lane reads it: byte offset of the cell in a ring
// slot, its probe, and its weight (0 for padding).
struct ProbeEntry {
    uint32_t lds_off;
    int32_t probe;  // -1: padding
    double weight;
};

// One batched launch over several instances (plans): the grid strides over
// items 0 .. total-1; item i belongs to selected instance j with
// first[j] <= i < first[j + 1] and is that instance's workgroup i - first[j].
// The instance's arguments are args[sel[j]].
struct BatchLaunch {
    const StageArgs* args;
    const int32_t* sel;    // [n_sel]
    const int32_t* first;  // [n_sel + 1]
    int32_t n_sel;
    int32_t total;
};

struct FinalizeArgs;
struct FinalizeBatch {
    const FinalizeArgs* args;
    const int32_t* sel;
    const int32_t* first;
    int32_t n_sel;
    int32_t total;
};

struct GhostArgs {
    void* psi;
    const OrdConst* ord;
    int64_t plane;
    int32_t nx, ny, pitch, M, ox;
    int32_t bc[4];
    float ghost[4];  // inflow value per side (0 for vacuum)
    int32_t all_dirs;  // 1 (order 3): every ordinate's ghost cells hold the side's ghost value
};

struct FinalizeArgs {
    const float* phi_part;  // [G] planes written by the stage
    float* phi;             // their sum: phi of the stage output
    int64_t plane;
    int32_t nx, ny, pitch, G, ox;
    int32_t n_phi_wg;       // workgroups reducing phi (0: the stage wrote no partials)
    const double* qpart;    // [nq][n_wg]
    const double* scale;    // [nq]
    double* inst;           // [nq] instantaneous QoIs of the stage input
    double* integ;          // [nq] running time integrals
    double* qchunk;         // [nq][q_split] chunk sums (q_split > 1)
    int32_t* qcount;        // [nq] chunks finished so far in this launch (0 between launches)
    int32_t q_split;        // chunks per QoI slot: ceil(n_wg / kQoiChunk)
    int32_t* flags;         // bit 0: a non-finite QoI was seen
    int32_t* counter;       // stages finalised so far (incremented once per finalize)
    double coef;            // weight of this stage in the time integral
    int32_t n_wg, nq;
    double* fluence;        // [ny][nx] running time integral of phi, or NULL
    // space-time probes: QoI slots qprobe + 3 p + m (p probe, m = phi, J_x,
    // J_y) also add pcoef times their total to the window of the current step
    double* pacc;           // [n_windows][n_probes][3]
    int32_t* pstep;         // [3 n_probes] steps finished so far, one counter per slot block
    double pcoef;           // coef / window length
    int32_t n_probes;       // 0: no window accumulation in this launch
    int32_t qprobe, n_windows, nt;
    int32_t last_stage;     // 1: this stage ends a step
};

// One piece of a block or line integral of sigma_a * fluence (the layout of
// sn_fluence_piece): the mean over cells a and b, entering with weight w.
struct FluencePiece {
    int32_t a, b;
    double w;
};

struct FluenceArgs {
    const double* fluence;      // [ny][nx]
    const uint8_t* region;      // padded plane: cell (i, j) at origin + j * pitch + i
    const double* sa;           // [n_regions] sigma_a in FP64
    const FluencePiece* pieces; // [n_pieces], sorted by set
    const int32_t* set_start;   // [n_blocks + 2]
    double* out;                // [4 + n_blocks]
    int32_t* status;            // 0, or 1 for a malformed piece list
    int64_t origin;
    int32_t pitch, nx, ny, n_pieces, n_blocks;
};

struct PhiInitArgs {
    const void* psi;
    float* phi;
    const OrdConst* ord;
    int64_t plane;
    int32_t nx, ny, pitch, M, ox;
};

// Launchers. dtype: 0 = f32, 1 = bf16.
hipError_t launch_stage(int order, int mode, int dtype, int rows_per_wave, int waves, const StageArgs& a,
                        hipStream_t s);
hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s);
// Batched forms. Stage: wgs_per_cu == 0 one workgroup per item, > 0 a
// persistent grid of that many workgroups per CU, < 0 a persistent grid of the
// resident capacity; modes kUpdate and kAverage only; face_lds: the largest
// face table (StageArgs::face_lds) of the launch's instances. Finalize: a
// persistent grid of `grid`.
hipError_t launch_stage_batch(int order, int mode, int dtype, int rows_per_wave, int waves, const BatchLaunch& L,
                              int wgs_per_cu, int cus, int face_lds, hipStream_t s);
hipError_t launch_finalize_batch(const FinalizeBatch& L, int grid, hipStream_t s);
hipError_t launch_ghost_fill(int dtype, const GhostArgs& a, hipStream_t s);
hipError_t launch_phi_init(int dtype, const PhiInitArgs& a, hipStream_t s);
hipError_t launch_fluence_functionals(const FluenceArgs& a, hipStream_t s);
bool supported_shape(int rows_per_wave, int waves);

// Per translation unit (sn_stage_o{1,2}_{f32,bf16}.hip).
hipError_t launch_stage_o1_f32(int mode, int rows, int waves, const StageArgs& a, hipStream_t s);
hipError_t launch_stage_o2_f32(int mode, int rows, int waves, const StageArgs& a, hipStream_t s);
hipError_t launch_stage_o1_bf16(int mode, int rows, int waves, const StageArgs& a, hipStream_t s);
hipError_t launch_stage_o2_bf16(int mode, int rows, int waves, const StageArgs& a, hipStream_t s);
hipError_t launch_stage_o3_f32(int mode, int rows, int waves, const StageArgs& a, hipStream_t s);
hipError_t launch_stage_o3_bf16(int mode, int rows, int waves, const StageArgs& a, hipStream_t s);
hipError_t launch_batch_o1_f32(int mode, int rows, int waves, const BatchLaunch& L, int wgs_per_cu, int cus,
                               int face_lds, hipStream_t s);
hipError_t launch_batch_o2_f32(int mode, int rows, int waves, const BatchLaunch& L, int wgs_per_cu, int cus,
                               int face_lds, hipStream_t s);
hipError_t launch_batch_o1_bf16(int mode, int rows, int waves, const BatchLaunch& L, int wgs_per_cu, int cus,
                               int face_lds, hipStream_t s);
hipError_t launch_batch_o2_bf16(int mode, int rows, int waves, const BatchLaunch& L, int wgs_per_cu, int cus,
                               int face_lds, hipStream_t s);
hipError_t launch_batch_o3_f32(int mode, int rows, int waves, const BatchLaunch& L, int wgs_per_cu, int cus,
                               int face_lds, hipStream_t s);
hipError_t launch_batch_o3_bf16(int mode, int rows, int waves, const BatchLaunch& L, int wgs_per_cu, int cus,
                               int face_lds, hipStream_t s);

}  // namespace snk
