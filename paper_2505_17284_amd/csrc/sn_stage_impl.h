// sn_stage_impl.h -- the gfx950 stage kernel of the explicit S_N finite-volume step.
//
// One stage evaluates, for every ordinate k and cell (i, j) of a uniform grid
// of square cells (arXiv 2505.17284, Sec. 4.2, eq. eq_sn_2d_eqn_fv divided by
// the cell area h^2),
//
//   dt F = -(dt xi_k / h)(trace_{i+1/2} - trace_{i-1/2})
//          -(dt eta_k / h)(trace_{j+1/2} - trace_{j-1/2})
//          - dt sigma_t psi + dt sigma_s / (2 pi) phi + dt Q,
//
// with the upwind trace of eq. eq_upwind1stOrder: the upwind cell's value for
// first order, its minmod-limited linear reconstruction at the face for
// second order, or (the third template order) its Green-Gauss gradient
// reconstruction with the Venkatakrishnan limiter of Sec. 4.2 (eq.
// eq_V_limiter). The stage update follows Sec. 4.3 (eq. eq_ODE): psi + dt F
// (Euler and Heun's first stage) or (psi^n + psi^(1) + dt F(psi^(1))) / 2
// (Heun's second stage, written in place over psi^n). The scalar flux
// phi = sum_k w_k psi_k of the written state (Sec. 4.1) leaves as a per-group
// epilogue, and FP64 partial sums of the QoIs of the stage input (mass,
// absorption per tally, outflow and inflow through rectangle boundaries,
// Sec. 3.1.2) leave per workgroup.
//
// Boundaries without boundary code: every psi plane carries a two-cell ghost
// frame. For an ordinate entering through a side, both ghost layers hold the
// ghost value of the end of Sec. 4.2 (the inflow value, 0 for vacuum, or the
// mirror ordinate's boundary value for a reflective wall); for an ordinate
// leaving through a side, the first ghost layer repeats the boundary cell.
// With those values the interior formula gives exactly the method's boundary
// traces: first order on boundary faces (the limiter sees a zero difference),
// and the ghost value in the slope of the first interior cell. The waves that
// write boundary cells also write the frame of the new state (write_frame);
// incoming vacuum/inflow ghosts are constant and set once.
//
// Mapping: a compute wave owns 128 consecutive output columns, two per lane
// (x-neighbours cross lanes through DPP wave shifts; the two cells beyond
// each end of the tile come from a separately staged x-halo), and TY rows;
// the W compute waves of a workgroup are stacked in y and share one LDS copy
// of each ordinate's rows, halo rows included, which a loader wave stages
// while they compute earlier ordinates. The loader wave also sums the QoIs
// that need few cells: the currents through rectangle boundaries and the
// space-time probes. Per-cell material data and the incoming scalar flux
// stay in registers across the ordinate loop. Global accesses are buffer
// instructions: one scalar resource per plane, wave-uniform row offsets, one
// per-lane offset. There is no MFMA: the stage is a bandwidth-bound stencil
// (order 3: bound by its arithmetic, still no contraction).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sn_device.h"

namespace snk {

// Stage arguments are read through the constant address space wherever they
// live (the kernel-argument segment, or a device table of a batched launch):
// uniform scalar loads.
using SArgs = const __attribute__((address_space(4))) StageArgs&;
using SArgsPtr = const __attribute__((address_space(4))) StageArgs*;

// ---------------------------------------------------------------- storage
template <typename T>
struct Store;

using rsrc_t = __amdgpu_buffer_rsrc_t;
using u32x2 = uint32_t __attribute__((ext_vector_type(2)));

// Buffer resource over `bytes` bytes from `base` (raw, untyped). Accesses whose
// per-lane offset is at or beyond `bytes` read 0 and write nothing.
__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// Cache policy of the stage's psi stores and of its psi^n row copies: both
// are touched once per stage (the stores are read back by the next stage,
// after ~0.5 GB of other traffic), so they are marked non-temporal (nt) and
// do not evict the stencil and halo lines that neighbouring tiles still
// read. Measured on the 700^2 x 256 lattice (FP32): 0.669 -> 0.604 ms per
// Heun step; the 1300^2 x 512 cavity 4.16 -> 3.72 ms. Marking the stencil
// copies as well was slower (0.620 ms; the cavity 4.32 ms): their halo rows
// are re-read.
#ifndef SN_STORE_CPOL
#define SN_STORE_CPOL 2
#endif
#ifndef SN_OLD_CPOL
#define SN_OLD_CPOL 2
#endif

// A per-lane byte offset that the buffer range check always rejects.
constexpr uint32_t kDropOffset = 0x80000000u;

template <>
struct Store<float> {
    static __device__ __forceinline__ float2 load2(const char* p) { return *reinterpret_cast<const float2*>(p); }
    static __device__ __forceinline__ float2 round2(float2 v, uint32_t) { return v; }
    static __device__ __forceinline__ void store2(char* p, float2 v) { *reinterpret_cast<float2*>(p) = v; }
    static __device__ __forceinline__ void store1(char* p, float v) { *reinterpret_cast<float*>(p) = v; }
    static __device__ __forceinline__ float2 bload2(rsrc_t r, uint32_t voff, uint32_t soff) {
        return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    }
    static __device__ __forceinline__ void bstore2(rsrc_t r, uint32_t voff, uint32_t soff, float2 v) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, SN_STORE_CPOL);
    }
    static __device__ __forceinline__ void bstore1(rsrc_t r, uint32_t voff, uint32_t soff, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
    }
};

// bfloat16 kept as raw 16-bit patterns: widening is exact, narrowing rounds
// to nearest even (NaN stays NaN).
__device__ __forceinline__ float bf16_widen(uint32_t b) { return __uint_as_float(b << 16); }
__device__ __forceinline__ uint32_t bf16_narrow(float v) {
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (u >> 16) | 0x40u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

using bf16x2_t = short __attribute__((ext_vector_type(2)));

// MurmurHash3's 32-bit finalizer (fmix32): a bijective mix of the input bits,
// used to derive a reproducible, well-mixed key per (stage, ordinate) for the
// rounding bits (wave-uniform: scalar instructions).
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

template <>
struct Store<uint16_t> {
    static __device__ __forceinline__ float2 load2(const char* p) {
        const uint32_t u = *reinterpret_cast<const uint32_t*>(p);
        return make_float2(bf16_widen(u & 0xffffu), bf16_widen(u >> 16));
    }
    // Stochastic rounding to bfloat16 with 16 random bits per value: adding
    // them to the magnitude bits below the kept 16 and truncating rounds up
    // with probability equal to the discarded fraction, so the stored value
    // is unbiased. Round-to-nearest would drop every update smaller than half
    // a bfloat16 ulp (2^-9 relative) and let slowly changing fluxes stagnate.
    // gfx950's v_cvt_sr_bf16_f32 does exactly this with the top 16 bits of
    // its random operand (NaN quieted, Inf kept), one instruction per value,
    // writing either half of the packed pair; the low half of the random
    // operand is not read (whole solves are bit-identical with it cleared).
    // From one mixed word h: the first value takes low(h) ^ high(h), the
    // second high(h). h << 16 is formed with a byte permute: as a shift the
    // compiler would fold it into a second (quarter-rate) integer multiply of
    // the hash. The pair starts from h's bits, both halves overwritten, so no
    // register is cleared first.
    static __device__ __forceinline__ float2 round2(float2 v, uint32_t h) {
        const uint32_t r0 = __builtin_amdgcn_perm(0u, h, 0x01000c0cu) ^ h;  // top half: low(h) ^ high(h)
        bf16x2_t p = __builtin_bit_cast(bf16x2_t, h);
        p = __builtin_amdgcn_cvt_sr_bf16_f32(p, v.y, h, true);
        p = __builtin_amdgcn_cvt_sr_bf16_f32(p, v.x, r0, false);
        const uint32_t u = __builtin_bit_cast(uint32_t, p);
        return make_float2(bf16_widen(u & 0xffffu), bf16_widen(u >> 16));
    }
    // v must already be representable (round2): narrowing is then exact.
    static __device__ __forceinline__ void store2(char* p, float2 v) {
        *reinterpret_cast<uint32_t*>(p) = (__float_as_uint(v.x) >> 16) | (__float_as_uint(v.y) & 0xffff0000u);
    }
    static __device__ __forceinline__ void store1(char* p, float v) {
        *reinterpret_cast<uint16_t*>(p) = (uint16_t)(__float_as_uint(v) >> 16);
    }
    static __device__ __forceinline__ float2 bload2(rsrc_t r, uint32_t voff, uint32_t soff) {
        const uint32_t u = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
        return make_float2(bf16_widen(u & 0xffffu), bf16_widen(u >> 16));
    }
    static __device__ __forceinline__ void bstore2(rsrc_t r, uint32_t voff, uint32_t soff, float2 v) {
        __builtin_amdgcn_raw_buffer_store_b32((__float_as_uint(v.x) >> 16) | (__float_as_uint(v.y) & 0xffff0000u), r,
                                              voff, soff, SN_STORE_CPOL);
    }
    static __device__ __forceinline__ void bstore1(rsrc_t r, uint32_t voff, uint32_t soff, float v) {
        __builtin_amdgcn_raw_buffer_store_b16((unsigned short)(__float_as_uint(v) >> 16), r, voff, soff, 0);
    }
};

// ---------------------------------------------------------------- helpers
// Lane l receives x from lane l-1; lane 0, which has no source lane, keeps
// `edge` (DPP wave_shr:1 with bound_ctrl off). One instruction over the full
// wave: writing this as a select on the lane index lets the compiler mask
// lane 0 out of EXEC around the move, and a masked-out lane is no valid
// source for lane 1.
__device__ __forceinline__ float lane_from_left(float x, float edge) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(x), 0x138, 0xf, 0xf, false));
}
// Lane l receives x from lane l+1; lane 63 keeps `edge` (DPP wave_shl:1).
__device__ __forceinline__ float lane_from_right(float x, float edge) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(x), 0x130, 0xf, 0xf, false));
}

// minmod(a, b): the argument of smaller magnitude when both have the same
// strict sign, else 0 -- which is the median of a, b and 0 (one v_med3_f32;
// it returns one of its operands exactly).
__device__ __forceinline__ float minmod(float a, float b) {
    return __builtin_amdgcn_fmed3f(a, b, 0.0f);
}

// Order 3 (Sec. 4.2, eq. eq_V_limiter). The limiter's factor of a face with
// reconstruction increment d is (b^2 + e^2 + 2 d b) / (b^2 + 2 d^2 + b d + e^2)
// with b = max - c for d > 0 and b = min - c for d < 0 (max, min over the cell
// and its four neighbours), and 1 for d = 0. The two faces of one direction
// have increments +A and -A (A = |increment|); negating both d and b leaves
// the factor unchanged, so they are the factors of A with b_up = max - c and
// b_dn = c - min, both >= 0. The quotient uses the hardware reciprocal
// (within 1 ulp): the factor only scales an increment, so its last bit is far
// below the FP32 error of the stage.
__device__ __forceinline__ float venkat_pair(float A, float b_up, float b_dn, float e2) {
    const float a2 = 2.0f * A * A;
    const float qu = fmaf(b_up, b_up, e2), qd = fmaf(b_dn, b_dn, e2);
    const float fu = fmaf(2.0f * A, b_up, qu) * __builtin_amdgcn_rcpf(fmaf(A, b_up, qu + a2));
    const float fd = fmaf(2.0f * A, b_dn, qd) * __builtin_amdgcn_rcpf(fmaf(A, b_dn, qd + a2));
    return A == 0.0f ? 1.0f : fminf(fu, fd);
}

// The limited reconstruction of a cell with value c and neighbours W, E, S,
// N: returns the limiter L (the minimum of the four faces' factors) and the
// increments to its east and north face midpoints, ax = g_x h/2 = (E - W)/4
// and ay = (N - S)/4 (the Green-Gauss gradient of a square cell is the
// central difference). Face values: c + L ax (east), c - L ax (west), c + L
// ay (north), c - L ay (south).
// The largest and smallest of three values, one instruction each. (Through
// fmaxf / fminf the compiler first quiets every operand that may be a
// signalling NaN, one more instruction per operand, because it cannot tell
// that staged values never are; for the values this code compares the
// results are the same.)
__device__ __forceinline__ float max3f(float a, float b, float c) {
    float r;
    asm("v_max3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ float min3f(float a, float b, float c) {
    float r;
    asm("v_min3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ float venkat_limit(float c, float W, float E, float S, float N, float e2, float& ax,
                                              float& ay) {
    ax = 0.25f * (E - W);
    ay = 0.25f * (N - S);
    const float mx = max3f(max3f(W, E, S), N, c);
    const float mn = min3f(min3f(W, E, S), N, c);
    const float b_up = mx - c, b_dn = c - mn;
    return fminf(venkat_pair(fabsf(ax), b_up, b_dn, e2), venkat_pair(fabsf(ay), b_up, b_dn, e2));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
    return v;
}

// ---------------------------------------------------------------- per-wave state
template <int TY>
struct WaveCtx {
    int y0;              // interior row of the wave's first output row (wave-uniform)
    int i0;              // interior column of the lane's first cell
    uint32_t lane_off;   // byte offset of the lane's cell pair within a padded row
    uint32_t store_off;  // lane_off for lanes storing a full pair, kDropOffset otherwise
    uint32_t single_off; // lane_off for a lane owning only its first cell, kDropOffset otherwise
    // Ghost frame of the written state (kDropOffset for lanes that own no
    // boundary cell): byte offsets in a row of ghost columns -1, -2 (lane
    // holding column 0) and nx, nx+1 (lane holding column nx-1).
    uint32_t gw1, gw2, ge1, ge2;
    bool ge_first;       // column nx-1 is the lane's first cell
    bool xb_w, xb_e0, xb_e1;  // the lane's cell 0 west face / cell 0 east face / cell 1 east face is on the grid's boundary
    bool ghost_wave;     // the wave holds a boundary cell (wave-uniform)
    uint32_t pitchb;     // bytes per padded row
    uint32_t seed;       // BF16 storage: stages finalised so far (rounding bits), else 0
    uint32_t planeb;     // bytes per plane
    bool ragged;         // some lane of the wave owns only its first cell (wave-uniform)
    bool v0, v1;         // the lane's cells are output cells of this wave
    float2 st[TY];       // dt sigma_t per cell
    float2 bb[TY];       // dt (sigma_s / (2 pi) phi + Q) per cell
    float2 phacc[TY];    // sum_k w_k psi_out over the group's ordinates
};

// ---------------------------------------------------------------- row staging
// A workgroup is W compute waves stacked in y plus one loader wave. For every
// ordinate the loader copies the workgroup's W TY + 4 stencil rows (and, for
// the averaging stage, the W TY rows of psi^n) from HBM straight into a ring
// of kSlots LDS slots (buffer loads with an LDS destination), kSlots - 1
// ordinates ahead of the compute waves; one barrier per ordinate hands a slot
// over. The compute waves issue no global loads in the ordinate loop and the
// loader no stores, so neither waits on the other's memory traffic (the wait
// counters are per wave). The depth is set by the latency of a copy under
// full load (several microseconds), not by its bytes: the stages without
// psi^n rows keep 4 ordinates in flight, the averaging stage, whose slots
// are almost twice as large, 2, both in ~32 KB of LDS per workgroup, plus
// the tile's face table (16 bytes per rectangle-boundary face, a few KB).
// A slot holds the stencil rows, the x-halo, the order-3 edge traces and the
// psi^n rows, in that order, so that a cell's offset in it does not depend
// on the stage kind (the host's face tables hold such offsets).
#ifndef SN_RING_SLOTS
#define SN_RING_SLOTS 3
#endif
#ifndef SN_RING_SLOTS_NO_OLD
#define SN_RING_SLOTS_NO_OLD 5
#endif

// XH: extra x-halo rows, one above and one below the output rows (order 3,
// whose limiter needs the cells beside the tile in the rows next to a face).
template <typename T, int TY, int W, int MODE, int XH = 0>
struct Ring {
    static constexpr int kSlots = MODE == kAverage ? SN_RING_SLOTS : SN_RING_SLOTS_NO_OLD;  // in flight + computed
    static_assert(kSlots >= 2 && kSlots <= 5, "ring depth");
    static constexpr int kRows = W * TY + 4;                             // stencil rows
    static constexpr int kOldRows = MODE == kAverage ? W * TY : 0;       // psi^n rows
    static constexpr int kRowBytes = kWave * 2 * (int)sizeof(T);         // 128 cells
    static constexpr int kDmaBytes = 16;                                   // bytes per lane per copy
    static constexpr int kRowsPerDma = kWave * kDmaBytes / kRowBytes;    // 2 (f32) or 4 (bf16)
    static constexpr int kLanesPerRow = kWave / kRowsPerDma;
    static constexpr int kDmaStencil = (kRows + kRowsPerDma - 1) / kRowsPerDma;
    static constexpr int kDmaOld = (kOldRows + kRowsPerDma - 1) / kRowsPerDma;
    // x-halo of the output rows (and XH / 2 more rows on each side): cells
    // -2, -1, 128, 129 of the tile, one dword per lane (4 lanes per row for
    // FP32, 2 for BF16)
    static constexpr int kHaloRows = W * TY + XH;
    static constexpr int kHaloRowBytes = 4 * (int)sizeof(T);
    static constexpr int kHaloLanesPerRow = kHaloRowBytes / 4;
    static constexpr int kHaloRowsPerDma = kWave / kHaloLanesPerRow;
    static constexpr int kDmaHalo = (kHaloRows + kHaloRowsPerDma - 1) / kHaloRowsPerDma;
    static constexpr int kHaloOffset = kDmaStencil * kRowsPerDma * kRowBytes;  // bytes into the slot
    static_assert(kHaloOffset == ring_halo_elem(kRows, (int)sizeof(T)) * (int)sizeof(T),
                  "slot layout of the host's face tables");
    // Order 3: the loader's trace of the one cell beyond the tile that each
    // output row's x-faces need (east face of cell -1 when xi > 0, west face
    // of cell 128 when xi < 0), one float per output row.
    static constexpr int kEdgeOffset = kHaloOffset + kDmaHalo * kWave * 4;
    static constexpr int kEdgeBytes = XH > 0 ? (W * TY * 4 + 15) / 16 * 16 : 0;
    static constexpr int kOldOffset = kEdgeOffset + kEdgeBytes;          // psi^n rows (averaging stage)
    static_assert(kOldOffset % 16 == 0, "copies land on 16-byte lanes");
    static constexpr int kSlotBytes = kOldOffset + kDmaOld * kRowsPerDma * kRowBytes;
    static constexpr int kDmaPerOrd = kDmaStencil + kDmaOld + kDmaHalo;  // copies per ordinate
    static constexpr int kBytes = kSlots * kSlotBytes;
    // outstanding copies allowed while waiting for the oldest ordinate when
    // `ahead` later ordinates are in flight (the counter field holds at most
    // 63: waiting for more is only conservative)
    static constexpr int wait_ahead(int ahead) { return kDmaPerOrd * ahead < 64 ? kDmaPerOrd * ahead : 63; }
};

// Extra x-halo rows of an order.
template <int ORDER>
constexpr int kExtraHalo = ORDER == 3 ? 2 : 0;

using lds_ptr = __attribute__((address_space(3))) void*;

// s_waitcnt with only the vector-memory count constrained (gfx9 encoding:
// vmcnt in bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at maximum).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Per-lane byte offsets of the loader's copies within a row, fixed for the
// whole launch. Copies of columns no output cell of the tile depends on (past
// the east ghost cells of the grid, or past the interior for psi^n) carry the
// dropped offset and fetch nothing.
struct LoaderOffsets {
    uint32_t stencil;  // rows of the stage input
    uint32_t old;      // rows of psi^n (averaging stage)
    uint32_t halo;     // x-halo dwords of the output rows
};

// Lane l copies kDmaBytes at column offset (l % kLanesPerRow) kDmaBytes of
// row l / kLanesPerRow of each kRowsPerDma-row block; the LDS copy lands at
// the block's base + l kDmaBytes, i.e. row-major [row][128 cells], the layout
// the compute lanes read. The x-halo dwords: lane l covers dword
// (l % kHaloLanesPerRow) of output row l / kHaloLanesPerRow, the first half
// of a row's dwords left of the tile, the rest right of it.
template <typename T, int TY, int W, int MODE, int XH>
__device__ __forceinline__ LoaderOffsets loader_offsets(SArgs a, int col0, uint32_t tile_off, uint32_t pitchb) {
    using R = Ring<T, TY, W, MODE, XH>;
    constexpr int kCellsPerCopy = R::kDmaBytes / (int)sizeof(T);
    const int lane = threadIdx.x & (kWave - 1);
    LoaderOffsets o;
    const int c = col0 + (lane % R::kLanesPerRow) * kCellsPerCopy;  // interior column of the copy's first cell
    const uint32_t voff = tile_off + (uint32_t)(lane % R::kLanesPerRow) * R::kDmaBytes +
                          (uint32_t)(lane / R::kLanesPerRow) * pitchb;
    o.stencil = c < a.nx + kGhost ? voff : kDropOffset;
    o.old = c < a.nx ? voff : kDropOffset;
    const int e = lane % R::kHaloLanesPerRow, hr = lane / R::kHaloLanesPerRow;
    const int half = R::kHaloLanesPerRow / 2;
    // rows past the workgroup's output rows, and east cells past the grid's
    // ghost cells, are not needed
    const bool right_needed = col0 + kTileX < a.nx + kGhost;
    o.halo = hr >= R::kHaloRows || (e >= half && !right_needed)
                 ? kDropOffset
                 : (e < half ? tile_off - 2 * (uint32_t)sizeof(T) + 4 * e
                             : tile_off + (uint32_t)(kTileX * sizeof(T)) + 4 * (e - half)) +
                       (uint32_t)hr * pitchb;
    return o;
}

// Loader: ordinate k's rows into ring slot `slot`.
template <typename T, int TY, int W, int MODE, int XH>
__device__ __forceinline__ void ring_issue(SArgs a, int k, int yw, const LoaderOffsets& lo, uint32_t pitchb,
                                           uint32_t planeb, char* slot) {
    using R = Ring<T, TY, W, MODE, XH>;
    const rsrc_t r = make_rsrc(static_cast<const char*>(a.psi_in) + (size_t)k * planeb, planeb);
#pragma unroll
    for (int i = 0; i < R::kDmaStencil; ++i)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)(slot + i * R::kRowsPerDma * R::kRowBytes),
                                                 R::kDmaBytes, lo.stencil,
                                                 (uint32_t)(yw + i * R::kRowsPerDma) * pitchb, 0, 0);
#pragma unroll
    for (int i = 0; i < R::kDmaHalo; ++i)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)(slot + R::kHaloOffset + i * kWave * 4), 4, lo.halo,
                                                 (uint32_t)(yw + kGhost - XH / 2 + i * R::kHaloRowsPerDma) * pitchb,
                                                 0, 0);
    if (MODE == kAverage) {
        const rsrc_t ro = make_rsrc(static_cast<const char*>(a.psi_old) + (size_t)k * planeb, planeb);
#pragma unroll
        for (int i = 0; i < R::kDmaOld; ++i)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                ro, (lds_ptr)(slot + R::kOldOffset + i * R::kRowsPerDma * R::kRowBytes), R::kDmaBytes, lo.old,
                (uint32_t)(yw + kGhost + i * R::kRowsPerDma) * pitchb, 0, SN_OLD_CPOL);
    }
}

// One staged cell pair of the compute lane `lane` from LDS.
template <typename T>
__device__ __forceinline__ float2 ring_read(const char* row, int lane);
template <>
__device__ __forceinline__ float2 ring_read<float>(const char* row, int lane) {
    return reinterpret_cast<const float2*>(row)[lane];
}
template <>
__device__ __forceinline__ float2 ring_read<uint16_t>(const char* row, int lane) {
    const uint32_t u = reinterpret_cast<const uint32_t*>(row)[lane];
    return make_float2(bf16_widen(u & 0xffffu), bf16_widen(u >> 16));
}

// The staged x-halo of one output row: cells -2, -1, 128, 129 of the tile
// (the same address in every lane: a broadcast read).
template <typename T>
__device__ __forceinline__ float4 halo_read(const char* h);
template <>
__device__ __forceinline__ float4 halo_read<float>(const char* h) {
    return *reinterpret_cast<const float4*>(h);
}
template <>
__device__ __forceinline__ float4 halo_read<uint16_t>(const char* h) {
    const uint2 u = *reinterpret_cast<const uint2*>(h);
    return make_float4(bf16_widen(u.x & 0xffffu), bf16_widen(u.x >> 16), bf16_widen(u.y & 0xffffu),
                       bf16_widen(u.y >> 16));
}

// Order 3, in the loader wave once ordinate k's rows have landed in `slot`:
// for every output row q of the workgroup, the trace at the tile's edge that
// lanes 0 / 63 of the compute waves need and no lane of theirs holds -- the
// east face of cell -1 (xi > 0) or the west face of cell 128 (xi < 0), the
// Venkatakrishnan-limited reconstruction of that cell from its staged x-halo
// and the halo of the rows above and below, evaluated as the compute waves
// would. One pass of W TY lanes instead of one 64-lane pass per output row in
// every compute wave.
using const_ord_ptr = const __attribute__((address_space(4))) OrdConst*;

template <typename T, int TY, int W, int MODE, int XH>
__device__ __forceinline__ void loader_edges(SArgs a, int k, char* slot) {
    using R = Ring<T, TY, W, MODE, XH>;
    const int q = threadIdx.x & (kWave - 1);  // output row of the workgroup
    const bool sx = (((const_ord_ptr)a.ord + k)->flags & 1) != 0;  // wave-uniform
    if (q < W * TY) {
        const float4 hu = halo_read<T>(slot + R::kHaloOffset + q * R::kHaloRowBytes);       // row above
        const float4 hv = halo_read<T>(slot + R::kHaloOffset + (q + 1) * R::kHaloRowBytes); // the row
        const float4 hd = halo_read<T>(slot + R::kHaloOffset + (q + 2) * R::kHaloRowBytes); // row below
        const char* row = slot + (q + 2) * R::kRowBytes;  // the row's staged cells 0 .. 127
        float e, ax, ay;
        if (sx) {
            const float L = venkat_limit(hv.y, hv.x, ring_read<T>(row, 0).x, hu.y, hd.y, a.eps2, ax, ay);
            e = fmaf(L, ax, hv.y);
        } else {
            const float L = venkat_limit(hv.z, ring_read<T>(row, kWave - 1).y, hv.w, hu.z, hd.z, a.eps2, ax, ay);
            e = fmaf(-L, ax, hv.z);
        }
        reinterpret_cast<float*>(slot + R::kEdgeOffset)[q] = e;
    }
}

// A staged cell of a ring slot by its element offset (face tables).
template <typename T>
__device__ __forceinline__ float slot_cell(const char* sb, uint32_t o) {
    o &= kFaceOffMask;
    if (sizeof(T) == 4) return *reinterpret_cast<const float*>(sb + 4 * o);
    return bf16_widen(*reinterpret_cast<const uint16_t*>(sb + 2 * o));
}

// Rectangle-boundary faces (outflow and inflow QoIs of Sec. 3.1.2), in the
// loader wave once ordinate k's rows are in slot `sb`: every face of the
// lane's table entries (all of one rectangle) adds w |Omega.n| times the
// face's upwind trace to the lane's outflow or inflow sum in FP64. The trace
// is reconstructed from the staged cells as the compute waves reconstruct
// it for the flux: the upwind cell (order 1), plus half its minmod slope
// along the normal (order 2), plus its Venkatakrishnan-limited gradient
// (order 3; first order on the grid's boundary). One lane per face instead
// of a 64-lane pass of every compute wave that owns one.
struct FaceOrd {
    bool sx, sy;    // xi > 0, eta > 0
    double fx, fy;  // w |xi|, w |eta|
};

template <int ORDER, typename T>
__device__ __forceinline__ void face_flux(const FaceOrd& fo, float eps2, const char* sb, uint4 raw, double& fout,
                                          double& fin) {
    const uint32_t o0 = raw.x & 0xffffu, o1 = raw.x >> 16, o2 = raw.y & 0xffffu, o3 = raw.y >> 16;
    const bool yaxis = (o1 >> 14) & 1u, holds_c2 = (o1 >> 15) & 1u;
    const bool first = (o2 >> 14) & 1u, valid = (o2 >> 15) & 1u;
    const bool dir = yaxis ? fo.sy : fo.sx;  // the flow crosses the face from c1 to c2
    const float c1 = slot_cell<T>(sb, o1), c2 = slot_cell<T>(sb, o2);
    float tr;
    if (ORDER == 1) {
        tr = dir ? c1 : c2;
    } else if (ORDER == 2) {
        const float c0 = slot_cell<T>(sb, o0), c3 = slot_cell<T>(sb, o3);
        const float d12 = c2 - c1;
        tr = dir ? fmaf(0.5f, minmod(c1 - c0, d12), c1) : fmaf(-0.5f, minmod(d12, c3 - c2), c2);
    } else {
        const float c0 = slot_cell<T>(sb, o0), c3 = slot_cell<T>(sb, o3);
        const float t1m = slot_cell<T>(sb, raw.z & 0xffffu), t1p = slot_cell<T>(sb, raw.z >> 16);
        const float t2m = slot_cell<T>(sb, raw.w & 0xffffu), t2p = slot_cell<T>(sb, raw.w >> 16);
        const float c = dir ? c1 : c2;                          // upwind cell
        const float nm = dir ? c0 : c1, np = dir ? c2 : c3;      // its neighbours along the normal
        const float tm = dir ? t1m : t2m, tp = dir ? t1p : t2p;  // and across it
        float gx, gy;
        const float L = venkat_limit(c, yaxis ? tm : nm, yaxis ? tp : np, yaxis ? nm : tm, yaxis ? np : tp, eps2,
                                     gx, gy);
        tr = first ? c : fmaf(dir ? L : -L, yaxis ? gy : gx, c);
    }
    const bool out = dir != holds_c2;
    const double r = fma(yaxis ? fo.fy : fo.fx, (double)tr, out ? fout : fin);
    if (valid) {
        if (out) fout = r;
        else fin = r;
    }
}

template <int ORDER, typename T>
__device__ __forceinline__ FaceOrd face_ord(SArgs a, int k) {
    const const_ord_ptr ok = (const_ord_ptr)a.ord + k;  // scalar loads
    const int fg = ok->flags;
    return FaceOrd{(fg & 1) != 0, (fg & 2) != 0, ok->fx, ok->fy};
}

// N entries held in registers (the common case: every load of the ordinate
// in flight together).
template <int ORDER, typename T, int N>
__device__ __forceinline__ void face_fluxes_regs(SArgs a, int k, const char* sb, const uint4 (&fr)[kFaceRegs],
                                                 double& fout, double& fin) {
    const FaceOrd fo = face_ord<ORDER, T>(a, k);
#pragma unroll
    for (int e = 0; e < N; ++e) face_flux<ORDER, T>(fo, a.eps2, sb, fr[e], fout, fin);
}

// fl entries from the tile's table in LDS (tiles with more faces per lane).
template <int ORDER, typename T>
__device__ __forceinline__ void face_fluxes_lds(SArgs a, int k, const char* sb, const FaceEntry* tab, int fl,
                                                double& fout, double& fin) {
    const FaceOrd fo = face_ord<ORDER, T>(a, k);
    for (int e = 0; e < fl; ++e)
        face_flux<ORDER, T>(fo, a.eps2, sb, *reinterpret_cast<const uint4*>(tab + e), fout, fin);
}

// Stores one cell pair (or the first cell only) at byte offset `off` of plane base `p`.
template <typename T>
__device__ __forceinline__ void put_pair(char* p, size_t off, float2 v, bool v0, bool v1) {
    if (v1) Store<T>::store2(p + off, v);
    else if (v0) Store<T>::store1(p + off, v.x);
}

// Keeps the ghost frame of the written state (the rule of the header comment):
// ordinate k leaving through a side repeats its boundary cell into the first
// ghost layer; on a reflective side the mirror ordinate, which enters there,
// gets the value in both layers. Lanes without a boundary cell carry the
// dropped offset, so the stores need no branches.
template <typename T, int TY, bool SX, bool SY>
__device__ __forceinline__ void write_frame(SArgs a, const OrdConst& o, int k, int j, uint32_t rowb,
                                            rsrc_t rout, const WaveCtx<TY>& w, float2 v) {
    const char* out = static_cast<const char*>(a.psi_out);
    if (!SX) {  // leaves through W
        Store<T>::bstore1(rout, w.gw1, rowb, v.x);
        if (a.bc[kW] == kReflect) {
            const rsrc_t rm = make_rsrc(out + (size_t)o.mx * w.planeb, w.planeb);
            Store<T>::bstore1(rm, w.gw1, rowb, v.x);
            Store<T>::bstore1(rm, w.gw2, rowb, v.x);
        }
    } else {  // leaves through E
        const float ve = w.ge_first ? v.x : v.y;
        Store<T>::bstore1(rout, w.ge1, rowb, ve);
        if (a.bc[kE] == kReflect) {
            const rsrc_t rm = make_rsrc(out + (size_t)o.mx * w.planeb, w.planeb);
            Store<T>::bstore1(rm, w.ge1, rowb, ve);
            Store<T>::bstore1(rm, w.ge2, rowb, ve);
        }
    }
    const int jg = SY ? a.ny - 1 : 0;  // boundary row the ordinate leaves through
    if (j == jg) {
        const uint32_t g1 = (uint32_t)(SY ? a.ny + kGhost : 1) * w.pitchb;  // first ghost row
        const uint32_t g2 = (uint32_t)(SY ? a.ny + kGhost + 1 : 0) * w.pitchb;
        Store<T>::bstore2(rout, w.store_off, g1, v);
        if (w.ragged) Store<T>::bstore1(rout, w.single_off, g1, v.x);
        if (a.bc[SY ? kN : kS] == kReflect) {
            const rsrc_t rm = make_rsrc(out + (size_t)o.my * w.planeb, w.planeb);
            Store<T>::bstore2(rm, w.store_off, g1, v);
            Store<T>::bstore2(rm, w.store_off, g2, v);
            if (w.ragged) {
                Store<T>::bstore1(rm, w.single_off, g1, v.x);
                Store<T>::bstore1(rm, w.single_off, g2, v.x);
            }
        }
    }
}

// Order 3: every ordinate's ghost cells hold the side's ghost value (set at
// init on vacuum and inflow sides, never rewritten). On a reflective side the
// ghost of ordinate k is its mirror's boundary cell, so every ordinate writes
// its boundary cells into its mirror's ghost layers, entering or leaving.
template <typename T, int TY>
__device__ __forceinline__ void write_frame_all(SArgs a, const OrdConst& o, int j, uint32_t rowb,
                                                const WaveCtx<TY>& w, float2 v) {
    const char* out = static_cast<const char*>(a.psi_out);
    if (a.bc[kW] == kReflect || a.bc[kE] == kReflect) {
        const rsrc_t rm = make_rsrc(out + (size_t)o.mx * w.planeb, w.planeb);
        if (a.bc[kW] == kReflect) {
            Store<T>::bstore1(rm, w.gw1, rowb, v.x);
            Store<T>::bstore1(rm, w.gw2, rowb, v.x);
        }
        if (a.bc[kE] == kReflect) {
            const float ve = w.ge_first ? v.x : v.y;
            Store<T>::bstore1(rm, w.ge1, rowb, ve);
            Store<T>::bstore1(rm, w.ge2, rowb, ve);
        }
    }
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const bool s_side = side == 0;
        if (a.bc[s_side ? kS : kN] != kReflect || j != (s_side ? 0 : a.ny - 1)) continue;
        const uint32_t g1 = (uint32_t)(s_side ? 1 : a.ny + kGhost) * w.pitchb;
        const uint32_t g2 = (uint32_t)(s_side ? 0 : a.ny + kGhost + 1) * w.pitchb;
        const rsrc_t rm = make_rsrc(out + (size_t)o.my * w.planeb, w.planeb);
        Store<T>::bstore2(rm, w.store_off, g1, v);
        Store<T>::bstore2(rm, w.store_off, g2, v);
        if (w.ragged) {
            Store<T>::bstore1(rm, w.single_off, g1, v.x);
            Store<T>::bstore1(rm, w.single_off, g2, v.x);
        }
    }
}

// ---------------------------------------------------------------- one ordinate
// Window row r holds grid row y0 - 2 + r; output row t is window row t + 2.
template <int ORDER, int MODE, typename T, int TY, int W, bool SX, bool SY>
__device__ __forceinline__ void stage_ordinate(SArgs a, const OrdConst& o, int k, WaveCtx<TY>& w,
                                               const float2 (&win)[TY + 4], const float4 (&halo)[TY + kExtraHalo<ORDER>],
                                               const float2 (&oldv)[TY], const float* edge) {
    constexpr int D = SY ? 0 : 1;  // y-traces of output row t: Ry[t + 1 + D] (south), Ry[t + 2 + D] (north)
    constexpr float HX = SX ? 0.5f : -0.5f;
    constexpr float HY = SY ? 0.5f : -0.5f;

    // Reconstructions at the downwind y-face of window rows (eta > 0: top face).
    float2 Ry[TY + 3];
    // Order 3: traces of the output rows' x-faces (west of cell 0, east of
    // cells 0 and 1), first order on the grid's boundary faces.
    float xw[TY], xe0[TY], xe1[TY];
    if (ORDER == 3) {
        // halo[h] is the x-halo of window row h + 1. Rows 1 + D .. TY + 1 + D
        // hold every upwind cell of the output rows' faces.
#pragma unroll
        for (int r = 1 + D; r <= TY + 1 + D; ++r) {
            const float c0 = win[r].x, c1 = win[r].y;
            const float4 hv = halo[r - 1];               // cells -2, -1, 128, 129 of window row r
            const float lf = lane_from_left(c1, hv.y);   // cell left of c0
            const float rt = lane_from_right(c0, hv.z);  // cell right of c1
            float ax0, ay0, ax1, ay1;
            const float L0 = venkat_limit(c0, lf, c1, win[r - 1].x, win[r + 1].x, a.eps2, ax0, ay0);
            const float L1 = venkat_limit(c1, c0, rt, win[r - 1].y, win[r + 1].y, a.eps2, ax1, ay1);
            {
                // downwind y-face of row r; on the grid's boundary faces (south
                // of row 0, north of row ny-1) the upwind cell's own value
                const int gy = w.y0 - 2 + r;
                const bool bnd = SY ? (gy == -1 || gy == a.ny - 1) : (gy == 0 || gy == a.ny);
                const float sy = SY ? 1.0f : -1.0f;
                Ry[r] = bnd ? win[r] : make_float2(fmaf(sy * L0, ay0, c0), fmaf(sy * L1, ay1, c1));
            }
            if (r >= 2 && r <= TY + 1) {
                const int t = r - 2;
                // the trace of the cell beyond the tile (loader_edges)
                const float e = edge[t];
                if (SX) {
                    // lane 0's west face is the east face of cell -1
                    const float REl = lane_from_left(fmaf(L1, ax1, c1), e);
                    xw[t] = w.xb_w ? lf : REl;
                    xe0[t] = w.xb_e0 ? c0 : fmaf(L0, ax0, c0);
                    xe1[t] = w.xb_e1 ? c1 : fmaf(L1, ax1, c1);
                } else {
                    // lane 63's east face is the west face of cell 128
                    const float RWr = lane_from_right(fmaf(-L0, ax0, c0), e);
                    xw[t] = w.xb_w ? c0 : fmaf(-L0, ax0, c0);
                    xe0[t] = w.xb_e0 ? c1 : fmaf(-L1, ax1, c1);
                    xe1[t] = w.xb_e1 ? rt : RWr;
                }
            }
        }
    } else if (ORDER == 2) {
        float2 dy[TY + 3];  // dy[r] = win[r + 1] - win[r]
#pragma unroll
        for (int r = D; r <= TY + 1 + D; ++r) dy[r] = make_float2(win[r + 1].x - win[r].x, win[r + 1].y - win[r].y);
#pragma unroll
        for (int r = 1 + D; r <= TY + 1 + D; ++r) {
            const float mx = minmod(dy[r - 1].x, dy[r].x);
            const float my = minmod(dy[r - 1].y, dy[r].y);
            Ry[r] = make_float2(fmaf(HY, mx, win[r].x), fmaf(HY, my, win[r].y));
        }
    } else {
#pragma unroll
        for (int r = 1 + D; r <= TY + 1 + D; ++r) Ry[r] = win[r];
    }

    char* const outk = static_cast<char*>(a.psi_out) + (size_t)k * w.planeb;
    const rsrc_t rout = make_rsrc(outk, w.planeb);
#pragma unroll
    for (int t = 0; t < TY; ++t) {
        const int j = w.y0 + t;
        if (j >= a.ny) break;  // wave-uniform
        const float c0 = win[t + 2].x, c1 = win[t + 2].y;
        const float4 hv = halo[ORDER == 3 ? t + 1 : t];  // cells -2, -1 and 128, 129 of the tile
        const float L = lane_from_left(c1, hv.y);    // cell left of c0 (lane 0: cell -1)
        const float Rn = lane_from_right(c0, hv.z);  // cell right of c1 (lane 63: cell 128)
        float dRx0, dRx1, tW0, tE0, tE1;       // x-differences and traces (west of cell 1 = east of cell 0)
        if (ORDER == 3) {
            tW0 = xw[t];
            tE0 = xe0[t];
            tE1 = xe1[t];
            dRx0 = tE0 - tW0;
            dRx1 = tE1 - tE0;
        } else if (ORDER == 2) {
            const float d01 = c1 - c0;
            const float m0 = minmod(c0 - L, d01), m1 = minmod(d01, Rn - c1);
            const float R0 = fmaf(HX, m0, c0), R1 = fmaf(HX, m1, c1);
            if (SX) {
                // lane 0: east-face value of cell -1 from the halo
                const float Rl = lane_from_left(R1, fmaf(HX, minmod(hv.y - hv.x, c0 - hv.y), hv.y));
                dRx0 = R0 - Rl;
                dRx1 = R1 - R0;
                tW0 = Rl;
                tE0 = R0;
                tE1 = R1;
            } else {
                // lane 63: west-face value of cell 128 from the halo
                const float Rr = lane_from_right(R0, fmaf(HX, minmod(hv.z - c1, hv.w - hv.z), hv.z));
                dRx0 = R1 - R0;
                dRx1 = Rr - R1;
                tW0 = R0;
                tE0 = R1;
                tE1 = Rr;
            }
        } else {
            if (SX) {
                dRx0 = c0 - L;
                dRx1 = c1 - c0;
                tW0 = L;
                tE0 = c0;
                tE1 = c1;
            } else {
                dRx0 = c1 - c0;
                dRx1 = Rn - c1;
                tW0 = c0;
                tE0 = c1;
                tE1 = Rn;
            }
        }
        const float2 tS = Ry[t + 1 + D], tN = Ry[t + 2 + D];

        if (MODE != kQoiOnly) {
            float2 v;
            float d0 = fmaf(-w.st[t].x, c0, w.bb[t].x);
            float d1 = fmaf(-w.st[t].y, c1, w.bb[t].y);
            d0 = fmaf(-o.cx, dRx0, d0);
            d1 = fmaf(-o.cx, dRx1, d1);
            d0 = fmaf(-o.cy, tN.x - tS.x, d0);
            d1 = fmaf(-o.cy, tN.y - tS.y, d1);
            v.x = c0 + d0;
            v.y = c1 + d1;
            if (MODE == kAverage) {
                v.x = 0.5f * (oldv[t].x + v.x);
                v.y = 0.5f * (oldv[t].y + v.y);
            }
            const uint32_t rowb = (uint32_t)(w.y0 + t + kGhost) * w.pitchb;
            uint32_t h = 0;
            if (sizeof(T) == 2) {  // rounding bits from (stage, ordinate, cell pair of the plane)
                const uint32_t sk = fmix32(fmix32(w.seed) + (uint32_t)k);  // wave-uniform
                // per cell pair: a multiplicative (Fibonacci) hash of the key
                // xor the pair's index, its two halves folded in round2. For a
                // fixed cell the bits follow the key, uniform over stages and
                // ordinates; one multiply instead of a second fmix32 (the
                // stage is bound by its VALU issue with BF16 storage).
                h = (sk ^ ((rowb + w.lane_off) / (uint32_t)sizeof(T))) * 0x9E3779B1u;
            }
            v = Store<T>::round2(v, h);
            Store<T>::bstore2(rout, w.store_off, rowb, v);  // halo and partial lanes drop the pair
            if (w.ragged) Store<T>::bstore1(rout, w.single_off, rowb, v.x);
            if (w.ghost_wave) {
                if (ORDER == 3) write_frame_all<T, TY>(a, o, j, rowb, w, v);
                else write_frame<T, TY, SX, SY>(a, o, k, j, rowb, rout, w, v);
            }
            w.phacc[t].x = fmaf(o.w, v.x, w.phacc[t].x);
            w.phacc[t].y = fmaf(o.w, v.y, w.phacc[t].y);
        }
    }
}

// The ordinate table is read-only for the whole launch: reading it through
// the constant address space makes it a scalar load, whose wait does not
// also wait for the next ordinate's window loads (const_ord_ptr).

template <int ORDER, int MODE, typename T, int TY, int W>
__device__ __forceinline__ void process_ordinate(SArgs a, int k, WaveCtx<TY>& w,
                                                 const float2 (&win)[TY + 4], const float4 (&halo)[TY + kExtraHalo<ORDER>],
                                                 const float2 (&oldv)[TY], const float* edge) {
    const const_ord_ptr q = (const_ord_ptr)a.ord + k;
    OrdConst o;
    o.cx = q->cx;
    o.cy = q->cy;
    o.w = q->w;
    o.flags = q->flags;
    o.mx = q->mx;
    o.my = q->my;
    o.fx = q->fx;
    o.fy = q->fy;
    switch (o.flags & 3) {
    case 3: stage_ordinate<ORDER, MODE, T, TY, W, true, true>(a, o, k, w, win, halo, oldv, edge); break;
    case 2: stage_ordinate<ORDER, MODE, T, TY, W, false, true>(a, o, k, w, win, halo, oldv, edge); break;
    case 1: stage_ordinate<ORDER, MODE, T, TY, W, true, false>(a, o, k, w, win, halo, oldv, edge); break;
    default: stage_ordinate<ORDER, MODE, T, TY, W, false, false>(a, o, k, w, win, halo, oldv, edge); break;
    }
}

// ---------------------------------------------------------------- one workgroup tile
// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// range of logical workgroups. Logical workgroups run ordinate group by
// ordinate group, each group's tiles row by row (x fastest), so an XCD works
// on one group (with 8 groups) over the whole grid: the tiles it holds at a
// time are each other's x- and y-neighbours, step through the same ordinates
// in lockstep, and read each other's halo lines from the XCD's L2. (With the
// groups of a tile adjacent instead, the halo lines mostly came from HBM:
// 1.35x the algorithmic reads in the averaging stage and 1.6x in the update
// stage on the 700 x 700 lattice, against 1.22x and 1.24x now.)
__device__ __forceinline__ int xcd_contiguous(int b, int nwg) {
    const int xcd = b & 7, q8 = b >> 3, per = nwg >> 3, rem = nwg & 7;
    return xcd < rem ? xcd * (per + 1) + q8 : rem * (per + 1) + (xcd - rem) * per + q8;
}

template <typename T, int TY, int W, int MODE, int XH>
struct StageLds {
    double red[W][kMaxQWave];
    double face_red[2 * kMaxRects];   // the loader wave's outflow, then inflow, per rectangle
    double probe_red[kMaxProbes][3];  // the loader wave's probe moments
    alignas(16) char ring[Ring<T, TY, W, MODE, XH>::kBytes];
};

using const_f64_ptr = const __attribute__((address_space(4))) double*;
using const_i32_ptr = const __attribute__((address_space(4))) int32_t*;

// The work of logical workgroup `logical` of one stage launch: tile and
// ordinate group, all ordinates of the group, epilogues. ftab: the dynamic
// LDS that holds the tile's face table (a.face_lds bytes).
template <int ORDER, int MODE, typename T, int TY, int W>
__device__ __forceinline__ void stage_tile(SArgs a, int logical, FaceEntry* ftab,
                                           StageLds<T, TY, W, MODE, kExtraHalo<ORDER>>& lds) {
    constexpr int XH = kExtraHalo<ORDER>;
    using R = Ring<T, TY, W, MODE, XH>;
    auto& red = lds.red;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int ntiles = a.ntx * a.nty;
    const int g = logical / ntiles;
    const int tile = logical - g * ntiles;
    const int tx = tile % a.ntx;
    const int tyi = tile / a.ntx;
    const int k0 = g * a.Mg;
    const int k1 = min(k0 + a.Mg, a.M);
    const int yw = tyi * W * TY;  // padded row of the workgroup's first staged row

    if (wave == W) {  // the loader wave
        const uint32_t es = (uint32_t)sizeof(T);
        const uint32_t pitchb = (uint32_t)a.pitch * es;
        const uint32_t planeb = (uint32_t)((size_t)a.plane * es);
        const uint32_t tile_off = (uint32_t)(a.ox + tx * kTileX) * es;  // 128-byte aligned
        const LoaderOffsets lo = loader_offsets<T, TY, W, MODE, XH>(a, tx * kTileX, tile_off, pitchb);
        // Space-time probes: between its copies the loader reads the tile's
        // probe cells of every staged ordinate from LDS. Lane l holds entries
        // pb + l pl .. pb + l pl + pl - 1, all of one probe (bit e of pvalid:
        // entry e is a cell, not padding). They are loaded here, before any
        // copy is in flight, so that waiting for them waits for no copy.
        int pl = 0;
        uint32_t poff[kProbePerLane];
        double pwt[kProbePerLane];
        uint32_t pvalid = 0;
        int my_probe = -1;
        double pm0 = 0.0, pm1 = 0.0, pm2 = 0.0;
#pragma unroll
        for (int e = 0; e < kProbePerLane; ++e) {
            poff[e] = 0;
            pwt[e] = 0.0;
        }
        // Rectangle-boundary faces: fl entries per lane, flanes lanes, a
        // lane's entries of one rectangle fq; up to kFaceRegs entries in
        // registers, more from a copy of the tile's table in LDS. Loaded
        // before any copy is in flight.
        int fl = 0, flanes = 0, fq = -1;
        double fout = 0.0, fin = 0.0;
        uint4 fr[kFaceRegs];
#pragma unroll
        for (int e = 0; e < kFaceRegs; ++e) fr[e] = make_uint4(0u, 0u, 0u, 0u);
        if (a.n_rects > 0) {
            const const_i32_ptr ft = (const_i32_ptr)a.ftile + 3 * tile;
            const int fb = ft[0];
            fl = ft[1];
            flanes = ft[2];
            const uint4* src = reinterpret_cast<const uint4*>(a.fent + fb);
            if (fl > face_regs(ORDER)) {
                for (int e = lane; e < fl * flanes; e += kWave) ftab[e] = a.fent[fb + e];
            } else if (lane < flanes) {
#pragma unroll
                for (int e = 0; e < kFaceRegs; ++e)
                    if (e < fl) fr[e] = src[lane * fl + e];
            }
            if (lane < flanes) fq = (int)(a.fent[fb + lane * fl].off[0] >> 14);
        }
        if (a.n_probes > 0) {
            const const_i32_ptr pt = (const_i32_ptr)a.ptile + 3 * tile;
            const int pb = pt[0];
            pl = pt[1];
            const int lanes = pt[2];
#pragma unroll
            for (int e = 0; e < kProbePerLane; ++e) {
                if (e < pl && lane < lanes) {
                    const ProbeEntry pe = a.pent[pb + lane * pl + e];
                    if (pe.probe >= 0) {
                        poff[e] = pe.lds_off;
                        pwt[e] = pe.weight;
                        pvalid |= 1u << e;
                        my_probe = pe.probe;
                    }
                }
            }
        }
        // ordinates k0 .. k0 + kSlots - 2 in flight before the first barrier
#pragma unroll
        for (int d = 0; d < R::kSlots - 1; ++d)
            if (k0 + d < k1)
                ring_issue<T, TY, W, MODE, XH>(a, k0 + d, yw, lo, pitchb, planeb, lds.ring + d * R::kSlotBytes);
        __syncthreads();
        int slot = 0;
        for (int k = k0; k < k1; ++k) {
            // ordinate k's copies are complete when at most the later
            // ordinates' copies are still outstanding
            const int ahead = min(R::kSlots - 2, k1 - 1 - k);
            if (ahead >= 3) wait_vmcnt<R::wait_ahead(3)>();
            else if (ahead == 2) wait_vmcnt<R::wait_ahead(2)>();
            else if (ahead == 1) wait_vmcnt<R::wait_ahead(1)>();
            else wait_vmcnt<0>();
            if (ORDER == 3) {
                loader_edges<T, TY, W, MODE, XH>(a, k, lds.ring + slot * R::kSlotBytes);
                // the edge values are in LDS before the compute waves pass the barrier
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            }
            __builtin_amdgcn_s_barrier();
            // the slot of ordinate k - 1 is free now: ordinate k + kSlots - 1 goes there
            const int s_free = slot == 0 ? R::kSlots - 1 : slot - 1;
            if (k + R::kSlots - 1 < k1)
                ring_issue<T, TY, W, MODE, XH>(a, k + R::kSlots - 1, yw, lo, pitchb, planeb,
                                               lds.ring + s_free * R::kSlotBytes);
            if (pl > 0) {  // workgroup-uniform
                // w, w xi, w eta of ordinate k: scalar loads, which leave the
                // copies' wait counter alone
                const const_f64_ptr mk = (const_f64_ptr)a.pmom + 3 * k;
                const double w0 = mk[0], w1 = mk[1], w2 = mk[2];
                const char* sb = lds.ring + slot * R::kSlotBytes;
                float x[kProbePerLane];  // all reads in flight together (padding reads cell 0)
#pragma unroll
                for (int e = 0; e < kProbePerLane; ++e)
                    x[e] = sizeof(T) == 4 ? *reinterpret_cast<const float*>(sb + poff[e])
                                          : bf16_widen(*reinterpret_cast<const uint16_t*>(sb + poff[e]));
                double v = 0.0;
#pragma unroll
                for (int e = 0; e < kProbePerLane; ++e)
                    if (pvalid >> e & 1u) v = fma(pwt[e], (double)x[e], v);
                pm0 = fma(w0, v, pm0);
                pm1 = fma(w1, v, pm1);
                pm2 = fma(w2, v, pm2);
            }
            if (fl > 0 && lane < flanes) {  // fl: workgroup-uniform
                const char* sb = lds.ring + slot * R::kSlotBytes;
                if (fl > face_regs(ORDER)) {
                    face_fluxes_lds<ORDER, T>(a, k, sb, ftab + lane * fl, fl, fout, fin);
                } else {
                    static_assert(kFaceRegs == 3, "one case per register count");
                    switch (fl) {
                    case 1: face_fluxes_regs<ORDER, T, 1>(a, k, sb, fr, fout, fin); break;
                    case 2: face_fluxes_regs<ORDER, T, 2>(a, k, sb, fr, fout, fin); break;
                    default: face_fluxes_regs<ORDER, T, 3>(a, k, sb, fr, fout, fin); break;
                    }
                }
            }
            slot = slot == R::kSlots - 1 ? 0 : slot + 1;
        }
        for (int q = 0; q < a.n_rects; ++q) {  // per rectangle, the wave's sums in lane order
            const double vo = wave_sum(fq == q ? fout : 0.0);
            const double vi = wave_sum(fq == q ? fin : 0.0);
            if (lane == 0) {
                lds.face_red[q] = vo;
                lds.face_red[a.n_rects + q] = vi;
            }
        }
        if (a.n_probes > 0) {  // per probe, the wave's sum in lane order
            for (int p = 0; p < a.n_probes; ++p) {
                const bool mine = my_probe == p;
                const double v0 = wave_sum(mine ? pm0 : 0.0);
                const double v1 = wave_sum(mine ? pm1 : 0.0);
                const double v2 = wave_sum(mine ? pm2 : 0.0);
                if (lane == 0) {
                    lds.probe_red[p][0] = v0;
                    lds.probe_red[p][1] = v1;
                    lds.probe_red[p][2] = v2;
                }
            }
        }
        __syncthreads();
        return;
    }

    WaveCtx<TY> w;
    w.y0 = (tyi * W + wave) * TY;
    w.i0 = tx * kTileX + 2 * lane;          // interior column of the lane's first cell
    const int pc = a.ox + w.i0;             // its column in the padded row
    const int pcc = min(pc, a.pitch - 2);   // lanes past the last column stay inside the row
    w.lane_off = (uint32_t)pcc * (uint32_t)sizeof(T);
    w.pitchb = (uint32_t)a.pitch * (uint32_t)sizeof(T);
    w.planeb = (uint32_t)((size_t)a.plane * sizeof(T));
    w.seed = sizeof(T) == 2 ? (uint32_t)*a.counter : 0u;
    w.v0 = w.i0 < a.nx;
    w.v1 = w.i0 + 1 < a.nx;
    w.store_off = w.v1 ? w.lane_off : kDropOffset;
    w.single_off = (w.v0 && !w.v1) ? w.lane_off : kDropOffset;
    w.ragged = __any(w.v0 && !w.v1);
    {
        const uint32_t es = (uint32_t)sizeof(T);
        const bool holds_w = w.v0 && w.i0 == 0;
        const bool holds_e0 = w.v0 && w.i0 == a.nx - 1, holds_e1 = w.v1 && w.i0 + 1 == a.nx - 1;
        w.gw1 = holds_w ? (uint32_t)(a.ox - 1) * es : kDropOffset;
        w.gw2 = holds_w ? (uint32_t)(a.ox - 2) * es : kDropOffset;
        w.ge1 = (holds_e0 || holds_e1) ? (uint32_t)(a.ox + a.nx) * es : kDropOffset;
        w.ge2 = (holds_e0 || holds_e1) ? (uint32_t)(a.ox + a.nx + 1) * es : kDropOffset;
        w.ge_first = holds_e0;
        w.xb_w = holds_w;
        w.xb_e0 = holds_e0;
        w.xb_e1 = holds_e1;
        w.ghost_wave = MODE != kQoiOnly && (__any(holds_w || holds_e0 || holds_e1) || w.y0 == 0 ||
                                            (w.y0 <= a.ny - 1 && a.ny - 1 < w.y0 + TY));
    }
    const int ny = a.ny;

    // Per-cell constants of the stage; mass and absorption of the stage input
    // (group-0 workgroups only).
    {
        double qm = 0.0;
        double qa[kMaxTallies];
#pragma unroll
        for (int t = 0; t < kMaxTallies; ++t) qa[t] = 0.0;
#pragma unroll
        for (int t = 0; t < TY; ++t) {
            const int j = w.y0 + t;
            w.st[t] = make_float2(0.0f, 0.0f);
            w.bb[t] = make_float2(0.0f, 0.0f);
            if (j < ny) {
                const size_t c = (size_t)(j + kGhost) * a.pitch + pcc;
                const RegConst r0 = a.reg[a.region[c]], r1 = a.reg[a.region[c + 1]];
                const float2 ph = *reinterpret_cast<const float2*>(a.phi + c);
                w.st[t] = make_float2(r0.st, r1.st);
                w.bb[t] = make_float2(fmaf(r0.cs, ph.x, r0.cq), fmaf(r1.cs, ph.y, r1.cq));
                if (g == 0) {
                    const double p0 = w.v0 ? (double)ph.x : 0.0, p1 = w.v1 ? (double)ph.y : 0.0;
                    qm += p0 + p1;
#pragma unroll
                    for (int tt = 0; tt < kMaxTallies; ++tt) {
                        if (tt == r0.tally) qa[tt] += r0.sa * p0;
                        if (tt == r1.tally) qa[tt] += r1.sa * p1;
                    }
                }
            }
        }
        const double v0 = wave_sum(qm);
        if (lane == 0) red[wave][0] = v0;
#pragma unroll
        for (int tt = 0; tt < kMaxTallies; ++tt) {
            if (tt < a.n_tallies) {
                const double v = wave_sum(qa[tt]);
                if (lane == 0) red[wave][1 + tt] = v;
            }
        }
    }

#pragma unroll
    for (int t = 0; t < TY; ++t) w.phacc[t] = make_float2(0.0f, 0.0f);

    {
        __syncthreads();  // set-up done; the loader's first copies are in flight
        int slot = 0;
        for (int k = k0; k < k1; ++k) {
            __syncthreads();  // ordinate k's rows are in slot `slot`
            const char* sb = lds.ring + slot * R::kSlotBytes;
            float2 win[TY + 4], oldv[TY];
            float4 halo[TY + XH];  // x-halo of window rows 2 - XH/2 .. TY + 1 + XH/2
#pragma unroll
            for (int r = 0; r < TY + 4; ++r) win[r] = ring_read<T>(sb + (wave * TY + r) * R::kRowBytes, lane);
#pragma unroll
            for (int t = 0; t < TY + XH; ++t)
                halo[t] = halo_read<T>(sb + R::kHaloOffset + (wave * TY + t) * R::kHaloRowBytes);
#pragma unroll
            for (int t = 0; t < TY; ++t)
                oldv[t] = MODE == kAverage ? ring_read<T>(sb + R::kOldOffset + (wave * TY + t) * R::kRowBytes, lane)
                                           : make_float2(0.0f, 0.0f);
            const float* edge = ORDER == 3 ? reinterpret_cast<const float*>(sb + R::kEdgeOffset) + wave * TY : nullptr;
            process_ordinate<ORDER, MODE, T, TY, W>(a, k, w, win, halo, oldv, edge);
            slot = slot == R::kSlots - 1 ? 0 : slot + 1;
        }
        if (MODE != kQoiOnly) {
            char* pphi = reinterpret_cast<char*>(a.phi_part + (size_t)g * (size_t)a.plane);
#pragma unroll
            for (int t = 0; t < TY; ++t) {
                const int j = w.y0 + t;
                if (j < ny) {
                    const size_t off = ((size_t)(j + kGhost) * a.pitch + pcc) * sizeof(float);
                    put_pair<float>(pphi, off, w.phacc[t], w.v0, w.v1);
                }
            }
        }
    }

    // Workgroup reduction of the QoI partial sums, fixed order.
    __syncthreads();
    if (tid < a.nq) {
        double tot;
        if (tid >= a.qprobe) {  // a probe moment, from the loader wave
            tot = lds.probe_red[(tid - a.qprobe) / 3][(tid - a.qprobe) % 3];
        } else if (tid > a.n_tallies) {  // a face current, from the loader wave
            tot = lds.face_red[tid - 1 - a.n_tallies];
        } else {
            tot = red[0][tid];
#pragma unroll
            for (int ww = 1; ww < W; ++ww) tot += red[ww][tid];
        }
        a.qpart[(size_t)tid * a.n_wg + logical] = tot;
    }
}

// ---------------------------------------------------------------- stage kernels
// Workgroup: W compute waves + 1 loader wave.
template <int ORDER, int MODE, typename T, int TY, int W>
__global__ void __launch_bounds__(kWave * (W + 1)) sn_stage_kernel(const StageArgs a) {
    extern __shared__ FaceEntry ftab[];  // the tile's face table (a.face_lds bytes)
    __shared__ StageLds<T, TY, W, MODE, kExtraHalo<ORDER>> lds;
    // The averaging stage runs its logical workgroups in reverse: it reads
    // psi^(1), which the update stage just wrote in forward order, so it
    // starts on the part most likely still held by the 256 MB Infinity Cache,
    // and it leaves psi^(n+1)'s first groups, which the next update stage
    // reads first, written last (700^2 x 256 lattice, FP32: 0.609 -> 0.601
    // ms per Heun step; 1300^2 x 512 cavity: 3.73 -> 3.69 ms).
    const int l = xcd_contiguous(blockIdx.x, gridDim.x);
    stage_tile<ORDER, MODE, T, TY, W>(*(SArgsPtr)&a, MODE == kAverage ? (int)gridDim.x - 1 - l : l, ftab, lds);
}

// The selected instance j holding item (first[j] <= item < first[j + 1]):
// returns its argument index sel[j] and its first item first[j]. Wave 0 tests
// 64 candidates per round, loading first[] and sel[] together with
// independent vector loads and taking the hit from a ballot (a binary search
// would chain dependent scalar loads at the start of every workgroup), and
// passes the pair to the other waves through LDS. The first barrier orders
// every LDS use of the previous item (the pair included) before this one's.
// Called by every thread of the workgroup.
struct InstanceRef {
    int sel, first;
};
__device__ __forceinline__ InstanceRef find_instance(const int32_t* first, const int32_t* sel, int n, int item,
                                                     int* slot) {
    __syncthreads();
    if (threadIdx.x < kWave) {
        const int lane = threadIdx.x;
        for (int base = 0; base < n; base += kWave) {  // wave-uniform
            const int c = base + lane;
            int f0 = 0, f1 = 0, sl = 0;
            if (c < n) {
                f0 = first[c];
                f1 = first[c + 1];
                sl = sel[c];
            }
            const bool hit = c < n && f0 <= item && item < f1;
            if (__ballot(hit)) {
                if (hit) {  // exactly one lane: the ranges are disjoint
                    slot[0] = sl;
                    slot[1] = f0;
                }
                break;
            }
        }
    }
    __syncthreads();
    return InstanceRef{__builtin_amdgcn_readfirstlane(slot[0]), __builtin_amdgcn_readfirstlane(slot[1])};
}

// One stage of many instances in one persistent launch: the grid strides over
// the concatenated workgroup lists of the selected instances.
template <int ORDER, int MODE, typename T, int TY, int W>
__global__ void __launch_bounds__(kWave * (W + 1)) sn_stage_batch_kernel(const BatchLaunch L) {
    extern __shared__ FaceEntry ftab[];  // the largest face table of the launch's instances
    __shared__ StageLds<T, TY, W, MODE, kExtraHalo<ORDER>> lds;
    __shared__ int inst[2];
    const int pos = xcd_contiguous(blockIdx.x, gridDim.x);
    for (int base = 0; base < L.total; base += gridDim.x) {
        const int item = base + pos;
        if (item >= L.total) break;  // workgroup-uniform; later rounds are past the end too
        const InstanceRef r = find_instance(L.first, L.sel, L.n_sel, item, inst);
        stage_tile<ORDER, MODE, T, TY, W>(*(SArgsPtr)(L.args + r.sel), item - r.first, ftab, lds);
    }
}

template <int ORDER, int MODE, typename T, int TY>
static void launch_w(int waves, const StageArgs& a, hipStream_t s) {
    const size_t lds = (size_t)a.face_lds;
    if (waves == 4)
        hipLaunchKernelGGL((sn_stage_kernel<ORDER, MODE, T, TY, 4>), dim3(a.n_wg), dim3(kWave * 5), lds, s, a);
    else
        hipLaunchKernelGGL((sn_stage_kernel<ORDER, MODE, T, TY, 8>), dim3(a.n_wg), dim3(kWave * 9), lds, s, a);
}

template <int ORDER, typename T>
static hipError_t launch_stage_tu(int mode, int rows, int waves, const StageArgs& a, hipStream_t s) {
    if (waves != 4 && waves != 8) return hipErrorInvalidValue;
    if (rows == 2) {
        if (mode == kUpdate) launch_w<ORDER, kUpdate, T, 2>(waves, a, s);
        else if (mode == kAverage) launch_w<ORDER, kAverage, T, 2>(waves, a, s);
        else launch_w<ORDER, kQoiOnly, T, 2>(waves, a, s);
    } else if (rows == 4) {
        if (mode == kUpdate) launch_w<ORDER, kUpdate, T, 4>(waves, a, s);
        else if (mode == kAverage) launch_w<ORDER, kAverage, T, 4>(waves, a, s);
        else launch_w<ORDER, kQoiOnly, T, 4>(waves, a, s);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Batched launch. wgs_per_cu == 0: one workgroup per item; > 0: a persistent
// grid of that many workgroups per compute unit strides over the L.total
// items; < 0: as many as are resident at once (occupancy of this kernel).
template <typename K>
static int batch_grid(K kernel, int threads, size_t lds, int total, int wgs_per_cu, int cus, int* cache) {
    if (wgs_per_cu == 0) return total > 0 ? total : 1;
    int per = wgs_per_cu;
    if (per < 0) {
        if (*cache <= 0) {
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, lds) != hipSuccess || nb < 1) nb = 1;
            *cache = nb;
        }
        per = *cache;
    }
    const long g = (long)per * cus;
    return (int)(g < total ? g : (total > 0 ? total : 1));
}

// Face tables take at most kFacePerLaneMax x kWave entries; the batched
// launch reserves the largest of its instances', rounded up to 4 KB steps
// (one residency figure cached per step).
constexpr int kFaceLdsStep = 4096;
constexpr int kFaceLdsSteps = kFacePerLaneMax * kWave * (int)sizeof(FaceEntry) / kFaceLdsStep;

template <int ORDER, int MODE, typename T, int TY, int W>
static void launch_batch_shape(const BatchLaunch& L, int wgs_per_cu, int cus, int face_lds, hipStream_t s) {
    static int resident[kFaceLdsSteps + 1] = {};  // per face-table size step, filled on first use
    const int step = (face_lds + kFaceLdsStep - 1) / kFaceLdsStep;
    const size_t lds = (size_t)step * kFaceLdsStep;
    auto kern = sn_stage_batch_kernel<ORDER, MODE, T, TY, W>;
    const int grid = batch_grid(kern, kWave * (W + 1), lds, L.total, wgs_per_cu, cus, &resident[step]);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWave * (W + 1)), lds, s, L);
}

template <int ORDER, int MODE, typename T, int TY>
static void launch_batch_w(int waves, const BatchLaunch& L, int wgs_per_cu, int cus, int face_lds, hipStream_t s) {
    if (waves == 4) launch_batch_shape<ORDER, MODE, T, TY, 4>(L, wgs_per_cu, cus, face_lds, s);
    else launch_batch_shape<ORDER, MODE, T, TY, 8>(L, wgs_per_cu, cus, face_lds, s);
}

template <int ORDER, typename T>
static hipError_t launch_batch_tu(int mode, int rows, int waves, const BatchLaunch& L, int wgs_per_cu, int cus,
                                  int face_lds, hipStream_t s) {
    if (waves != 4 && waves != 8) return hipErrorInvalidValue;
    if (mode != kUpdate && mode != kAverage) return hipErrorInvalidValue;
    if (face_lds < 0 || face_lds > kFaceLdsSteps * kFaceLdsStep) return hipErrorInvalidValue;
    if (rows == 2) {
        if (mode == kUpdate) launch_batch_w<ORDER, kUpdate, T, 2>(waves, L, wgs_per_cu, cus, face_lds, s);
        else launch_batch_w<ORDER, kAverage, T, 2>(waves, L, wgs_per_cu, cus, face_lds, s);
    } else if (rows == 4) {
        if (mode == kUpdate) launch_batch_w<ORDER, kUpdate, T, 4>(waves, L, wgs_per_cu, cus, face_lds, s);
        else launch_batch_w<ORDER, kAverage, T, 4>(waves, L, wgs_per_cu, cus, face_lds, s);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace snk
