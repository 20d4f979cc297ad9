// sn_stage.hip -- gfx950 kernels of one explicit S_N finite-volume stage.
//
// One stage evaluates, for every ordinate k and cell (i, j) of a uniform grid
// of square cells (arXiv 2505.17284, Sec. 4.2, eq. eq_sn_2d_eqn_fv divided by
// the cell area h^2),
//
//   dt F = -(dt xi_k / h)(trace_{i+1/2} - trace_{i-1/2})
//          -(dt eta_k / h)(trace_{j+1/2} - trace_{j-1/2})
//          - dt sigma_t psi + dt sigma_s / (2 pi) phi + dt Q,
//
// with the upwind trace of eq. eq_upwind1stOrder (the upwind cell's value,
// or its minmod-limited linear reconstruction at the face for second order;
// boundary faces first order with ghost values, end of Sec. 4.2), and then the
// stage update of Sec. 4.3 (eq. eq_ODE): psi + dt F for Euler and Heun's first
// stage, (psi^n + psi^(1) + dt F(psi^(1))) / 2 for Heun's second stage. The
// scalar flux phi = sum_k w_k psi_k of the written state (Sec. 4.1) is produced
// as an epilogue, per ordinate group, so the next stage reads phi without
// re-reading psi. QoI partial sums of the stage input (mass, absorption per
// tally, outflow/inflow through rectangle boundaries, Sec. 3.1.2) are reduced
// per workgroup in FP64.
//
// Mapping: psi is [M][ny][pitch], x fastest. A wavefront owns 64 consecutive
// columns (60 output columns plus 2 halo lanes on each side; neighbours come
// through DPP wave shifts) and `TY` rows, and marches over the ordinates of
// its workgroup's group. Per-cell material data and the incoming scalar flux
// stay in registers across the ordinate loop. There is no MFMA: the stage is
// a bandwidth-bound stencil.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sn_device.h"

namespace snk {

// ---------------------------------------------------------------- storage
template <typename T>
struct Store;

template <>
struct Store<float> {
    static __device__ __forceinline__ float load(const float* p) { return *p; }
    // Stores v and returns the value as stored.
    static __device__ __forceinline__ float store(float* p, float v) {
        *p = v;
        return v;
    }
};

// bfloat16 kept as raw 16-bit patterns: widening is exact, narrowing rounds
// to nearest even (NaN stays NaN).
template <>
struct Store<uint16_t> {
    static __device__ __forceinline__ float widen(uint32_t b) { return __uint_as_float(b << 16); }
    static __device__ __forceinline__ uint32_t narrow(float v) {
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (u >> 16) | 0x40u;
        u += 0x7fffu + ((u >> 16) & 1u);
        return u >> 16;
    }
    static __device__ __forceinline__ float load(const uint16_t* p) { return widen(*p); }
    static __device__ __forceinline__ float store(uint16_t* p, float v) {
        uint32_t b = narrow(v);
        *p = (uint16_t)b;
        return widen(b);
    }
};

// ---------------------------------------------------------------- helpers
// Lane l receives x from lane l-1 (lane 0 keeps x): DPP wave_shr:1.
__device__ __forceinline__ float lane_from_left(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x),
                                                      0x138, 0xf, 0xf, false));
}
// Lane l receives x from lane l+1 (lane 63 keeps x): DPP wave_shl:1.
__device__ __forceinline__ float lane_from_right(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x),
                                                      0x130, 0xf, 0xf, false));
}

// minmod(a, b): the argument of smaller magnitude when both have the same
// strict sign, else 0. Exactly one of the two terms is non-zero, so the sum
// is exact.
__device__ __forceinline__ float minmod(float a, float b) {
    return fmaxf(fminf(a, b), 0.0f) + fminf(fmaxf(a, b), 0.0f);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
    return v;
}

// Load element `off` (32-bit element offset) of the plane starting at `base`:
// the base is wave-uniform, so the address is a scalar base plus a 32-bit
// vector offset.
template <typename T>
__device__ __forceinline__ float load_at(const T* base, uint32_t off) {
    return Store<T>::load(reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                                     (size_t)off * sizeof(T)));
}

// Face-QoI tags of one cell: bit (4 * kind + q) is set when the cell's face of
// that kind (0 W, 1 E, 2 S, 3 N) lies on the boundary of rectangle q. Each
// rectangle-boundary face is assigned to the cell inside the rectangle.
__device__ __forceinline__ uint32_t face_tags(const StageArgs& a, int i, int j, bool out_lane) {
    uint32_t tg = 0;
    if (!out_lane || j >= a.ny) return 0;
    for (int q = 0; q < a.n_rects; ++q) {
        const int i0 = a.rect[q][0], j0 = a.rect[q][1], i1 = a.rect[q][2], j1 = a.rect[q][3];
        const bool rows = j >= j0 && j < j1, cols = i >= i0 && i < i1;
        if (rows && i == i0) tg |= 1u << (0 + q);
        if (rows && i == i1 - 1) tg |= 1u << (4 + q);
        if (cols && j == j0) tg |= 1u << (8 + q);
        if (cols && j == j1 - 1) tg |= 1u << (12 + q);
    }
    return tg;
}

// Adds w |Omega.n| trace to the lane's outflow or inflow accumulator of every
// rectangle whose boundary holds one of the tagged faces. West face: Omega.n =
// -xi; east: xi; south: -eta; north: eta.
__device__ __forceinline__ void face_accumulate(uint32_t tg, float tW, float tE, float tS,
                                                          float tN, double fx, double fy, bool sx, bool sy,
                                                          int n_rects, double* facc) {
#pragma unroll 1
    while (tg) {
        const int b = __builtin_ctz(tg);
        tg &= tg - 1;
        const int kind = b >> 2, q = b & 3;
        const float tr = kind == 0 ? tW : (kind == 1 ? tE : (kind == 2 ? tS : tN));
        const bool out = kind == 0 ? !sx : (kind == 1 ? sx : (kind == 2 ? !sy : sy));
        const double wgt = kind < 2 ? fx : fy;
        double* slot = facc + (out ? q : n_rects + q) * (kWave * kWavesPerWG);
        *slot = fma(wgt, (double)tr, *slot);
    }
}

// ---------------------------------------------------------------- one ordinate
// Processes ordinate k for the wave's TY rows. SY: eta_k > 0. The window holds
// TY + 3 rows: 2 upwind halo rows and 1 downwind halo row along y.
template <int ORDER, int MODE, typename T, int TY, bool SY>
__device__ __forceinline__ void stage_ordinate(const StageArgs& a, const OrdConst& o, int k, int i,
                                               uint32_t ic, int y0, bool in_x, bool out_lane,
                                               bool ghost_wave, const float (&st)[TY],
                                               const float (&bb)[TY], float (&phacc)[TY],
                                               const uint32_t (&tags)[(TY + 1) / 2], bool any_tag,
                                               double* facc) {
    constexpr int OFF = SY ? 2 : 1;  // window row of output row 0
    const bool sx = (o.flags & 1) != 0;
    const int nx = a.nx, ny = a.ny;
    const uint32_t pitch = (uint32_t)a.pitch;
    const T* pk = static_cast<const T*>(a.psi_in) + (size_t)k * (size_t)a.plane;

    // Columns outside the grid: a constant ghost (vacuum or inflow) unless the
    // side reflects, in which case the wave reloads them below.
    float lane_c = 0.0f;
    bool lane_refl = false;
    if (i == -1 && sx) {
        if (a.bc[kW] == kReflect) lane_refl = true;
        else lane_c = a.ghost[kW];
    } else if (i == nx && !sx) {
        if (a.bc[kE] == kReflect) lane_refl = true;
        else lane_c = a.ghost[kE];
    }

    float win[TY + 3];
#pragma unroll
    for (int r = 0; r < TY + 3; ++r) {
        const int jj = y0 + r - OFF;
        float v = 0.0f;
        if (jj >= 0 && jj < ny) {
            v = load_at(pk, (uint32_t)jj * pitch + ic);
            v = in_x ? v : lane_c;
        } else if (SY && jj == -1) {  // south ghost row (incoming for eta > 0)
            if (a.bc[kS] == kReflect)
                v = load_at(static_cast<const T*>(a.psi_in) + (size_t)o.my * (size_t)a.plane, ic);
            else
                v = a.ghost[kS];
        } else if (!SY && jj == ny) {  // north ghost row (incoming for eta < 0)
            if (a.bc[kN] == kReflect)
                v = load_at(static_cast<const T*>(a.psi_in) + (size_t)o.my * (size_t)a.plane,
                            (uint32_t)(ny - 1) * pitch + ic);
            else
                v = a.ghost[kN];
        }
        win[r] = v;
    }
    if (ghost_wave && __any(lane_refl)) {  // reflective ghost column: mirror ordinate's boundary cell
        const T* pm = static_cast<const T*>(a.psi_in) + (size_t)o.mx * (size_t)a.plane;
#pragma unroll
        for (int r = 0; r < TY + 3; ++r) {
            const int jj = y0 + r - OFF;
            if (jj >= 0 && jj < ny) {
                const float g = load_at(pm, (uint32_t)jj * pitch + ic);
                win[r] = lane_refl ? g : win[r];
            }
        }
    }

    float oldv[TY];
    if (MODE == kAverage) {
        const T* po = static_cast<const T*>(a.psi_old) + (size_t)k * (size_t)a.plane;
#pragma unroll
        for (int t = 0; t < TY; ++t) {
            const int j = y0 + t;
            oldv[t] = (j < ny) ? load_at(po, (uint32_t)j * pitch + ic) : 0.0f;
        }
    }

    // Traces on the y-faces: Ry[r] is the reconstruction of window row r at its
    // downwind face (eta > 0: top face; eta < 0: bottom face).
    float Ry[TY + 2];
#pragma unroll
    for (int r = 1; r <= TY + 1; ++r) {
        const float c = win[r];
        if (ORDER == 2) {
            const float m = minmod(c - win[r - 1], win[r + 1] - c);
            const float R = SY ? fmaf(0.5f, m, c) : fmaf(-0.5f, m, c);
            const int jj = y0 + r - OFF;
            const bool first = SY ? (jj == -1 || jj == ny - 1) : (jj == ny || jj == 0);
            Ry[r] = first ? c : R;
        } else {
            Ry[r] = c;
        }
    }

    T* pout = static_cast<T*>(a.psi_out) + (size_t)k * (size_t)a.plane;  // may alias psi_old
#pragma unroll
    for (int t = 0; t < TY; ++t) {
        const int j = y0 + t;
        if (j >= ny) break;  // wave-uniform
        const float c = win[t + OFF];
        float Rx = c;
        if (ORDER == 2) {
            const float cl = lane_from_left(c);
            const float cr = lane_from_right(c);
            const float m = minmod(c - cl, cr - c);
            const float R = sx ? fmaf(0.5f, m, c) : fmaf(-0.5f, m, c);
            const bool first = sx ? (i == -1 || i == nx - 1) : (i == nx || i == 0);
            Rx = first ? c : R;
        }
        const float Rxl = lane_from_left(Rx);
        const float Rxr = lane_from_right(Rx);
        const float dRx = sx ? (Rx - Rxl) : (Rxr - Rx);
        const float dRy = Ry[t + 2] - Ry[t + 1];

        if (MODE != kQoiOnly) {
            float d = fmaf(-st[t], c, bb[t]);
            d = fmaf(-o.cx, dRx, d);
            d = fmaf(-o.cy, dRy, d);
            float v = c + d;
            if (MODE == kAverage) v = 0.5f * (oldv[t] + v);
            if (out_lane) {
                char* addr = reinterpret_cast<char*>(pout) + (size_t)((uint32_t)j * pitch + ic) * sizeof(T);
                v = Store<T>::store(reinterpret_cast<T*>(addr), v);
                phacc[t] = fmaf(o.w, v, phacc[t]);
            }
        }

        if (any_tag) {  // wave-uniform: some lane of this wave owns a rectangle-boundary face
            const uint32_t tg = (tags[t >> 1] >> ((t & 1) * 16)) & 0xffffu;
            if (tg) {
                const float tW = sx ? Rxl : Rx;  // trace on face i - 1/2
                const float tE = sx ? Rx : Rxr;  // trace on face i + 1/2
                face_accumulate(tg, tW, tE, Ry[t + 1], Ry[t + 2], o.fx, o.fy, sx, SY, a.n_rects, facc);
            }
        }
    }
}

// ---------------------------------------------------------------- stage kernel
template <int ORDER, int MODE, typename T, int TY>
__global__ void __launch_bounds__(kWave * kWavesPerWG)
sn_stage_kernel(const StageArgs a) {
    extern __shared__ double facc_all[];  // [2 n_rects][256] per-thread FP64 face accumulators
    __shared__ double red[kWavesPerWG][kMaxQ];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);  // wave-uniform: keeps row math scalar
    const int wg = blockIdx.x;
    const int g = wg % a.G;  // neighbouring workgroups share a tile: phi_in and region hit in L2
    const int tile = wg / a.G;
    const int tx = tile % a.ntx;
    const int tyi = tile / a.ntx;
    const int i = tx * kXOut - kXHalo + lane;
    const int y0 = (tyi * kWavesPerWG + wave) * TY;
    const int nx = a.nx, ny = a.ny;
    const uint32_t pitch = (uint32_t)a.pitch;
    const bool in_x = i >= 0 && i < nx;
    const uint32_t ic = (uint32_t)min(max(i, 0), nx - 1);  // in-bounds column for every lane
    const bool out_lane = in_x && lane >= kXHalo && lane < kXHalo + kXOut;
    const bool ghost_wave = tx == 0 || tx == a.ntx - 1;
    double* facc = facc_all + tid;
    for (int s = 0; s < 2 * a.n_rects; ++s) facc[s * kWave * kWavesPerWG] = 0.0;

    // Per-cell constants of the stage: dt sigma_t and dt (sigma_s/(2 pi) phi + Q);
    // mass and absorption of the stage input (group-0 workgroups only).
    float st[TY], bb[TY];
    {
        double qm = 0.0;
        double qa[kMaxTallies];
#pragma unroll
        for (int t = 0; t < kMaxTallies; ++t) qa[t] = 0.0;
#pragma unroll
        for (int t = 0; t < TY; ++t) {
            const int j = y0 + t;
            st[t] = 0.0f;
            bb[t] = 0.0f;
            if (in_x && j < ny) {
                const uint32_t c = (uint32_t)j * pitch + ic;
                const RegConst rc = a.reg[a.region[c]];
                float ph = 0.0f;
                for (int p = 0; p < a.G; ++p) ph += load_at(a.phi_in + (size_t)p * (size_t)a.plane, c);
                st[t] = rc.st;
                bb[t] = fmaf(rc.cs, ph, rc.cq);
                if (g == 0 && out_lane) {
                    qm += (double)ph;
#pragma unroll
                    for (int tt = 0; tt < kMaxTallies; ++tt)
                        if (tt == rc.tally) qa[tt] += rc.sa * (double)ph;
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

    uint32_t tags[(TY + 1) / 2];
    uint32_t my_tags = 0;
#pragma unroll
    for (int t = 0; t < (TY + 1) / 2; ++t) {
        const uint32_t lo = face_tags(a, i, y0 + 2 * t, out_lane);
        const uint32_t hi = (2 * t + 1 < TY) ? face_tags(a, i, y0 + 2 * t + 1, out_lane) : 0u;
        tags[t] = lo | (hi << 16);
        my_tags |= tags[t];
    }
    const bool any_tag = __any(my_tags != 0);

    float phacc[TY];
#pragma unroll
    for (int t = 0; t < TY; ++t) phacc[t] = 0.0f;

    if (y0 < ny) {
        const int k0 = g * a.Mg;
        const int k1 = min(k0 + a.Mg, a.M);
        for (int k = k0; k < k1; ++k) {
            const OrdConst o = a.ord[k];
            if (o.flags & 2)
                stage_ordinate<ORDER, MODE, T, TY, true>(a, o, k, i, ic, y0, in_x, out_lane, ghost_wave, st, bb,
                                                         phacc, tags, any_tag, facc);
            else
                stage_ordinate<ORDER, MODE, T, TY, false>(a, o, k, i, ic, y0, in_x, out_lane, ghost_wave, st, bb,
                                                          phacc, tags, any_tag, facc);
        }
        if (MODE != kQoiOnly) {
            float* pphi = a.phi_out + (size_t)g * (size_t)a.plane;
#pragma unroll
            for (int t = 0; t < TY; ++t) {
                const int j = y0 + t;
                if (out_lane && j < ny) pphi[(uint32_t)j * pitch + ic] = phacc[t];
            }
        }
    }

    // Workgroup reduction of the QoI partial sums, fixed order.
    const int nt = a.n_tallies, nr = a.n_rects;
    for (int s = 0; s < 2 * nr; ++s) {
        const double v = wave_sum(facc[s * kWave * kWavesPerWG]);
        if (lane == 0) red[wave][1 + nt + s] = v;
    }
    __syncthreads();
    if (tid < a.nq) {
        double tot = red[0][tid];
#pragma unroll
        for (int w = 1; w < kWavesPerWG; ++w) tot += red[w][tid];
        a.qpart[(size_t)tid * a.n_wg + wg] = tot;
    }
}

// ---------------------------------------------------------------- finalize
// One workgroup per QoI slot: sums the per-workgroup partials in a fixed
// order (deterministic), scales, and accumulates the time integral.
__global__ void __launch_bounds__(256) sn_qoi_finalize_kernel(const FinalizeArgs a) {
    const int s = blockIdx.x;
    double acc = 0.0;
    for (int w = threadIdx.x; w < a.n_wg; w += 256) acc += a.qpart[(int64_t)s * a.n_wg + w];
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int m = 128; m >= 1; m >>= 1) {
        if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double tot = red[0] * a.scale[s];
        a.inst[s] = tot;
        a.integ[s] += a.coef * tot;
        if (!isfinite(tot)) a.flags[0] = 1;
    }
}

// ---------------------------------------------------------------- phi of a given state
template <typename T>
__global__ void __launch_bounds__(256) sn_phi_init_kernel(const PhiInitArgs a) {
    const int64_t cells = (int64_t)a.ny * a.pitch;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    if (c >= cells) return;
    const int i = (int)(c % a.pitch);
    if (i >= a.nx) return;
    const T* psi = static_cast<const T*>(a.psi);
    const int k0 = g * a.Mg, k1 = min(k0 + a.Mg, a.M);
    float acc = 0.0f;
    for (int k = k0; k < k1; ++k) acc = fmaf(a.ord[k].w, Store<T>::load(psi + (int64_t)k * a.plane + c), acc);
    a.phi[(int64_t)g * a.plane + c] = acc;
}

// ---------------------------------------------------------------- launchers
template <int ORDER, int MODE, typename T>
static hipError_t launch_rows(int rows, const StageArgs& a, hipStream_t s) {
    dim3 grid(a.n_wg), block(kWave * kWavesPerWG);
    const size_t lds = (size_t)2 * a.n_rects * kWave * kWavesPerWG * sizeof(double);
    switch (rows) {
    case 4:
        hipLaunchKernelGGL((sn_stage_kernel<ORDER, MODE, T, 4>), grid, block, lds, s, a);
        break;
    case 8:
        hipLaunchKernelGGL((sn_stage_kernel<ORDER, MODE, T, 8>), grid, block, lds, s, a);
        break;
    case 16:
        hipLaunchKernelGGL((sn_stage_kernel<ORDER, MODE, T, 16>), grid, block, lds, s, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool supported_rows_per_wave(int rows) { return rows == 4 || rows == 8 || rows == 16; }

template <int ORDER, typename T>
static hipError_t launch_mode(int mode, int rows, const StageArgs& a, hipStream_t s) {
    switch (mode) {
    case kUpdate: return launch_rows<ORDER, kUpdate, T>(rows, a, s);
    case kAverage: return launch_rows<ORDER, kAverage, T>(rows, a, s);
    case kQoiOnly: return launch_rows<ORDER, kQoiOnly, T>(rows, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stage(int order, int mode, int dtype, int rows, const StageArgs& a, hipStream_t s) {
    if (order == 1)
        return dtype == 0 ? launch_mode<1, float>(mode, rows, a, s) : launch_mode<1, uint16_t>(mode, rows, a, s);
    if (order == 2)
        return dtype == 0 ? launch_mode<2, float>(mode, rows, a, s) : launch_mode<2, uint16_t>(mode, rows, a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(sn_qoi_finalize_kernel, dim3(a.nq), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_phi_init(int dtype, const PhiInitArgs& a, hipStream_t s) {
    const int64_t cells = (int64_t)a.ny * a.pitch;
    dim3 grid((unsigned)((cells + 255) / 256), a.G), block(256);
    if (dtype == 0)
        hipLaunchKernelGGL(sn_phi_init_kernel<float>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(sn_phi_init_kernel<uint16_t>, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace snk
