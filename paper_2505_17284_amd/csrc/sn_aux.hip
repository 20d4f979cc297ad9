// sn_aux.hip -- the small kernels around the stage: QoI/phi finalize, the
// ghost-frame fill of a freshly set state, phi of a given state, and the
// launch dispatch over (order, storage type).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sn_device.h"
#include "sn_stage_impl.h"

namespace snk {

template <typename T>
__device__ __forceinline__ float ld(const T* p);
template <>
__device__ __forceinline__ float ld<float>(const float* p) { return *p; }
template <>
__device__ __forceinline__ float ld<uint16_t>(const uint16_t* p) { return bf16_widen(*p); }
template <typename T>
__device__ __forceinline__ void st(T* p, float v);
template <>
__device__ __forceinline__ void st<float>(float* p, float v) { *p = v; }
template <>
__device__ __forceinline__ void st<uint16_t>(uint16_t* p, float v) { *p = (uint16_t)bf16_narrow(v); }

// ---------------------------------------------------------------- ghost frame
// Sets the ghost frame of every ordinate from the interior of the same state
// (the rule the stage kernels maintain): an ordinate entering through a side
// gets the side's ghost value in both layers (inflow value, 0 for vacuum, or
// the mirror ordinate's boundary cell for a reflective side); an ordinate
// leaving through a side gets a copy of its boundary cell in the first layer.
// This is ordinate k's frame along row/column idx; it reads only interior
// cells, so every (k, idx) can run concurrently. Used when a state is set
// from outside; the stage kernels maintain the frame of what they write.
template <typename T>
__device__ __forceinline__ void ghost_update(const GhostArgs& a, int k, int idx) {
    const OrdConst o = a.ord[k];
    const bool sx = (o.flags & 1) != 0, sy = (o.flags & 2) != 0;
    T* psi = static_cast<T*>(a.psi);
    T* pk = psi + (int64_t)k * a.plane;
    const T* pmx = psi + (int64_t)o.mx * a.plane;
    const T* pmy = psi + (int64_t)o.my * a.plane;
    const int64_t P = a.pitch;
    const int nx = a.nx, ny = a.ny, ox = a.ox;
    // with all_dirs (order 3) the side's ghost value also goes to the
    // ordinates leaving through it
    const bool all = a.all_dirs != 0;
    if (idx < ny) {
        const int64_t row = (int64_t)(idx + kGhost) * P;
        if (sx || all) {  // enters through W
            const float g = a.bc[kW] == kReflect ? ld(pmx + row + ox) : a.ghost[kW];
            st(pk + row + ox - 1, g);
            st(pk + row + ox - 2, g);
        } else {
            st(pk + row + ox - 1, ld(pk + row + ox));
        }
        if (!sx || all) {  // enters through E
            const float g = a.bc[kE] == kReflect ? ld(pmx + row + ox + nx - 1) : a.ghost[kE];
            st(pk + row + ox + nx, g);
            st(pk + row + ox + nx + 1, g);
        } else {
            st(pk + row + ox + nx, ld(pk + row + ox + nx - 1));
        }
    }
    if (idx < nx) {
        const int64_t col = idx + ox;
        if (sy || all) {  // enters through S
            const float g = a.bc[kS] == kReflect ? ld(pmy + kGhost * P + col) : a.ghost[kS];
            st(pk + 1 * P + col, g);
            st(pk + 0 * P + col, g);
        } else {
            st(pk + 1 * P + col, ld(pk + kGhost * P + col));
        }
        if (!sy || all) {  // enters through N
            const float g = a.bc[kN] == kReflect ? ld(pmy + (int64_t)(ny - 1 + kGhost) * P + col) : a.ghost[kN];
            st(pk + (int64_t)(ny + kGhost) * P + col, g);
            st(pk + (int64_t)(ny + kGhost + 1) * P + col, g);
        } else {
            st(pk + (int64_t)(ny + kGhost) * P + col, ld(pk + (int64_t)(ny - 1 + kGhost) * P + col));
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) sn_ghost_fill_kernel(const GhostArgs a) {
    ghost_update<T>(a, blockIdx.y, blockIdx.x * 256 + threadIdx.x);
}

// ---------------------------------------------------------------- finalize
// Workgroups [0, nq q_split): QoI slot s = blk / q_split, chunk blk % q_split
// of its per-workgroup partials (kQoiChunk of them, 8 per thread, all loads
// in flight at once), summed in a fixed order; with more than one chunk, the
// chunk that finishes last (a device-scope counter per slot) adds the chunk
// sums in chunk order. Either way the slot's total is scaled and accumulated
// into the time integral by one thread. The order of every sum is fixed, so
// the result does not depend on which chunk finishes last.
// Workgroups [nq q_split, + n_phi_wg): phi = sum over groups of the stage's
// partial scalar fluxes, in group order, for every interior cell (4 padded
// columns per thread, ny * pitch / 4 threads), first adding the replaced phi
// (the stage input's) to the fluence when that is kept. The QoI slots of the
// space-time probes also accumulate into the window of the current step.
using FArgs = const __attribute__((address_space(4))) FinalizeArgs&;
using FArgsPtr = const __attribute__((address_space(4))) FinalizeArgs*;

__device__ double block_sum(double v, double* red) {
    __syncthreads();  // red may still be read by the previous reduction
    red[threadIdx.x] = v;
    __syncthreads();
    for (int m = 128; m >= 1; m >>= 1) {
        if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
        __syncthreads();
    }
    return red[0];
}

// The total of QoI slot s: scaled, stored, integrated in time.
__device__ __forceinline__ void finish_slot(FArgs a, int s, double sum) {
    const double tot = sum * a.scale[s];
    a.inst[s] = tot;
    a.integ[s] += a.coef * tot;
    if (!isfinite(tot)) a.flags[0] = 1;
    // one finalize per stage; the next stage reads it. The QoI-only pass
    // (no phi partials) is no stage and leaves the count alone, so that
    // reading QoIs mid-run does not change later rounding bits.
    if (s == 0 && a.n_phi_wg > 0) a.counter[0] += 1;
    if (a.n_probes > 0 && s >= a.qprobe) {
        // a probe moment: also into the window of the step (this slot's
        // finishing thread owns the slot's step counter)
        const int q = s - a.qprobe;
        const int32_t step = a.pstep[q];
        const int64_t w = (int64_t)step * a.n_windows / a.nt;
        if (w < a.n_windows) a.pacc[(w * a.n_probes + q / 3) * 3 + q % 3] += a.pcoef * tot;
        if (a.last_stage) a.pstep[q] = step + 1;
    }
}

__device__ __forceinline__ void finalize_block(FArgs a, int blk) {
    const int nqb = a.nq * a.q_split;
    if (blk >= nqb) {
        // four consecutive padded columns per thread (16-byte aligned: the
        // pitch is a multiple of 16 elements); only interior cells are written
        const int per_row = a.pitch / 4;
        const int64_t u = (int64_t)(blk - nqb) * 256 + threadIdx.x;
        if (u >= (int64_t)a.ny * per_row) return;
        const int j = (int)(u / per_row), c4 = (int)(u - (int64_t)j * per_row);
        const int64_t off = (int64_t)(j + kGhost) * a.pitch + 4 * c4;
        float4 part[16];
        const int G = a.G;
#pragma unroll
        for (int g = 0; g < 16; ++g)
            if (g < G) part[g] = *reinterpret_cast<const float4*>(a.phi_part + (int64_t)g * a.plane + off);
        float4 acc = part[0];
#pragma unroll
        for (int g = 1; g < 16; ++g) {
            if (g < G) {
                acc.x += part[g].x;
                acc.y += part[g].y;
                acc.z += part[g].z;
                acc.w += part[g].w;
            }
        }
        for (int g = 16; g < G; ++g) {
            const float4 p = *reinterpret_cast<const float4*>(a.phi_part + (int64_t)g * a.plane + off);
            acc.x += p.x;
            acc.y += p.y;
            acc.z += p.z;
            acc.w += p.w;
        }
        const int i0 = 4 * c4 - a.ox;  // interior column of the first of the four
        if (a.fluence != nullptr) {
            // phi still holds the stage input's scalar flux: add its share of
            // the time integral before it is replaced
            const float4 o = *reinterpret_cast<const float4*>(a.phi + off);
            const float ov[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (i0 + e >= 0 && i0 + e < a.nx) a.fluence[(int64_t)j * a.nx + i0 + e] += a.coef * (double)ov[e];
        }
        if (i0 >= 0 && i0 + 3 < a.nx) {
            *reinterpret_cast<float4*>(a.phi + off) = acc;
        } else {
            const float v[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (i0 + e >= 0 && i0 + e < a.nx) a.phi[off + e] = v[e];
        }
        return;
    }
    const int s = blk / a.q_split;
    const int chunk = blk - s * a.q_split;
    const int lo = chunk * kQoiChunk;
    const int hi = min(lo + kQoiChunk, a.n_wg);
    // eight independent loads per thread, combined in a fixed order
    const double* qp = a.qpart + (int64_t)s * a.n_wg;
    double acc8[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int w = lo + (int)threadIdx.x + u * 256;
        acc8[u] = w < hi ? qp[w] : 0.0;
    }
    double acc = ((acc8[0] + acc8[1]) + (acc8[2] + acc8[3])) + ((acc8[4] + acc8[5]) + (acc8[6] + acc8[7]));
    __shared__ double red[256];
    __syncthreads();  // a previous block of a batched launch may still read red
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int m = 128; m >= 1; m >>= 1) {
        if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double csum = red[0];
    if (a.q_split == 1) {
        finish_slot(a, s, csum);
        return;
    }
    // Publish the chunk sum, then count it; the chunk that brings the count to
    // q_split sees every chunk sum (release before the count, acquire after)
    // and resets the count for the next launch.
    double* cs = a.qchunk + (int64_t)s * a.q_split;
    __hip_atomic_store(cs + chunk, csum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int done = __hip_atomic_fetch_add(a.qcount + s, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (done != a.q_split - 1) return;
    double tot = 0.0;
    for (int c = 0; c < a.q_split; ++c) tot += __hip_atomic_load(cs + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(a.qcount + s, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    finish_slot(a, s, tot);
}

__global__ void __launch_bounds__(256) sn_qoi_finalize_kernel(const FinalizeArgs a) {
    finalize_block(*(FArgsPtr)&a, blockIdx.x);
}

// Finalize of many instances in one persistent launch.
__global__ void __launch_bounds__(256) sn_finalize_batch_kernel(const FinalizeBatch L) {
    __shared__ int inst[2];
    for (int item = blockIdx.x; item < L.total; item += gridDim.x) {
        const InstanceRef r = find_instance(L.first, L.sel, L.n_sel, item, inst);
        finalize_block(*(FArgsPtr)(L.args + r.sel), item - r.first);
    }
}

// ---------------------------------------------------------------- phi of a given state
template <typename T>
__global__ void __launch_bounds__(256) sn_phi_init_kernel(const PhiInitArgs a) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (int64_t)a.nx * a.ny) return;
    const int64_t j = c / a.nx, i = c - j * a.nx;
    const int64_t off = (j + kGhost) * a.pitch + i + a.ox;
    const T* psi = static_cast<const T*>(a.psi);
    float acc = 0.0f;
    for (int k = 0; k < a.M; ++k) acc = fmaf(a.ord[k].w, ld(psi + (int64_t)k * a.plane + off), acc);
    a.phi[off] = acc;
}

// ---------------------------------------------------------------- fluence functionals
// One workgroup, FP64 throughout, fixed reduction order. The value of a piece
// is the mean of sigma_a * fluence over its two cells; every set's weighted
// sum is a strided partial per thread followed by a tree over the workgroup.
__device__ __forceinline__ double fl_cell(const FluenceArgs& a, int32_t c) {
    const int32_t j = c / a.nx, i = c - j * a.nx;
    return a.sa[a.region[a.origin + (int64_t)j * a.pitch + i]] * a.fluence[c];
}

__global__ void __launch_bounds__(256) sn_fluence_functionals_kernel(const FluenceArgs a) {
    __shared__ double red[256];
    __shared__ double setsum[kMaxFluenceBlocks + 1];
    __shared__ int bad;
    const int nsets = a.n_blocks + 1;
    const int64_t ncell = (int64_t)a.nx * a.ny;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int g = threadIdx.x; g <= nsets; g += 256) {
        const int32_t lo = g == 0 ? 0 : a.set_start[g - 1], hi = a.set_start[g];
        const bool ok = g == 0 ? hi == 0 : (lo <= hi && (g < nsets || hi == a.n_pieces));
        if (!ok) atomicOr(&bad, 1);
    }
    for (int p = threadIdx.x; p < a.n_pieces; p += 256) {
        const FluencePiece q = a.pieces[p];
        if (q.a < 0 || q.a >= ncell || q.b < 0 || q.b >= ncell || !isfinite(q.w)) atomicOr(&bad, 1);
    }
    __syncthreads();
    if (bad) {  // uniform: every thread leaves here
        if (threadIdx.x == 0) a.status[0] = 1;
        for (int e = threadIdx.x; e < 4 + a.n_blocks; e += 256) a.out[e] = __builtin_nan("");
        return;
    }
    for (int g = 0; g < nsets; ++g) {
        double v = 0.0;
        for (int p = a.set_start[g] + threadIdx.x; p < a.set_start[g + 1]; p += 256) {
            const FluencePiece q = a.pieces[p];
            v += q.w * (0.5 * (fl_cell(a, q.a) + fl_cell(a, q.b)));
        }
        const double tot = block_sum(v, red);
        if (threadIdx.x == 0) setsum[g] = tot;
    }
    __syncthreads();
    double A_G = 0.0, V_G = 0.0;
    for (int g = 0; g < a.n_blocks; ++g) A_G += setsum[g];
    A_G /= a.n_blocks;
    for (int g = 0; g < a.n_blocks; ++g) V_G += (A_G - setsum[g]) * (A_G - setsum[g]);
    V_G /= a.n_blocks;
    const double A_L = setsum[a.n_blocks];
    double v = 0.0;
    for (int p = a.set_start[a.n_blocks] + threadIdx.x; p < a.set_start[a.n_blocks + 1]; p += 256) {
        const FluencePiece q = a.pieces[p];
        const double d = A_L - 0.5 * (fl_cell(a, q.a) + fl_cell(a, q.b));
        v += q.w * d * d;
    }
    const double V_L = block_sum(v, red);
    if (threadIdx.x == 0) {
        a.out[0] = A_G;
        a.out[1] = V_G;
        a.out[2] = A_L;
        a.out[3] = V_L;
        a.status[0] = 0;
    }
    for (int g = threadIdx.x; g < a.n_blocks; g += 256) a.out[4 + g] = setsum[g];
}

// ---------------------------------------------------------------- launchers
bool supported_shape(int rows, int waves) {
    return (rows == 2 || rows == 4) && (waves == 4 || waves == 8);
}

hipError_t launch_stage(int order, int mode, int dtype, int rows, int waves, const StageArgs& a, hipStream_t s) {
    if (order == 1)
        return dtype == 0 ? launch_stage_o1_f32(mode, rows, waves, a, s) : launch_stage_o1_bf16(mode, rows, waves, a, s);
    if (order == 2)
        return dtype == 0 ? launch_stage_o2_f32(mode, rows, waves, a, s) : launch_stage_o2_bf16(mode, rows, waves, a, s);
    if (order == 3)
        return dtype == 0 ? launch_stage_o3_f32(mode, rows, waves, a, s) : launch_stage_o3_bf16(mode, rows, waves, a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_stage_batch(int order, int mode, int dtype, int rows, int waves, const BatchLaunch& L, int wgs_per_cu,
                              int cus, int face_lds, hipStream_t s) {
    if (order == 1)
        return dtype == 0 ? launch_batch_o1_f32(mode, rows, waves, L, wgs_per_cu, cus, face_lds, s)
                          : launch_batch_o1_bf16(mode, rows, waves, L, wgs_per_cu, cus, face_lds, s);
    if (order == 2)
        return dtype == 0 ? launch_batch_o2_f32(mode, rows, waves, L, wgs_per_cu, cus, face_lds, s)
                          : launch_batch_o2_bf16(mode, rows, waves, L, wgs_per_cu, cus, face_lds, s);
    if (order == 3)
        return dtype == 0 ? launch_batch_o3_f32(mode, rows, waves, L, wgs_per_cu, cus, face_lds, s)
                          : launch_batch_o3_bf16(mode, rows, waves, L, wgs_per_cu, cus, face_lds, s);
    return hipErrorInvalidValue;
}

hipError_t launch_finalize_batch(const FinalizeBatch& L, int grid, hipStream_t s) {
    hipLaunchKernelGGL(sn_finalize_batch_kernel, dim3(grid), dim3(256), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(sn_qoi_finalize_kernel, dim3(a.nq * a.q_split + a.n_phi_wg), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ghost_fill(int dtype, const GhostArgs& a, hipStream_t s) {
    const int n = a.nx > a.ny ? a.nx : a.ny;
    const dim3 grid((unsigned)((n + 255) / 256), (unsigned)a.M), block(256);
    if (dtype == 0)
        hipLaunchKernelGGL(sn_ghost_fill_kernel<float>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(sn_ghost_fill_kernel<uint16_t>, grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fluence_functionals(const FluenceArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(sn_fluence_functionals_kernel, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_phi_init(int dtype, const PhiInitArgs& a, hipStream_t s) {
    const int64_t cells = (int64_t)a.nx * a.ny;
    const dim3 grid((unsigned)((cells + 255) / 256)), block(256);
    if (dtype == 0)
        hipLaunchKernelGGL(sn_phi_init_kernel<float>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(sn_phi_init_kernel<uint16_t>, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace snk
