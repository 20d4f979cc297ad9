// sn_host.h -- host-side internals of libsnrt shared by the plan and batch
// translation units: the plan object, error reporting, argument builders.
// Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "sn_device.h"
#include "snrt.h"

namespace snh {

// Sets the thread's last-error text and returns s.
sn_status fail(sn_status s, const char* fmt, ...);
sn_status hip_fail(hipError_t e, const char* what);
const char* last_error();

#define HIP_TRY(expr, what)                                \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return snh::hip_fail(e_, what); \
    } while (0)

constexpr double kTwoPi = 6.283185307179586476925286766559;

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace snh

struct sn_plan {
    // statement (copied)
    int nx = 0, ny = 0, M = 0;
    double h = 0;
    std::vector<double> xi, eta, w;
    std::vector<int32_t> mx, my;
    std::vector<uint8_t> region;
    std::vector<double> sa, ss, q;
    std::vector<uint8_t> tally;
    int n_regions = 0, n_tallies = 0, n_rects = 0;
    int bc[4] = {0, 0, 0, 0};
    double inflow[4] = {0, 0, 0, 0};
    int order = 1, stepper = 0, dtype = 0;
    double cfl = 0, t_end = 0;
    int rects[snk::kMaxRects][4] = {};

    // derived
    int nt = 0;
    double dt = 0;
    int pitch = 0, ny_alloc = 0, ox = 2;
    int64_t plane = 0, origin = 0;
    // Ordinate groups per stage layout: [0] update stage (Euler, Heun stage 1,
    // QoI pass), [1] Heun's averaging stage. Buffers hold the larger of each.
    int G_l[2] = {1, 1}, Mg_l[2] = {1, 1}, n_wg_l[2] = {0, 0};
    int G = 1, n_wg = 0;  // maxima over the layouts (buffer sizes)
    int rows = 2, waves = 4;
    int ntx = 0, nty = 0, nq = 0;
    size_t elem = 4, psi_bytes = 0, scratch_bytes = 0;
    size_t off_phi = 0, off_phi_part = 0, off_ord = 0, off_reg = 0, off_region = 0, off_qpart = 0,
           off_scale = 0, off_inst = 0, off_integ = 0, off_mass0 = 0, off_flags = 0, off_qchunk = 0,
           off_qcount = 0;
    // fluence (time integral of phi per cell, FP64 [ny][nx]) and what its
    // functionals read: sigma_a in FP64 and a status word
    bool fluence = false;
    size_t off_fluence = 0, off_sa64 = 0, off_fstatus = 0;
    // space-time probes: the caller's cells, the loader waves' per-tile entry
    // tables, the moments table, the window accumulators and the step
    // counters of the probe QoI slots
    int n_probes = 0, n_windows = 0;
    std::vector<sn_probe_cell> pcell_h;
    std::vector<snk::ProbeEntry> pent_h;
    std::vector<int32_t> ptile_h;  // [ntiles][3]: first entry, entries per lane, lanes
    std::vector<double> pmom_h;    // [M][3]
    size_t off_pent = 0, off_ptile = 0, off_pmom = 0, off_pacc = 0, off_pstep = 0;
    // rectangle-boundary faces: the loader waves' per-tile entry tables
    std::vector<snk::FaceEntry> fent_h;
    std::vector<int32_t> ftile_h;  // [ntiles][3]: first entry, entries per lane, lanes
    int face_lds = 0;              // bytes of the largest table read from LDS (more than kFaceRegs per lane)
    size_t off_fent = 0, off_ftile = 0;
    double source = 0;  // (sum w) h^2 sum_cells Q
    std::vector<snk::OrdConst> ord_h;
    std::vector<snk::RegConst> reg_h;
    std::vector<uint8_t> region_h;  // [ny][pitch]
    std::vector<double> scale_h;

    // device
    char* psi[2] = {nullptr, nullptr};
    char* scratch = nullptr;
    int static_dev = -1;  // device whose library-held scratch area the plan is bound to, or -1
    bool bound = false, inited = false;
    int64_t step = 0;
    int cur = 0;  // buffer holding the current state

    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev_start, ev_stop;
    std::vector<int> ev_kind;
    int ev_used = 0;
    double kernel_ms[4] = {0, 0, 0, 0};
    int64_t kernel_count[4] = {0, 0, 0, 0};

    // membership of a batch (a plan in a batch is advanced only by it)
    const sn_batch* batch = nullptr;

    // graph replay
    int graph_steps = 0;
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t graph_stream = nullptr;

    template <typename P>
    P* sp(size_t off) const { return reinterpret_cast<P*>(scratch + off); }
};

namespace snh {

// Kernel arguments of one stage of plan P (see launch_stage_pair in
// snrt_plan.cpp for the buffer roles of each kind). A stage with psi^n
// (old != NULL) is Heun's averaging stage and takes that stage's layout.
snk::StageArgs stage_args(const sn_plan* P, const char* in, const char* old, char* out);
// Finalize arguments of a stage of P; kind 0 Euler, 1/2 Heun stages, -1 QoI
// only.
snk::FinalizeArgs finalize_args(const sn_plan* P, int kind);
// Workgroups of that finalize.
int finalize_workgroups(const sn_plan* P, int kind);
// Issue n whole steps of P on s with plain launches (no graph, no timing);
// advances P's step counter and buffer parity. Used by a batch for plans
// that fill the GPU on their own.
sn_status issue_steps(sn_plan* P, int n, hipStream_t s);
// Validate and lend buffers to P (the body of sn_plan_bind, without touching
// a static-scratch binding; P->static_dev becomes -1 on success).
sn_status bind_buffers(sn_plan* P, void* psi_a, void* psi_b, void* scratch);
// P no longer holds the library-held scratch area of device dev (snrt_static.hip).
void release_static_scratch(const sn_plan* P, int dev);

}  // namespace snh
