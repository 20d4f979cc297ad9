// snrt_batch.cpp -- host side of the batched-solve ABI (include/snrt.h,
// sn_batch_*): many independent plans advanced together, each stage of all
// unfinished plans as one persistent launch (sn_stage_batch_kernel) followed
// by one batched finalize (sn_finalize_batch_kernel).
//
// Device tables (in the caller's workspace):
//   stage   [max_instances][2] StageArgs: Heun stage 1 / stage 2, or Euler
//                                         from buffer A / from buffer B
//   final   [max_instances][2] FinalizeArgs of the same two stages
//   run     launch records (stage sel, stage first, finalize first,
//           finalize sel) of every launch of one run
// A run of K steps is planned entirely on the host: which plans are still
// unfinished at each step is known from their step counters, so every launch
// gets its own instance list and no device-side bookkeeping is needed. Small
// plans are grouped so that a group's steps run out of the Infinity Cache.
// The launches of a run are captured into a hipGraph and replayed as long as
// the admitted set and the active pattern repeat.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "sn_host.h"

using namespace snk;
using namespace snh;

struct sn_batch {
    sn_batch_opts o{};
    char* ws = nullptr;
    size_t off_stage = 0, off_final = 0, off_run = 0, run_ints = 0;
    int launches_per_step = 0;  // stage launches per step (1 Euler, 2 Heun)
    int cus = 0;
    std::vector<sn_plan*> slot;  // nullptr = free
    std::vector<int32_t> quota;  // per slot: most steps per run (0 = none)
    uint64_t bytes_admitted = 0;
    int64_t launches = 0, graph_replays = 0;
    uint64_t epoch = 0;  // changes with every admission or retirement

    // pinned staging of the run tables, two halves used alternately; an upload
    // may reuse a half once the event recorded after its previous upload has
    // completed
    int32_t* pinned[2] = {nullptr, nullptr};
    hipEvent_t pinned_done[2] = {nullptr, nullptr};
    int pinned_next = 0;

    // the last captured run
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<int32_t> graph_key;
    uint64_t graph_epoch = ~uint64_t(0);
};

namespace {

uint64_t footprint(const sn_plan* P) { return 2 * (uint64_t)P->psi_bytes + (uint64_t)P->scratch_bytes; }

sn_status check_opts(const sn_batch_opts* o) {
    if (!o) return fail(SN_ERR_INVALID, "opts is NULL");
    if (o->max_instances < 1 || o->max_instances > 4096)
        return fail(SN_ERR_INVALID, "max_instances = %d out of range [1, 4096]", o->max_instances);
    if (o->max_steps_per_run < 1 || o->max_steps_per_run > 256)
        return fail(SN_ERR_INVALID, "max_steps_per_run = %d out of range [1, 256]", o->max_steps_per_run);
    if (o->order < 1 || o->order > 3) return fail(SN_ERR_INVALID, "order must be 1, 2 or 3");
    if (o->stepper != SN_EULER && o->stepper != SN_HEUN) return fail(SN_ERR_INVALID, "stepper must be Euler or Heun");
    if (o->psi_dtype != SN_F32 && o->psi_dtype != SN_BF16) return fail(SN_ERR_INVALID, "psi_dtype must be F32 or BF16");
    const int rows = o->rows_per_wave ? o->rows_per_wave : 2;
    const int waves = o->waves_per_group ? o->waves_per_group : 4;
    if (!supported_shape(rows, waves))
        return fail(SN_ERR_UNSUPPORTED, "launch shape rows_per_wave %d, waves %d not compiled", rows, waves);
    if (o->workgroups_per_cu < -1 || o->workgroups_per_cu > 64)
        return fail(SN_ERR_INVALID, "workgroups_per_cu = %d out of range [-1, 64]", o->workgroups_per_cu);
    if (o->direct_min_workgroups < -1)
        return fail(SN_ERR_INVALID, "direct_min_workgroups = %d (>= -1 expected)", o->direct_min_workgroups);
    return SN_OK;
}

// Workspace layout for the options. A run holds at most max_steps x stage
// launches per step x (cache groups) launch records of 4 n + 2 ints, n the
// members of the group; summed over the groups of one stage that is at most
// 6 max_instances ints.
void layout(const sn_batch_opts* o, size_t* off_stage, size_t* off_final, size_t* off_run, size_t* run_ints,
            size_t* total) {
    const size_t n = (size_t)o->max_instances;
    const int lps = o->stepper == SN_HEUN ? 2 : 1;
    size_t off = 0;
    *off_stage = off;
    off += align256(2 * n * sizeof(StageArgs));
    *off_final = off;
    off += align256(2 * n * sizeof(FinalizeArgs));
    *off_run = off;
    *run_ints = (size_t)o->max_steps_per_run * lps * (6 * n + 2);
    off += align256(*run_ints * sizeof(int32_t));
    *total = off;
}

void drop_graph(sn_batch* B) {
    if (B->graph_exec) (void)hipGraphExecDestroy(B->graph_exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->graph_exec = nullptr;
    B->graph = nullptr;
    B->graph_key.clear();
}

int grid_for(const sn_batch* B, int total, int per_cu) {
    const long cap = (long)B->cus * per_cu;
    return (int)std::max<long>(1, std::min<long>(total, cap));
}

}  // namespace

extern "C" {

sn_status sn_batch_workspace_bytes(const sn_batch_opts* opts, uint64_t* bytes) {
    if (!bytes) return fail(SN_ERR_INVALID, "bytes is NULL");
    sn_status st = check_opts(opts);
    if (st != SN_OK) return st;
    size_t a, b, c, d, total;
    layout(opts, &a, &b, &c, &d, &total);
    *bytes = total;
    return SN_OK;
}

sn_status sn_batch_create(const sn_batch_opts* opts, void* workspace, sn_batch** out) {
    if (!out) return fail(SN_ERR_INVALID, "out is NULL");
    *out = nullptr;
    sn_status st = check_opts(opts);
    if (st != SN_OK) return st;
    if (!workspace || ((uintptr_t)workspace & 255)) return fail(SN_ERR_INVALID, "workspace must be 256-byte aligned");
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
    sn_batch* B = new (std::nothrow) sn_batch();
    if (!B) return fail(SN_ERR_OOM, "batch allocation failed");
    try {
        B->slot.assign(opts->max_instances, nullptr);
        B->quota.assign(opts->max_instances, 0);
    } catch (const std::bad_alloc&) {
        delete B;
        return fail(SN_ERR_OOM, "batch allocation failed");
    }
    B->o = *opts;
    if (!B->o.rows_per_wave) B->o.rows_per_wave = 2;
    if (!B->o.waves_per_group) B->o.waves_per_group = 4;
    B->ws = (char*)workspace;
    B->cus = std::max(cus, 1);
    B->launches_per_step = opts->stepper == SN_HEUN ? 2 : 1;
    size_t total;
    layout(opts, &B->off_stage, &B->off_final, &B->off_run, &B->run_ints, &total);
    const size_t run_bytes = B->run_ints * sizeof(int32_t);
    for (int h = 0; h < 2; ++h) {
        hipError_t e = hipHostMalloc((void**)&B->pinned[h], run_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&B->pinned_done[h], hipEventDisableTiming);
        if (e != hipSuccess) {
            sn_batch_destroy(B);
            return hip_fail(e, "pinned run tables");
        }
    }
    *out = B;
    return SN_OK;
}

sn_status sn_plan_footprint(const sn_plan* P, uint64_t* bytes) {
    if (!P || !bytes) return fail(SN_ERR_INVALID, "NULL argument");
    *bytes = footprint(P);
    return SN_OK;
}

sn_status sn_batch_admit(sn_batch* B, sn_plan* P, int32_t* slot) {
    if (!B || !P || !slot) return fail(SN_ERR_INVALID, "NULL argument");
    *slot = -1;
    if (!P->bound || !P->inited) return fail(SN_ERR_STATE, "plan not bound and initialised");
    if (P->batch) return fail(SN_ERR_STATE, "plan is already admitted to a batch");
    if (P->order != B->o.order || P->stepper != B->o.stepper || P->dtype != B->o.psi_dtype)
        return fail(SN_ERR_INVALID, "plan (order %d, stepper %d, dtype %d) does not match the batch (%d, %d, %d)",
                    P->order, P->stepper, P->dtype, B->o.order, B->o.stepper, B->o.psi_dtype);
    if (P->rows != B->o.rows_per_wave || P->waves != B->o.waves_per_group)
        return fail(SN_ERR_INVALID, "plan launch shape (%d rows, %d waves) differs from the batch's (%d, %d)",
                    P->rows, P->waves, B->o.rows_per_wave, B->o.waves_per_group);
    if (P->n_wg > (1 << 24)) return fail(SN_ERR_UNSUPPORTED, "plan has too many workgroups for a batch");
    const uint64_t need = footprint(P);
    if (B->o.hbm_budget_bytes && B->bytes_admitted + need > B->o.hbm_budget_bytes)
        return fail(SN_ERR_BUSY, "admitting %llu bytes would exceed the budget (%llu of %llu in use)",
                    (unsigned long long)need, (unsigned long long)B->bytes_admitted,
                    (unsigned long long)B->o.hbm_budget_bytes);
    int s = -1;
    for (int i = 0; i < (int)B->slot.size(); ++i)
        if (!B->slot[i]) {
            s = i;
            break;
        }
    if (s < 0) return fail(SN_ERR_BUSY, "no free slot (%d admitted)", (int)B->slot.size());
    StageArgs sa[2];
    if (P->stepper == SN_HEUN) {
        sa[0] = stage_args(P, P->psi[0], nullptr, P->psi[1]);     // psi^(1) = psi^n + dt F(psi^n): A -> B
        sa[1] = stage_args(P, P->psi[1], P->psi[0], P->psi[0]);  // (psi^n + psi^(1) + dt F(psi^(1))) / 2 -> A
    } else {
        sa[0] = stage_args(P, P->psi[0], nullptr, P->psi[1]);
        sa[1] = stage_args(P, P->psi[1], nullptr, P->psi[0]);
    }
    // one finalize per stage-argument variant
    FinalizeArgs fa[2];
    fa[0] = finalize_args(P, P->stepper == SN_HEUN ? 1 : 0);
    fa[1] = finalize_args(P, P->stepper == SN_HEUN ? 2 : 0);
    HIP_TRY(hipMemcpy(B->ws + B->off_stage + (size_t)s * 2 * sizeof(StageArgs), sa, sizeof sa, hipMemcpyHostToDevice),
            "upload stage arguments");
    HIP_TRY(hipMemcpy(B->ws + B->off_final + (size_t)s * 2 * sizeof(FinalizeArgs), fa, sizeof fa, hipMemcpyHostToDevice),
            "upload finalize arguments");
    B->slot[s] = P;
    P->batch = B;
    B->bytes_admitted += need;
    B->epoch++;
    *slot = s;
    return SN_OK;
}

sn_status sn_batch_run(sn_batch* B, int32_t n_steps, void* stream) {
    if (!B) return fail(SN_ERR_INVALID, "batch is NULL");
    if (n_steps < 1 || n_steps > B->o.max_steps_per_run)
        return fail(SN_ERR_INVALID, "n_steps = %d out of range [1, %d]", n_steps, B->o.max_steps_per_run);
    hipStream_t s = (hipStream_t)stream;
    const int n_slots = (int)B->slot.size();
    const int lps = B->launches_per_step;

    // Plan the run. By default all unfinished plans form one group, so that
    // every stage of all of them is one launch that fills the GPU. With a
    // cache-group size set, plans whose two psi buffers fit it are packed
    // (slot order) into groups of at most that many bytes, so that a group's
    // K steps run back to back out of the 256 MB Infinity Cache; larger plans
    // form one group. Each group takes its steps in turn; within a group every
    // stage of every member is one launch (plus one finalize), members
    // dropping out as they finish.
    std::vector<int64_t> left(n_slots, 0);
    int face_lds = 0;  // the largest face table of the run's plans
    std::vector<std::vector<int>> groups;
    {
        std::vector<int> big;
        std::vector<int> cur;
        uint64_t cur_bytes = 0;
        const uint64_t cap = B->o.cache_group_bytes;  // 0: no cache groups
        for (int i = 0; i < n_slots; ++i) {
            if (!B->slot[i]) continue;
            left[i] = std::max<int64_t>(0, B->slot[i]->nt - B->slot[i]->step);
            left[i] = std::min<int64_t>(left[i], n_steps);
            if (B->quota[i] > 0) left[i] = std::min<int64_t>(left[i], B->quota[i]);
            if (B->quota[i] == SN_STEPS_PAUSED) left[i] = 0;
            if (left[i] == 0) continue;
            face_lds = std::max(face_lds, B->slot[i]->face_lds);
            const uint64_t f = 2 * (uint64_t)B->slot[i]->psi_bytes;
            if (cap == 0 || f > cap) {
                big.push_back(i);
                continue;
            }
            if (!cur.empty() && cur_bytes + f > cap) {
                groups.push_back(cur);
                cur.clear();
                cur_bytes = 0;
            }
            cur.push_back(i);
            cur_bytes += f;
        }
        if (!cur.empty()) groups.push_back(cur);
        if (!big.empty()) groups.push_back(big);
    }
    if (groups.empty()) return SN_OK;
    // Members with at least this many workgroups per stage (default 2 per
    // CU: with 4 per CU the serving mix ran 7% slower batched than one at a
    // time, its mid-size plans going through the shared launch) take their steps
    // as launches of their own (plain kernel arguments, no instance lookup at
    // the start of every workgroup), all steps of the run of one member back
    // to back, after the shared launches: they fill the GPU by themselves,
    // and consecutive stages of one plan reuse what the cache holds of it.
    const int64_t direct_min = B->o.direct_min_workgroups < 0
                                   ? INT64_MAX
                                   : (B->o.direct_min_workgroups > 0 ? B->o.direct_min_workgroups : 2 * (int64_t)B->cus);
    struct Rec {
        size_t off;  // ints into the run area: sel [n], first [n+1], ffirst [n+1], fsel [n]
        int32_t n, total, ftotal, mode;
    };
    std::vector<Rec> recs;
    std::vector<int32_t> host;
    std::vector<int> direct;  // slots advanced with launches of their own
    int64_t stage_launches = 0;
    try {
        for (const auto& g : groups) {
            int64_t steps = 0;
            for (int i : g) steps = std::max(steps, left[i]);
            for (int t = 0; t < steps; ++t) {
                for (int st = 0; st < lps; ++st) {
                    Rec r{host.size(), 0, 0, 0, (B->o.stepper == SN_HEUN && st == 1) ? (int32_t)kAverage : (int32_t)kUpdate};
                    std::vector<int32_t> sel, first, ffirst, fsel;
                    for (int i : g) {
                        if (left[i] <= t) continue;
                        const sn_plan* P = B->slot[i];
                        const int variant = P->stepper == SN_EULER ? ((P->cur + t) & 1) : st;
                        if (P->n_wg_l[0] >= direct_min) {
                            if (t == 0 && st == 0) direct.push_back(i);
                            stage_launches++;
                            continue;
                        }
                        // the averaging stage has a layout (groups, workgroups) of its own
                        const int layout = (P->stepper == SN_HEUN && st == 1) ? 1 : 0;
                        sel.push_back(2 * i + variant);
                        fsel.push_back(2 * i + variant);
                        first.push_back(r.total);
                        ffirst.push_back(r.ftotal);
                        r.total += P->n_wg_l[layout];
                        r.ftotal += finalize_workgroups(P, P->stepper == SN_HEUN ? 1 + st : 0);
                    }
                    r.n = (int32_t)sel.size();
                    first.push_back(r.total);
                    ffirst.push_back(r.ftotal);
                    host.insert(host.end(), sel.begin(), sel.end());
                    host.insert(host.end(), first.begin(), first.end());
                    host.insert(host.end(), ffirst.begin(), ffirst.end());
                    host.insert(host.end(), fsel.begin(), fsel.end());
                    if (r.n > 0) {
                        recs.push_back(r);
                        ++stage_launches;
                    }
                }
            }
        }
    } catch (const std::bad_alloc&) {
        return fail(SN_ERR_OOM, "host run tables");
    }
    if (host.size() > B->run_ints) return fail(SN_ERR_INVALID, "run tables exceed the workspace (internal)");

    auto issue = [&](hipStream_t q) -> sn_status {
        const int32_t* base = reinterpret_cast<const int32_t*>(B->ws + B->off_run);
        for (const Rec& r : recs) {
            const int32_t* d = base + r.off;
            BatchLaunch bl{};
            bl.args = reinterpret_cast<const StageArgs*>(B->ws + B->off_stage);
            bl.sel = d;
            bl.first = d + r.n;
            bl.n_sel = r.n;
            bl.total = r.total;
            HIP_TRY(launch_stage_batch(B->o.order, r.mode, B->o.psi_dtype, B->o.rows_per_wave, B->o.waves_per_group,
                                       bl, B->o.workgroups_per_cu, B->cus, face_lds, q),
                    "batched stage launch");
            FinalizeBatch fb{};
            fb.args = reinterpret_cast<const FinalizeArgs*>(B->ws + B->off_final);
            fb.first = d + 2 * r.n + 1;
            fb.sel = d + 3 * r.n + 2;
            fb.n_sel = r.n;
            fb.total = r.ftotal;
            HIP_TRY(launch_finalize_batch(fb, grid_for(B, fb.total, 8), q), "batched finalize launch");
        }
        return SN_OK;
    };

    // The run's tables and launch sequence are a function of host-side state
    // only; an identical run under an unchanged admitted set replays the graph.
    std::vector<int32_t> key;
    if (B->o.use_graph) {
        key.reserve(host.size() + 5 * recs.size() + 2);
        key.push_back((int32_t)recs.size());
        key.push_back(face_lds);
        for (const Rec& r : recs) {
            key.push_back((int32_t)r.off);
            key.push_back(r.n);
            key.push_back(r.total);
            key.push_back(r.ftotal);
            key.push_back(r.mode);
        }
        key.insert(key.end(), host.begin(), host.end());
    }
    const bool replay = B->o.use_graph && B->graph_exec && B->graph_epoch == B->epoch && key == B->graph_key;
    if (recs.empty()) {
        // only members with launches of their own this run
    } else if (replay) {
        HIP_TRY(hipGraphLaunch(B->graph_exec, s), "hipGraphLaunch");
        B->graph_replays++;
    } else {
        // Stage through pinned memory: the copy is asynchronous, so the half
        // is not rewritten until the event after its last upload has passed.
        // The device tables are rewritten in stream order, after every launch
        // already queued on `s` that reads them.
        const int h = B->pinned_next;
        B->pinned_next ^= 1;
        HIP_TRY(hipEventSynchronize(B->pinned_done[h]), "hipEventSynchronize");
        std::memcpy(B->pinned[h], host.data(), host.size() * sizeof(int32_t));
        HIP_TRY(hipMemcpyAsync(B->ws + B->off_run, B->pinned[h], host.size() * sizeof(int32_t), hipMemcpyHostToDevice, s),
                "upload run tables");
        HIP_TRY(hipEventRecord(B->pinned_done[h], s), "hipEventRecord");
        if (B->o.use_graph) {
            drop_graph(B);
            hipStream_t cs;
            HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
            HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            sn_status st = issue(cs);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(cs, &g);
            (void)hipStreamDestroy(cs);
            if (st != SN_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            B->graph = g;
            HIP_TRY(hipGraphInstantiate(&B->graph_exec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
            B->graph_key.swap(key);
            B->graph_epoch = B->epoch;
            HIP_TRY(hipGraphLaunch(B->graph_exec, s), "hipGraphLaunch");
        } else {
            sn_status st = issue(s);
            if (st != SN_OK) return st;
        }
    }
    // Members with launches of their own: all their steps of the run back to
    // back, in stream order after the shared launches.
    std::vector<char> is_direct(n_slots, 0);
    for (int i : direct) {
        is_direct[i] = 1;
        sn_status st = issue_steps(B->slot[i], (int)left[i], s);
        if (st != SN_OK) return st;
    }
    B->launches += stage_launches;
    for (int i = 0; i < n_slots; ++i) {
        sn_plan* P = B->slot[i];
        if (!P || is_direct[i]) continue;  // issue_steps advanced the direct members
        P->step += left[i];
        if (P->stepper == SN_EULER) P->cur ^= (int)(left[i] & 1);
    }
    return SN_OK;
}

sn_status sn_batch_set_steps(sn_batch* B, int32_t slot, int32_t steps) {
    if (!B) return fail(SN_ERR_INVALID, "batch is NULL");
    if (slot < 0 || slot >= (int)B->slot.size() || !B->slot[slot]) return fail(SN_ERR_INVALID, "slot %d is not admitted", slot);
    if (steps < SN_STEPS_PAUSED || steps > B->o.max_steps_per_run)
        return fail(SN_ERR_INVALID, "steps = %d out of range [%d, %d]", steps, SN_STEPS_PAUSED, B->o.max_steps_per_run);
    B->quota[slot] = steps;
    return SN_OK;
}

sn_status sn_batch_status(const sn_batch* B, int32_t slot, int32_t* done, int64_t* step) {
    if (!B || !done || !step) return fail(SN_ERR_INVALID, "NULL argument");
    if (slot < 0 || slot >= (int)B->slot.size() || !B->slot[slot]) return fail(SN_ERR_INVALID, "slot %d is not admitted", slot);
    const sn_plan* P = B->slot[slot];
    *step = P->step;
    *done = P->step >= P->nt ? 1 : 0;
    return SN_OK;
}

sn_status sn_batch_retire(sn_batch* B, int32_t slot) {
    if (!B) return fail(SN_ERR_INVALID, "batch is NULL");
    if (slot < 0 || slot >= (int)B->slot.size() || !B->slot[slot]) return fail(SN_ERR_INVALID, "slot %d is not admitted", slot);
    sn_plan* P = B->slot[slot];
    B->bytes_admitted -= footprint(P);
    P->batch = nullptr;
    B->slot[slot] = nullptr;
    B->quota[slot] = 0;
    B->epoch++;
    return SN_OK;
}

sn_status sn_batch_get_info(const sn_batch* B, sn_batch_info* out) {
    if (!B || !out) return fail(SN_ERR_INVALID, "NULL argument");
    std::memset(out, 0, sizeof *out);
    for (const sn_plan* P : B->slot) {
        if (!P) continue;
        out->n_admitted++;
        if (P->step < P->nt) out->n_unfinished++;
    }
    out->bytes_admitted = B->bytes_admitted;
    out->hbm_budget_bytes = B->o.hbm_budget_bytes;
    out->launches = B->launches;
    out->graph_replays = B->graph_replays;
    return SN_OK;
}

void sn_batch_destroy(sn_batch* B) {
    if (!B) return;
    for (sn_plan* P : B->slot)
        if (P) P->batch = nullptr;
    drop_graph(B);
    for (int h = 0; h < 2; ++h) {
        if (B->pinned_done[h]) {
            (void)hipEventSynchronize(B->pinned_done[h]);
            (void)hipEventDestroy(B->pinned_done[h]);
        }
        if (B->pinned[h]) (void)hipHostFree(B->pinned[h]);
    }
    delete B;
}

}  // extern "C"
