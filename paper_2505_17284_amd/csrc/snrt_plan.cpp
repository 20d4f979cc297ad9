// snrt_plan.cpp -- host side of the C ABI in include/snrt.h: validation of a
// problem statement, derived constants, device-buffer layout, and the launch
// sequence of Euler / Heun steps (arXiv 2505.17284, Sec. 4.3, eq. eq_ODE).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "sn_host.h"

using namespace snk;

namespace snh {

namespace {
thread_local std::string g_err;
}

sn_status fail(sn_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

sn_status hip_fail(hipError_t e, const char* what) {
    return fail(SN_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error() { return g_err.c_str(); }

}  // namespace snh

using namespace snh;

namespace {

sn_status validate_and_copy(const sn_problem* p, sn_plan* P) {
    if (!p) return fail(SN_ERR_INVALID, "problem is NULL");
    if (p->nx < 1 || p->ny < 1 || p->nx > (1 << 20) || p->ny > (1 << 20))
        return fail(SN_ERR_INVALID, "grid %d x %d out of range [1, 2^20]", p->nx, p->ny);
    if (!(p->h > 0) || !std::isfinite(p->h)) return fail(SN_ERR_INVALID, "cell size h must be finite and > 0");
    if (p->M < 1 || p->M > SN_MAX_ORDINATES)
        return fail(SN_ERR_INVALID, "M = %d out of range [1, %d]", p->M, SN_MAX_ORDINATES);
    if (!p->xi || !p->eta || !p->w) return fail(SN_ERR_INVALID, "quadrature arrays are NULL");
    if (!p->region || !p->sigma_a || !p->sigma_s || !p->q || !p->tally)
        return fail(SN_ERR_INVALID, "material arrays are NULL");
    if (p->n_regions < 1 || p->n_regions > SN_MAX_REGIONS)
        return fail(SN_ERR_INVALID, "n_regions = %d out of range [1, %d]", p->n_regions, SN_MAX_REGIONS);
    if (p->n_tallies < 1 || p->n_tallies > SN_MAX_TALLIES)
        return fail(SN_ERR_INVALID, "n_tallies = %d out of range [1, %d]", p->n_tallies, SN_MAX_TALLIES);
    if (p->n_rects < 0 || p->n_rects > SN_MAX_RECTS)
        return fail(SN_ERR_INVALID, "n_rects = %d out of range [0, %d]", p->n_rects, SN_MAX_RECTS);
    if (p->n_rects > 0 && !p->rects) return fail(SN_ERR_INVALID, "rects is NULL");
    if (p->order < 1 || p->order > 3) return fail(SN_ERR_INVALID, "order must be 1, 2 or 3");
    if (p->stepper != SN_EULER && p->stepper != SN_HEUN) return fail(SN_ERR_INVALID, "stepper must be Euler or Heun");
    if (p->psi_dtype != SN_F32 && p->psi_dtype != SN_BF16) return fail(SN_ERR_INVALID, "psi_dtype must be F32 or BF16");
    if (p->fluence != 0 && p->fluence != 1) return fail(SN_ERR_INVALID, "fluence must be 0 or 1");
    if (p->n_probes < 0 || p->n_probes > SN_MAX_PROBES)
        return fail(SN_ERR_INVALID, "n_probes = %d out of range [0, %d]", p->n_probes, SN_MAX_PROBES);
    if (p->n_probes > 0) {
        if (p->n_windows < 1 || p->n_windows > SN_MAX_WINDOWS)
            return fail(SN_ERR_INVALID, "n_windows = %d out of range [1, %d]", p->n_windows, SN_MAX_WINDOWS);
        if (p->n_probe_cells < 0 || p->n_probe_cells > SN_MAX_PROBE_CELLS)
            return fail(SN_ERR_INVALID, "n_probe_cells = %d out of range [0, %d]", p->n_probe_cells,
                        SN_MAX_PROBE_CELLS);
        if (p->n_probe_cells > 0 && !p->probe_cells) return fail(SN_ERR_INVALID, "probe_cells is NULL");
        for (int c = 0; c < p->n_probe_cells; ++c) {
            const sn_probe_cell& pc = p->probe_cells[c];
            if (pc.cell < 0 || (int64_t)pc.cell >= (int64_t)p->nx * p->ny)
                return fail(SN_ERR_INVALID, "probe cell %d: cell index %d out of range", c, pc.cell);
            if (pc.probe < 0 || pc.probe >= p->n_probes)
                return fail(SN_ERR_INVALID, "probe cell %d: probe %d out of range", c, pc.probe);
            if (!std::isfinite(pc.weight)) return fail(SN_ERR_INVALID, "probe cell %d: weight not finite", c);
        }
    }
    if (p->fluence && (int64_t)p->nx * p->ny > 0x7fffffff)
        return fail(SN_ERR_UNSUPPORTED, "fluence needs nx * ny < 2^31 (cell indices are 32-bit)");
    if (!(p->cfl > 0) || !std::isfinite(p->cfl)) return fail(SN_ERR_INVALID, "cfl must be finite and > 0");
    if (!(p->t_end > 0) || !std::isfinite(p->t_end)) return fail(SN_ERR_INVALID, "t_end must be finite and > 0");

    const int M = p->M;
    double sw = 0;
    for (int k = 0; k < M; ++k) {
        const double a = p->xi[k], b = p->eta[k], c = p->w[k];
        if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(c))
            return fail(SN_ERR_INVALID, "ordinate %d is not finite", k);
        if (c < 0) return fail(SN_ERR_INVALID, "weight %d is negative", k);
        if (a * a + b * b > 1.0 + 1e-12) return fail(SN_ERR_INVALID, "ordinate %d is not a unit direction", k);
        sw += c;
    }
    if (std::fabs(sw - kTwoPi) > 1e-10 * kTwoPi)
        return fail(SN_ERR_INVALID, "weights sum to %.17g, not 2 pi", sw);

    bool need_mx = p->bc[0] == SN_BC_REFLECT || p->bc[1] == SN_BC_REFLECT;
    bool need_my = p->bc[2] == SN_BC_REFLECT || p->bc[3] == SN_BC_REFLECT;
    for (int s = 0; s < 4; ++s) {
        if (p->bc[s] < SN_BC_VACUUM || p->bc[s] > SN_BC_REFLECT)
            return fail(SN_ERR_INVALID, "boundary kind %d on side %d", p->bc[s], s);
        if (!std::isfinite(p->inflow[s])) return fail(SN_ERR_INVALID, "inflow on side %d not finite", s);
    }
    P->mx.assign(M, 0);
    P->my.assign(M, 0);
    for (int pass = 0; pass < 2; ++pass) {
        const int32_t* m = pass == 0 ? p->mirror_x : p->mirror_y;
        const bool need = pass == 0 ? need_mx : need_my;
        std::vector<int32_t>& dst = pass == 0 ? P->mx : P->my;
        if (!m) {
            if (need) return fail(SN_ERR_INVALID, "reflective side needs mirror_%c", pass == 0 ? 'x' : 'y');
            for (int k = 0; k < M; ++k) dst[k] = k;
            continue;
        }
        for (int k = 0; k < M; ++k) {
            const int32_t l = m[k];
            if (l < 0 || l >= M) return fail(SN_ERR_INVALID, "mirror index %d of ordinate %d out of range", l, k);
            if (need) {
                const bool ok = pass == 0 ? (p->xi[l] == -p->xi[k] && p->eta[l] == p->eta[k])
                                          : (p->eta[l] == -p->eta[k] && p->xi[l] == p->xi[k]);
                if (!ok || p->w[l] != p->w[k])
                    return fail(SN_ERR_INVALID, "ordinate %d has no exact mirror partner along %c", k,
                                pass == 0 ? 'x' : 'y');
            }
            dst[k] = l;
        }
    }

    for (int r = 0; r < p->n_regions; ++r) {
        if (!(p->sigma_a[r] >= 0) || !(p->sigma_s[r] >= 0) || !std::isfinite(p->sigma_a[r]) ||
            !std::isfinite(p->sigma_s[r]))
            return fail(SN_ERR_INVALID, "cross-sections of region %d must be finite and >= 0", r);
        if (!std::isfinite(p->q[r])) return fail(SN_ERR_INVALID, "source of region %d not finite", r);
        if (p->tally[r] >= p->n_tallies) return fail(SN_ERR_INVALID, "tally of region %d out of range", r);
    }
    const size_t ncell = (size_t)p->nx * p->ny;
    for (size_t c = 0; c < ncell; ++c)
        if (p->region[c] >= p->n_regions)
            return fail(SN_ERR_INVALID, "region id %d of cell %zu >= n_regions", p->region[c], c);
    for (int r = 0; r < p->n_rects; ++r) {
        const int32_t* R = p->rects + 4 * r;
        if (!(R[0] >= 0 && R[0] < R[2] && R[2] <= p->nx && R[1] >= 0 && R[1] < R[3] && R[3] <= p->ny))
            return fail(SN_ERR_INVALID, "rect %d = (%d, %d, %d, %d) not a non-empty cell range", r, R[0], R[1],
                        R[2], R[3]);
        for (int e = 0; e < 4; ++e) P->rects[r][e] = R[e];
    }

    P->nx = p->nx;
    P->ny = p->ny;
    P->M = M;
    P->h = p->h;
    P->xi.assign(p->xi, p->xi + M);
    P->eta.assign(p->eta, p->eta + M);
    P->w.assign(p->w, p->w + M);
    P->region.assign(p->region, p->region + ncell);
    P->n_regions = p->n_regions;
    P->sa.assign(p->sigma_a, p->sigma_a + p->n_regions);
    P->ss.assign(p->sigma_s, p->sigma_s + p->n_regions);
    P->q.assign(p->q, p->q + p->n_regions);
    P->tally.assign(p->tally, p->tally + p->n_regions);
    P->n_tallies = p->n_tallies;
    P->n_rects = p->n_rects;
    for (int s = 0; s < 4; ++s) {
        P->bc[s] = p->bc[s];
        P->inflow[s] = p->inflow[s];
    }
    P->order = p->order;
    P->stepper = p->stepper;
    P->dtype = p->psi_dtype;
    P->fluence = p->fluence == 1;
    P->n_probes = p->n_probes;
    P->n_windows = p->n_probes > 0 ? p->n_windows : 0;
    P->pcell_h.clear();
    if (P->n_probes > 0) P->pcell_h.assign(p->probe_cells, p->probe_cells + p->n_probe_cells);
    P->cfl = p->cfl;
    P->t_end = p->t_end;
    return SN_OK;
}

void default_shape(const sn_plan* P, int* group_size, int* group_size_avg, int* rows, int* waves) {
    // Two rows per wave keep the staged windows, the per-cell constants and the
    // reconstructions within ~80 VGPRs. Four waves per workgroup by default;
    // ordinate groups as below; at least 8 ordinates per group keep the
    // per-workgroup set-up and the group's phi partial small.
    *rows = 2;
    *waves = 4;
    const int64_t cells = (int64_t)P->nx * P->ny;
    // FP32 storage, orders 1 and 2, no probes: eight waves per workgroup
    // (16-row tiles stage 1.25x instead of 1.5x the stencil rows) on grids of
    // 10^6 cells or more, and of 4 10^5 or more with 512 ordinates or more,
    // 32 ordinates per group in both stages. Timed over minmod-Heun lattice
    // and cavity classes (grid side 200 to 1300, 64 to 512 ordinates, ms per
    // step against four waves): the 1300^2 x 512 cavity 3.58 -> 3.48, the
    // 1000^2 lattice 2.6-6% faster at every ordinate count, 700^2 x 512 4%;
    // slower on smaller grids (700^2 x 256: +2%), at order 3 (1.22 vs 0.95 ms
    // on the 700^2 lattice) and with BF16 storage (+5-15%).
    if (P->dtype == SN_F32 && P->order < 3 && P->n_probes == 0 &&
        (cells >= 1000000 || (cells >= 400000 && P->M >= 512))) {
        *waves = 8;
        *group_size = std::min(P->M, 32);
        *group_size_avg = *group_size;
        return;
    }
    const int wg_rows = *waves * *rows;
    const long tiles = (long)((P->nx + kTileX - 1) / kTileX) * ((P->ny + wg_rows - 1) / wg_rows);
    if (P->dtype == SN_F32) {
        // 32 ordinates per group, halved (down to 8) while the launch would
        // hold fewer than 400 workgroups. Timed over the lattice at grid sides
        // 200 to 1000 with 64 to 512 ordinates, 32 per group is the fastest
        // or within 5% everywhere but the smallest launches (200^2 x 64: 8
        // per group, 2x faster; 200^2 x 128 and 300^2 x 64: 16), while aiming
        // at 4 K workgroups had split mid-size grids into groups of 8 (500^2 x
        // 256: 0.42 vs 0.31 ms per step). More than 32 per group is slower on
        // large M (700 x 700 with 1936 ordinates, stage 1: 1.83 ms with 32
        // per group, 2.27 ms with 242). Launches of 1,000 to 5,000 workgroups
        // at 32 per group take 16 (re-timed after the face currents left the
        // compute waves, which freed LDS for a fourth workgroup per compute
        // unit: the 700^2 lattice 1.9-6% faster at 64 to 256 ordinates,
        // 560^2 and 400^2 1.3-2%; the 700^2 x 256 benchmark lattice 0.525 ->
        // 0.515 ms per step).
        int gs = std::min(P->M, 32);
        while (gs > 8 && tiles * ((P->M + gs - 1) / gs) < 400) gs = (gs + 1) / 2;
        if (gs == 32 && P->order < 3) {  // order 3 (bound by its arithmetic) not re-timed
            const long wg = tiles * ((P->M + gs - 1) / gs);
            if (wg >= 1000 && wg < 5000) gs = 16;
        }
        *group_size = gs;
    } else {
        // BF16 storage favours larger groups: 64 ordinates per group (M / 8
        // when that is more: 242 per group on the 1936-ordinate lattice, 1.74
        // vs 1.85 ms with 32), halved (down to 8) while the launch would hold
        // fewer than 700 workgroups. Timed over the same lattice classes, 64
        // per group is the fastest or within a few percent from 500^2 up (the
        // 700^2 x 256 lattice: 0.554 vs 0.577 ms per step with 32; the 1300^2
        // x 256 Hohlraum: 1.48 vs 1.57 ms), the smaller grids want 8 to 32.
        int gs = std::max(std::min(P->M, 64), (P->M + 7) / 8);
        while (gs > 8 && tiles * ((P->M + gs - 1) / gs) < 700) gs = (gs + 1) / 2;
        *group_size = gs;
    }
    // Heun's averaging stage also streams psi^n; with FP32 storage its LDS
    // slots are twice those of the update stage, and twice the groups (half
    // the ordinates each, while that leaves at least 16) measured faster on
    // the 700 x 700 grids: 356 vs 372 us per launch with 256 ordinates, 2.61
    // vs 2.69 ms with 1936. On grids of more than 2^20 cells the finalize's
    // extra phi partials (one plane per group) cost more than that gains
    // (the 1300 x 1300 x 512 cavity: 4.16 vs 4.22 ms per step). With BF16
    // storage the halving measured slower (368 vs 330 us on the lattice), and
    // with the Venkatakrishnan limiter (order 3), whose stage is bound by its
    // arithmetic rather than by the copies in flight, too (572 vs 533 us).
    // Re-timed with the reversed averaging stage, the halving is worth little
    // any more: 1-3.5% slower than whole groups at 256 and 512 ordinates on
    // grids from 400^2 to 1000^2 (the benchmark lattice: level), 2-10% slower
    // at 64 and 128; it is kept only at 256 ordinates and more.
    const bool halve = *group_size >= 32 && P->dtype == SN_F32 && P->order < 3 && P->M >= 256 &&
                       (int64_t)P->nx * P->ny <= (1 << 20);
    *group_size_avg = halve ? (*group_size + 1) / 2 : *group_size;
}

// The stage kernels' loader wave of a tile reads the tile's probe cells from
// its LDS ring (the stencil rows of every ordinate it stages) and sums
// w_k weight psi_k, w_k xi_k weight psi_k and w_k eta_k weight psi_k, in FP64.
// Per tile: the cells grouped by probe (caller's order within a probe), dealt
// pl to a lane, a lane's cells all of one probe (the last lane of a probe
// padded), pl the smallest that fits the tile's cells into one wave.
sn_status probe_tables(sn_plan* P) {
    const int ntiles = P->ntx * P->nty;
    const int tile_rows = P->waves * P->rows;
    P->ptile_h.assign((size_t)3 * ntiles, 0);
    P->pent_h.clear();
    if (P->n_probes == 0) return SN_OK;
    const int n = (int)P->pcell_h.size();
    std::vector<int64_t> key(n);
    std::vector<int32_t> idx(n);
    for (int c = 0; c < n; ++c) {
        const sn_probe_cell& pc = P->pcell_h[c];
        const int j = pc.cell / P->nx, i = pc.cell - j * P->nx;
        const int tile = (j / tile_rows) * P->ntx + i / kTileX;
        key[c] = (int64_t)tile * P->n_probes + pc.probe;
        idx[c] = c;
    }
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return key[x] < key[y]; });
    for (int b = 0; b < n;) {
        const int tile = (int)(key[idx[b]] / P->n_probes);
        int e = b;
        while (e < n && key[idx[e]] / P->n_probes == tile) ++e;
        int cnt[kMaxProbes] = {};
        for (int c = b; c < e; ++c) cnt[P->pcell_h[idx[c]].probe]++;
        int pl = 0, lanes = 0;
        for (int cand = 1; cand <= kProbePerLane && pl == 0; ++cand) {
            int l = 0;
            for (int q = 0; q < P->n_probes; ++q) l += (cnt[q] + cand - 1) / cand;
            if (l <= kWave) {
                pl = cand;
                lanes = l;
            }
        }
        if (pl == 0)
            return fail(SN_ERR_UNSUPPORTED,
                        "%d probe cells in the tile of columns %d.. and rows %d..: at most %d per tile (%d lanes of "
                        "%d, a lane's cells of one probe)",
                        e - b, (tile % P->ntx) * kTileX, (tile / P->ntx) * tile_rows, kWave * kProbePerLane, kWave,
                        kProbePerLane);
        P->ptile_h[3 * tile] = (int32_t)P->pent_h.size();
        P->ptile_h[3 * tile + 1] = pl;
        P->ptile_h[3 * tile + 2] = lanes;
        for (int c = b; c < e;) {  // one probe's cells
            const int q = P->pcell_h[idx[c]].probe;
            int m = 0;
            for (; c < e && P->pcell_h[idx[c]].probe == q; ++c, ++m) {
                const sn_probe_cell& pc = P->pcell_h[idx[c]];
                const int j = pc.cell / P->nx, i = pc.cell - j * P->nx;
                const uint32_t off = (uint32_t)(((j % tile_rows) + kGhost) * kTileX + i % kTileX) * (uint32_t)P->elem;
                P->pent_h.push_back(ProbeEntry{off, q, pc.weight});
            }
            for (; m % pl != 0; ++m) P->pent_h.push_back(ProbeEntry{0u, -1, 0.0});
        }
        b = e;
    }
    return SN_OK;
}

// The stage kernels' loader wave sums the outflow and inflow through the
// rectangles' boundaries (Sec. 3.1.2, R11): each boundary face of a
// rectangle is assigned to the cell inside it, so to that cell's tile. Per
// tile: the faces grouped by rectangle (west, east, south, north faces, in
// cell order), dealt fl to a lane, a lane's faces all of one rectangle (the
// last lane of a rectangle padded), fl the smallest that fits the tile's
// faces into one wave. An entry holds the ring-slot offsets of the cells the
// face's trace is reconstructed from (FaceEntry); every such cell is staged
// with the tile: the line c0..c3 lies in the face's row or column within
// two cells of the tile, and at order 3 the cells across it lie in the rows
// next to an output row, whose x-halo is staged too.
sn_status face_tables(sn_plan* P) {
    const int ntiles = P->ntx * P->nty;
    const int tile_rows = P->waves * P->rows;
    const int xh = P->order == 3 ? 1 : 0;  // x-halo rows staged above and below the output rows
    const int halo0 = ring_halo_elem(tile_rows + 4, (int)P->elem);
    P->ftile_h.assign((size_t)3 * ntiles, 0);
    P->fent_h.clear();
    P->face_lds = 0;
    if (P->n_rects == 0) return SN_OK;

    struct Face {
        int tile, q;
        FaceEntry e;
    };
    std::vector<Face> faces;
    bool staged = true;
    // element offset in the slot of tile (tx, ty) of grid cell (i, j), ghost cells included
    auto off = [&](int tx, int ty, int i, int j) -> uint16_t {
        const int c = i - tx * kTileX, r = j - ty * tile_rows + kGhost;
        int o = -1;
        if (c >= 0 && c < kTileX) {
            if (r >= 0 && r < tile_rows + 4) o = r * kTileX + c;
        } else if (c >= -2 && c < kTileX + 2) {
            const int hr = r - kGhost + xh;
            if (hr >= 0 && hr < tile_rows + 2 * xh) o = halo0 + hr * 4 + (c < 0 ? c + 2 : c - kTileX + 2);
        }
        if (o < 0 || o > (int)kFaceOffMask) {
            staged = false;
            return 0;
        }
        return (uint16_t)o;
    };
    // face between cells (i1c, j1c) and (i2c, j2c) = (i1c, j1c) + d, d the unit step along the axis
    auto add = [&](int q, int iin, int jin, bool yaxis, bool holds_c2, int i1c, int j1c, bool first) {
        const int tx = iin / kTileX, ty = jin / tile_rows;
        const int dx = yaxis ? 0 : 1, dy = yaxis ? 1 : 0;  // along the normal
        const int ex = yaxis ? 1 : 0, ey = yaxis ? 0 : 1;  // across it
        FaceEntry e{};
        e.off[0] = off(tx, ty, i1c - dx, j1c - dy);
        e.off[1] = off(tx, ty, i1c, j1c);
        e.off[2] = off(tx, ty, i1c + dx, j1c + dy);
        e.off[3] = off(tx, ty, i1c + 2 * dx, j1c + 2 * dy);
        if (P->order == 3) {
            e.off[4] = off(tx, ty, i1c - ex, j1c - ey);
            e.off[5] = off(tx, ty, i1c + ex, j1c + ey);
            e.off[6] = off(tx, ty, i1c + dx - ex, j1c + dy - ey);
            e.off[7] = off(tx, ty, i1c + dx + ex, j1c + dy + ey);
        }
        e.off[0] |= (uint16_t)(q << 14);
        e.off[1] |= (uint16_t)((yaxis ? 1 : 0) << 14 | (holds_c2 ? 1 : 0) << 15);
        e.off[2] |= (uint16_t)((first ? 1 : 0) << 14 | 1 << 15);
        faces.push_back(Face{ty * P->ntx + tx, q, e});
    };
    for (int q = 0; q < P->n_rects; ++q) {
        const int i0 = P->rects[q][0], j0 = P->rects[q][1], i1 = P->rects[q][2], j1 = P->rects[q][3];
        for (int j = j0; j < j1; ++j) add(q, i0, j, false, true, i0 - 1, j, i0 == 0);             // west
        for (int j = j0; j < j1; ++j) add(q, i1 - 1, j, false, false, i1 - 1, j, i1 == P->nx);    // east
        for (int i = i0; i < i1; ++i) add(q, i, j0, true, true, i, j0 - 1, j0 == 0);              // south
        for (int i = i0; i < i1; ++i) add(q, i, j1 - 1, true, false, i, j1 - 1, j1 == P->ny);     // north
    }
    if (!staged) return fail(SN_ERR_UNSUPPORTED, "a rectangle face reads a cell its tile does not stage");
    std::stable_sort(faces.begin(), faces.end(), [](const Face& x, const Face& y) {
        return x.tile != y.tile ? x.tile < y.tile : x.q < y.q;
    });
    for (size_t b = 0; b < faces.size();) {
        const int tile = faces[b].tile;
        size_t e = b;
        int cnt[kMaxRects] = {};
        while (e < faces.size() && faces[e].tile == tile) cnt[faces[e++].q]++;
        int fl = 0, lanes = 0;
        for (int cand = 1; cand <= kFacePerLaneMax && fl == 0; ++cand) {
            int l = 0;
            for (int q = 0; q < P->n_rects; ++q) l += (cnt[q] + cand - 1) / cand;
            if (l <= kWave) {
                fl = cand;
                lanes = l;
            }
        }
        if (fl == 0)  // a tile holds at most 4 x (2 x 128 + 2 x 8 x 4) faces
            return fail(SN_ERR_UNSUPPORTED, "%zu rectangle faces in one tile", e - b);
        P->ftile_h[3 * tile] = (int32_t)P->fent_h.size();
        P->ftile_h[3 * tile + 1] = fl;
        P->ftile_h[3 * tile + 2] = lanes;
        for (size_t c = b; c < e;) {  // one rectangle's faces
            const int q = faces[c].q;
            int m = 0;
            for (; c < e && faces[c].q == q; ++c, ++m) P->fent_h.push_back(faces[c].e);
            for (; m % fl != 0; ++m) {
                FaceEntry pad{};
                pad.off[0] = (uint16_t)(q << 14);
                P->fent_h.push_back(pad);
            }
        }
        if (fl > face_regs(P->order)) P->face_lds = std::max(P->face_lds, fl * lanes * (int)sizeof(FaceEntry));
        b = e;
    }
    return SN_OK;
}

sn_status derive(sn_plan* P, int group_size, int group_size_avg, int rows, int waves) {
    // dt = CFL * h (Sec. 5.1.3), adjusted so that N_t dt = T (Sec. 4.3).
    const double r = P->t_end / (P->cfl * P->h);
    P->nt = std::max(1, (int)std::ceil(r - 1e-9));
    P->dt = P->t_end / P->nt;

    int gs = 0, gsa = 0, rw = 0, wv = 0;
    default_shape(P, &gs, &gsa, &rw, &wv);
    if (group_size > 0) gs = std::min(group_size, P->M);
    if (group_size_avg > 0) gsa = std::min(group_size_avg, P->M);
    if (rows > 0) rw = rows;
    if (waves > 0) wv = waves;
    if (!supported_shape(rw, wv))
        return fail(SN_ERR_UNSUPPORTED, "launch shape rows_per_wave %d, waves %d not compiled", rw, wv);
    P->Mg_l[0] = gs;
    P->Mg_l[1] = gsa;
    for (int l = 0; l < 2; ++l) P->G_l[l] = (P->M + P->Mg_l[l] - 1) / P->Mg_l[l];
    P->G = std::max(P->G_l[0], P->G_l[1]);
    P->rows = rw;
    P->waves = wv;
    P->elem = P->dtype == SN_F32 ? 4 : 2;
    // Rows of 64-byte multiples holding the interior plus the two-cell ghost
    // frame; enough rows that every window of the last row of tiles is inside.
    // Rows of whole 128-byte lines; the interior starts one line in (ox
    // columns), so that 128-column tiles are line-aligned.
    const int line_elems = (int)(128 / P->elem);
    P->ox = line_elems;
    P->pitch = (P->ox + P->nx + kGhost + line_elems - 1) / line_elems * line_elems;
    P->ntx = (P->nx + kTileX - 1) / kTileX;
    P->nty = (P->ny + wv * rw - 1) / (wv * rw);
    P->ny_alloc = P->nty * wv * rw + 2 * kGhost;
    P->plane = (int64_t)P->ny_alloc * P->pitch;
    P->origin = (int64_t)kGhost * P->pitch + P->ox;
    if ((uint64_t)P->plane * P->elem >= (1ull << 31))
        return fail(SN_ERR_UNSUPPORTED, "one psi plane exceeds 2 GiB (grid %d x %d)", P->nx, P->ny);
    const int64_t n_wg = (int64_t)P->ntx * P->nty * P->G;
    if (n_wg > (int64_t)0x7fffffff) return fail(SN_ERR_UNSUPPORTED, "too many workgroups");
    P->n_wg = (int)n_wg;
    for (int l = 0; l < 2; ++l) P->n_wg_l[l] = P->ntx * P->nty * P->G_l[l];
    P->nq = 1 + P->n_tallies + 2 * P->n_rects + 3 * P->n_probes;
    {
        const sn_status st = probe_tables(P);
        if (st != SN_OK) return st;
        const sn_status sf = face_tables(P);
        if (sf != SN_OK) return sf;
    }

    P->psi_bytes = align256((size_t)P->M * (size_t)P->plane * P->elem);
    size_t off = 0;
    P->off_phi = off;
    off += align256((size_t)P->plane * sizeof(float));
    P->off_phi_part = off;
    off += align256((size_t)P->G * (size_t)P->plane * sizeof(float));
    P->off_ord = off;
    off += align256((size_t)P->M * sizeof(OrdConst));
    P->off_reg = off;
    off += align256((size_t)P->n_regions * sizeof(RegConst));
    P->off_region = off;
    off += align256((size_t)P->plane);
    P->off_qpart = off;
    off += align256((size_t)P->nq * P->n_wg * sizeof(double));
    P->off_qchunk = off;
    off += align256((size_t)P->nq * ((P->n_wg + kQoiChunk - 1) / kQoiChunk) * sizeof(double));
    P->off_qcount = off;
    off += align256(kMaxQ * sizeof(int32_t));
    P->off_scale = off;
    off += align256(kMaxQ * sizeof(double));
    P->off_inst = off;
    off += align256(kMaxQ * sizeof(double));
    P->off_integ = off;
    off += align256(kMaxQ * sizeof(double));
    P->off_mass0 = off;
    off += align256(sizeof(double));
    P->off_flags = off;
    off += align256(2 * sizeof(int32_t));
    P->off_sa64 = off;
    off += align256((size_t)P->n_regions * sizeof(double));
    P->off_fstatus = off;
    off += align256(sizeof(int32_t));
    P->off_fluence = off;
    if (P->fluence) off += align256((size_t)P->nx * P->ny * sizeof(double));
    P->off_pent = off;
    P->off_ptile = off;
    P->off_pmom = off;
    P->off_pacc = off;
    P->off_pstep = off;
    if (P->n_probes > 0) {
        P->off_pent = off;
        off += align256(std::max<size_t>(1, P->pent_h.size()) * sizeof(ProbeEntry));
        P->off_ptile = off;
        off += align256(P->ptile_h.size() * sizeof(int32_t));
        P->off_pmom = off;
        off += align256((size_t)P->M * 3 * sizeof(double));
        P->off_pacc = off;
        off += align256((size_t)P->n_windows * P->n_probes * 3 * sizeof(double));
        P->off_pstep = off;
        off += align256((size_t)3 * P->n_probes * sizeof(int32_t));
    }
    P->off_fent = off;
    P->off_ftile = off;
    if (P->n_rects > 0) {
        off += align256(std::max<size_t>(1, P->fent_h.size()) * sizeof(FaceEntry));
        P->off_ftile = off;
        off += align256(P->ftile_h.size() * sizeof(int32_t));
    }
    P->scratch_bytes = off;

    // Tables, computed in FP64 and rounded once.
    P->ord_h.assign(P->M, OrdConst{});
    for (int k = 0; k < P->M; ++k) {
        OrdConst& o = P->ord_h[k];
        o.cx = (float)(P->dt * P->xi[k] / P->h);
        o.cy = (float)(P->dt * P->eta[k] / P->h);
        o.w = (float)P->w[k];
        o.flags = (P->xi[k] > 0 ? 1 : 0) | (P->eta[k] > 0 ? 2 : 0);
        o.mx = P->mx[k];
        o.my = P->my[k];
        o.fx = P->w[k] * std::fabs(P->xi[k]);
        o.fy = P->w[k] * std::fabs(P->eta[k]);
    }
    P->reg_h.assign(P->n_regions, RegConst{});
    for (int r = 0; r < P->n_regions; ++r) {
        RegConst& c = P->reg_h[r];
        c.st = (float)(P->dt * (P->sa[r] + P->ss[r]));
        c.cs = (float)(P->dt * P->ss[r] / kTwoPi);
        c.cq = (float)(P->dt * P->q[r]);
        c.tally = P->tally[r];
        c.sa = P->sa[r];
    }
    P->pmom_h.assign((size_t)P->M * 3, 0.0);
    for (int k = 0; k < P->M; ++k) {
        P->pmom_h[3 * k] = P->w[k];
        P->pmom_h[3 * k + 1] = P->w[k] * P->xi[k];
        P->pmom_h[3 * k + 2] = P->w[k] * P->eta[k];
    }
    P->region_h.assign((size_t)P->plane, 0);
    for (int j = 0; j < P->ny; ++j)
        std::memcpy(&P->region_h[(size_t)(P->origin + (int64_t)j * P->pitch)], &P->region[(size_t)j * P->nx], P->nx);
    const double h2 = P->h * P->h;
    P->scale_h.assign(kMaxQ, 0.0);
    P->scale_h[0] = h2;
    for (int t = 0; t < P->n_tallies; ++t) P->scale_h[1 + t] = h2;
    for (int r = 0; r < 2 * P->n_rects; ++r) P->scale_h[1 + P->n_tallies + r] = P->h;
    for (int m = 0; m < 3 * P->n_probes; ++m) P->scale_h[1 + P->n_tallies + 2 * P->n_rects + m] = 1.0;
    double sw = 0;
    for (int k = 0; k < P->M; ++k) sw += P->w[k];
    double sq = 0;
    for (size_t c = 0; c < P->region.size(); ++c) sq += P->q[P->region[c]];
    P->source = sw * h2 * sq;
    return SN_OK;
}

}  // namespace

StageArgs snh::stage_args(const sn_plan* P, const char* in, const char* old, char* out) {
    const int l = old ? 1 : 0;  // only the averaging stage reads psi^n
    StageArgs a{};
    a.psi_in = in;
    a.psi_old = old;
    a.psi_out = out;
    a.phi = P->sp<float>(P->off_phi);
    a.phi_part = P->sp<float>(P->off_phi_part);
    a.ord = P->sp<OrdConst>(P->off_ord);
    a.reg = P->sp<RegConst>(P->off_reg);
    a.region = P->sp<uint8_t>(P->off_region);
    a.qpart = P->sp<double>(P->off_qpart);
    a.counter = P->sp<int32_t>(P->off_flags) + 1;
    a.plane = P->plane;
    a.nx = P->nx;
    a.ny = P->ny;
    a.pitch = P->pitch;
    a.M = P->M;
    a.ox = P->ox;
    a.G = P->G_l[l];
    a.Mg = P->Mg_l[l];
    a.ntx = P->ntx;
    a.nty = P->nty;
    a.n_wg = P->n_wg_l[l];
    a.n_tallies = P->n_tallies;
    a.n_rects = P->n_rects;
    a.nq = P->nq;
    for (int s = 0; s < 4; ++s) a.bc[s] = P->bc[s];
    if (P->n_rects > 0) {
        a.fent = P->sp<FaceEntry>(P->off_fent);
        a.ftile = P->sp<int32_t>(P->off_ftile);
        a.face_lds = P->face_lds;
    }
    {
        const double A = P->h * P->h, eps = A * A * A;  // K A^3 with K = 1 (Sec. 4.2)
        a.eps2 = (float)(eps * eps);
    }
    a.n_probes = P->n_probes;
    a.qprobe = 1 + P->n_tallies + 2 * P->n_rects;
    if (P->n_probes > 0) {
        a.pent = P->sp<ProbeEntry>(P->off_pent);
        a.ptile = P->sp<int32_t>(P->off_ptile);
        a.pmom = P->sp<double>(P->off_pmom);
    }
    return a;
}

int snh::finalize_workgroups(const sn_plan* P, int kind) {
    const int l = kind == 2 ? 1 : 0;
    const int phi_wg = kind < 0 ? 0 : (int)(((int64_t)P->ny * (P->pitch / 4) + 255) / 256);
    return P->nq * ((P->n_wg_l[l] + kQoiChunk - 1) / kQoiChunk) + phi_wg;
}

FinalizeArgs snh::finalize_args(const sn_plan* P, int kind) {
    const int l = kind == 2 ? 1 : 0;  // layout of the stage just run
    FinalizeArgs f{};
    f.phi_part = P->sp<float>(P->off_phi_part);
    f.phi = P->sp<float>(P->off_phi);
    f.plane = P->plane;
    f.nx = P->nx;
    f.ny = P->ny;
    f.pitch = P->pitch;
    f.G = P->G_l[l];
    f.ox = P->ox;
    f.n_phi_wg = kind < 0 ? 0 : (int)(((int64_t)P->ny * (P->pitch / 4) + 255) / 256);
    f.qpart = P->sp<double>(P->off_qpart);
    f.scale = P->sp<double>(P->off_scale);
    f.inst = P->sp<double>(P->off_inst);
    f.integ = P->sp<double>(P->off_integ);
    f.qchunk = P->sp<double>(P->off_qchunk);
    f.qcount = P->sp<int32_t>(P->off_qcount);
    f.q_split = (P->n_wg_l[l] + kQoiChunk - 1) / kQoiChunk;
    f.flags = P->sp<int32_t>(P->off_flags);
    f.counter = P->sp<int32_t>(P->off_flags) + 1;
    f.coef = kind == 0 ? P->dt : (kind > 0 ? 0.5 * P->dt : 0.0);
    f.n_wg = P->n_wg_l[l];
    f.nq = P->nq;
    f.fluence = P->fluence ? P->sp<double>(P->off_fluence) : nullptr;
    f.n_probes = kind < 0 ? 0 : P->n_probes;
    f.qprobe = 1 + P->n_tallies + 2 * P->n_rects;
    if (P->n_probes > 0) {
        f.pacc = P->sp<double>(P->off_pacc);
        f.pstep = P->sp<int32_t>(P->off_pstep);
        f.pcoef = f.coef / (P->t_end / P->n_windows);
        f.n_windows = P->n_windows;
        f.nt = P->nt;
        f.last_stage = kind == 0 || kind == 2 ? 1 : 0;
    }
    return f;
}

namespace {

GhostArgs ghost_args(const sn_plan* P, char* psi) {
    GhostArgs ga{};
    ga.psi = psi;
    ga.ord = P->sp<OrdConst>(P->off_ord);
    ga.plane = P->plane;
    ga.nx = P->nx;
    ga.ny = P->ny;
    ga.pitch = P->pitch;
    ga.M = P->M;
    ga.ox = P->ox;
    for (int side = 0; side < 4; ++side) {
        ga.bc[side] = P->bc[side];
        ga.ghost[side] = P->bc[side] == SN_BC_INFLOW ? (float)P->inflow[side] : 0.0f;
    }
    ga.all_dirs = P->order == 3 ? 1 : 0;
    return ga;
}

sn_status flush_events(sn_plan* P) {
    for (int e = 0; e < P->ev_used; ++e) {
        HIP_TRY(hipEventSynchronize(P->ev_stop[e]), "hipEventSynchronize");
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, P->ev_start[e], P->ev_stop[e]), "hipEventElapsedTime");
        P->kernel_ms[P->ev_kind[e]] += ms;
        P->kernel_count[P->ev_kind[e]] += 1;
    }
    P->ev_used = 0;
    return SN_OK;
}

// Launch one stage kernel and its QoI finalize. kind: 0 Euler, 1 Heun-1,
// 2 Heun-2, -1 QoI only.
sn_status launch_stage_pair(sn_plan* P, int kind, hipStream_t s, bool allow_timing) {
    int mode = kind == 2 ? kAverage : (kind < 0 ? kQoiOnly : kUpdate);
    const char* in = P->psi[P->cur];
    char* out = P->psi[P->cur ^ 1];
    const char* old = nullptr;
    if (kind == 2) {  // Heun stage 2: reads psi^(1) in B, psi^n in A, writes A
        in = P->psi[1];
        old = P->psi[0];
        out = P->psi[0];
    }
    if (kind < 0) out = nullptr;
    StageArgs a = stage_args(P, in, old, out);
    const bool timed = P->timing && allow_timing && kind >= 0;
    if (timed) {
        if (P->ev_used == (int)P->ev_start.size()) {
            sn_status st = flush_events(P);
            if (st != SN_OK) return st;
        }
        HIP_TRY(hipEventRecord(P->ev_start[P->ev_used], s), "hipEventRecord");
    }
    HIP_TRY(launch_stage(P->order, mode, P->dtype, P->rows, P->waves, a, s), "stage launch");
    if (timed) {
        HIP_TRY(hipEventRecord(P->ev_stop[P->ev_used], s), "hipEventRecord");
        P->ev_kind[P->ev_used] = kind;
        P->ev_used++;
    }
    const FinalizeArgs f = finalize_args(P, kind);
    HIP_TRY(launch_finalize(f, s), "finalize launch");
    return SN_OK;
}

sn_status launch_steps(sn_plan* P, int n, hipStream_t s, bool allow_timing) {
    for (int it = 0; it < n; ++it) {
        sn_status st;
        if (P->stepper == SN_EULER) {
            st = launch_stage_pair(P, 0, s, allow_timing);
            if (st != SN_OK) return st;
            P->cur ^= 1;
        } else {
            st = launch_stage_pair(P, 1, s, allow_timing);
            if (st != SN_OK) return st;
            st = launch_stage_pair(P, 2, s, allow_timing);
            if (st != SN_OK) return st;
        }
        P->step++;
    }
    return SN_OK;
}

void drop_graph(sn_plan* P) {
    if (P->graph_exec) (void)hipGraphExecDestroy(P->graph_exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    P->graph_exec = nullptr;
    P->graph = nullptr;
}

sn_status run_steps(sn_plan* P, int n, hipStream_t s) {
    if (!P->bound || !P->inited) return fail(SN_ERR_STATE, "plan not bound and initialised");
    if (P->batch) return fail(SN_ERR_STATE, "plan is admitted to a batch; the batch advances it");
    if (n <= 0) return SN_OK;
    int done = 0;
    if (P->graph_steps > 0 && !P->timing) {
        const int K = P->graph_steps;
        // the graph covers K steps and starts from buffer parity 0
        if (n >= K && P->cur == 0) {
            if (!P->graph_exec) {
                hipStream_t cs;
                HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
                HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
                const int64_t step0 = P->step;
                sn_status st = launch_steps(P, K, cs, false);
                P->step = step0;
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamEndCapture(cs, &g);
                (void)hipStreamDestroy(cs);
                if (st != SN_OK) {
                    if (g) (void)hipGraphDestroy(g);
                    return st;
                }
                if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
                P->graph = g;
                HIP_TRY(hipGraphInstantiate(&P->graph_exec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
            }
            while (n - done >= K) {
                HIP_TRY(hipGraphLaunch(P->graph_exec, s), "hipGraphLaunch");
                P->step += K;
                done += K;
            }
        }
    }
    return launch_steps(P, n - done, s, true);
}

}  // namespace

sn_status snh::issue_steps(sn_plan* P, int n, hipStream_t s) { return launch_steps(P, n, s, false); }

sn_status snh::bind_buffers(sn_plan* P, void* psi_a, void* psi_b, void* scratch) {
    if (!P || !psi_a || !psi_b || !scratch) return fail(SN_ERR_INVALID, "NULL argument");
    if (P->batch) return fail(SN_ERR_STATE, "plan is admitted to a batch");
    const uintptr_t pa = (uintptr_t)psi_a, pb = (uintptr_t)psi_b, ps = (uintptr_t)scratch;
    if ((pa | pb | ps) & 255) return fail(SN_ERR_INVALID, "device buffers must be 256-byte aligned");
    auto overlap = [](uintptr_t a, size_t na, uintptr_t b, size_t nb) { return a < b + nb && b < a + na; };
    if (overlap(pa, P->psi_bytes, pb, P->psi_bytes) || overlap(pa, P->psi_bytes, ps, P->scratch_bytes) ||
        overlap(pb, P->psi_bytes, ps, P->scratch_bytes))
        return fail(SN_ERR_INVALID, "device buffers overlap");
    drop_graph(P);
    P->psi[0] = (char*)psi_a;
    P->psi[1] = (char*)psi_b;
    P->scratch = (char*)scratch;
    P->static_dev = -1;
    P->bound = true;
    P->inited = false;
    return SN_OK;
}

extern "C" {

const char* sn_last_error(void) { return snh::last_error(); }

const char* sn_status_str(sn_status s) {
    switch (s) {
    case SN_OK: return "ok";
    case SN_ERR_INVALID: return "invalid argument";
    case SN_ERR_OOM: return "out of memory";
    case SN_ERR_DEVICE: return "device error";
    case SN_ERR_UNSUPPORTED: return "unsupported";
    case SN_ERR_NONFINITE: return "non-finite QoI";
    case SN_ERR_BUSY: return "over budget";
    case SN_ERR_STATE: return "bad call order";
    default: return "unknown status";
    }
}

sn_status sn_plan_create_shaped(const sn_problem* problem, int32_t group_size, int32_t group_size_avg,
                                int32_t rows_per_wave, int32_t waves_per_group, sn_plan** out) {
    if (!out) return fail(SN_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (group_size < 0 || group_size_avg < 0 || rows_per_wave < 0 || waves_per_group < 0)
        return fail(SN_ERR_INVALID, "negative launch shape");
    sn_plan* P = new (std::nothrow) sn_plan();
    if (!P) return fail(SN_ERR_OOM, "plan allocation failed");
    sn_status st;
    try {
        st = validate_and_copy(problem, P);
        if (st == SN_OK) st = derive(P, group_size, group_size_avg, rows_per_wave, waves_per_group);
    } catch (const std::bad_alloc&) {
        st = fail(SN_ERR_OOM, "host allocation failed");
    }
    if (st != SN_OK) {
        delete P;
        return st;
    }
    *out = P;
    return SN_OK;
}

sn_status sn_plan_create_tuned(const sn_problem* problem, int32_t group_size, int32_t rows_per_wave,
                               int32_t waves_per_group, sn_plan** out) {
    return sn_plan_create_shaped(problem, group_size, group_size, rows_per_wave, waves_per_group, out);
}

sn_status sn_plan_create(const sn_problem* problem, sn_plan** out) {
    return sn_plan_create_shaped(problem, 0, 0, 0, 0, out);
}

sn_status sn_plan_get_info(const sn_plan* P, sn_plan_info* out) {
    if (!P || !out) return fail(SN_ERR_INVALID, "NULL argument");
    out->n_steps = P->nt;
    out->dt = P->dt;
    out->nx = P->nx;
    out->ny = P->ny;
    out->M = P->M;
    out->pitch = P->pitch;
    out->n_groups = P->G_l[0];
    out->group_size = P->Mg_l[0];
    out->rows_per_wave = P->rows;
    out->waves_per_group = P->waves;
    out->n_workgroups = P->n_wg_l[0];
    out->n_groups_average = P->G_l[1];
    out->group_size_average = P->Mg_l[1];
    out->n_workgroups_average = P->n_wg_l[1];
    out->psi_bytes = P->psi_bytes;
    out->scratch_bytes = P->scratch_bytes;
    out->psi_dtype = P->dtype;
    out->step = (int32_t)P->step;
    return SN_OK;
}

sn_status sn_plan_bind(sn_plan* P, void* psi_a, void* psi_b, void* scratch) {
    if (!P) return fail(SN_ERR_INVALID, "NULL argument");
    const int old_dev = P->static_dev;
    const sn_status st = snh::bind_buffers(P, psi_a, psi_b, scratch);
    if (st == SN_OK && old_dev >= 0) snh::release_static_scratch(P, old_dev);
    return st;
}


sn_status sn_plan_init(sn_plan* P, const float* psi0, void* stream) {
    if (!P) return fail(SN_ERR_INVALID, "plan is NULL");
    if (P->batch) return fail(SN_ERR_STATE, "plan is admitted to a batch");
    if (!P->bound) return fail(SN_ERR_STATE, "plan not bound");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(P->sp<char>(P->off_ord), P->ord_h.data(), P->M * sizeof(OrdConst),
                           hipMemcpyHostToDevice, s), "upload ordinates");
    HIP_TRY(hipMemcpyAsync(P->sp<char>(P->off_reg), P->reg_h.data(), P->n_regions * sizeof(RegConst),
                           hipMemcpyHostToDevice, s), "upload regions");
    HIP_TRY(hipMemcpyAsync(P->sp<char>(P->off_region), P->region_h.data(), P->region_h.size(),
                           hipMemcpyHostToDevice, s), "upload region map");
    HIP_TRY(hipMemcpyAsync(P->sp<char>(P->off_scale), P->scale_h.data(), kMaxQ * sizeof(double),
                           hipMemcpyHostToDevice, s), "upload scales");
    HIP_TRY(hipMemsetAsync(P->sp<char>(P->off_integ), 0, kMaxQ * sizeof(double), s), "clear integrals");
    HIP_TRY(hipMemsetAsync(P->sp<char>(P->off_inst), 0, kMaxQ * sizeof(double), s), "clear QoIs");
    HIP_TRY(hipMemsetAsync(P->sp<char>(P->off_flags), 0, 2 * sizeof(int32_t), s), "clear flags and stage counter");
    HIP_TRY(hipMemsetAsync(P->sp<char>(P->off_qcount), 0, kMaxQ * sizeof(int32_t), s), "clear QoI chunk counts");
    HIP_TRY(hipMemsetAsync(P->sp<char>(P->off_phi), 0, P->plane * sizeof(float), s), "clear phi");
    HIP_TRY(hipMemcpyAsync(P->sp<char>(P->off_sa64), P->sa.data(), P->n_regions * sizeof(double),
                           hipMemcpyHostToDevice, s), "upload sigma_a");
    if (P->fluence)
        HIP_TRY(hipMemsetAsync(P->sp<char>(P->off_fluence), 0, (size_t)P->nx * P->ny * sizeof(double), s),
                "clear fluence");
    if (P->n_rects > 0) {
        if (!P->fent_h.empty())
            HIP_TRY(hipMemcpyAsync(P->sp<char>(P->off_fent), P->fent_h.data(), P->fent_h.size() * sizeof(FaceEntry),
                                   hipMemcpyHostToDevice, s), "upload face entries");
        HIP_TRY(hipMemcpyAsync(P->sp<char>(P->off_ftile), P->ftile_h.data(), P->ftile_h.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, s), "upload face tiles");
    }
    if (P->n_probes > 0) {
        if (!P->pent_h.empty())
            HIP_TRY(hipMemcpyAsync(P->sp<char>(P->off_pent), P->pent_h.data(), P->pent_h.size() * sizeof(ProbeEntry),
                                   hipMemcpyHostToDevice, s), "upload probe entries");
        HIP_TRY(hipMemcpyAsync(P->sp<char>(P->off_ptile), P->ptile_h.data(), P->ptile_h.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, s), "upload probe tiles");
        HIP_TRY(hipMemcpyAsync(P->sp<char>(P->off_pmom), P->pmom_h.data(), P->pmom_h.size() * sizeof(double),
                               hipMemcpyHostToDevice, s), "upload probe moments");
        HIP_TRY(hipMemsetAsync(P->sp<char>(P->off_pacc), 0,
                               (size_t)P->n_windows * P->n_probes * 3 * sizeof(double), s), "clear probe windows");
        HIP_TRY(hipMemsetAsync(P->sp<char>(P->off_pstep), 0, (size_t)3 * P->n_probes * sizeof(int32_t), s),
                "clear probe steps");
    }
    HIP_TRY(hipMemsetAsync(P->psi[0], 0, P->psi_bytes, s), "clear psi A");
    HIP_TRY(hipMemsetAsync(P->psi[1], 0, P->psi_bytes, s), "clear psi B");
    P->cur = 0;
    P->step = 0;
    drop_graph(P);
    if (psi0) {
        if (P->dtype == SN_F32) {
            for (int k = 0; k < P->M; ++k)
                HIP_TRY(hipMemcpy2DAsync(P->psi[0] + (k * P->plane + P->origin) * sizeof(float), P->pitch * sizeof(float),
                                         psi0 + (size_t)k * P->ny * P->nx, P->nx * sizeof(float), P->nx * sizeof(float),
                                         P->ny, hipMemcpyHostToDevice, s), "upload psi0");
            HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        } else {
            std::vector<uint16_t> tmp;
            try {
                tmp.resize((size_t)P->M * P->ny * P->nx);
            } catch (const std::bad_alloc&) {
                return fail(SN_ERR_OOM, "host staging for psi0");
            }
            for (size_t e = 0; e < tmp.size(); ++e) {
                uint32_t u;
                std::memcpy(&u, &psi0[e], 4);
                if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
                    u = (u >> 16) | 0x40u;
                else
                    u = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
                tmp[e] = (uint16_t)u;
            }
            for (int k = 0; k < P->M; ++k)
                HIP_TRY(hipMemcpy2DAsync(P->psi[0] + (k * P->plane + P->origin) * 2, P->pitch * 2,
                                         tmp.data() + (size_t)k * P->ny * P->nx, P->nx * 2, P->nx * 2, P->ny,
                                         hipMemcpyHostToDevice, s), "upload psi0");
            HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        }
        PhiInitArgs pa{};
        pa.psi = P->psi[0];
        pa.phi = P->sp<float>(P->off_phi);
        pa.ord = P->sp<OrdConst>(P->off_ord);
        pa.plane = P->plane;
        pa.nx = P->nx;
        pa.ny = P->ny;
        pa.pitch = P->pitch;
        pa.M = P->M;
        pa.ox = P->ox;
        HIP_TRY(launch_phi_init(P->dtype, pa, s), "phi init launch");
    }
    // Ghost frames of both buffers: B's incoming vacuum/inflow ghosts are
    // constants the stages never rewrite.
    for (int b = 0; b < 2; ++b) HIP_TRY(launch_ghost_fill(P->dtype, ghost_args(P, P->psi[b]), s), "ghost fill launch");
    // QoIs of the initial state: keep mass(0) for the balance residual.
    P->inited = true;
    sn_status st = launch_stage_pair(P, -1, s, false);
    if (st != SN_OK) return st;
    HIP_TRY(hipMemcpyAsync(P->sp<char>(P->off_mass0), P->sp<char>(P->off_inst), sizeof(double),
                           hipMemcpyDeviceToDevice, s), "save mass0");
    return SN_OK;
}

sn_status sn_plan_run(sn_plan* P, int32_t n_steps, void* stream) {
    if (!P) return fail(SN_ERR_INVALID, "plan is NULL");
    if (n_steps < 0) return fail(SN_ERR_INVALID, "n_steps < 0");
    const int64_t left = P->nt - P->step;
    const int n = (int)std::min<int64_t>(n_steps, std::max<int64_t>(left, 0));
    return run_steps(P, n, (hipStream_t)stream);
}

sn_status sn_plan_run_unbounded(sn_plan* P, int32_t n_steps, void* stream) {
    if (!P) return fail(SN_ERR_INVALID, "plan is NULL");
    if (n_steps < 0) return fail(SN_ERR_INVALID, "n_steps < 0");
    return run_steps(P, n_steps, (hipStream_t)stream);
}

sn_status sn_plan_qoi(sn_plan* P, sn_qoi* out, void* stream) {
    if (!P || !out) return fail(SN_ERR_INVALID, "NULL argument");
    if (!P->bound || !P->inited) return fail(SN_ERR_STATE, "plan not bound and initialised");
    hipStream_t s = (hipStream_t)stream;
    sn_status st = launch_stage_pair(P, -1, s, false);
    if (st != SN_OK) return st;
    double inst[kMaxQ], integ[kMaxQ], mass0 = 0;
    int32_t flags = 0;
    HIP_TRY(hipMemcpyAsync(inst, P->sp<char>(P->off_inst), sizeof inst, hipMemcpyDeviceToHost, s), "read QoIs");
    HIP_TRY(hipMemcpyAsync(integ, P->sp<char>(P->off_integ), sizeof integ, hipMemcpyDeviceToHost, s),
            "read integrals");
    HIP_TRY(hipMemcpyAsync(&mass0, P->sp<char>(P->off_mass0), sizeof mass0, hipMemcpyDeviceToHost, s),
            "read mass0");
    HIP_TRY(hipMemcpyAsync(&flags, P->sp<char>(P->off_flags), sizeof flags, hipMemcpyDeviceToHost, s),
            "read flags");
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    std::memset(out, 0, sizeof *out);
    const int T = P->n_tallies, R = P->n_rects;
    out->step = P->step;
    out->t = P->step * P->dt;
    out->n_tallies = T;
    out->n_rects = R;
    out->mass = inst[0];
    out->source = P->source;
    out->int_mass = integ[0];
    out->int_source = P->source * out->t;
    double sum_abs = 0;
    for (int t = 0; t < T; ++t) {
        out->absorption[t] = inst[1 + t];
        out->int_absorption[t] = integ[1 + t];
        sum_abs += integ[1 + t];
    }
    for (int r = 0; r < R; ++r) {
        out->outflow[r] = inst[1 + T + r];
        out->inflow[r] = inst[1 + T + R + r];
        out->int_outflow[r] = integ[1 + T + r];
        out->int_inflow[r] = integ[1 + T + R + r];
    }
    const bool domain_rect =
        R > 0 && P->rects[0][0] == 0 && P->rects[0][1] == 0 && P->rects[0][2] == P->nx && P->rects[0][3] == P->ny;
    if (domain_rect) {
        out->balance_residual =
            out->mass - (mass0 + out->int_source + out->int_inflow[0] - out->int_outflow[0] - sum_abs);
    } else {
        out->balance_residual = 0.0;
    }
    bool nonfinite = flags != 0;
    for (int e = 0; e < P->nq; ++e) nonfinite = nonfinite || !std::isfinite(inst[e]) || !std::isfinite(integ[e]);
    out->nonfinite = nonfinite ? 1 : 0;
    if (nonfinite) return fail(SN_ERR_NONFINITE, "a QoI is NaN or infinite at step %lld", (long long)P->step);
    return SN_OK;
}

sn_status sn_plan_read_psi(const sn_plan* P, float* host_out, void* stream) {
    if (!P || !host_out) return fail(SN_ERR_INVALID, "NULL argument");
    if (!P->bound || !P->inited) return fail(SN_ERR_STATE, "plan not bound and initialised");
    hipStream_t s = (hipStream_t)stream;
    if (P->dtype == SN_F32) {
        for (int k = 0; k < P->M; ++k)
            HIP_TRY(hipMemcpy2DAsync(host_out + (size_t)k * P->ny * P->nx, P->nx * sizeof(float),
                                     P->psi[P->cur] + (k * P->plane + P->origin) * sizeof(float),
                                     P->pitch * sizeof(float), P->nx * sizeof(float), P->ny, hipMemcpyDeviceToHost, s),
                    "read psi");
        HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    } else {
        std::vector<uint16_t> tmp((size_t)P->M * P->ny * P->nx);
        for (int k = 0; k < P->M; ++k)
            HIP_TRY(hipMemcpy2DAsync(tmp.data() + (size_t)k * P->ny * P->nx, P->nx * 2,
                                     P->psi[P->cur] + (k * P->plane + P->origin) * 2, P->pitch * 2, P->nx * 2, P->ny,
                                     hipMemcpyDeviceToHost, s), "read psi");
        HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        for (size_t e = 0; e < tmp.size(); ++e) {
            uint32_t u = (uint32_t)tmp[e] << 16;
            std::memcpy(&host_out[e], &u, 4);
        }
    }
    return SN_OK;
}

sn_status sn_plan_read_phi(const sn_plan* P, float* host_out, void* stream) {
    if (!P || !host_out) return fail(SN_ERR_INVALID, "NULL argument");
    if (!P->bound || !P->inited) return fail(SN_ERR_STATE, "plan not bound and initialised");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpy2DAsync(host_out, P->nx * sizeof(float), P->sp<char>(P->off_phi) + P->origin * sizeof(float),
                             P->pitch * sizeof(float),
                             P->nx * sizeof(float), P->ny, hipMemcpyDeviceToHost, s), "read phi");
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    return SN_OK;
}

sn_status sn_plan_read_probes(const sn_plan* P, double* host_out, void* stream) {
    if (!P || !host_out) return fail(SN_ERR_INVALID, "NULL argument");
    if (!P->bound || !P->inited) return fail(SN_ERR_STATE, "plan not bound and initialised");
    if (P->n_probes == 0) return fail(SN_ERR_STATE, "plan has no probes");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(host_out, P->sp<char>(P->off_pacc), (size_t)P->n_windows * P->n_probes * 3 * sizeof(double),
                           hipMemcpyDeviceToHost, s), "read probes");
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    return SN_OK;
}

sn_status sn_plan_read_fluence(const sn_plan* P, double* host_out, void* stream) {
    if (!P || !host_out) return fail(SN_ERR_INVALID, "NULL argument");
    if (!P->bound || !P->inited) return fail(SN_ERR_STATE, "plan not bound and initialised");
    if (!P->fluence) return fail(SN_ERR_STATE, "plan does not accumulate the fluence");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(host_out, P->sp<char>(P->off_fluence), (size_t)P->nx * P->ny * sizeof(double),
                           hipMemcpyDeviceToHost, s), "read fluence");
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    return SN_OK;
}

sn_status sn_plan_fluence_functionals(const sn_plan* P, const sn_fluence_piece* pieces, int32_t n_pieces,
                                      const int32_t* set_start, int32_t n_blocks, double* out, void* stream) {
    static_assert(sizeof(sn_fluence_piece) == sizeof(FluencePiece), "piece layout");
    if (!P || !set_start || !out || (n_pieces > 0 && !pieces)) return fail(SN_ERR_INVALID, "NULL argument");
    if (!P->bound || !P->inited) return fail(SN_ERR_STATE, "plan not bound and initialised");
    if (!P->fluence) return fail(SN_ERR_STATE, "plan does not accumulate the fluence");
    if (n_pieces < 0) return fail(SN_ERR_INVALID, "n_pieces < 0");
    if (n_blocks < 1 || n_blocks > kMaxFluenceBlocks)
        return fail(SN_ERR_INVALID, "n_blocks = %d out of range [1, %d]", n_blocks, kMaxFluenceBlocks);
    if (((uintptr_t)pieces & 7) || ((uintptr_t)set_start & 3) || ((uintptr_t)out & 7))
        return fail(SN_ERR_INVALID, "misaligned device array");
    hipStream_t s = (hipStream_t)stream;
    FluenceArgs a{};
    a.fluence = P->sp<double>(P->off_fluence);
    a.region = P->sp<uint8_t>(P->off_region);
    a.sa = P->sp<double>(P->off_sa64);
    a.pieces = reinterpret_cast<const FluencePiece*>(pieces);
    a.set_start = set_start;
    a.out = out;
    a.status = P->sp<int32_t>(P->off_fstatus);
    a.origin = P->origin;
    a.pitch = P->pitch;
    a.nx = P->nx;
    a.ny = P->ny;
    a.n_pieces = n_pieces;
    a.n_blocks = n_blocks;
    HIP_TRY(launch_fluence_functionals(a, s), "fluence functionals launch");
    int32_t status = -1;
    HIP_TRY(hipMemcpyAsync(&status, a.status, sizeof status, hipMemcpyDeviceToHost, s), "read status");
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (status != 0) return fail(SN_ERR_INVALID, "malformed piece list (cell index, weight or set_start)");
    return SN_OK;
}

sn_status sn_plan_use_graph(sn_plan* P, int32_t steps_per_graph) {
    if (!P) return fail(SN_ERR_INVALID, "plan is NULL");
    if (steps_per_graph < 0 || steps_per_graph == 1 || (steps_per_graph & 1))
        return fail(SN_ERR_INVALID, "steps_per_graph must be 0 or an even number >= 2");
    drop_graph(P);
    P->graph_steps = steps_per_graph;
    return SN_OK;
}

sn_status sn_plan_set_timing(sn_plan* P, int32_t on) {
    if (!P) return fail(SN_ERR_INVALID, "plan is NULL");
    if (on && P->ev_start.empty()) {
        const int cap = 512;
        P->ev_start.resize(cap);
        P->ev_stop.resize(cap);
        P->ev_kind.resize(cap);
        for (int e = 0; e < cap; ++e) {
            HIP_TRY(hipEventCreate(&P->ev_start[e]), "hipEventCreate");
            HIP_TRY(hipEventCreate(&P->ev_stop[e]), "hipEventCreate");
        }
    }
    if (!on) {
        sn_status st = flush_events(P);
        if (st != SN_OK) return st;
    }
    P->timing = on != 0;
    for (int k = 0; k < 4; ++k) {
        P->kernel_ms[k] = 0;
        P->kernel_count[k] = 0;
    }
    return SN_OK;
}

sn_status sn_plan_kernel_ms(sn_plan* P, double ms[4], int64_t counts[4]) {
    if (!P || !ms || !counts) return fail(SN_ERR_INVALID, "NULL argument");
    sn_status st = flush_events(P);
    if (st != SN_OK) return st;
    for (int k = 0; k < 4; ++k) {
        ms[k] = P->kernel_ms[k];
        counts[k] = P->kernel_count[k];
    }
    return SN_OK;
}

void sn_plan_destroy(sn_plan* P) {
    if (!P) return;
    if (P->static_dev >= 0) snh::release_static_scratch(P, P->static_dev);
    drop_graph(P);
    for (auto e : P->ev_start) (void)hipEventDestroy(e);
    for (auto e : P->ev_stop) (void)hipEventDestroy(e);
    delete P;
}

}  // extern "C"
