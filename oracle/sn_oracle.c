/*
 * sn_oracle.c -- FP64 reference of the explicit S_N finite-volume transport
 * step on a uniform Cartesian grid.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the checker that the HIP path is
 * compared against. Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it. It shares no code, header, table or constant
 * with the product library.
 *
 * It follows arXiv 2505.17284 as written, with plain loops and no blocking,
 * fusion or reordering:
 *   - S_N system, scalar flux phi = sum_l w_l psi_l, scattering sigma_s/(2 pi)
 *     phi, isotropic source Q added to every ordinate: Sec. 4.1, eq. eq_sn_2d.
 *   - cell balance with the upwind numerical trace (Heaviside selection of the
 *     reconstruction of the upwind cell): Sec. 4.2, eqs. eq_sn_2d_eqn_fv and
 *     eq_upwind1stOrder, on square cells (edge length h, area h^2; the flux sum
 *     is divided by the cell area).
 *   - order 3: the Green-Gauss gradient with the Venkatakrishnan limiter
 *     (Sec. 4.2, eq. eq_V_limiter) on square cells.
 *   - ghost cells carrying the inflow value, first-order fluxes on boundary
 *     faces: end of Sec. 4.2.
 *   - forward Euler and Heun's method (SSP-RK2) with dt = T / N_t: Sec. 4.3,
 *     eq. eq_ODE; dt = CFL * dx: Sec. 5.1.3.
 *   - QoIs: mass (QoI-5), absorption per region (QoI-3/4), outflow through the
 *     boundary of a rectangle (QoI-1/2): Sec. 3.1.2.
 *   - optional: the time integral of phi per cell (fluence) and space-time
 *     probe averages of phi, J_x, J_y (the Hohlraum QoIs of Sec. 3.2.2).
 * The readings taken where the paper is silent (minmod reconstruction on the
 * Cartesian grid, reflective walls, the time rule for integrated QoIs, the
 * boundary-slope rule) are listed in the design notes and restated where they
 * are used below.
 *
 * Layout: psi[(k * ny + j) * nx + i], k = ordinate, j = row (y), i = column (x).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_VACUUM 0
#define ORC_INFLOW 1
#define ORC_REFLECT 2
#define ORC_W 0
#define ORC_E 1
#define ORC_S 2
#define ORC_N 3

typedef struct {
    int nx, ny;
    double h;
    int M;
    const double *xi, *eta, *w;
    const int *mirror_x, *mirror_y;
    const unsigned char *region;
    int n_regions;
    const double *sigma_a, *sigma_s, *q;
    const unsigned char *tally;
    int n_tallies;
    int bc[4];
    double inflow[4];
    int order, stepper;
    double cfl, t_end;
    int n_rects;
    const int *rects; /* [n_rects][4] = i0, j0, i1, j1 (half-open cell ranges) */
} orc_problem;

static const double TWO_PI = 6.283185307179586476925286766559;

static double PSI(const orc_problem *P, const double *psi, int k, int j, int i)
{
    return psi[((size_t)k * P->ny + j) * P->nx + i];
}

int orc_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Number of steps: dt = CFL * h (Sec. 5.1.3) rounded so that N_t dt = T
 * exactly (Sec. 4.3): N_t = ceil(T / (CFL h) - 1e-9), dt = T / N_t. */
int orc_num_steps(const orc_problem *P, double *dt)
{
    double r = P->t_end / (P->cfl * P->h);
    int nt = (int)ceil(r - 1e-9);
    if (nt < 1) nt = 1;
    if (dt) *dt = P->t_end / nt;
    return nt;
}

/* phi = sum_l w_l psi_l (eq. eq_sn_2d), summed in ordinate order. */
void orc_scalar_flux(const orc_problem *P, const double *psi, double *phi)
{
    int c, l;
    int ncell = P->nx * P->ny;
#pragma omp parallel for private(l)
    for (c = 0; c < ncell; ++c) {
        double s = 0.0;
        for (l = 0; l < P->M; ++l) s += P->w[l] * psi[(size_t)l * ncell + c];
        phi[c] = s;
    }
}

/* Ghost value on a side for ordinate k at position idx along that side (row j
 * for W/E, column i for S/N). Vacuum: 0. Inflow: the isotropic inflow value
 * (end of Sec. 4.2). Reflective: the mirror ordinate's value in the adjacent
 * boundary cell. */
static double ghost(const orc_problem *P, const double *psi, int side, int k, int idx)
{
    switch (P->bc[side]) {
    case ORC_INFLOW:
        return P->inflow[side];
    case ORC_REFLECT:
        if (side == ORC_W) return PSI(P, psi, P->mirror_x[k], idx, 0);
        if (side == ORC_E) return PSI(P, psi, P->mirror_x[k], idx, P->nx - 1);
        if (side == ORC_S) return PSI(P, psi, P->mirror_y[k], 0, idx);
        return PSI(P, psi, P->mirror_y[k], P->ny - 1, idx);
    default:
        return 0.0;
    }
}

static double minmod(double a, double b)
{
    if (a > 0.0 && b > 0.0) return a < b ? a : b;
    if (a < 0.0 && b < 0.0) return a > b ? a : b;
    return 0.0;
}

/* Value of ordinate k in cell i of row j, or the ghost value when i is outside. */
static double cell_x(const orc_problem *P, const double *psi, int k, int j, int i)
{
    if (i < 0) return ghost(P, psi, ORC_W, k, j);
    if (i >= P->nx) return ghost(P, psi, ORC_E, k, j);
    return PSI(P, psi, k, j, i);
}

static double cell_y(const orc_problem *P, const double *psi, int k, int j, int i)
{
    if (j < 0) return ghost(P, psi, ORC_S, k, i);
    if (j >= P->ny) return ghost(P, psi, ORC_N, k, i);
    return PSI(P, psi, k, j, i);
}

/* Venkatakrishnan-limited reconstruction (Sec. 4.2, eq. eq_V_limiter) of
 * ordinate k in cell (i, j) at the midpoint of one of its faces: dir 0 for an
 * x-face, 1 for a y-face; sgn +1 for the face on the cell's + side.
 *   gradient  g = (1/A) sum_faces l n (psi_i + psi_j)/2; on a square cell of
 *             side h the cell's own value cancels: g = ((E - W), (N - S)) / (2h)
 *   face      R = psi_i + L g . r, r from the cell centre to the face midpoint
 *             (|r| = h/2), so g . r = +-(E - W)/4 or +-(N - S)/4
 *   limiter   L = min over the four faces of
 *             ((b^2 + e^2) + 2 D b) / (b^2 + 2 D^2 + b D + e^2), and 1 where D = 0,
 *             with D = g . r of that face (reading: the increment g . r; the
 *             printed factor 1/2 would let face values leave the
 *             neighbourhood's range), b = max - psi_i for D > 0 and
 *             min - psi_i for D < 0 over the cell and its four neighbours,
 *             e = K A^3 with K = 1, A = h^2.
 * Neighbours outside the grid are ghost cells holding the side's ghost value
 * for every ordinate. */
static double venkat(const orc_problem *P, const double *psi, int k, int j, int i, int dir, int sgn)
{
    double c = PSI(P, psi, k, j, i);
    double W = cell_x(P, psi, k, j, i - 1), E = cell_x(P, psi, k, j, i + 1);
    double S = cell_y(P, psi, k, j - 1, i), N = cell_y(P, psi, k, j + 1, i);
    double ax = 0.25 * (E - W), ay = 0.25 * (N - S);
    double mx = c, mn = c, bM, bm, e, e2, L = HUGE_VAL, D[4];
    int f;
    if (W > mx) mx = W;
    if (E > mx) mx = E;
    if (S > mx) mx = S;
    if (N > mx) mx = N;
    if (W < mn) mn = W;
    if (E < mn) mn = E;
    if (S < mn) mn = S;
    if (N < mn) mn = N;
    bM = mx - c;
    bm = mn - c;
    e = P->h * P->h * P->h * P->h * P->h * P->h;
    e2 = e * e;
    D[0] = ax;
    D[1] = -ax;
    D[2] = ay;
    D[3] = -ay;
    for (f = 0; f < 4; ++f) {
        double d = D[f], b, v;
        if (d == 0.0) {
            v = 1.0;
        } else {
            b = d > 0.0 ? bM : bm;
            v = (b * b + e2 + 2.0 * d * b) / (b * b + 2.0 * d * d + b * d + e2);
        }
        if (v < L) L = v; /* may exceed 1: the factor peaks near 1.094 */
    }
    return c + sgn * L * (dir == 0 ? ax : ay);
}

/* Upwind numerical trace on the x-face f (between cells f-1 and f) of row j,
 * f = 0..nx (eq. eq_upwind1stOrder). Boundary faces take the ghost for
 * incoming ordinates and the boundary cell value for outgoing ones (first
 * order). Interior faces take the reconstruction of the upwind cell u at the
 * face: psi_u for order 1; psi_u +- 1/2 minmod(psi_u - psi_{u-1},
 * psi_{u+1} - psi_u) for order 2, "+" when the face is the cell's right face;
 * the Venkatakrishnan-limited reconstruction (venkat) for order 3;
 * a neighbour outside the grid is the ghost value. */
double orc_face_x(const orc_problem *P, const double *psi, int k, int f, int j)
{
    double xi = P->xi[k];
    if (f == 0) return xi > 0.0 ? ghost(P, psi, ORC_W, k, j) : PSI(P, psi, k, j, 0);
    if (f == P->nx) return xi < 0.0 ? ghost(P, psi, ORC_E, k, j) : PSI(P, psi, k, j, P->nx - 1);
    {
        int u = xi > 0.0 ? f - 1 : f;
        double pu = PSI(P, psi, k, j, u);
        double slope;
        if (P->order == 1) return pu;
        if (P->order == 3) return venkat(P, psi, k, j, u, 0, xi > 0.0 ? 1 : -1);
        slope = minmod(pu - cell_x(P, psi, k, j, u - 1), cell_x(P, psi, k, j, u + 1) - pu);
        return xi > 0.0 ? pu + 0.5 * slope : pu - 0.5 * slope;
    }
}

/* The same for the y-face f (between rows f-1 and f) of column i. */
double orc_face_y(const orc_problem *P, const double *psi, int k, int i, int f)
{
    double eta = P->eta[k];
    if (f == 0) return eta > 0.0 ? ghost(P, psi, ORC_S, k, i) : PSI(P, psi, k, 0, i);
    if (f == P->ny) return eta < 0.0 ? ghost(P, psi, ORC_N, k, i) : PSI(P, psi, k, P->ny - 1, i);
    {
        int u = eta > 0.0 ? f - 1 : f;
        double pu = PSI(P, psi, k, u, i);
        double slope;
        if (P->order == 1) return pu;
        if (P->order == 3) return venkat(P, psi, k, u, i, 1, eta > 0.0 ? 1 : -1);
        slope = minmod(pu - cell_y(P, psi, k, u - 1, i), cell_y(P, psi, k, u + 1, i) - pu);
        return eta > 0.0 ? pu + 0.5 * slope : pu - 0.5 * slope;
    }
}

/* F(psi) of eq. eq_ODE: for every ordinate k and cell (i, j),
 *   F = -(xi_k/h)(trace_{i+1/2} - trace_{i-1/2}) - (eta_k/h)(trace_{j+1/2} - trace_{j-1/2})
 *       - sigma_t psi_k + sigma_s/(2 pi) phi + Q,     sigma_t = sigma_a + sigma_s.
 * phi must hold the scalar flux of psi. */
void orc_rhs(const orc_problem *P, const double *psi, const double *phi, double *F)
{
    int k;
#pragma omp parallel for schedule(dynamic, 1)
    for (k = 0; k < P->M; ++k) {
        int i, j;
        for (j = 0; j < P->ny; ++j) {
            for (i = 0; i < P->nx; ++i) {
                int r = P->region[j * P->nx + i];
                double sa = P->sigma_a[r], ss = P->sigma_s[r], q = P->q[r];
                double st = sa + ss;
                double p = PSI(P, psi, k, j, i);
                double dx = orc_face_x(P, psi, k, i + 1, j) - orc_face_x(P, psi, k, i, j);
                double dy = orc_face_y(P, psi, k, i, j + 1) - orc_face_y(P, psi, k, i, j);
                F[((size_t)k * P->ny + j) * P->nx + i] =
                    -(P->xi[k] / P->h) * dx - (P->eta[k] / P->h) * dy - st * p
                    + ss / TWO_PI * phi[j * P->nx + i] + q;
            }
        }
    }
}

/* Number of entries in a QoI vector:
 *   [0] mass = int_D phi                                   (QoI-5)
 *   [1] source emission = (sum_k w_k) int_D Q
 *   [2 .. 2+T) absorption int_{tally t} sigma_a phi         (QoI-3)
 *   [2+T .. 2+T+R) outflow  through the boundary of rect r   (QoI-1)
 *   [2+T+R .. 2+T+2R) inflow through the boundary of rect r */
int orc_qoi_len(const orc_problem *P) { return 2 + P->n_tallies + 2 * P->n_rects; }

static void add_face(double wn, double trace, double len, double *out, double *in)
{
    /* wn = w_k (Omega_k . n) for the outward normal n */
    if (wn > 0.0) *out += wn * trace * len;
    else if (wn < 0.0) *in += -wn * trace * len;
}

/* Instantaneous QoIs of the state psi (phi = its scalar flux), in FP64 with
 * sequential sums. Outflow/inflow use the scheme's numerical trace on the
 * faces of the rectangle, split by the sign of Omega_k . n (Sec. 3.1.2). */
void orc_qoi(const orc_problem *P, const double *psi, const double *phi, double *qv)
{
    int T = P->n_tallies, R = P->n_rects;
    int i, j, k, r, t;
    double h2 = P->h * P->h, sw = 0.0;
    for (t = 0; t < orc_qoi_len(P); ++t) qv[t] = 0.0;
    for (k = 0; k < P->M; ++k) sw += P->w[k];
    for (j = 0; j < P->ny; ++j) {
        for (i = 0; i < P->nx; ++i) {
            int reg = P->region[j * P->nx + i];
            double ph = phi[j * P->nx + i];
            qv[0] += h2 * ph;
            qv[1] += sw * h2 * P->q[reg];
            qv[2 + P->tally[reg]] += h2 * P->sigma_a[reg] * ph;
        }
    }
    for (r = 0; r < R; ++r) {
        int i0 = P->rects[4 * r], j0 = P->rects[4 * r + 1];
        int i1 = P->rects[4 * r + 2], j1 = P->rects[4 * r + 3];
        double *out = &qv[2 + T + r], *in = &qv[2 + T + R + r];
        for (k = 0; k < P->M; ++k) {
            double w = P->w[k], xi = P->xi[k], eta = P->eta[k];
            for (j = j0; j < j1; ++j) {
                add_face(-w * xi, orc_face_x(P, psi, k, i0, j), P->h, out, in); /* west, n = -x */
                add_face(w * xi, orc_face_x(P, psi, k, i1, j), P->h, out, in);  /* east, n = +x */
            }
            for (i = i0; i < i1; ++i) {
                add_face(-w * eta, orc_face_y(P, psi, k, i, j0), P->h, out, in); /* south */
                add_face(w * eta, orc_face_y(P, psi, k, i, j1), P->h, out, in);  /* north */
            }
        }
    }
}

/* Advance psi by n_steps time steps (Sec. 4.3):
 *   Euler: psi <- psi + dt F(psi)
 *   Heun:  psi1 = psi + dt F(psi); psi2 = psi1 + dt F(psi1); psi <- (psi + psi2) / 2.
 * qint accumulates the time integral of the QoI vector with the rule that
 * matches the stepper: Euler dt q(psi^n); Heun dt/2 (q(psi^n) + q(psi1)).
 * fluence (NULL to skip) accumulates the time integral of phi per cell,
 * [ny][nx], with the same rule; the Hohlraum QoI-3 to QoI-6 (Sec. 3.2.2)
 * integrate sigma_a times it over blocks and a line.
 * Returns 0, or -1 if memory could not be allocated. */
static void add_fluence(const orc_problem *P, double coef, const double *phi, double *fluence)
{
    size_t c, ncell = (size_t)P->nx * P->ny;
    if (!fluence) return;
    for (c = 0; c < ncell; ++c) fluence[c] += coef * phi[c];
}

/* Space-time probes (Hohlraum QoI-1, Sec. 3.2.2): probe p averages phi,
 * J_x = sum_l w_l xi_l psi_l and J_y = sum_l w_l eta_l psi_l over its cells
 * with the given weights (area of the cell inside the probe's ball over the
 * ball's area) and over each of n_windows equal time windows of [0, T]. A
 * step's contributions (the same time rule as the integrated QoIs) fall in the
 * window that holds the step's start time: window floor(step n_windows / N_t). */
typedef struct {
    int n_probes, n_windows, n_cells;
    const int *cell_i, *cell_j, *probe; /* [n_cells] */
    const double *weight;               /* [n_cells] */
} orc_probes;

static void add_probes(const orc_problem *P, const orc_probes *pr, int step, int nt, double coef,
                       const double *psi, double *pacc)
{
    int c, k, w;
    double win;
    if (!pr || !pacc || pr->n_probes <= 0) return;
    w = (int)(((long long)step * pr->n_windows) / nt);
    if (w >= pr->n_windows) return;
    win = P->t_end / pr->n_windows; /* the window's length: the average's time measure */
    for (c = 0; c < pr->n_cells; ++c) {
        double m0 = 0.0, mx = 0.0, my = 0.0;
        double *a = &pacc[((size_t)w * pr->n_probes + pr->probe[c]) * 3];
        for (k = 0; k < P->M; ++k) {
            double v = PSI(P, psi, k, pr->cell_j[c], pr->cell_i[c]);
            m0 += P->w[k] * v;
            mx += P->w[k] * P->xi[k] * v;
            my += P->w[k] * P->eta[k] * v;
        }
        a[0] += coef / win * pr->weight[c] * m0;
        a[1] += coef / win * pr->weight[c] * mx;
        a[2] += coef / win * pr->weight[c] * my;
    }
}

int orc_advance(const orc_problem *P, int n_steps, double *psi, double *qint, double *fluence,
                const orc_probes *probes, int step0, double *pacc)
{
    size_t n = (size_t)P->M * P->nx * P->ny;
    size_t ncell = (size_t)P->nx * P->ny;
    int L = orc_qoi_len(P);
    double dt;
    int nt;
    double *F = malloc(n * sizeof(double));
    double *psi1 = P->stepper == 1 ? malloc(n * sizeof(double)) : NULL;
    double *phi = malloc(ncell * sizeof(double));
    double *qv = malloc((size_t)L * sizeof(double));
    int s, t;
    long long e;
    nt = orc_num_steps(P, &dt);
    if (!F || !phi || !qv || (P->stepper == 1 && !psi1)) {
        free(F); free(psi1); free(phi); free(qv);
        return -1;
    }
    for (s = 0; s < n_steps; ++s) {
        orc_scalar_flux(P, psi, phi);
        orc_qoi(P, psi, phi, qv);
        orc_rhs(P, psi, phi, F);
        if (P->stepper == 0) {
            for (t = 0; t < L; ++t) qint[t] += dt * qv[t];
            add_fluence(P, dt, phi, fluence);
            add_probes(P, probes, step0 + s, nt, dt, psi, pacc);
#pragma omp parallel for
            for (e = 0; e < (long long)n; ++e) psi[e] = psi[e] + dt * F[e];
        } else {
            for (t = 0; t < L; ++t) qint[t] += 0.5 * dt * qv[t];
            add_fluence(P, 0.5 * dt, phi, fluence);
            add_probes(P, probes, step0 + s, nt, 0.5 * dt, psi, pacc);
#pragma omp parallel for
            for (e = 0; e < (long long)n; ++e) psi1[e] = psi[e] + dt * F[e];
            orc_scalar_flux(P, psi1, phi);
            orc_qoi(P, psi1, phi, qv);
            orc_rhs(P, psi1, phi, F);
            for (t = 0; t < L; ++t) qint[t] += 0.5 * dt * qv[t];
            add_fluence(P, 0.5 * dt, phi, fluence);
            add_probes(P, probes, step0 + s, nt, 0.5 * dt, psi1, pacc);
#pragma omp parallel for
            for (e = 0; e < (long long)n; ++e) {
                double psi2 = psi1[e] + dt * F[e];
                psi[e] = 0.5 * (psi[e] + psi2);
            }
        }
    }
    free(F); free(psi1); free(phi); free(qv);
    return 0;
}
