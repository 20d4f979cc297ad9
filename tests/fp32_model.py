"""A dtype-generic NumPy model of the S_N stage, used to measure what FP32
arithmetic alone does to the scheme's results.

It is neither the oracle nor the GPU path: it evaluates the same cell balance
(arXiv 2505.17284, Sec. 4.2, eqs. eq_sn_2d_eqn_fv / eq_upwind1stOrder, minmod
reconstruction, ghost values at the boundary) and Heun's method (Sec. 4.3) in
a chosen float width, with the per-cell coefficients dt sigma_t, dt sigma_s /
(2 pi), dt Q computed in FP64 and rounded once. Run in float64 it must agree
with the oracle to rounding; run in float32 it shows how far an FP32 state
can drift from the FP64 result, which sets the field tolerances of the GPU
parity tests for long runs.
"""

import numpy as np


def _mm(a, b, zero):
    return np.maximum(np.minimum(a, b), zero) + np.minimum(np.maximum(a, b), zero)


def _ghost_value(p, P, side, k):
    kind = p.bc[side]
    if kind == 1:
        return p.inflow[side]
    if kind == 2:
        m = p.quad.mirror_x[k] if side < 2 else p.quad.mirror_y[k]
        nx, ny = p.nx, p.ny
        return {0: P[m][2:-2, 2], 1: P[m][2:-2, nx + 1], 2: P[m][2, 2:-2], 3: P[m][ny + 1, 2:-2]}[side]
    return 0.0


def fill_frame(p, P):
    """Ghost frame: entering ordinates see the side's ghost value in both
    layers, leaving ordinates a copy of the boundary cell."""
    nx, ny = p.nx, p.ny
    for k in range(p.M):
        xi, eta = p.quad.xi[k], p.quad.eta[k]
        if xi > 0:
            P[k][2:-2, 0] = P[k][2:-2, 1] = _ghost_value(p, P, 0, k)
            P[k][2:-2, nx + 2] = P[k][2:-2, nx + 1]
        else:
            P[k][2:-2, 1] = P[k][2:-2, 2]
            P[k][2:-2, nx + 2] = P[k][2:-2, nx + 3] = _ghost_value(p, P, 1, k)
        if eta > 0:
            P[k][0, 2:-2] = P[k][1, 2:-2] = _ghost_value(p, P, 2, k)
            P[k][ny + 2, 2:-2] = P[k][ny + 1, 2:-2]
        else:
            P[k][1, 2:-2] = P[k][2, 2:-2]
            P[k][ny + 2, 2:-2] = P[k][ny + 3, 2:-2] = _ghost_value(p, P, 3, k)


def stage(p, P, dt, dtype, old=None):
    f = dtype
    zero, half = f(0), f(0.5)
    h = p.h
    psi = P[:, 2:-2, 2:-2]
    phi = np.zeros((p.ny, p.nx), f)
    for k in range(p.M):
        phi = phi + f(p.quad.w[k]) * psi[k]
    st = (dt * (p.sigma_a + p.sigma_s))[p.region].astype(f)
    cs = (dt * p.sigma_s / (2 * np.pi))[p.region].astype(f)
    cq = (dt * p.q)[p.region].astype(f)
    bb = cs * phi + cq
    out = np.zeros_like(P)
    for k in range(p.M):
        xi, eta = p.quad.xi[k], p.quad.eta[k]
        A = P[k]
        row = A[2:-2]
        c, L, R = row[:, 1:-1], row[:, :-2], row[:, 2:]
        m = _mm(c - L, R - c, zero) if p.order == 2 else zero * c
        Rx = c + (half if xi > 0 else -half) * m
        dRx = Rx[:, 1:-1] - Rx[:, :-2] if xi > 0 else Rx[:, 2:] - Rx[:, 1:-1]
        col = A[:, 2:-2]
        c, L, R = col[1:-1], col[:-2], col[2:]
        m = _mm(c - L, R - c, zero) if p.order == 2 else zero * c
        Ry = c + (half if eta > 0 else -half) * m
        dRy = Ry[1:-1] - Ry[:-2] if eta > 0 else Ry[2:] - Ry[1:-1]
        d = bb - st * psi[k] - f(dt * xi / h) * dRx - f(dt * eta / h) * dRy
        v = psi[k] + d
        if old is not None:
            v = half * (old[k, 2:-2, 2:-2] + v)
        out[k, 2:-2, 2:-2] = v
    fill_frame(p, out)
    return out


def run(p, steps, dt, dtype):
    """Heun steps from psi = 0; returns psi [M][ny][nx] as float64."""
    P = np.zeros((p.M, p.ny + 4, p.nx + 4), dtype)
    fill_frame(p, P)
    for _ in range(steps):
        P1 = stage(p, P, dt, dtype)
        P = stage(p, P1, dt, dtype, old=P)
    return P[:, 2:-2, 2:-2].astype(np.float64)
