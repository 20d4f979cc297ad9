"""Brute-force forms of the S_N finite-volume operator for tiny grids.

These are independent of the oracle's loops: the first-order operator is
assembled face by face in conservative form (each face's flux leaves one cell
and enters the other) as a dense matrix, and the second-order operators
(minmod; the Venkatakrishnan-limited gradient, as vectors) are evaluated face
by face in Python on a ghost-padded array. All follow the cell balance with
the upwind trace of arXiv 2505.17284 Sec. 4.2 (eqs. eq_sn_2d_eqn_fv,
eq_upwind1stOrder, eq_V_limiter) on square cells.
"""

import numpy as np

VAC, INF, REF = 0, 1, 2


def _idx(p, k, j, i):
    return (k * p.ny + j) * p.nx + i


def dense_first_order(p):
    """(A, b) with F(psi) = A psi + b for order 1, psi flattened [M][ny][nx]."""
    M, nx, ny, h = p.M, p.nx, p.ny, p.h
    N = M * nx * ny
    A = np.zeros((N, N))
    b = np.zeros(N)
    xi, eta, w = p.quad.xi, p.quad.eta, p.quad.w
    sa = p.sigma_a[p.region]
    ss = p.sigma_s[p.region]
    q = p.q[p.region]
    inv_area = 1.0 / (h * h)

    def add_flux(k, wn, src_cell, dst_cell, value_row, value_const):
        """A flux wn * h * value leaves src_cell (if any) and enters dst_cell (if any).
        value = value_row . psi + value_const."""
        for cell, sign in ((src_cell, -1.0), (dst_cell, +1.0)):
            if cell is None:
                continue
            r = _idx(p, k, *cell)
            for col, coef in value_row:
                A[r, col] += sign * wn * h * coef * inv_area
            b[r] += sign * wn * h * value_const * inv_area

    def ghost(side, k, j, i):
        """(row entries, constant) of the ghost value behind boundary cell (i, j)."""
        kind = p.bc[side]
        if kind == INF:
            return [], p.inflow[side]
        if kind == REF:
            m = p.quad.mirror_x[k] if side in (0, 1) else p.quad.mirror_y[k]
            return [(_idx(p, m, j, i), 1.0)], 0.0
        return [], 0.0

    for k in range(M):
        # x-faces: face f between cells f-1 and f, normal +x (from f-1 into f)
        for j in range(ny):
            for f in range(nx + 1):
                L = (j, f - 1) if f >= 1 else None
                R = (j, f) if f < nx else None
                wn = xi[k]  # Omega . (+x)
                if wn > 0:  # upwind = left
                    row, const = ([(_idx(p, k, j, f - 1), 1.0)], 0.0) if L else ghost(0, k, j, 0)
                else:
                    row, const = ([(_idx(p, k, j, f), 1.0)], 0.0) if R else ghost(1, k, j, nx - 1)
                add_flux(k, wn, L, R, row, const)
        # y-faces: face f between rows f-1 and f, normal +y
        for i in range(nx):
            for f in range(ny + 1):
                L = (f - 1, i) if f >= 1 else None
                R = (f, i) if f < ny else None
                wn = eta[k]
                if wn > 0:
                    row, const = ([(_idx(p, k, f - 1, i), 1.0)], 0.0) if L else ghost(2, k, 0, i)
                else:
                    row, const = ([(_idx(p, k, f, i), 1.0)], 0.0) if R else ghost(3, k, ny - 1, i)
                add_flux(k, wn, L, R, row, const)
        # collision, isotropic scattering, source
        for j in range(ny):
            for i in range(nx):
                r = _idx(p, k, j, i)
                A[r, r] -= sa[j, i] + ss[j, i]
                for l in range(M):
                    A[r, _idx(p, l, j, i)] += ss[j, i] / (2 * np.pi) * w[l]
                b[r] += q[j, i]
    return A, b


def _padded(p, psi, k):
    """Ordinate k of psi with one ghost layer on every side (corners unused)."""
    nx, ny = p.nx, p.ny
    g = np.zeros((ny + 2, nx + 2))
    g[1:-1, 1:-1] = psi[k]
    mx, my = p.quad.mirror_x[k], p.quad.mirror_y[k]
    sides = {
        0: (np.s_[1:-1, 0], lambda: psi[mx][:, 0]),
        1: (np.s_[1:-1, -1], lambda: psi[mx][:, nx - 1]),
        2: (np.s_[0, 1:-1], lambda: psi[my][0, :]),
        3: (np.s_[-1, 1:-1], lambda: psi[my][ny - 1, :]),
    }
    for side, (sl, refl) in sides.items():
        kind = p.bc[side]
        if kind == INF:
            g[sl] = p.inflow[side]
        elif kind == REF:
            g[sl] = refl()
    return g


def _minmod(a, b):
    if a * b <= 0:
        return 0.0
    return a if abs(a) < abs(b) else b


def rhs_second_order(p, psi):
    """F(psi) for order 2, face by face, on ghost-padded ordinates."""
    M, nx, ny, h = p.M, p.nx, p.ny, p.h
    psi = np.asarray(psi).reshape(M, ny, nx)
    phi = np.einsum("k,kji->ji", p.quad.w, psi)
    F = np.zeros_like(psi)
    sa = p.sigma_a[p.region]
    ss = p.sigma_s[p.region]
    q = p.q[p.region]
    for k in range(M):
        g = _padded(p, psi, k)  # g[j+1, i+1] = cell (i, j)
        xi, eta = p.quad.xi[k], p.quad.eta[k]
        fx = np.zeros((ny, nx + 1))
        fy = np.zeros((ny + 1, nx))
        for j in range(ny):
            row = g[j + 1]  # row[i+1] = cell i, row[0] / row[nx+1] ghosts
            for f in range(nx + 1):
                if f == 0 or f == nx:  # boundary faces: first order
                    fx[j, f] = row[f] if xi > 0 else row[f + 1]
                    continue
                if xi > 0:
                    c = f  # padded index of the upwind cell f-1
                    fx[j, f] = row[c] + 0.5 * _minmod(row[c] - row[c - 1], row[c + 1] - row[c])
                else:
                    c = f + 1  # padded index of the upwind cell f
                    fx[j, f] = row[c] - 0.5 * _minmod(row[c] - row[c - 1], row[c + 1] - row[c])
        for i in range(nx):
            col = g[:, i + 1]
            for f in range(ny + 1):
                if f == 0 or f == ny:
                    fy[f, i] = col[f] if eta > 0 else col[f + 1]
                    continue
                if eta > 0:
                    c = f
                    fy[f, i] = col[c] + 0.5 * _minmod(col[c] - col[c - 1], col[c + 1] - col[c])
                else:
                    c = f + 1
                    fy[f, i] = col[c] - 0.5 * _minmod(col[c] - col[c - 1], col[c + 1] - col[c])
        div = xi * (fx[:, 1:] - fx[:, :-1]) / h + eta * (fy[1:, :] - fy[:-1, :]) / h
        F[k] = -div - (sa + ss) * psi[k] + ss / (2 * np.pi) * phi + q
    return F


def rhs_venkat(p, psi):
    """F(psi) for order 3 (Venkatakrishnan-limited Green-Gauss reconstruction,
    Sec. 4.2), face by face on ghost-padded ordinates: every interior face
    takes the upwind cell's limited linear reconstruction at the face
    midpoint, boundary faces are first order."""
    M, nx, ny, h = p.M, p.nx, p.ny, p.h
    psi = np.asarray(psi).reshape(M, ny, nx)
    phi = np.einsum("k,kji->ji", p.quad.w, psi)
    F = np.zeros_like(psi)
    sa = p.sigma_a[p.region]
    ss = p.sigma_s[p.region]
    q = p.q[p.region]
    eps2 = (h ** 2) ** 6  # (K A^3)^2 with K = 1, A = h^2

    def limited(g, jp, ip, normal):
        """Face value of padded cell (jp, ip) at its face with outward unit normal."""
        c = g[jp, ip]
        nb = [g[jp, ip - 1], g[jp, ip + 1], g[jp - 1, ip], g[jp + 1, ip]]  # W E S N
        grad = np.array([(nb[1] - nb[0]) / (2 * h), (nb[3] - nb[2]) / (2 * h)])
        lo, hi = min([c] + nb), max([c] + nb)
        factors = []
        for n in ((-1, 0), (1, 0), (0, -1), (0, 1)):
            d = grad @ (np.array(n) * h / 2)  # increment to that face's midpoint
            if d > 0:
                b = hi - c
            elif d < 0:
                b = lo - c
            else:
                factors.append(1.0)
                continue
            factors.append(((b * b + eps2) * d + 2 * d * d * b) / d / (b * b + 2 * d * d + b * d + eps2))
        return c + min(factors) * (grad @ (np.array(normal) * h / 2))

    for k in range(M):
        g = _padded(p, psi, k)
        xi, eta = p.quad.xi[k], p.quad.eta[k]
        fx = np.zeros((ny, nx + 1))
        fy = np.zeros((ny + 1, nx))
        for j in range(ny):
            for f in range(nx + 1):
                if f == 0 or f == nx:
                    fx[j, f] = g[j + 1, f] if xi > 0 else g[j + 1, f + 1]
                elif xi > 0:
                    fx[j, f] = limited(g, j + 1, f, (1, 0))  # cell f-1, its east face
                else:
                    fx[j, f] = limited(g, j + 1, f + 1, (-1, 0))  # cell f, its west face
        for i in range(nx):
            for f in range(ny + 1):
                if f == 0 or f == ny:
                    fy[f, i] = g[f, i + 1] if eta > 0 else g[f + 1, i + 1]
                elif eta > 0:
                    fy[f, i] = limited(g, f, i + 1, (0, 1))
                else:
                    fy[f, i] = limited(g, f + 1, i + 1, (0, -1))
        div = xi * (fx[:, 1:] - fx[:, :-1]) / h + eta * (fy[1:, :] - fy[:-1, :]) / h
        F[k] = -div - (sa + ss) * psi[k] + ss / (2 * np.pi) * phi + q
    return F
