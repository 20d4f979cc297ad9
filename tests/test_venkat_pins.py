"""Pins of the oracle's order-3 reconstruction: the Green-Gauss gradient with
the Venkatakrishnan limiter (Sec. 4.2, eq. eq_V_limiter).

Against a face-by-face Python evaluation written from the paper's vector
form (tests/bruteforce.py); against what the limiter is for: linear data is
reconstructed exactly, face values stay inside the range of the cell and its
neighbours, a local extremum falls back to its cell value; and the scheme's
conservation, symmetry and accuracy on the beam.
"""

import numpy as np
import pytest

from paper_2505_17284_amd import inputs as I
from tests import bruteforce as BF


@pytest.mark.parametrize("shape", [(3, 3), (4, 5), (6, 4)])
@pytest.mark.parametrize("bcs", [0, 1, 2])
def test_matches_facewise_python(orc, shape, bcs):
    b = [(I.BC_VACUUM,) * 4, (I.BC_INFLOW, I.BC_REFLECT, I.BC_REFLECT, I.BC_INFLOW),
         (I.BC_REFLECT, I.BC_INFLOW, I.BC_VACUUM, I.BC_REFLECT)][bcs]
    nx, ny = shape
    p = I.random_materials(nx, ny, 3, seed=bcs, order=3, bc=b, inflow=(0.9, 0.4, 0.6, 0.2))
    for s, kind in ((0, "uniform"), (1, "smooth")):
        psi = I.random_state(p, 40 + s, kind)
        np.testing.assert_allclose(orc.rhs(p, psi), BF.rhs_venkat(p, psi), rtol=1e-12, atol=1e-12)


def test_linear_data_reconstructed_exactly(orc):
    """On 2-D linear data the face along the steepest direction has
    b / D = 2, where the limiter's factor is exactly 1, and no face's factor
    is below 1: L = 1, the face value is the linear function's."""
    p = I.random_materials(9, 8, 1, seed=0, order=3)
    a, bx, by = 2.0, 0.3, -0.2
    jj, ii = np.meshgrid(np.arange(p.ny), np.arange(p.nx), indexing="ij")
    psi = np.broadcast_to(a + bx * ii + by * jj, (p.M, p.ny, p.nx)).copy()
    for k in (0, 5, 13, 27):
        for j in range(1, p.ny - 1):
            for f in range(2, p.nx - 1):
                assert orc.face_x(p, psi, k, f, j) == pytest.approx(a + bx * (f - 0.5) + by * j, abs=1e-13)
        for i in range(1, p.nx - 1):
            for f in range(2, p.ny - 1):
                assert orc.face_y(p, psi, k, i, f) == pytest.approx(a + bx * i + by * (f - 0.5), abs=1e-13)


def test_face_values_stay_in_the_neighbourhood_range(orc):
    """For random data every interior face value lies between the minimum and
    the maximum of its upwind cell and that cell's four neighbours."""
    p = I.random_materials(9, 7, 1, seed=2, order=3)
    rng = np.random.Generator(np.random.PCG64(3))
    psi = rng.uniform(-1.0, 2.0, (p.M, p.ny, p.nx))
    for k in range(0, p.M, 3):
        xi, eta = p.quad.xi[k], p.quad.eta[k]
        for j in range(1, p.ny - 1):
            for f in range(2, p.nx - 1):
                u = f - 1 if xi > 0 else f
                nb = psi[k, j, u - 1:u + 2].tolist() + [psi[k, j - 1, u], psi[k, j + 1, u]]
                v = orc.face_x(p, psi, k, f, j)
                assert min(nb) - 1e-14 <= v <= max(nb) + 1e-14
        for i in range(1, p.nx - 1):
            for f in range(2, p.ny - 1):
                u = f - 1 if eta > 0 else f
                nb = psi[k, u - 1:u + 2, i].tolist() + [psi[k, u, i - 1], psi[k, u, i + 1]]
                v = orc.face_y(p, psi, k, i, f)
                assert min(nb) - 1e-14 <= v <= max(nb) + 1e-14


def test_extremum_falls_back_to_first_order(orc):
    p = I.random_materials(7, 7, 1, seed=1, order=3)
    psi = np.ones((p.M, p.ny, p.nx))
    psi[:, 3, 3] = 5.0  # strict local maximum
    psi[:, 3, 4] = 2.0  # a non-zero gradient at the peak
    for k in range(p.M):
        fe = 4 if p.quad.xi[k] > 0 else 3   # the peak's downwind x-face
        fn = 4 if p.quad.eta[k] > 0 else 3  # its downwind y-face
        assert orc.face_x(p, psi, k, fe, 3) == pytest.approx(5.0, abs=1e-12)
        assert orc.face_y(p, psi, k, 3, fn) == pytest.approx(5.0, abs=1e-12)


@pytest.mark.parametrize("stepper", [I.EULER, I.HEUN])
def test_particle_balance(orc, stepper):
    bcs = (I.BC_INFLOW, I.BC_REFLECT, I.BC_VACUUM, I.BC_INFLOW)
    p = I.random_materials(11, 9, 4, seed=5, order=3, stepper=stepper, bc=bcs, inflow=(0.8, 0, 0, 0.3))
    r = orc.solve(p, steps=12, psi0=I.random_state(p, 6))
    q = dict(zip(r["names"], r["qoi"]))
    qi = dict(zip(r["names"], r["qoi_int"]))
    q0 = dict(zip(r["names"], orc.qoi(p, I.random_state(p, 6))))
    gain = qi["source"] + qi["in:r0"] - qi["out:r0"] - sum(qi[f"abs:t{t}"] for t in range(3))
    assert q["mass"] == pytest.approx(q0["mass"] + gain, rel=1e-12, abs=1e-12)


def test_symmetric_lattice_stays_symmetric(orc):
    p = I.lattice(28, 32, order=3, stepper=I.HEUN, d4=True, t_end=0.6)
    r = orc.solve(p)
    phi = r["phi"]
    for a, b in ((phi, phi[:, ::-1]), (phi, phi[::-1, :]), (phi, phi.T)):
        np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-13 * phi.max())


def test_beam_more_accurate_than_first_order(orc):
    """Against the continuum cell average of the beam, the limited scheme at
    h beats first order at h/2."""
    sigma, g, L = 1.0, 1.0, 1.0

    def err(nx, order):
        h = L / nx
        p = I.beam(nx=nx, ny=3, M=32, sigma=sigma, g=g, h=h, order=order, stepper=I.HEUN, t_end=4.0)
        r = orc.solve(p)
        i = np.arange(nx)
        e = 0.0
        for k in range(p.M):
            xi = p.quad.xi[k]
            if xi <= 0:
                continue
            exact = (xi / (sigma * h)) * (np.exp(-sigma * i * h / xi) - np.exp(-sigma * (i + 1) * h / xi))
            e += p.quad.w[k] * np.sum(np.abs(r["psi"][k, 1] - exact)) * h
        return e

    assert err(20, 3) < err(40, 1)
