"""Pins of the oracle's space-time probes (Hohlraum QoI-1, Sec. 3.2.2).

The probe weights are pinned by closed-form areas of a disc cut by the grid;
the window averages by the homogeneous medium under Euler (phi in closed
form, zero currents), by the steady beam (J_x in closed form, J_y zero by the
reflective symmetry), by the pinned fluence (the windows of phi add up to the
ball's share of it), and by splitting a run across calls.
"""

import math

import numpy as np
import pytest

from paper_2505_17284_amd import inputs as I


@pytest.fixture(scope="module")
def hq():
    from oracle import hohlraum_qoi
    return hohlraum_qoi


def test_disc_areas_closed_form(hq):
    h = 0.3
    r = 2 * h
    # disc centred on a grid vertex with r = 2h: the cell at the centre is
    # inside (far corner at h sqrt 2), the side cell [h, 2h] x [0, h] holds
    # (sqrt3/2 - 1 + pi/3) h^2, the corner cell (pi/3 + 1 - sqrt3) h^2
    assert hq.disc_cell_area(0, 0, r, 0, h, 0, h) == pytest.approx(h * h, rel=1e-12)
    assert hq.disc_cell_area(0, 0, r, h, 2 * h, 0, h) == pytest.approx(
        (math.sqrt(3) / 2 - 1 + math.pi / 3) * h * h, rel=1e-11)
    assert hq.disc_cell_area(0, 0, r, h, 2 * h, h, 2 * h) == pytest.approx(
        (math.pi / 3 + 1 - math.sqrt(3)) * h * h, rel=1e-11)
    assert hq.disc_cell_area(0, 0, r, -3 * h, 3 * h, -3 * h, 3 * h) == pytest.approx(math.pi * r * r, rel=1e-12)
    assert hq.disc_cell_area(0, 0, r, 2 * h, 3 * h, 0, h) == 0.0
    # a small disc inside one cell
    assert hq.disc_cell_area(0.11, 0.12, 0.01, 0.0, 0.3, 0.0, 0.3) == pytest.approx(math.pi * 1e-4, rel=1e-12)


@pytest.mark.parametrize("n", [104, 260, 333])
def test_hohlraum_probe_weights(hq, n):
    p = I.hohlraum(n=n, M=32)
    pc = hq.probe_cells(p)
    assert pc["n_probes"] == 4 and pc["n_windows"] == 10
    for q in range(4):
        w = pc["weight"][pc["probe"] == q]
        assert w.sum() == pytest.approx(1.0, rel=1e-12)  # each ball lies inside the domain
        assert np.all(w > 0) and np.all(w <= (p.h ** 2) / (math.pi * 1e-4) * (1 + 1e-12))
    if n == 260:  # every centre is a grid vertex and r = 2h: 16 cells, three kinds
        for q in range(4):
            w = np.sort(pc["weight"][pc["probe"] == q])
            assert len(w) == 16
            unit = 1.0 / (4 * math.pi)
            np.testing.assert_allclose(w[:4], (math.pi / 3 + 1 - math.sqrt(3)) * unit, rtol=1e-10)
            np.testing.assert_allclose(w[4:12], (math.sqrt(3) / 2 - 1 + math.pi / 3) * unit, rtol=1e-10)
            np.testing.assert_allclose(w[12:], unit, rtol=1e-10)


def _probes_at(p, hq, centres, r, n_windows):
    return hq.probe_cells(p, centres=centres, r=r, n_windows=n_windows)


def test_homogeneous_euler_window_averages_closed_form(orc, hq):
    # phi^n = (2 pi q / sigma_a)(1 - r^n) everywhere; the windows average it
    # over their steps; the currents vanish (the quadrature is symmetric and
    # psi is the same for every ordinate).
    sa, q = 0.7, 1.3
    p = I.homogeneous(nx=6, ny=5, sigma_a=sa, sigma_s=0.4, q=q)
    nt, dt = orc.num_steps(p)
    nw = 5
    pr = _probes_at(p, hq, [(0.3, 0.25), (0.21, 0.33)], 0.08, nw)
    r = orc.solve(p, probes=pr)
    rr = 1.0 - dt * sa
    phi = (2 * math.pi * q / sa) * (1.0 - rr ** np.arange(nt))
    win = p.t_end / nw
    for w in range(nw):
        steps = [n for n in range(nt) if (n * nw) // nt == w]
        want = dt * phi[steps].sum() / win
        np.testing.assert_allclose(r["probes"][w, :, 0], want, rtol=1e-12)
    assert np.abs(r["probes"][:, :, 1:]).max() < 1e-12 * np.abs(r["probes"][:, :, 0]).max()


def test_steady_beam_current_closed_form(orc, hq):
    # steady first-order beam: psi_k(i) = g (1 + sigma h / xi_k)^-(i+1) for
    # xi_k > 0, else 0; J_x of cell i is the quadrature sum of xi psi; the
    # reflective S/N walls keep psi even in eta, so J_y = 0.
    sigma, g = 2.0, 1.5
    p = I.beam(nx=24, ny=3, M=32, sigma=sigma, g=g, h=0.05, t_end=0.4)
    psi0 = np.zeros((p.M, p.ny, p.nx))
    i = np.arange(p.nx)
    for k in range(p.M):
        if p.quad.xi[k] > 0:
            psi0[k] = g * (1 + sigma * p.h / p.quad.xi[k]) ** (-(i + 1.0))
    # a ball of radius 0.02 inside cell (7, 1): weight 1 on that cell
    pr = _probes_at(p, hq, [(7.5 * 0.05, 1.5 * 0.05)], 0.02, 4)
    assert list(pr["cell_i"]) == [7] and pr["weight"][0] == pytest.approx(1.0, rel=1e-12)
    r = orc.solve(p, psi0=psi0, probes=pr)
    xi, w = np.asarray(p.quad.xi), np.asarray(p.quad.w)
    jx = sum(w[k] * xi[k] * g * (1 + sigma * p.h / xi[k]) ** (-8.0) for k in range(p.M) if xi[k] > 0)
    phi = sum(w[k] * g * (1 + sigma * p.h / xi[k]) ** (-8.0) for k in range(p.M) if xi[k] > 0)
    np.testing.assert_allclose(r["probes"][:, 0, 0], phi, rtol=1e-12)
    np.testing.assert_allclose(r["probes"][:, 0, 1], jx, rtol=1e-12)
    assert np.abs(r["probes"][:, 0, 2]).max() < 1e-13 * jx


@pytest.mark.parametrize("stepper", [I.EULER, I.HEUN])
def test_windows_add_up_to_the_fluence(orc, hq, stepper):
    p = I.random_materials(17, 13, 4, seed=4, order=2, stepper=stepper, t_end=0.4)
    pr = _probes_at(p, hq, [(0.3, 0.2), (0.52, 0.41)], 0.06, 3)
    r = orc.solve(p, psi0=I.random_state(p, 9), fluence=True, probes=pr)
    win = p.t_end / 3
    for q in range(2):
        m = pr["probe"] == q
        ball = np.sum(pr["weight"][m] * r["fluence"][pr["cell_j"][m], pr["cell_i"][m]])
        assert win * r["probes"][:, q, 0].sum() == pytest.approx(ball, rel=1e-12)


def test_split_run_matches_single_call(orc, hq):
    p = I.random_materials(11, 9, 3, seed=6, order=2, stepper=I.HEUN, t_end=0.5)
    pr = _probes_at(p, hq, [(0.2, 0.2)], 0.05, 4)
    nt, _ = orc.num_steps(p)
    psi0 = I.random_state(p, 3)
    one = np.zeros((4, 1, 3))
    orc.advance(p, psi0, nt, probes=pr, probe_acc=one)
    two = np.zeros((4, 1, 3))
    k = nt // 3 + 1
    psi, _ = orc.advance(p, psi0, k, probes=pr, probe_acc=two)
    orc.advance(p, psi, nt - k, probes=pr, step0=k, probe_acc=two)
    np.testing.assert_allclose(two, one, rtol=1e-13, atol=0)
