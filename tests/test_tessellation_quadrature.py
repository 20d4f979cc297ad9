"""The tessellation quadrature of Sec. 5.1.1 (M = 4 N^2), built by the input
generator; pinned by what its construction fixes exactly (the weights tile
the hemisphere; the octahedral symmetry makes the second moments exact) and
by its convergence on the first moment."""

import math

import numpy as np
import pytest

from paper_2505_17284_amd import inputs as I


@pytest.mark.parametrize("N", [1, 2, 3, 7, 18, 22])
def test_counts_weights_and_symmetric_moments(N):
    q = I.tessellation_quadrature(N)
    assert q.M == 4 * N * N
    assert q.w.sum() == pytest.approx(2 * math.pi, rel=1e-13)
    assert np.all(q.w > 0) and np.all(q.mu > 0)
    np.testing.assert_allclose(q.xi ** 2 + q.eta ** 2 + q.mu ** 2, 1.0, rtol=1e-14)
    # permuting the axes maps the first face's triangulation onto itself, so
    # the three second moments are equal and add up to sum w = 2 pi
    for m in (q.xi ** 2, q.eta ** 2, q.mu ** 2):
        assert np.sum(q.w * m) == pytest.approx(2 * math.pi / 3, rel=1e-13)
    assert abs(np.sum(q.w * q.xi)) < 1e-13 and abs(np.sum(q.w * q.eta)) < 1e-13
    assert np.array_equal(q.xi[q.mirror_x], -q.xi) and np.array_equal(q.eta[q.mirror_x], q.eta)
    assert np.array_equal(q.eta[q.mirror_y], -q.eta) and np.array_equal(q.xi[q.mirror_y], q.xi)
    assert np.array_equal(q.w[q.mirror_x], q.w) and np.array_equal(q.w[q.mirror_y], q.w)


def test_one_triangle_per_face():
    # N = 1: the whole face; centroid (1, 1, 1)/sqrt 3, weight = the octant's area pi/2
    q = I.tessellation_quadrature(1)
    np.testing.assert_allclose(np.abs(q.xi), 1 / math.sqrt(3), rtol=1e-15)
    np.testing.assert_allclose(q.mu, 1 / math.sqrt(3), rtol=1e-15)
    np.testing.assert_allclose(q.w, math.pi / 2, rtol=1e-15)


def test_first_moment_converges_at_second_order():
    # int over S^2_+ of mu = pi; the centroid rule errs by O(1/N^2)
    err = [abs(np.sum(q.w * q.mu) - math.pi) for q in map(I.tessellation_quadrature, (6, 12, 24))]
    assert 3.6 < err[0] / err[1] < 4.4 and 3.6 < err[1] / err[2] < 4.4


def test_plan_accepts_it_with_reflective_sides():
    from paper_2505_17284_amd import solver

    p = I.lattice(14, 32, bc=(I.BC_REFLECT,) * 4).replace(quad=I.tessellation_quadrature(5))
    info = solver.plan_info(p)
    assert info["M"] == 100 and info["n_steps"] > 0
