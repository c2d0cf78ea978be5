"""Pins of the oracle's kernel and direct sum (Section 1: N-body sum, 3D
Laplace kernel) against closed forms."""
import math

import numpy as np

from oracle import kernel


def test_two_charges_closed_form():
    y = np.array([[0.1, 0.2, 0.3]])
    x = np.array([[0.4, -0.2, 1.5]])
    q = np.array([[2.5]])
    r = math.sqrt(0.3 ** 2 + 0.4 ** 2 + 1.2 ** 2)
    assert abs(kernel.direct(y, q, x)[0, 0] - 2.5 / (4 * math.pi * r)) < 1e-15


def test_cube_corners_closed_form():
    # unit charges on the 8 corners of a unit cube: at a corner the other
    # corners sit at distance 1 (x3), sqrt(2) (x3) and sqrt(3) (x1); the
    # coincident corner contributes nothing.
    pts = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], dtype=float)
    q = np.ones((1, 8))
    phi = kernel.direct(pts, q, pts)
    want = (3 + 3 / math.sqrt(2) + 1 / math.sqrt(3)) / (4 * math.pi)
    assert np.allclose(phi, want, rtol=1e-15, atol=0)


def test_symmetry_and_self_term():
    rng = np.random.default_rng(0)
    p = rng.random((50, 3))
    k = kernel.kernel_matrix(p, p)
    assert np.all(np.diag(k) == 0.0)
    assert np.array_equal(k, k.T)


def test_exact_summation_at_a_few_targets():
    rng = np.random.default_rng(1)
    y = rng.random((300, 3))
    q = rng.random((1, 300))
    x = rng.random((4, 3)) + 2.0
    phi = kernel.direct(y, q, x)[0]
    for i in range(4):
        terms = [q[0, j] / (4 * math.pi * math.dist(x[i], y[j])) for j in range(300)]
        assert abs(phi[i] - math.fsum(terms)) <= 1e-14 * abs(phi[i])


def test_rel_l2():
    a = np.array([1.0, 2.0, 2.0])
    assert kernel.rel_l2(a, a) == 0.0
    assert abs(kernel.rel_l2(a + np.array([0, 0, 0.3]), a) - 0.1) < 1e-15
