"""Pins of the backward-stable pseudo-inverse (Section 2.1.1): the paper's
rule is SciPy's default, so scipy.linalg.pinv is its library special case."""
import numpy as np
import pytest
import scipy.linalg

from oracle import kernel, linalg, surfaces


@pytest.mark.parametrize("shape", [(7, 7), (9, 5), (5, 9)])
def test_matches_scipy_on_random(shape):
    rng = np.random.default_rng(3)
    a = rng.standard_normal(shape)
    v, ut = linalg.pinv_factors(a)
    assert np.allclose(v @ ut, scipy.linalg.pinv(a), rtol=1e-12, atol=1e-12)


def test_rank_deficient_drops_small_singular_values():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((8, 3)) @ rng.standard_normal((3, 8))
    v, ut = linalg.pinv_factors(a)
    assert v.shape == (8, 3) and ut.shape == (3, 8)
    pa = v @ ut
    assert np.allclose(pa, scipy.linalg.pinv(a), atol=1e-10)
    # Moore-Penrose identities
    assert np.allclose(a @ pa @ a, a, atol=1e-12)
    assert np.allclose(pa @ a @ pa, pa, atol=1e-12)
    assert np.allclose((a @ pa).T, a @ pa, atol=1e-12)
    assert np.allclose((pa @ a).T, pa @ a, atol=1e-12)


def test_check_to_equivalent_solve():
    # the kiFMM solve: ill-conditioned, but the recovered density reproduces
    # the check potential of a smooth exterior field to high accuracy
    p = 6
    uc = surfaces.surface(p, 2.95, 0.5)
    ue = surfaces.surface(p, 1.05, 0.5)
    k = kernel.kernel_matrix(uc, ue)
    src = np.array([[0.1, -0.2, 0.3], [-0.4, 0.1, 0.05]])
    phi = kernel.kernel_matrix(uc, src) @ np.array([1.0, -0.5])
    q = linalg.pinv_apply(linalg.pinv_factors(k), phi)
    assert np.linalg.norm(k @ q - phi) < 1e-9 * np.linalg.norm(phi)
