"""Pins of the oracle's M2L forms: dense M2L (Section 2.2, the M2L matvec),
FFT-M2L (Appendix A.1; exact per Section 5.1) and SVD-compressed M2L
(Section 3.1)."""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import blas_m2l, fft_m2l, fmm, kernel, surfaces
from oracle.tree import TRANSFER_VECTORS


def test_dense_m2l_equals_explicit_pair_products():
    # build K(DC_tau, UE_sigma) from the actual box centres of every pair and
    # compare with the oracle's per-transfer-vector matrices
    pts = workloads.uniform_cube(4000, 21)
    f = fmm.KiFMM(pts, pts, 3, 4)
    rng = np.random.default_rng(22)
    lev = 3
    nb = len(f.tree.levels[lev])
    mult = rng.standard_normal((nb, f.ns, 2))
    got = f.m2l_level(lev, mult)
    offs, src, _ = f.tree.interactions(lev)
    r = f.r(lev)
    cen = f.tree.center(lev, np.arange(nb))
    for tau in range(0, nb, 37):
        dc = surfaces.surface(4, 1.05, r, cen[tau])
        want = np.zeros((f.ns, 2))
        for s in src[offs[tau]:offs[tau + 1]]:
            want += kernel.kernel_matrix(dc, surfaces.surface(4, 1.05, r, cen[s])) @ mult[s]
        assert np.allclose(got[tau], want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("p", [2, 3, 4, 6])
@pytest.mark.parametrize("grid", ["2p", "2p-1"])
def test_fft_m2l_equals_dense_toeplitz_product(p, grid):
    rng = np.random.default_rng(p)
    r = 0.125
    h = 2 * 1.05 * r / (p - 1)
    n = 2 * p if grid == "2p" else 2 * p - 1
    x = surfaces.surface(p, 1.05, r)
    for it in range(0, 316, 5):
        t = TRANSFER_VECTORS[it] * 2 * r
        q = rng.standard_normal(surfaces.n_surface(p))
        dense = kernel.kernel_matrix(x, surfaces.surface(p, 1.05, r, t)) @ q
        fft = fft_m2l.check_potential(p, h, -t, q, n)
        assert np.linalg.norm(fft - dense) <= 1e-13 * np.linalg.norm(dense) * p


def test_fft_grid_below_2p_minus_1_wraps():
    # one point fewer than 2p - 1 folds the kernel onto used entries
    p, r = 4, 0.125
    with pytest.raises(ValueError):
        fft_m2l.kernel_grid(p, 2 * 1.05 * r / (p - 1), np.array([0.5, 0.0, 0.0]), 2 * p - 2)


def test_fft_storage_matches_paper_table(repo_root):
    with open(os.path.join(repo_root, "tests", "golden", "paper_counts.json")) as fh:
        rows = json.load(fh)["fft_m2l_storage_mb"]["rows"]
    for row in rows:
        p = row["P"]
        spec = fft_m2l.kernel_spectrum(p, 0.1, np.array([2.0, 0.0, 0.0]))
        assert spec.size == (2 * p) ** 2 * (p + 1)
        # the table counts two such sets of 26 x 64 spectra
        mib = 2 * fft_m2l.storage_words(p) * row["bytes_per_word"] / 2 ** 20
        assert abs(mib - row["mb"]) < 0.01  # the table truncates or rounds to 2 decimals


def test_fft_mode_equals_dense_mode_whole_fmm():
    pts = workloads.uniform_cube(800, 23)
    q = workloads.charges(800, 1, 24, "u01")
    a = fmm.KiFMM(pts, pts, 2, 3, m2l="dense").evaluate(q)
    b = fmm.KiFMM(pts, pts, 2, 3, m2l="fft").evaluate(q)
    assert kernel.rel_l2(b, a) < 1e-13


def test_full_rank_blas_equals_dense():
    ks = blas_m2l.m2l_matrices(4, 0.25)
    comp = blas_m2l.compress(ks, 0.0, -1.0)
    assert comp["k"] == surfaces.n_surface(4)
    for it in range(0, 316, 7):
        assert np.allclose(blas_m2l.applied_operator(comp, it), ks[it], rtol=0,
                           atol=1e-13 * np.abs(ks[it]).max())
    # Fong's identity K_t = U C_t S^T also holds with full-rank recompression
    comp2 = blas_m2l.compress(ks, 0.0, 0.0)
    for it in range(0, 316, 11):
        assert np.allclose(blas_m2l.applied_operator(comp2, it), ks[it], rtol=0,
                           atol=1e-13 * np.abs(ks[it]).max())


@pytest.mark.parametrize("tol,tol_dir", [(1e-4, -1.0), (1e-6, 1e-6), (1e-3, 1e-2)])
def test_truncated_blas_error_bound(tol, tol_dir):
    ks = blas_m2l.m2l_matrices(5, 0.25)
    comp = blas_m2l.compress(ks, tol, tol_dir)
    k = comp["k"]
    bound0 = comp["sigma_fat"][k] + comp["sigma_thin"][k]
    for it in range(0, 316, 3):
        err = np.linalg.norm(ks[it] - blas_m2l.applied_operator(comp, it), 2)
        c = comp["U"].T @ ks[it] @ comp["S"]
        sc = np.linalg.svd(c, compute_uv=False)
        kt = comp["kt"][it]
        extra = sc[kt] if kt < len(sc) else 0.0
        assert err <= (bound0 + extra) * (1 + 1e-9) + 1e-15


def test_compression_basis_independent():
    # the applied operator does not depend on the singular-vector signs
    ks = blas_m2l.m2l_matrices(4, 0.25)
    comp = blas_m2l.compress(ks, 1e-5, 1e-5)
    rng = np.random.default_rng(9)
    s1 = np.diag(rng.choice([-1.0, 1.0], comp["k"]))
    s2 = np.diag(rng.choice([-1.0, 1.0], comp["k"]))
    u, s = comp["U"] @ s1, comp["S"] @ s2
    for it in range(0, 316, 13):
        c = u.T @ ks[it] @ s
        cu, cs, cvt = np.linalg.svd(c)
        r = comp["kt"][it]
        op = u @ cu[:, :r] @ (cvt[:r].T * cs[:r]).T @ s.T
        assert np.allclose(op, blas_m2l.applied_operator(comp, it), atol=1e-12 * np.abs(ks[it]).max())


def test_probe_ranks_p6():
    # rank at the 1e-6 relative threshold for p = 6 (both stacks agree when the
    # check and equivalent surfaces are discretised alike)
    ks = blas_m2l.m2l_matrices(6, 0.5)
    comp = blas_m2l.compress(ks, 1e-6, 1e-6)
    kthin = int(np.sum(comp["sigma_thin"] > 1e-6 * comp["sigma_thin"][0]))
    assert comp["k"] == kthin
    assert 80 <= comp["k"] <= 152
    assert 5 <= comp["kt"].min() and comp["kt"].max() <= comp["k"]


def test_check_order_above_expansion_order():
    """P_c > P_e (Section 5.1; the P_e / P_c columns of Section 4's BLAS-M2L
    parameter table), with rectangular n_c x n_e M2L matrices.  More check points
    never make the dense fit worse against the direct sum.  The compressed form
    keeps one rank k <= n_e for both sides, so at full rank it drops the part of
    K_fat beyond its n_e-th singular value: it differs from the dense form by no
    more than sigma_(n_e) / sigma_0 of K_fat, and equals it when P_c = P_e."""
    pts = workloads.uniform_cube(3000, 5)
    q = workloads.charges(3000, 2, 6, "normal")
    direct = kernel.direct(pts, q, pts)
    ne = surfaces.n_surface(4)
    errs = []
    for pc in (4, 5, 6):
        dense = fmm.KiFMM(pts, pts, 3, 4, check_order=pc).evaluate(q)
        blas = fmm.KiFMM(pts, pts, 3, 4, m2l="blas", check_order=pc).evaluate(q)
        s = np.linalg.svd(np.hstack(blas_m2l.m2l_matrices(4, 0.5, check_order=pc)), compute_uv=False)
        bound = s[ne] / s[0] if s.size > ne else 1e-13
        assert kernel.rel_l2(blas, dense) < bound
        errs.append(kernel.rel_l2(dense, direct))
    assert errs[0] > errs[1] > errs[2]
    with pytest.raises(ValueError):
        fmm.KiFMM(pts, pts, 3, 4, m2l="fft", check_order=5)
    with pytest.raises(ValueError):
        fmm.KiFMM(pts, pts, 3, 4, check_order=3)
