"""Pins of the oracle's whole kiFMM (Sections 2, 2.1.1, 2.2) against the
direct sum, with error magnitudes from the paper's grid search (Table 5)."""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import fmm, kernel, surfaces


@pytest.fixture(scope="module")
def problem():
    pts = workloads.uniform_cube(2000, 31)
    q = workloads.charges(2000, 2, 32, "u01")
    return pts, q, kernel.direct(pts, q, pts)


def test_error_falls_with_order(problem, repo_root):
    pts, q, ex = problem
    with open(os.path.join(repo_root, "tests", "golden", "paper_counts.json")) as fh:
        orders = {r["P"]: r["eps"] for r in json.load(fh)["kifmm_error_order"]["rows"]}
    for depth in (2, 3):
        errs = {}
        for p in (3, 4, 5, 6, 7, 8):
            errs[p] = kernel.rel_l2(fmm.KiFMM(pts, pts, depth, p).evaluate(q), ex)
        for a, b in ((3, 5), (4, 6), (5, 7), (6, 8)):
            assert errs[b] < errs[a]
        for p, eps in orders.items():
            assert errs[p] < 5 * eps, (depth, p, errs[p])


def test_sources_differ_from_targets():
    src = workloads.uniform_cube(1500, 33)
    tgt = workloads.uniform_cube(700, 34)
    q = workloads.charges(1500, 1, 35, "upm1")
    ex = kernel.direct(src, q, tgt)
    got = fmm.KiFMM(src, tgt, 3, 6).evaluate(q)
    assert kernel.rel_l2(got, ex) < 5e-6


def test_sphere_pruned_tree():
    pts = workloads.sphere_surface(3000, 36)
    q = workloads.charges(3000, 1, 37, "normal")
    ex = kernel.direct(pts, q, pts)
    got = fmm.KiFMM(pts, pts, 4, 6, origin=(-1, -1, -1), width=2.0).evaluate(q)
    assert kernel.rel_l2(got, ex) < 1e-5


def test_sampled_equals_full():
    pts = workloads.uniform_cube(3000, 38)
    q = workloads.charges(3000, 2, 39, "u01")
    f = fmm.KiFMM(pts, pts, 3, 4)
    full = f.evaluate(q)
    s = workloads.sample_indices(3000, 40, 40)
    assert np.allclose(f.evaluate(q, s), full[:, s], rtol=1e-13, atol=0)


def test_p2m_monopole_and_far_field():
    # the upward equivalent densities carry the source monopole, and their far
    # field converges to the sources' with p
    rng = np.random.default_rng(41)
    y = rng.random((40, 3)) * 0.25
    q = rng.random(40)
    far = np.array([[3.0, 0.2, -1.0], [-2.0, 2.5, 0.7]])
    c = np.full(3, 0.125)
    prev = None
    for p in (3, 5, 7):
        f = fmm.KiFMM(np.vstack([y, [[1, 1, 1]]]), np.vstack([y, [[1, 1, 1]]]), 2, p)
        uc = surfaces.surface(p, 2.95, 0.125, c)
        ue = surfaces.surface(p, 1.05, 0.125, c)
        qe = f._apply_pinv(f.up_pinv(2), (kernel.kernel_matrix(uc, y) @ q)[None, :, None])[0, :, 0]
        assert abs(qe.sum() - q.sum()) < 1e-2 * q.sum()
        err = np.abs(kernel.kernel_matrix(far, ue) @ qe - kernel.kernel_matrix(far, y) @ q).max()
        if prev is not None:
            assert err < prev
        prev = err


@pytest.mark.parametrize("mistake", ["t_sign", "l2l_transposed", "no_l2l", "m2m_octant"])
def test_planted_mistakes_are_caught(problem, mistake, monkeypatch):
    # a plausible mistake in the oracle must break the error pin above
    pts, q, ex = problem
    f = fmm.KiFMM(pts, pts, 3, 6)
    if mistake == "t_sign":
        orig = f.m2l_matrix
        monkeypatch.setattr(f, "m2l_matrix", lambda lev, it: orig(lev, 315 - it))
    elif mistake == "l2l_transposed":
        orig = f.l2l_matrix
        monkeypatch.setattr(f, "l2l_matrix", lambda lev, o: orig(lev, o).T)
    elif mistake == "no_l2l":
        monkeypatch.setattr(f, "l2l_matrix", lambda lev, o: np.zeros((f.ns, f.ns)))
    elif mistake == "m2m_octant":
        orig = f.m2m_matrix
        monkeypatch.setattr(f, "m2m_matrix", lambda lev, o: orig(lev, 7 - o))
    assert kernel.rel_l2(f.evaluate(q), ex) > 1e-4
