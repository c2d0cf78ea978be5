"""Moving points: kifmm_update_points builds the tree of the new positions
on the device (Section 5.1's re-setup).  With the box set unchanged the
point order and potentials must equal those of a fresh kifmm_set_points bit
for bit; when the box set changes, the device-built levels, point order,
interaction and near lists must equal the oracle's tree entry for entry, the
potentials must equal a fresh handle's bit for bit (same domain cube) and
pass the oracle's element-wise gates; a point outside the domain cube is
refused and changes nothing."""
import numpy as np
import pytest

import workloads
from oracle import tree as T

from gpu_util import E2E_GATES, check_parity, say

K = pytest.importorskip("paper_2408_07436_amd")
torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def fresh(order, depth, m2l, prec, src, tgt=None, **kw):
    return K.KiFMM(order, depth, m2l=m2l, prec=prec, **kw).set_points(src, tgt).precompute()


@pytest.mark.parametrize("m2l,prec,distinct", [("fft", "fp32", False), ("fft", "fp64", True),
                                               ("blas", "fp32", False)])
def test_update_points_matches_fresh_tree(m2l, prec, distinct):
    kw = dict(svd_rel_tol=1e-6, svd_rel_tol_dir=1e-6) if m2l == "blas" else {}
    n, depth, order = 20000, 3, 5
    p0 = workloads.uniform_cube(n, 301)
    p1 = workloads.uniform_cube(n, 302)
    t0 = workloads.uniform_cube(7000, 303) if distinct else None
    t1 = workloads.uniform_cube(7000, 304) if distinct else None
    q = workloads.charges(n, 2, 305, "upm1")
    say(f"case: update points {m2l} {prec} 20k depth 3 p5 distinct={distinct}")
    dt = torch.float64 if prec == "fp64" else torch.float32
    qt = torch.as_tensor(q, dtype=dt, device="cuda")
    f = fresh(order, depth, m2l, prec, p0, t0, **kw)
    f.evaluate(qt)
    g = fresh(order, depth, m2l, prec, p1, t1, **kw)
    assert np.array_equal(f.box_keys(depth), g.box_keys(depth)), "box sets differ"
    s1 = torch.as_tensor(p1, device="cuda")
    f.update_points(s1, torch.as_tensor(t1, device="cuda") if distinct else None)
    a = f.evaluate(qt)
    b = g.evaluate(qt)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert np.array_equal(f.point_perm(0), g.point_perm(0))
    assert np.array_equal(f.point_perm(1), g.point_perm(1))


def test_update_points_three_pass_sort_permuted():
    """262,144 leaves (three 8-bit passes of the radix sort): the same points
    in another order give the fresh tree's point order and potentials."""
    pts = workloads.sphere_surface(150000, 311)
    q = workloads.charges(150000, 1, 312, "normal")
    perm = np.random.default_rng(313).permutation(150000)
    say("case: update points, permuted sphere 150k depth 6 p4 fft fp64")
    f = fresh(4, 6, "fft", "fp64", pts, origin=(-1, -1, -1), width=2.0)
    g = fresh(4, 6, "fft", "fp64", pts[perm], origin=(-1, -1, -1), width=2.0)
    qt = torch.as_tensor(q, device="cuda")
    f.evaluate(qt)
    f.update_points(torch.as_tensor(pts[perm], device="cuda"))
    a = f.evaluate(qt[:, torch.as_tensor(perm, device="cuda")].contiguous())
    b = g.evaluate(qt[:, torch.as_tensor(perm, device="cuda")].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert np.array_equal(f.point_perm(0), g.point_perm(0))


def test_update_points_refuses_points_outside_the_cube():
    pts = workloads.sphere_surface(20000, 321)
    q = workloads.charges(20000, 1, 322, "normal")
    say("case: update points refused (sphere 20k depth 4 p4 fft fp32)")
    f = fresh(4, 4, "fft", "fp32", pts, origin=(-1, -1, -1), width=2.0)
    qt = torch.as_tensor(q, dtype=torch.float32, device="cuda")
    before = f.evaluate(qt).clone()
    perm_before = f.point_perm(0).copy()
    keys_before = f.box_keys(4).copy()
    moved = pts.copy()
    moved[123] = np.array([1.5, 0.0, 0.0])
    with pytest.raises(K.KifmmError) as e:
        f.update_points(torch.as_tensor(moved, device="cuda"))
    assert e.value.code == 2
    after = f.evaluate(qt)
    torch.cuda.synchronize()
    assert torch.equal(before, after)
    assert np.array_equal(perm_before, f.point_perm(0))
    assert np.array_equal(keys_before, f.box_keys(4))


def check_tree(f, src, tgt, depth, origin, width):
    """Device-built tree of f against the oracle's, entry for entry."""
    tr = T.Tree(src, tgt, depth, origin, width)
    for lev in range(depth + 1):
        assert f.num_boxes(lev) == len(tr.levels[lev]), f"box count, level {lev}"
        assert np.array_equal(f.box_keys(lev), tr.levels[lev]), f"keys, level {lev}"
    assert np.array_equal(f.point_perm(0), tr.src_perm)
    assert np.array_equal(f.point_perm(1), tr.tgt_perm)
    for lev in range(2, depth + 1):
        for x, y in zip(f.interactions(lev), tr.interactions(lev)):
            assert np.array_equal(x, y), f"interaction lists, level {lev}"
    for x, y in zip(f.near(), tr.near()):
        assert np.array_equal(x, y), "near lists"
    return tr


def contract(p, c, s):
    return np.asarray(c) + s * (p - np.asarray(c))


def rotate(p, angle, c):
    ca, sa = np.cos(angle), np.sin(angle)
    r = np.array([[ca, -sa, 0.0], [sa, ca, 0.0], [0.0, 0.0, 1.0]])
    r = r @ np.array([[1.0, 0.0, 0.0], [0.0, np.cos(0.3), -np.sin(0.3)], [0.0, np.sin(0.3), np.cos(0.3)]])
    return np.asarray(c) + (p - np.asarray(c)) @ r.T


# (m2l, prec, order, depth, nvec list per step, kind)
REBUILD = [
    ("fft", "fp32", 4, 4, [1], "uniform"),
    ("fft", "fp64", 4, 5, [2], "sphere"),
    ("blas", "fp32", 4, 4, [2, 1], "uniform"),
    ("blas", "fp64", 4, 4, [1], "distinct"),
    ("dense", "fp64", 3, 3, [1], "uniform"),
]


@pytest.mark.parametrize("m2l,prec,order,depth,nvecs,kind", REBUILD,
                         ids=[f"{r[0]}-{r[1]}-{r[5]}" for r in REBUILD])
def test_update_points_rebuilds_tree(m2l, prec, order, depth, nvecs, kind):
    from oracle import fmm
    kw = dict(svd_rel_tol=1e-6, svd_rel_tol_dir=1e-6) if m2l == "blas" else {}
    if kind == "sphere":
        origin, width, c = (-1.0, -1.0, -1.0), 2.0, (0.0, 0.0, 0.0)
        p0 = workloads.sphere_surface(30000, 331)
        steps = [rotate(p0, 0.35, c), contract(rotate(p0, 0.7, c), c, 0.55), p0]
        t0, tsteps = None, [None] * 3
    else:
        origin, width, c = (0.0, 0.0, 0.0), 1.0, (0.5, 0.5, 0.5)
        n = 12000 if m2l == "dense" else 20000
        p0 = workloads.uniform_cube(n, 341)
        blob = contract(p0, c, 0.45)
        steps = [blob, blob + np.array([0.2, -0.15, 0.1]), workloads.uniform_cube(n, 342)]
        if kind == "distinct":
            t0 = workloads.uniform_cube(6000, 343)
            tsteps = [contract(t0, (0.2, 0.3, 0.7), 0.3), contract(t0, c, 0.8), t0]
        else:
            t0, tsteps = None, [None] * 3
    say(f"case: update points with a new box set, {m2l} {prec} p{order} depth {depth} {kind}")
    f = fresh(order, depth, m2l, prec, p0, t0, origin=origin, width=width, **kw)
    dt = torch.float64 if prec == "fp64" else torch.float32
    nsrc = p0.shape[0]
    for k, (p, tp) in enumerate(zip(steps, tsteps)):
        before = [f.num_boxes(lev) for lev in range(depth + 1)]
        f.update_points(torch.as_tensor(p, device="cuda"),
                        None if tp is None else torch.as_tensor(tp, device="cuda"))
        counts = [f.num_boxes(lev) for lev in range(depth + 1)]
        say(f"  step {k}: boxes per level {before} -> {counts}")
        tgt = p if tp is None else tp
        check_tree(f, p, tgt, depth, origin, width)
        g = fresh(order, depth, m2l, prec, p, tp, origin=origin, width=width, **kw)
        for nvec in nvecs:
            q = workloads.charges(nsrc, nvec, 350 + k, "upm1")
            qt = torch.as_tensor(q, dtype=dt, device="cuda")
            a = f.evaluate(qt)
            b = g.evaluate(qt)
            torch.cuda.synchronize()
            assert torch.equal(a, b), f"step {k}, {nvec} vectors: potentials differ from a fresh tree"
        if k == 1:
            okw = dict(m2l="blas", svd_rel_tol=1e-6, svd_rel_tol_dir=1e-6) if m2l == "blas" else {}
            ref = fmm.KiFMM(p, tgt, depth, order, origin=origin, width=width, **okw).evaluate(q)
            check_parity(a.double().cpu().numpy(), ref, E2E_GATES[prec], what=f"step {k} vs oracle")
        g.close()
    # the moved handle still serves a batch (recorded launches read the new buffers)
    phi = torch.full_like(a, float("nan"))
    bt = K.Batch([(f, qt, phi)])
    bt.launch()
    torch.cuda.synchronize()
    bt.close()
    assert torch.equal(phi, a)
