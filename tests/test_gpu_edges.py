"""Degenerate and ragged inputs through the C ABI against the oracle: one
point (its own potential is exactly zero, the self term being excluded), two
and nine points at depths 2 and 3 (levels with a single box, halos that are
all absent), all points in one corner of the domain (a heavily pruned tree
whose FFT-M2L source blocks are partly filled), two far-apart clusters, zero
charges (exactly zero potentials), coincident points (copies of other points:
the kernel is zero for bitwise-equal points) and points on the domain's faces
(coordinates exactly 0 and exactly 1, which the leaf anchor clamps into the
last leaf), and FFT-M2L at orders 2, 7 and 8 (the smallest and largest
built).  Gates as in the parity tests (gpu_util), element by element and in
relative L2."""
import numpy as np
import pytest

import workloads
from oracle import fmm, kernel

from gpu_util import E2E_GATES, STAGE_GATES, check_parity, evaluate, say

K = pytest.importorskip("paper_2408_07436_amd")
torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MODES = [("fft", "fp64"), ("fft", "fp32"), ("blas", "fp64"), ("blas", "fp32")]


def corner(n, seed):
    rng = np.random.default_rng(seed)
    return 0.2 * rng.random((n, 3)) + 0.001


def two_clusters(n, seed):
    rng = np.random.default_rng(seed)
    h = n // 2
    return np.concatenate([0.1 * rng.random((h, 3)) + 0.02, 0.1 * rng.random((n - h, 3)) + 0.85])


@pytest.mark.parametrize("m2l,prec", MODES)
def test_single_point_has_zero_potential(m2l, prec):
    pts = workloads.uniform_cube(1, 901)
    q = workloads.charges(1, 2, 911, "normal")
    say(f"case: one point depth 2 p4 {m2l} {prec}")
    got, _ = evaluate(K, pts, q, 2, 4, m2l, prec)
    say(f"  potentials {got.ravel()}")
    assert np.all(got == 0.0)


@pytest.mark.parametrize("m2l,prec", MODES)
@pytest.mark.parametrize("n,depth", [(2, 2), (9, 3)])
def test_few_points(m2l, prec, n, depth):
    pts = workloads.uniform_cube(n, 900 + n)
    q = workloads.charges(n, 2, 910 + n, "normal")
    say(f"case: {n} points depth {depth} p4 {m2l} {prec}")
    got, _ = evaluate(K, pts, q, depth, 4, m2l, prec)
    ref = fmm.KiFMM(pts, pts, depth, 4).evaluate(q)
    check_parity(got, ref, E2E_GATES[prec])


@pytest.mark.parametrize("m2l,prec", MODES)
@pytest.mark.parametrize("shape", ["corner", "two_clusters"])
def test_pruned_trees(m2l, prec, shape):
    n = 6000
    pts = corner(n, 921) if shape == "corner" else two_clusters(n, 922)
    q = workloads.charges(n, 1, 923, "normal")
    say(f"case: {shape} {n} points depth 5 p4 {m2l} {prec}")
    got, _ = evaluate(K, pts, q, 5, 4, m2l, prec)
    ref = fmm.KiFMM(pts, pts, 5, 4).evaluate(q)
    check_parity(got, ref, E2E_GATES[prec])


@pytest.mark.parametrize("m2l,prec", MODES)
def test_zero_charges_give_zero(m2l, prec):
    pts = workloads.uniform_cube(5000, 931)
    q = np.zeros((3, 5000))
    say(f"case: zero charges 5000 points depth 4 p4 {m2l} {prec}")
    got, _ = evaluate(K, pts, q, 4, 4, m2l, prec)
    assert np.all(got == 0.0)


@pytest.mark.parametrize("p", [2, 7, 8])
@pytest.mark.parametrize("prec,gate", [("fp64", STAGE_GATES["fp64"]), ("fp32", STAGE_GATES["fp32"])])
def test_fft_extreme_orders_stage(p, prec, gate):
    """FFT-M2L at the smallest and the largest orders the library builds (grids
    of 3 and 15 points per axis): one level at a time, in check-potential space."""
    pts = workloads.sphere_surface(8000, 990 + p)
    ora = fmm.KiFMM(pts, pts, 4, p, origin=(-1, -1, -1), width=2.0)
    f = K.KiFMM(p, 4, m2l="fft", prec=prec, origin=(-1, -1, -1), width=2.0).set_points(pts).precompute()
    rng = np.random.default_rng(991)
    for lev in (2, 3, 4):
        nb = len(ora.tree.levels[lev])
        mult = rng.standard_normal((nb, 2, ora.ns))
        say(f"case: fft stage p{p} {prec} level {lev} boxes {nb}")
        out = f.stage_m2l(lev, torch.as_tensor(mult, device="cuda"))
        torch.cuda.synchronize()
        ref = ora.m2l_level(lev, mult.transpose(0, 2, 1)).transpose(0, 2, 1)
        check_parity(out.cpu().numpy(), ref, gate, vec_axis=1, what="check potentials vs oracle")


@pytest.mark.parametrize("p", [2, 8])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fft_extreme_orders_end_to_end(p, prec):
    pts = workloads.sphere_surface(8000, 992 + p)
    q = workloads.charges(8000, 1, 993 + p, "normal")
    say(f"case: fft end to end p{p} {prec} sphere 8000 depth 4")
    got, _ = evaluate(K, pts, q, 4, p, "fft", prec, origin=(-1, -1, -1), width=2.0)
    ref = fmm.KiFMM(pts, pts, 4, p, origin=(-1, -1, -1), width=2.0).evaluate(q)
    check_parity(got, ref, E2E_GATES[prec])


def duplicates_and_faces(n, seed):
    """n uniform points, then 300 exact copies of some of them, then 200 points
    with one, two or three coordinates exactly 0.0 or 1.0 (domain faces, edges
    and corners of [0, 1]^3), and a second copy of 20 of those."""
    rng = np.random.default_rng(seed)
    base = rng.random((n, 3))
    dup = base[rng.choice(n, 300, replace=False)]
    face = rng.random((200, 3))
    for i in range(200):
        axes = rng.choice(3, size=1 + i % 3, replace=False)
        face[i, axes] = rng.integers(0, 2, size=axes.size).astype(np.float64)
    pts = np.concatenate([base, dup, face, face[:20]])
    return pts[rng.permutation(pts.shape[0])]


@pytest.mark.parametrize("m2l,prec", MODES)
def test_coincident_points_and_domain_faces(m2l, prec):
    pts = duplicates_and_faces(6000, 941)
    n = pts.shape[0]
    assert np.sum(pts == 1.0) > 0 and np.unique(pts, axis=0).shape[0] < n
    q = workloads.charges(n, 2, 942, "normal")
    say(f"case: {n} points with 320 coincident copies and 220 on the faces, depth 4 p4 {m2l} {prec}")
    got, _ = evaluate(K, pts, q, 4, 4, m2l, prec)
    ref = fmm.KiFMM(pts, pts, 4, 4).evaluate(q)
    check_parity(got, ref, E2E_GATES[prec])
