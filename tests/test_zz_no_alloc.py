"""kifmm_evaluate_noalloc (work buffers from the library's fixed device scratch
array, no allocation) against kifmm_evaluate on the same handles and inputs:
two calls in a row, the second on a smaller problem (fewer points and
vectors), then the first problem again with new charges, so each call runs on
the array as the previous call left it.  Gates: the parity gates of the
potentials (FP64 1e-10, FP32 / BF16x3 1e-5 relative L2 and element-wise);
the two entry points run the same kernels in the same schedule, so the
potentials are also expected bit for bit."""
import numpy as np
import pytest

import workloads
from oracle import fmm

from gpu_util import E2E_GATES, check_parity, say

K = pytest.importorskip("paper_2408_07436_amd")
torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (m2l, prec, order, depth, blas tol, (points, vectors) of the two problems)
CASES = [("fft", "fp64", 4, 4, 0.0, (30000, 3), (9000, 1)),
         ("fft", "fp32", 6, 4, 0.0, (40000, 2), (8000, 1)),
         ("blas", "fp32", 5, 3, 1e-6, (20000, 4), (6000, 2)),
         ("blas", "bf16x3", 5, 3, 1e-6, (12000, 2), (5000, 1)),
         ("blas", "bf16x6", 5, 3, 1e-6, (12000, 3), (5000, 2)),
         ("dense", "fp64", 3, 3, 0.0, (20000, 1), (5000, 1))]


def make(m2l, prec, order, depth, tol, n, nvec, seed):
    kw = dict(svd_rel_tol=tol, svd_rel_tol_dir=tol) if m2l == "blas" else {}
    pts = workloads.uniform_cube(n, seed)
    f = K.KiFMM(order, depth, m2l=m2l, prec=prec, **kw).set_points(pts).precompute()
    q = torch.as_tensor(workloads.charges(n, nvec, seed + 1, "upm1"), dtype=f.dtype, device="cuda")
    return f, pts, q


@pytest.mark.parametrize("m2l,prec,order,depth,tol,big,small", CASES)
def test_noalloc_matches_evaluate(m2l, prec, order, depth, tol, big, small):
    gates = E2E_GATES[prec]
    fa, _, qa = make(m2l, prec, order, depth, tol, big[0], big[1], 7100)
    fb, pts_b, qb = make(m2l, prec, order, depth, tol, small[0], small[1], 7200)
    # the regular entry point first: it places the tree and operators on the device
    ref_a = fa.evaluate(qa).clone()
    ref_b = fb.evaluate(qb).clone()
    torch.cuda.synchronize()
    for name, f, q, ref in (("first (larger)", fa, qa, ref_a), ("second (smaller)", fb, qb, ref_b)):
        say(f"case: noalloc {m2l} {prec} p{order} depth {depth}, {name}: {f.n_src} points, "
            f"{q.shape[0]} vectors")
        out = torch.full_like(ref, float("nan"))
        f.evaluate_noalloc(q, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
        check_parity(got, ref.cpu().numpy().astype(np.float64), gates, what="vs kifmm_evaluate")
        assert torch.equal(out, ref), "no-allocation potentials differ from kifmm_evaluate's"
    # the larger problem again, new charges, after the smaller one used the array
    qa2 = -0.5 * qa + 0.25
    ref_a2 = fa.evaluate(qa2).clone()
    out = torch.empty_like(ref_a2)
    fa.evaluate_noalloc(qa2, out)
    torch.cuda.synchronize()
    check_parity(out.cpu().numpy().astype(np.float64), ref_a2.cpu().numpy().astype(np.float64), gates,
                 what="first problem again vs kifmm_evaluate")
    assert torch.equal(out, ref_a2)
    # the handle's own buffers are untouched: the regular entry point still agrees
    assert torch.equal(fb.evaluate(qb), ref_b)
    if m2l == "fft":
        ora = fmm.KiFMM(pts_b, pts_b, depth, order).evaluate(qb.cpu().numpy().astype(np.float64))
        out = torch.empty_like(ref_b)
        fb.evaluate_noalloc(qb, out)
        torch.cuda.synchronize()
        check_parity(out.cpu().numpy().astype(np.float64), ora, gates, what="vs oracle")
    fa.close()
    fb.close()


def test_noalloc_refuses_problem_above_scratch_and_stale_tiles():
    """A problem whose work buffers exceed the scratch array is refused with EINVAL
    (nothing enqueued, output untouched); BLAS tiles built for another width, ESTATE."""
    f, _, q = make("fft", "fp32", 6, 5, 0.0, 300000, 1, 7300)
    f.evaluate(q)
    out = torch.full((1, f.n_tgt), 7.0, dtype=torch.float32, device="cuda")
    with pytest.raises(K.KifmmError) as e:
        f.evaluate_noalloc(q, out)
    say(f"  refused: {e.value}")
    assert e.value.code == 1 and "MiB" in str(e.value)
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0))
    f.close()
    g, _, qg = make("blas", "fp32", 4, 3, 1e-6, 5000, 2, 7400)
    g.evaluate(qg)          # tiles of 64 boxes (128 / 2 vectors)
    q1 = qg[:1].contiguous()
    out1 = torch.empty((1, g.n_tgt), dtype=torch.float32, device="cuda")
    with pytest.raises(K.KifmmError) as e:
        g.evaluate_noalloc(q1, out1)   # one vector wants tiles of 128 boxes
    assert e.value.code == 2
    ref1 = g.evaluate(q1).clone()      # rebuilds the tiles
    g.evaluate_noalloc(q1, out1)
    torch.cuda.synchronize()
    assert torch.equal(out1, ref1)
    g.close()
