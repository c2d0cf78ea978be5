"""Batches of independent problems run as one graph of grouped launches (one
launch per stage and kernel instance across all problems): every replay must
reproduce the eager evaluate of each problem bit for bit, also after the
charges change, with eager work between replays and with other buffers per
launch; the serving workload's 128 problems are each checked against the
oracle."""
import numpy as np
import pytest

import workloads
from oracle import fmm, kernel

from gpu_util import E2E_GATES, check_parity, say

K = pytest.importorskip("paper_2408_07436_amd")
torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PROBLEMS = [
    # n, depth, p, m2l, prec, nvec
    (4000, 3, 4, "fft", "fp32", 1),
    (12000, 3, 5, "fft", "fp32", 3),
    (20000, 4, 6, "fft", "fp32", 2),
    (9000, 3, 4, "blas", "bf16x3", 4),
    (7000, 3, 3, "dense", "fp64", 1),
    (15000, 4, 5, "fft", "fp64", 5),
    (8000, 3, 5, "blas", "bf16x6", 2),
]


def build(i, n, depth, p, m2l, prec, nvec):
    pts = workloads.uniform_cube(n, 7000 + i)
    q = workloads.charges(n, nvec, 7100 + i, "upm1")
    kw = dict(svd_rel_tol=1e-6, svd_rel_tol_dir=1e-6) if m2l == "blas" else {}
    f = K.KiFMM(p, depth, m2l=m2l, prec=prec, **kw).set_points(pts).precompute()
    qt = torch.as_tensor(q, dtype=f.dtype, device="cuda")
    return f, pts, q, qt


def test_batch_graph_replays_match_eager():
    items, eager, hosts = [], [], []
    for i, spec in enumerate(PROBLEMS):
        f, pts, q, qt = build(i, *spec)
        ref = f.evaluate(qt).clone()
        phi = torch.full_like(ref, float("nan"))
        items.append((f, qt, phi))
        eager.append(ref)
        hosts.append((pts, q))
    torch.cuda.synchronize()
    say(f"case: batch of {len(items)} problems, grouped launches in one graph")
    b = K.Batch(items)
    info = b.info()
    say(f"  {info}")
    assert info["problems"] == len(items)
    # one launch per stage and kernel instance, not one per problem: the FFT
    # problems' launches are all grouped; the BLAS problem adds its own
    assert info["grouped"] >= 10 and info["launches"] <= 100
    for rep in range(3):
        for _, _, phi in items:
            phi.fill_(float("nan"))
        b.launch()
        torch.cuda.synchronize()
        for i, (_, _, phi) in enumerate(items):
            assert torch.equal(phi, eager[i]), f"replay {rep} problem {i}"
        # eager work between replays
        items[0][0].evaluate(items[0][1])
        torch.cuda.synchronize()
    # new charges in place: the replay reads them
    for _, qt, _ in items:
        qt.mul_(2.0)
    b.launch()
    torch.cuda.synchronize()
    for i, (_, _, phi) in enumerate(items):
        assert torch.equal(phi, 2.0 * eager[i]), f"scaled charges problem {i}"
    # other buffers per launch (kifmm_batch_evaluate): new charges in new
    # tensors, potentials into new tensors; the creation buffers stay as they were
    q_new = [(-0.5 * qt + 0.125).contiguous() for _, qt, _ in items]
    phi_new = [torch.full_like(phi, float("nan")) for _, _, phi in items]
    before = [phi.clone() for _, _, phi in items]
    b.evaluate(q_new, phi_new)
    torch.cuda.synchronize()
    for i, (f, _, phi) in enumerate(items):
        assert torch.equal(phi, before[i]), f"creation buffer changed, problem {i}"
    b.close()
    for i, (f, _, _) in enumerate(items):
        assert torch.equal(phi_new[i], f.evaluate(q_new[i])), f"batch_evaluate problem {i}"
    # every problem against the oracle (the replays equal the eager results)
    for i, (n, depth, p, m2l, prec, nvec) in enumerate(PROBLEMS):
        pts, q = hosts[i]
        kw = dict(m2l="blas", svd_rel_tol=1e-6, svd_rel_tol_dir=1e-6) if m2l == "blas" else {}
        ref = fmm.KiFMM(pts, pts, depth, p, **kw).evaluate(q)
        check_parity(eager[i].cpu().numpy().astype(np.float64), ref, E2E_GATES[prec],
                     what=f"problem {i} ({m2l} {prec}) vs oracle")


def test_batch_rejects_repeated_handle():
    f, _, _, qt = build(0, *PROBLEMS[0])
    phi = torch.empty((1, 4000), dtype=f.dtype, device="cuda")
    with pytest.raises(K.KifmmError) as e:
        K.Batch([(f, qt, phi), (f, qt, phi)])
    assert e.value.code == 1


def test_batch_autotune_keeps_results():
    """The batch autotuner times whole-batch candidates (BLAS tile widths and
    forms), keeps one, and the kept batch replays the eager results of the
    kept knobs bit for bit (and the default knobs' results to rounding)."""
    items, eager = [], []
    for i, spec in enumerate(PROBLEMS):
        f, _, _, qt = build(i, *spec)
        ref = f.evaluate(qt).clone()
        items.append((f, qt, torch.full_like(ref, float("nan"))))
        eager.append(ref)
    torch.cuda.synchronize()
    say(f"case: batch autotune over {len(items)} problems")
    b = K.Batch(items, autotune=True, reps=2)
    say(f"  kept {[f.tuning() for f, _, _ in items]}, {b.best_ms:.3f} ms")
    assert b.best_ms > 0.0
    for i, ((f, _, _), spec) in enumerate(zip(items, PROBLEMS)):
        t = f.tuning()
        m2l, prec, nvec = spec[3], spec[4], spec[5]
        if m2l == "fft":
            assert t["blas_tile"] == 0 and t["hadamard"] == 0
        else:
            assert t["blas_tile"] in [max(1, (128 // nvec) >> k) for k in range(4)]
    for rep in range(2):
        for _, _, phi in items:
            phi.fill_(float("nan"))
        b.launch()
        torch.cuda.synchronize()
        replay = [phi.clone() for _, _, phi in items]
        for i in range(len(items)):
            check_parity(replay[i].double().cpu().numpy(), eager[i].double().cpu().numpy(),
                         E2E_GATES[PROBLEMS[i][4]], what=f"replay {rep} problem {i} vs default knobs")
    b.close()
    for i, (f, qt, _) in enumerate(items):
        assert torch.equal(f.evaluate(qt), replay[i]), f"eager with kept knobs, problem {i}"


def test_serving_batch_every_problem_vs_oracle():
    """The batched serving workload as the benchmark runs it (128 problems, 1e4 to
    2e5 uniform points, depth 3-4, p 4-6, 1-8 vectors, FFT-M2L FP32 with FP64
    local accumulation): every problem's potentials from one grouped graph
    launch against the oracle at 100 sampled targets, element by element."""
    import batch_oracle
    specs = workloads.batch_problems(128)
    say(f"case: serving batch, {len(specs)} problems, oracle at {batch_oracle.N_SAMPLE} targets each")
    items = []
    for sp in specs:
        pts = workloads.uniform_cube(sp["n"], sp["seed_points"])
        q = workloads.charges(sp["n"], sp["nvec"], sp["seed_charges"], "u01")
        f = K.KiFMM(sp["order"], sp["depth"], m2l="fft", prec="fp32").set_points(pts).precompute()
        qt = torch.as_tensor(q, dtype=torch.float32, device="cuda")
        items.append((f, qt, torch.full((sp["nvec"], sp["n"]), float("nan"), dtype=torch.float32,
                                        device="cuda")))
    b = K.Batch(items)
    say(f"  {b.info()}")
    b.launch()
    torch.cuda.synchronize()
    got = [phi.cpu().numpy().astype(np.float64) for _, _, phi in items]
    b.close()
    worst = (0.0, 0.0)
    for i, s, ref in batch_oracle.references(specs):
        e2, ei = check_parity(got[i][:, s], ref, E2E_GATES["fp32"], what=f"problem {i}")
        worst = (max(worst[0], e2), max(worst[1], ei))
    say(f"  worst over {len(specs)} problems: rel L2 {worst[0]:.3e}, element-wise {worst[1]:.3e}")
