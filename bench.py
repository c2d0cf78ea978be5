#!/usr/bin/env python3
"""Benchmark of the kiFMM hot path on one MI355X.

Workload: 1,000,000 points uniform in the unit cube (sources = targets),
charges uniform in [0, 1), one charge vector, uniform octree of depth 5,
expansion order p = 6 (152 surface points, 12^3 convolution grid), FFT-M2L.
A step is one full evaluate: P2M, M2M, M2L (FFT forward, Hadamard, inverse)
per level, L2L and pseudo-inverses, L2P + P2P, written back in the caller's
order.  Inputs are resident in device memory before the timed region.

The headline value is the M2L time per evaluate of the mixed-precision run
(FP32 complex transforms and Hadamard products, FP64 local accumulation);
the same path in FP64 is timed beside it.  The JSON line also carries the
roofline of the dominant kernel, measured live with HIP events (the leaf
level's M2L kernels on their own through single-level stage calls, since the
levels of an evaluate overlap), and the FP64 CPU oracle timed on a bounded
sample.  Further sections (each can be switched off): the plain kiFMM
workload (20k points, dense M2L, FP64), moving points, BLAS-M2L with a finer
check surface, BLAS-M2L with 32 vectors in FP64 / FP32 / BF16x3 beside FP64
with one vector per launch, the 4M-point sphere with 64 vectors (FFT- and
BLAS-M2L, mixed against FP64), the batched serving workload and the 8M-point
uniform cube; errors against the FP64 direct sum at sampled targets.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "M2L ms & GB/s, Laplace 1M pts p=6: mixed/batched vs FP64, rel err ≤1e-5"
PEAK_HBM = 8.0e12           # bytes/s
PEAK_MFMA = {"fp32": 157.3e12, "fp64": 78.6e12, "bf16": 2500e12}
# Issue-slot model of the point kernels (bound "alu"): a SIMD issues one wave64
# VALU instruction per 4 cycles (16 lanes a cycle), a transcendental one
# (v_rsq_f32 / v_rsq_f64) per 16 cycles; 256 CUs x 4 SIMDs at 2.4 GHz.  VALU
# instructions per interaction, counted in the inner loops of this build's
# gfx950 assembly: near field (FP32 P2P) 42 + 4 v_rsq_f32 per 2 sources x 2
# targets; P2M (FP64) 48 + 3 v_rsq_f64 per source x 3 check points; L2P
# (FP64) 67 + 4 v_rsq_f64 per 2 equivalent points x 2 targets.
SIMDS, CLOCK_HZ = 256 * 4, 2.4e9
VALU_PER_PAIR = {"near_field": (42 / 4, 1.0), "p2m": (48 / 3, 1.0), "far_field": (67 / 4, 1.0)}


def pair_peak(kind):
    """Interactions per second at full VALU issue (the issue-slot model above)."""
    v, t = VALU_PER_PAIR[kind]
    return SIMDS * CLOCK_HZ * 64 / (4 * v + 16 * t)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(kernel_source: str, record: str):
    """HBM bytes per dispatch from the committed rocprofv3 counter record, or
    None when the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", record)
    try:
        with open(path) as fh:
            rec = json.load(fh)
        with open(os.path.join(ROOT, kernel_source), "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
    except OSError:
        return None
    if rec.get("source_sha256") != sha:
        return None
    return rec["traffic_bytes_per_dispatch"]


def m2l_work(f, depth, order, nvec, prec):
    """Algorithmic flops of the Hadamard launches and HBM bytes of the M2L."""
    n = 2 * order - 1
    F = n * n * (n // 2 + 1)
    ns = 6 * (order - 1) ** 2 + 2
    cb = 8 if prec == "fp32" else 16
    had_flops = 0.0
    had_bytes = 0.0
    m2l_bytes = 0.0
    for lev in range(2, depth + 1):
        c = f.m2l_counts(lev)
        had_flops += 8.0 * 64 * F * c["cluster_pairs"] * nvec
        spec = c["clusters"] * 8 * F * cb * nvec
        kern = 26 * 64 * F * cb
        had_bytes += 2 * spec + kern
        m2l_bytes += 2 * c["boxes"] * ns * 8 * nvec + 4 * spec + kern
    return had_flops, had_bytes, m2l_bytes


def leaf_level_m2l(torch, f, w, reps):
    """The leaf level's M2L on its own: one event-timed stage call at a time
    (forward transform, Hadamard, inverse) on synthetic FP64 densities."""
    lev = w.depth
    ns = 6 * (w.order - 1) ** 2 + 2
    g = torch.Generator(device="cuda")
    g.manual_seed(w.order * 1000 + lev)
    mult = torch.randn((f.num_boxes(lev), w.nvec, ns), dtype=torch.float64, device="cuda", generator=g)
    out = torch.empty_like(mult)
    for _ in range(3):
        f.stage_m2l(lev, mult, out)
    f.set_timing(True)
    acc = np.zeros(3)
    for _ in range(reps):
        f.stage_m2l(lev, mult, out)
        t = f.timings()
        acc += (t["m2l_first"], t["m2l_main"], t["m2l_last"])
    f.set_timing(False)
    torch.cuda.synchronize()
    return dict(zip(("fft_forward", "hadamard", "fft_inverse"), acc / reps))


def leaf_level_work(f, w, prec):
    """Algorithmic flops / HBM bytes of the leaf level's M2L kernels."""
    n = 2 * w.order - 1
    F = n * n * (n // 2 + 1)
    ns = 6 * (w.order - 1) ** 2 + 2
    cb = 8 if prec == "fp32" else 16
    c = f.m2l_counts(w.depth)
    spec = c["clusters"] * 8 * F * cb * w.nvec        # spectra of one side
    dens = c["boxes"] * ns * 8 * w.nvec               # FP64 densities / check potentials
    return {"hadamard_flops": 8.0 * 64 * F * c["cluster_pairs"] * w.nvec,
            "hadamard_bytes": 2 * spec + 26 * 64 * F * cb,
            "fft_forward_bytes": dens + spec, "fft_inverse_bytes": spec + dens}


def p2p_work(pts, depth):
    """Near-field interactions of the P2P (27-leaf neighbourhoods)."""
    a = np.minimum(np.floor(pts * 2 ** depth).astype(np.int64), 2 ** depth - 1)
    n = 2 ** depth
    counts = np.zeros((n + 2, n + 2, n + 2), dtype=np.int64)
    np.add.at(counts, (a[:, 0] + 1, a[:, 1] + 1, a[:, 2] + 1), 1)
    nb = np.zeros_like(counts)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                nb[1:-1, 1:-1, 1:-1] += counts[1 + dx:n + 1 + dx, 1 + dy:n + 1 + dy, 1 + dz:n + 1 + dz]
    return float(np.sum(counts[1:-1, 1:-1, 1:-1] * nb[1:-1, 1:-1, 1:-1]))


def run_precision(K, torch, w, prec, steps, warmup):
    dt = torch.float64 if prec == "fp64" else torch.float32
    t0 = time.perf_counter()
    f = K.KiFMM(w.order, w.depth, m2l="fft", prec=prec).set_points(w.points).precompute()
    setup_s = time.perf_counter() - t0
    q = torch.as_tensor(w.q, dtype=dt, device="cuda")
    out = torch.empty((w.nvec, w.n), dtype=dt, device="cuda")
    for _ in range(warmup):
        f.evaluate(q, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        f.evaluate(q, out)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) / steps * 1e3
    # per-kernel timing: HIP events recorded between launches on the stream
    f.set_timing(True)
    acc = {}
    for _ in range(steps):
        f.evaluate(q, out)
        for k, v in f.timings().items():
            acc[k] = acc.get(k, 0.0) + v
    f.set_timing(False)
    torch.cuda.synchronize()
    tm = {k: v / steps for k, v in acc.items()}
    tm["m2l_levels"] = int(round(tm["m2l_levels"]))
    return f, out, ms_step, tm, setup_s


def direct_potentials(torch, w, sample):
    """FP64 direct sum (Section 1's N-body sum, K = 0 for coincident points) of every
    charge vector at the sampled targets: (nvec, len(sample)) on the device."""
    src = torch.as_tensor(w.points, device="cuda")
    q = torch.as_tensor(np.ascontiguousarray(w.q.T), device="cuda")      # (n, nvec)
    tgt = src[torch.as_tensor(sample, device="cuda")]
    ref = torch.zeros((len(sample), w.nvec), dtype=torch.float64, device="cuda")
    for c in range(0, w.n, 65536):
        diff = tgt[:, None, :] - src[None, c:c + 65536, :]
        r2 = (diff * diff).sum(-1)
        inv = torch.where(r2 > 0, torch.rsqrt(torch.where(r2 > 0, r2, torch.ones_like(r2))),
                          torch.zeros_like(r2))
        ref += inv @ q[c:c + 65536]
    return (ref / (4 * np.pi)).T.contiguous()


def direct_errors(torch, w, phi, ref, sample):
    """Relative L2 errors against the FP64 direct sum at the sampled targets: the
    largest over the charge vectors and the Frobenius value over all of them."""
    got = phi[:, torch.as_tensor(sample, device="cuda")].double()
    per = torch.linalg.norm(got - ref, dim=1) / torch.linalg.norm(ref, dim=1)
    return {"max_over_vectors": float(per.max()),
            "frobenius": float(torch.linalg.norm(got - ref) / torch.linalg.norm(ref))}


def direct_error(torch, w, phi, n_sample=1000):
    """Relative L2 error of the first charge vector against the FP64 direct sum at
    sampled targets."""
    import workloads
    s = workloads.sample_indices(w.n, n_sample, workloads.SEED_SAMPLES + 2)
    w1 = workloads.Workload(w.name, w.points, w.q[:1], w.depth, w.order, w.origin, w.width, w.m2l)
    ref = direct_potentials(torch, w1, s)
    return direct_errors(torch, w1, phi[:1], ref, s)["frobenius"]


def run_blas(K, torch, steps, warmup):
    """The 32-vector BLAS-M2L workload in FP64, FP32, bf16x3 and bf16x6."""
    import workloads
    w = workloads.config(3)
    out = {"workload": w.name, "n_vec": w.nvec, "svd_rel_tol": 1e-6, "svd_rel_tol_dir": 1e-6}
    ref_phi = None
    flops = None
    sample = workloads.sample_indices(w.n, 1000, workloads.SEED_SAMPLES + 3)
    ref_direct = direct_potentials(torch, w, sample)
    for prec in ("fp64", "fp32", "bf16x3", "bf16x6"):
        dt = torch.float64 if prec == "fp64" else torch.float32
        t0 = time.perf_counter()
        f = K.KiFMM(w.order, w.depth, m2l="blas", prec=prec, svd_rel_tol=1e-6,
                    svd_rel_tol_dir=1e-6).set_points(w.points)
        t1 = time.perf_counter()
        f.precompute()
        precompute_s = time.perf_counter() - t1
        setup_s = time.perf_counter() - t0
        if flops is None:
            ranks = f.operator(K.OP_BLAS_RANKS)
            k, kt = int(ranks[0]), ranks[1:]
            flops = 0.0
            for lev in range(2, w.depth + 1):
                _, _, tid = f.interactions(lev)
                cnt = np.bincount(tid, minlength=316)
                flops += float(np.sum(cnt * 4.0 * k * kt)) * w.nvec
            out["k"] = k
            out["kt_mean"] = round(float(kt.mean()), 2)
        q = torch.as_tensor(w.q, dtype=dt, device="cuda")
        phi = torch.empty((w.nvec, w.n), dtype=dt, device="cuda")
        tune_ms = f.autotune(q, phi, reps=2)
        tuning = f.tuning()
        # BF16x6 has only the stacked form, whatever the form knob holds
        form = "stacked" if prec == "bf16x6" else ("stacked", "fused")[tuning["blas_form"]]
        for _ in range(warmup):
            f.evaluate(q, phi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            f.evaluate(q, phi)
        torch.cuda.synchronize()
        ms_step = (time.perf_counter() - t0) / steps * 1e3
        f.set_timing(True)
        acc = {}
        for _ in range(steps):
            f.evaluate(q, phi)
            for kk, v in f.timings().items():
                acc[kk] = acc.get(kk, 0.0) + v
        f.set_timing(False)
        tm = {kk: v / steps for kk, v in acc.items()}
        if ref_phi is None:
            ref_phi = phi.double().clone()
        rel = float(torch.linalg.norm(phi.double() - ref_phi) / torch.linalg.norm(ref_phi))
        derr = direct_errors(torch, w, phi, ref_direct, sample)
        main_s = tm["m2l_main"] * 1e-3
        peak = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16x3": 2500e12 / 3, "bf16x6": 2500e12 / 6}[prec]
        out[prec] = {"m2l_ms": round(tm["m2l"], 3), "m2l_ms_per_vector": round(tm["m2l"] / w.nvec, 4),
                     "fused_kernel_ms": round(tm["m2l_main"], 3), "ms_per_step": round(ms_step, 3),
                     "fused_tflops": round(flops / main_s / 1e12, 2),
                     "fused_frac_of_peak": round(flops / main_s / peak, 4),
                     "rel_err_vs_fp64_run": rel, "rel_err_vs_direct": derr,
                     "setup_s": round(setup_s, 2),
                     "precompute_s": round(precompute_s, 3),
                     "autotuned_tile_boxes": tuning["blas_tile"],
                     "autotuned_form": form,
                     "autotune_best_ms": round(tune_ms, 3)}
        log(f"  blas {prec}: step {ms_step:.2f} ms, m2l {tm['m2l']:.2f} ms (fused {tm['m2l_main']:.2f}), "
            f"{flops / main_s / 1e12:.1f} TFLOP/s, rel vs fp64 {rel:.2e}, vs direct "
            f"{derr['max_over_vectors']:.2e} (max over vectors), autotuned tile {tuning['blas_tile']} boxes, "
            f"form {form}")
        if prec == "fp64":
            # the plain FP64 comparator: the same M2L form, one charge vector per launch
            q1 = q[:1].contiguous()
            phi1 = torch.empty((1, w.n), dtype=dt, device="cuda")
            f.autotune(q1, phi1, reps=2)
            out["fp64_one_rhs_per_launch"] = one_rhs_m2l(torch, f, q1, phi1, steps)
            out["fp64_one_rhs_per_launch"]["autotuned_tile_boxes"] = f.tuning()["blas_tile"]
            out["fp64_one_rhs_per_launch"]["autotuned_form"] = ("stacked", "fused")[f.tuning()["blas_form"]]
            log(f"  blas fp64, one vector per launch: m2l {out['fp64_one_rhs_per_launch']['m2l_ms']:.3f} ms")
        del f, q, phi
        torch.cuda.empty_cache()
    # K_fat compressed by the one-shot randomized SVD on the device (rank k + 4,
    # oversampling 10) instead of the deterministic host SVD, FP64 operators
    rank = out["k"] + 4
    f = K.KiFMM(w.order, w.depth, m2l="blas", prec="fp64", svd_rel_tol=1e-6, svd_rel_tol_dir=1e-6)
    f.set_svd("randomized", rank=rank, oversample=10, seed=1).set_points(w.points)
    t1 = time.perf_counter()
    f.precompute()
    rnd_s = time.perf_counter() - t1
    q = torch.as_tensor(w.q, dtype=torch.float64, device="cuda")
    phi = torch.empty((w.nvec, w.n), dtype=torch.float64, device="cuda")
    f.evaluate(q, phi)
    torch.cuda.synchronize()
    rel = float(torch.linalg.norm(phi - ref_phi) / torch.linalg.norm(ref_phi))
    out["randomized_svd"] = {"precompute_s": round(rnd_s, 3),
                             "deterministic_precompute_s": out["fp64"]["precompute_s"],
                             "rank": rank, "oversample": 10, "k": int(f.operator(K.OP_BLAS_RANKS)[0]),
                             "rel_diff_vs_deterministic_fp64": rel}
    log(f"  blas fp64 randomized SVD: precompute {rnd_s:.3f} s (deterministic "
        f"{out['fp64']['precompute_s']:.3f} s), potentials vs deterministic {rel:.2e}")
    del f, q, phi
    torch.cuda.empty_cache()
    out["algorithmic_gflop"] = round(flops / 1e9, 1)
    out["peaks_tflops"] = {"fp64": 78.6, "fp32": 157.3, "bf16x3": round(2500 / 3, 1), "bf16x6": round(2500 / 6, 1)}
    one = out["fp64_one_rhs_per_launch"]["m2l_ms"]
    out["m2l_per_vector_speedup_vs_fp64_one_rhs"] = {
        p: round(one / out[p]["m2l_ms_per_vector"], 2) for p in ("fp64", "fp32", "bf16x3", "bf16x6")}
    out["error_targets"] = len(sample)
    return out


def one_rhs_m2l(torch, f, q1, phi1, steps):
    """M2L time of evaluates with one charge vector (timed evaluates, HIP events)."""
    f.evaluate(q1, phi1)
    f.set_timing(True)
    m2l = 0.0
    for _ in range(steps):
        f.evaluate(q1, phi1)
        m2l += f.timings()["m2l"]
    f.set_timing(False)
    torch.cuda.synchronize()
    return {"m2l_ms": round(m2l / steps, 4)}


def run_check_order(K, torch, w, steps):
    """BLAS-M2L (FP64, SVD tolerance 1e-6, no directional recompression: a configuration
    no other section precomputes, so both setups are timed uncached) on the main
    workload with check surfaces of the expansion order and of one order more: setup,
    M2L time and the error against the FP64 direct sum."""
    out = {"workload": w.name + " (BLAS-M2L FP64, tol 1e-6, no recompression)", "order": w.order}
    q = torch.as_tensor(w.q, dtype=torch.float64, device="cuda")
    for pc in (w.order, w.order + 1):
        f = K.KiFMM(w.order, w.depth, m2l="blas", prec="fp64", svd_rel_tol=1e-6, svd_rel_tol_dir=-1.0,
                    check_order=pc).set_points(w.points)
        t0 = time.perf_counter()
        f.precompute()
        pre_s = time.perf_counter() - t0
        phi = torch.empty((w.nvec, w.n), dtype=torch.float64, device="cuda")
        f.evaluate(q, phi)
        f.set_timing(True)
        m2l = 0.0
        for _ in range(steps):
            f.evaluate(q, phi)
            m2l += f.timings()["m2l"]
        f.set_timing(False)
        torch.cuda.synchronize()
        err = direct_error(torch, w, phi)
        out[f"check_order_{pc}"] = {"n_check": 6 * (pc - 1) ** 2 + 2, "precompute_s": round(pre_s, 2),
                                    "k": int(f.operator(K.OP_BLAS_RANKS)[0]),
                                    "m2l_ms": round(m2l / steps, 3), "rel_err_vs_direct": err}
        log(f"  blas fp64 check order {pc}: m2l {m2l / steps:.3f} ms, err vs direct {err:.2e}, "
            f"precompute {pre_s:.2f} s")
        del f, phi
        torch.cuda.empty_cache()
    return out


def run_scale(K, torch, steps, warmup):
    """The paper's larger problem size: 8,000,000 uniform points, depth 6, p = 6,
    FFT-M2L, mixed and FP64, with the error against the FP64 direct sum."""
    import workloads
    w = workloads.config(6)
    out = {"workload": w.name, "n_points": w.n, "depth": w.depth, "order": w.order, "n_vec": w.nvec}
    for prec in ("fp32", "fp64"):
        f, phi, ms_step, tm, setup_s = run_precision(K, torch, w, prec, steps, warmup)
        err = direct_error(torch, w, phi)
        out[prec] = {"ms_per_step": round(ms_step, 3), "m2l_ms": round(tm["m2l"], 3),
                     "near_field_ms": round(tm["near_field"], 3), "setup_s": round(setup_s, 2),
                     "rel_err_vs_direct": err}
        log(f"  8M {prec}: step {ms_step:.2f} ms, m2l {tm['m2l']:.3f} ms, near field "
            f"{tm['near_field']:.3f} ms, err vs direct {err:.2e}")
        del f, phi
        torch.cuda.empty_cache()
    out["m2l_speedup_mixed_vs_fp64"] = round(out["fp64"]["m2l_ms"] / out["fp32"]["m2l_ms"], 3)
    out["error_targets"] = 1000
    return out


def timed_run(torch, f, q, phi, steps, warmup):
    """Wall time per evaluate (synchronised) and the event-timed phases."""
    for _ in range(warmup):
        f.evaluate(q, phi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        f.evaluate(q, phi)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) / steps * 1e3
    f.set_timing(True)
    acc = {}
    for _ in range(steps):
        f.evaluate(q, phi)
        for kk, v in f.timings().items():
            acc[kk] = acc.get(kk, 0.0) + v
    f.set_timing(False)
    torch.cuda.synchronize()
    return ms_step, {kk: v / steps for kk, v in acc.items()}


def run_sphere(K, torch, steps, warmup):
    """The non-uniform workload: 4,000,000 points on the unit sphere (domain [-1,1]^3,
    depth 6, empty boxes pruned), p = 6, 64 standard-normal charge vectors.  FFT-M2L in
    FP32 complex and FP64, BLAS-M2L (SVD tolerance 1e-6 / 1e-6) in FP32, BF16x3 and FP64,
    all 64 vectors through each launch, beside the plain FP64 form with one vector per
    launch; errors of every vector against the FP64 direct sum at 1,000 sampled targets."""
    import workloads
    w = workloads.config(4)
    sample = workloads.sample_indices(w.n, 1000, workloads.SEED_SAMPLES + 4)
    ref = direct_potentials(torch, w, sample)
    out = {"workload": w.name, "n_points": w.n, "depth": w.depth, "order": w.order, "n_vec": w.nvec,
           "error_targets": len(sample)}
    for m2l, precs in (("fft", ("fp32", "fp64")), ("blas", ("fp32", "bf16x3", "bf16x6", "fp64"))):
        for prec in precs:
            dt = torch.float64 if prec == "fp64" else torch.float32
            kw = dict(svd_rel_tol=1e-6, svd_rel_tol_dir=1e-6) if m2l == "blas" else {}
            t0 = time.perf_counter()
            f = K.KiFMM(w.order, w.depth, m2l=m2l, prec=prec, origin=w.origin, width=w.width,
                        **kw).set_points(w.points).precompute()
            setup_s = time.perf_counter() - t0
            q = torch.as_tensor(w.q, dtype=dt, device="cuda")
            phi = torch.empty((w.nvec, w.n), dtype=dt, device="cuda")
            if m2l == "blas":
                f.autotune(q, phi, reps=2)
            ms_step, tm = timed_run(torch, f, q, phi, steps, warmup)
            derr = direct_errors(torch, w, phi, ref, sample)
            key = f"{m2l}_{prec}"
            out[key] = {"ms_per_step": round(ms_step, 3), "m2l_ms": round(tm["m2l"], 3),
                        "m2l_ms_per_vector": round(tm["m2l"] / w.nvec, 4),
                        "m2l_main_kernel_ms": round(tm["m2l_main"], 3),
                        "setup_s": round(setup_s, 2), "rel_err_vs_direct": derr}
            log(f"  sphere {key}: step {ms_step:.2f} ms, m2l {tm['m2l']:.3f} ms "
                f"({tm['m2l'] / w.nvec:.4f} per vector), err vs direct {derr['max_over_vectors']:.2e}")
            if prec == "fp64":
                q1 = q[:1].contiguous()
                phi1 = torch.empty((1, w.n), dtype=dt, device="cuda")
                if m2l == "blas":
                    f.autotune(q1, phi1, reps=2)
                one = one_rhs_m2l(torch, f, q1, phi1, steps)
                out[f"{m2l}_fp64_one_rhs_per_launch"] = one
                log(f"  sphere {m2l} fp64, one vector per launch: m2l {one['m2l_ms']:.3f} ms")
                del q1, phi1
            f.close()
            del f, q, phi
            torch.cuda.empty_cache()
    for m2l, mixed in (("fft", ("fp32",)), ("blas", ("fp32", "bf16x3", "bf16x6"))):
        one = out[f"{m2l}_fp64_one_rhs_per_launch"]["m2l_ms"]
        for prec in mixed + ("fp64",):
            out[f"{m2l}_{prec}"]["m2l_per_vector_speedup_vs_fp64_one_rhs"] = round(
                one / out[f"{m2l}_{prec}"]["m2l_ms_per_vector"], 2)
    return out


def run_plain(K, torch, steps, warmup):
    """The plain kiFMM workload: 20,000 uniform points, depth 3, p = 3, dense M2L in
    FP64, one vector; error against the FP64 direct sum at every target."""
    import workloads
    w = workloads.config(1)
    f = K.KiFMM(w.order, w.depth, m2l="dense", prec="fp64").set_points(w.points).precompute()
    q = torch.as_tensor(w.q, device="cuda")
    phi = torch.empty((w.nvec, w.n), dtype=torch.float64, device="cuda")
    ms_step, tm = timed_run(torch, f, q, phi, steps, warmup)
    sample = np.arange(w.n)
    derr = direct_errors(torch, w, phi, direct_potentials(torch, w, sample), sample)
    out = {"workload": w.name, "ms_per_step": round(ms_step, 4), "m2l_ms": round(tm["m2l"], 4),
           "upward_ms": round(tm["upward"], 4), "downward_ms": round(tm["downward"], 4),
           "leaves_ms": round(tm["leaves"], 4), "rel_err_vs_direct_all_targets": derr["frobenius"]}
    log(f"  plain kiFMM 20k: step {ms_step:.3f} ms, m2l {tm['m2l']:.4f} ms, err vs direct "
        f"{derr['frobenius']:.2e}")
    f.close()
    return out


def run_resetup(K, torch, w, reps=3):
    """Moving points (the dynamic-particle re-setup of Section 5.1) on the 1M
    workload: the host tree build (kifmm_set_points, plus the upload and tile
    build of the first evaluate) against the device re-setup
    (kifmm_update_points) for moves that keep the leaves (new point order and
    ranges) and moves that change the box set (levels, near and interaction
    lists, FFT-M2L halos and source blocks rebuilt on the device; BLAS-M2L
    target tiles at the next evaluate, timed as that evaluate's extra time)."""
    import workloads
    out = {"n_points": w.n, "depth": w.depth}
    c = np.array([0.5, 0.5, 0.5])
    moves = [c + 0.6 * (workloads.uniform_cube(w.n, 9100 + r) - c) + 0.05 * r for r in range(reps)]
    for m2l in ("fft", "blas"):
        kw = dict(svd_rel_tol=1e-6, svd_rel_tol_dir=1e-6) if m2l == "blas" else {}
        t0 = time.perf_counter()
        f = K.KiFMM(w.order, w.depth, m2l=m2l, prec="fp32", **kw).set_points(w.points)
        host_ms = (time.perf_counter() - t0) * 1e3
        f.precompute()
        q = torch.as_tensor(w.q[:1], dtype=torch.float32, device="cuda")

        def timed_eval():
            torch.cuda.synchronize()
            t = time.perf_counter()
            f.evaluate(q)
            torch.cuda.synchronize()
            return (time.perf_counter() - t) * 1e3

        first_ms = timed_eval()
        steady_ms = float(np.median([timed_eval() for _ in range(3)]))
        same, new, extra, boxes = [], [], [], []
        for r in range(reps):
            # same leaves: every leaf of the 1M cube stays occupied
            pts = torch.as_tensor(workloads.uniform_cube(w.n, 9000 + r), device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f.update_points(pts)
            torch.cuda.synchronize()
            same.append((time.perf_counter() - t0) * 1e3)
            timed_eval()
            # a new box set: the points contracted into a smaller cube
            pts = torch.as_tensor(moves[r], device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f.update_points(pts)
            torch.cuda.synchronize()
            new.append((time.perf_counter() - t0) * 1e3)
            boxes.append(f.num_boxes(w.depth))
            extra.append(timed_eval() - steady_ms)
        out[m2l] = {"host_set_points_ms": round(host_ms, 2),
                    "host_first_evaluate_extra_ms": round(first_ms - steady_ms, 2),
                    "device_update_same_leaves_ms": round(float(np.median(same)), 3),
                    "device_update_new_box_set_ms": round(float(np.median(new)), 3),
                    "first_evaluate_extra_after_rebuild_ms": round(float(np.median(extra)), 3),
                    "leaves_after_move": int(np.median(boxes))}
        log(f"  {m2l}: host tree build {host_ms:.1f} ms (+{first_ms - steady_ms:.1f} ms upload at the "
            f"first evaluate); device re-setup, same leaves {np.median(same):.2f} ms, new box set "
            f"{np.median(new):.2f} ms (+{np.median(extra):.2f} ms at the next evaluate)")
        del f, q
        torch.cuda.empty_cache()
    return out


def run_batch(K, torch, launches):
    """128 independent problems (log-uniform sizes 1e4..2e5, depth 3-4,
    p in {4,5,6}, 1-8 vectors), FFT-M2L in FP32 with FP64 local
    accumulation, replayed as one graph launch."""
    import workloads
    specs = workloads.batch_problems(128)
    t0 = time.perf_counter()
    items = []
    total_pts = 0
    for sp in specs:
        pts = workloads.uniform_cube(sp["n"], sp["seed_points"])
        q = workloads.charges(sp["n"], sp["nvec"], sp["seed_charges"], "u01")
        f = K.KiFMM(sp["order"], sp["depth"], m2l="fft", prec="fp32").set_points(pts).precompute()
        qt = torch.as_tensor(q, dtype=torch.float32, device="cuda")
        phi = torch.empty((sp["nvec"], sp["n"]), dtype=torch.float32, device="cuda")
        items.append((f, qt, phi))
        total_pts += sp["n"]
    setup_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    b = K.Batch(items, autotune=True, reps=3)
    capture_s = time.perf_counter() - t0
    info = b.info()
    s = torch.cuda.current_stream()
    for _ in range(5):
        b.launch()
    torch.cuda.synchronize()
    dev_ms, host_ms = [], []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(launches):
        t0 = time.perf_counter()
        ev0.record(s)
        b.launch()
        ev1.record(s)
        ev1.synchronize()
        host_ms.append((time.perf_counter() - t0) * 1e3)
        dev_ms.append(ev0.elapsed_time(ev1))
    dev = np.array(dev_ms)
    host = np.array(host_ms)
    # the same problems evaluated one by one (eager, one stream) for comparison
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        for f, qt, phi in items:
            f.evaluate(qt, phi)
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) / 3 * 1e3
    b.close()
    p50 = float(np.percentile(host, 50))
    out = {"problems": len(items), "total_points": total_pts,
           "total_vectors": int(sum(sp["nvec"] for sp in specs)),
           "launches": launches,
           "latency_ms_p50": round(p50, 3), "latency_ms_p99": round(float(np.percentile(host, 99)), 3),
           "device_ms_p50": round(float(np.percentile(dev, 50)), 3),
           "device_ms_p99": round(float(np.percentile(dev, 99)), 3),
           "problems_per_s": round(len(items) / (p50 * 1e-3), 1),
           "points_per_s": round(total_pts / (p50 * 1e-3), 1),
           "eager_sequential_ms": round(eager_ms, 3),
           "setup_s": round(setup_s, 2), "autotune_and_capture_s": round(capture_s, 2),
           "launches_per_replay": info["launches"], "grouped_launches": info["grouped"],
           "autotune_best_ms": round(b.best_ms, 3),
           "precision": "fp32 M2L, fp64 local accumulation", "m2l": "fft"}
    log(f"  batch: p50 {p50:.2f} ms, p99 {out['latency_ms_p99']:.2f} ms, eager sequential {eager_ms:.2f} ms, "
        f"{info['launches']} launches per replay ({info['grouped']} grouped)")
    del items
    torch.cuda.empty_cache()
    return out


def cpu_baseline(w, min_seconds=10.0, max_reps=3):
    """FP64 oracle dense M2L of every level (the whole M2L of one evaluate), timed on the
    host cores; repeated until about ten seconds of CPU work (at most three times)."""
    from oracle import fmm
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    ora = fmm.KiFMM(w.points, w.points, w.depth, w.order)
    rng = np.random.default_rng(7)
    levels = list(range(2, w.depth + 1))
    mult, total_pairs = {}, 0
    for lev in levels:
        offs, _, _ = ora.tree.interactions(lev)
        total_pairs += int(offs[-1])
        mult[lev] = rng.standard_normal((len(ora.tree.levels[lev]), ora.ns, w.nvec))
    reps, elapsed = 0, 0.0
    while reps < max_reps and (reps == 0 or elapsed < min_seconds):
        t0 = time.perf_counter()
        for lev in levels:
            ora.m2l_level(lev, mult[lev], np.arange(len(ora.tree.levels[lev])))
        elapsed += time.perf_counter() - t0
        reps += 1
    return {"value": round(elapsed * 1e3 / reps, 1), "unit": "ms (M2L per evaluate, all levels, FP64)",
            "cores": int(threads), "kind": "oracle",
            "sample": f"complete dense M2L of levels 2-{w.depth} (every target box, {total_pairs} "
                      f"M2L pairs), {reps} repetitions, {elapsed:.1f} s in total",
            "host_cpus": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-blas", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-scale", action="store_true")
    ap.add_argument("--no-resetup", action="store_true")
    ap.add_argument("--no-check-order", action="store_true")
    ap.add_argument("--no-sphere", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the FMM here is a single-GPU build; "
              "use --gpus 1", file=sys.stderr)
        return 2
    import torch
    import paper_2408_07436_amd as K
    import workloads

    w = workloads.config(2)
    log(f"workload {w.name}: n={w.n} depth={w.depth} p={w.order} nvec={w.nvec}")
    res = {}
    for prec in ("fp32", "fp64"):
        log(f"run {prec}: warmup {args.warmup}, steps {args.steps}")
        f, out, ms_step, tm, setup_s = run_precision(K, torch, w, prec, args.steps, args.warmup)
        err = direct_error(torch, w, out)
        res[prec] = dict(f=f, out=out, ms_step=ms_step, tm=tm, setup_s=setup_s, err=err)
        log(f"  {prec}: step {ms_step:.3f} ms; phases: upward {tm['upward']:.3f}, m2l {tm['m2l']:.3f} "
            f"(kernel sums fwd {tm['m2l_first']:.3f} had {tm['m2l_main']:.3f} inv {tm['m2l_last']:.3f}), "
            f"downward {tm['downward']:.3f}, near field {tm['near_field']:.3f}, far field "
            f"{tm['far_field']:.3f} ms; err vs direct {err:.2e}")
    mix, ref = res["fp32"], res["fp64"]
    rel_mix_vs_fp64 = float(torch.linalg.norm(mix["out"].double() - ref["out"]) / torch.linalg.norm(ref["out"]))

    had_flops, had_bytes, m2l_bytes = m2l_work(mix["f"], w.depth, w.order, w.nvec, "fp32")
    tm = mix["tm"]
    # the leaf level's M2L kernels timed on their own (levels overlap inside
    # an evaluate, so per-kernel times come from single-level stage calls)
    lk = leaf_level_m2l(torch, mix["f"], w, args.steps)
    lw = leaf_level_work(mix["f"], w, "fp32")
    log(f"  leaf-level M2L kernels (level {w.depth}, alone): fwd {lk['fft_forward']:.4f} "
        f"had {lk['hadamard']:.4f} inv {lk['fft_inverse']:.4f} ms")
    # the same Hadamard with its products on FP32 MFMA (the other product form)
    mix["f"].set_tuning(products=1)
    lk_f32 = leaf_level_m2l(torch, mix["f"], w, args.steps)
    mix["f"].set_tuning(products=0)
    log(f"  leaf-level Hadamard with FP32 MFMA products: {lk_f32['hadamard']:.4f} ms")
    # the same for the FP64 run (its Hadamard is the gather form on FP64 MFMA)
    lk64 = leaf_level_m2l(torch, ref["f"], w, args.steps)
    lw64 = leaf_level_work(ref["f"], w, "fp64")
    log(f"  leaf-level M2L kernels, fp64 (level {w.depth}, alone): fwd {lk64['fft_forward']:.4f} "
        f"had {lk64['hadamard']:.4f} inv {lk64['fft_inverse']:.4f} ms")
    interactions = p2p_work(w.points, w.depth)
    # the headline metric is the M2L's time, so its dominant kernel (the
    # longest of the leaf level's three M2L kernels) carries `roofline`; the
    # near field, about as long, is reported with the others
    kernels = dict(lk)
    dominant = max(kernels, key=kernels.get)
    had_s = lk["hadamard"] * 1e-3
    # the FP32 Hadamard runs as BF16 MFMAs: six part products per FP32
    # product, so its MFMA work is 6x the method's flops, against the BF16 peak
    roof_had = {"kernel": "hadamard_split_kernel (v_mfma_f32_16x16x32_bf16: FP32 operands as three BF16 "
                          "parts, six part products per FP32 product), leaf level", "bound": "mfma",
                "achieved": 6.0 * lw["hadamard_flops"] / had_s / 1e12, "peak": PEAK_MFMA["bf16"] / 1e12,
                "unit": "TFLOP/s",
                "traffic": measured_traffic("paper_2408_07436_amd/csrc/k_fft.hip",
                                            "hadamard_f32_uniform1M_p6_traffic.json"),
                "algorithmic_bytes": round(lw["hadamard_bytes"]),
                "fp32_equivalent": {"achieved": round(lw["hadamard_flops"] / had_s / 1e12, 2),
                                    "fp32_mfma_peak": PEAK_MFMA["fp32"] / 1e12,
                                    "fp32_mfma_form_ms": round(lk_f32["hadamard"], 4)},
                "per_launch": f"{lw['hadamard_flops'] / 1e9:.2f} GFLOP of FP32 complex products (8 flops x "
                              f"64 pairs x F per cluster pair at level {w.depth}), run as "
                              f"{6 * lw['hadamard_flops'] / 1e9:.1f} GFLOP of BF16 MFMA, avg "
                              f"{lk['hadamard']:.4f} ms"}
    roof_had["frac"] = roof_had["achieved"] / roof_had["peak"]
    fwd_s, inv_s = lk["fft_forward"] * 1e-3, lk["fft_inverse"] * 1e-3
    roof_fwd = {"kernel": "fft_forward_kernel<float, 6>, leaf level", "bound": "hbm",
                "achieved": lw["fft_forward_bytes"] / fwd_s / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s",
                "traffic": measured_traffic("paper_2408_07436_amd/csrc/k_fft.hip",
                                            "fft_forward_f32_uniform1M_p6_traffic.json"),
                "per_launch": f"{lw['fft_forward_bytes'] / 1e6:.1f} MB (FP64 densities in, FP32 "
                              f"spectra out), avg {lk['fft_forward']:.4f} ms"}
    roof_inv = {"kernel": "fft_inverse_kernel<float, 6>, leaf level", "bound": "hbm",
                "achieved": lw["fft_inverse_bytes"] / inv_s / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s",
                "traffic": measured_traffic("paper_2408_07436_amd/csrc/k_fft.hip",
                                            "fft_inverse_f32_uniform1M_p6_traffic.json"),
                "per_launch": f"{lw['fft_inverse_bytes'] / 1e6:.1f} MB (FP32 products in, FP64 "
                              f"check potentials out), avg {lk['fft_inverse']:.4f} ms"}
    roof_had64 = {"kernel": "hadamard_gather_kernel<double> (v_mfma_f64_16x16x4f64), leaf level, FP64 run",
                  "bound": "mfma", "achieved": lw64["hadamard_flops"] / (lk64["hadamard"] * 1e-3) / 1e12,
                  "peak": PEAK_MFMA["fp64"] / 1e12, "unit": "TFLOP/s", "traffic": None,
                  "algorithmic_bytes": round(lw64["hadamard_bytes"]),
                  "per_launch": f"{lw64['hadamard_flops'] / 1e9:.2f} GFLOP, avg {lk64['hadamard']:.4f} ms"}
    for r in (roof_fwd, roof_inv, roof_had64):
        r["frac"] = r["achieved"] / r["peak"]
    near_s = tm["near_field"] * 1e-3
    # interactions per second against the issue-slot peak (VALU_PER_PAIR)
    roof_leaf = {"kernel": "leaf_eval_kernel<float, float, 1, 1> (near field, P2P FP32)", "bound": "alu",
                 "achieved": interactions / near_s / 1e9, "peak": pair_peak("near_field") / 1e9,
                 "unit": "Ginteractions/s",
                 "traffic": measured_traffic("paper_2408_07436_amd/csrc/k_leaf.hip",
                                             "leaf_eval_f32_uniform1M_p6_traffic.json"),
                 "per_launch": f"{interactions:.3e} P2P interactions, avg {tm['near_field']:.4f} ms; peak: "
                               f"{VALU_PER_PAIR['near_field'][0]} VALU + 1 v_rsq_f32 per interaction at "
                               f"full issue"}
    roof_leaf["frac"] = roof_leaf["achieved"] / roof_leaf["peak"]
    # the passes around the M2L (mixed run): P2M and L2P on the FP64 VALU
    # (issue-slot model, as for P2P), the composite-operator GEMMs of the
    # upward and downward passes on FP64 MFMA
    ns = 6 * (w.order - 1) ** 2 + 2
    nb = [mix["f"].num_boxes(lev) for lev in range(w.depth + 1)]
    up_flops = 2.0 * ns * ns * nb[w.depth] * w.nvec + sum(
        2.0 * ns * 8 * ns * nb[lev] * w.nvec for lev in range(2, w.depth))
    down_flops = sum(2.0 * ns * ns * nb[lev] * w.nvec for lev in range(2, w.depth + 1)) + sum(
        2.0 * 8 * ns * ns * nb[lev - 1] * w.nvec for lev in range(3, w.depth + 1))
    surf_pairs = float(ns) * w.n
    roof_p2m = {"kernel": "p2m_kernel (FP64, leaf check potentials)", "bound": "alu",
                "achieved": surf_pairs / (tm["p2m"] * 1e-3) / 1e9,
                "peak": pair_peak("p2m") / 1e9, "unit": "Ginteractions/s", "traffic": None,
                "per_launch": f"{surf_pairs:.3e} (check point, source) pairs, avg {tm['p2m']:.4f} ms; "
                              f"peak: {VALU_PER_PAIR['p2m'][0]} VALU + 1 v_rsq_f64 per pair"}
    roof_l2p = {"kernel": "leaf_eval_kernel<float, float, 1, 2> (far field, L2P FP64)", "bound": "alu",
                "achieved": surf_pairs / (tm["far_field"] * 1e-3) / 1e9,
                "peak": pair_peak("far_field") / 1e9, "unit": "Ginteractions/s", "traffic": None,
                "per_launch": f"{surf_pairs:.3e} (target, equivalent point) pairs, avg "
                              f"{tm['far_field']:.4f} ms; peak: {VALU_PER_PAIR['far_field'][0]} VALU + "
                              f"1 v_rsq_f64 per pair"}
    up_gemm_ms = tm["upward"] - tm["p2m"]
    roof_up = {"kernel": "gemm64_kernel, upward pass (leaf pseudo-inverse, M2M with it folded in)",
               "bound": "mfma", "achieved": up_flops / (up_gemm_ms * 1e-3) / 1e12,
               "peak": PEAK_MFMA["fp64"] / 1e12, "unit": "TFLOP/s", "traffic": None,
               "per_launch": f"{up_flops / 1e9:.2f} GFLOP per evaluate, {up_gemm_ms:.4f} ms "
                             f"(upward phase minus P2M, includes the charge gather)"}
    roof_down = {"kernel": "gemm64_kernel, downward pass (down pseudo-inverse, L2L with it folded in)",
                 "bound": "mfma", "achieved": down_flops / (tm["downward"] * 1e-3) / 1e12,
                 "peak": PEAK_MFMA["fp64"] / 1e12, "unit": "TFLOP/s", "traffic": None,
                 "per_launch": f"{down_flops / 1e9:.2f} GFLOP per evaluate, {tm['downward']:.4f} ms"}
    for r in (roof_p2m, roof_l2p, roof_up, roof_down):
        r["frac"] = r["achieved"] / r["peak"]
    roofs = {"hadamard": roof_had, "fft_forward": roof_fwd, "fft_inverse": roof_inv,
             "hadamard_fp64": roof_had64, "near_field": roof_leaf,
             "p2m": roof_p2m, "far_field": roof_l2p, "upward_gemm": roof_up, "downward_gemm": roof_down}
    for r in roofs.values():
        for k in ("achieved", "peak", "frac"):
            r[k] = round(r[k], 4)
    roofline = roofs[dominant]

    m2l_ms = tm["m2l"]
    line = {
        "metric": METRIC,
        "value": round(m2l_ms, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mix["ms_step"], 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP32 complex M2L, Hadamard products as three-part BF16 on MFMA, FP64 local "
                 "accumulation)",
        "data": "synthetic",
        "config": {"workload": w.name, "n_points": w.n, "depth": w.depth, "order": w.order,
                   "n_vec": w.nvec, "m2l": "fft", "distribution": "uniform unit cube, seed 1002"},
        "m2l_gbps": round(m2l_bytes / (m2l_ms * 1e-3) / 1e9, 1),
        "m2l_ms_fp64": round(ref["tm"]["m2l"], 4),
        "m2l_gbps_fp64": round(m2l_work(ref["f"], w.depth, w.order, w.nvec, "fp64")[2]
                               / (ref["tm"]["m2l"] * 1e-3) / 1e9, 1),
        "m2l_speedup_mixed_vs_fp64": round(ref["tm"]["m2l"] / m2l_ms, 3),
        "ms_per_step_fp64": round(ref["ms_step"], 4),
        "rel_err_vs_direct": {"mixed": mix["err"], "fp64": ref["err"], "targets": 1000},
        "rel_err_mixed_vs_fp64": rel_mix_vs_fp64,
        "stage_ms": {k: round(v, 4) for k, v in tm.items() if k != "m2l_levels"},
        "stage_ms_fp64": {k: round(v, 4) for k, v in ref["tm"].items() if k != "m2l_levels"},
        "roofline": roofline,
        "roofline_other": [r for k, r in roofs.items() if k != dominant],
        "leaf_level_m2l_kernel_ms": {k: round(v, 4) for k, v in lk.items()},
        "leaf_level_m2l_kernel_ms_fp64": {k: round(v, 4) for k, v in lk64.items()},
        "paper_context": "FFT-M2L FP64, N=1e6, P=6, depth 5: T_M2L 813 ms on Apple M1 Pro "
                         "(8 cores); 240 ms on AMD 3790X at depth 4 (32 cores) - CPU context only",
        "setup_s": {"fp32": round(mix["setup_s"], 2), "fp64": round(ref["setup_s"], 2)},
    }
    if not args.no_plain:
        log("plain kiFMM workload: 20k points, dense M2L, fp64")
        line["plain_20k"] = run_plain(K, torch, args.steps, args.warmup)
    # the BLAS section first: operators are cached per configuration, and it
    # times the deterministic precompute uncached (the re-setup and check-order
    # sections build BLAS-M2L handles of the same configuration)
    if not args.no_blas:
        log("blas-m2l workload: 32 vectors, fp64 / fp32 / bf16x3 / bf16x6")
        line["blas_32rhs"] = run_blas(K, torch, max(1, min(args.steps, 3)), 1)
    if not args.no_resetup:
        log("moving points: host tree build vs device re-setup")
        line["resetup_1M"] = run_resetup(K, torch, w)
    if not args.no_check_order:
        log("blas-m2l with a finer check surface: check order p and p + 1")
        line["check_order_blas"] = run_check_order(K, torch, w, max(1, min(args.steps, 3)))
    if not args.no_sphere:
        log("sphere workload: 4M points, depth 6, p = 6, 64 vectors")
        line["sphere_4M"] = run_sphere(K, torch, max(1, min(args.steps, 3)), 1)
    if not args.no_batch:
        log("batched serving workload: 128 problems, one graph launch")
        line["batch_128"] = run_batch(K, torch, 200)
    if not args.no_scale:
        log("scale workload: 8M uniform points, depth 6, p = 6")
        line["scale_8M"] = run_scale(K, torch, max(1, min(args.steps, 5)), 1)
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle dense M2L of every level")
        line["cpu_baseline"] = cpu_baseline(w)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
