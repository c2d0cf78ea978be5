"""Shared helpers of the GPU tests: run the HIP library through the C ABI."""
import sys

import numpy as np


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def evaluate(K, pts, q, depth, order, m2l, prec, tgt=None, origin=(0, 0, 0), width=1.0,
             tol=0.0, tol_dir=-1.0, ld_pad=0, tune=None):
    import torch
    f = K.KiFMM(order, depth, m2l=m2l, prec=prec, origin=origin, width=width, svd_rel_tol=tol,
                svd_rel_tol_dir=tol_dir)
    f.set_points(pts, tgt)
    f.precompute()
    if tune:
        f.set_tuning(**tune)
    dt = torch.float64 if prec == "fp64" else torch.float32
    n_src = pts.shape[0]
    n_tgt = n_src if tgt is None else tgt.shape[0]
    nvec = q.shape[0]
    qbuf = torch.zeros((nvec, n_src + ld_pad), dtype=dt, device="cuda")
    qbuf[:, :n_src] = torch.as_tensor(q, dtype=dt)
    out = torch.full((nvec, n_tgt + ld_pad), float("nan"), dtype=dt, device="cuda")
    f.evaluate(qbuf[:, :n_src], out[:, :n_tgt])
    torch.cuda.synchronize()
    res = out.cpu().numpy().astype(np.float64)
    if ld_pad:
        assert np.all(np.isnan(res[:, n_tgt:])), "write beyond n_tgt"
    return res[:, :n_tgt], f


# Parity gates (relative L2 over every entry, largest element-wise error):
# the element-wise error of a vector is max |got - ref| over its entries
# divided by max |ref| of the same vector, and the gate applies to the
# largest such value over the vectors.  End to end (potentials): FP64
# agrees with the oracle to rounding (1e-10 both ways); FP32 M2L with FP64
# accumulation to 1e-5 both ways; BF16x3 (operands split into two bf16
# parts, about 16 significant bits, relative error up to ~2^-16 = 1.5e-5
# per product) to 1e-5 in L2 and 3e-5 element-wise.  Per M2L stage (check
# potentials of one level): FP64 1e-12 / 1e-11; FP32 1e-6 / 1e-5 (inner
# products of up to ~1000 FP32 terms, error ~sqrt(n) 2^-24 relative to the
# largest term); BF16x3 2e-5 / 1e-4.  BF16x6 (three bf16 parts, 24 significant
# bits, the dropped products of order three ~2^-24 relative) takes the FP32
# gates.
E2E_GATES = {"fp64": (1e-10, 1e-10), "fp32": (1e-5, 1e-5), "bf16x3": (1e-5, 3e-5),
             "bf16x6": (1e-5, 1e-5)}
STAGE_GATES = {"fp64": (1e-12, 1e-11), "fp32": (1e-6, 1e-5), "bf16x3": (2e-5, 1e-4),
               "bf16x6": (1e-6, 1e-5)}


def max_rel_inf(got, ref, vec_axis=0):
    """Largest element-wise error relative to the vector's max |ref|, over vectors."""
    g = np.moveaxis(np.asarray(got, dtype=np.float64), vec_axis, 0)
    r = np.moveaxis(np.asarray(ref, dtype=np.float64), vec_axis, 0)
    g = g.reshape(g.shape[0], -1)
    r = r.reshape(r.shape[0], -1)
    num = np.max(np.abs(g - r), axis=1)
    den = np.max(np.abs(r), axis=1)
    out = np.where(den > 0, num / np.where(den > 0, den, 1.0), num)
    return float(np.max(out))


def check_parity(got, ref, gates, vec_axis=0, what="vs oracle"):
    """Assert both gates (rel L2, element-wise max) and report the values."""
    from oracle import kernel
    e2 = kernel.rel_l2(got, ref)
    ei = max_rel_inf(got, ref, vec_axis)
    say(f"  {what}: rel L2 {e2:.3e} (gate {gates[0]:.0e}), max element-wise {ei:.3e} "
        f"(gate {gates[1]:.0e})")
    assert np.all(np.isfinite(got)), "non-finite values"
    assert e2 <= gates[0], f"rel L2 {e2} > {gates[0]}"
    assert ei <= gates[1], f"element-wise {ei} > {gates[1]}"
    return e2, ei
