"""Shared helpers of the GPU tests: run the HIP library through the C ABI."""
import sys

import numpy as np


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def evaluate(K, pts, q, depth, order, m2l, prec, tgt=None, origin=(0, 0, 0), width=1.0,
             tol=0.0, tol_dir=-1.0, ld_pad=0):
    import torch
    f = K.KiFMM(order, depth, m2l=m2l, prec=prec, origin=origin, width=width, svd_rel_tol=tol,
                svd_rel_tol_dir=tol_dir)
    f.set_points(pts, tgt)
    f.precompute()
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
