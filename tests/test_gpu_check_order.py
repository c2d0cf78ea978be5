"""BLAS-M2L with check surfaces finer than the equivalent surfaces (P_c > P_e;
Section 5.1, and the P_e / P_c columns of Section 4's BLAS-M2L parameter
table) against the oracle with the same orders and truncation: per M2L stage
in check-potential space (n_c points) and end to end, FP64 and FP32, at the
parity gates (FP64 1e-12 per stage, 1e-10 end to end; FP32 2e-6 / 1e-5)."""
import numpy as np
import pytest

import workloads
from oracle import fmm, kernel

from gpu_util import check_parity, say

K = pytest.importorskip("paper_2408_07436_amd")
torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("pc", [5, 6])
@pytest.mark.parametrize("prec,gate", [("fp64", (1e-12, 1e-11)), ("fp32", (2e-6, 1e-5))])
def test_finer_check_surface_stage(pc, prec, gate):
    p = 4
    pts = workloads.sphere_surface(12000, 960 + pc)
    ora = fmm.KiFMM(pts, pts, 4, p, origin=(-1, -1, -1), width=2.0, m2l="blas", svd_rel_tol=1e-6,
                    svd_rel_tol_dir=1e-6, check_order=pc)
    f = K.KiFMM(p, 4, m2l="blas", prec=prec, origin=(-1, -1, -1), width=2.0, svd_rel_tol=1e-6,
                svd_rel_tol_dir=1e-6, check_order=pc).set_points(pts).precompute()
    rng = np.random.default_rng(961)
    for lev in (2, 3, 4):
        nb = len(ora.tree.levels[lev])
        mult = rng.standard_normal((nb, 2, ora.ns))
        say(f"case: blas stage P_e {p} P_c {pc} {prec} level {lev} boxes {nb}")
        out = f.stage_m2l(lev, torch.as_tensor(mult, device="cuda"))
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert got.shape == (nb, 2, ora.nc)
        ref = ora.m2l_level(lev, mult.transpose(0, 2, 1)).transpose(0, 2, 1)
        check_parity(got, ref, gate, vec_axis=1, what="check potentials vs oracle")


@pytest.mark.parametrize("prec,gate", [("fp64", (1e-10, 1e-10)), ("fp32", (1e-5, 1e-5))])
def test_finer_check_surface_end_to_end(prec, gate):
    p = 4
    pts = workloads.uniform_cube(20000, 962)
    q = workloads.charges(20000, 2, 963, "normal")
    direct = kernel.direct(pts, q, pts)
    direct_err = []
    for pc in (4, 5, 6):
        say(f"case: blas end to end P_e {p} P_c {pc} {prec} 20k depth 4")
        f = K.KiFMM(p, 4, m2l="blas", prec=prec, svd_rel_tol=1e-6, svd_rel_tol_dir=1e-6, check_order=pc)
        f.set_points(pts).precompute()
        qd = torch.as_tensor(q, dtype=f.dtype, device="cuda")
        got = f.evaluate(qd).double().cpu().numpy()
        ref = fmm.KiFMM(pts, pts, 4, p, m2l="blas", svd_rel_tol=1e-6, svd_rel_tol_dir=1e-6,
                        check_order=pc).evaluate(q)
        direct_err.append(kernel.rel_l2(got, direct))
        say(f"  rel err vs direct {direct_err[-1]:.3e}")
        check_parity(got, ref, gate)
    # more check points fit the equivalent densities better
    assert direct_err[0] > direct_err[1] > direct_err[2]
