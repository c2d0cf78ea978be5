"""All-box parity of single M2L levels at full size: every target box of the
leaf level of the 1M-point uniform workload (level 5, 32,768 boxes, p = 6)
and of the 4M-point sphere (level 6, 18,886 non-empty boxes, p = 6) through
kifmm_stage, against the oracle's M2L of the same level (the dense sum of
Section 2.2, which the convolution form of Appendix A.1 reaches exactly, and
the compressed operator of Section 3.1 for BLAS-M2L), compared element by
element in check-potential space.  These launches run the kernels' full-size
work splits (the FP32 Hadamard's persistent schedule over 4,096 clusters,
the BLAS tiles of every octant class) that smaller trees do not reach.  The
FP32 FFT-M2L runs in both Hadamard product forms (BF16 parts, the default,
and FP32 MFMA)."""
import numpy as np
import pytest

import workloads
from oracle import fmm

from gpu_util import STAGE_GATES, check_parity, say

K = pytest.importorskip("paper_2408_07436_amd")
torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BLAS_TOL = 1e-6
NVEC_BLAS = 4


class Level:
    """One full level: points, oracle and seeded densities; references cached."""

    def __init__(self, points, depth, order, origin, width, seed):
        self.points, self.depth, self.order = points, depth, order
        self.origin, self.width = origin, width
        self.seed = seed
        self._ref = {}
        self._mult = {}
        self._ora = {}

    def mult(self, nvec):
        if nvec not in self._mult:
            ora = self.oracle("dense")
            nb = len(ora.tree.levels[self.depth])
            rng = np.random.default_rng(self.seed + nvec)
            self._mult[nvec] = rng.standard_normal((nb, nvec, ora.ns))
        return self._mult[nvec]

    def oracle(self, m2l):
        if m2l not in self._ora:
            kw = dict(m2l="blas", svd_rel_tol=BLAS_TOL, svd_rel_tol_dir=BLAS_TOL) if m2l == "blas" else {}
            self._ora[m2l] = fmm.KiFMM(self.points, self.points, self.depth, self.order,
                                       origin=self.origin, width=self.width, **kw)
        return self._ora[m2l]

    def ref(self, m2l, nvec):
        key = (m2l, nvec)
        if key not in self._ref:
            ora = self.oracle(m2l)
            m = self.mult(nvec)
            self._ref[key] = ora.m2l_level(self.depth, m.transpose(0, 2, 1)).transpose(0, 2, 1)
        return self._ref[key]

    def run(self, m2l, prec, nvec, products=0):
        kw = dict(svd_rel_tol=BLAS_TOL, svd_rel_tol_dir=BLAS_TOL) if m2l == "blas" else {}
        f = K.KiFMM(self.order, self.depth, m2l=m2l, prec=prec, origin=self.origin,
                    width=self.width, **kw).set_points(self.points).precompute()
        f.set_tuning(products=products)
        out = f.stage_m2l(self.depth, torch.as_tensor(self.mult(nvec), device="cuda"))
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        f.close()
        del out
        torch.cuda.empty_cache()
        return got


@pytest.fixture(scope="module")
def uniform_1m():
    w = workloads.config(2)
    return Level(w.points, w.depth, w.order, w.origin, w.width, 4100)


@pytest.fixture(scope="module")
def sphere_4m():
    w = workloads.config(4)
    return Level(w.points, w.depth, w.order, w.origin, w.width, 4200)


# (M2L form, precision, vectors, FP32 Hadamard products: 0 BF16 parts, 1 FP32 MFMA)
CASES = [("fft", "fp64", 1, 0), ("fft", "fp32", 1, 0), ("fft", "fp32", 1, 1), ("blas", "fp32", NVEC_BLAS, 0),
         ("blas", "bf16x3", NVEC_BLAS, 0), ("blas", "bf16x6", NVEC_BLAS, 0),
         ("blas", "fp64", NVEC_BLAS, 0)]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("m2l,prec,nvec,products", CASES)
def test_uniform_1M_leaf_level_all_boxes(uniform_1m, m2l, prec, nvec, products):
    L = uniform_1m
    say(f"case: uniform 1M level {L.depth} all boxes, {m2l} {prec} nvec {nvec} products {products}")
    got = L.run(m2l, prec, nvec, products)
    ref = L.ref("blas" if m2l == "blas" else "dense", nvec)
    assert got.shape == ref.shape
    check_parity(got, ref, STAGE_GATES[prec], vec_axis=1, what="check potentials vs oracle")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("m2l,prec,nvec,products", CASES)
def test_sphere_4M_leaf_level_all_boxes(sphere_4m, m2l, prec, nvec, products):
    L = sphere_4m
    say(f"case: sphere 4M level {L.depth} all boxes, {m2l} {prec} nvec {nvec} products {products}")
    got = L.run(m2l, prec, nvec, products)
    ref = L.ref("blas" if m2l == "blas" else "dense", nvec)
    assert got.shape == ref.shape
    check_parity(got, ref, STAGE_GATES[prec], vec_axis=1, what="check potentials vs oracle")
