"""Host-side checks of the C-ABI library (no GPU needed): exported symbols,
tree and lists bit-exact against the oracle, FP64 precompute against the
oracle, and the documented error codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads
from oracle import blas_m2l, fft_m2l, kernel, linalg, surfaces
from oracle import tree as T

K = pytest.importorskip("paper_2408_07436_amd")


def header_symbols(repo_root):
    with open(os.path.join(repo_root, "include", "kifmm.h")) as fh:
        txt = fh.read()
    return sorted(set(re.findall(r"\b(kifmm_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol(repo_root):
    lib = K.lib()
    names = header_symbols(repo_root)
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert set(K.EXPORTS) <= set(names)


@pytest.mark.parametrize("kind", ["uniform", "sphere", "distinct"])
def test_tree_and_lists_bit_exact(kind):
    if kind == "uniform":
        src = tgt = workloads.uniform_cube(20000, 51)
        depth, origin, width = 4, (0, 0, 0), 1.0
    elif kind == "sphere":
        src = tgt = workloads.sphere_surface(20000, 52)
        depth, origin, width = 5, (-1, -1, -1), 2.0
    else:
        src = workloads.uniform_cube(5000, 53)
        tgt = workloads.uniform_cube(3000, 54) * 0.5
        depth, origin, width = 4, (0, 0, 0), 1.0
    f = K.KiFMM(4, depth, origin=origin, width=width).set_points(src, tgt)
    tr = T.Tree(src, tgt, depth, origin, width)
    for lev in range(depth + 1):
        assert np.array_equal(f.box_keys(lev), tr.levels[lev])
    assert np.array_equal(f.point_perm(0), tr.src_perm)
    assert np.array_equal(f.point_perm(1), tr.tgt_perm)
    for lev in range(2, depth + 1):
        a, b = f.interactions(lev), tr.interactions(lev)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    for x, y in zip(f.near(), tr.near()):
        assert np.array_equal(x, y)


def test_fft_spectra_match_oracle():
    p = 6
    f = K.KiFMM(p, 3, m2l="fft").set_points(workloads.uniform_cube(100, 55)).precompute()
    spec = f.operator(K.OP_FFT_SPECTRA).reshape(316, -1, 2)
    h = 2 * surfaces.ALPHA_INNER * 0.5 / (p - 1)
    n = 2 * p - 1
    assert spec.shape[1] == n * n * (n // 2 + 1)
    for it in range(0, 316, 3):
        ref = fft_m2l.kernel_spectrum(p, h, -T.TRANSFER_VECTORS[it].astype(float), n).ravel()
        got = spec[it, :, 0] + 1j * spec[it, :, 1]
        assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


def test_pinv_factors_reproduce_oracle_solution():
    p = 6
    f = K.KiFMM(p, 3).set_points(workloads.uniform_cube(100, 56)).precompute()
    ns = surfaces.n_surface(p)
    V, Ut = f.operator(K.OP_UP_V), f.operator(K.OP_UP_UT)
    r = Ut.size // ns
    kmat = kernel.kernel_matrix(surfaces.surface(p, 2.95, 0.5), surfaces.surface(p, 1.05, 0.5))
    fac = linalg.pinv_factors(kmat)
    assert r == fac[0].shape[1]
    # compare in potential space: both solutions reproduce the check potential
    y = np.array([[0.1, 0.2, -0.3], [0.3, -0.1, 0.2]])
    phi = kernel.kernel_matrix(surfaces.surface(p, 2.95, 0.5), y) @ np.array([1.0, 0.7])
    q_lib = V.reshape(ns, r) @ (Ut.reshape(r, ns) @ phi)
    q_ora = linalg.pinv_apply(fac, phi)
    far = surfaces.surface(p, 5.0, 0.5)
    e = kernel.kernel_matrix(far, surfaces.surface(p, 1.05, 0.5))
    assert np.linalg.norm(e @ (q_lib - q_ora)) < 1e-12 * np.linalg.norm(e @ q_ora)


@pytest.mark.parametrize("tol,tol_dir", [(1e-6, 1e-6), (1e-4, -1.0), (0.0, -1.0)])
def test_blas_operators_match_oracle(tol, tol_dir):
    p = 4
    f = K.KiFMM(p, 3, m2l="blas", svd_rel_tol=tol, svd_rel_tol_dir=tol_dir)
    f.set_points(workloads.uniform_cube(100, 57)).precompute()
    ns = surfaces.n_surface(p)
    comp = blas_m2l.compress(blas_m2l.m2l_matrices(p, 0.5), tol, tol_dir)
    ranks = f.operator(K.OP_BLAS_RANKS)
    assert int(ranks[0]) == comp["k"]
    assert np.array_equal(ranks[1:].astype(int), comp["kt"])
    app = f.operator(K.OP_BLAS_APPLIED).reshape(316, ns, ns)
    for it in range(316):
        ref = blas_m2l.applied_operator(comp, it)
        assert np.abs(app[it] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_error_codes():
    with pytest.raises(K.KifmmError) as e:
        K.KiFMM(1, 3)
    assert e.value.code == 1
    with pytest.raises(K.KifmmError) as e:
        K.KiFMM(4, 1)
    assert e.value.code == 1
    with pytest.raises(K.KifmmError) as e:
        K.KiFMM(4, 3, m2l="fft", prec="bf16x3")
    assert e.value.code == 5
    for m2l in ("fft", "dense"):
        with pytest.raises(K.KifmmError) as e:
            K.KiFMM(4, 3, m2l=m2l, prec="bf16x6")
        assert e.value.code == 5
    # three-part BF16 runs the stacked BLAS form only: no directional
    # recompression is refused once the operators are known
    g = K.KiFMM(3, 3, m2l="blas", prec="bf16x6", svd_rel_tol=1e-6, svd_rel_tol_dir=-1.0)
    with pytest.raises(K.KifmmError) as e:
        g.precompute()
    assert e.value.code == 5
    with pytest.raises(K.KifmmError) as e:  # refused again from the operator cache
        g.precompute()
    assert e.value.code == 5
    K.KiFMM(3, 3, m2l="blas", prec="bf16x6", svd_rel_tol=1e-6, svd_rel_tol_dir=1e-6).precompute()
    f = K.KiFMM(4, 3)
    with pytest.raises(K.KifmmError) as e:
        f.set_points(np.array([[0.5, 0.5, 1.5]]))
    assert e.value.code == 1
    with pytest.raises(K.KifmmError) as e:
        f.num_boxes(2)
    assert e.value.code == 2
    f.set_points(workloads.uniform_cube(500, 58))
    with pytest.raises(K.KifmmError) as e:
        f.num_boxes(9)
    assert e.value.code == 1
    # evaluate before precompute: state error, raised before any device use
    lib = K.lib()
    rc = lib.kifmm_evaluate(f._h, ctypes.c_void_p(1), 500, 1, ctypes.c_void_p(1), 500, None)
    assert rc == 2
    assert b"precompute" in lib.kifmm_last_error()
    f.precompute()
    rc = lib.kifmm_evaluate(f._h, ctypes.c_void_p(1), 499, 1, ctypes.c_void_p(1), 500, None)
    assert rc == 1


def test_tuning_knobs_host():
    """Knob defaults, round trip and range checks; autotune argument errors
    raised before any device use."""
    f = K.KiFMM(4, 3, m2l="blas", prec="fp32")
    assert f.tuning() == {"blas_tile": 0, "schedule": 0, "hadamard": 0, "blas_form": 0, "products": 0}
    f.set_tuning(blas_tile=16, schedule=1, hadamard=1, blas_form=1, products=1)
    set_knobs = {"blas_tile": 16, "schedule": 1, "hadamard": 1, "blas_form": 1, "products": 1}
    assert f.tuning() == set_knobs
    lib = K.lib()
    for bad in ([129, 0, 0, 0, 0], [-1, 0, 0, 0, 0], [0, 2, 0, 0, 0], [0, 0, 2, 0, 0], [0, 0, 0, 2, 0],
                [0, 0, 0, 0, 2]):
        k = np.array(bad, dtype=np.int32)
        rc = lib.kifmm_set_tuning(f._h, k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 5)
        assert rc == 1
        assert f.tuning() == set_knobs
    k = np.zeros(6, dtype=np.int32)
    assert lib.kifmm_set_tuning(f._h, k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 6) == 1
    assert lib.kifmm_get_tuning(f._h, k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 4) == 1
    # partial update: only the first knob
    k1 = np.array([32], dtype=np.int32)
    assert lib.kifmm_set_tuning(f._h, k1.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 1) == 0
    assert f.tuning() == dict(set_knobs, blas_tile=32)
    best = ctypes.c_double(0.0)
    rc = lib.kifmm_autotune(f._h, ctypes.c_void_p(1), 500, 1, ctypes.c_void_p(1), 500, None, 3,
                            ctypes.byref(best))
    assert rc == 2  # no points yet
    f.set_points(workloads.uniform_cube(500, 59))
    f.precompute()
    for reps in (0, 101):
        rc = lib.kifmm_autotune(f._h, ctypes.c_void_p(1), 500, 1, ctypes.c_void_p(1), 500, None,
                                reps, ctypes.byref(best))
        assert rc == 1
    rc = lib.kifmm_autotune(f._h, ctypes.c_void_p(1), 499, 1, ctypes.c_void_p(1), 500, None, 3,
                            ctypes.byref(best))
    assert rc == 1


def test_update_points_argument_errors():
    """Refused before any device use: null buffers, no points, no operators."""
    lib = K.lib()
    f = K.KiFMM(4, 3)
    one = ctypes.c_void_p(1)
    assert lib.kifmm_update_points(f._h, None, one, None) == 1
    assert lib.kifmm_update_points(f._h, one, one, None) == 2
    f.set_points(workloads.uniform_cube(500, 60))
    assert lib.kifmm_update_points(f._h, one, one, None) == 2
    assert b"precompute" in lib.kifmm_last_error()


def test_set_svd_argument_and_state_errors():
    """The K_fat compression is chosen before precompute; bad modes and sizes are refused."""
    lib = K.lib()
    f = K.KiFMM(4, 3, m2l="blas", svd_rel_tol=1e-6)
    assert lib.kifmm_set_svd(None, 1, 0, 10, 0) == 1
    assert lib.kifmm_set_svd(f._h, 2, 0, 10, 0) == 1
    assert lib.kifmm_set_svd(f._h, 1, -1, 10, 0) == 1
    assert lib.kifmm_set_svd(f._h, 1, 0, -1, 0) == 1
    assert lib.kifmm_set_svd(f._h, 0, 0, 0, 0) == 0
    f.set_points(workloads.uniform_cube(500, 61))
    f.precompute()  # deterministic: host only
    assert lib.kifmm_set_svd(f._h, 1, 0, 10, 0) == 2
    assert b"precompute" in lib.kifmm_last_error()


@pytest.mark.parametrize("tol,tol_dir", [(1e-6, 1e-6), (1e-6, -1.0)])
def test_blas_operators_with_finer_check_surface_match_oracle(tol, tol_dir):
    """P_c = 5 check points over P_e = 4 equivalent points: the library's ranks and
    applied n_c x n_e operators equal the oracle's projected ones (host precompute)."""
    p, pc = 4, 5
    f = K.KiFMM(p, 3, m2l="blas", svd_rel_tol=tol, svd_rel_tol_dir=tol_dir, check_order=pc)
    f.set_points(workloads.uniform_cube(100, 58)).precompute()
    ne, nc = surfaces.n_surface(p), surfaces.n_surface(pc)
    comp = blas_m2l.compress(blas_m2l.m2l_matrices(p, 0.5, check_order=pc), tol, tol_dir)
    ranks = f.operator(K.OP_BLAS_RANKS)
    assert int(ranks[0]) == comp["k"] and comp["k"] <= ne
    assert np.array_equal(ranks[1:].astype(int), comp["kt"])
    app = f.operator(K.OP_BLAS_APPLIED).reshape(316, nc, ne)
    for it in range(316):
        ref = blas_m2l.applied_operator(comp, it)
        assert np.abs(app[it] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert f.operator(K.OP_UP_UT).size == f.operator(K.OP_UP_V).size // ne * nc


def test_check_order_validation():
    with pytest.raises(K.KifmmError) as e:
        K.KiFMM(4, 3, m2l="blas", check_order=3)
    assert e.value.code == 1
    for m2l in ("fft", "dense"):
        with pytest.raises(K.KifmmError) as e:
            K.KiFMM(4, 3, m2l=m2l, check_order=5)
        assert e.value.code == 5


def test_vector_limits_refused_before_device_use():
    """Vector counts beyond a kernel's limit are refused with EUNSUPPORTED before
    anything is enqueued (no device is touched here)."""
    lib = K.lib()
    one = ctypes.c_void_p(1)
    f = K.KiFMM(4, 3, m2l="blas", prec="fp32", svd_rel_tol=1e-6, svd_rel_tol_dir=1e-6)
    f.set_points(workloads.uniform_cube(500, 62)).precompute()
    assert lib.kifmm_evaluate(f._h, one, 500, 129, one, 500, None) == 5
    assert b"128" in lib.kifmm_last_error()
    assert lib.kifmm_stage(f._h, 0, 3, one, one, 129, None) == 5
    best = ctypes.c_double(0.0)
    assert lib.kifmm_autotune(f._h, one, 500, 129, one, 500, None, 2, ctypes.byref(best)) == 5
    # FFT: a level's spectra (clusters x vectors x 128 bytes in FP32) stay below 4 GiB
    g = K.KiFMM(4, 3, m2l="fft", prec="fp32").set_points(workloads.uniform_cube(500, 63)).precompute()
    nvec = (1 << 26) // (g.num_boxes(2) + 1) + 1
    assert lib.kifmm_evaluate(g._h, one, 500, nvec, one, 500, None) == 5
    assert b"4 GiB" in lib.kifmm_last_error()


def test_binding_checks_shapes_before_calls():
    """The binding refuses tensors whose shapes do not cover the problem (the C
    entry points take raw pointers and cannot see sizes)."""
    torch = pytest.importorskip("torch")
    f = K.KiFMM(4, 3, m2l="fft", prec="fp64").set_points(workloads.uniform_cube(500, 64)).precompute()
    nb = f.num_boxes(3)
    with pytest.raises(AssertionError):
        f.stage_m2l(3, torch.zeros((nb - 1, 1, f.n_equiv), dtype=torch.float64))
    with pytest.raises(AssertionError):
        f.evaluate(torch.zeros((1, 499), dtype=torch.float64))


def test_evaluate_noalloc_refused_before_device_setup():
    """kifmm_evaluate_noalloc allocates nothing, so it refuses (ESTATE, nothing
    enqueued) a handle whose tree and operators are not on the device yet, and
    checks its arguments like kifmm_evaluate (no device is touched here)."""
    lib = K.lib()
    one = ctypes.c_void_p(1)
    f = K.KiFMM(4, 3, m2l="fft", prec="fp32").set_points(workloads.uniform_cube(500, 65)).precompute()
    assert lib.kifmm_evaluate_noalloc(f._h, one, 500, 1, one, 500, None) == 2
    assert b"not on the device" in lib.kifmm_last_error()
    assert lib.kifmm_evaluate_noalloc(f._h, None, 500, 1, one, 500, None) == 1
    assert lib.kifmm_evaluate_noalloc(f._h, one, 499, 1, one, 500, None) == 1
    assert lib.kifmm_evaluate_noalloc(None, one, 500, 1, one, 500, None) == 1
    g = K.KiFMM(4, 3, m2l="fft", prec="fp32")
    assert lib.kifmm_evaluate_noalloc(g._h, one, 500, 1, one, 500, None) == 2
    assert K.NOALLOC_SCRATCH_BYTES == 256 << 20
