"""Python binding of libkifmm, the MI355X kernel-independent FMM library.

Argument marshalling only: every step of the FMM runs in the HIP library
(``csrc/``) behind the C ABI of ``include/kifmm.h``.  PyTorch supplies device
memory and streams.  There is no CPU fallback: importing the binding fails
loudly when ``libkifmm.so`` has not been built.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkifmm.so")

M2L = {"dense": 0, "fft": 1, "blas": 2}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
STATUS = {0: "OK", 1: "EINVAL", 2: "ESTATE", 3: "ENOMEM", 4: "EDEVICE", 5: "EUNSUPPORTED",
          6: "ENUMERIC"}

EXPORTS = [
    "kifmm_config_default", "kifmm_create", "kifmm_set_points", "kifmm_precompute",
    "kifmm_evaluate", "kifmm_destroy", "kifmm_last_error", "kifmm_num_boxes", "kifmm_box_keys",
    "kifmm_point_perm", "kifmm_interactions", "kifmm_near", "kifmm_operator", "kifmm_stage",
    "kifmm_set_timing", "kifmm_timings", "kifmm_m2l_counts", "kifmm_get_tuning",
    "kifmm_set_tuning", "kifmm_autotune", "kifmm_update_points", "kifmm_batch_create", "kifmm_batch_autotune",
    "kifmm_batch_launch", "kifmm_batch_destroy", "kifmm_set_svd", "kifmm_evaluate_noalloc",
    "kifmm_batch_evaluate", "kifmm_batch_info",
]
NOALLOC_SCRATCH_BYTES = 256 << 20  # KIFMM_NOALLOC_SCRATCH_BYTES
TUNE_KNOBS = ("blas_tile", "schedule", "hadamard", "blas_form", "products")


class KifmmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [
        ("size", ctypes.c_uint32),
        ("order", ctypes.c_int32),
        ("depth", ctypes.c_int32),
        ("m2l", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("svd_rel_tol", ctypes.c_double),
        ("svd_rel_tol_dir", ctypes.c_double),
        ("alpha_inner", ctypes.c_double),
        ("alpha_outer", ctypes.c_double),
        ("origin", ctypes.c_double * 3),
        ("width", ctypes.c_double),
        ("check_order", ctypes.c_int32),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libkifmm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2408_07436_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    L.kifmm_config_default.argtypes = [ctypes.POINTER(Config)]
    L.kifmm_config_default.restype = None
    L.kifmm_create.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(vp)]
    L.kifmm_set_points.argtypes = [vp, dp, i64, dp, i64]
    L.kifmm_precompute.argtypes = [vp]
    L.kifmm_evaluate.argtypes = [vp, vp, i64, i32, vp, i64, vp]
    L.kifmm_evaluate_noalloc.argtypes = [vp, vp, i64, i32, vp, i64, vp]
    L.kifmm_destroy.argtypes = [vp]
    L.kifmm_last_error.restype = ctypes.c_char_p
    L.kifmm_num_boxes.argtypes = [vp, i32, ctypes.POINTER(i64)]
    L.kifmm_box_keys.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_uint64), i64]
    L.kifmm_point_perm.argtypes = [vp, i32, ctypes.POINTER(i64), i64]
    L.kifmm_interactions.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                     ctypes.POINTER(i32), i64, ctypes.POINTER(i64)]
    L.kifmm_near.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), i64, ctypes.POINTER(i64)]
    L.kifmm_operator.argtypes = [vp, i32, dp, i64, ctypes.POINTER(i64)]
    L.kifmm_stage.argtypes = [vp, i32, i32, vp, vp, i32, vp]
    L.kifmm_set_timing.argtypes = [vp, i32]
    L.kifmm_timings.argtypes = [vp, dp, i32]
    L.kifmm_m2l_counts.argtypes = [vp, i32, ctypes.POINTER(i64), i32]
    L.kifmm_update_points.argtypes = [vp, vp, vp, vp]
    L.kifmm_get_tuning.argtypes = [vp, ctypes.POINTER(i32), i32]
    L.kifmm_set_tuning.argtypes = [vp, ctypes.POINTER(i32), i32]
    L.kifmm_set_svd.argtypes = [vp, i32, i32, i32, ctypes.c_uint64]
    L.kifmm_autotune.argtypes = [vp, vp, i64, i32, vp, i64, vp, i32, dp]
    L.kifmm_batch_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp), ctypes.POINTER(i64),
                                     ctypes.POINTER(i32), ctypes.POINTER(vp), ctypes.POINTER(i64), vp,
                                     ctypes.POINTER(vp)]
    L.kifmm_batch_autotune.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp),
                                       ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(vp),
                                       ctypes.POINTER(i64), vp, i32, ctypes.POINTER(vp), dp]
    L.kifmm_batch_launch.argtypes = [vp, vp]
    L.kifmm_batch_evaluate.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    L.kifmm_batch_info.argtypes = [vp, ctypes.POINTER(i64), i32]
    L.kifmm_batch_destroy.argtypes = [vp]
    for name in EXPORTS:
        if name not in ("kifmm_config_default", "kifmm_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(code: int):
    if code != 0:
        raise KifmmError(code, lib().kifmm_last_error().decode())


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class KiFMM:
    """A kiFMM problem: configuration, points, precomputed operators.

    ``m2l`` is "dense", "fft" or "blas"; ``prec`` is "fp64", "fp32", "bf16x3"
    or "bf16x6" (see ``include/kifmm.h``).
    """

    def __init__(self, order: int, depth: int, m2l: str = "fft", prec: str = "fp64",
                 origin=(0.0, 0.0, 0.0), width: float = 1.0, svd_rel_tol: float = 0.0,
                 svd_rel_tol_dir: float = -1.0, device: int = 0, alpha_inner: float = 1.05,
                 alpha_outer: float = 2.95, check_order: int = 0):
        L = lib()
        cfg = Config()
        L.kifmm_config_default(ctypes.byref(cfg))
        cfg.order, cfg.depth = order, depth
        cfg.m2l, cfg.prec = M2L[m2l], PREC[prec]
        cfg.device = device
        cfg.svd_rel_tol, cfg.svd_rel_tol_dir = svd_rel_tol, svd_rel_tol_dir
        cfg.alpha_inner, cfg.alpha_outer = alpha_inner, alpha_outer
        cfg.origin[:] = list(origin)
        cfg.width = width
        cfg.check_order = check_order
        h = ctypes.c_void_p()
        _check(L.kifmm_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.order, self.depth, self.m2l, self.prec = order, depth, m2l, prec
        self.check_order = check_order if check_order > 0 else order
        self.n_equiv = 6 * (order - 1) ** 2 + 2              # points of an equivalent surface
        self.n_check = 6 * (self.check_order - 1) ** 2 + 2  # points of a check surface
        self.n_src = self.n_tgt = 0

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().kifmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.prec == "fp64" else torch.float32

    def set_points(self, sources: np.ndarray, targets: np.ndarray | None = None):
        s = np.ascontiguousarray(sources, dtype=np.float64)
        t = s if targets is None else np.ascontiguousarray(targets, dtype=np.float64)
        _check(lib().kifmm_set_points(self._h, _ptr(s, ctypes.c_double), s.shape[0],
                                      _ptr(t, ctypes.c_double), t.shape[0]))
        self.n_src, self.n_tgt = s.shape[0], t.shape[0]
        return self

    def set_svd(self, mode: str = "randomized", rank: int = 0, oversample: int = 10, seed: int = 0):
        """Compression of K_fat for BLAS-M2L: "deterministic" (host SVD) or "randomized"
        (one-shot randomized SVD on the device; ``rank`` 0 = ceil(n_s / 2)).  Before
        ``precompute``."""
        modes = {"deterministic": 0, "randomized": 1}
        _check(lib().kifmm_set_svd(self._h, modes[mode], int(rank), int(oversample), int(seed)))
        return self

    def precompute(self):
        _check(lib().kifmm_precompute(self._h))
        return self

    def _eval_args(self, q, out, stream):
        import torch
        if q.dim() == 1:
            q = q[None]
        assert q.is_cuda and q.dtype == self.dtype and q.stride(1) == 1
        assert q.dim() == 2 and q.shape[1] == self.n_src, "charges must be (nvec, n_src)"
        nvec = q.shape[0]
        if out is None:
            out = torch.empty((nvec, self.n_tgt), dtype=self.dtype, device=q.device)
        assert out.is_cuda and out.dtype == self.dtype and out.stride(1) == 1
        assert tuple(out.shape) == (nvec, self.n_tgt), "potentials must be (nvec, n_tgt)"
        s = torch.cuda.current_stream(q.device) if stream is None else stream
        return q, out, nvec, s

    def evaluate(self, q, out=None, stream=None):
        """Potentials (nvec, n_tgt) on the device for charges ``q`` (nvec, n_src)."""
        q, out, nvec, s = self._eval_args(q, out, stream)
        _check(lib().kifmm_evaluate(self._h, q.data_ptr(), q.stride(0), nvec, out.data_ptr(),
                                    out.stride(0), ctypes.c_void_p(s.cuda_stream)))
        return out

    def evaluate_noalloc(self, q, out, stream=None):
        """As ``evaluate`` through kifmm_evaluate_noalloc: the library allocates no device
        memory (its work buffers come from its fixed scratch array); ``out`` is required."""
        q, out, nvec, s = self._eval_args(q, out, stream)
        _check(lib().kifmm_evaluate_noalloc(self._h, q.data_ptr(), q.stride(0), nvec, out.data_ptr(),
                                            out.stride(0), ctypes.c_void_p(s.cuda_stream)))
        return out

    def stage_m2l(self, level: int, mult, out=None, stream=None):
        """M2L check potentials (n_boxes, nvec, n_check) of one level for equivalent
        densities ``mult`` (n_boxes, nvec, n_equiv), FP64."""
        import torch
        assert mult.is_cuda and mult.dtype == torch.float64 and mult.is_contiguous()
        assert mult.dim() == 3 and mult.shape[2] == self.n_equiv
        assert mult.shape[0] == self.num_boxes(level), "densities must cover every box of the level"
        if out is None:
            out = torch.empty((mult.shape[0], mult.shape[1], self.n_check), dtype=torch.float64,
                              device=mult.device)
        assert out.shape == (mult.shape[0], mult.shape[1], self.n_check) and out.is_contiguous()
        s = torch.cuda.current_stream(mult.device) if stream is None else stream
        _check(lib().kifmm_stage(self._h, 0, level, mult.data_ptr(), out.data_ptr(), mult.shape[1],
                                 ctypes.c_void_p(s.cuda_stream)))
        return out

    # ---- introspection -----------------------------------------------------
    def num_boxes(self, level: int) -> int:
        n = ctypes.c_int64()
        _check(lib().kifmm_num_boxes(self._h, level, ctypes.byref(n)))
        return n.value

    def box_keys(self, level: int) -> np.ndarray:
        n = self.num_boxes(level)
        out = np.zeros(n, dtype=np.uint64)
        _check(lib().kifmm_box_keys(self._h, level, _ptr(out, ctypes.c_uint64), n))
        return out

    def point_perm(self, which: int = 0) -> np.ndarray:
        n = self.n_src if which == 0 else self.n_tgt
        out = np.zeros(n, dtype=np.int64)
        _check(lib().kifmm_point_perm(self._h, which, _ptr(out, ctypes.c_int64), n))
        return out

    def interactions(self, level: int):
        L = lib()
        cnt = ctypes.c_int64()
        _check(L.kifmm_interactions(self._h, level, None, None, None, 0, ctypes.byref(cnt)))
        nb = self.num_boxes(level)
        offs = np.zeros(nb + 1, dtype=np.int64)
        src = np.zeros(max(cnt.value, 1), dtype=np.int64)
        tid = np.zeros(max(cnt.value, 1), dtype=np.int32)
        _check(L.kifmm_interactions(self._h, level, _ptr(offs, ctypes.c_int64), _ptr(src, ctypes.c_int64),
                                    _ptr(tid, ctypes.c_int32), src.size, ctypes.byref(cnt)))
        return offs, src[:cnt.value], tid[:cnt.value]

    def near(self):
        L = lib()
        cnt = ctypes.c_int64()
        _check(L.kifmm_near(self._h, None, None, 0, ctypes.byref(cnt)))
        offs = np.zeros(self.num_boxes(self.depth) + 1, dtype=np.int64)
        src = np.zeros(cnt.value, dtype=np.int64)
        _check(L.kifmm_near(self._h, _ptr(offs, ctypes.c_int64), _ptr(src, ctypes.c_int64), src.size,
                            ctypes.byref(cnt)))
        return offs, src

    def operator(self, which: int) -> np.ndarray:
        L = lib()
        n = ctypes.c_int64()
        _check(L.kifmm_operator(self._h, which, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, dtype=np.float64)
        _check(L.kifmm_operator(self._h, which, _ptr(out, ctypes.c_double), n.value, ctypes.byref(n)))
        return out

    def set_timing(self, on: bool = True):
        _check(lib().kifmm_set_timing(self._h, 1 if on else 0))

    def timings(self) -> dict:
        ms = np.zeros(12, dtype=np.float64)
        _check(lib().kifmm_timings(self._h, _ptr(ms, ctypes.c_double), 12))
        return dict(upward=ms[0], m2l=ms[1], downward=ms[2], leaves=ms[3], total=ms[4],
                    m2l_first=ms[5], m2l_main=ms[6], m2l_last=ms[7], m2l_levels=int(ms[8]),
                    near_field=ms[9], far_field=ms[10], p2m=ms[11])

    def update_points(self, sources, targets=None, stream=None):
        """Move the points on the device (kifmm_update_points): ``sources``
        (and ``targets``, default the sources) are FP64 device tensors (n, 3)
        with the counts of set_points; the tree of the new positions over the
        same domain cube is built on the device."""
        import torch
        tgt = sources if targets is None else targets
        for a, n in ((sources, self.n_src), (tgt, self.n_tgt)):
            assert a.is_cuda and a.dtype == torch.float64 and a.is_contiguous()
            assert a.dim() == 2 and tuple(a.shape) == (n, 3), "points must be (n, 3) as in set_points"
        s = torch.cuda.current_stream(sources.device) if stream is None else stream
        _check(lib().kifmm_update_points(self._h, sources.data_ptr(), tgt.data_ptr(),
                                         ctypes.c_void_p(s.cuda_stream)))
        return self

    # ---- autotuning -------------------------------------------------------
    def tuning(self) -> dict:
        k = np.zeros(len(TUNE_KNOBS), dtype=np.int32)
        _check(lib().kifmm_get_tuning(self._h, _ptr(k, ctypes.c_int32), len(TUNE_KNOBS)))
        return {n: int(v) for n, v in zip(TUNE_KNOBS, k)}

    def set_tuning(self, **knobs):
        cur = self.tuning()
        for n, v in knobs.items():
            if n not in cur:
                raise KeyError(n)
            cur[n] = int(v)
        k = np.array([cur[n] for n in TUNE_KNOBS], dtype=np.int32)
        _check(lib().kifmm_set_tuning(self._h, _ptr(k, ctypes.c_int32), len(TUNE_KNOBS)))

    def autotune(self, q, out=None, stream=None, reps: int = 3) -> float:
        """Time the candidate knob settings on charges ``q`` and keep the fastest; returns its
        median evaluate time in ms (``out`` receives the potentials)."""
        import torch
        if q.dim() == 1:
            q = q[None]
        assert q.is_cuda and q.dtype == self.dtype and q.stride(1) == 1
        assert q.dim() == 2 and q.shape[1] == self.n_src, "charges must be (nvec, n_src)"
        nvec = q.shape[0]
        if out is None:
            out = torch.empty((nvec, self.n_tgt), dtype=self.dtype, device=q.device)
        assert out.is_cuda and out.dtype == self.dtype and out.stride(1) == 1
        assert tuple(out.shape) == (nvec, self.n_tgt), "potentials must be (nvec, n_tgt)"
        s = torch.cuda.current_stream(q.device) if stream is None else stream
        best = ctypes.c_double(0.0)
        _check(lib().kifmm_autotune(self._h, q.data_ptr(), q.stride(0), nvec, out.data_ptr(),
                                    out.stride(0), ctypes.c_void_p(s.cuda_stream), reps,
                                    ctypes.byref(best)))
        return best.value

    def m2l_counts(self, level: int) -> dict:
        c = np.zeros(4, dtype=np.int64)
        _check(lib().kifmm_m2l_counts(self._h, level, _ptr(c, ctypes.c_int64), 4))
        return dict(boxes=int(c[0]), pairs=int(c[1]), clusters=int(c[2]), cluster_pairs=int(c[3]))


class Batch:
    """Independent problems replayed with one graph launch (see kifmm_batch_create).

    ``items`` is a list of (KiFMM, q, phi) with device tensors q (nvec, n_src)
    and phi (nvec, n_tgt) that stay alive as long as the batch.
    """

    def __init__(self, items, stream=None, autotune: bool = False, reps: int = 3):
        """With ``autotune`` the knob settings that apply to the handles are timed as whole
        batches (kifmm_batch_autotune) and the fastest is kept; ``best_ms`` is its median
        launch time (None without autotuning)."""
        import torch
        n = len(items)
        self._items = items
        hs = (ctypes.c_void_p * n)(*[f._h.value for f, _, _ in items])
        qs = (ctypes.c_void_p * n)(*[q.data_ptr() for _, q, _ in items])
        ps = (ctypes.c_void_p * n)(*[p.data_ptr() for _, _, p in items])
        ldq = (ctypes.c_int64 * n)(*[q.stride(0) for _, q, _ in items])
        ldp = (ctypes.c_int64 * n)(*[p.stride(0) for _, _, p in items])
        nv = (ctypes.c_int32 * n)(*[q.shape[0] for _, q, _ in items])
        for f, q, p in items:
            assert q.is_cuda and p.is_cuda and q.dtype == f.dtype and p.dtype == f.dtype
            assert q.dim() == 2 and q.shape[1] == f.n_src and q.stride(1) == 1
            assert tuple(p.shape) == (q.shape[0], f.n_tgt) and p.stride(1) == 1
        s = torch.cuda.current_stream() if stream is None else stream
        b = ctypes.c_void_p()
        self.best_ms = None
        if autotune:
            best = ctypes.c_double(0.0)
            _check(lib().kifmm_batch_autotune(hs, n, qs, ldq, nv, ps, ldp,
                                              ctypes.c_void_p(s.cuda_stream), reps, ctypes.byref(b),
                                              ctypes.byref(best)))
            self.best_ms = best.value
        else:
            _check(lib().kifmm_batch_create(hs, n, qs, ldq, nv, ps, ldp,
                                            ctypes.c_void_p(s.cuda_stream), ctypes.byref(b)))
        self._b = b

    def launch(self, stream=None):
        import torch
        s = torch.cuda.current_stream() if stream is None else stream
        _check(lib().kifmm_batch_launch(self._b, ctypes.c_void_p(s.cuda_stream)))

    def evaluate(self, qs, phis, stream=None):
        """Launch with other charge / potential tensors (kifmm_batch_evaluate): one
        (q, phi) per problem, shapes and dtypes as at creation."""
        import torch
        n = len(self._items)
        assert len(qs) == n and len(phis) == n
        for (f, q0, p0), q, p in zip(self._items, qs, phis):
            assert q.is_cuda and p.is_cuda and q.dtype == f.dtype and p.dtype == f.dtype
            assert q.shape == q0.shape and q.stride() == q0.stride()
            assert p.shape == p0.shape and p.stride() == p0.stride()
        qa = (ctypes.c_void_p * n)(*[q.data_ptr() for q in qs])
        pa = (ctypes.c_void_p * n)(*[p.data_ptr() for p in phis])
        s = torch.cuda.current_stream() if stream is None else stream
        _check(lib().kifmm_batch_evaluate(self._b, qa, pa, ctypes.c_void_p(s.cuda_stream)))

    def info(self) -> dict:
        """Problems, launches per replay, and how many of those are grouped."""
        a = np.zeros(3, dtype=np.int64)
        _check(lib().kifmm_batch_info(self._b, _ptr(a, ctypes.c_int64), 3))
        return dict(problems=int(a[0]), launches=int(a[1]), grouped=int(a[2]))

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            lib().kifmm_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


OP_UP_V, OP_UP_UT, OP_DOWN_V, OP_DOWN_UT, OP_FFT_SPECTRA, OP_BLAS_U, OP_BLAS_RANKS, OP_BLAS_APPLIED = range(8)
