"""Python binding of librss (ctypes over include/rss.h).

Argument marshalling only: every step of the factorization, solve, apply, exact
operator and GMRES runs in the HIP library.  torch provides device memory and the
current HIP stream.  Importing this module fails loudly when librss.so has not been
built (`python -m paper_1609_08130_amd.build` or `__graft_entry__.build()`).
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np
# torch ships its own HIP runtime (SONAME libamdhip64.so.7).  It must be loaded before
# librss so that librss binds to that same runtime instead of pulling a second copy
# from /opt/rocm into the process (two runtimes cannot share the device).
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librss.so")

RSS_FP64 = 0
RSS_MIXED = 1

RSS_K_LAPLACE2D = 0
RSS_K_LAPLACE3D = 1
RSS_K_HELMHOLTZ2D = 2
KERNELS = {"laplace2d": RSS_K_LAPLACE2D, "laplace3d": RSS_K_LAPLACE3D, "helmholtz2d": RSS_K_HELMHOLTZ2D}

STATUS = {0: "RSS_OK", 1: "RSS_E_ARG", 2: "RSS_E_NOMEM", 3: "RSS_E_DEVICE", 4: "RSS_E_SINGULAR",
          5: "RSS_E_UNSUPPORTED", 6: "RSS_E_NOCONV", 7: "RSS_E_ARENA"}

# exported names declared in include/rss.h
EXPORTS = ["rss_params_default", "rss_factor_create", "rss_solve", "rss_apply", "rss_sqrt_apply", "rss_matvec", "rss_gmres",
           "rss_gmres_noalloc",
           "rss_logdet", "rss_shape", "rss_box_sets", "rss_box_record", "rss_top_set", "rss_info",
           "rss_factor_destroy", "rss_last_error", "rss_trim"]


class RSSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("dim", ctypes.c_int32),
        ("kernel", ctypes.c_int32),
        ("symmetric", ctypes.c_int32),
        ("diag", ctypes.c_double),
        ("weight", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("leaf_size", ctypes.c_int32),
        ("n_proxy", ctypes.c_int32),
        ("proxy_radius", ctypes.c_double),
        ("root_lo", ctypes.c_double * 3),
        ("root_side", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("method", ctypes.c_int32),
        ("level_graphs", ctypes.c_int32),
        ("max_box", ctypes.c_int32),
        ("arena_bytes", ctypes.c_uint64),
    ]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"librss.so not built at {path}; run `python -m paper_1609_08130_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    lib.rss_params_default.argtypes = [P(Params), i32, i32]
    lib.rss_params_default.restype = None
    lib.rss_factor_create.argtypes = [vp, i64, P(Params), vp, P(vp)]
    lib.rss_solve.argtypes = [vp, vp, vp, i32, i64, i32, vp]
    lib.rss_apply.argtypes = [vp, vp, vp, i32, i64, vp]
    lib.rss_sqrt_apply.argtypes = [vp, vp, vp, i32, i64, i32, vp]
    lib.rss_matvec.argtypes = [vp, vp, vp, i32, i64, vp]
    lib.rss_gmres.argtypes = [vp, vp, vp, dbl, i32, i32, i32, vp, P(i32), P(dbl)]
    lib.rss_gmres_noalloc.argtypes = [vp, vp, vp, dbl, i32, i32, i32, vp, P(i32), P(dbl)]
    lib.rss_logdet.argtypes = [vp, P(dbl), P(dbl)]
    lib.rss_shape.argtypes = [vp, P(i32), P(i64)]
    lib.rss_box_sets.argtypes = [vp, i32, i64, i32, P(i64), i32, P(i32), P(i64), i32, P(i32)]
    lib.rss_box_record.argtypes = [vp, i32, i64, i32, P(dbl), P(dbl), P(dbl), P(dbl), P(i64), i64, P(i32), P(i32),
                                   P(i32)]
    lib.rss_top_set.argtypes = [vp, P(i64), i64, P(i64)]
    lib.rss_info.argtypes = [vp, ctypes.c_char_p, i64]
    lib.rss_factor_destroy.argtypes = [vp]
    lib.rss_trim.argtypes = []
    lib.rss_last_error.argtypes = []
    lib.rss_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("rss_params_default", "rss_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    return lib


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def _check(st: int):
    if st != 0:
        raise RSSError(st, lib().rss_last_error().decode())


def make_params(dim: int = 2, kernel="laplace2d", **kw) -> Params:
    p = Params()
    lib().rss_params_default(ctypes.byref(p), int(dim), KERNELS.get(kernel, kernel))
    for k, v in kw.items():
        if k == "root_lo":
            for i, c in enumerate(v):
                p.root_lo[i] = float(c)
        elif k == "precision":
            p.precision = {"fp64": RSS_FP64, "mixed": RSS_MIXED}.get(v, v)
        elif k == "method":
            p.method = {"rs-s": 0, "rs-ws": 1}.get(v, v)
        elif k == "hybrid":
            p.method = 1 if v else 0
        elif hasattr(p, k):
            setattr(p, k, type(getattr(p, k))(v))
        else:
            raise KeyError(k)
    return p


def trim():
    """Return the library's cached device blocks to the device."""
    _check(lib().rss_trim())


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Factor:
    """RS-S factorization F ~ A of the matrix defined by `points` and the parameters."""

    def __init__(self, points, **params):
        import torch
        self._torch = torch
        if not (points.is_cuda and points.dtype == torch.float64 and points.dim() == 2):
            raise ValueError("points must be a CUDA float64 tensor of shape (N, dim)")
        params.setdefault("dim", int(points.shape[1]))
        self.points = points.contiguous()
        self.n = int(points.shape[0])
        self.params = make_params(**params)
        h = ctypes.c_void_p()
        _check(lib().rss_factor_create(ctypes.c_void_p(self.points.data_ptr()), self.n, ctypes.byref(self.params),
                                       _stream(torch), ctypes.byref(h)))
        self._h = h

    def _vec(self, b):
        torch = self._torch
        if not (b.is_cuda and b.dtype == torch.float64):
            raise ValueError("vectors must be CUDA float64 tensors")
        if b.shape[0] != self.n:
            raise ValueError("leading dimension must equal N")
        single = b.dim() == 1
        bb = b.reshape(self.n, 1) if single else b
        # column-major N x nrhs storage
        bb = bb.t().contiguous().t()
        return bb, single

    def solve(self, b, use_fp32: bool = False):
        bb, single = self._vec(b)
        x = self._torch.empty_like(bb).t().contiguous().t()
        nrhs = bb.shape[1]
        _check(lib().rss_solve(self._h, ctypes.c_void_p(bb.data_ptr()), ctypes.c_void_p(x.data_ptr()), nrhs,
                               self.n, int(bool(use_fp32)), _stream(self._torch)))
        return x.reshape(-1) if single else x

    def apply(self, x):
        xx, single = self._vec(x)
        y = self._torch.empty_like(xx).t().contiguous().t()
        _check(lib().rss_apply(self._h, ctypes.c_void_p(xx.data_ptr()), ctypes.c_void_p(y.data_ptr()), xx.shape[1],
                               self.n, _stream(self._torch)))
        return y.reshape(-1) if single else y

    def matvec(self, x):
        xx, single = self._vec(x)
        y = self._torch.empty_like(xx).t().contiguous().t()
        _check(lib().rss_matvec(self._h, ctypes.c_void_p(xx.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                xx.shape[1], self.n, _stream(self._torch)))
        return y.reshape(-1) if single else y

    def gmres(self, b, rtol: float = 1e-10, maxit: int = 100, restart: int = 30, use_fp32: bool = False,
              raise_on_noconv: bool = True):
        bb = b.contiguous()
        x = self._torch.empty_like(bb)
        it = ctypes.c_int32()
        rr = ctypes.c_double()
        st = lib().rss_gmres(self._h, ctypes.c_void_p(bb.data_ptr()), ctypes.c_void_p(x.data_ptr()), float(rtol),
                             int(maxit), int(restart), int(bool(use_fp32)), _stream(self._torch), ctypes.byref(it),
                             ctypes.byref(rr))
        if st != 6 or raise_on_noconv:
            _check(st)
        return x, it.value, rr.value

    def gmres_noalloc(self, b, x, rtol: float = 1e-10, maxit: int = 100, restart: int = 8, use_fp32: bool = False):
        """rss_gmres_noalloc: the same iteration with the library's own device work array (no
        allocation); x is a caller-provided output (no allocation here either).  Returns
        (status, iterations, relres) without raising on RSS_E_NOCONV."""
        it = ctypes.c_int32()
        rr = ctypes.c_double()
        st = lib().rss_gmres_noalloc(self._h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                     float(rtol), int(maxit), int(restart), int(bool(use_fp32)),
                                     _stream(self._torch), ctypes.byref(it), ctypes.byref(rr))
        if st not in (0, 6):
            _check(st)
        return st, it.value, rr.value

    def sqrt_apply(self, x, adjoint: bool = False):
        """y = F^{1/2} x, or (F^{1/2})^* x with adjoint (generalized square root, Section 3.3)."""
        xx, single = self._vec(x)
        y = self._torch.empty_like(xx).t().contiguous().t()
        _check(lib().rss_sqrt_apply(self._h, ctypes.c_void_p(xx.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                    xx.shape[1], self.n, int(bool(adjoint)), _stream(self._torch)))
        return y.reshape(-1) if single else y

    def logdet(self):
        """(sign, log|det F|) of a real factor, from rss_logdet's log det = re + i im."""
        re, im = ctypes.c_double(), ctypes.c_double()
        _check(lib().rss_logdet(self._h, ctypes.byref(re), ctypes.byref(im)))
        return (-1.0 if im.value != 0.0 else 1.0), re.value

    def box_record(self, depth: int, box: int, weak: bool = False) -> dict:
        """T, X_RR, X_JR, G and the global J indices of one skeletonization step (empty
        arrays when the box has no record); weak selects the weak step of RS-WS."""
        ns, nr, nj = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        w = int(bool(weak))
        _check(lib().rss_box_record(self._h, depth, box, w, None, None, None, None, None, 0, ctypes.byref(ns),
                                    ctypes.byref(nr), ctypes.byref(nj)))
        k, r, J = ns.value, nr.value, nj.value
        cap = max(k * r, r * r, J * r, J, 1)
        bufs = [(ctypes.c_double * cap)() for _ in range(4)]
        jb = (ctypes.c_int64 * cap)()
        _check(lib().rss_box_record(self._h, depth, box, w, *bufs, jb, cap, ctypes.byref(ns), ctypes.byref(nr),
                                    ctypes.byref(nj)))
        col = lambda b, rows, cols: np.array(b[:rows * cols], dtype=np.float64).reshape(cols, rows).T.copy()
        return dict(T=col(bufs[0], k, r), XRR=col(bufs[1], r, r), XJR=col(bufs[2], J, r), G=col(bufs[3], r, J),
                    J=np.array(jb[:J], dtype=np.int64))

    def shape(self):
        d, nt = ctypes.c_int32(), ctypes.c_int64()
        _check(lib().rss_shape(self._h, ctypes.byref(d), ctypes.byref(nt)))
        return d.value, nt.value

    def box_sets(self, depth: int, box: int, weak: bool = False):
        cap = 8192
        S = (ctypes.c_int64 * cap)()
        R = (ctypes.c_int64 * cap)()
        ns, nr = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().rss_box_sets(self._h, depth, box, int(bool(weak)), S, cap, ctypes.byref(ns), R, cap,
                                  ctypes.byref(nr)))
        return (np.array(S[:ns.value], dtype=np.int64), np.array(R[:nr.value], dtype=np.int64))

    def top_set(self):
        d, nt = self.shape()
        buf = (ctypes.c_int64 * max(nt, 1))()
        cnt = ctypes.c_int64()
        _check(lib().rss_top_set(self._h, buf, nt, ctypes.byref(cnt)))
        return np.array(buf[:cnt.value], dtype=np.int64)

    def info(self) -> dict:
        buf = ctypes.create_string_buffer(1 << 20)
        _check(lib().rss_info(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().rss_factor_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
