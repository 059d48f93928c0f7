"""Thin ctypes binding of libfftfem.so (include/fftfem.h).

Argument marshalling only: every step of a solve runs in the HIP library.
Device arrays are torch tensors on a ROCm device (torch is used for memory
and streams).  If the library has not been built this module raises on
import of the library handle; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfftfem.so")

FFTFEM_FP64, FFTFEM_FP32, FFTFEM_FP32_REFINE = 0, 1, 2
MAX_DIMS, MAX_ITERS = 3, 16
PRECISIONS = {"fp64": FFTFEM_FP64, "fp32": FFTFEM_FP32, "fp32_refine": FFTFEM_FP32_REFINE}

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESPECTRUM", -5: "EINDEF",
          -6: "ENOCONV", -7: "ENOTIMPL"}

EXPORTS = [
    "fftfem_plan", "fftfem_plan_ex", "fftfem_solve", "fftfem_apply_A", "fftfem_get_stats",
    "fftfem_workspace_bytes", "fftfem_destroy", "fftfem_status_string", "fftfem_plan_tables",
    "fftfem_debug_transform", "fftfem_axis_tables_host", "fftfem_element_matrices_host",
    "fftfem_set_timing", "fftfem_get_timing",
    "fftfem_plan_batch", "fftfem_solve_batch", "fftfem_batch_get_stats", "fftfem_batch_workspace_bytes",
    "fftfem_destroy_batch", "fftfem_tune", "fftfem_implicit_euler", "fftfem_tune_save", "fftfem_tune_load",
    "fftfem_coefficients", "fftfem_synthesize", "fftfem_dirichlet_load", "fftfem_dirichlet_load_noalloc",
]
BATCH_TUNE = 1
ALGORITHM_B = 1  # fftfem_desc.flags: algorithm (b) of Sect. 4


class FftfemError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS.get(status, status)} ({status})")
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int),
        ("K", ctypes.c_int64 * MAX_DIMS),
        ("n", ctypes.c_int),
        ("diff", ctypes.c_double * MAX_DIMS),
        ("react", ctypes.c_double),
        ("X", ctypes.c_double * MAX_DIMS),
        ("precision", ctypes.c_int),
        ("max_iter", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("nrhs", ctypes.c_int),
        ("flags", ctypes.c_uint),
        ("n_axis", ctypes.c_int * MAX_DIMS),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("rel_correction", ctypes.c_double * (MAX_ITERS + 1)),
        ("stop", ctypes.c_int),
    ]


ENOCONV = -6
STOP_REASONS = {0: "none", 1: "tol", 2: "max_iter", 3: "nonfinite", 4: "stalled"}


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        # FFTFEM_LIBRARY selects another build of the same library (e.g. one
        # compiled with different kernel parameters)
        path = os.environ.get("FFTFEM_LIBRARY", LIB_PATH)
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with "
                               "`python -m paper_1701_03967_amd.build`")
        L = ctypes.CDLL(path)
        vp, i64p, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
        L.fftfem_plan.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i64p, ctypes.c_int, dp, ctypes.c_double]
        L.fftfem_plan_ex.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Desc)]
        L.fftfem_solve.argtypes = [vp, vp, vp, vp]
        L.fftfem_apply_A.argtypes = [vp, vp, vp, vp]
        L.fftfem_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.fftfem_workspace_bytes.argtypes = [vp]
        L.fftfem_workspace_bytes.restype = ctypes.c_size_t
        L.fftfem_destroy.argtypes = [vp]
        L.fftfem_destroy.restype = None
        L.fftfem_status_string.argtypes = [ctypes.c_int]
        L.fftfem_status_string.restype = ctypes.c_char_p
        L.fftfem_plan_tables.argtypes = [vp, ctypes.c_int, dp, dp]
        L.fftfem_debug_transform.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int, vp]
        L.fftfem_axis_tables_host.argtypes = [ctypes.c_int, ctypes.c_int64, dp, dp]
        L.fftfem_element_matrices_host.argtypes = [ctypes.c_int, dp, dp]
        L.fftfem_set_timing.argtypes = [vp, ctypes.c_int]
        L.fftfem_get_timing.argtypes = [vp, ctypes.c_int, ctypes.c_char_p, dp,
                                        ctypes.POINTER(ctypes.c_int)]
        L.fftfem_plan_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(Desc), ctypes.c_int]
        L.fftfem_solve_batch.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
        L.fftfem_batch_get_stats.argtypes = [vp, ctypes.c_int, ctypes.POINTER(Stats)]
        L.fftfem_batch_workspace_bytes.argtypes = [vp]
        L.fftfem_batch_workspace_bytes.restype = ctypes.c_size_t
        L.fftfem_destroy_batch.argtypes = [vp]
        L.fftfem_destroy_batch.restype = None
        L.fftfem_tune.argtypes = [vp, vp]
        L.fftfem_implicit_euler.argtypes = [vp, vp, vp, vp, ctypes.c_int, vp]
        L.fftfem_tune_save.argtypes = [ctypes.c_char_p]
        L.fftfem_coefficients.argtypes = [vp, vp, vp, ctypes.c_int, vp]
        L.fftfem_synthesize.argtypes = [vp, vp, vp, vp]
        L.fftfem_dirichlet_load.argtypes = [vp, vp, vp, vp, vp, vp]
        L.fftfem_dirichlet_load_noalloc.argtypes = [vp, vp, vp, vp, vp]
        L.fftfem_tune_load.argtypes = [ctypes.c_char_p]
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise FftfemError(rc, what)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def axis_tables_host(n: int, K: int):
    """(lam, Q) of one axis computed on the host (no device needed)."""
    lam = np.zeros(n * K - 1)
    Q = np.zeros(K * n * n)
    _check(lib().fftfem_axis_tables_host(n, K, _dptr(lam), _dptr(Q)), "axis_tables_host")
    return lam, Q.reshape(K, n, n)


def element_matrices_host(n: int):
    A = np.zeros((n + 1) * (n + 1))
    C = np.zeros((n + 1) * (n + 1))
    _check(lib().fftfem_element_matrices_host(n, _dptr(A), _dptr(C)), "element_matrices_host")
    return A.reshape(n + 1, n + 1), C.reshape(n + 1, n + 1)


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _tptr(t):
    return ctypes.c_void_p(t.data_ptr())


def orders(n, N: int):
    """Element order per axis: an int (every axis) or a sequence of N ints."""
    if isinstance(n, (int, np.integer)):
        return (int(n),) * N
    ns = tuple(int(x) for x in n)
    if len(ns) != N:
        raise ValueError("one element order per axis")
    return ns


def tune_save(path: str) -> int:
    """Write the process-wide line-pass parameter table; returns its size."""
    rc = lib().fftfem_tune_save(os.fsencode(path))
    if rc < 0:
        _check(rc, "fftfem_tune_save")
    return rc


def tune_load(path: str) -> int:
    """Add a saved line-pass parameter table; returns the entries loaded."""
    rc = lib().fftfem_tune_load(os.fsencode(path))
    if rc < 0:
        _check(rc, "fftfem_tune_load")
    return rc


def make_desc(K: Sequence[int], n, diff: Sequence[float], react: float = 0.0,
              X: Optional[Sequence[float]] = None, precision: str = "fp64", max_iter: int = 0,
              tol: float = 0.0, nrhs: int = 1, algorithm: str = "a") -> "Desc":
    """n: one element order for every axis, or one per axis.  algorithm: "a"
    (FC_n transforms along every axis) or "b" (transforms along axes 2..N and
    a banded solve along axis 1; fp64 only)."""
    if algorithm not in ("a", "b"):
        raise ValueError("algorithm must be 'a' or 'b'")
    d = Desc()
    d.N = len(K)
    ns = orders(n, d.N)
    for i, k in enumerate(K):
        d.K[i] = int(k)
        d.diff[i] = float(diff[i])
        d.X[i] = float(X[i]) if X is not None else 0.0
        d.n_axis[i] = ns[i]
    d.n = ns[0]
    d.react = float(react)
    d.precision = PRECISIONS[precision]
    d.max_iter = int(max_iter)
    d.tol = float(tol)
    d.nrhs = int(nrhs)
    d.flags = ALGORITHM_B if algorithm == "b" else 0
    return d


def _stats_dict(s):
    return {"iterations": s.iterations, "converged": bool(s.converged),
            "rel_correction": list(s.rel_correction)[:max(1, s.iterations + 1)],
            "stop": STOP_REASONS.get(s.stop, s.stop)}


def _get_stats(fn, *args):
    """Statistics; FFTFEM_ENOCONV (an unconverged or non-finite solve) is
    reported in the result, not raised."""
    s = Stats()
    rc = fn(*args, ctypes.byref(s))
    if rc != ENOCONV:
        _check(rc, fn.__name__)
    return _stats_dict(s)


class Batch:
    """Independent problems solved together (one graph launch per solve).

    problems: sequence of dicts with the Plan arguments (K, n, diff, react,
    precision, max_iter, tol, nrhs).  tune: measure line-pass parameters on
    the first solve.
    """

    def __init__(self, problems, tune: bool = False):
        descs = (Desc * len(problems))()
        self.shapes = []
        for i, pr in enumerate(problems):
            descs[i] = make_desc(**pr)
            nrhs = int(pr.get("nrhs", 1))
            shape = tuple(m * int(k) - 1 for m, k in zip(orders(pr["n"], len(pr["K"])), pr["K"]))
            self.shapes.append(((nrhs,) if nrhs > 1 else ()) + shape)
        h = ctypes.c_void_p()
        _check(lib().fftfem_plan_batch(ctypes.byref(h), len(problems), descs, BATCH_TUNE if tune else 0),
               "fftfem_plan_batch")
        self._h = h
        self.count = len(problems)

    def close(self):
        if self._h:
            lib().fftfem_destroy_batch(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, fs, us, stream=None):
        """fs, us: lists of contiguous float64 device tensors (problem shapes)."""
        import torch
        if len(fs) != self.count or len(us) != self.count:
            raise ValueError("one f and one u tensor per problem")
        for t, shp in zip(list(fs) + list(us), self.shapes * 2):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                    and t.is_contiguous() and tuple(t.shape) == shp):
                raise ValueError(f"expected a contiguous float64 device tensor of shape {shp}")
        fp = (ctypes.c_void_p * self.count)(*[t.data_ptr() for t in fs])
        up = (ctypes.c_void_p * self.count)(*[t.data_ptr() for t in us])
        _check(lib().fftfem_solve_batch(self._h, fp, up, _stream_ptr(stream)), "fftfem_solve_batch")
        return us

    def stats(self, i: int):
        return _get_stats(lib().fftfem_batch_get_stats, self._h, int(i))

    def workspace_bytes(self) -> int:
        return int(lib().fftfem_batch_workspace_bytes(self._h))


class Plan:
    """A solver plan: fixed sizes, coefficients and precision mode."""

    def __init__(self, K: Sequence[int], n, diff: Sequence[float], react: float = 0.0,
                 X: Optional[Sequence[float]] = None, precision: str = "fp64",
                 max_iter: int = 0, tol: float = 0.0, nrhs: int = 1, algorithm: str = "a"):
        d = make_desc(K, n, diff, react, X, precision, max_iter, tol, nrhs, algorithm)
        h = ctypes.c_void_p()
        _check(lib().fftfem_plan_ex(ctypes.byref(h), ctypes.byref(d)), "fftfem_plan_ex")
        self._h = h
        self.K = tuple(int(k) for k in K)
        self.orders = orders(n, len(self.K))
        self.n = n if isinstance(n, (int, np.integer)) else self.orders
        self.nrhs = int(nrhs)
        self.shape = tuple(m * k - 1 for m, k in zip(self.orders, self.K))
        self.precision = precision
        self.algorithm = algorithm

    def close(self):
        if self._h:
            lib().fftfem_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _full_shape(self):
        return ((self.nrhs,) if self.nrhs > 1 else ()) + self.shape

    def _check_tensor(self, t, name):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and t.is_contiguous() and tuple(t.shape) == self._full_shape()):
            raise ValueError(f"{name} must be a contiguous float64 device tensor of shape "
                             f"{self._full_shape()}")

    def solve(self, f, u=None, stream=None):
        import torch
        self._check_tensor(f, "f")
        if u is None:
            u = torch.empty_like(f)
        self._check_tensor(u, "u")
        _check(lib().fftfem_solve(self._h, _tptr(f), _tptr(u), _stream_ptr(stream)), "fftfem_solve")
        return u

    def apply_A(self, u, y=None, stream=None):
        import torch
        self._check_tensor(u, "u")
        if y is None:
            y = torch.empty_like(u)
        self._check_tensor(y, "y")
        _check(lib().fftfem_apply_A(self._h, _tptr(u), _tptr(y), _stream_ptr(stream)), "fftfem_apply_A")
        return y

    def coefficients(self, x, out=None, kind: str = "values", stream=None):
        """Expansion coefficients in the tensor eigenbasis: of grid values
        (kind "values", the direct F_n transform) or of a load ("loads",
        the direct FC_n transform)."""
        import torch
        self._check_tensor(x, "x")
        if out is None:
            out = torch.empty_like(x)
        self._check_tensor(out, "out")
        k = {"values": 0, "loads": 1}[kind]
        _check(lib().fftfem_coefficients(self._h, _tptr(x), _tptr(out), k, _stream_ptr(stream)),
               "fftfem_coefficients")
        return out

    def synthesize(self, c, out=None, stream=None):
        """Grid values of the expansion with coefficients c."""
        import torch
        self._check_tensor(c, "c")
        if out is None:
            out = torch.empty_like(c)
        self._check_tensor(out, "out")
        _check(lib().fftfem_synthesize(self._h, _tptr(c), _tptr(out), _stream_ptr(stream)), "fftfem_synthesize")
        return out

    @property
    def extended_shape(self):
        """Shape of boundary data: every axis with its two boundary points."""
        sh = tuple(m + 2 for m in self.shape)
        return (self.nrhs,) + sh if self.nrhs > 1 else sh

    def dirichlet_load(self, b, f, out=None, work=None, stream=None):
        """f - A_IB b: the load of the homogeneous system whose solution is
        the interior of the solution with boundary values b (extended-grid
        float64 device tensor; only its boundary entries are read)."""
        import torch
        if not (isinstance(b, torch.Tensor) and b.is_cuda and b.dtype == torch.float64 and b.is_contiguous()
                and tuple(b.shape) == self.extended_shape):
            raise ValueError(f"b must be a contiguous float64 device tensor of shape {self.extended_shape}")
        self._check_tensor(f, "f")
        if out is None:
            out = torch.empty_like(f)
        self._check_tensor(out, "out")
        ne = 1
        for m in self.shape:
            ne *= m + 2
        if work is None:
            work = torch.empty(2 * ne, dtype=torch.float64, device=f.device)
        if not (isinstance(work, torch.Tensor) and work.is_cuda and work.dtype == torch.float64
                and work.is_contiguous() and work.numel() >= 2 * ne):
            raise ValueError(f"work must be a contiguous float64 device tensor of at least {2 * ne} values")
        _check(lib().fftfem_dirichlet_load(self._h, _tptr(b), _tptr(f), _tptr(out), _tptr(work),
                                           _stream_ptr(stream)), "fftfem_dirichlet_load")
        return out

    def dirichlet_load_noalloc(self, b, f, out, stream=None):
        """dirichlet_load with the library's static device work area instead of
        a work array (fftfem_dirichlet_load_noalloc): nothing is allocated,
        so `out` must be given."""
        import torch
        if not (isinstance(b, torch.Tensor) and b.is_cuda and b.dtype == torch.float64 and b.is_contiguous()
                and tuple(b.shape) == self.extended_shape):
            raise ValueError(f"b must be a contiguous float64 device tensor of shape {self.extended_shape}")
        self._check_tensor(f, "f")
        self._check_tensor(out, "out")
        _check(lib().fftfem_dirichlet_load_noalloc(self._h, _tptr(b), _tptr(f), _tptr(out), _stream_ptr(stream)),
               "fftfem_dirichlet_load_noalloc")
        return out

    def implicit_euler(self, u, nsteps: int, F=None, work=None, stream=None):
        """nsteps implicit Euler steps of C du/dt + A_diff u = F with
        tau = 1/react, in place on u (float64 device tensor); F: constant load
        or None; work: scratch of u's shape (allocated when None)."""
        import torch
        self._check_tensor(u, "u")
        if F is not None:
            self._check_tensor(F, "F")
        if work is None:
            work = torch.empty_like(u)
        self._check_tensor(work, "work")
        _check(lib().fftfem_implicit_euler(self._h, _tptr(F) if F is not None else None, _tptr(u), _tptr(work),
                                           int(nsteps), _stream_ptr(stream)), "fftfem_implicit_euler")
        return u

    def tune(self, stream=None):
        """Measures this plan's line-pass parameters (2D plans; the choice is
        kept process-wide for plans of the same kind)."""
        _check(lib().fftfem_tune(self._h, _stream_ptr(stream)), "fftfem_tune")

    def stats(self):
        """Refinement statistics of the last solve: iterations, converged,
        rel_correction (per iteration), stop (why the refinement stopped:
        none, tol, max_iter, nonfinite, stalled)."""
        return _get_stats(lib().fftfem_get_stats, self._h)

    def tables(self, axis: int):
        M = self.shape[axis]
        K = self.K[axis]
        lam = np.zeros(M)
        m = self.orders[axis]
        Q = np.zeros(K * m * m)
        _check(lib().fftfem_plan_tables(self._h, axis, _dptr(lam), _dptr(Q)), "fftfem_plan_tables")
        return lam, Q.reshape(K, m, m)

    def set_timing(self, enable: bool = True):
        _check(lib().fftfem_set_timing(self._h, int(enable)), "fftfem_set_timing")

    def get_timing(self):
        """{kernel name: (mean ms, launches)} since the last call."""
        mx = 64
        names = ctypes.create_string_buffer(32 * mx)
        avg = np.zeros(mx)
        cnt = (ctypes.c_int * mx)()
        nk = lib().fftfem_get_timing(self._h, mx, names, _dptr(avg), cnt)
        if nk < 0:
            _check(nk, "fftfem_get_timing")
        out = {}
        for i in range(min(nk, mx)):
            nm = names.raw[32 * i:32 * (i + 1)].split(b"\0", 1)[0].decode()
            out[nm] = (float(avg[i]), int(cnt[i]))
        return out

    def workspace_bytes(self) -> int:
        return int(lib().fftfem_workspace_bytes(self._h))

    def debug_transform(self, axis: int, direction: int, x, out=None, dtype: str = "fp64",
                        stream=None):
        import torch
        self._check_tensor(x, "x")
        if out is None:
            out = torch.empty_like(x)
        _check(lib().fftfem_debug_transform(self._h, axis, direction, _tptr(x), _tptr(out),
                                            0 if dtype == "fp64" else 1, _stream_ptr(stream)),
               "fftfem_debug_transform")
        return out
