"""Python binding of libtdsolve.so (ctypes).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels.  PyTorch supplies device memory and the current HIP stream.
If the shared library is missing this module raises on first use; there is
no CPU fallback.

Arrays use the library's RHS-interleaved layout: a tensor of shape (M, N)
whose column n is right-hand side n (row-major, contiguous).
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os
import weakref
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdsolve.so")

MODES = {"f64": 0, "f32_refined": 1, "f32": 2, "f32_wide": 3}
_F_DTYPE = {0: "float64", 1: "float32", 2: "float32", 3: "float32"}
_X_DTYPE = {0: "float64", 1: "float64", 2: "float32", 3: "float64"}

SYMBOLS = [
    "tdsolve_prepare", "tdsolve_prepare_general", "tdsolve_series", "tdsolve_components",
    "tdsolve_backward",
    "tdsolve_residual", "tdsolve_set_refinement", "tdsolve_info", "tdsolve_prepare_host",
    "tdsolve_default_blocks", "tdsolve_destroy", "tdsolve_strerror",
    "tdsolve_batch_prepare", "tdsolve_batch_series", "tdsolve_timing_enable",
    "tdsolve_timing_read", "tdsolve_autotune", "tdsolve_batch_autotune", "tdsolve_autotune_plan",
    "tdsolve_prepare_host_general", "tdsolve_set_interface", "tdsolve_dense_table_host",
    "tdsolve_status", "tdsolve_strided_copy", "tdsolve_series_noalloc", "tdsolve_set_fused",
    "tdsolve_batch_set_fused",
]

_lib = None


class TdsError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.tdsolve_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} (status {code})")
        self.code = code


class Tuning(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int32), ("order", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("fuse_lag", ctypes.c_int32), ("fuse_tile", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("ms", ctypes.c_double), ("r2", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("P", ctypes.c_int32), ("max_block", ctypes.c_int32),
                ("dominant", ctypes.c_int32), ("refine_passes", ctypes.c_int32),
                ("max_ratio", ctypes.c_double), ("general", ctypes.c_int32),
                ("sweep_halves", ctypes.c_int32)]


def lib():
    """Load libtdsolve.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c "
                           "'import __graft_entry__ as g; g.build()'` (no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    L.tdsolve_prepare.argtypes = [dp, dp, i64, i32, ctypes.POINTER(vp)]
    L.tdsolve_prepare_general.argtypes = [dp, dp, dp, i64, i32, ctypes.POINTER(vp)]
    L.tdsolve_series.argtypes = [vp, vp, vp, i64, i32, vp]
    L.tdsolve_series_noalloc.argtypes = [vp, vp, vp, i64, i32, vp]
    L.tdsolve_components.argtypes = [vp, vp, vp, i64, i32, vp]
    L.tdsolve_backward.argtypes = [vp, vp, vp, vp, vp, vp, i64, i32, vp]
    L.tdsolve_residual.argtypes = [vp, vp, vp, i64, i32, vp, vp]
    L.tdsolve_set_refinement.argtypes = [vp, i32]
    L.tdsolve_set_fused.argtypes = [vp, i32, i32]
    L.tdsolve_batch_set_fused.argtypes = [vp, i32]
    L.tdsolve_set_interface.argtypes = [vp, i32]
    L.tdsolve_info.argtypes = [vp, ctypes.POINTER(Info)]
    L.tdsolve_prepare_host.argtypes = [dp, dp, i64, i32, dp, dp, dp, dp, dp, dp]
    L.tdsolve_prepare_host_general.argtypes = [dp, dp, dp, i64, i32, dp, dp, dp, dp, dp, dp]
    L.tdsolve_dense_table_host.argtypes = [dp, dp, i64, i32, dp]
    L.tdsolve_default_blocks.argtypes = [i64]
    L.tdsolve_default_blocks.restype = i32
    L.tdsolve_destroy.argtypes = [vp]
    L.tdsolve_strerror.argtypes = [ctypes.c_int]
    L.tdsolve_strerror.restype = ctypes.c_char_p
    L.tdsolve_batch_prepare.argtypes = [i32, vp, vp, vp, vp, ctypes.POINTER(vp)]
    L.tdsolve_batch_series.argtypes = [vp, vp, vp, vp, i32, vp]
    L.tdsolve_status.argtypes = [vp, vp, vp, vp]
    L.tdsolve_strided_copy.argtypes = [vp, vp, i32, i64, i64, i64, vp, vp, ctypes.c_double, vp]
    L.tdsolve_timing_enable.argtypes = [vp, i32]
    L.tdsolve_timing_read.argtypes = [vp, vp, vp]
    L.tdsolve_autotune.argtypes = [dp, dp, i64, i64, i32, i32, vp, vp, vp]
    L.tdsolve_batch_autotune.argtypes = [i32, vp, vp, vp, vp, i32, i32, vp, vp, vp, vp, vp]
    L.tdsolve_autotune_plan.argtypes = [dp, dp, i64, i64, i32, i32, vp, i32,
                                        ctypes.POINTER(Tuning), vp]
    for name in SYMBOLS:
        if name not in ("tdsolve_default_blocks", "tdsolve_strerror"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(code: int, where: str):
    if code != 0:
        raise TdsError(code, where)


def _host_f64(x) -> np.ndarray:
    if hasattr(x, "detach"):
        x = x.detach().to("cpu").numpy()
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _ptr(arr: np.ndarray):
    return arr.ctypes.data_as(ctypes.c_void_p)


def mode_id(mode) -> int:
    if isinstance(mode, str):
        return MODES[mode]
    return int(mode)


def default_blocks(M: int) -> int:
    return int(lib().tdsolve_default_blocks(M))


def prepare_host(a, b, P: int):
    """FP64 tables of the preliminary step computed on the host (no GPU)."""
    L = lib()
    b = _host_f64(b)
    M = b.shape[0]
    a = _host_f64(a) if M > 1 else np.zeros(1)
    if P == 0:
        P = default_blocks(M)
    starts = np.zeros(P + 1, dtype=np.int64)
    wR, wL, dinv = np.zeros(M), np.zeros(M), np.zeros(M)
    rho, lam = np.zeros(P), np.zeros(P)
    _check(L.tdsolve_prepare_host(_ptr(a), _ptr(b), M, P, _ptr(starts), _ptr(wR), _ptr(wL),
                                  _ptr(rho), _ptr(lam), _ptr(dinv)), "tdsolve_prepare_host")
    return dict(starts=starts, wR=wR, wL=wL, rho=rho, lam=lam, diag_inv=dinv, P=P, M=M)


def dense_table_host(a, b, P: int):
    """Theorem 2's coefficients as the (P-1) x 2P matrix of the dense
    interface order (tdsolve_dense_table_host), computed on the host."""
    L = lib()
    b = _host_f64(b)
    M = b.shape[0]
    a = _host_f64(a) if M > 1 else np.zeros(1)
    K = np.zeros((max(P - 1, 0), 2 * P))
    _check(L.tdsolve_dense_table_host(_ptr(a), _ptr(b), M, P, _ptr(K)), "tdsolve_dense_table_host")
    return K


def prepare_host_general(lower, diag, upper, P: int):
    """prepare_host() for a non-symmetric A (tdsolve_prepare_host_general)."""
    L = lib()
    d = _host_f64(diag)
    M = d.shape[0]
    lo = _host_f64(lower) if M > 1 else np.zeros(1)
    up = _host_f64(upper) if M > 1 else np.zeros(1)
    if P == 0:
        P = default_blocks(M)
    starts = np.zeros(P + 1, dtype=np.int64)
    wR, wL, dinv = np.zeros(M), np.zeros(M), np.zeros(M)
    rho, lam = np.zeros(P), np.zeros(P)
    _check(L.tdsolve_prepare_host_general(_ptr(lo), _ptr(d), _ptr(up), M, P, _ptr(starts),
                                          _ptr(wR), _ptr(wL), _ptr(rho), _ptr(lam), _ptr(dinv)),
           "tdsolve_prepare_host_general")
    return dict(starts=starts, wR=wR, wL=wL, rho=rho, lam=lam, diag_inv=dinv, P=P, M=M)


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def strided_copy(dst, src, alpha: float = 1.0, stream=None):
    """dst = alpha * src for two device views of one shape (S, M, L) and one
    dtype (float32 or float64), any non-negative strides
    (tdsolve_strided_copy: LDS tiles of (s, l) per i, so a transposing copy
    reads and writes whole rows)."""
    import torch
    if tuple(dst.shape) != tuple(src.shape) or dst.dim() != 3:
        raise ValueError("dst and src must be views of one (S, M, L) shape")
    if dst.dtype != src.dtype or src.dtype not in (torch.float32, torch.float64):
        raise TypeError("dst and src must both be float32 or both float64")
    if not (dst.is_cuda and src.is_cuda):
        raise ValueError("dst and src must be device tensors")
    S, M, L = src.shape
    ss = np.array(src.stride(), dtype=np.int64)
    ds = np.array(dst.stride(), dtype=np.int64)
    _check(lib().tdsolve_strided_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                      int(src.dtype == torch.float64), S, M, L, _ptr(ss), _ptr(ds),
                                      float(alpha), _stream_ptr(stream)), "tdsolve_strided_copy")
    return dst


def _status(h, stream):
    err = ctypes.c_double()
    passes = ctypes.c_int32()
    _check(lib().tdsolve_status(h, _stream_ptr(stream), ctypes.byref(err), ctypes.byref(passes)),
           "tdsolve_status")
    return float(err.value), int(passes.value)


class Plan:
    """A prepared matrix (preliminary step of the method, done once)."""

    def __init__(self, a, b, P: Optional[int] = None):
        L = lib()
        b = _host_f64(b)
        M = int(b.shape[0])
        a = _host_f64(a) if M > 1 else np.zeros(1)
        h = ctypes.c_void_p()
        _check(L.tdsolve_prepare(_ptr(a), _ptr(b), M, int(P or 0), ctypes.byref(h)),
               "tdsolve_prepare")
        self._h = h
        self.M = M
        info = self.info()
        self.P = info.P

    @classmethod
    def general(cls, lower, diag, upper, P: Optional[int] = None):
        """Plan for a non-symmetric tridiagonal matrix (row i: lower[i-1]
        x_{i-1} + diag[i] x_i + upper[i] x_{i+1}); needs lower[i] * upper[i]
        > 0 (tdsolve_prepare_general).  No backward()."""
        L = lib()
        d = _host_f64(diag)
        M = int(d.shape[0])
        lo = _host_f64(lower) if M > 1 else np.zeros(1)
        up = _host_f64(upper) if M > 1 else np.zeros(1)
        if M > 1 and (lo.shape[0] != M - 1 or up.shape[0] != M - 1):
            raise ValueError("lower and upper need M-1 entries")
        h = ctypes.c_void_p()
        _check(L.tdsolve_prepare_general(_ptr(lo), _ptr(d), _ptr(up), M, int(P or 0),
                                         ctypes.byref(h)), "tdsolve_prepare_general")
        self = cls.__new__(cls)
        self._h = h
        self.M = M
        self.P = self.info().P
        return self

    def info(self) -> Info:
        out = Info()
        _check(lib().tdsolve_info(self._h, ctypes.byref(out)), "tdsolve_info")
        return out

    def timing(self, on: bool = True):
        _check(lib().tdsolve_timing_enable(self._h, int(bool(on))), "tdsolve_timing_enable")

    def timing_read(self):
        """(ms_beta, ms_interface, ms_sweep, calls) accumulated since the last read."""
        ms = np.zeros(3)
        calls = np.zeros(1, dtype=np.int64)
        _check(lib().tdsolve_timing_read(self._h, _ptr(ms), _ptr(calls)), "tdsolve_timing_read")
        return float(ms[0]), float(ms[1]), float(ms[2]), int(calls[0])

    def status(self, stream=None):
        """(largest normwise backward error, refinement passes) of the last
        solve; synchronises (tdsolve_status)."""
        return _status(self._h, stream)

    def set_interface(self, order: str):
        """'recurrence' (default, Theorem 2 as two recurrences), 'dichotomy'
        (Algorithm 4, level by level) or 'dense' (Theorem 2's double sum as
        one product on the FP64 matrix cores; P <= 1024)."""
        code = {"recurrence": 0, "dichotomy": 1, "dense": 2}[order]
        _check(lib().tdsolve_set_interface(self._h, code), "tdsolve_set_interface")

    def set_refinement(self, passes: int):
        _check(lib().tdsolve_set_refinement(self._h, int(passes)), "tdsolve_set_refinement")

    def set_fused(self, lag: int, tile: int = 1024):
        """The fused order (one launch; the sweeps of a tile of `tile`
        right-hand sides `lag` tiles behind its weights), or the three
        launches (lag 0)."""
        _check(lib().tdsolve_set_fused(self._h, int(lag), int(tile)), "tdsolve_set_fused")

    def _check_tensor(self, t, dtype: str, name: str, rows: Optional[int] = None):
        import torch
        want = getattr(torch, dtype)
        rows = self.M if rows is None else rows
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
        if t.dtype != want:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if t.dim() != 2 or t.shape[0] != rows or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous ({rows}, N) tensor")

    def solve(self, F, X=None, mode=None, stream=None):
        """X = A^{-1} F for every column of F (device tensors, (M, N))."""
        import torch
        m = mode_id(mode if mode is not None else ("f64" if F.dtype == torch.float64 else "f32_refined"))
        self._check_tensor(F, _F_DTYPE[m], "F")
        N = F.shape[1]
        if X is None:
            X = torch.empty((self.M, N), dtype=getattr(torch, _X_DTYPE[m]), device=F.device)
        self._check_tensor(X, _X_DTYPE[m], "X")
        if X.shape[1] != N:
            raise ValueError("X and F differ in N")
        _check(lib().tdsolve_series(self._h, ctypes.c_void_p(F.data_ptr()),
                                    ctypes.c_void_p(X.data_ptr()), N, m, _stream_ptr(stream)),
               "tdsolve_series")
        return X

    def solve_noalloc(self, F, X, mode=None, stream=None):
        """As solve() into a given X, by the entry point that allocates
        nothing (tdsolve_series_noalloc: the work area is the library's fixed
        device scratch, shared by every call on the GPU)."""
        import torch
        m = mode_id(mode if mode is not None else ("f64" if F.dtype == torch.float64 else "f32_refined"))
        self._check_tensor(F, _F_DTYPE[m], "F")
        self._check_tensor(X, _X_DTYPE[m], "X")
        if X.shape[1] != F.shape[1]:
            raise ValueError("X and F differ in N")
        _check(lib().tdsolve_series_noalloc(self._h, ctypes.c_void_p(F.data_ptr()),
                                            ctypes.c_void_p(X.data_ptr()), F.shape[1], m,
                                            _stream_ptr(stream)), "tdsolve_series_noalloc")
        return X

    def components(self, F, mode=None, stream=None):
        """Algorithm 3 alone: x at the P-1 interface rows, shape (P-1, N), FP64."""
        import torch
        m = mode_id(mode if mode is not None else ("f64" if F.dtype == torch.float64 else "f32_refined"))
        self._check_tensor(F, _F_DTYPE[m], "F")
        N = F.shape[1]
        out = torch.empty((max(self.P - 1, 0), N), dtype=torch.float64, device=F.device)
        if self.P > 1 and N > 0:
            _check(lib().tdsolve_components(self._h, ctypes.c_void_p(F.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()), N, m,
                                            _stream_ptr(stream)), "tdsolve_components")
        return out

    def residual(self, F, X, mode=None, stream=None):
        """(eta, r2) per right-hand side, each an FP64 device tensor of N."""
        import torch
        m = mode_id(mode if mode is not None else ("f64" if F.dtype == torch.float64 else "f32_refined"))
        self._check_tensor(F, _F_DTYPE[m], "F")
        self._check_tensor(X, _X_DTYPE[m], "X")
        N = F.shape[1]
        out = torch.zeros(2 * N, dtype=torch.float64, device=F.device)
        _check(lib().tdsolve_residual(self._h, ctypes.c_void_p(F.data_ptr()),
                                      ctypes.c_void_p(X.data_ptr()), N, m,
                                      ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
               "tdsolve_residual")
        return out[:N], out[N:]

    def backward(self, X, gX, mode=None, want_ga=True, want_gb=True, stream=None):
        """Adjoint: (gF, ga, gb) for dL/dX = gX at the solution X."""
        import torch
        m = mode_id(mode if mode is not None else ("f64" if X.dtype == torch.float64 else "f32"))
        self._check_tensor(X, _X_DTYPE[m], "X")
        self._check_tensor(gX, _X_DTYPE[m], "gX")
        N = X.shape[1]
        gF = torch.empty((self.M, N), dtype=getattr(torch, _F_DTYPE[m]), device=X.device)
        ga = torch.empty(max(self.M - 1, 0), dtype=torch.float64, device=X.device) if want_ga else None
        gb = torch.empty(self.M, dtype=torch.float64, device=X.device) if want_gb else None
        pga = ctypes.c_void_p(ga.data_ptr()) if (ga is not None and ga.numel()) else None
        pgb = ctypes.c_void_p(gb.data_ptr()) if gb is not None else None
        _check(lib().tdsolve_backward(self._h, ctypes.c_void_p(X.data_ptr()),
                                      ctypes.c_void_p(gX.data_ptr()),
                                      ctypes.c_void_p(gF.data_ptr()), pga, pgb, N, m,
                                      _stream_ptr(stream)), "tdsolve_backward")
        return gF, ga, gb

    def close(self):
        if getattr(self, "_h", None):
            lib().tdsolve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """K independent matrices of uneven sizes prepared together; every
    series solve of the batch is one launch per step of the method for all
    K matrices (tdsolve_batch_series)."""

    def __init__(self, a_list, b_list, P_list=None):
        L = lib()
        K = len(b_list)
        if K < 1 or len(a_list) != K:
            raise ValueError("need K >= 1 matrices with matching a and b")
        self._bs = [_host_f64(b) for b in b_list]
        self._as = [(_host_f64(a) if len(b) > 1 else np.zeros(1)) for a, b in zip(a_list, self._bs)]
        self.M = [int(b.shape[0]) for b in self._bs]
        Ms = np.array(self.M, dtype=np.int64)
        Ps = np.array(P_list if P_list is not None else [0] * K, dtype=np.int32)
        ap = (ctypes.c_void_p * K)(*[x.ctypes.data for x in self._as])
        bp = (ctypes.c_void_p * K)(*[x.ctypes.data for x in self._bs])
        h = ctypes.c_void_p()
        _check(L.tdsolve_batch_prepare(K, ap, bp, _ptr(Ms), _ptr(Ps), ctypes.byref(h)),
               "tdsolve_batch_prepare")
        self._h = h
        self.K = K

    def timing(self, on: bool = True):
        _check(lib().tdsolve_timing_enable(self._h, int(bool(on))), "tdsolve_timing_enable")

    def timing_read(self):
        """(ms_beta, ms_interface, ms_sweep, calls) accumulated since the last read."""
        ms = np.zeros(3)
        calls = np.zeros(1, dtype=np.int64)
        _check(lib().tdsolve_timing_read(self._h, _ptr(ms), _ptr(calls)), "tdsolve_timing_read")
        return float(ms[0]), float(ms[1]), float(ms[2]), int(calls[0])

    def status(self, stream=None):
        """(largest normwise backward error over all matrices, refinement
        passes) of the last batch solve; synchronises (tdsolve_status)."""
        return _status(self._h, stream)

    def set_refinement(self, passes: int):
        _check(lib().tdsolve_set_refinement(self._h, int(passes)), "tdsolve_set_refinement")

    def set_fused(self, lag: int):
        """The one-launch order (every matrix's items in one grid, the
        interface items `lag` tiles of 256 right-hand sides and the sweeps 2
        `lag` tiles behind the weights; taken when every matrix has blocks
        of at most 32 rows), or the separate launches (lag 0)."""
        _check(lib().tdsolve_batch_set_fused(self._h, int(lag)), "tdsolve_batch_set_fused")

    def solve(self, F_list, X_list=None, mode="f32_refined", stream=None):
        import torch
        m = mode_id(mode)
        if len(F_list) != self.K:
            raise ValueError("one right-hand-side array per matrix")
        if X_list is None:
            X_list = [torch.empty((self.M[k], F_list[k].shape[1]),
                                  dtype=getattr(torch, _X_DTYPE[m]), device=F_list[k].device)
                      for k in range(self.K)]
        Ns = np.zeros(self.K, dtype=np.int64)
        for k in range(self.K):
            F, X = F_list[k], X_list[k]
            for t_, name, dt in ((F, "F", _F_DTYPE[m]), (X, "X", _X_DTYPE[m])):
                if not t_.is_cuda or t_.dtype != getattr(torch, dt) or t_.dim() != 2 \
                        or t_.shape[0] != self.M[k] or not t_.is_contiguous():
                    raise ValueError(f"{name}[{k}] must be a contiguous ({self.M[k]}, N) {dt} device tensor")
            if X.shape[1] != F.shape[1]:
                raise ValueError(f"X[{k}] and F[{k}] differ in N")
            Ns[k] = F.shape[1]
        Fp = (ctypes.c_void_p * self.K)(*[F.data_ptr() for F in F_list])
        Xp = (ctypes.c_void_p * self.K)(*[X.data_ptr() for X in X_list])
        _check(lib().tdsolve_batch_series(self._h, Fp, Xp, _ptr(Ns), m, _stream_ptr(stream)),
               "tdsolve_batch_series")
        return X_list

    def solve_stacked(self, F, X=None, mode="f32_refined", stream=None):
        """The batch with every matrix of the same size M and the same series
        length N, given as one contiguous (K, M, N) tensor (matrix k's
        right-hand sides in F[k]); returns X of the same shape."""
        import torch
        m = mode_id(mode)
        if not (F.is_cuda and F.dim() == 3 and F.shape[0] == self.K and F.is_contiguous()
                and F.dtype == getattr(torch, _F_DTYPE[m])):
            raise ValueError(f"F must be a contiguous (K, M, N) {_F_DTYPE[m]} device tensor")
        K, M, N = F.shape
        if any(mk != M for mk in self.M):
            raise ValueError("solve_stacked needs matrices of one size")
        if X is None:
            X = torch.empty((K, M, N), dtype=getattr(torch, _X_DTYPE[m]), device=F.device)
        elif not (X.is_cuda and tuple(X.shape) == (K, M, N) and X.is_contiguous()
                  and X.dtype == getattr(torch, _X_DTYPE[m])):
            raise ValueError("X must match F")
        k = np.arange(K, dtype=np.uint64)
        Fp = (F.data_ptr() + k * np.uint64(M * N * F.element_size())).astype(np.uint64)
        Xp = (X.data_ptr() + k * np.uint64(M * N * X.element_size())).astype(np.uint64)
        Ns = np.full(K, N, dtype=np.int64)
        _check(lib().tdsolve_batch_series(self._h, _ptr(Fp), _ptr(Xp), _ptr(Ns), m,
                                          _stream_ptr(stream)), "tdsolve_batch_series")
        return X

    def close(self):
        if getattr(self, "_h", None):
            lib().tdsolve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _cache_path():
    return os.environ.get("TDSOLVE_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "tdsolve",
                                       "autotune.json"))


def _device_key():
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(p, 'gcnArchName', p.name)}:{p.multi_processor_count}"


def _cache_load():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _cache_store(key, value):
    path = _cache_path()
    data = _cache_load()
    data[key] = value
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass                     # an unwritable cache only costs a re-measurement


def autotune(a, b, N: int, mode="f32_refined", reps: int = 5, cache: bool = True,
             stream=None):
    """Block count P for solving series of N right-hand sides with the
    tridiagonal matrix (a, b) in `mode`, measured on the current device by
    tdsolve_autotune (fastest of blocks of <= 16/32/64/128 rows).  Results
    are cached in a JSON file (TDSOLVE_AUTOTUNE_CACHE, default
    ~/.cache/tdsolve/autotune.json) by device, M, N and mode: the timing
    does not depend on the matrix values.  Returns (P, ms per solve)."""
    m = mode_id(mode)
    b = _host_f64(b)
    M = int(b.shape[0])
    a = _host_f64(a) if M > 1 else np.zeros(1)
    key = f"single|{_device_key()}|M={M}|N={int(N)}|mode={m}"
    if cache:
        hit = _cache_load().get(key)
        if hit is not None:
            return int(hit["P"]), float(hit["ms"])
    P = ctypes.c_int32()
    ms = ctypes.c_double()
    _check(lib().tdsolve_autotune(_ptr(a), _ptr(b), M, int(N), m, int(reps), ctypes.byref(P),
                                  ctypes.byref(ms), _stream_ptr(stream)), "tdsolve_autotune")
    if cache:
        _cache_store(key, {"P": P.value, "ms": ms.value})
    return P.value, ms.value


def batch_autotune(a_list, b_list, N_list, mode="f32_refined", reps: int = 5,
                   cache: bool = True, stream=None, with_passes: bool = False,
                   with_order: bool = False):
    """Block counts for an uneven batch (tdsolve_batch_autotune: 32 or 64
    rows per block for every matrix, then per class of matrices by size,
    timed on the whole batch, the refinement passes of the refined mode
    chosen by accuracy, then the launch order).  Cached like autotune(), by
    device, mode and the digest of the (M, N) list.  Returns (list of P, ms
    per batch solve), (list of P, passes, ms) with with_passes, or (list of
    P, passes, lag of the one-launch order (0: separate launches), ms) with
    with_order."""
    m = mode_id(mode)
    K = len(b_list)
    bs = [_host_f64(b) for b in b_list]
    as_ = [(_host_f64(a) if len(b) > 1 else np.zeros(1)) for a, b in zip(a_list, bs)]
    Ms = np.array([x.shape[0] for x in bs], dtype=np.int64)
    Ns = np.array([int(n) for n in N_list], dtype=np.int64)
    digest = hashlib.sha256(Ms.tobytes() + Ns.tobytes()).hexdigest()[:16]
    key = f"batch-order|{_device_key()}|K={K}|MN={digest}|mode={m}"
    hit = _cache_load().get(key) if cache else None
    if hit is not None and "lag" in hit:
        Pl, passes, lag = [int(p) for p in hit["P"]], int(hit["passes"]), int(hit["lag"])
        ms = float(hit["ms"])
    else:
        ap = (ctypes.c_void_p * K)(*[x.ctypes.data for x in as_])
        bp = (ctypes.c_void_p * K)(*[x.ctypes.data for x in bs])
        Ps = np.zeros(K, dtype=np.int32)
        npass = ctypes.c_int32()
        nlag = ctypes.c_int32()
        msv = ctypes.c_double()
        _check(lib().tdsolve_batch_autotune(K, ap, bp, _ptr(Ms), _ptr(Ns), m, int(reps),
                                            _ptr(Ps), ctypes.byref(npass), ctypes.byref(nlag),
                                            ctypes.byref(msv), _stream_ptr(stream)),
               "tdsolve_batch_autotune")
        Pl, passes, lag, ms = Ps.tolist(), int(npass.value), int(nlag.value), float(msv.value)
        if cache:
            _cache_store(key, {"P": Pl, "passes": passes, "lag": lag, "ms": ms})
    if with_order:
        return Pl, passes, lag, ms
    return (Pl, passes, ms) if with_passes else (Pl, ms)


def autotune_plan(a, b, N: int, mode="f32_refined", P: int = 0, F=None, reps: int = 5,
                  stream=None):
    """Measured configuration of a single-matrix plan (tdsolve_autotune_plan):
    block count (P = 0: chosen; else fixed), interface order, fused order and
    the refined mode's passes, on the device right-hand sides F ((M, N), the
    mode's input type) or generated ones.  Returns a dict with P, order
    ('recurrence' or 'dense'), passes, fuse_lag, fuse_tile, ms, r2."""
    m = mode_id(mode)
    b = _host_f64(b)
    M = int(b.shape[0])
    a = _host_f64(a) if M > 1 else np.zeros(1)
    fp = None
    if F is not None:
        Plan._check_tensor(None, F, _F_DTYPE[m], "F", rows=M)
        if F.shape[1] != N:
            raise ValueError("F must have N columns")
        fp = ctypes.c_void_p(F.data_ptr())
    out = Tuning()
    _check(lib().tdsolve_autotune_plan(_ptr(a), _ptr(b), M, int(N), m, int(P), fp, int(reps),
                                       ctypes.byref(out), _stream_ptr(stream)),
           "tdsolve_autotune_plan")
    return {"P": out.P, "order": {0: "recurrence", 2: "dense"}.get(out.order, "recurrence"),
            "passes": out.passes, "fuse_lag": out.fuse_lag, "fuse_tile": out.fuse_tile,
            "ms": out.ms, "r2": out.r2}


# Plans of the differentiable solve, reused while a and b are the same
# tensors with the same in-place version (weak references: a freed tensor,
# or one whose storage address is reused, never matches).
_PLAN_CACHE_SIZE = 8
_plan_cache: list = []


def _version(x):
    return getattr(x, "_version", None)


def cached_plan(a, b, P=None):
    """A Plan for (a, b, P), taken from the cache while a and b are the same
    objects, unmodified in place since the plan was made (torch tensors carry
    an in-place version counter; other arrays are matched by identity only,
    so they must not be modified in place between calls)."""
    for ra, rb, va, vb, p, plan in reversed(_plan_cache):
        if ra() is a and rb() is b and va == _version(a) and vb == _version(b) and p == P:
            return plan
    plan = Plan(a, b, P)
    try:
        entry = (weakref.ref(a), weakref.ref(b), _version(a), _version(b), P, plan)
    except TypeError:                 # objects without weak references: no caching
        return plan
    _plan_cache.append(entry)
    del _plan_cache[:-_PLAN_CACHE_SIZE]
    return plan


def _autograd_fn():
    import torch

    class TDSolveFn(torch.autograd.Function):
        """X = A(a, b)^{-1} F with gradients for F, a and b.

        The backward pass reuses the forward's prepared plan: A is symmetric,
        so gF = A^{-1} gX is another solve with the same tables (Lemma 2)."""

        @staticmethod
        def forward(ctx, F, a, b, P=None, mode=None):
            plan = cached_plan(a, b, P)
            m = mode_id(mode if mode is not None else ("f64" if F.dtype == torch.float64 else "f32_refined"))
            X = plan.solve(F.contiguous(), mode=m)
            ctx.plan, ctx.mode = plan, m
            ctx.a_meta = (a.dtype, a.device)
            ctx.b_meta = (b.dtype, b.device)
            ctx.save_for_backward(X)
            return X

        @staticmethod
        def backward(ctx, gX):
            (X,) = ctx.saved_tensors
            need_F, need_a, need_b = ctx.needs_input_grad[:3]
            gF, ga, gb = ctx.plan.backward(X, gX.contiguous().to(X.dtype), mode=ctx.mode,
                                           want_ga=need_a, want_gb=need_b)
            ga = ga.to(dtype=ctx.a_meta[0], device=ctx.a_meta[1]) if (need_a and ga is not None) else None
            gb = gb.to(dtype=ctx.b_meta[0], device=ctx.b_meta[1]) if (need_b and gb is not None) else None
            return (gF if need_F else None), ga, gb, None, None

    return TDSolveFn


_TDSolveFn = None


def TDSolveFn():
    global _TDSolveFn
    if _TDSolveFn is None:
        _TDSolveFn = _autograd_fn()
    return _TDSolveFn


def tdsolve(F, a, b, P=None, mode=None):
    """Differentiable solve of the series A(a, b) X = F."""
    return TDSolveFn().apply(F, a, b, P, mode)
