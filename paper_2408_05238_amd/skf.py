"""Thin Python binding of libskf (ctypes).  Argument marshalling only: every step
of the computation runs in the HIP kernels of ``libskf.so``.

Matrices are PyTorch CUDA tensors in column-major layout: ``A.stride(0) == 1``
and ``A.stride(1) = lda >= n`` (see :func:`colmajor`).  PyTorch supplies device
memory and streams; nothing here computes.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libskf.so")

PREC_F64 = 0
PREC_F32_TRAILING = 1

OK = 0
ENOMEM = -100
EDEVICE = -101
ENOTIMPL = -102
ENONFINITE = -103
EWORK = -104
ETIMEOUT = -105
ESCRATCH = -106
SOLVE_NOALLOC_MAX_N = 4096

# Every symbol declared in include/skf.h (checked by the CPU test suite).
EXPORTS = [
    "skf_version", "skf_last_error", "skf_ltlt_workspace", "skf_ltlt", "skf_pfonly", "skf_logpf_from_factors",
    "skf_logpf_workspace", "skf_logpf", "skf_pfaffian", "skf_skr2k", "skf_skr2k_f32",
    "skf_solve_workspace", "skf_solve", "skf_solve_noalloc", "skf_pf_ratio_workspace", "skf_pf_ratio", "skf_pfonly_c128_workspace",
    "skf_pfonly_c128", "skf_logpf_c128_from_factors", "skf_ltlt_c128_workspace", "skf_ltlt_c128",
    "skf_solve_c128_workspace", "skf_solve_c128", "skf_refine_workspace",
    "skf_solve_refine",
    "skf_batched_workspace", "skf_ltlt_batched", "skf_pfonly_batched", "skf_logpf_batched",
    "skf_solve_batched_workspace", "skf_solve_batched",
    "skf_profile_enable", "skf_profile_read", "skf_tune_set", "skf_tune_get", "skf_tune_clear",
]

_lib = None
_lock = threading.Lock()


class SkfError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = f"{where} failed with status {code}"
        try:
            le = _load().skf_last_error().decode()
            if le:
                msg += f" ({le})"
        except Exception:  # pragma: no cover - message decoration only
            pass
        super().__init__(msg)
        self.code = code


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it first (paper_2408_05238_amd.build.build())")
            lib = ctypes.CDLL(LIB_PATH)
            i64, vp, sz, d = ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_double
            ci = ctypes.c_int
            sig = {
                "skf_version": (ctypes.c_char_p, []),
                "skf_last_error": (ctypes.c_char_p, []),
                "skf_ltlt_workspace": (sz, [i64, ci]),
                "skf_ltlt": (ci, [i64, vp, i64, vp, vp, ci, vp, sz, vp, vp]),
                "skf_pfonly": (ci, [i64, vp, i64, vp, vp, ci, vp, sz, vp, vp]),
                "skf_logpf_from_factors": (ci, [i64, vp, vp, vp, vp, vp]),
                "skf_logpf_workspace": (sz, [i64, ci]),
                "skf_logpf": (ci, [i64, vp, i64, vp, vp, ci, vp, sz, vp, vp]),
                "skf_pfaffian": (ci, [i64, vp, i64, vp, ci, vp, sz, vp, vp]),
                "skf_skr2k": (ci, [i64, i64, d, vp, i64, vp, i64, d, vp, i64, vp]),
                "skf_skr2k_f32": (ci, [i64, i64, d, vp, i64, vp, i64, d, vp, i64, vp]),
                "skf_solve_workspace": (sz, [i64, i64]),
                "skf_solve": (ci, [i64, i64, vp, i64, vp, vp, vp, i64, vp, sz, vp, vp]),
                "skf_solve_noalloc": (ci, [i64, i64, vp, i64, vp, vp, vp, i64, vp, vp]),
                "skf_pfonly_c128_workspace": (sz, [i64]),
                "skf_pfonly_c128": (ci, [i64, vp, i64, vp, vp, vp, sz, vp, vp]),
                "skf_logpf_c128_from_factors": (ci, [i64, vp, vp, vp, vp, vp]),
                "skf_ltlt_c128_workspace": (sz, [i64]),
                "skf_ltlt_c128": (ci, [i64, vp, i64, vp, vp, vp, sz, vp, vp]),
                "skf_solve_c128_workspace": (sz, [i64, i64]),
                "skf_solve_c128": (ci, [i64, i64, vp, i64, vp, vp, vp, i64, vp, sz, vp, vp]),
                "skf_pf_ratio_workspace": (sz, [i64, i64]),
                "skf_pf_ratio": (ci, [i64, i64, vp, i64, vp, vp, vp, i64, vp, i64, vp, vp, vp, sz, vp, vp]),
                "skf_refine_workspace": (sz, [i64, i64]),
                "skf_solve_refine": (ci, [i64, i64, vp, i64, vp, i64, vp, vp, vp, i64, vp, i64, d, ci,
                                          ctypes.POINTER(ci), ctypes.POINTER(d), vp, sz, vp]),
                "skf_batched_workspace": (sz, [i64, vp]),
                "skf_ltlt_batched": (ci, [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]),
                "skf_pfonly_batched": (ci, [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]),
                "skf_logpf_batched": (ci, [i64, vp, vp, vp, vp, vp, vp, vp, sz, vp]),
                "skf_solve_batched_workspace": (sz, [i64, vp, vp]),
                "skf_solve_batched": (ci, [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]),
                "skf_tune_set": (ci, [ci, i64, i64, ci]),
                "skf_tune_get": (ci, [ci, i64]),
                "skf_tune_clear": (ci, []),
                "skf_profile_enable": (ci, [ci]),
                "skf_profile_read": (ci, [vp, vp, vp, ci]),
            }
            for name, (res, args) in sig.items():
                if hasattr(lib, name):
                    f = getattr(lib, name)
                    f.restype = res
                    f.argtypes = args
            load_tuning(lib=lib)
            _lib = lib
    return _lib


# Tuning table persisted by tune.py; SKF_TUNING=<path> selects another file,
# SKF_TUNING=off keeps the built-in rules.
TUNE_PARAMS = {"ltlt_nb": 0, "pfonly_nb": 1, "skr2k_band": 2}
TUNING_PATH = os.path.join(HERE, "tuning", "mi355x.json")


def load_tuning(path: str | None = None, lib=None) -> int:
    """Load a tuning table (JSON, ``{"entries": [{"param", "n_lo", "n_hi", "value"}, ...]}``)
    into the library, replacing what it held; returns the number of entries.
    A missing default file leaves the built-in rules; a malformed one raises."""
    import json
    lib = lib or _load()
    if path is None:
        path = os.environ.get("SKF_TUNING", TUNING_PATH)
    lib.skf_tune_clear()
    if path == "off" or not os.path.exists(path):
        return 0
    with open(path) as f:
        table = json.load(f)
    count = 0
    for e in table.get("entries", []):
        rc = lib.skf_tune_set(TUNE_PARAMS[e["param"]], int(e["n_lo"]), int(e["n_hi"]), int(e["value"]))
        if rc != 0:
            raise ValueError(f"{path}: entry {e} rejected by skf_tune_set (status {rc})")
        count += 1
    return count


def tune_get(param: str, n: int) -> int:
    """The value in effect for order n (table entry, SKF_NB override or built-in rule)."""
    return int(_load().skf_tune_get(TUNE_PARAMS[param], int(n)))


def lib():
    return _load()


def version() -> str:
    return _load().skf_version().decode()


# ----------------------------------------------------------------------------
# torch helpers (memory and streams only)
# ----------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def colmajor(n_rows: int, n_cols: int, device="cuda", dtype=None, ld: int | None = None):
    """Empty column-major tensor (stride(0) == 1, stride(1) == ld)."""
    torch = _torch()
    dtype = dtype or torch.float64
    ld = ld or max(n_rows, 1)
    buf = torch.empty((max(n_cols, 1), ld), device=device, dtype=dtype)
    return buf.t()[:n_rows, :n_cols]


def to_device_colmajor(a, device="cuda"):
    """Copy a numpy array (any order) into a new column-major device tensor."""
    import numpy as np
    torch = _torch()
    a = np.asfortranarray(a)
    t = colmajor(a.shape[0], a.shape[1] if a.ndim > 1 else 1, device=device,
                 dtype=torch.from_numpy(np.zeros(1, a.dtype)).dtype)
    t.copy_(torch.from_numpy(a.reshape(t.shape, order="F")))
    return t


def _ld(A) -> int:
    if A.dim() != 2 or (A.shape[0] > 1 and A.stride(0) != 1):
        raise ValueError("expected a column-major 2-D tensor (stride(0) == 1)")
    return max(A.stride(1), A.shape[0], 1)


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _ptr_array(tensors, dev, stream):
    """Device array of the tensors' data pointers for an asynchronous call.

    The caller must keep the returned tensor alive until the call is enqueued;
    when the call runs on a stream other than the current one the block is also
    recorded on that stream, so the caching allocator cannot hand it out before
    the call's kernels have read it.
    """
    torch = _torch()
    arr = torch.tensor([t.data_ptr() for t in tensors] or [0], dtype=torch.int64, device=dev)
    if stream is not None and stream != torch.cuda.current_stream(dev):
        arr.record_stream(stream)
    return arr


def workspace(nbytes: int, device="cuda"):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# Numerical outcomes a synchronous call returns instead of raising.
NUMERICAL = (ENONFINITE, ETIMEOUT)


def _check(rc: int, where: str):
    if rc < 0 and rc not in NUMERICAL:
        raise SkfError(rc, where)
    return rc


# ----------------------------------------------------------------------------
# Entry points (names follow the C ABI)
# ----------------------------------------------------------------------------

def ltlt_workspace(n: int, prec: int = PREC_F64) -> int:
    return int(_load().skf_ltlt_workspace(n, prec))


def ltlt(A, ipiv=None, T=None, prec: int = PREC_F64, work=None, dinfo=None, stream=None):
    """Factor A (column-major, strict lower triangle read) in place.

    Returns (ipiv, T, info); info is an int when ``dinfo`` is None (the call then
    synchronizes the stream), else the device tensor ``dinfo``.
    """
    torch = _torch()
    n = A.shape[0]
    lda = _ld(A)
    dev = A.device
    if ipiv is None:
        ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    if T is None:
        T = torch.empty(max(n - 1, 1), dtype=torch.float64, device=dev)
    if work is None:
        work = workspace(ltlt_workspace(n, prec), dev)
    rc = _load().skf_ltlt(n, _ptr(A), lda, _ptr(ipiv), _ptr(T), prec, _ptr(work), work.numel(),
                          _ptr(dinfo), _stream(stream))
    _check(rc, "skf_ltlt")
    return ipiv[:n], T[:max(n - 1, 0)], (rc if dinfo is None else dinfo)


def pfonly(A, ipiv=None, T=None, prec: int = PREC_F64, work=None, dinfo=None, stream=None):
    """Pfaffian-only reduction of A (column-major; destroyed).

    Returns (ipiv, T, info) as ``ltlt``: ipiv holds the interchanges of the even
    steps (at odd positions), T the pivots at even positions (odd entries 0).
    """
    torch = _torch()
    n = A.shape[0]
    lda = _ld(A)
    dev = A.device
    if ipiv is None:
        ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    if T is None:
        T = torch.empty(max(n - 1, 1), dtype=torch.float64, device=dev)
    if work is None:
        work = workspace(ltlt_workspace(n, prec), dev)
    rc = _load().skf_pfonly(n, _ptr(A), lda, _ptr(ipiv), _ptr(T), prec, _ptr(work), work.numel(),
                            _ptr(dinfo), _stream(stream))
    _check(rc, "skf_pfonly")
    return ipiv[:n], T[:max(n - 1, 0)], (rc if dinfo is None else dinfo)


def logpf_from_factors(n: int, ipiv, T, stream=None):
    torch = _torch()
    dev = ipiv.device
    la = torch.empty(1, dtype=torch.float64, device=dev)
    sg = torch.empty(1, dtype=torch.int32, device=dev)
    Tp = T if T.numel() > 0 else torch.zeros(1, dtype=torch.float64, device=dev)
    rc = _load().skf_logpf_from_factors(n, _ptr(ipiv), _ptr(Tp), _ptr(la), _ptr(sg), _stream(stream))
    _check(rc, "skf_logpf_from_factors")
    return la, sg


def logpf_workspace(n: int, prec: int = PREC_F64) -> int:
    return int(_load().skf_logpf_workspace(n, prec))


def logpf(A, prec: int = PREC_F64, work=None, dinfo=None, stream=None):
    """(logabs, sign, info) of the Pfaffian; A is destroyed.  logabs/sign are device tensors."""
    torch = _torch()
    n = A.shape[0]
    lda = _ld(A)
    dev = A.device
    la = torch.empty(1, dtype=torch.float64, device=dev)
    sg = torch.empty(1, dtype=torch.int32, device=dev)
    if work is None:
        work = workspace(logpf_workspace(n, prec), dev)
    rc = _load().skf_logpf(n, _ptr(A), lda, _ptr(la), _ptr(sg), prec, _ptr(work), work.numel(),
                           _ptr(dinfo), _stream(stream))
    _check(rc, "skf_logpf")
    return la, sg, (rc if dinfo is None else dinfo)


def pfaffian(A, prec: int = PREC_F64, work=None, dinfo=None, stream=None):
    torch = _torch()
    n = A.shape[0]
    lda = _ld(A)
    pf = torch.empty(1, dtype=torch.float64, device=A.device)
    if work is None:
        work = workspace(logpf_workspace(n, prec), A.device)
    rc = _load().skf_pfaffian(n, _ptr(A), lda, _ptr(pf), prec, _ptr(work), work.numel(), _ptr(dinfo),
                              _stream(stream))
    _check(rc, "skf_pfaffian")
    return pf, (rc if dinfo is None else dinfo)


def skr2k(alpha: float, A, B, beta: float, C, f32: bool = False, stream=None):
    """C := beta C + alpha (A B^T - B A^T) on the strict lower triangle of C (in place)."""
    n, k = A.shape
    fn = _load().skf_skr2k_f32 if f32 else _load().skf_skr2k
    rc = fn(n, k, float(alpha), _ptr(A), _ld(A) if k > 0 else max(n, 1), _ptr(B),
            _ld(B) if k > 0 else max(n, 1), float(beta), _ptr(C), _ld(C), _stream(stream))
    _check(rc, "skf_skr2k")
    return C


def solve_workspace(n: int, nrhs: int) -> int:
    return int(_load().skf_solve_workspace(n, nrhs))


def solve(LT, ipiv, T, B, work=None, dinfo=None, stream=None):
    """X = A^{-1} B with the factors of :func:`ltlt`, in place over B (column-major n x nrhs).

    Returns info (int) when ``dinfo`` is None (synchronous), else ``dinfo``.
    """
    torch = _torch()
    n = LT.shape[0]
    nrhs = B.shape[1] if B.dim() == 2 else 1
    if work is None:
        work = workspace(solve_workspace(n, nrhs), LT.device)
    Tp = T if T.numel() > 0 else torch.zeros(1, dtype=torch.float64, device=LT.device)
    rc = _load().skf_solve(n, nrhs, _ptr(LT), _ld(LT), _ptr(ipiv), _ptr(Tp), _ptr(B), _ld(B), _ptr(work),
                           work.numel(), _ptr(dinfo), _stream(stream))
    _check(rc, "skf_solve")
    return rc if dinfo is None else dinfo


def solve_noalloc(LT, ipiv, T, B, dinfo=None, stream=None):
    """:func:`solve` through ``skf_solve_noalloc`` (no workspace: the library's
    fixed device scratch, n <= SOLVE_NOALLOC_MAX_N)."""
    torch = _torch()
    n = LT.shape[0]
    nrhs = B.shape[1] if B.dim() == 2 else 1
    Tp = T if T.numel() > 0 else torch.zeros(1, dtype=torch.float64, device=LT.device)
    rc = _load().skf_solve_noalloc(n, nrhs, _ptr(LT), _ld(LT), _ptr(ipiv), _ptr(Tp), _ptr(B), _ld(B),
                                   _ptr(dinfo), _stream(stream))
    _check(rc, "skf_solve_noalloc")
    return rc if dinfo is None else dinfo


def pfonly_c128(A, ipiv=None, T=None, work=None, dinfo=None, stream=None):
    """Pfaffian-only reduction of a complex128 skew matrix (column-major device
    tensor, strict lower triangle read, not modified): (ipiv, T, info)."""
    torch = _torch()
    n = A.shape[0]
    lda = _ld(A)
    dev = A.device
    if A.dtype != torch.complex128:
        raise ValueError("expected a complex128 tensor")
    if ipiv is None:
        ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    if T is None:
        T = torch.empty(max(n - 1, 1), dtype=torch.complex128, device=dev)
    if work is None:
        work = workspace(int(_load().skf_pfonly_c128_workspace(n)), dev)
    rc = _load().skf_pfonly_c128(n, _ptr(A), lda, _ptr(ipiv), _ptr(T), _ptr(work), work.numel(), _ptr(dinfo),
                                 _stream(stream))
    _check(rc, "skf_pfonly_c128")
    return ipiv[:n], T[:max(n - 1, 0)], (rc if dinfo is None else dinfo)


def ltlt_c128(A, ipiv=None, T=None, work=None, dinfo=None, stream=None):
    """LTL^T of a complex128 skew matrix (column-major device tensor, strict lower
    triangle read) in place: (ipiv, T, info) as :func:`ltlt`."""
    torch = _torch()
    n = A.shape[0]
    lda = _ld(A)
    dev = A.device
    if A.dtype != torch.complex128:
        raise ValueError("expected a complex128 tensor")
    if ipiv is None:
        ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    if T is None:
        T = torch.empty(max(n - 1, 1), dtype=torch.complex128, device=dev)
    if work is None:
        work = workspace(max(int(_load().skf_ltlt_c128_workspace(n)), 256), dev)
    rc = _load().skf_ltlt_c128(n, _ptr(A), lda, _ptr(ipiv), _ptr(T), _ptr(work), work.numel(), _ptr(dinfo),
                               _stream(stream))
    _check(rc, "skf_ltlt_c128")
    return ipiv[:n], T[:max(n - 1, 0)], (rc if dinfo is None else dinfo)


def solve_c128(LT, ipiv, T, B, work=None, dinfo=None, stream=None):
    """X = A^-1 B in place over B (complex128, column-major) with the factors of
    :func:`ltlt_c128`; returns info (an int when ``dinfo`` is None)."""
    torch = _torch()
    n = LT.shape[0]
    nrhs = B.shape[1] if B.dim() == 2 else 1
    dev = LT.device
    if work is None:
        work = workspace(int(_load().skf_solve_c128_workspace(n, nrhs)), dev)
    Tp = T if T.numel() > 0 else torch.zeros(1, dtype=torch.complex128, device=dev)
    rc = _load().skf_solve_c128(n, nrhs, _ptr(LT), _ld(LT), _ptr(ipiv), _ptr(Tp), _ptr(B),
                                _ld(B) if B.dim() == 2 else max(n, 1), _ptr(work), work.numel(), _ptr(dinfo),
                                _stream(stream))
    _check(rc, "skf_solve_c128")
    return rc if dinfo is None else dinfo


def logpf_c128_from_factors(n: int, ipiv, T, stream=None):
    """(logabs, phase) device tensors: log|Pf| and Pf/|Pf| as complex128."""
    torch = _torch()
    dev = ipiv.device
    la = torch.empty(1, dtype=torch.float64, device=dev)
    ph = torch.empty(1, dtype=torch.complex128, device=dev)
    Tp = T if T.numel() > 0 else torch.zeros(1, dtype=torch.complex128, device=dev)
    rc = _load().skf_logpf_c128_from_factors(n, _ptr(ipiv), _ptr(Tp), _ptr(la), _ptr(ph), _stream(stream))
    _check(rc, "skf_logpf_c128_from_factors")
    return la, ph


def pf_ratio_workspace(n: int, r: int) -> int:
    return int(_load().skf_pf_ratio_workspace(n, r))


def pf_ratio(LT, ipiv, T, U, V, work=None, dinfo=None, stream=None):
    """(log|ratio|, sign, info) of Pf(A + U V^T - V U^T) / Pf(A) from the factors of A.

    U, V: column-major n x r device tensors (r <= 32).  logabs and sign are device
    tensors; info is an int when ``dinfo`` is None (synchronous), else ``dinfo``.
    """
    torch = _torch()
    n = LT.shape[0]
    r = U.shape[1]
    dev = LT.device
    la = torch.empty(1, dtype=torch.float64, device=dev)
    sg = torch.empty(1, dtype=torch.int32, device=dev)
    if work is None:
        work = workspace(pf_ratio_workspace(n, r), dev)
    Tp = T if T.numel() > 0 else torch.zeros(1, dtype=torch.float64, device=dev)
    rc = _load().skf_pf_ratio(n, r, _ptr(LT), _ld(LT), _ptr(ipiv), _ptr(Tp), _ptr(U), _ld(U), _ptr(V), _ld(V),
                              _ptr(la), _ptr(sg), _ptr(work), work.numel(), _ptr(dinfo), _stream(stream))
    _check(rc, "skf_pf_ratio")
    return la, sg, (rc if dinfo is None else dinfo)


def refine_workspace(n: int, nrhs: int) -> int:
    return int(_load().skf_refine_workspace(n, nrhs))


def solve_refine(A0, LT, ipiv, T, B, X=None, tol: float = 1e-13, maxit: int = 10, work=None, stream=None):
    """Iterative refinement; returns (X, status, iters, berr).  A0 is the original matrix."""
    torch = _torch()
    n = LT.shape[0]
    nrhs = B.shape[1]
    if X is None:
        X = colmajor(n, nrhs, device=LT.device)
    if work is None:
        work = workspace(refine_workspace(n, nrhs), LT.device)
    it = ctypes.c_int(0)
    be = ctypes.c_double(0.0)
    Tp = T if T.numel() > 0 else torch.zeros(1, dtype=torch.float64, device=LT.device)
    rc = _load().skf_solve_refine(n, nrhs, _ptr(A0), _ld(A0), _ptr(LT), _ld(LT), _ptr(ipiv), _ptr(Tp), _ptr(B),
                                  _ld(B), _ptr(X), _ld(X), float(tol), int(maxit), ctypes.byref(it),
                                  ctypes.byref(be), _ptr(work), work.numel(), _stream(stream))
    _check(rc, "skf_solve_refine")
    return X, rc, int(it.value), float(be.value)


def batched_workspace(n_list) -> int:
    import numpy as np
    arr = np.ascontiguousarray(np.asarray(n_list, dtype=np.int64))
    return int(_load().skf_batched_workspace(len(arr), arr.ctypes.data_as(ctypes.c_void_p)))


def ltlt_batched(mats, with_factors: bool = True, work=None, stream=None):
    """Factor a list of column-major skew matrices (n <= 512) in one persistent launch
    (L is left in place).

    Returns (logabs, sign, info, ipivs, Ts) as device tensors (ipivs / Ts are
    lists, or None when ``with_factors`` is False: then they are not stored).
    Asynchronous on the stream.  For log|Pf| alone see :func:`logpf_batched`.
    """
    import numpy as np
    torch = _torch()
    dev = mats[0].device if mats else torch.device("cuda")
    B = len(mats)
    n_h = np.array([m.shape[0] for m in mats], dtype=np.int64)
    lda_h = np.array([_ld(m) if m.shape[0] > 0 else 1 for m in mats], dtype=np.int64)
    aptr = _ptr_array(mats, dev, stream)
    logabs = torch.empty(max(B, 1), dtype=torch.float64, device=dev)
    sign = torch.empty(max(B, 1), dtype=torch.int32, device=dev)
    info = torch.empty(max(B, 1), dtype=torch.int32, device=dev)
    if work is None:
        work = workspace(batched_workspace(n_h), dev)
    ipivs = Ts = None
    if with_factors:
        ipivs = [torch.empty(max(int(n), 1), dtype=torch.int32, device=dev) for n in n_h]
        Ts = [torch.empty(max(int(n) - 1, 1), dtype=torch.float64, device=dev) for n in n_h]
        pp = _ptr_array(ipivs, dev, stream)
        tp = _ptr_array(Ts, dev, stream)
        rc = _load().skf_ltlt_batched(B, n_h.ctypes.data_as(ctypes.c_void_p), _ptr(aptr),
                                      lda_h.ctypes.data_as(ctypes.c_void_p), _ptr(pp), _ptr(tp), _ptr(logabs),
                                      _ptr(sign), _ptr(info), _ptr(work), work.numel(), _stream(stream))
        ipivs = [ip[:int(n)] for ip, n in zip(ipivs, n_h)]
        Ts = [t[:max(int(n) - 1, 0)] for t, n in zip(Ts, n_h)]
    else:
        rc = _load().skf_ltlt_batched(B, n_h.ctypes.data_as(ctypes.c_void_p), _ptr(aptr),
                                      lda_h.ctypes.data_as(ctypes.c_void_p), None, None, _ptr(logabs),
                                      _ptr(sign), _ptr(info), _ptr(work), work.numel(), _stream(stream))
    _check(rc, "skf_ltlt_batched")
    return logabs[:B], sign[:B], info[:B], ipivs, Ts


def logpf_batched(mats, work=None, stream=None):
    """log|Pf| and sign of a list of column-major skew matrices (n <= 512) by the
    Pfaffian-only reduction, one persistent launch; the matrices are scratch.
    Returns (logabs, sign, info) as device tensors."""
    import numpy as np
    torch = _torch()
    dev = mats[0].device if mats else torch.device("cuda")
    B = len(mats)
    n_h = np.array([m.shape[0] for m in mats], dtype=np.int64)
    lda_h = np.array([_ld(m) if m.shape[0] > 0 else 1 for m in mats], dtype=np.int64)
    aptr = _ptr_array(mats, dev, stream)
    logabs = torch.empty(max(B, 1), dtype=torch.float64, device=dev)
    sign = torch.empty(max(B, 1), dtype=torch.int32, device=dev)
    info = torch.empty(max(B, 1), dtype=torch.int32, device=dev)
    if work is None:
        work = workspace(batched_workspace(n_h), dev)
    rc = _load().skf_logpf_batched(B, n_h.ctypes.data_as(ctypes.c_void_p), _ptr(aptr),
                                   lda_h.ctypes.data_as(ctypes.c_void_p), _ptr(logabs), _ptr(sign), _ptr(info),
                                   _ptr(work), work.numel(), _stream(stream))
    _check(rc, "skf_logpf_batched")
    return logabs[:B], sign[:B], info[:B]


def pfonly_batched(mats, work=None, stream=None):
    """Pfaffian-only reduction of a list of column-major skew matrices (n <= 512),
    one persistent launch.  Returns (logabs, sign, info, ipivs, Ts) as device
    tensors; the matrices are used as scratch."""
    import numpy as np
    torch = _torch()
    dev = mats[0].device if mats else torch.device("cuda")
    B = len(mats)
    n_h = np.array([m.shape[0] for m in mats], dtype=np.int64)
    lda_h = np.array([_ld(m) if m.shape[0] > 0 else 1 for m in mats], dtype=np.int64)
    aptr = _ptr_array(mats, dev, stream)
    logabs = torch.empty(max(B, 1), dtype=torch.float64, device=dev)
    sign = torch.empty(max(B, 1), dtype=torch.int32, device=dev)
    info = torch.empty(max(B, 1), dtype=torch.int32, device=dev)
    if work is None:
        work = workspace(batched_workspace(n_h), dev)
    ipivs = [torch.empty(max(int(n), 1), dtype=torch.int32, device=dev) for n in n_h]
    Ts = [torch.empty(max(int(n) - 1, 1), dtype=torch.float64, device=dev) for n in n_h]
    pp = _ptr_array(ipivs, dev, stream)
    tp = _ptr_array(Ts, dev, stream)
    rc = _load().skf_pfonly_batched(B, n_h.ctypes.data_as(ctypes.c_void_p), _ptr(aptr),
                                    lda_h.ctypes.data_as(ctypes.c_void_p), _ptr(pp), _ptr(tp), _ptr(logabs),
                                    _ptr(sign), _ptr(info), _ptr(work), work.numel(), _stream(stream))
    _check(rc, "skf_pfonly_batched")
    return (logabs[:B], sign[:B], info[:B], [ip[:int(n)] for ip, n in zip(ipivs, n_h)],
            [t[:max(int(n) - 1, 0)] for t, n in zip(Ts, n_h)])


def logpf_batched_packed(buf, offsets, n_list, work=None, stream=None):
    """log|Pf| of matrices packed in one device buffer (matrix b at element offset
    offsets[b], column-major with lda = n_b).  One persistent launch."""
    import numpy as np
    torch = _torch()
    dev = buf.device
    n_h = np.ascontiguousarray(np.asarray(n_list, dtype=np.int64))
    lda_h = np.maximum(n_h, 1)
    B = len(n_h)
    base = buf.data_ptr()
    aptr = torch.tensor((base + 8 * np.asarray(offsets, dtype=np.int64)).tolist() or [0], dtype=torch.int64,
                        device=dev)
    if stream is not None and stream != torch.cuda.current_stream(dev):
        aptr.record_stream(stream)
    logabs = torch.empty(max(B, 1), dtype=torch.float64, device=dev)
    sign = torch.empty(max(B, 1), dtype=torch.int32, device=dev)
    info = torch.empty(max(B, 1), dtype=torch.int32, device=dev)
    if work is None:
        work = workspace(batched_workspace(n_h), dev)
    rc = _load().skf_logpf_batched(B, n_h.ctypes.data_as(ctypes.c_void_p), _ptr(aptr),
                                   lda_h.ctypes.data_as(ctypes.c_void_p), _ptr(logabs), _ptr(sign), _ptr(info),
                                   _ptr(work), work.numel(), _stream(stream))
    _check(rc, "skf_logpf_batched")
    return logabs[:B], sign[:B], info[:B], aptr


def solve_batched(LTs, ipivs, Ts, Bs, work=None, stream=None):
    """X_b = A_b^{-1} B_b in place over each B_b, with the factors of
    :func:`ltlt_batched` (or :func:`ltlt`).  Returns the device info array."""
    import numpy as np
    torch = _torch()
    nb = len(LTs)
    dev = LTs[0].device if nb else torch.device("cuda")
    n_h = np.array([m.shape[0] for m in LTs], dtype=np.int64)
    lda_h = np.array([_ld(m) if m.shape[0] > 0 else 1 for m in LTs], dtype=np.int64)
    nr_h = np.array([b.shape[1] if b.dim() == 2 else 1 for b in Bs], dtype=np.int64)
    ldb_h = np.array([_ld(b) if b.dim() == 2 and b.shape[0] > 0 else max(int(n), 1) for b, n in zip(Bs, n_h)],
                     dtype=np.int64)
    if work is None:
        need = int(_load().skf_solve_batched_workspace(nb, n_h.ctypes.data_as(ctypes.c_void_p),
                                                        nr_h.ctypes.data_as(ctypes.c_void_p)))
        work = workspace(max(need, 256), dev)
    lt_arr = _ptr_array(LTs, dev, stream)
    ip_arr = _ptr_array(ipivs, dev, stream)
    t_arr = _ptr_array(Ts, dev, stream)
    b_arr = _ptr_array(Bs, dev, stream)
    info = torch.empty(max(nb, 1), dtype=torch.int32, device=dev)
    rc = _load().skf_solve_batched(nb, n_h.ctypes.data_as(ctypes.c_void_p), _ptr(lt_arr),
                                   lda_h.ctypes.data_as(ctypes.c_void_p), _ptr(ip_arr), _ptr(t_arr),
                                   nr_h.ctypes.data_as(ctypes.c_void_p), _ptr(b_arr),
                                   ldb_h.ctypes.data_as(ctypes.c_void_p), _ptr(info), _ptr(work), work.numel(),
                                   _stream(stream))
    _check(rc, "skf_solve_batched")
    return info[:nb]
