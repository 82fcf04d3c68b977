"""Thin ctypes binding of libskltlt.so (C ABI in include/skltlt.h).

Argument marshalling only: every step of the factorization runs in the HIP
kernels of the library.  PyTorch supplies device memory and the stream.  If the
library is missing this module raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libskltlt.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "skltlt.h")

SKLTLT_OK = 0
SKLTLT_EINVAL = -1
SKLTLT_ENOMEM = -2
SKLTLT_EDEVICE = -3
SKLTLT_ENOTSUP = -4
FP64 = 0
FP32_UPDATE = 1

_lib = None


class SkltltError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = lib().skltlt_status_string(status).decode()
        if status == SKLTLT_EDEVICE:
            msg += " [" + lib().skltlt_last_device_error().decode() + "]"
        super().__init__(f"{what}: {msg} ({status})")


def lib():
    """Load libskltlt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        # torch bundles its own HIP runtime with the same SONAME as ROCm's;
        # loading torch first makes the library bind to that one runtime
        # instead of pulling a second HIP/HSA runtime into the process.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
        L.skltlt_status_string.argtypes = [i]
        L.skltlt_status_string.restype = ctypes.c_char_p
        L.skltlt_last_device_error.argtypes = []
        L.skltlt_last_device_error.restype = ctypes.c_char_p
        L.skltlt_default_block_size.argtypes = [i]
        L.skltlt_default_block_size.restype = i
        L.skltlt_workspace_size.argtypes = [i, i, i, ctypes.POINTER(sz)]
        L.skltlt_workspace_size.restype = i
        L.skltlt_factor.argtypes = [i, vp, i, vp, vp, i, i, vp, sz, vp]
        L.skltlt_factor.restype = i
        L.skltlt_pfaffian.argtypes = [i, vp, i, vp, vp, vp, vp, i, i, vp, sz, vp]
        L.skltlt_pfaffian.restype = i
        L.skltlt_left_workspace_size.argtypes = [i, i, ctypes.POINTER(sz)]
        L.skltlt_left_workspace_size.restype = i
        L.skltlt_factor_left.argtypes = [i, vp, i, vp, vp, i, i, vp, sz, vp]
        L.skltlt_factor_left.restype = i
        L.skltlt_pfaffian_left.argtypes = [i, vp, i, vp, vp, vp, vp, i, i, vp, sz, vp]
        L.skltlt_pfaffian_left.restype = i
        L.skltlt_factor_nopiv.argtypes = [i, vp, i, vp, vp, i, i, vp, sz, vp]
        L.skltlt_factor_nopiv.restype = i
        L.skltlt_pfaffian_nopiv.argtypes = [i, vp, i, vp, vp, vp, vp, i, i, vp, sz, vp]
        L.skltlt_pfaffian_nopiv.restype = i
        L.skltlt_pfaffian_partial.argtypes = [i, vp, i, vp, vp, vp, vp, i, i, vp, sz, vp]
        L.skltlt_pfaffian_partial.restype = i
        L.skltlt_batched_max_n.argtypes = []
        L.skltlt_batched_max_n.restype = i
        L.skltlt_tune_batched_wgpc.argtypes = [i]
        L.skltlt_tune_batched_wgpc.restype = i
        L.skltlt_tune_skr2k_small_tiles.argtypes = [i]
        L.skltlt_tune_skr2k_small_tiles.restype = i
        L.skltlt_batched_workspace_size.argtypes = [i, ctypes.POINTER(sz)]
        L.skltlt_batched_workspace_size.restype = i
        L.skltlt_batched.argtypes = [i, vp, vp, vp, vp, vp, vp, vp, vp, i, i, i, vp, sz, vp]
        L.skltlt_batched.restype = i
        L.skltlt_batched_noalloc_max_batch.argtypes = []
        L.skltlt_batched_noalloc_max_batch.restype = i
        L.skltlt_batched_noalloc.argtypes = [i, vp, vp, vp, vp, vp, vp, vp, vp, i, i, i, vp]
        L.skltlt_batched_noalloc.restype = i
        L.skltlt_solve_workspace_size.argtypes = [i, i, ctypes.POINTER(sz)]
        L.skltlt_solve_workspace_size.restype = i
        L.skltlt_solve.argtypes = [i, i, vp, i, vp, vp, vp, i, vp, sz, vp]
        L.skltlt_solve.restype = i
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared in include/skltlt.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(skltlt_[a-z0-9_]+)\s*\(", txt)))


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def default_block_size(n: int) -> int:
    return lib().skltlt_default_block_size(int(n))


def workspace_size(n: int, block_size: int = 0, precision: int = FP64) -> int:
    out = ctypes.c_size_t(0)
    st = lib().skltlt_workspace_size(int(n), int(block_size), int(precision), ctypes.byref(out))
    if st != SKLTLT_OK:
        raise SkltltError(st, "skltlt_workspace_size")
    return int(out.value)


def alloc_workspace(nbytes: int, device="cuda"):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _lda_of(A):
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be a square 2-D tensor")
    n = A.shape[0]
    if n > 1 and A.stride(0) != 1:
        raise ValueError("A must be column-major (stride(0) == 1)")
    return max(A.stride(1), 1) if n > 1 else 1


def factor(A, t, ipiv, block_size: int = 0, precision: int = FP64, work=None, stream=None):
    """skltlt_factor on device tensors: A (n x n fp64, column-major view),
    t (n-1 fp64), ipiv (n int32).  Returns the status (raises on error)."""
    n = A.shape[0]
    lda = _lda_of(A)
    if work is None:
        work = alloc_workspace(workspace_size(n, block_size, precision), A.device)
    st = lib().skltlt_factor(n, _ptr(A), lda, _ptr(t), _ptr(ipiv), int(block_size),
                             int(precision), _ptr(work), work.numel(), _stream(stream))
    if st != SKLTLT_OK:
        raise SkltltError(st, "skltlt_factor")
    return st


def pfaffian(A, t, ipiv, log_abs_pf, sign, block_size: int = 0, precision: int = FP64,
             work=None, stream=None):
    """skltlt_pfaffian on device tensors (log_abs_pf: 1 fp64, sign: 1 int32)."""
    n = A.shape[0]
    lda = _lda_of(A)
    if work is None:
        work = alloc_workspace(workspace_size(n, block_size, precision), A.device)
    st = lib().skltlt_pfaffian(n, _ptr(A), lda, _ptr(t), _ptr(ipiv), _ptr(log_abs_pf),
                               _ptr(sign), int(block_size), int(precision), _ptr(work),
                               work.numel(), _stream(stream))
    if st != SKLTLT_OK:
        raise SkltltError(st, "skltlt_pfaffian")
    return st


def factor_nopiv(A, t, ipiv, block_size: int = 0, precision: int = FP64, work=None,
                 stream=None):
    """skltlt_factor_nopiv (no pivoting) on device tensors; ipiv receives the
    identity."""
    n = A.shape[0]
    lda = _lda_of(A)
    if work is None:
        work = alloc_workspace(workspace_size(n, block_size, precision), A.device)
    st = lib().skltlt_factor_nopiv(n, _ptr(A), lda, _ptr(t), _ptr(ipiv), int(block_size),
                                   int(precision), _ptr(work), work.numel(), _stream(stream))
    if st != SKLTLT_OK:
        raise SkltltError(st, "skltlt_factor_nopiv")
    return st


def pfaffian_nopiv(A, t, ipiv, log_abs_pf, sign, block_size: int = 0, precision: int = FP64,
                   work=None, stream=None):
    """skltlt_pfaffian_nopiv on device tensors."""
    n = A.shape[0]
    lda = _lda_of(A)
    if work is None:
        work = alloc_workspace(workspace_size(n, block_size, precision), A.device)
    st = lib().skltlt_pfaffian_nopiv(n, _ptr(A), lda, _ptr(t), _ptr(ipiv), _ptr(log_abs_pf),
                                     _ptr(sign), int(block_size), int(precision), _ptr(work),
                                     work.numel(), _stream(stream))
    if st != SKLTLT_OK:
        raise SkltltError(st, "skltlt_pfaffian_nopiv")
    return st


def left_workspace_size(n: int, block_size: int = 0) -> int:
    out = ctypes.c_size_t(0)
    st = lib().skltlt_left_workspace_size(int(n), int(block_size), ctypes.byref(out))
    if st != SKLTLT_OK:
        raise SkltltError(st, "skltlt_left_workspace_size")
    return int(out.value)


def factor_left(A, t, ipiv, block_size: int = 0, work=None, stream=None):
    """skltlt_factor_left (left-looking, no pivoting) on device tensors."""
    n = A.shape[0]
    lda = _lda_of(A)
    if work is None:
        work = alloc_workspace(left_workspace_size(n, block_size), A.device)
    st = lib().skltlt_factor_left(n, _ptr(A), lda, _ptr(t), _ptr(ipiv), int(block_size), FP64,
                                  _ptr(work), work.numel(), _stream(stream))
    if st != SKLTLT_OK:
        raise SkltltError(st, "skltlt_factor_left")
    return st


def pfaffian_left(A, t, ipiv, log_abs_pf, sign, block_size: int = 0, work=None, stream=None):
    """skltlt_pfaffian_left on device tensors."""
    n = A.shape[0]
    lda = _lda_of(A)
    if work is None:
        work = alloc_workspace(left_workspace_size(n, block_size), A.device)
    st = lib().skltlt_pfaffian_left(n, _ptr(A), lda, _ptr(t), _ptr(ipiv), _ptr(log_abs_pf),
                                    _ptr(sign), int(block_size), FP64, _ptr(work), work.numel(),
                                    _stream(stream))
    if st != SKLTLT_OK:
        raise SkltltError(st, "skltlt_pfaffian_left")
    return st


def pfaffian_partial(A, t, ipiv, log_abs_pf, sign, block_size: int = 0, precision: int = FP64,
                     work=None, stream=None):
    """skltlt_pfaffian_partial on device tensors: the Pfaffian by the
    pairwise reduction; A is only read, t and ipiv receive the pairs' tau
    and pivots."""
    n = A.shape[0]
    lda = _lda_of(A)
    if work is None:
        work = alloc_workspace(workspace_size(n, block_size, precision), A.device)
    st = lib().skltlt_pfaffian_partial(n, _ptr(A), lda, _ptr(t), _ptr(ipiv), _ptr(log_abs_pf),
                                       _ptr(sign), int(block_size), int(precision), _ptr(work),
                                       work.numel(), _stream(stream))
    if st != SKLTLT_OK:
        raise SkltltError(st, "skltlt_pfaffian_partial")
    return st


def batched_max_n() -> int:
    return lib().skltlt_batched_max_n()


def batched_workspace_size(batch: int) -> int:
    out = ctypes.c_size_t(0)
    st = lib().skltlt_batched_workspace_size(int(batch), ctypes.byref(out))
    if st != SKLTLT_OK:
        raise SkltltError(st, "skltlt_batched_workspace_size")
    return int(out.value)


def batched(n_dev, A_ptrs, lda_dev, t_ptrs, ipiv_ptrs, log_abs_pf, sign, info, max_n: int,
            block_size: int = 0, precision: int = FP64, work=None, stream=None):
    """skltlt_batched with device descriptor arrays (int32 n/lda, int64 pointer arrays)."""
    batch = n_dev.numel()
    if work is None:
        work = alloc_workspace(batched_workspace_size(batch), n_dev.device)
    st = lib().skltlt_batched(batch, _ptr(n_dev), _ptr(A_ptrs), _ptr(lda_dev), _ptr(t_ptrs),
                              _ptr(ipiv_ptrs), _ptr(log_abs_pf), _ptr(sign), _ptr(info),
                              int(max_n), int(block_size), int(precision), _ptr(work),
                              work.numel(), _stream(stream))
    if st != SKLTLT_OK:
        raise SkltltError(st, "skltlt_batched")
    return st


def batched_noalloc_max_batch() -> int:
    return lib().skltlt_batched_noalloc_max_batch()


def batched_noalloc(n_dev, A_ptrs, lda_dev, t_ptrs, ipiv_ptrs, log_abs_pf, sign, info,
                    max_n: int, block_size: int = 0, precision: int = FP64, stream=None):
    """skltlt_batched_noalloc: as batched() with no workspace (the library's
    per-device static scratch array)."""
    batch = n_dev.numel()
    st = lib().skltlt_batched_noalloc(batch, _ptr(n_dev), _ptr(A_ptrs), _ptr(lda_dev),
                                      _ptr(t_ptrs), _ptr(ipiv_ptrs), _ptr(log_abs_pf),
                                      _ptr(sign), _ptr(info), int(max_n), int(block_size),
                                      int(precision), _stream(stream))
    if st != SKLTLT_OK:
        raise SkltltError(st, "skltlt_batched_noalloc")
    return st


def solve_workspace_size(n: int, nrhs: int = 1) -> int:
    out = ctypes.c_size_t(0)
    st = lib().skltlt_solve_workspace_size(int(n), int(nrhs), ctypes.byref(out))
    if st != SKLTLT_OK:
        raise SkltltError(st, "skltlt_solve_workspace_size")
    return int(out.value)


def solve(LT, t, ipiv, B, work=None, stream=None):
    """skltlt_solve on device tensors: LT the factored matrix (column-major
    view), t (n-1), ipiv (n), B overwritten by X: a 1-D tensor of length n or
    an n x nrhs column-major view."""
    n = LT.shape[0]
    lda = _lda_of(LT)
    if B.dim() == 1:
        nrhs, ldb = 1, max(n, 1)
        if B.shape[0] != n:
            raise ValueError("B must have n entries")
    else:
        if B.shape[0] != n or (n > 1 and B.stride(0) != 1):
            raise ValueError("B must be an n x nrhs column-major view")
        nrhs, ldb = B.shape[1], max(B.stride(1), n, 1)
    if work is None:
        work = alloc_workspace(solve_workspace_size(n, max(nrhs, 1)), LT.device)
    st = lib().skltlt_solve(n, int(nrhs), _ptr(LT), lda, _ptr(t), _ptr(ipiv), _ptr(B), ldb,
                            _ptr(work), work.numel(), _stream(stream))
    if st != SKLTLT_OK:
        raise SkltltError(st, "skltlt_solve")
    return st


# ---------------------------------------------------------------- helpers
def to_device_colmajor(A_np, device="cuda"):
    """Copy a host numpy matrix into a column-major device tensor (lda = n)."""
    import numpy as np
    import torch
    A_np = np.asfortranarray(A_np, dtype=np.float64)
    n = A_np.shape[0]
    host = torch.from_numpy(A_np)  # strides (1, n)
    dev = torch.empty_strided((n, n), (1, max(n, 1)), dtype=torch.float64, device=device)
    dev.copy_(host)
    return dev


def from_device_colmajor(A_dev):
    import numpy as np
    host = A_dev.cpu()
    return np.asfortranarray(host.numpy())
