"""CPU oracle for the pivoted skew-symmetric LTL^T factorization and Pfaffian.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The GPU library never imports,
links or calls anything here, and this module never touches the GPU library.

The factorization's arithmetic lives in ``skltlt_oracle.c`` (plain C, fp64,
full storage); this module compiles it with gcc and marshals numpy arrays
through ctypes.  ``solve`` is the definition of a linear solve written out
with numpy's dense LU (a library primitive as the one step).
Paper: arXiv 2411.09859, Sec. 2.4 (eq. (1), the Parlett-Reid step), Sec. 3.7
(pivoting) and Sec. 1 (the Pfaffian; skew systems as the factorization's use).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "skltlt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

MUTATIONS = {
    "none": 0,
    "drop_second_term": 1,
    "no_pivoting": 2,
    "no_l_row_swap": 3,
    "pf_no_detp": 4,
    "pf_paper_product": 5,
    "l_from_upper": 6,
    "last_index_ties": 7,
    "wrong_l_column": 8,
    "partial_update_sign": 9,
    "partial_unscaled_l": 10,
    "second_largest": 11,
}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-std=c11", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_ltlt.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, dp, dp, ip,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.oracle_ltlt.restype = ctypes.c_int
        lib.oracle_pfaffian.argtypes = [ctypes.c_int, dp, ip, dp, ip, ctypes.c_int]
        lib.oracle_pfaffian.restype = ctypes.c_int
        lib.oracle_ltlt_partial.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, ip,
                                            ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.oracle_ltlt_partial.restype = ctypes.c_int
        lib.oracle_pack.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int]
        lib.oracle_pack.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def ltlt(A: np.ndarray, max_steps: int = -1, nthreads: int = 0, mutation: int | str = 0,
         pivot: bool = True):
    """Factor the skew matrix whose strict lower triangle is ``A`` (n x n).

    Returns a dict with ``X`` (state after the steps; T when complete), ``L``
    (unit lower, first column e_0), ``t`` (n-1 subdiagonal entries of T) and
    ``ipiv`` (absolute, 0-based, ipiv[0] = 0).  The relation P A P^T = L T L^T
    holds with P the product of the transpositions (r, ipiv[r]) applied in
    order r = 1, 2, ... (P(pi) of Sec. 3.7.1 with absolute pivots).  With
    ``pivot=False`` every step pivots on its own subdiagonal entry (P = I),
    the unpivoted algorithm for inputs known to need no pivoting.
    """
    if isinstance(mutation, str):
        mutation = MUTATIONS[mutation]
    A = np.asfortranarray(A, dtype=np.float64)
    n = A.shape[0]
    assert A.shape == (n, n)
    X = np.empty((n, n), dtype=np.float64, order="F")
    L = np.empty((n, n), dtype=np.float64, order="F")
    t = np.zeros(max(n - 1, 1), dtype=np.float64)
    ipiv = np.zeros(max(n, 1), dtype=np.int32)
    rc = _load().oracle_ltlt(n, _dp(A), max(n, 1), _dp(X), _dp(L), _dp(t), _ip(ipiv),
                             int(max_steps), int(bool(pivot)), int(nthreads), int(mutation))
    if rc != 0:
        raise ValueError(f"oracle_ltlt failed with status {rc}")
    return {"X": X, "L": L, "t": t[: max(n - 1, 0)], "ipiv": ipiv[:n]}


def ltlt_partial(A: np.ndarray, max_pairs: int = -1, nthreads: int = 0,
                 mutation: int | str = 0):
    """The Pfaffian-only reduction (one pivot and one rank-2 Schur complement
    per pair of columns) of the skew matrix whose strict lower triangle is
    ``A``.  Returns ``t`` (tau of the even steps, 0 at odd positions) and
    ``ipiv`` (exchanges at the even steps only); :func:`pfaffian` of the two
    gives Pf(A).  ``max_pairs`` >= 0 stops after that many pairs."""
    if isinstance(mutation, str):
        mutation = MUTATIONS[mutation]
    A = np.asfortranarray(A, dtype=np.float64)
    n = A.shape[0]
    assert A.shape == (n, n)
    t = np.zeros(max(n - 1, 1), dtype=np.float64)
    ipiv = np.zeros(max(n, 1), dtype=np.int32)
    rc = _load().oracle_ltlt_partial(n, _dp(A), max(n, 1), _dp(t), _ip(ipiv), int(max_pairs),
                                     int(nthreads), int(mutation))
    if rc != 0:
        raise ValueError(f"oracle_ltlt_partial failed with status {rc}")
    return {"t": t[: max(n - 1, 0)], "ipiv": ipiv[:n]}


def pfaffian(n: int, t: np.ndarray, ipiv: np.ndarray, mutation: int | str = 0):
    """(log|Pf|, sign) from the factors: Pf = det(P) * prod_i (-t[2i])."""
    if isinstance(mutation, str):
        mutation = MUTATIONS[mutation]
    t = np.ascontiguousarray(t, dtype=np.float64)
    if t.size == 0:
        t = np.zeros(1)
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int32)
    if ipiv.size == 0:
        ipiv = np.zeros(1, dtype=np.int32)
    la = np.zeros(1, dtype=np.float64)
    sg = np.zeros(1, dtype=np.int32)
    rc = _load().oracle_pfaffian(int(n), _dp(t), _ip(ipiv), _dp(la), _ip(sg), int(mutation))
    if rc != 0:
        raise ValueError(f"oracle_pfaffian failed with status {rc}")
    return float(la[0]), int(sg[0])


def pack(L: np.ndarray, t: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Return a copy of ``A`` with the factors written in the packed layout."""
    n = L.shape[0]
    out = np.array(A, dtype=np.float64, order="F", copy=True)
    Lf = np.asfortranarray(L, dtype=np.float64)
    tt = np.ascontiguousarray(t, dtype=np.float64)
    if tt.size == 0:
        tt = np.zeros(1)
    rc = _load().oracle_pack(n, _dp(Lf), _dp(tt), _dp(out), max(n, 1))
    if rc != 0:
        raise ValueError("oracle_pack failed")
    return out


def solve(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """X with A X = B for the skew matrix whose strict lower triangle is ``A``:
    the definition written out, a dense LU solve of the full matrix (the use
    of the factorization for skew systems, Sec. 1, is checked against it)."""
    A = np.asarray(A, dtype=np.float64)
    low = np.tril(A, -1)
    return np.linalg.solve(low - low.T, np.asarray(B, dtype=np.float64))
