"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module only draws random numbers and arranges them into skew-symmetric
matrices; it holds no step of the factorization.  Every generator uses numpy's
PCG64 (``np.random.default_rng(seed)``) so the GPU path and the oracle consume
the very same host buffers.

Recipes (the paper names no test distribution; these stand in for its random
matrices and for the application matrices it motivates in Sec. 1):

* ``skew_normal``: strict lower entries i.i.d. N(0, 1), drawn in column-major
  order of the strict lower triangle; upper = -lower^T; zero diagonal.
* ``skew_graded``: the same entry times 10**U(-6, 6) (normal draws first, then
  the uniform exponents, both in the same column-major order).
* ``skew_odd_blocks``: a symmetric permutation of diag(S1, S2) with odd-order
  skew blocks S1, S2 -- structurally singular, Pf = 0 exactly.
* ``skew_zero_line``: N(0, 1) entries with one zero row and column -- Pf = 0.
* ``batch_sizes``: even n uniform over [lo, hi], a seeded 5% marked singular.
* ``serving_requests``: n log-uniform over [32, 2048] rounded to even, a
  precision tag per request and Poisson arrival times.
"""
from __future__ import annotations

import numpy as np


def _fill_lower(n: int, values: np.ndarray, full: bool) -> np.ndarray:
    A = np.zeros((n, n), dtype=np.float64, order="F")
    off = 0
    for j in range(n - 1):
        cnt = n - j - 1
        A[j + 1:, j] = values[off:off + cnt]
        off += cnt
    if full:
        A = np.asfortranarray(A - A.T)
    return A


def skew_normal(n: int, seed: int, full: bool = True) -> np.ndarray:
    """n x n skew matrix, strict lower entries N(0,1) (Fortran order).

    With ``full=False`` the upper triangle is left zero (the library and the
    oracle read only the strict lower triangle)."""
    rng = np.random.default_rng(seed)
    vals = rng.standard_normal(n * (n - 1) // 2)
    return _fill_lower(n, vals, full)


def skew_graded(n: int, seed: int, full: bool = True, decades: float = 6.0) -> np.ndarray:
    """Entries N(0,1) * 10**U(-decades, decades), independent per entry."""
    rng = np.random.default_rng(seed)
    cnt = n * (n - 1) // 2
    vals = rng.standard_normal(cnt)
    expo = rng.uniform(-decades, decades, cnt)
    vals *= np.power(10.0, expo)
    return _fill_lower(n, vals, full)


def random_permutation(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).permutation(n)


def skew_odd_blocks(n: int, seed: int, full: bool = True) -> np.ndarray:
    """Q diag(S1, S2) Q^T with S1, S2 skew of odd orders n1 + n2 = n (n even).

    Each odd-order skew block is singular, so the matrix is singular and its
    Pfaffian is exactly zero."""
    assert n % 2 == 0 and n >= 2
    rng = np.random.default_rng(seed)
    n1 = 2 * int(rng.integers(0, n // 2)) + 1
    B = np.zeros((n, n), dtype=np.float64)
    for lo, sz in ((0, n1), (n1, n - n1)):
        v = rng.standard_normal((sz, sz))
        B[lo:lo + sz, lo:lo + sz] = np.tril(v, -1) - np.tril(v, -1).T
    q = rng.permutation(n)
    A = B[np.ix_(q, q)]
    if not full:
        A = np.tril(A, -1)
    return np.asfortranarray(A)


def skew_zero_line(n: int, seed: int, full: bool = True) -> np.ndarray:
    """N(0,1) skew matrix with row and column ``z`` set to zero."""
    rng = np.random.default_rng(seed)
    A = _fill_lower(n, rng.standard_normal(n * (n - 1) // 2), True)
    z = int(rng.integers(0, n))
    A[z, :] = 0.0
    A[:, z] = 0.0
    if not full:
        A = np.asfortranarray(np.tril(A, -1))
    return A


def skew_known_factor(n: int, seed: int, lmax: float = 0.9, full: bool = True):
    """A = L0 T0 L0^T with unit lower L0 (first column e_0, entries below
    the diagonal uniform in [-lmax, lmax] / sqrt(n)) and skew tridiagonal T0
    with |t0| uniform in [1, 1.01] and random signs.  Returns (A, L0, t0): a
    matrix whose factors without pivoting are known in advance (with lmax
    above 1/2 partial pivoting would exchange rows, without it the factors
    are L0 and t0)."""
    rng = np.random.default_rng(seed)
    L0 = np.tril(rng.uniform(-lmax, lmax, (n, n)) / np.sqrt(max(n, 1)), -1)
    L0[:, 0] = 0.0
    L0 += np.eye(n)
    t0 = rng.uniform(1.0, 1.01, max(n - 1, 0)) * rng.choice([-1.0, 1.0], max(n - 1, 0))
    T0 = np.diag(t0, -1) - np.diag(t0, 1) if n > 1 else np.zeros((n, n))
    A = L0 @ T0 @ L0.T
    A = np.asfortranarray(A if full else np.tril(A, -1))
    return A, L0, t0


def batch_sizes(count: int, seed: int, lo: int = 16, hi: int = 256,
                singular_fraction: float = 0.05):
    """Even sizes uniform over [lo, hi] and a seeded set of singular members.

    Returns (sizes int array, singular bool array); exactly
    round(count * singular_fraction) members are singular."""
    rng = np.random.default_rng(seed)
    evens = np.arange(lo, hi + 1, 2)
    sizes = rng.choice(evens, size=count)
    nsing = int(round(count * singular_fraction))
    sing = np.zeros(count, dtype=bool)
    sing[rng.choice(count, size=nsing, replace=False)] = True
    return sizes.astype(np.int64), sing


def batch_matrices(sizes, singular, seed: int):
    """One matrix per entry: N(0,1), or (singular) half odd-block / half
    zero-line constructions, alternating by position among the singular."""
    out = []
    k = 0
    for i, (n, s) in enumerate(zip(sizes, singular)):
        sd = seed * 1_000_003 + i
        if s:
            A = skew_odd_blocks(int(n), sd) if k % 2 == 0 else skew_zero_line(int(n), sd)
            k += 1
        else:
            A = skew_normal(int(n), sd)
        out.append(A)
    return out


def serving_requests(count: int, seed: int, rate_per_s: float, lo: int = 32, hi: int = 2048,
                     p_fp32: float = 0.5, p_factor: float = 0.5):
    """Request stream: sizes, precision tags (0 = FP64, 1 = FP32 update),
    arrival times (s) of a Poisson process with the given rate, seeds, and
    kinds (1 = factorization, 0 = Pfaffian only)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(np.log(lo), np.log(hi), count)
    sizes = 2 * np.round(np.exp(u) / 2.0).astype(np.int64)
    sizes = np.clip(sizes, lo, hi)
    prec = (rng.uniform(0.0, 1.0, count) < p_fp32).astype(np.int64)
    gaps = rng.exponential(1.0 / rate_per_s, count)
    arrivals = np.cumsum(gaps)
    seeds = rng.integers(0, 2**31 - 1, count)
    kinds = (rng.uniform(0.0, 1.0, count) < p_factor).astype(np.int64)
    return sizes, prec, arrivals, seeds, kinds
