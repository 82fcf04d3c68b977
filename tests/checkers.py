"""Independent checks used by the tests (numpy only; no step of the method).

Each check states a property fixed by the paper or by textbook mathematics:

* ``pf_definition``: the Pfaffian as the signed sum over all permutations of
  Sec. 1 (literal, for order <= 8).
* ``pf_expand``: the row-0 expansion Pf(A) = sum_j (-1)^(j+1) a_0j Pf(A minus
  rows/cols 0, j), itself checked against ``pf_definition`` in the tests.
* ``residual``: ||P A P^T - L T L^T||_F / ||A||_F for the postcondition of
  Sec. 3.2 with the pivoting of Sec. 3.7.
* ``T_from_t``: the skew-symmetric tridiagonal T of Sec. 1 (T[k+1,k] = t[k]).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def full_skew(A: np.ndarray) -> np.ndarray:
    """Full skew matrix from the strict lower triangle of A."""
    lo = np.tril(np.asarray(A, dtype=np.float64), -1)
    return lo - lo.T


def perm_sign(perm) -> int:
    perm = list(perm)
    s = 1
    seen = [False] * len(perm)
    for i in range(len(perm)):
        if seen[i]:
            continue
        j, cyc = i, 0
        while not seen[j]:
            seen[j] = True
            j = perm[j]
            cyc += 1
        if cyc % 2 == 0:
            s = -s
    return s


def pf_definition(X: np.ndarray) -> float:
    """(1 / (2^m m!)) sum_{sigma in S_2m} sgn(sigma) prod_i x[sigma(2i), sigma(2i+1)]."""
    n = X.shape[0]
    if n % 2:
        return 0.0
    m = n // 2
    total = 0.0
    for sigma in itertools.permutations(range(n)):
        prod = 1.0
        for i in range(m):
            prod *= X[sigma[2 * i], sigma[2 * i + 1]]
        total += perm_sign(sigma) * prod
    return total / (2 ** m * math.factorial(m))


def pf_expand(X: np.ndarray) -> float:
    """Recursive expansion along row 0 (exact for the definition)."""
    n = X.shape[0]
    if n == 0:
        return 1.0
    if n % 2:
        return 0.0
    total = 0.0
    for j in range(1, n):
        if X[0, j] == 0.0:
            continue
        keep = [k for k in range(n) if k not in (0, j)]
        sub = X[np.ix_(keep, keep)]
        total += (-1.0) ** (j + 1) * X[0, j] * pf_expand(sub)
    return total


def T_from_t(t: np.ndarray) -> np.ndarray:
    n = len(t) + 1
    T = np.zeros((n, n))
    for k in range(n - 1):
        T[k + 1, k] = t[k]
        T[k, k + 1] = -t[k]
    return T


def perm_index(ipiv) -> np.ndarray:
    """q with (P A P^T)[i, j] = A[q[i], q[j]], transpositions (r, ipiv[r]) in order r."""
    n = len(ipiv)
    q = np.arange(n)
    for r in range(n):
        p = int(ipiv[r])
        if p != r:
            q[r], q[p] = q[p], q[r]
    return q


def residual(A_full: np.ndarray, L: np.ndarray, t: np.ndarray, ipiv) -> float:
    q = perm_index(ipiv)
    PAP = A_full[np.ix_(q, q)]
    R = PAP - L @ T_from_t(t) @ L.T
    den = np.linalg.norm(A_full)
    return float(np.linalg.norm(R) / (den if den > 0 else 1.0))


def unpack(Apacked: np.ndarray, n: int):
    """(L, t) from the packed in-place layout (t on the subdiagonal, L[i][j+1] at (i, j))."""
    L = np.eye(n)
    t = np.zeros(max(n - 1, 0))
    for j in range(n - 1):
        t[j] = Apacked[j + 1, j]
        L[j + 2:, j + 1] = Apacked[j + 2:, j]
    return L, t


def slog_pf_from_det(A_full: np.ndarray):
    """(sign of det, 0.5 * log|det|) from an LU-based determinant (numpy)."""
    s, ld = np.linalg.slogdet(A_full)
    return float(s), 0.5 * float(ld)
