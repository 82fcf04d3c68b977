"""Full-size checks of a factorization on the GPU (torch fp64 arithmetic in
the test harness; no step of the method here).

* ``unpack_L``: the unit lower L from the packed in-place layout (L[i][j+1]
  stored at (i, j) for i >= j+2, column 0 = e_0).
* ``permuted``: P A P^T for the full skew matrix whose strict lower triangle
  is A's, with P from the absolute pivots (transpositions (r, ipiv[r]) in
  order r).
* ``exact_residual``: ||P A P^T - L T L^T||_F / ||A||_F, the postcondition of
  the factorization (Sec. 3.2) with the pivoting of Sec. 3.7, from one dense
  product.
* ``probe_residual``: the same ratio estimated from random probes v:
  sqrt(sum_k ||E v_k||^2 / sum_k ||P A P^T v_k||^2) with E = P A P^T - L T L^T.
  For Gaussian v, E ||M v||^2 = ||M||_F^2 for any M, so numerator and
  denominator estimate ||E||_F^2 and ||A||_F^2 (normalizing by ||v|| instead
  would divide the estimate by sqrt(n)).
"""
from __future__ import annotations

import numpy as np

from tests import checkers as ck


def unpack_L(torch, Af):
    n = Af.shape[0]
    L = torch.roll(torch.tril(Af, -2), shifts=1, dims=1)
    L[:, 0] = 0
    L += torch.eye(n, dtype=torch.float64, device=Af.device)
    return L


def permuted(torch, A0, ipiv_host):
    low = torch.tril(A0, -1)
    Afull = low - low.T
    del low
    q = torch.from_numpy(ck.perm_index(np.asarray(ipiv_host))).to(A0.device)
    PAP = Afull.index_select(0, q).index_select(1, q)
    del Afull
    return PAP


def t_times(torch, t, w):
    """T w for the skew tridiagonal T with T[k+1][k] = t[k], T[k][k+1] = -t[k]
    (w may be a vector or a matrix whose rows are T's index)."""
    out = torch.zeros_like(w)
    if w.dim() == 1:
        out[1:] += t * w[:-1]
        out[:-1] -= t * w[1:]
    else:
        out[1:] += t[:, None] * w[:-1]
        out[:-1] -= t[:, None] * w[1:]
    return out


def exact_residual(torch, PAP, L, t):
    """||PAP - L T L^T||_F / ||PAP||_F with one dense fp64 product."""
    # (L T)[:, j] = t[j] L[:, j+1] - t[j-1] L[:, j-1]
    LT = torch.zeros_like(L)
    LT[:, :-1] += L[:, 1:] * t[None, :]
    LT[:, 1:] -= L[:, :-1] * t[None, :]
    R = torch.matmul(LT, L.T.contiguous())
    del LT
    R -= PAP
    out = (torch.linalg.norm(R) / torch.linalg.norm(PAP)).item()
    del R
    return out


def probe_residual(torch, PAP, L, t, nprobe=8, seed=1):
    g = torch.Generator(device=PAP.device)
    g.manual_seed(seed)
    num = den = 0.0
    worst = 0.0
    for _ in range(nprobe):
        v = torch.randn(PAP.shape[0], dtype=torch.float64, device=PAP.device, generator=g)
        av = PAP @ v
        ev = av - L @ t_times(torch, t, L.T @ v)
        e2 = float(torch.dot(ev, ev).item())
        a2 = float(torch.dot(av, av).item())
        num += e2
        den += a2
        worst = max(worst, (e2 / a2) ** 0.5 if a2 > 0 else 0.0)
    return (num / den) ** 0.5 if den > 0 else 0.0, worst
