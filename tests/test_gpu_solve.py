"""Solving A X = B with the factors (skltlt_solve) against the oracle's dense
solve, on the same seeded inputs.

X = P^T L^{-T} T^{-1} L^{-1} P B with P A P^T = L T L^T (the factorization's
use for skew systems, paper Sec. 1).  Criteria: the backward error
||A X - B||_F / (||A||_F ||X||_F) <= 1e-13 (conditioning-free), and the
forward difference to the oracle ||X - X_o|| / ||X_o|| <= 1e-13 * cond-proxy,
with cond-proxy = ||A||_F ||A^{-1}||_F from the oracle (the solve is backward
stable, so its forward error is bounded by the condition number times the
backward error).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2411_09859_amd import binding, inputs
from tests.gpu_util import note

pytestmark = pytest.mark.gpu


def factor_and_solve(A_np, B_np, block_size=0):
    import torch
    n = A_np.shape[0]
    Ad = binding.to_device_colmajor(A_np)
    t = torch.zeros(max(n - 1, 1), dtype=torch.float64, device="cuda")
    ipiv = torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")
    binding.factor(Ad, t, ipiv, block_size)
    B2 = np.atleast_2d(B_np.T).T if B_np.ndim == 1 else B_np
    Bd = torch.empty_strided(B2.shape, (1, max(n, 1)), dtype=torch.float64, device="cuda")
    Bd.copy_(torch.from_numpy(np.ascontiguousarray(B2)))
    binding.solve(Ad, t, ipiv, Bd)
    torch.cuda.synchronize()
    return Bd.cpu().numpy()


def check(A_np, B_np, X):
    low = np.tril(A_np, -1)
    Af = low - low.T
    Xo = oracle.solve(A_np, B_np)
    X = X.reshape(Xo.shape)
    nA = np.linalg.norm(Af)
    back = np.linalg.norm(Af @ X - B_np) / (nA * np.linalg.norm(X))
    cond = nA * np.linalg.norm(np.linalg.inv(Af))
    fwd = np.linalg.norm(X - Xo) / np.linalg.norm(Xo)
    assert back <= 1e-13, back
    assert fwd <= 1e-13 * cond, (fwd, cond)
    return back, fwd, cond


# up to four right-hand sides take the single-launch triangular solves, more
# the block-sequential ones; n = 130 and 200 end in a ragged block
CASES = [(2, 1, 0), (4, 1, 0), (10, 3, 0), (64, 1, 16), (128, 2, 32), (130, 2, 0), (130, 9, 32),
         (200, 4, 32), (300, 17, 64), (514, 1, 128), (1000, 5, 256)]


@pytest.mark.parametrize("n,nrhs,b", CASES)
def test_solve_matches_oracle(n, nrhs, b):
    note(f"[solve] n={n} nrhs={nrhs} b={b}")
    A = inputs.skew_normal(n, 600 + n)
    B = np.random.default_rng(n).standard_normal((n, nrhs))
    X = factor_and_solve(A, B, b)
    back, fwd, cond = check(A, B, X)
    note(f"[solve] n={n}: backward {back:.2e} forward {fwd:.2e} cond {cond:.1e}")


def test_solve_vector_rhs_graded():
    n = 400
    note(f"[solve] graded n={n}, 1-D right-hand side")
    A = inputs.skew_graded(n, 8, decades=2.0)
    B = np.random.default_rng(1).standard_normal(n)
    X = factor_and_solve(A, B, 64)
    check(A, B, X)


def test_solve_closed_form_block_diagonal():
    from tests.test_oracle_pins import _block_diag_system
    n = 512
    note(f"[solve] permuted block diagonal n={n}")
    A, w, v = _block_diag_system(n, 7)
    X = factor_and_solve(A, w, 128)
    assert np.allclose(X, v, rtol=1e-12, atol=1e-12)


def test_solve_argument_errors():
    import torch
    note("[solve] argument errors")
    n = 8
    Ad = torch.zeros((n, n), dtype=torch.float64, device="cuda").t()
    t = torch.zeros(n - 1, dtype=torch.float64, device="cuda")
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    B = torch.zeros(n, dtype=torch.float64, device="cuda")
    Ao = torch.zeros((7, 7), dtype=torch.float64, device="cuda").t()
    with pytest.raises(binding.SkltltError) as e:
        binding.solve(Ao, t[:6], ipiv[:7], B[:7])  # odd order
    assert e.value.status == binding.SKLTLT_EINVAL
    work = binding.alloc_workspace(16)
    with pytest.raises(binding.SkltltError) as e:
        binding.solve(Ad, t, ipiv, B, work=work)  # short workspace
    assert e.value.status == binding.SKLTLT_EINVAL


def test_solve_n8192_residual():
    import torch
    n = 8192
    note(f"[solve] n={n} residual on the GPU")
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    low = torch.tril(torch.randn((n, n), generator=g, dtype=torch.float64, device="cuda"), -1)
    Af = low - low.T
    Ad = low.T.contiguous().T.clone(memory_format=torch.preserve_format)  # column-major lower
    t = torch.zeros(n - 1, dtype=torch.float64, device="cuda")
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    binding.factor(Ad, t, ipiv)
    B = torch.randn((n, 2), generator=g, dtype=torch.float64, device="cuda")
    X = B.T.contiguous().T.clone(memory_format=torch.preserve_format)
    binding.solve(Ad, t, ipiv, X)
    torch.cuda.synchronize()
    back = (torch.linalg.norm(Af @ X - B) / (torch.linalg.norm(Af) * torch.linalg.norm(X))).item()
    note(f"[solve] n={n} backward error {back:.2e}")
    assert back <= 1e-13
