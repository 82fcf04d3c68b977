"""Full-size GPU checks (n = 8192 and 16384, the benchmark's launch shapes).

At these sizes the whole oracle is too slow for a test, so each check uses
what can be computed exactly:
* the first column steps against the oracle run for the same number of
  steps (pivots identical, columns of L and t within 1e-12 relative);
* the backward error ||P A P^T - L T L^T||_F / ||A||_F <= 1e-12, estimated
  from 8 random probes (tests/gpu_full.py), and max |L| <= 1;
* matrices whose factors or Pfaffian are known in closed form (known-factor
  construction, permuted block-diagonal).
The FP32-update variant is held to a bound derived from its arithmetic: the
trailing update is an fp32 product with fp32 accumulation (unit roundoff
u32 = 2^-24), so the backward error is bounded by about n u32 (an inner
product of length at most n, with |L| <= 1 from partial pivoting).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2411_09859_amd import binding, inputs
from tests import checkers as ck
from tests import gpu_full as gf
from tests.gpu_util import note, rel

pytestmark = pytest.mark.gpu


def device_factor(Adev, b=0, prec=binding.FP64):
    import torch
    n = Adev.shape[0]
    t = torch.zeros(n - 1, dtype=torch.float64, device="cuda")
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    la = torch.zeros(1, dtype=torch.float64, device="cuda")
    sg = torch.zeros(1, dtype=torch.int32, device="cuda")
    binding.pfaffian(Adev, t, ipiv, la, sg, b, prec)
    torch.cuda.synchronize()
    return t, ipiv, float(la.item()), int(sg.item())


def probe_residual(torch, A0dev, Af, t, ipiv, nprobe=8):
    """Estimate of ||P A P^T - L T L^T||_F / ||A||_F from random probes
    (tests/gpu_full.py); also checks max |L| <= 1 (partial pivoting)."""
    PAP = gf.permuted(torch, A0dev, ipiv.cpu().numpy())
    L = gf.unpack_L(torch, Af)
    assert torch.max(torch.abs(L)).item() <= 1.0
    est, _ = gf.probe_residual(torch, PAP, L, t, nprobe)
    del PAP, L
    return est


@pytest.mark.parametrize("b", [0, 128])
def test_n16384_graded_prefix_parity_and_residual(b):
    import torch
    n, steps = 16384, 48
    note(f"[large] n={n} b={b} graded: factor + oracle prefix of {steps} steps")
    A = inputs.skew_graded(n, 3, full=False)
    A0 = binding.to_device_colmajor(A)
    Af = A0.clone()
    t, ipiv, la, sg = device_factor(Af, b=b)
    ref = oracle.ltlt(A, max_steps=steps)
    gp = ipiv.cpu().numpy()
    assert gp[0] == 0 and np.array_equal(gp[: steps + 1], ref["ipiv"][: steps + 1])
    tg = t.cpu().numpy()
    assert rel(tg[:steps], ref["t"][:steps]) <= 1e-12
    # The stored columns of L carry the row exchanges of all later steps;
    # apply the same exchanges (from the GPU pivots) to the oracle's prefix
    # columns: row i of the result is row G[i] of the prefix.
    G = np.arange(n)
    pos = np.arange(n)
    for c in range(n - 2, steps - 1, -1):
        a, b = c + 1, int(gp[c + 1])
        if a != b:
            ia, ib = pos[a], pos[b]
            G[ia], G[ib] = b, a
            pos[a], pos[b] = ib, ia
    Ah = Af[:, : steps].cpu().numpy()
    for j in range(1, steps):  # L column j is stored in A column j-1 (rows >= j+1)
        got = Ah[j + 1:, j - 1]
        want = ref["L"][G[j + 1:], j]
        assert rel(got, want) <= 1e-12, j
    assert np.all(np.isfinite(tg)) and np.all(gp >= np.arange(n))
    res = probe_residual(torch, A0, Af, t, ipiv)
    note(f"[large] residual probe {res:.3e}, log|Pf| {la:.6f} sign {sg}")
    assert res <= 1e-12
    assert sg in (-1, 1)


def test_n8192_known_factors():
    import torch
    n = 8192
    note(f"[large] n={n} known factors")
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    scale = 0.5 * 4.0 / math.sqrt(n)
    L0 = torch.tril((torch.rand((n, n), generator=g, dtype=torch.float64, device="cuda") * 2 - 1) * scale, -1)
    L0[:, 0] = 0
    L0 += torch.eye(n, dtype=torch.float64, device="cuda")
    # |t| nearly constant: the step for column c pivots on row c+1, so the
    # sensitivity of the factors runs through products of the ratios
    # |t[a+1] / t[a]| along two interleaved chains; magnitudes drawn from
    # [1, 2] make the log of those products a random walk and the forward
    # error grows faster than any power of n (the backward error stays at
    # rounding level, but t is no longer recovered to 1e-12 at this order).
    t0 = (1.0 + 0.01 * torch.rand(n - 1, generator=g, dtype=torch.float64, device="cuda")) * \
        torch.where(torch.rand(n - 1, generator=g, device="cuda") < 0.5, -1.0, 1.0).double()
    T0 = torch.diag(t0, -1) - torch.diag(t0, 1)
    A = (L0 @ T0) @ L0.T.contiguous()
    Adev = A.T.contiguous().T  # column-major view of the same values
    Af = Adev.clone(memory_format=torch.preserve_format)
    t, ipiv, la, sg = device_factor(Af)
    assert torch.equal(ipiv.cpu(), torch.arange(n, dtype=torch.int32))
    assert (torch.linalg.norm(t - t0) / torch.linalg.norm(t0)).item() <= 1e-12
    # L column j is stored in A column j-1 below the subdiagonal
    L = torch.roll(torch.tril(Af, -2), shifts=1, dims=1)
    L[:, 0] = 0
    L += torch.eye(n, dtype=torch.float64, device="cuda")
    assert (torch.linalg.norm(L - L0) / torch.linalg.norm(L0)).item() <= 1e-12
    del L
    want_la = torch.sum(torch.log(torch.abs(t0[0::2]))).item()
    want_sg = int(torch.prod(torch.sign(-t0[0::2])).item())
    assert sg == want_sg and abs(la - want_la) <= 1e-12 * max(1.0, abs(want_la))
    assert probe_residual(torch, Adev, Af, t, ipiv) <= 1e-12


def test_n16384_permuted_block_diagonal_pfaffian():
    import torch
    n = 16384
    note(f"[large] n={n} permuted block diagonal")
    rng = np.random.default_rng(n)
    a = rng.uniform(0.5, 2.0, n // 2) * rng.choice([-1.0, 1.0], n // 2)
    q = rng.permutation(n)
    qi = np.empty(n, dtype=np.int64)
    qi[q] = np.arange(n)
    # A[i, j] = B[q[i], q[j]] with B = diag([[0, a_k], [-a_k, 0]])
    Adev = torch.zeros((n, n), dtype=torch.float64, device="cuda").t()
    rows = torch.from_numpy(qi[np.arange(0, n, 2)]).to("cuda")
    cols = torch.from_numpy(qi[np.arange(1, n, 2)]).to("cuda")
    av = torch.from_numpy(a).to("cuda")
    Adev[rows, cols] = av
    Adev[cols, rows] = -av
    t, ipiv, la, sg = device_factor(Adev)
    want_sg = ck.perm_sign(q) * int(np.prod(np.sign(a)))
    assert sg == want_sg
    assert abs(la - float(np.sum(np.log(np.abs(a))))) <= 1e-10 * n


@pytest.mark.parametrize("n", [1024, 2048])
def test_fp32_update_backward_error_vs_oracle(n):
    import torch
    note(f"[fp32] n={n}")
    A = inputs.skew_normal(n, 21)
    A0 = binding.to_device_colmajor(A)
    Af = A0.clone()
    t, ipiv, la, sg = device_factor(Af, prec=binding.FP32_UPDATE)
    res = probe_residual(torch, A0, Af, t, ipiv)
    ref = oracle.ltlt(A)
    rla, rsg = oracle.pfaffian(n, ref["t"], ref["ipiv"])
    note(f"[fp32] n={n} residual {res:.3e}, |dlog|Pf|| {abs(la - rla):.3e}")
    assert res <= n * 2.0 ** -24
    assert sg == rsg
    assert abs(la - rla) <= 1e-4 * abs(rla)


def test_b256_shape_parity():
    note("[large] b=256 panel shape")
    n = 1500
    A = inputs.skew_normal(n, 31)
    from tests.gpu_util import run_factor
    from tests.test_gpu_factor import check_against_oracle
    res = run_factor(A, block_size=256, pfaffian=True)
    check_against_oracle(A, res, check_pf=True)
