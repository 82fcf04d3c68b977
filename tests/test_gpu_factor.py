"""GPU parity of skltlt_factor / skltlt_pfaffian against the CPU oracle.

Bar (FP64): pivots identical to the oracle; ||t - t_oracle|| / ||t_oracle|| and
||L - L_oracle||_F / ||L_oracle||_F <= 1e-12; reconstruction residual
||P A P^T - L T L^T||_F / ||A||_F <= 1e-12; the diagonal and upper triangle of
A (and padding rows when lda > n) bit-for-bit untouched; Pfaffian sign equal
and |log|Pf| - log|Pf|_oracle| <= 1e-12 * max(1, |log|Pf||).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2411_09859_amd import binding, inputs
from tests import checkers as ck
from tests.gpu_util import note, rel, run_factor

pytestmark = pytest.mark.gpu

TOL = 1e-12


def check_against_oracle(A, res, tol=TOL, check_pf=False):
    n = A.shape[0]
    ref = oracle.ltlt(A, nthreads=0)
    assert np.array_equal(res["ipiv"], ref["ipiv"]), "pivot sequence differs from the oracle"
    if n <= 1:
        return ref
    assert rel(res["t"], ref["t"]) <= tol
    L, t = ck.unpack(res["A"], n)
    assert np.array_equal(t, res["t"])  # t moved onto the subdiagonal
    assert rel(L, ref["L"]) <= tol
    assert np.max(np.abs(L)) <= 1.0
    assert ck.residual(A, L, t, res["ipiv"]) <= tol
    # diagonal and upper triangle untouched
    assert np.array_equal(np.triu(res["A"]), np.triu(A))
    if check_pf:
        la, sg = oracle.pfaffian(n, ref["t"], ref["ipiv"])
        assert res["sign"] == sg
        if sg != 0:
            assert abs(res["log_abs_pf"] - la) <= 1e-12 * max(1.0, abs(la))
        else:
            assert res["log_abs_pf"] == -math.inf
    return ref


SMALL = [(2, 0), (3, 0), (4, 1), (5, 2), (16, 0), (17, 4), (33, 8), (64, 0), (65, 16),
         (127, 32), (128, 32), (129, 32), (200, 64), (256, 0), (257, 64), (300, 128),
         (513, 128), (600, 256)]


@pytest.mark.parametrize("n,b", SMALL)
def test_parity_normal(n, b):
    note(f"[parity] n={n} b={b}")
    A = inputs.skew_normal(n, 1000 + n)
    res = run_factor(A, block_size=b, pfaffian=True)
    check_against_oracle(A, res, check_pf=True)


@pytest.mark.parametrize("b", [1, 2, 3, 5, 8, 31, 64])
def test_parity_block_sizes(b):
    n = 150
    note(f"[parity-b] n={n} b={b}")
    A = inputs.skew_normal(n, 77)
    res = run_factor(A, block_size=b, pfaffian=True)
    check_against_oracle(A, res, check_pf=True)


def test_parity_config_n256():
    """The n = 256 single-matrix workload (N(0,1), seed 1)."""
    note("[parity] n=256 config")
    A = inputs.skew_normal(256, 1)
    res = run_factor(A, pfaffian=True)
    check_against_oracle(A, res, check_pf=True)


@pytest.mark.parametrize("n,b", [(1024, 128), (2048, 128), (2048, 64)])
def test_parity_medium(n, b):
    note(f"[parity] n={n} b={b}")
    A = inputs.skew_normal(n, 5 + n)
    res = run_factor(A, block_size=b, pfaffian=True)
    check_against_oracle(A, res, check_pf=True)


def test_parity_graded():
    n = 700
    note(f"[parity] graded n={n}")
    A = inputs.skew_graded(n, 3)
    res = run_factor(A, block_size=64, pfaffian=True)
    check_against_oracle(A, res, check_pf=True)


def test_lda_padding_untouched():
    n, lda = 130, 161
    note("[parity] lda padding")
    A = inputs.skew_normal(n, 9)
    res = run_factor(A, block_size=32, lda=lda)
    check_against_oracle(A, res)
    assert np.all(res["buf"][n:, :] == 7.25)


def test_degenerate_sizes():
    note("[edge] n=0,1,2")
    for n in (0, 1):
        A = np.zeros((n, n))
        res = run_factor(A, pfaffian=(n == 1))
        if n == 1:
            assert res["ipiv"][0] == 0
            assert res["sign"] == 0 and res["log_abs_pf"] == -math.inf
    A = np.array([[0.0, -3.0], [3.0, 0.0]])
    res = run_factor(A, pfaffian=True)
    assert res["t"][0] == 3.0 and res["ipiv"].tolist() == [0, 1]
    # Pf of [[0, a], [-a, 0]] with a = -3
    assert res["sign"] == -1 and abs(res["log_abs_pf"] - math.log(3.0)) < 1e-15


def test_exact_zero_pfaffians_and_zero_matrix():
    note("[edge] singular")
    for n, b in ((64, 16), (250, 32)):
        for A in (inputs.skew_odd_blocks(n, 4), inputs.skew_zero_line(n, 4)):
            res = run_factor(A, block_size=b, pfaffian=True)
            check_against_oracle(A, res, check_pf=True)
            assert res["sign"] == 0
    Z = np.zeros((70, 70))
    res = run_factor(Z, block_size=16, pfaffian=True)
    assert np.array_equal(res["ipiv"], np.arange(70))
    assert np.all(res["t"] == 0) and res["sign"] == 0


def test_permuted_block_diagonal_pfaffian():
    """Closed form Pf(Q diag(J(a_i)) Q^T) = det(Q) prod a_i (pins the sign)."""
    note("[pin] permuted block diagonal")
    for n in (128, 1000):
        rng = np.random.default_rng(n)
        a = rng.uniform(0.5, 2.0, n // 2) * rng.choice([-1.0, 1.0], n // 2)
        B = np.zeros((n, n))
        for i in range(n // 2):
            B[2 * i, 2 * i + 1], B[2 * i + 1, 2 * i] = a[i], -a[i]
        q = rng.permutation(n)
        A = np.asfortranarray(B[np.ix_(q, q)])
        res = run_factor(A, block_size=64, pfaffian=True)
        assert res["sign"] == ck.perm_sign(q) * int(np.prod(np.sign(a)))
        assert abs(res["log_abs_pf"] - np.sum(np.log(np.abs(a)))) < 1e-12 * n


def test_ties_first_index():
    """Column 0 holds several entries of exactly the largest magnitude: the
    first of them is the pivot (iamax reading), as in the oracle."""
    note("[edge] ties")
    n = 40
    A = inputs.skew_normal(n, 31)
    A[:, 0] = 0.0
    A[0, :] = 0.0
    col = np.random.default_rng(2).uniform(-1, 1, n - 1)
    col[[4, 9, 17]] = [5.0, -5.0, 5.0]
    A[1:, 0] = col
    A[0, 1:] = -col
    res = run_factor(A, block_size=8)
    assert res["ipiv"][1] == 5
    check_against_oracle(A, res)


def test_deterministic():
    note("[det] repeat")
    A = inputs.skew_normal(700, 12)
    r1 = run_factor(A, block_size=64)
    r2 = run_factor(A, block_size=64)
    assert np.array_equal(r1["A"], r2["A"]) and np.array_equal(r1["ipiv"], r2["ipiv"])


@pytest.mark.parametrize("precision", [binding.FP64, binding.FP32_UPDATE])
def test_trailing_update_tilings_bit_identical(precision):
    """The 128x128-tile and the 64x64-tile trailing updates sum every element
    in the same K order: forcing either tiling for every update of an
    n = 2600 factorization (ragged against both tile sizes, trailing blocks
    from 2599 down to a few rows) gives the same bytes, and the FP64 result
    matches the oracle."""
    L = binding.lib()
    n = 2600
    A = inputs.skew_normal(n, 77)
    note(f"[tilings] n={n} precision={precision}")
    try:
        assert L.skltlt_tune_skr2k_small_tiles(0) == 0            # 128-tiles only
        r_big = run_factor(A, block_size=128, precision=precision)
        assert L.skltlt_tune_skr2k_small_tiles(1 << 30) == 0      # 64-tiles only
        r_small = run_factor(A, block_size=128, precision=precision)
    finally:
        L.skltlt_tune_skr2k_small_tiles(-1)
    assert np.array_equal(r_big["ipiv"], r_small["ipiv"])
    assert np.array_equal(r_big["t"], r_small["t"])
    assert np.array_equal(r_big["A"], r_small["A"])
    if precision == binding.FP64:
        check_against_oracle(A, r_small)


def test_concurrent_streams_bit_identical():
    """Factorizations and Pfaffian-only runs of several orders whose panels
    take ordinary (not cooperative) launches, issued on four streams at once,
    give the same bytes as the same calls run one at a time; one of them is
    also checked against the oracle."""
    import torch
    sizes = [1100, 1536, 2048, 1800, 1300, 2000, 1024, 1700]
    mats = [inputs.skew_normal(n, 500 + k) for k, n in enumerate(sizes)]
    note(f"[streams] sizes {sizes}")

    def launch(k, stream):
        n = sizes[k]
        A = binding.to_device_colmajor(mats[k])
        t = torch.zeros(n - 1, dtype=torch.float64, device="cuda")
        ip = torch.zeros(n, dtype=torch.int32, device="cuda")
        la = torch.zeros(1, dtype=torch.float64, device="cuda")
        sg = torch.zeros(1, dtype=torch.int32, device="cuda")
        work = binding.alloc_workspace(binding.workspace_size(n, 0, binding.FP64))
        torch.cuda.synchronize()
        if k % 2 == 0:
            binding.pfaffian(A, t, ip, la, sg, 0, binding.FP64, work, stream)
        else:
            binding.pfaffian_partial(A, t, ip, la, sg, 0, binding.FP64, work, stream)
        return (A, t, ip, la, sg, work)

    def host(bufs):
        A, t, ip, la, sg, _ = bufs
        return (A.cpu().numpy(), t.cpu().numpy(), ip.cpu().numpy(), float(la.item()),
                int(sg.item()))

    seq = []
    for k in range(len(sizes)):
        bufs = launch(k, torch.cuda.current_stream())
        torch.cuda.synchronize()
        seq.append(host(bufs))
    streams = [torch.cuda.Stream() for _ in range(4)]
    conc = [launch(k, streams[k % 4]) for k in range(len(sizes))]
    torch.cuda.synchronize()
    for k in range(len(sizes)):
        got = host(conc[k])
        assert got[3] == seq[k][3] and got[4] == seq[k][4], f"Pfaffian differs, n={sizes[k]}"
        assert np.array_equal(got[2], seq[k][2]), f"ipiv differs, n={sizes[k]}"
        assert np.array_equal(got[1], seq[k][1]), f"t differs, n={sizes[k]}"
        if k % 2 == 0:  # full factorization: L as well
            assert np.array_equal(got[0], seq[k][0]), f"L differs, n={sizes[k]}"
    res = {"A": np.asfortranarray(seq[0][0]), "t": seq[0][1], "ipiv": seq[0][2],
           "log_abs_pf": seq[0][3], "sign": seq[0][4]}
    check_against_oracle(mats[0], res, check_pf=True)
