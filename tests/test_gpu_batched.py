"""GPU tests of skltlt_batched (one persistent launch for many small matrices).

Bar: every member matches the CPU oracle as skltlt_factor does (pivots
identical, factors and residual within 1e-12, Pfaffian sign equal); a member's
result is bitwise the same alone and in any mix or order; invalid members are
rejected without touching their buffers; a captured hipGraph replays the
eager result on every replay.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2411_09859_amd import binding, inputs
from tests.gpu_util import DeviceBatch, note
from tests.test_gpu_factor import check_against_oracle

pytestmark = pytest.mark.gpu


def mixed_batch(count, seed):
    sizes, sing = inputs.batch_sizes(count, seed)
    mats = inputs.batch_matrices(sizes, sing, seed)
    return mats


def test_batched_parity_mixed():
    note("[batched] mixed parity")
    mats = mixed_batch(48, 11)
    mats += [np.zeros((0, 0)), np.zeros((1, 1)), inputs.skew_normal(2, 1), inputs.skew_normal(3, 2),
             inputs.skew_normal(255, 3), inputs.skew_normal(256, 4), np.zeros((40, 40))]
    db = DeviceBatch(mats)
    db.run()
    res = db.results()
    for M, r in zip(mats, res):
        assert r["info"] == 0
        check_against_oracle(M, r, check_pf=True)


@pytest.mark.parametrize("bs", [1, 2, 3, 8, 12, 15, 16])
def test_batched_block_sizes(bs):
    note(f"[batched] bs={bs}")
    mats = [inputs.skew_normal(n, 100 + n) for n in (5, 33, 100, 199, 256)]
    db = DeviceBatch(mats)
    db.run(block_size=bs)
    for M, r in zip(mats, db.results()):
        check_against_oracle(M, r, check_pf=True)


def test_batched_alone_equals_in_mix_and_order_free():
    note("[batched] alone vs mix")
    mats = mixed_batch(40, 5)
    db = DeviceBatch(mats)
    db.run(max_n=256)
    mix = db.results()
    order = np.random.default_rng(3).permutation(len(mats))
    db2 = DeviceBatch([mats[k] for k in order])
    db2.run(max_n=256)
    shuf = db2.results()
    for pos, k in enumerate(order):
        assert np.array_equal(shuf[pos]["A"], mix[k]["A"])
        assert np.array_equal(shuf[pos]["ipiv"], mix[k]["ipiv"])
        assert shuf[pos]["log_abs_pf"] == mix[k]["log_abs_pf"] or (
            np.isinf(shuf[pos]["log_abs_pf"]) and np.isinf(mix[k]["log_abs_pf"]))
    for k in (0, 7, 23):
        alone = DeviceBatch([mats[k]])
        alone.run(max_n=256)
        a = alone.results()[0]
        assert np.array_equal(a["A"], mix[k]["A"]) and np.array_equal(a["ipiv"], mix[k]["ipiv"])
        assert a["sign"] == mix[k]["sign"]


def test_batched_rejects_invalid_members():
    note("[batched] invalid members")
    good = inputs.skew_normal(20, 1)
    big = inputs.skew_normal(30, 2)
    db = DeviceBatch([good, big, good], ldas=[20, 30, 10])  # lda < n for the third
    db.run(max_n=25)  # the second exceeds max_n
    res = db.results()
    assert res[0]["info"] == 0 and res[1]["info"] == -1 and res[2]["info"] == -1
    assert np.array_equal(res[1]["A"], big)
    for r in res[1:]:  # no result: NaN log|Pf| and sign 0, t and ipiv untouched
        assert np.isnan(r["log_abs_pf"]) and r["sign"] == 0
        assert np.all(r["t"] == -5.0) and np.all(r["ipiv"] == -1)
    check_against_oracle(good, res[0], check_pf=True)


def test_batched_rejects_member_spanning_2gib():
    """A member whose matrix spans 2 GiB or more ((n-1) lda + n doubles) is
    rejected like the other invalid members; the buffer given for it is
    allocated in full (3.4 GB), so no address the kernel could form lies
    outside it.  The other member of the batch is factored as usual."""
    import torch
    note("[batched] member spanning 2 GiB")
    n, lda = 200, 1 << 21
    assert ((n - 1) * lda + n) * 8 >= 2 ** 31 - 1
    big = torch.zeros((n, lda), dtype=torch.float64, device="cuda")  # column-major lda x n
    M = inputs.skew_normal(n, 3)
    big[:, :n] = torch.from_numpy(np.ascontiguousarray(M.T)).to("cuda")
    good = inputs.skew_normal(40, 4)
    gbuf = torch.from_numpy(np.asfortranarray(good)).to("cuda")  # stride (1, 40)
    ts = [torch.full((n - 1,), -5.0, dtype=torch.float64, device="cuda") for n in (40, n)]
    ps = [torch.full((n,), -1, dtype=torch.int32, device="cuda") for n in (40, n)]
    dev = "cuda"
    n_dev = torch.tensor([40, n], dtype=torch.int32, device=dev)
    lda_dev = torch.tensor([40, lda], dtype=torch.int32, device=dev)
    A_ptrs = torch.tensor([gbuf.data_ptr(), big.data_ptr()], dtype=torch.int64, device=dev)
    t_ptrs = torch.tensor([t.data_ptr() for t in ts], dtype=torch.int64, device=dev)
    p_ptrs = torch.tensor([p.data_ptr() for p in ps], dtype=torch.int64, device=dev)
    la = torch.zeros(2, dtype=torch.float64, device=dev)
    sg = torch.full((2,), 9, dtype=torch.int32, device=dev)
    info = torch.full((2,), 5, dtype=torch.int32, device=dev)
    work = binding.alloc_workspace(binding.batched_workspace_size(2))
    binding.batched(n_dev, A_ptrs, lda_dev, t_ptrs, p_ptrs, la, sg, info, 256, 0, binding.FP64, work)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, -1]
    assert np.isnan(float(la[1])) and int(sg[1]) == 0
    assert np.all(ts[1].cpu().numpy() == -5.0) and np.all(ps[1].cpu().numpy() == -1)
    assert np.array_equal(big[:, :n].cpu().numpy().T, M)
    del big
    res = {"A": np.asfortranarray(gbuf.cpu().numpy()), "t": ts[0].cpu().numpy(),
           "ipiv": ps[0].cpu().numpy(), "log_abs_pf": float(la[0]), "sign": int(sg[0]),
           "info": 0}
    check_against_oracle(good, res, check_pf=True)


def test_batched_argument_errors():
    import torch
    n = torch.zeros(1, dtype=torch.int32, device="cuda")
    p = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(binding.SkltltError):
        binding.batched(n, p, n, p, p, None, None, None, max_n=300)
    with pytest.raises(binding.SkltltError):
        binding.batched(n, p, n, p, p, None, None, None, max_n=10, precision=binding.FP32_UPDATE)


def test_batched_hipgraph_replays():
    """Capture one batched launch in a graph and replay it; every replay must
    reproduce the eager result (inputs restored between replays)."""
    import torch
    note("[batched] hipGraph")
    mats = mixed_batch(24, 17)
    db = DeviceBatch(mats)
    db.run(max_n=256)
    eager = db.results()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    db.restore()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        db.run(max_n=256, stream=s)
    for rep in range(3):
        db.restore()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = db.results()
        for a, b in zip(got, eager):
            assert np.array_equal(a["A"], b["A"]) and np.array_equal(a["ipiv"], b["ipiv"])
            assert a["sign"] == b["sign"]
