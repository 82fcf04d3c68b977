"""The allocation-free batched entry point (skltlt_batched_noalloc) against
skltlt_batched on the same inputs: two calls in a row, the second with a
smaller batch, each bit for bit equal to the workspace call (same kernels,
same per-matrix arithmetic) and checked against the oracle."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2411_09859_amd import binding, inputs
from tests.gpu_util import DeviceBatch, note
from tests.test_gpu_factor import check_against_oracle

pytestmark = pytest.mark.gpu


def run_noalloc(db, max_n=None, block_size=0):
    mx = max(db.ns) if max_n is None else max_n
    binding.batched_noalloc(db.n_dev, db.A_ptrs, db.lda_dev, db.t_ptrs, db.p_ptrs, db.la, db.sg,
                            db.info, max(mx, 0), block_size, binding.FP64)


def clear(db):
    """Restore the inputs and overwrite every output of an earlier run."""
    db.restore()
    for t in db.ts:
        t.fill_(-5.0)
    for p in db.ipivs:
        p.fill_(-1)
    db.la.fill_(123.0)
    db.sg.fill_(9)
    db.info.fill_(5)


def same(a, b):
    for x, y in zip(a, b):
        assert x["info"] == y["info"]
        assert np.array_equal(x["buf"], y["buf"])
        assert np.array_equal(x["t"], y["t"]) and np.array_equal(x["ipiv"], y["ipiv"])
        assert x["sign"] == y["sign"]
        assert np.array_equal(np.array(x["log_abs_pf"]), np.array(y["log_abs_pf"]))


@pytest.mark.parametrize("count,seed,oracle_every", [(96, 31, 7), (9, 32, 1)])
def test_noalloc_equals_workspace_call(count, seed, oracle_every):
    note(f"[noalloc] batch of {count} (seed {seed})")
    sizes, sing = inputs.batch_sizes(count, seed)
    mats = inputs.batch_matrices(sizes, sing, seed)
    db = DeviceBatch(mats)
    db.run()
    ref = db.results()
    clear(db)
    run_noalloc(db)
    got = db.results()
    same(got, ref)
    for k in range(0, count, oracle_every):
        check_against_oracle(mats[k], got[k], check_pf=True)


def test_noalloc_two_calls_second_smaller():
    """Back to back on one stream: a batch, then a smaller one; the second
    must not see anything the first left in the shared scratch array."""
    note("[noalloc] two calls in a row")
    big = inputs.batch_matrices(*inputs.batch_sizes(200, 41), 41)
    small = inputs.batch_matrices(*inputs.batch_sizes(5, 42), 42)
    d1, d2 = DeviceBatch(big), DeviceBatch(small)
    d1.run()
    d2.run()
    r1, r2 = d1.results(), d2.results()
    clear(d1)
    clear(d2)
    run_noalloc(d1)
    run_noalloc(d2)
    same(d1.results(), r1)
    same(d2.results(), r2)
    for k, M in enumerate(small):
        check_against_oracle(M, d2.results()[k], check_pf=True)


def test_noalloc_rejects_oversized_batch():
    import torch
    mx = binding.batched_noalloc_max_batch()
    n = torch.zeros(1, dtype=torch.int32, device="cuda")
    p = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = binding.lib().skltlt_batched_noalloc(mx + 1, n.data_ptr(), p.data_ptr(), n.data_ptr(),
                                              p.data_ptr(), p.data_ptr(), None, None, None, 16,
                                              0, binding.FP64, None)
    assert st == binding.SKLTLT_ENOTSUP
