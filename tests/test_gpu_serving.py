"""GPU tests of the serving loop: results alone and in a concurrent mix are
identical, match the oracle, and a real-time Poisson stream completes."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2411_09859_amd import inputs
from paper_2411_09859_amd.serving import GpuExecutor, Request, Server, make_requests, summarize
from tests.gpu_util import note

pytestmark = pytest.mark.gpu


def serve(reqs, **kw):
    srv = Server(GpuExecutor(n_streams=4), budget_bytes=8 << 30, **kw)
    res = srv.run(reqs, time_limit_s=300)
    return {r.rid: r for r in res}, srv


def test_alone_equals_mix_and_oracle():
    """Factorization and Pfaffian requests of both paths (batched for
    n <= 256, alone above: full factorization or the partial reduction)."""
    note("[serving] alone vs mix")
    sizes = [32, 48, 100, 130, 256, 300, 520, 770, 34, 64, 1030, 200, 302, 1030]
    mats = [inputs.skew_normal(n, 500 + k) for k, n in enumerate(sizes)]
    kind = [k % 2 == 0 for k in range(len(sizes))]  # True: factorization request
    mix = [Request(k, n, precision=0, arrival=0.0, matrix=M, factor=kind[k]) for k, (n, M) in
           enumerate(zip(sizes, mats))]
    got, srv = serve(mix)
    assert len(got) == len(sizes) and srv.used == 0
    for k, M in enumerate(mats):
        n = sizes[k]
        alone, _ = serve([Request(k, n, arrival=0.0, matrix=M, factor=kind[k])])
        a, b = alone[k], got[k]
        assert a.path == b.path
        assert b.path == ("batched" if n <= 256 else ("single" if kind[k] else "partial"))
        assert a.sign == b.sign
        assert a.log_abs_pf == b.log_abs_pf  # bitwise: no dependence on the mix
        ref = oracle.ltlt(M)
        la, sg = oracle.pfaffian(n, ref["t"], ref["ipiv"])
        assert b.sign == sg
        assert abs(b.log_abs_pf - la) <= 1e-12 * max(1.0, abs(la))
        if kind[k]:
            A_d, t_d, ip_d = b.factors
            assert np.array_equal(ip_d.cpu().numpy()[:n], ref["ipiv"])
            assert np.linalg.norm(t_d.cpu().numpy()[: n - 1] - ref["t"]) <= \
                1e-12 * np.linalg.norm(ref["t"])
        else:
            assert b.factors is None


def test_poisson_stream_completes():
    note("[serving] poisson stream")
    reqs = make_requests(300, seed=5, rate_per_s=400.0, hi=1024)
    got, srv = serve(reqs)
    assert len(got) == 300
    assert all(r.error is None and r.sign in (-1, 0, 1) for r in got.values())
    assert srv.peak_used <= srv.budget
    s = summarize(list(got.values()), wall_s=max(r.done for r in got.values()) -
                  min(r.arrival for r in got.values()))
    note(f"[serving] {s}")
    assert s["p99_ms"] >= s["p50_ms"] > 0
