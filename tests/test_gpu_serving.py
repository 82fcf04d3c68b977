"""GPU tests of the serving loop: results alone and in a concurrent mix are
identical, match the oracle, and a real-time Poisson stream completes."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2411_09859_amd import inputs
from paper_2411_09859_amd.serving import GpuExecutor, Request, Server, make_requests, summarize
from tests import checkers as ck
from tests.gpu_util import note

pytestmark = pytest.mark.gpu


def serve(reqs, **kw):
    srv = Server(GpuExecutor(n_streams=4), budget_bytes=8 << 30, **kw)
    res = srv.run(reqs, time_limit_s=300)
    return {r.rid: r for r in res}, srv


U32 = 2.0 ** -24


def check_vs_oracle(res, M, n, fp32):
    """A served result against the oracle: FP64 to 1e-12; an FP32-update
    result (pivots may differ) by its sign and the bound n u32 of its
    arithmetic on log|Pf| and on the backward error of its factors."""
    ref = oracle.ltlt(M)
    la, sg = oracle.pfaffian(n, ref["t"], ref["ipiv"])
    assert res.sign == sg
    tol = (n * U32) if fp32 else 1e-12
    assert abs(res.log_abs_pf - la) <= tol * max(1.0, abs(la))
    if res.factors is not None:
        A_d, t_d, ip_d = res.factors
        ip = ip_d.cpu().numpy()[:n]
        t = t_d.cpu().numpy()[: n - 1]
        if fp32:
            L, tt = ck.unpack(np.asfortranarray(A_d.cpu().numpy()), n)
            assert np.array_equal(tt, t)
            assert ck.residual(ck.full_skew(M), L, t, ip) <= n * U32
        else:
            assert np.array_equal(ip, ref["ipiv"])
            assert np.linalg.norm(t - ref["t"]) <= 1e-12 * np.linalg.norm(ref["t"])


def test_alone_equals_mix_and_oracle():
    """Factorization and Pfaffian requests of both paths (batched for
    n <= 256, alone above: full factorization or the partial reduction), with
    both precision tags."""
    note("[serving] alone vs mix")
    sizes = [32, 48, 100, 130, 256, 300, 520, 770, 34, 64, 1030, 200, 302, 1030,
             40, 250, 400, 900, 36, 128, 600, 1024]
    mats = [inputs.skew_normal(n, 500 + k) for k, n in enumerate(sizes)]
    kind = [k % 2 == 0 for k in range(len(sizes))]  # True: factorization request
    prec = [0] * 14 + [1] * 8                         # the last eight FP32-tagged
    mix = [Request(k, n, precision=prec[k], arrival=0.0, matrix=M, factor=kind[k])
           for k, (n, M) in enumerate(zip(sizes, mats))]
    got, srv = serve(mix)
    assert len(got) == len(sizes) and srv.used == 0
    for k, M in enumerate(mats):
        n = sizes[k]
        alone, _ = serve([Request(k, n, precision=prec[k], arrival=0.0, matrix=M,
                                  factor=kind[k])])
        a, b = alone[k], got[k]
        assert a.error is None and b.error is None
        assert a.path == b.path
        assert b.path == ("batched" if n <= 256 else ("single" if kind[k] else "partial"))
        assert b.precision == prec[k]
        assert b.precision_used == (0 if n <= 256 else prec[k])
        assert a.sign == b.sign
        assert a.log_abs_pf == b.log_abs_pf  # bitwise: no dependence on the mix
        if kind[k]:
            for x, y in zip(a.factors, b.factors):
                assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
        else:
            assert b.factors is None
        check_vs_oracle(b, M, n, fp32=(b.precision_used == 1))


def test_poisson_stream_matches_oracle():
    """A real-time Poisson stream completes within the memory budget, and a
    sample of its results (matrices regenerated from the requests' seeds)
    matches the oracle."""
    import torch
    note("[serving] poisson stream")
    reqs = make_requests(300, seed=5, rate_per_s=400.0, hi=1024)
    by_id = {r.rid: (r.n, r.seed, r.precision) for r in reqs}
    got, srv = serve(reqs)
    assert len(got) == 300
    assert all(r.error is None and r.sign in (-1, 0, 1) for r in got.values())
    assert srv.peak_used <= srv.budget
    s = summarize(list(got.values()), wall_s=max(r.done for r in got.values()) -
                  min(r.arrival for r in got.values()))
    note(f"[serving] {s}")
    assert s["p99_ms"] >= s["p50_ms"] > 0
    assert s["by_tag"]["fp64"]["requests"] + s["by_tag"]["fp32_update"]["requests"] == 300
    for rid in range(0, 300, 15):
        n, seed, pr = by_id[rid]
        g = torch.Generator(device="cuda")
        g.manual_seed(int(seed))
        M = torch.randn((n, n), generator=g, dtype=torch.float64, device="cuda").t().cpu().numpy()
        r = got[rid]
        assert r.precision == pr
        check_vs_oracle(r, np.asfortranarray(M), n, fp32=(r.precision_used == 1))
