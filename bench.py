#!/usr/bin/env python
"""Benchmark: FP64 pivoted skew LTL^T + Pfaffian of one n = 16384 matrix.

One step = one skltlt_pfaffian call (panel, skr2k update, row gathers,
Pfaffian) on a device-resident graded skew matrix A_ij = N(0,1) * 10^U(-6,6).
The input is restored from a pristine device copy before every step, outside
the timed region.  Prints ONE JSON line on stdout; progress goes to stderr.

Reported value: GFLOP/s at the nominal n^3/3 flops of the paper (Sec. 3.6).
Also reported: the same step with the FP32-MFMA update variant (backward error
and Pfaffian difference stated), a per-kernel time breakdown measured with HIP
events on the library's stream during the timed steps, the roofline of the
dominant kernel, and the CPU oracle timed on a bounded sample (first column
steps of the same matrix) on this host.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6    # MI355X dense FP64 MFMA
PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 MFMA
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_times(lib):
    out = {}
    names = ["panel", "skr2k", "finalize", "pfaffian", "batched", "other", "solve"]
    for k, nm in enumerate(names):
        ms = ctypes.c_double(0)
        cnt = ctypes.c_int(0)
        fl = ctypes.c_double(0)
        st = lib.skltlt_timing_read(k, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(fl))
        if st != 0:
            raise RuntimeError(f"skltlt_timing_read failed {st}")
        if cnt.value:
            out[nm] = {"total_ms": ms.value, "launches": cnt.value, "flops": fl.value}
    return out


def skr2k_bytes(n, b):
    """Algorithmic HBM bytes of all skr2k launches of one factorization: each
    launch reads the strict lower triangle of the trailing block once (8 B
    per element, at permuted positions), writes it and its negated mirror
    (16 B per element) and reads the two m x K operand panels once."""
    tot = 0.0
    k0 = 0
    while k0 < n - 1:
        nb = min(b, n - 1 - k0)
        cp = k0 + nb
        m = n - cp
        if cp < n - 1 and m >= 2:
            K = 2 * ((nb + 1) // 2)
            tot += 24.0 * m * (m - 1) / 2.0 + 16.0 * m * K
        k0 = cp
    return tot


def panel_flops(n, b):
    """FP64 flops of the panel's left-looking products x = y - L h (2 flops
    per stored L entry of every candidate row at every column step)."""
    tot = 0.0
    for c in range(n - 1):
        j = c % b
        tot += 2.0 * (n - c - 1) * (j + 1)
    return tot


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "skr2k_n16384_b256_traffic.txt")
MFMA_SUMMARY = os.path.join(ROOT, "profiles", "skr2k_n16384_b256_mfma_counters.txt")


def _committed_counters(path, n, b, key):
    """A figure from a committed counter summary, or None with the reason
    when the summary does not describe this kernel source and workload."""
    from paper_2411_09859_amd import profsum
    if not os.path.exists(path):
        return None, "no counter summary"
    v = profsum.read_summary(path)
    if v.get("workload") != f"n={n} b={b}":
        return None, "counters were taken at another workload"
    srcs = [os.path.join(ROOT, x.strip()) for x in v.get("source", "").split(",") if x.strip()]
    if not srcs or not all(os.path.exists(x) for x in srcs) or \
            profsum.sha256_of(",".join(srcs)) != v.get("source_sha256"):
        return None, "kernel source changed since the counters were taken"
    return float(v[key]), os.path.relpath(path, ROOT)


def measured_traffic(n, b):
    """Counter-measured HBM bytes per skr2k launch from the committed summary."""
    return _committed_counters(TRAFFIC_SUMMARY, n, b, "traffic_bytes_per_launch")


def measured_mfma_busy(n, b):
    """Counter-measured MFMA busy fraction of the skr2k from the committed
    summary."""
    return _committed_counters(MFMA_SUMMARY, n, b, "mfma_busy_fraction")


def resid_probe(torch, A0, Af, t, ipiv, nprobe=4, seed=0):
    """max over probes of ||(P A P^T - L T L^T) v|| / (||A||_F ||v||), O(n^2) each."""
    n = A0.shape[0]
    low = torch.tril(A0, -1)
    Afull = low - low.T
    del low
    q = torch.arange(n, device=A0.device)
    piv = ipiv.to(torch.int64).cpu().numpy()
    qq = np.arange(n)
    for r in range(n):
        p = int(piv[r])
        if p != r:
            qq[r], qq[p] = qq[p], qq[r]
    q = torch.from_numpy(qq).to(A0.device)
    PAP = Afull.index_select(0, q).index_select(1, q)
    del Afull
    L = torch.tril(Af, -2)
    L = torch.roll(L, shifts=1, dims=1)  # L[i][j+1] stored at (i, j)
    L[:, 0] = 0
    L = L + torch.eye(n, dtype=L.dtype, device=L.device)
    normA = torch.linalg.norm(PAP).item()
    g = torch.Generator(device=A0.device)
    g.manual_seed(seed)
    worst = 0.0
    for _ in range(nprobe):
        v = torch.randn(n, dtype=torch.float64, device=A0.device, generator=g)
        w = L.T @ v
        tw = torch.zeros_like(w)
        tw[1:] += t * w[:-1]
        tw[:-1] -= t * w[1:]
        lhs = PAP @ v
        rhs = L @ tw
        worst = max(worst, (torch.linalg.norm(lhs - rhs) / (normA * torch.linalg.norm(v))).item())
    del PAP, L
    return worst


def bench_batched(torch, binding, inputs, count, seed=4, reps=3):
    """4096 matrices, even n uniform over [16, 256], 5% singular: one batched
    launch vs a loop of per-matrix skltlt_pfaffian launches on one stream."""
    from paper_2411_09859_amd.batch import Arena
    log(f"[bench] batched: building {count} matrices")
    sizes, sing = inputs.batch_sizes(count, seed)
    mats = inputs.batch_matrices(sizes, sing, seed)
    ar = Arena(mats)
    flops = float(np.sum(sizes.astype(np.float64) ** 3) / 3.0)
    for _ in range(1):
        ar.restore()
        ar.run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        ar.restore()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ar.run()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms_eager = float(np.median(ts))
    signs = ar.sign.cpu().numpy()
    logpf = ar.log_abs_pf.cpu().numpy()
    # the same launch captured once in a hipGraph and replayed (inputs
    # restored between replays, outside the timed region); every replay must
    # reproduce the eager Pfaffians bit for bit
    gs = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    ar.restore()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=gs):
        ar.run(stream=gs)
    gts = []
    graph_equal = True
    for _ in range(reps):
        ar.restore()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(gs):  # replay() launches on the current stream
            e0.record()
            graph.replay()
            e1.record()
        torch.cuda.synchronize()
        gts.append(e0.elapsed_time(e1))
        graph_equal = graph_equal and np.array_equal(ar.sign.cpu().numpy(), signs) and \
            np.array_equal(ar.log_abs_pf.cpu().numpy(), logpf)
    ms = float(np.median(gts))
    # baseline: per-matrix launches over a prefix of the same batch
    nbase = min(256, count)
    ar.restore()
    torch.cuda.synchronize()
    t = torch.zeros(256, dtype=torch.float64, device="cuda")
    ip = torch.zeros(256, dtype=torch.int32, device="cuda")
    la = torch.zeros(1, dtype=torch.float64, device="cuda")
    sg = torch.zeros(1, dtype=torch.int32, device="cuda")
    work = binding.alloc_workspace(binding.workspace_size(256, 0, binding.FP64))
    base_signs = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(nbase):
        binding.pfaffian(ar.matrix(k), t, ip, la, sg, 0, binding.FP64, work)
    e1.record()
    torch.cuda.synchronize()
    base_ms_per = e0.elapsed_time(e1) / nbase
    out = {"workload": f"{count} matrices, even n uniform in [16,256], N(0,1), "
                       f"{int(sing.sum())} structurally singular, seed {seed}",
           "ms": ms, "launch": "hipGraph replay", "ms_eager_launch": ms_eager,
           "graph_replays_equal_eager": bool(graph_equal), "pfaffians_per_s": count / (ms * 1e-3),
           "gflops_nominal": flops / (ms * 1e-3) / 1e9,
           "zero_pfaffians": int(np.sum(signs == 0)),
           "per_matrix_launch_baseline": {"matrices_timed": nbase, "ms_per_matrix": base_ms_per,
                                          "pfaffians_per_s": 1e3 / base_ms_per},
           "speedup_vs_per_matrix": (count / (ms * 1e-3)) / (1e3 / base_ms_per)}
    log(f"[bench] batched {out}")
    return out


def bench_serving(torch, count, seed=5):
    """Serving stream: n log-uniform over even values in [32, 2048], FP64 /
    FP32-update tags, 64 GB budget.  A closed-loop run (all requests at t=0)
    measures capacity; Poisson runs at 50 %, 80 % and 95 % of it measure
    latency under load."""
    from paper_2411_09859_amd.serving import GpuExecutor, Server, make_requests, summarize
    reqs = make_requests(count, seed, rate_per_s=1.0)
    for r in reqs:
        r.arrival = 0.0
    srv = Server(GpuExecutor(n_streams=4), budget_bytes=64 << 30)
    t0 = time.perf_counter()
    res = srv.run(reqs, time_limit_s=600)
    wall = time.perf_counter() - t0
    closed = summarize(res, wall)
    cap = closed["solves_per_s"]
    log(f"[bench] serving closed loop {closed}")
    out = {"workload": f"{count} requests (of the 100000-request stream), n log-uniform even in "
                       f"[32,2048], FP64/FP32-update 50/50, Poisson arrivals, 64 GB budget",
           "closed_loop": closed}
    for pct, sd in ((80, seed + 1), (50, seed + 2), (95, seed + 3)):
        rate = pct / 100.0 * cap
        reqs = make_requests(count, sd, rate_per_s=rate)
        srv = Server(GpuExecutor(n_streams=4), budget_bytes=64 << 30)
        t0 = time.perf_counter()
        res = srv.run(reqs, time_limit_s=600)
        wall = time.perf_counter() - t0
        openl = summarize(res, wall)
        log(f"[bench] serving poisson at {pct}% {openl}")
        out[f"poisson_at_{pct}pct"] = dict(openl, rate_per_s=rate)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--fp32-steps", type=int, default=2)
    ap.add_argument("--cpu-steps", type=int, default=160,
                    help="oracle column steps in the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--serving-count", type=int, default=2000,
                    help="requests in the serving runs (the full stream has 100000)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--solve-steps", type=int, default=3,
                    help="timed solves with the factors (0: skip)")
    ap.add_argument("--partial-steps", type=int, default=2,
                    help="timed Pfaffian-only (partial) reductions (0: skip)")
    ap.add_argument("--nopiv-steps", type=int, default=2,
                    help="timed unpivoted factorizations of a known-factor matrix (0: skip)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(a single factorization is not sharded); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2411_09859_amd import binding, inputs

    lib = binding.lib()
    n = args.n
    b = args.block if args.block > 0 else binding.default_block_size(n)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    log(f"[bench] generating graded skew matrix n={n} seed={args.seed}")
    t0 = time.time()
    A_np = inputs.skew_graded(n, args.seed, full=False)
    log(f"[bench] generated in {time.time() - t0:.1f}s")
    A0 = binding.to_device_colmajor(A_np)
    Aw = torch.empty_strided((n, n), (1, n), dtype=torch.float64, device=dev)
    t = torch.zeros(n - 1, dtype=torch.float64, device=dev)
    ipiv = torch.zeros(n, dtype=torch.int32, device=dev)
    la = torch.zeros(1, dtype=torch.float64, device=dev)
    sg = torch.zeros(1, dtype=torch.int32, device=dev)
    ws_bytes = max(binding.workspace_size(n, b, binding.FP64),
                   binding.workspace_size(n, b, binding.FP32_UPDATE))
    work = binding.alloc_workspace(ws_bytes, dev)
    stream = torch.cuda.current_stream()

    def one(prec):
        Aw.copy_(A0)
        binding.pfaffian(Aw, t, ipiv, la, sg, b, prec, work, stream)

    log(f"[bench] warmup {args.warmup} (b={b})")
    for _ in range(args.warmup):
        one(binding.FP64)
    torch.cuda.synchronize()

    nblk = (n - 1 + b - 1) // b
    lib.skltlt_timing_enable(args.steps * (2 * nblk + 8) + 16)
    step_ms = []
    for s in range(args.steps):
        Aw.copy_(A0)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        binding.pfaffian(Aw, t, ipiv, la, sg, b, binding.FP64, work, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        step_ms.append(ev0.elapsed_time(ev1))
        log(f"[bench] step {s}: {step_ms[-1]:.2f} ms")
    lib.skltlt_timing_disable()
    kt = kernel_times(lib)
    ms = float(np.mean(step_ms))
    nominal = n ** 3 / 3.0
    gflops = nominal / (ms * 1e-3) / 1e9
    log(f"[bench] FP64 mean {ms:.2f} ms -> {gflops:.1f} GFLOP/s (n^3/3); kernels {kt}")

    sign64 = int(sg.item())
    logpf64 = float(la.item())
    ipiv64 = ipiv.clone()
    checks = {}
    if not args.no_check:
        checks["resid_probe_fp64"] = resid_probe(torch, A0, Aw, t, ipiv)
        log(f"[bench] fp64 residual probe {checks['resid_probe_fp64']:.3e}")

    # solving A x = w with the factors just computed (one right-hand side)
    solve = None
    if args.solve_steps > 0:
        g = torch.Generator(device=dev)
        g.manual_seed(args.seed)
        w = torch.randn(n, dtype=torch.float64, device=dev, generator=g)
        x = torch.empty_like(w)
        swork = binding.alloc_workspace(binding.solve_workspace_size(n, 1), dev)
        x.copy_(w)
        binding.solve(Aw, t, ipiv, x, swork, stream)
        torch.cuda.synchronize()
        sms = []
        for _ in range(args.solve_steps):
            x.copy_(w)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            binding.solve(Aw, t, ipiv, x, swork, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            sms.append(e0.elapsed_time(e1))
        low = torch.tril(A0, -1)
        r = (low - low.T) @ x - w
        nA = torch.linalg.norm(low) * 2 ** 0.5
        solve = {"n": n, "nrhs": 1, "ms": float(np.median(sms)),
                 "backward_error": (torch.linalg.norm(r) / (nA * torch.linalg.norm(x))).item()}
        del low, r
        log(f"[bench] solve {solve}")

    # Pfaffian only by the pairwise (partial) reduction of the same matrix
    partial = None
    if args.partial_steps > 0:
        tp = torch.zeros_like(t)
        ipp = torch.zeros_like(ipiv)
        lap = torch.zeros_like(la)
        sgp = torch.zeros_like(sg)
        binding.pfaffian_partial(A0, tp, ipp, lap, sgp, b, binding.FP64, work, stream)
        torch.cuda.synchronize()
        pms = []
        for _ in range(args.partial_steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            binding.pfaffian_partial(A0, tp, ipp, lap, sgp, b, binding.FP64, work, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            pms.append(e0.elapsed_time(e1))
        pm = float(np.median(pms))
        partial = {"n": n, "ms": pm, "speedup_vs_full": ms / pm,
                   "sign_equal_full": int(sgp.item()) == sign64,
                   "log_abs_pf_rel_diff_full":
                       abs(float(lap.item()) - logpf64) / max(1.0, abs(logpf64))}
        del tp, ipp
        log(f"[bench] partial {partial}")

    # unpivoted factorization (for inputs that need no pivoting) on a matrix
    # assembled from known factors, A = L0 T0 L0^T, of the same order
    nopiv = None
    if args.nopiv_steps > 0:
        g = torch.Generator(device=dev)
        g.manual_seed(args.seed + 11)
        L0 = torch.tril((torch.rand((n, n), generator=g, dtype=torch.float64, device=dev) * 2 - 1)
                        * (2.0 / n ** 0.5), -1)
        L0[:, 0] = 0
        L0 += torch.eye(n, dtype=torch.float64, device=dev)
        t0 = (1.0 + 0.01 * torch.rand(n - 1, generator=g, dtype=torch.float64, device=dev)) * \
            torch.where(torch.rand(n - 1, generator=g, device=dev) < 0.5, -1.0, 1.0).double()
        K = torch.diag(t0, -1) - torch.diag(t0, 1)
        K = (L0 @ K) @ L0.T.contiguous()
        del L0
        Kc = K.T.contiguous().T
        del K
        bn = min(b, 128)
        tn = torch.zeros_like(t)
        ipn = torch.zeros_like(ipiv)
        lan = torch.zeros_like(la)
        sgn = torch.zeros_like(sg)
        nms = []
        for s_ in range(args.nopiv_steps + 1):
            Aw.copy_(Kc)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            binding.pfaffian_nopiv(Aw, tn, ipn, lan, sgn, bn, binding.FP64, work, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            if s_ > 0:  # the first run is the warmup
                nms.append(e0.elapsed_time(e1))
        nm = float(np.mean(nms))
        nopiv = {"workload": f"n={n} A = L0 T0 L0^T, |L0| <= 2/sqrt(n), |t0| in [1, 1.01]",
                 "block": bn, "ms": nm, "gflops_nominal": nominal / (nm * 1e-3) / 1e9,
                 "frac_fp64_peak": nominal / (nm * 1e-3) / 78.6e12,
                 "t_rel_err_vs_t0": (torch.linalg.norm(tn - t0) / torch.linalg.norm(t0)).item()}
        # the same factorization by the left-looking algorithm
        lwork = binding.alloc_workspace(binding.left_workspace_size(n, bn), dev)
        lms = []
        for s_ in range(args.nopiv_steps + 1):
            Aw.copy_(Kc)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            binding.pfaffian_left(Aw, tn, ipn, lan, sgn, bn, lwork, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            if s_ > 0:
                lms.append(e0.elapsed_time(e1))
        del lwork
        lm = float(np.mean(lms))
        nopiv["left_looking"] = {
            "ms": lm, "gflops_nominal": nominal / (lm * 1e-3) / 1e9,
            "t_rel_err_vs_t0": (torch.linalg.norm(tn - t0) / torch.linalg.norm(t0)).item()}
        del Kc, tn, ipn, t0
        log(f"[bench] nopiv {nopiv}")

    # FP32-update variant
    fp32 = None
    if args.fp32_steps > 0:
        one(binding.FP32_UPDATE)
        torch.cuda.synchronize()
        tms = []
        for _ in range(args.fp32_steps):
            Aw.copy_(A0)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            binding.pfaffian(Aw, t, ipiv, la, sg, b, binding.FP32_UPDATE, work, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            tms.append(e0.elapsed_time(e1))
        ms32 = float(np.mean(tms))
        fp32 = {"ms_per_step": ms32, "gflops_nominal": nominal / (ms32 * 1e-3) / 1e9,
                "sign": int(sg.item()), "log_abs_pf": float(la.item()),
                "sign_matches_fp64": int(sg.item()) == sign64,
                "abs_dlog_pf_vs_fp64": abs(float(la.item()) - logpf64),
                "pivots_equal_fp64": bool(torch.equal(ipiv, ipiv64))}
        if not args.no_check:
            fp32["resid_probe"] = resid_probe(torch, A0, Aw, t, ipiv)
        log(f"[bench] FP32-update {fp32}")

    # roofline of the throughput-bound kernel (the trailing update); the
    # panel is latency-bound and reported by its per-step time
    dom = max(("skr2k", "panel"), key=lambda k: kt.get(k, {}).get("total_ms", 0.0))
    roof = None
    if "skr2k" in kt:
        sk = kt["skr2k"]
        steps = args.steps
        per_launch_ms = sk["total_ms"] / sk["launches"]
        flops_per_launch = sk["flops"] / sk["launches"]
        achieved = flops_per_launch / (per_launch_ms * 1e-3) / 1e12
        bytes_per_launch = skr2k_bytes(n, b) * steps / sk["launches"]
        traffic, traffic_src = measured_traffic(n, b)
        busy, busy_src = measured_mfma_busy(n, b)
        roof = {"kernel": "skr2k_kernel<double>", "bound": "mfma", "achieved": achieved,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": traffic, "traffic_source": traffic_src,
                "mfma_busy": busy, "mfma_busy_source": busy_src,
                "flops_per_launch": flops_per_launch,
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "avg_launch_ms": per_launch_ms,
                "hbm_gbs_algorithmic": bytes_per_launch / (per_launch_ms * 1e-3) / 1e9,
                "hbm_frac_algorithmic": bytes_per_launch / (per_launch_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                "dominant_class_by_time": dom}
    panel = None
    if "panel" in kt:
        pk = kt["panel"]
        pms = pk["total_ms"] / args.steps
        pf = panel_flops(n, b)
        panel = {"bound": "latency", "ms_per_step": pms,
                 "us_per_column_step": pms * 1e3 / (n - 1),
                 "alu_flops": pf, "alu_tflops": pf / (pms * 1e-3) / 1e12,
                 "alu_frac": pf / (pms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}

    # CPU oracle on a bounded sample
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        nthr = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, os.cpu_count() or 1)
        s_steps = min(args.cpu_steps, n - 1)
        log(f"[bench] oracle sample: first {s_steps} column steps, {nthr} threads")
        tt = time.time()
        oracle.ltlt(A_np, max_steps=0, nthreads=nthr)
        t_setup = time.time() - tt
        tt = time.time()
        ref = oracle.ltlt(A_np, max_steps=s_steps, nthreads=nthr)
        t_s = time.time() - tt - t_setup
        w_s = sum((n - k - 1) ** 2 for k in range(s_steps))
        w_all = sum((n - k - 1) ** 2 for k in range(n - 1))
        t_full = t_s * w_all / w_s
        cpu = {"value": nominal / t_full / 1e9, "unit": "GFLOP/s", "cores": nthr, "kind": "oracle",
               "sample": (f"first {s_steps} of {n - 1} column steps of the same n={n} matrix "
                          f"({t_s:.1f} s measured after {t_setup:.1f} s setup), extrapolated by the "
                          f"per-step work (n-k-1)^2 to {t_full:.0f} s for the whole factorization")}
        gp = ipiv64.cpu().numpy()
        checks["oracle_prefix_steps"] = s_steps
        checks["ipiv_prefix_equal_oracle"] = bool(np.array_equal(gp[: s_steps + 1],
                                                                   ref["ipiv"][: s_steps + 1]))
        log(f"[bench] oracle {cpu}")

    batched = None if args.no_batched else bench_batched(torch, binding, inputs, args.batch_count)
    serving = None if args.no_serving else bench_serving(torch, args.serving_count)

    out = {
        "metric": "FP64 skew-LTLt GFLOP/s (n^3/3) at n=16384; batched Pfaffians/s + p99 latency",
        "value": gflops,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"pivoted skew LTL^T + Pfaffian, one n={n} matrix, graded "
                               f"N(0,1)*10^U(-6,6), seed {args.seed}, FP64",
                   "n": n, "block_size": b},
        "roofline": roof,
        "step_ms": {"mean": ms, "median": float(np.median(step_ms)), "min": float(np.min(step_ms)),
                    "max": float(np.max(step_ms))},
        "panel": panel,
        "solve": solve,
        "pfaffian_partial": partial,
        "nopiv": nopiv,
        "cpu_baseline": cpu,
        "kernels": kt,
        "fp32_update": fp32,
        "pfaffian_fp64": {"sign": sign64, "log_abs_pf": logpf64},
        "batched": batched,
        "serving": serving,
        "checks": checks,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
