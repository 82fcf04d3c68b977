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
dominant kernel (the panel, by time) and of the trailing update, the CPU
oracle timed on the whole factorization of the same matrix on this host's
cores, and the full-length comparison of both precisions with that oracle.
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


def skr2k_bytes(n, b, per_elem=16.0):
    """HBM bytes of all skr2k launches of one factorization: each launch reads
    the strict lower triangle of the trailing block once and writes it
    (per_elem = 16 B per element, the algorithmic minimum, which the
    lower-triangle storage of the work matrices also moves) and reads the two
    m x K operand panels once."""
    tot = 0.0
    k0 = 0
    while k0 < n - 1:
        nb = min(b, n - 1 - k0)
        cp = k0 + nb
        m = n - cp
        if cp < n - 1 and m >= 2:
            K = 2 * ((nb + 1) // 2)
            tot += per_elem * m * (m - 1) / 2.0 + 16.0 * m * K
        k0 = cp
    return tot


def panel_tpr(b):
    """Threads per register row of the panel kernel for panel width b."""
    return 1 if b + 1 <= 65 else (2 if b + 1 <= 130 else 4)


def panel_flops(n, b):
    """FP64 flops of the panel's left-looking products x = y - L h (2 flops
    per stored L entry of every candidate row at every column step)."""
    tot = 0.0
    for c in range(n - 1):
        j = c % b
        tot += 2.0 * (n - c - 1) * (j + 1)
    return tot


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "skr2k_n16384_b256_traffic.txt")
PANEL_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "panel_n16384_b256_traffic.txt")
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


def measured_panel_traffic(n, b):
    """Counter-measured HBM bytes per panel launch from the committed summary."""
    return _committed_counters(PANEL_TRAFFIC_SUMMARY, n, b, "traffic_bytes_per_launch")


def panel_bytes(n, b):
    """Algorithmic HBM bytes of all panel launches of one factorization: the
    new column of every trailing row at each step, the panel's columns of L
    and the operands U, V written once."""
    tot = 0.0
    k0 = 0
    while k0 < n - 1:
        nb = min(b, n - 1 - k0)
        m = n - k0 - 1
        cp = k0 + nb
        tot += 16.0 * m * nb + (16.0 * (n - cp) * ((nb + 1) // 2) if cp < n - 1 else 0.0)
        k0 = cp
    return tot


def measured_mfma_busy(n, b):
    """Counter-measured MFMA busy fraction of the skr2k from the committed
    summary."""
    return _committed_counters(MFMA_SUMMARY, n, b, "mfma_busy_fraction")


def unpack_L(torch, Af):
    """Unit lower L from the packed layout (L[i][j+1] at (i, j), column 0 = e_0)."""
    n = Af.shape[0]
    L = torch.roll(torch.tril(Af, -2), shifts=1, dims=1)
    L[:, 0] = 0
    L += torch.eye(n, dtype=torch.float64, device=Af.device)
    return L


def permuted_full(torch, A0, ipiv_host):
    """P A P^T of the full skew matrix whose strict lower triangle is A0's."""
    n = A0.shape[0]
    qq = np.arange(n)
    for r in range(n):
        p = int(ipiv_host[r])
        if p != r:
            qq[r], qq[p] = qq[p], qq[r]
    low = torch.tril(A0, -1)
    Afull = low - low.T
    del low
    q = torch.from_numpy(qq).to(A0.device)
    PAP = Afull.index_select(0, q).index_select(1, q)
    del Afull
    return PAP


def exact_residual(torch, A0, Af, t, ipiv_host):
    """||P A P^T - L T L^T||_F / ||A||_F from one dense fp64 product."""
    PAP = permuted_full(torch, A0, ipiv_host)
    L = unpack_L(torch, Af)
    LT = torch.zeros_like(L)  # (L T)[:, j] = t[j] L[:, j+1] - t[j-1] L[:, j-1]
    LT[:, :-1] += L[:, 1:] * t[None, :]
    LT[:, 1:] -= L[:, :-1] * t[None, :]
    R = torch.matmul(LT, L.T.contiguous())
    del LT, L
    R -= PAP
    out = (torch.linalg.norm(R) / torch.linalg.norm(PAP)).item()
    del R, PAP
    torch.cuda.empty_cache()
    return out


def compare_with_oracle(torch, Af, t, ipiv_host, ref):
    """Pivots, t and L of a GPU factorization against the oracle's."""
    L = unpack_L(torch, Af)
    Lref = torch.from_numpy(np.asfortranarray(ref["L"])).to(Af.device)
    l_rel = (torch.linalg.norm(L - Lref) / torch.linalg.norm(Lref)).item()
    max_l = torch.max(torch.abs(L)).item()
    del L, Lref
    torch.cuda.empty_cache()
    th = t.cpu().numpy()
    eq = bool(np.array_equal(ipiv_host, ref["ipiv"]))
    out = {"ipiv_equal_oracle_full": eq,
           "t_rel_err": float(np.linalg.norm(th - ref["t"]) / np.linalg.norm(ref["t"])),
           "L_rel_err": l_rel, "max_abs_L": max_l}
    if not eq:
        d = np.nonzero(ipiv_host != ref["ipiv"])[0]
        out["pivot_steps_differing"] = int(d.size)
        out["first_pivot_step_differing"] = int(d[0])
    return out


def host_info():
    import platform
    import subprocess
    info = {"nproc": os.cpu_count(), "machine": platform.machine()}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            k = k.strip()
            if k in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core"):
                info[k] = v.strip()
    except Exception as exc:  # lscpu missing: say so
        info["lscpu"] = f"unavailable ({exc.__class__.__name__})"
    return info


def batched_vs_oracle(ar, sizes):
    """Every member of a batch against the oracle: pivots, t, Pfaffian."""
    import oracle
    pp = ar.ipiv.cpu().numpy()
    tt = ar.t.cpu().numpy()
    las = ar.log_abs_pf.cpu().numpy()
    sgs = ar.sign.cpu().numpy()
    piv_ok = sign_ok = 0
    worst_t = worst_pf = 0.0
    for k in range(len(sizes)):
        n = int(sizes[k])
        M = ar.pristine[int(ar.offs[k]):int(ar.offs[k]) + n * n].cpu().numpy().reshape((n, n), order="F")
        ref = oracle.ltlt(M, nthreads=1)
        p = pp[int(ar.ioffs[k]):int(ar.ioffs[k]) + n]
        piv_ok += int(np.array_equal(p, ref["ipiv"]))
        if n > 1:
            tk = tt[int(ar.toffs[k]):int(ar.toffs[k]) + n - 1]
            nr = np.linalg.norm(ref["t"])
            worst_t = max(worst_t, float(np.linalg.norm(tk - ref["t"]) / (nr if nr > 0 else 1.0)))
        la, sg = oracle.pfaffian(n, ref["t"], ref["ipiv"])
        sign_ok += int(sgs[k] == sg)
        if sg != 0 and sgs[k] == sg:
            worst_pf = max(worst_pf, abs(las[k] - la) / max(1.0, abs(la)))
    return {"members": len(sizes), "ipiv_equal_oracle": piv_ok, "sign_equal_oracle": sign_ok,
            "max_t_rel_err": worst_t, "max_rel_dlog_pf": worst_pf}


def bench_batched(torch, binding, inputs, count, seed=4, reps=3, check=True):
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
    oracle_check = None
    if check:
        log(f"[bench] batched: every member against the oracle")
        oracle_check = batched_vs_oracle(ar, sizes)
        log(f"[bench] batched oracle check {oracle_check}")
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
           "oracle_check": oracle_check,
           "per_matrix_launch_baseline": {"matrices_timed": nbase, "ms_per_matrix": base_ms_per,
                                          "pfaffians_per_s": 1e3 / base_ms_per},
           "speedup_vs_per_matrix": (count / (ms * 1e-3)) / (1e3 / base_ms_per)}
    log(f"[bench] batched {out}")
    return out


def bench_serving(torch, count, short_count, seed=5, deadline=None):
    """Serving stream: n log-uniform over even values in [32, 2048], FP64 /
    FP32-update tags, 64 GB budget.  A closed-loop run (all requests at t=0)
    measures capacity after an untimed warm-up run; Poisson runs at 80 %
    (``count`` requests), 50 % and 95 % (``short_count``) of it measure
    latency under load.  A run that would
    end after ``deadline`` (perf_counter seconds) is shortened, and the
    request count actually run is stated."""
    from paper_2411_09859_amd.serving import GpuExecutor, Server, make_requests, summarize

    def fit(want, rate):
        if deadline is None:
            return want
        left = deadline - time.perf_counter()
        return int(max(1000, min(want, 0.9 * left * rate)))

    # warm-up (untimed): a server in steady state, with torch's caching
    # allocator already holding blocks of the sizes the stream asks for (the
    # first requests of a cold process pay synchronous device allocations)
    warm = make_requests(min(2000, count), seed + 10, rate_per_s=1.0)
    for r in warm:
        r.arrival = 0.0
    Server(GpuExecutor(n_streams=4), budget_bytes=64 << 30, keep_factors=False).run(
        warm, time_limit_s=300)
    torch.cuda.synchronize()
    reqs = make_requests(count, seed, rate_per_s=1.0)
    for r in reqs:
        r.arrival = 0.0
    srv = Server(GpuExecutor(n_streams=4), budget_bytes=64 << 30, keep_factors=False)
    t0 = time.perf_counter()
    res = srv.run(reqs, time_limit_s=900)
    wall = time.perf_counter() - t0
    closed = summarize(res, wall)
    del res, srv
    cap = closed["solves_per_s"]
    log(f"[bench] serving closed loop {closed}")
    out = {"workload": f"n log-uniform even in [32,2048], FP64/FP32-update 50/50, "
                       f"factorization/Pfaffian 50/50, Poisson arrivals, 64 GB budget",
           "single_request_streams": 4,
           "closed_loop": closed}
    for pct, sd, want in ((80, seed + 1, count), (50, seed + 2, short_count),
                          (95, seed + 3, short_count)):
        rate = pct / 100.0 * cap
        cnt = fit(want, rate)
        reqs = make_requests(cnt, sd, rate_per_s=rate)
        srv = Server(GpuExecutor(n_streams=4), budget_bytes=64 << 30, keep_factors=False)
        t0 = time.perf_counter()
        res = srv.run(reqs, time_limit_s=900)
        wall = time.perf_counter() - t0
        openl = summarize(res, wall)
        del res, srv
        log(f"[bench] serving poisson at {pct}% {openl}")
        out[f"poisson_at_{pct}pct"] = dict(openl, rate_per_s=rate)
    torch.cuda.empty_cache()
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
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle column steps in the CPU baseline (0: the whole "
                         "factorization, which also gives the full-length oracle checks)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--serving-count", type=int, default=100000,
                    help="requests in the closed-loop and 80 %% runs (the full stream)")
    ap.add_argument("--serving-short", type=int, default=10000,
                    help="requests in the 50 %% and 95 %% runs")
    ap.add_argument("--time-budget", type=float, default=540.0,
                    help="seconds the whole run may take; later serving runs shrink to fit")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--solve-steps", type=int, default=3,
                    help="timed solves with the factors (0: skip)")
    ap.add_argument("--partial-steps", type=int, default=2,
                    help="timed Pfaffian-only (partial) reductions (0: skip)")
    ap.add_argument("--n8192-steps", type=int, default=3,
                    help="timed factorizations of the n = 8192 N(0,1) matrix (0: skip)")
    ap.add_argument("--nopiv-steps", type=int, default=2,
                    help="timed unpivoted factorizations of a known-factor matrix (0: skip)")
    args = ap.parse_args()

    t_start = time.perf_counter()
    deadline = t_start + args.time_budget
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
    ipiv64 = ipiv.cpu().numpy()
    t64 = t.clone()
    Af64 = Aw.clone()  # the FP64 factors, kept for the oracle comparison
    checks = {}

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
                "pivots_equal_fp64": bool(np.array_equal(ipiv.cpu().numpy(), ipiv64))}
        if not args.no_check:
            fp32["backward_error_exact"] = exact_residual(torch, A0, Aw, t, ipiv.cpu().numpy())
        log(f"[bench] FP32-update {fp32}")

    fp32_ipiv = ipiv.cpu().numpy() if fp32 is not None else None

    # the n = 8192 N(0,1) single-matrix workload at the block size the
    # library's tuned table picks for that order
    n8192 = None
    if args.n8192_steps > 0:
        n2 = 8192
        b2 = binding.default_block_size(n2)
        A2 = binding.to_device_colmajor(inputs.skew_normal(n2, 2, full=False))
        A2w = torch.empty_like(A2)
        t2 = torch.zeros(n2 - 1, dtype=torch.float64, device=dev)
        ip2 = torch.zeros(n2, dtype=torch.int32, device=dev)
        work2 = binding.alloc_workspace(binding.workspace_size(n2, b2, binding.FP64), dev)
        ms2 = []
        for s_ in range(args.n8192_steps + 1):
            A2w.copy_(A2)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            binding.pfaffian(A2w, t2, ip2, la, sg, b2, binding.FP64, work2, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            if s_ > 0:
                ms2.append(e0.elapsed_time(e1))
        m2 = float(np.median(ms2))
        n8192 = {"workload": "n=8192 N(0,1) seed 2, FP64", "block_size": b2,
                 "block_size_source": "tuned table (skltlt_default_block_size)",
                 "ms": m2, "gflops_nominal": n2 ** 3 / 3.0 / (m2 * 1e-3) / 1e9,
                 "frac_fp64_peak": n2 ** 3 / 3.0 / (m2 * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}
        del A2, A2w, work2
        torch.cuda.empty_cache()
        log(f"[bench] n=8192 {n8192}")

    # roofline of each kernel class; the line's "roofline" is the dominant
    # one by time, the other is reported beside it
    steps = args.steps
    roofs = {}
    if "skr2k" in kt:
        sk = kt["skr2k"]
        per_launch_ms = sk["total_ms"] / sk["launches"]
        flops_per_launch = sk["flops"] / sk["launches"]
        achieved = flops_per_launch / (per_launch_ms * 1e-3) / 1e12
        alg = skr2k_bytes(n, b, 16.0) * steps / sk["launches"]
        traffic, traffic_src = measured_traffic(n, b)
        busy, busy_src = measured_mfma_busy(n, b)
        roofs["skr2k"] = {
            "kernel": "skr2k_kernel<double> (128x128 tiles) and skr2k_small_kernel<double> "
                      "(64x64 tiles, trailing blocks with fewer 128-tiles than CUs)",
            "bound": "mfma", "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": traffic, "traffic_source": traffic_src,
            "traffic_over_algorithmic": (traffic / alg) if traffic else None,
            "mfma_busy": busy, "mfma_busy_source": busy_src,
            "flops_per_launch": flops_per_launch, "launches": sk["launches"] // steps,
            "algorithmic_bytes_per_launch": alg,
            "avg_launch_ms": per_launch_ms,
            "hbm_gbs_algorithmic": alg / (per_launch_ms * 1e-3) / 1e9,
            "hbm_frac_algorithmic": alg / (per_launch_ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
    panel = None
    if "panel" in kt:
        pk = kt["panel"]
        pms = pk["total_ms"] / steps
        launches = pk["launches"] // steps
        pf = panel_flops(n, b)
        us_col = pms * 1e3 / (n - 1)
        per_launch_ms = pk["total_ms"] / pk["launches"]
        achieved = (pf / launches) / (per_launch_ms * 1e-3) / 1e12
        panel = {"ms_per_step": pms, "us_per_column_step": us_col,
                 "alu_flops": pf, "alu_tflops": pf / (pms * 1e-3) / 1e12,
                 "alu_frac": pf / (pms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}
        ptraffic, ptraffic_src = measured_panel_traffic(n, b)
        palg = panel_bytes(n, b) / launches
        roofs["panel"] = {
            "kernel": f"panel_kernel<512,{panel_tpr(b)},65>", "bound": "alu",
            "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS, "traffic": ptraffic,
            "traffic_source": ptraffic_src,
            "traffic_over_algorithmic": (ptraffic / palg) if ptraffic else None,
            "algorithmic_bytes_per_launch": palg,
            "hbm_gbs_algorithmic": palg / (per_launch_ms * 1e-3) / 1e9,
            "flops_per_launch": pf / launches, "launches": launches,
            "avg_launch_ms": per_launch_ms,
            "latency": {"us_per_column_step": us_col, "budget_us_per_column_step": 2.0,
                        "note": "bound by the latency of the per-column pivot exchange "
                                "between workgroups, not by ALU or HBM"}}
    dom = max(roofs, key=lambda k: kt[k]["total_ms"]) if roofs else None
    roof = dict(roofs[dom], dominant_class_by_time=dom) if dom else None
    roof_other = {k: v for k, v in roofs.items() if k != dom}

    # CPU oracle: the whole factorization of the same matrix on this host,
    # which also gives the full-length checks of both precisions
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        nthr = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
        s_steps = n - 1 if args.cpu_steps <= 0 else min(args.cpu_steps, n - 1)
        log(f"[bench] oracle: {s_steps} of {n - 1} column steps, {nthr} threads")
        tt = time.time()
        ref = oracle.ltlt(A_np, max_steps=s_steps, nthreads=nthr)
        t_s = time.time() - tt
        del ref["X"]
        w_s = sum((n - k - 1) ** 2 for k in range(s_steps))
        w_all = sum((n - k - 1) ** 2 for k in range(n - 1))
        host = host_info()
        cpu = {"value": nominal * (w_s / w_all) / t_s / 1e9, "unit": "GFLOP/s", "cores": nthr,
               "kind": "oracle", "seconds": t_s, "host": host}
        if s_steps == n - 1:
            cpu["sample"] = (f"the whole factorization of the same n={n} matrix (all {n - 1} "
                             f"column steps), {t_s:.1f} s on {nthr} threads, GFLOP/s at the "
                             f"nominal n^3/3")
        else:
            cpu["sample"] = (f"first {s_steps} of {n - 1} column steps of the same n={n} matrix "
                             f"({t_s:.1f} s), scaled by their share (n-k-1)^2 of the work")
        log(f"[bench] oracle {cpu}")
        if s_steps == n - 1 and not args.no_check:
            la_o, sg_o = oracle.pfaffian(n, ref["t"], ref["ipiv"])
            c64 = compare_with_oracle(torch, Af64, t64, ipiv64, ref)
            c64["residual_exact"] = exact_residual(torch, A0, Af64, t64, ipiv64)
            c64["sign_equal_oracle"] = sign64 == sg_o
            c64["abs_dlog_pf_vs_oracle"] = abs(logpf64 - la_o)
            checks["fp64_vs_oracle"] = c64
            if fp32 is not None:
                fp32["sign_matches_oracle"] = fp32["sign"] == sg_o
                fp32["abs_dlog_pf_vs_oracle"] = abs(fp32["log_abs_pf"] - la_o)
                fp32["rel_dlog_pf_vs_oracle"] = abs(fp32["log_abs_pf"] - la_o) / max(1.0, abs(la_o))
                fp32["pivots_equal_oracle"] = bool(np.array_equal(fp32_ipiv, ref["ipiv"]))
                fp32["pivot_steps_equal_oracle"] = int(np.sum(fp32_ipiv == ref["ipiv"]))
            checks["oracle_pfaffian"] = {"sign": sg_o, "log_abs_pf": la_o}
            log(f"[bench] checks {checks}")
        elif s_steps < n - 1:
            checks["oracle_prefix_steps"] = s_steps
            checks["ipiv_prefix_equal_oracle"] = bool(np.array_equal(ipiv64[: s_steps + 1],
                                                                       ref["ipiv"][: s_steps + 1]))
        del ref
    elif not args.no_check:
        checks["residual_exact_fp64"] = exact_residual(torch, A0, Af64, t64, ipiv64)
    del Af64

    batched = None if args.no_batched else bench_batched(torch, binding, inputs, args.batch_count,
                                                         check=not args.no_check)
    serving = None if args.no_serving else bench_serving(
        torch, args.serving_count, args.serving_short, deadline=deadline)

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
        "roofline_other": roof_other,
        "step_ms": {"mean": ms, "median": float(np.median(step_ms)), "min": float(np.min(step_ms)),
                    "max": float(np.max(step_ms))},
        "panel": panel,
        "solve": solve,
        "pfaffian_partial": partial,
        "nopiv": nopiv,
        "n8192": n8192,
        "cpu_baseline": cpu,
        "kernels": kt,
        "fp32_update": fp32,
        "pfaffian_fp64": {"sign": sign64, "log_abs_pf": logpf64},
        "batched": batched,
        "serving": serving,
        "checks": checks,
        "elapsed_s": time.perf_counter() - t_start,
    }
    print(json.dumps(out), flush=True)
    # release the timing events and finish all device work before the
    # runtime's teardown at exit
    torch.cuda.synchronize()
    lib.skltlt_timing_release()


if __name__ == "__main__":
    main()
