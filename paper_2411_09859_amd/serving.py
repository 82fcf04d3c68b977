"""Continuous-batching server for Pfaffian / factorization requests.

Requests of uneven order arrive over time.  The scheduler admits them in
arrival order while the device-memory budget allows (back-pressure when it is
full), keeps every admitted request's matrix and factors on the device, and
overlaps their work on the GPU:

* small requests (n <= ``small_n``) are collected and factored together by
  one ``skltlt_batched`` launch, in FP64 whatever their tag (the batched
  kernel runs FP64 only; FP64 is at least as accurate as the FP32-update
  variant asked for, and at these orders the update is a small share of the
  work); requests admitted while a batch runs join the next batch, which
  starts as soon as the batch stream is free;
* the others run alone, each on the stream of a pool with the least queued
  work, in the precision their tag asks for: a factorization request by ``skltlt_pfaffian`` (its
  factors are handed back on the device), a Pfaffian request by
  ``skltlt_pfaffian_partial`` (half the pivot steps, nothing but the
  Pfaffian).

Each result records the precision it was computed in (``precision_used``).
A batched member the library rejects (``info != 0``) comes back as an error.

Completion is detected by polling HIP events, never by blocking the device.
Latency is measured from a request's arrival to the host observing its
completion.  The executor is pluggable: ``GpuExecutor`` drives the library,
``FakeExecutor`` runs the same scheduling logic on the CPU (tests of
admission, back-pressure, failure handling and latency accounting).

A request's result does not depend on which other requests share the GPU or
its batch: the batched kernel and the blocked factorization compute each
matrix independently and deterministically.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    n: int
    precision: int = 0            # 0 FP64, 1 FP32 update
    arrival: float = 0.0          # seconds on the server clock
    seed: int = 0                 # for device-side generation of the input
    matrix: Optional[np.ndarray] = None  # host input (strict lower used), optional
    factor: bool = False          # factorization request: the factors (A, t, ipiv)
                                  # come back on the device; else Pfaffian only


@dataclasses.dataclass
class Result:
    rid: int
    n: int
    log_abs_pf: float
    sign: int
    arrival: float
    admitted: float
    done: float
    path: str
    error: Optional[str] = None
    factors: object = None
    precision: int = 0          # the request's tag
    precision_used: int = 0     # the precision it was computed in

    @property
    def latency(self):
        return self.done - self.arrival


def request_bytes(n: int, precision: int = 0) -> int:
    """Device bytes a request holds while admitted (matrix, t, ipiv, work)."""
    from . import binding
    b = binding.default_block_size(max(n, 1))
    ws = binding.workspace_size(max(n, 1), b, precision) if n > 256 else 0
    return 8 * n * n + 16 * n + ws + 4096


class FakeExecutor:
    """CPU stand-in: a request 'runs' for a modelled time and its Pfaffian is
    computed by a supplied function (e.g. the oracle).  Same interface as the
    GPU executor."""

    def __init__(self, clock: Callable[[], float], duration: Callable[[Request], float],
                 pf: Optional[Callable[[Request], tuple]] = None,
                 fail: Optional[Callable[[Request], bool]] = None, bytes_of=None):
        self.clock = clock
        self.duration = duration
        self.pf = pf
        self.fail = fail
        self.inflight = []
        self.bytes_of = bytes_of or (lambda r: 8 * r.n * r.n + 4096)

    def nbytes(self, req):
        return self.bytes_of(req)

    def launch_batch(self, reqs):
        t = self.clock()
        end = t + sum(self.duration(r) for r in reqs) / max(len(reqs), 1)
        self.inflight.append((end, reqs, "batched"))

    def launch_single(self, req):
        self.inflight.append((self.clock() + self.duration(req), [req], "single"))

    def batch_busy(self):
        return any(p == "batched" for _, _, p in self.inflight)

    def poll(self):
        now = self.clock()
        done, keep = [], []
        for item in self.inflight:
            (done if item[0] <= now else keep).append(item)
        self.inflight = keep
        out = []
        for _, reqs, path in done:
            for r in reqs:
                used = 0 if path == "batched" else r.precision
                if self.fail and self.fail(r):
                    out.append((r, float("nan"), 0, path, "device error", None, used))
                    continue
                la, sg = self.pf(r) if self.pf else (0.0, 1)
                out.append((r, la, sg, path, None, None, used))
        return out

    def idle(self):
        return not self.inflight


class GpuExecutor:
    """Drives libskltlt on cuda:0: one batch stream, a pool of streams."""

    def __init__(self, n_streams: int = 4, small_n: int = 256, device="cuda",
                 policy: str = "least_loaded"):
        if policy not in ("least_loaded", "round_robin"):
            raise ValueError(f"unknown stream policy {policy!r}")
        import torch
        from . import binding
        self.torch = torch
        self.binding = binding
        self.device = device
        self.small_n = small_n
        self.batch_stream = torch.cuda.Stream(device=device)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        self.policy = policy
        self.next_stream = 0
        # work queued on each stream and not yet seen complete, in units of
        # the order n (a single request's time grows about linearly with n at
        # these orders: its column steps)
        self.load = [0] * n_streams
        self.inflight = []  # (event, payload)

    def _pick_stream(self, n):
        """Round robin, or the stream with the least queued work (ties go to
        the next stream in round-robin order, so an idle pool is used in
        turn).  Under load, round robin queues a long request ahead of short
        ones on one stream while another idles."""
        ns = len(self.streams)
        if self.policy == "round_robin":
            k = self.next_stream
        else:
            order = [(self.next_stream + i) % ns for i in range(ns)]
            k = min(order, key=lambda q: self.load[q])
        self.next_stream = (k + 1) % ns
        self.load[k] += n
        return k

    def nbytes(self, req):
        return request_bytes(req.n, req.precision)

    def _materialize(self, req, stream):
        """Device input for a request: the host matrix if given, else seeded
        N(0,1) entries drawn on the device (only the strict lower triangle is
        read by the library)."""
        torch = self.torch
        n = req.n
        with torch.cuda.stream(stream):
            if req.matrix is not None:
                host = torch.from_numpy(np.asfortranarray(req.matrix, dtype=np.float64))
                dev = torch.empty_strided((n, n), (1, max(n, 1)), dtype=torch.float64,
                                          device=self.device)
                dev.copy_(host, non_blocking=False)
            else:
                g = torch.Generator(device=self.device)
                g.manual_seed(int(req.seed))
                dev = torch.randn((n, n), generator=g, dtype=torch.float64,
                                  device=self.device).t()  # column-major view
        return dev

    def launch_batch(self, reqs):
        torch, binding = self.torch, self.binding
        s = self.batch_stream
        with torch.cuda.stream(s):
            mats = [self._materialize(r, s) for r in reqs]
            ns = [r.n for r in reqs]
            ts = [torch.empty(max(n - 1, 1), dtype=torch.float64, device=self.device) for n in ns]
            ps = [torch.empty(max(n, 1), dtype=torch.int32, device=self.device) for n in ns]
            # the descriptor arrays go up in one asynchronous copy from pinned
            # memory (a device tensor built from a Python list is a blocking
            # pageable copy that waits for the GPU)
            k = len(reqs)
            desc_h = torch.empty(5 * k, dtype=torch.int64, pin_memory=True)
            desc_h[0:k] = torch.tensor(ns, dtype=torch.int64)
            desc_h[k:2 * k] = torch.tensor([max(n, 1) for n in ns], dtype=torch.int64)
            desc_h[2 * k:3 * k] = torch.tensor([m.data_ptr() for m in mats], dtype=torch.int64)
            desc_h[3 * k:4 * k] = torch.tensor([t.data_ptr() for t in ts], dtype=torch.int64)
            desc_h[4 * k:5 * k] = torch.tensor([p.data_ptr() for p in ps], dtype=torch.int64)
            desc = desc_h.to(self.device, non_blocking=True)
            n_dev = desc[0:k].to(torch.int32)
            lda = desc[k:2 * k].to(torch.int32)
            A_ptr, t_ptr, p_ptr = desc[2 * k:3 * k], desc[3 * k:4 * k], desc[4 * k:5 * k]
            la = torch.empty(len(reqs), dtype=torch.float64, device=self.device)
            sg = torch.empty(len(reqs), dtype=torch.int32, device=self.device)
            info = torch.empty(len(reqs), dtype=torch.int32, device=self.device)
            work = binding.alloc_workspace(binding.batched_workspace_size(len(reqs)), self.device)
            binding.batched(n_dev, A_ptr, lda, t_ptr, p_ptr, la, sg, info, max(ns), 0,
                            binding.FP64, work, s)
            la_h = torch.empty(len(reqs), dtype=torch.float64, pin_memory=True)
            sg_h = torch.empty(len(reqs), dtype=torch.int32, pin_memory=True)
            in_h = torch.empty(len(reqs), dtype=torch.int32, pin_memory=True)
            la_h.copy_(la, non_blocking=True)
            sg_h.copy_(sg, non_blocking=True)
            in_h.copy_(info, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        keep = (mats, ts, ps, desc_h, desc, n_dev, lda, A_ptr, t_ptr, p_ptr, la, sg, info, work)
        facs = [(mats[k], ts[k], ps[k]) if r.factor else None for k, r in enumerate(reqs)]
        self.inflight.append((ev, ("batched", reqs, la_h, sg_h, keep, facs, in_h)))

    def launch_single(self, req):
        torch, binding = self.torch, self.binding
        k = self._pick_stream(req.n)
        s = self.streams[k]
        with torch.cuda.stream(s):
            A = self._materialize(req, s)
            n = req.n
            t = torch.empty(max(n - 1, 1), dtype=torch.float64, device=self.device)
            ip = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
            la = torch.empty(1, dtype=torch.float64, device=self.device)
            sg = torch.empty(1, dtype=torch.int32, device=self.device)
            work = binding.alloc_workspace(
                binding.workspace_size(max(n, 1), 0, req.precision), self.device)
            if req.factor:
                binding.pfaffian(A, t, ip, la, sg, 0, req.precision, work, s)
            else:
                binding.pfaffian_partial(A, t, ip, la, sg, 0, req.precision, work, s)
            la_h = torch.empty(1, dtype=torch.float64, pin_memory=True)
            sg_h = torch.empty(1, dtype=torch.int32, pin_memory=True)
            la_h.copy_(la, non_blocking=True)
            sg_h.copy_(sg, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        path = "single" if req.factor else "partial"
        facs = [(A, t, ip)] if req.factor else [None]
        self.inflight.append((ev, (path, [req], la_h, sg_h, (A, t, ip, la, sg, work, k), facs,
                                   None)))

    def batch_busy(self):
        return any(p[0] == "batched" for _, p in self.inflight)

    def poll(self):
        out, keep = [], []
        for ev, payload in self.inflight:
            if ev.query():
                path, reqs, la_h, sg_h, bufs, facs, in_h = payload
                if path != "batched":
                    self.load[bufs[-1]] -= reqs[0].n
                for k, r in enumerate(reqs):
                    err = None
                    if in_h is not None and int(in_h[k]) != 0:
                        err = f"rejected by the batched kernel (info {int(in_h[k])})"
                    used = 0 if path == "batched" else r.precision
                    out.append((r, float(la_h[k]), int(sg_h[k]), path, err, facs[k], used))
            else:
                keep.append((ev, payload))
        self.inflight = keep
        return out

    def idle(self):
        return not self.inflight


class Server:
    """Admission by memory budget, continuous batching, latency accounting."""

    def __init__(self, executor, budget_bytes: int = 64 << 30, small_n: int = 256,
                 max_batch: int = 4096, max_inflight_single: int = 64,
                 clock: Callable[[], float] = time.perf_counter, keep_factors: bool = True):
        self.ex = executor
        # keep_factors=False: a factorization request's device factors are
        # released when it completes (a client that reads only the Pfaffian;
        # otherwise every completed request would keep its matrix on the
        # device for as long as its result is held)
        self.keep_factors = keep_factors
        self.budget = budget_bytes
        self.small_n = small_n
        self.max_batch = max_batch
        self.max_inflight_single = max_inflight_single
        self.clock = clock
        self.used = 0
        self.peak_used = 0
        self.waiting = collections.deque()   # arrived, not admitted (FIFO)
        self.pending_small = []              # admitted, waiting for the next batch
        self.inflight_single = 0
        self.held = {}                       # rid -> bytes held
        self.admit_time = {}
        self.results = []
        self.rejected = []

    def submit(self, req: Request):
        if req.n < 0 or req.n > 1 << 16:
            self.rejected.append((req, "invalid order"))
            return
        if req.matrix is not None and not np.all(np.isfinite(np.tril(req.matrix, -1))):
            self.rejected.append((req, "non-finite input"))
            return
        if self.ex.nbytes(req) > self.budget:
            self.rejected.append((req, "larger than the memory budget"))
            return
        self.waiting.append(req)

    def _admit(self):
        now = self.clock()
        while self.waiting:
            r = self.waiting[0]
            need = self.ex.nbytes(r)
            small = r.n <= self.small_n
            if self.used + need > self.budget:
                break  # back-pressure: FIFO, no overtaking
            if not small and self.inflight_single >= self.max_inflight_single:
                break
            self.waiting.popleft()
            self.used += need
            self.peak_used = max(self.peak_used, self.used)
            self.held[r.rid] = need
            self.admit_time[r.rid] = now
            if small:
                self.pending_small.append(r)
            else:
                self.inflight_single += 1
                self.ex.launch_single(r)

    def _launch_batch(self):
        if self.pending_small and not self.ex.batch_busy():
            reqs = self.pending_small[: self.max_batch]
            self.pending_small = self.pending_small[self.max_batch:]
            self.ex.launch_batch(reqs)

    def _collect(self):
        now = self.clock()
        for r, la, sg, path, err, facs, used in self.ex.poll():
            self.used -= self.held.pop(r.rid)
            if path != "batched":
                self.inflight_single -= 1
            self.results.append(Result(r.rid, r.n, la, sg, r.arrival,
                                       self.admit_time.pop(r.rid), now, path, err,
                                       facs if self.keep_factors else None,
                                       r.precision, used))

    def tick(self):
        self._collect()
        self._admit()
        self._launch_batch()

    def busy(self):
        return bool(self.waiting or self.pending_small or not self.ex.idle())

    def run(self, requests, sleep_s: float = 20e-6, time_limit_s: float = 3600.0):
        """Replay ``requests`` (sorted by arrival, seconds from start) in real
        time and return the results."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        i = 0
        while i < len(reqs) or self.busy():
            now = self.clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                r = reqs[i]
                r.arrival = t0 + r.arrival
                self.submit(r)
                i += 1
            self.tick()
            if now > time_limit_s:
                raise TimeoutError("serving run exceeded its time limit")
            if i < len(reqs) and not self.busy():
                wait = reqs[i].arrival - (self.clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
            elif sleep_s:
                time.sleep(sleep_s)
        return self.results


def summarize(results, wall_s: float):
    ok = [r for r in results if r.error is None]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    return {
        "requests": len(results),
        "errors": len(results) - len(ok),
        "solves_per_s": len(ok) / wall_s if wall_s > 0 else 0.0,
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "batched_fraction": float(np.mean([r.path == "batched" for r in ok])) if ok else 0.0,
        "partial_fraction": float(np.mean([r.path == "partial" for r in ok])) if ok else 0.0,
        "by_tag": {tag: {"requests": sum(r.precision == p for r in results),
                         "computed_fp64": sum(r.precision == p and r.precision_used == 0
                                              for r in ok),
                         "computed_fp32_update": sum(r.precision == p and r.precision_used == 1
                                                     for r in ok)}
                   for tag, p in (("fp64", 0), ("fp32_update", 1))},
    }


def make_requests(count: int, seed: int, rate_per_s: float, lo=32, hi=2048, p_fp32=0.5,
                  p_factor=0.5):
    sizes, prec, arrivals, seeds, kinds = __import__(
        "paper_2411_09859_amd.inputs", fromlist=["serving_requests"]).serving_requests(
        count, seed, rate_per_s, lo, hi, p_fp32, p_factor)
    return [Request(rid=k, n=int(sizes[k]), precision=int(prec[k]), arrival=float(arrivals[k]),
                    seed=int(seeds[k]), factor=bool(kinds[k])) for k in range(count)]
