"""Autotuner for the panel width of the single-matrix factorization.

For each measured order it times skltlt_pfaffian (pivoted FP64 LTL^T plus the
Pfaffian) on a seeded N(0,1) skew matrix for every candidate panel width
(HIP events, median of a few repetitions, the input restored before each run
outside the timed region) and keeps the fastest.  Orders between two measured
ones use the width of the nearer one on a log scale.  The result is written
twice: ``tune_factor.json`` (the measurements) and ``csrc/factor_table.h``
(the compiled-in lookup behind skltlt_default_block_size).  Rebuild the
library after tuning.

    python -m paper_2411_09859_amd.tune_factor
"""
from __future__ import annotations

import argparse
import json
import math
import os

import numpy as np

from . import binding, inputs

PKG = os.path.dirname(os.path.abspath(__file__))
ORDERS = [256, 512, 1024, 2048, 4096, 8192, 16384]
CANDIDATES = [16, 32, 64, 128, 256]


def time_factor(torch, n, b, reps=3, seed=2):
    A0 = binding.to_device_colmajor(inputs.skew_normal(n, seed, full=False))
    Aw = torch.empty_like(A0)
    t = torch.zeros(max(n - 1, 1), dtype=torch.float64, device="cuda")
    ip = torch.zeros(n, dtype=torch.int32, device="cuda")
    la = torch.zeros(1, dtype=torch.float64, device="cuda")
    sg = torch.zeros(1, dtype=torch.int32, device="cuda")
    work = binding.alloc_workspace(binding.workspace_size(n, b, binding.FP64))
    ts = []
    for _ in range(reps + 1):
        Aw.copy_(A0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        binding.pfaffian(Aw, t, ip, la, sg, b, binding.FP64, work)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts[1:]))


def tune(orders=ORDERS, verbose=True):
    import torch
    meas = {}
    table = []
    for n in orders:
        res = {b: time_factor(torch, n, b) for b in CANDIDATES if b <= n // 2}
        best = min(res, key=res.get)
        meas[str(n)] = {"ms": res, "best": best}
        table.append((n, best))
        if verbose:
            print(f"[tune] n={n}: " + " ".join(f"b{b}={t:.2f}ms" for b, t in res.items())
                  + f" -> {best}", flush=True)
    return table, meas


def write_outputs(table, meas, out_dir=None):
    jdir = out_dir or PKG
    hdir = out_dir or os.path.join(PKG, "csrc")
    with open(os.path.join(jdir, "tune_factor.json"), "w") as f:
        json.dump({"device": "MI355X (gfx950)", "input": "N(0,1) skew, seed 2",
                   "orders": meas}, f, indent=1)
    # class boundaries at the geometric midpoints between measured orders
    rows = []
    for k, (n, b) in enumerate(table):
        hi = int(math.sqrt(n * table[k + 1][0])) if k + 1 < len(table) else 1 << 30
        rows.append((hi, b))
    lines = ["// Panel width of the single-matrix factorization per matrix order,",
             "// measured on MI355X by paper_2411_09859_amd/tune_factor.py (written by",
             "// the tuner): the first entry whose n_max is at least the order applies.",
             "#pragma once",
             "namespace skl {",
             "struct FactorTune { int n_max; int b; };",
             "constexpr FactorTune kFactorTune[] = {"]
    lines += [f"    {{{hi}, {b}}}," for hi, b in rows]
    lines += ["};", "}  // namespace skl", ""]
    with open(os.path.join(hdir, "factor_table.h"), "w") as f:
        f.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--no-write", action="store_true")
    ap.add_argument("--out-dir", default=None, help="write both files here instead")
    args = ap.parse_args()
    binding.lib()
    table, meas = tune()
    if not args.no_write:
        write_outputs(table, meas, args.out_dir)
    print(json.dumps({"table": table}))


if __name__ == "__main__":
    main()
