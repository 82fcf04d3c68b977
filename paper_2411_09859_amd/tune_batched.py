"""Autotuner for the batched kernel: panel width per matrix order and
persistent workgroups per CU.

Two measurements per size class (HIP events, median of a few repetitions):
1. the panel width: a seeded batch of matrices of that class only, timed for
   every candidate pair (panel width, workgroups per CU); the width of the
   fastest pair applies to the matrices of that class;
2. the workgroups per CU: they apply to a whole batch, chosen by the batch's
   largest order (the host knows no more of a batch than its bound), so they
   are timed on a mixed batch whose orders spread evenly from 16 up to the
   class's upper end, each matrix at the compiled table's width.
(On a batch of [226, 256] alone three workgroups per CU beat four by 3 %;
on a batch spread over [16, 256], which a largest order of 256 also
describes, four beat three by 6 %.)
The result is written twice: ``tune_batched.json`` (the measurements) and
``csrc/batched_table.h`` (the compiled-in lookup used when block_size = 0).
Rebuild the library after tuning; if the widths changed, tune again so that
the second measurement sees them.

    python -m paper_2411_09859_amd.tune_batched [--count 4096]
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

from . import binding, inputs
from .batch import Arena

PKG = os.path.dirname(os.path.abspath(__file__))
CLASSES = [(16, 32), (34, 64), (66, 96), (98, 128), (130, 160), (162, 192), (194, 224), (226, 256)]
WIDTHS = [4, 6, 8, 10, 12, 14, 16]
WGPC = [1, 2, 3, 4]


def time_arena(torch, arena, bs, reps=3):
    ts = []
    for _ in range(reps + 1):
        arena.restore()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        arena.run(block_size=bs)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts[1:]))


def tune(count=4096, seed=7, verbose=True):
    import torch
    L = binding.lib()
    table = []
    meas = {}
    try:
        for lo, hi in CLASSES:
            # 1. panel width on a batch of this class only
            sizes, sing = inputs.batch_sizes(count, seed + lo, lo=lo, hi=hi,
                                             singular_fraction=0.0)
            arena = Arena(inputs.batch_matrices(sizes, sing, seed + lo))
            res = {}
            for g in WGPC:
                if L.skltlt_tune_batched_wgpc(g) != 0:
                    raise RuntimeError("skltlt_tune_batched_wgpc refused")
                for bs in WIDTHS:
                    res[f"{bs}x{g}"] = time_arena(torch, arena, bs)
            best = min(res, key=res.get)
            bs = int(best.split("x")[0])
            del arena
            # 2. workgroups per CU on a batch spread over [16, hi]
            sizes, sing = inputs.batch_sizes(count, seed + 1000 + hi, lo=16, hi=hi,
                                             singular_fraction=0.0)
            arena = Arena(inputs.batch_matrices(sizes, sing, seed + 1000 + hi))
            mixed = {}
            for g in WGPC:
                L.skltlt_tune_batched_wgpc(g)
                mixed[str(g)] = time_arena(torch, arena, 0)
            del arena
            g = int(min(mixed, key=mixed.get))
            meas[f"{lo}-{hi}"] = {"ms": res, "best_width": bs,
                                  "mixed_16_to_hi_ms_by_wgpc": mixed, "best_wgpc": g,
                                  "count": count}
            table.append((hi, bs, g))
            if verbose:
                print(f"[tune] n in [{lo},{hi}]: width {bs} ({res[best]:.3f} ms alone); "
                      f"batch over [16,{hi}]: {g} per CU {mixed[str(g)]:.3f} ms "
                      f"(4 per CU {mixed['4']:.3f} ms)", flush=True)
    finally:
        L.skltlt_tune_batched_wgpc(0)
    return table, meas


def write_outputs(table, meas, out_dir=None):
    jdir = out_dir or PKG
    hdir = out_dir or os.path.join(PKG, "csrc")
    with open(os.path.join(jdir, "tune_batched.json"), "w") as f:
        json.dump({"device": "MI355X (gfx950)", "classes": meas}, f, indent=1)
    lines = ["// Panel width of the batched kernel per matrix order and persistent",
             "// workgroups per CU per largest order of a batch, measured on MI355X by",
             "// paper_2411_09859_amd/tune_batched.py (written by the tuner).",
             "#pragma once",
             "namespace skl {",
             "struct BatchedTune { int n_max; int bs; int wgpc; };",
             "constexpr BatchedTune kBatchedTune[] = {"]
    lines += [f"    {{{hi}, {bs}, {g}}}," for hi, bs, g in table]
    lines += ["};", "}  // namespace skl", ""]
    with open(os.path.join(hdir, "batched_table.h"), "w") as f:
        f.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--no-write", action="store_true")
    ap.add_argument("--out-dir", default=None, help="write both files here instead")
    args = ap.parse_args()
    binding.lib()
    table, meas = tune(args.count)
    if not args.no_write:
        write_outputs(table, meas, args.out_dir)
    print(json.dumps({"table": table}))


if __name__ == "__main__":
    main()
