"""Autotuner for the batched kernel: panel width per matrix order and
persistent workgroups per CU.

For each size class it times skltlt_batched on a seeded batch of that class
for every candidate pair (panel width, workgroups per CU) (HIP events, median
of a few repetitions) and keeps the fastest.  The width applies to the
matrices of that class; the workgroups per CU to batches whose largest order
falls in the class.  The result is written twice: ``tune_batched.json`` (the
measurements) and ``csrc/batched_table.h`` (the compiled-in lookup used when
block_size = 0).  Rebuild the library after tuning.

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
            sizes, sing = inputs.batch_sizes(count, seed + lo, lo=lo, hi=hi,
                                             singular_fraction=0.0)
            mats = inputs.batch_matrices(sizes, sing, seed + lo)
            arena = Arena(mats)
            res = {}
            for g in WGPC:
                if L.skltlt_tune_batched_wgpc(g) != 0:
                    raise RuntimeError("skltlt_tune_batched_wgpc refused")
                for bs in WIDTHS:
                    res[f"{bs}x{g}"] = time_arena(torch, arena, bs)
            best = min(res, key=res.get)
            bs, g = (int(x) for x in best.split("x"))
            meas[f"{lo}-{hi}"] = {"ms": res, "best": {"width": bs, "wgpc": g}, "count": count}
            table.append((hi, bs, g))
            if verbose:
                print(f"[tune] n in [{lo},{hi}]: best width {bs} x {g} per CU "
                      f"{res[best]:.3f} ms; width 16 x 4: {res['16x4']:.3f} ms", flush=True)
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
