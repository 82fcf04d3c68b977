"""Summaries of rocprofv3 output for the kernels of this library.

Subcommands:

  copy --mib M
      A calibration program: one elementwise pass (torch.neg) over M MiB of
      fp64, so that each dispatch reads M MiB and writes M MiB.  Run it under
      ``rocprofv3 --pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE`` to learn what
      those counters read for a known number of bytes.

  stats --dir D --cmd "..." --out F
      Writes the per-kernel table of a ``rocprofv3 --kernel-trace --stats -f
      csv`` run found under D (its ``*kernel_stats.csv``).

  counters --dir D --kernel REGEX --counters C1,C2,... --source FILE[,FILE...]
           --workload W --cmd "..." --out F [--cus N] [--algo-flops F]
      Per-launch means of SQ/GRBM counters of one ``rocprofv3 --pmc`` run for
      the kernels matching REGEX, the MFMA busy fraction and the F64 MFMA
      operations as flops when those counters are present.

  traffic --fetch D1 --write D2 --calib-fetch D3 --calib-write D4 --mib M
          --kernel REGEX --source FILE[,FILE...] --algo-bytes B --cmd "..." --out F
      Per-launch HBM traffic of the kernels matching REGEX from two counter
      runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by the
      factor (known bytes / counter reading) of the calibration runs, with the
      SHA-256 of the kernel's source files (concatenated, in the order given)
      so a reader can tell when the figure no longer describes the kernel.  The output is ``key: value`` text.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import sys


def _find(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits


def counter_per_dispatch(d, counter, kernel_re):
    """{dispatch id: (kernel name, summed value)} of ``counter`` for the
    dispatches whose kernel name matches ``kernel_re``."""
    pat = re.compile(kernel_re)
    out = {}
    for path in _find(d, "counter_collection.csv"):
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                name = row.get("Kernel_Name", "")
                if not pat.search(name):
                    continue
                key = (path, row.get("Dispatch_Id"))
                val = float(row.get("Counter_Value", 0) or 0)
                prev = out.get(key)
                out[key] = (name, val + (prev[1] if prev else 0.0))
    return out


def sha256_of(paths):
    """SHA-256 of the files (a path, or comma-separated paths) concatenated."""
    h = hashlib.sha256()
    for path in str(paths).split(","):
        with open(path.strip(), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def read_summary(path):
    """``key: value`` lines of a summary file (comments and others skipped)."""
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    return vals


def cmd_copy(args):
    import torch
    n = args.mib * (1 << 20) // 8
    x = torch.randn(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(args.reps):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(f"copy: {args.reps} passes of {args.mib} MiB read + {args.mib} MiB written", flush=True)


def cmd_stats(args):
    path = _find(args.dir, "kernel_stats.csv")[0]
    with open(path, newline="") as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: -float(r.get("TotalDurationNs", 0) or 0))
    lines = [f"# {args.title}", f"# command: {args.cmd}", "#",
             f"{'calls':>7} {'total_ms':>10} {'avg_us':>10} {'min_us':>9} {'max_us':>9} {'pct':>6}  kernel"]
    for r in rows[: args.top]:
        lines.append(f"{int(r['Calls']):7d} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                     f"{float(r['AverageNs']) / 1e3:10.2f} {float(r['MinNs']) / 1e3:9.2f} "
                     f"{float(r['MaxNs']) / 1e3:9.2f} {float(r['Percentage']):6.2f}  {r['Name'][:150]}")
    txt = "\n".join(lines) + "\n"
    with open(args.out, "w") as f:
        f.write(txt)
    sys.stdout.write(txt)


def cmd_traffic(args):
    known = args.mib * (1 << 20)
    cf = counter_per_dispatch(args.calib_fetch, "FETCH_SIZE", args.calib_kernel)
    cw = counter_per_dispatch(args.calib_write, "WRITE_SIZE", args.calib_kernel)
    if not cf or not cw:
        raise SystemExit("calibration dispatches not found")
    # the median reading over the passes
    cf_kib = sorted(v for _, v in cf.values())[len(cf) // 2]
    cw_kib = sorted(v for _, v in cw.values())[len(cw) // 2]
    f_fac = known / (cf_kib * 1024.0)
    w_fac = known / (cw_kib * 1024.0)
    kf = counter_per_dispatch(args.fetch, "FETCH_SIZE", args.kernel)
    kw = counter_per_dispatch(args.write, "WRITE_SIZE", args.kernel)
    if not kf or not kw:
        raise SystemExit("kernel dispatches not found")
    nf, nw = len(kf), len(kw)
    fetch_b = sum(v for _, v in kf.values()) * 1024.0 * f_fac / nf
    write_b = sum(v for _, v in kw.values()) * 1024.0 * w_fac / nw
    tot = fetch_b + write_b
    lines = [f"# {args.title}",
             f"# fetch run:  {args.cmd_fetch}",
             f"# write run:  {args.cmd_write}",
             f"# calibration: {args.cmd_calib} (FETCH_SIZE and WRITE_SIZE runs)",
             f"workload: {args.workload}",
             f"kernel_regex: {args.kernel}",
             f"source: {args.source}",
             f"source_sha256: {sha256_of(args.source)}",
             f"launches_fetch_run: {nf}",
             f"launches_write_run: {nw}",
             f"calib_bytes_each_way: {known}",
             f"calib_fetch_kib: {cf_kib:.1f}",
             f"calib_write_kib: {cw_kib:.1f}",
             f"calib_factor_fetch: {f_fac:.4f}",
             f"calib_factor_write: {w_fac:.4f}",
             f"fetch_bytes_per_launch: {fetch_b:.6e}",
             f"write_bytes_per_launch: {write_b:.6e}",
             f"traffic_bytes_per_launch: {tot:.6e}",
             f"algorithmic_bytes_per_launch: {args.algo_bytes:.6e}",
             f"traffic_over_algorithmic: {tot / args.algo_bytes:.4f}"]
    txt = "\n".join(lines) + "\n"
    with open(args.out, "w") as f:
        f.write(txt)
    sys.stdout.write(txt)


def cmd_counters(args):
    """Per-launch means of SQ/GRBM counters for the kernels matching REGEX,
    with the MFMA busy fraction and the F64 MFMA operations as flops (the
    counter counts units of 512 flops) beside the algorithmic flops per
    launch.  GRBM_GUI_ACTIVE of a dispatch is summed over the XCDs (each has
    its own GRBM), so one XCD's active cycles are the value over the XCD
    count, and the busy fraction is the MFMA busy cycles (summed over all
    SIMDs) over those cycles times CUs times 4 SIMDs."""
    names = [c.strip() for c in args.counters.split(",") if c.strip()]
    per = {c: counter_per_dispatch(args.dir, c, args.kernel) for c in names}
    nl = max((len(v) for v in per.values()), default=0)
    if nl == 0:
        raise SystemExit("kernel dispatches not found")
    mean = {c: (sum(x for _, x in v.values()) / len(v) if v else float("nan"))
            for c, v in per.items()}
    lines = [f"# {args.title}", f"# command: {args.cmd}",
             f"workload: {args.workload}", f"kernel_regex: {args.kernel}",
             f"source: {args.source}", f"source_sha256: {sha256_of(args.source)}",
             f"launches: {nl}"]
    for c in names:
        lines.append(f"{c}_per_launch: {mean[c]:.6e}")
    if "SQ_VALU_MFMA_BUSY_CYCLES" in mean and "GRBM_GUI_ACTIVE" in mean:
        act = mean["GRBM_GUI_ACTIVE"] / args.xcds
        busy = mean["SQ_VALU_MFMA_BUSY_CYCLES"] / (act * args.cus * 4)
        lines.append(f"active_cycles_per_launch_one_xcd: {act:.6e}")
        lines.append(f"mfma_busy_fraction: {busy:.4f}")
        if "SQ_BUSY_CU_CYCLES" in mean:
            lines.append(f"cu_busy_fraction: {mean['SQ_BUSY_CU_CYCLES'] / (act * args.cus):.4f}")
    if "SQ_INSTS_VALU_MFMA_MOPS_F64" in mean:
        fl = mean["SQ_INSTS_VALU_MFMA_MOPS_F64"] * 512.0
        lines.append(f"mfma_f64_flops_per_launch: {fl:.6e}")
        if args.algo_flops:
            lines.append(f"algorithmic_flops_per_launch: {args.algo_flops:.6e}")
            lines.append(f"mfma_flops_over_algorithmic: {fl / args.algo_flops:.4f}")
    if "SQ_LDS_BANK_CONFLICT" in mean and "SQ_INSTS_LDS" in mean and mean["SQ_INSTS_LDS"]:
        lines.append(f"lds_bank_conflict_cycles_per_lds_instruction: "
                     f"{mean['SQ_LDS_BANK_CONFLICT'] / mean['SQ_INSTS_LDS']:.4f}")
    txt = "\n".join(lines) + "\n"
    with open(args.out, "w") as f:
        f.write(txt)
    sys.stdout.write(txt)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="sub", required=True)
    a = sub.add_parser("copy")
    a.add_argument("--mib", type=int, default=1024)
    a.add_argument("--reps", type=int, default=3)
    a = sub.add_parser("stats")
    a.add_argument("--dir", required=True)
    a.add_argument("--cmd", required=True)
    a.add_argument("--title", default="rocprofv3 kernel statistics")
    a.add_argument("--top", type=int, default=25)
    a.add_argument("--out", required=True)
    a = sub.add_parser("counters")
    a.add_argument("--dir", required=True)
    a.add_argument("--kernel", required=True)
    a.add_argument("--counters", required=True)
    a.add_argument("--cus", type=int, default=256)
    a.add_argument("--xcds", type=int, default=8)
    a.add_argument("--algo-flops", type=float, default=0.0)
    a.add_argument("--source", required=True)
    a.add_argument("--workload", required=True)
    a.add_argument("--cmd", required=True)
    a.add_argument("--title", default="rocprofv3 counters")
    a.add_argument("--out", required=True)
    a = sub.add_parser("traffic")
    for k in ("fetch", "write", "calib_fetch", "calib_write"):
        a.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    a.add_argument("--mib", type=int, required=True)
    a.add_argument("--kernel", required=True)
    a.add_argument("--calib-kernel", default="neg")
    a.add_argument("--source", required=True)
    a.add_argument("--algo-bytes", type=float, required=True)
    a.add_argument("--cmd-fetch", required=True)
    a.add_argument("--cmd-write", required=True)
    a.add_argument("--cmd-calib", required=True)
    a.add_argument("--title", default="HBM traffic per launch")
    a.add_argument("--workload", required=True, help='e.g. "n=16384 b=256"')
    a.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    {"copy": cmd_copy, "stats": cmd_stats, "traffic": cmd_traffic,
     "counters": cmd_counters}[args.sub](args)


if __name__ == "__main__":
    main()
