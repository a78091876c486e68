"""Summaries of rocprofv3 output for profiles/ and for bench.py's traffic field.

    python -m paper_1001_5460_amd.rocprof_summary trace  OUT.md  TRACE.csv  --cmd "..." [--title ...]
    python -m paper_1001_5460_amd.rocprof_summary counters OUT.md OUT.json --run NAME=COUNTERS.csv ...
        [--calib-fetch CSV --calib-write CSV] [--kernels bench-name=symbol-substring ...] --cmd "..."

`trace` reads a `*_kernel_trace.csv` (rocprofv3 --kernel-trace --output-format csv) and writes
per-kernel launch counts and average durations.  `counters` reads `*_counter_collection.csv`
files (rocprofv3 --pmc ... --output-format csv), averages each counter per kernel over the
active dispatches, and derives

* HBM-side traffic from FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by what the
  same counter reads for the library's plain FP32 copy kernel of known size (--calib-*);
* MFMA work from SQ_INSTS_VALU_MFMA_MOPS_BF16 (units of 512 flops per count) over the kernel's
  duration, as a fraction of the BF16 dense peak, and the MFMA-busy share
  SQ_VALU_MFMA_BUSY_CYCLES / (4 SIMDs x SQ_BUSY_CU_CYCLES);
* DRAM reads from TCC_EA0_RDREQ_DRAM, in bytes per request measured on the same copy kernel
  (--calib-dram: bytes the copy reads / its requests), wave stall share
  SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES and LDS bank-conflict cycles per LDS instruction.

A dispatch is active when its duration (or, without timestamps, its first counter) is at least a
tenth of the kernel's 90th-percentile value: launches enqueued past a solve's convergence exit at
once on the device-side flag and are left out, as bench.py's tracer does.
"""
import argparse
import collections
import csv
import json
import os
import sys

BF16_PEAK_TFLOPS = 2500.0


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _active(values):
    if not values:
        return []
    s = sorted(values)
    cut = 0.1 * s[(len(s) - 1) * 9 // 10]
    return [v for v in values if v >= cut]


def trace(args):
    rows = _rows(args.trace)
    dur = collections.defaultdict(list)
    for r in rows:
        name = r.get("Kernel_Name") or r.get("Name")
        try:
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        except (KeyError, ValueError):
            continue
        dur[name].append(d)
    out = [f"# {args.title}", "", "Command (GPU box, repo root = $R):", "", "```", args.cmd, "```", "",
           "Average over active launches (those of at least a tenth of the kernel's 90th-percentile "
           "duration; launches enqueued past a converged solve exit at once).", "",
           "| kernel | launches | active | avg active us | total ms |", "|---|---:|---:|---:|---:|"]
    for name, d in sorted(dur.items(), key=lambda kv: -sum(kv[1])):
        a = _active(d)
        out.append(f"| `{name[:110]}` | {len(d)} | {len(a)} | {sum(a) / max(len(a), 1):.1f} | "
                   f"{sum(d) / 1e3:.3f} |")
    with open(args.out, "w") as f:
        f.write("\n".join(out) + "\n")


def _per_kernel(path):
    """{kernel: {counter: [value per dispatch]}, "_dur": {kernel: [us per dispatch]}}"""
    per = collections.defaultdict(lambda: collections.defaultdict(dict))
    for r in _rows(path):
        k = r.get("Kernel_Name")
        disp = r.get("Dispatch_Id") or r.get("Correlation_Id")
        c = r.get("Counter_Name")
        try:
            v = float(r.get("Counter_Value"))
        except (TypeError, ValueError):
            continue
        per[k][disp][c] = per[k][disp].get(c, 0.0) + v
        try:
            per[k][disp]["_us"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        except (KeyError, ValueError):
            pass
    return per


def _avg_active(disp, counter):
    vals = [(d.get("_us", 0.0), d[counter]) for d in disp.values() if counter in d]
    if not vals:
        return None, 0, None
    key = [u for u, _ in vals] if any(u > 0 for u, _ in vals) else [v for _, v in vals]
    cut = 0.1 * sorted(key)[(len(key) - 1) * 9 // 10]
    act = [(u, v) for (u, v), kk in zip(vals, key) if kk >= cut]
    n = len(act)
    return sum(v for _, v in act) / n, n, (sum(u for u, _ in act) / n if n else None)


def counters(args):
    runs = {}
    for spec in args.run:
        name, path = spec.split("=", 1)
        runs[name] = _per_kernel(path)
    scale = {"FETCH_SIZE": 1.0, "WRITE_SIZE": 1.0}
    calib = {}
    if args.calib_fetch and args.calib_write:
        for ctr, path in (("FETCH_SIZE", args.calib_fetch), ("WRITE_SIZE", args.calib_write)):
            per = _per_kernel(path)
            copy = [k for k in per if "k_cast<float, float>" in k]
            if not copy:
                raise SystemExit(f"no copy kernel in {path}")
            kib, n, _ = _avg_active(per[copy[0]], ctr)
            calib[ctr] = kib
            scale[ctr] = (args.calib_bytes / 1024.0) / kib
    dram_req = None
    if args.calib_dram:
        per = _per_kernel(args.calib_dram)
        copy = [k for k in per if "k_cast<float, float>" in k]
        if not copy:
            raise SystemExit(f"no copy kernel in {args.calib_dram}")
        req, n, _ = _avg_active(per[copy[0]], "TCC_EA0_RDREQ_DRAM")
        dram_req = args.calib_bytes / req
        calib["TCC_EA0_RDREQ_DRAM"] = req
    wanted = dict(s.split("=", 1) for s in args.kernels)
    summary = {}
    for bench_name, sub in wanted.items():
        row = {"symbol": None}
        for rname, per in runs.items():
            match = [k for k in per if sub in k]
            if not match:
                continue
            k = max(match, key=lambda kk: len(per[kk]))
            row["symbol"] = k
            for ctr in sorted({c for d in per[k].values() for c in d if c != "_us"}):
                v, n, us = _avg_active(per[k], ctr)
                row[ctr] = v
                row["active_dispatches"] = max(row.get("active_dispatches", 0), n)
                if us:
                    row.setdefault("avg_us", us)
        if "FETCH_SIZE" in row:
            row["fetch_bytes_per_launch"] = int(row["FETCH_SIZE"] * 1024 * scale["FETCH_SIZE"])
        if "WRITE_SIZE" in row:
            row["write_bytes_per_launch"] = int(row["WRITE_SIZE"] * 1024 * scale["WRITE_SIZE"])
        if "fetch_bytes_per_launch" in row and "write_bytes_per_launch" in row:
            row["traffic_bytes_per_launch"] = row["fetch_bytes_per_launch"] + row["write_bytes_per_launch"]
        if row.get("SQ_INSTS_VALU_MFMA_MOPS_BF16") is not None and row.get("avg_us"):
            fl = row["SQ_INSTS_VALU_MFMA_MOPS_BF16"] * 512.0
            row["mfma_bf16_tflops"] = fl / (row["avg_us"] * 1e-6) / 1e12
            row["mfma_frac_of_bf16_peak"] = row["mfma_bf16_tflops"] / BF16_PEAK_TFLOPS
        if row.get("SQ_VALU_MFMA_BUSY_CYCLES") is not None and row.get("SQ_BUSY_CU_CYCLES"):
            row["mfma_busy_share"] = row["SQ_VALU_MFMA_BUSY_CYCLES"] / (4.0 * row["SQ_BUSY_CU_CYCLES"])
        if row.get("SQ_WAIT_INST_ANY") is not None and row.get("SQ_WAVE_CYCLES"):
            row["wait_share"] = row["SQ_WAIT_INST_ANY"] / row["SQ_WAVE_CYCLES"]
        if row.get("SQ_LDS_BANK_CONFLICT") is not None and row.get("SQ_INSTS_LDS"):
            row["lds_conflict_cycles_per_instr"] = row["SQ_LDS_BANK_CONFLICT"] / row["SQ_INSTS_LDS"]
        if row.get("TCC_EA0_RDREQ_DRAM") is not None and dram_req:
            row["dram_read_bytes_per_launch"] = int(row["TCC_EA0_RDREQ_DRAM"] * dram_req)
        summary[bench_name] = row
    js = {"workload": args.workload, "tuning": json.loads(args.tuning) if args.tuning else None,
          "read_scale": scale["FETCH_SIZE"], "write_scale": scale["WRITE_SIZE"], "dram_request_bytes": dram_req,
          "calibration_kib": calib, "source": args.out, "command": args.cmd,
          "sources": args.sources, "kernels": {}}
    for k, row in summary.items():
        e = {kk: (round(v, 6) if isinstance(v, float) else v) for kk, v in row.items()}
        e["sources"] = args.sources
        js["kernels"][k] = e
    with open(args.json_out, "w") as f:
        json.dump(js, f, indent=1)
    lines = [f"# {args.title}", "", "Commands (GPU box, repo root = $R; one counter group per run):", "",
             "```", args.cmd, "```", "",
             "Per kernel, averages over active dispatches (a tenth of the 90th-percentile duration or "
             "more). FETCH_SIZE counts what the L2 fetches from the fabric (Infinity Cache hits "
             "included), so it bounds HBM reads from above; TCC_EA0_RDREQ_DRAM counts DRAM read "
             "requests. Copy calibration (the library's FP32 copy kernel, "
             f"{args.calib_bytes} bytes read and written per launch): "
             f"FETCH x{scale['FETCH_SIZE']:.4f}, WRITE x{scale['WRITE_SIZE']:.4f}"
             + (f", {dram_req:.1f} bytes per DRAM read request." if dram_req else "."), ""]
    cols = [("avg_us", "avg us", "{:.1f}"), ("traffic_bytes_per_launch", "traffic MB", "{:.1f}"),
            ("dram_read_bytes_per_launch", "DRAM read MB", "{:.1f}"),
            ("mfma_bf16_tflops", "MFMA BF16 TFLOP/s", "{:.2f}"),
            ("mfma_frac_of_bf16_peak", "MFMA frac of peak", "{:.4f}"),
            ("mfma_busy_share", "MFMA busy share", "{:.4f}"), ("wait_share", "wait share", "{:.3f}"),
            ("lds_conflict_cycles_per_instr", "LDS conflict cyc/instr", "{:.2f}")]
    lines.append("| kernel | " + " | ".join(c[1] for c in cols) + " |")
    lines.append("|---|" + "---:|" * len(cols))
    for k, row in summary.items():
        vals = []
        for key, _, fmt in cols:
            v = row.get(key)
            if v is None:
                vals.append("")
            elif key.endswith("bytes_per_launch"):
                vals.append(fmt.format(v / 1e6))
            else:
                vals.append(fmt.format(v))
        lines.append(f"| `{k}` | " + " | ".join(vals) + " |")
    lines += ["", "Raw counter averages per active dispatch:", ""]
    for k, row in summary.items():
        raw = {c: row[c] for c in row if c.isupper() or c.startswith(("SQ_", "TCC_", "FETCH", "WRITE"))}
        lines.append(f"* `{k}` ({row.get('symbol')}): " + ", ".join(f"{c} {v:.4g}" for c, v in sorted(raw.items())))
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("out")
    t.add_argument("trace")
    t.add_argument("--cmd", required=True)
    t.add_argument("--title", default="Kernel trace")
    c = sub.add_parser("counters")
    c.add_argument("out")
    c.add_argument("json_out")
    c.add_argument("--run", action="append", default=[], required=True)
    c.add_argument("--calib-fetch")
    c.add_argument("--calib-write")
    c.add_argument("--calib-dram")
    c.add_argument("--calib-bytes", type=int, default=4 * 37748736)
    c.add_argument("--kernels", nargs="+", default=[])
    c.add_argument("--cmd", required=True)
    c.add_argument("--title", default="Counters")
    c.add_argument("--workload", default="")
    c.add_argument("--tuning", default="")
    c.add_argument("--sources", default="")
    args = ap.parse_args(argv)
    if args.mode == "trace":
        trace(args)
    else:
        counters(args)


if __name__ == "__main__":
    sys.exit(main())
