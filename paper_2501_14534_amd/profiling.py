"""Summaries of rocprofv3 output for the kernels of libgs.

  python -m paper_2501_14534_amd.profiling stats DIR --cmd "..." --out profiles/NAME.md
      per-kernel call count and average/total duration from a
      `rocprofv3 --kernel-trace --stats --output-format csv` run.
  python -m paper_2501_14534_amd.profiling counters DIR --issue-dir IDIR --stats-dir SDIR --kernel K
      --workload W --cmd "..." [--json profiles/pmc_valu_lds.json] [--out profiles/NAME.md]
      LDS utilisation, LDS bank conflicts and LDS bytes per launch of kernel K from a `rocprofv3 --pmc
      VALUBusy VALUUtilization LdsUtil LdsBankConflict SQ_INSTS_LDS_LOAD_BANDWIDTH
      SQ_INSTS_LDS_STORE_BANDWIDTH` run (DIR), and its VALU and LDS instruction issue from a raw
      `--pmc SQ_INSTS_VALU SQ_INSTS_LDS SQ_WAVES ...` run (IDIR) over the kernel's average duration
      in a `--kernel-trace --stats` run (SDIR); medians over dispatches.  rocprofv3's derived
      VALUBusy and VALUUtilization read above 100 % on this chip and are not used.
  python -m paper_2501_14534_amd.profiling traffic FETCH_DIR WRITE_DIR --kernel K --workload W
      --copy-bytes B --cmd "..." [--json profiles/pmc_traffic.json] [--key NAME] [--out profiles/NAME.md]
      HBM bytes per launch of kernel K from two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs
      (KiB per dispatch), each scaled by what the same counter reads for the plain copy kernel
      of B bytes that `bench.py --calibration-copy-bytes B` launches (an elementwise multiply
      by one: B read, B written).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _csvs(d, suffix):
    return sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))


def kernel_stats(d):
    rows = []
    for f in _csvs(d, "kernel_stats.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append(dict(name=r["Name"], calls=int(r["Calls"]), total_ns=float(r["TotalDurationNs"]),
                                 avg_ns=float(r["AverageNs"]), pct=float(r["Percentage"])))
    rows.sort(key=lambda r: -r["total_ns"])
    return rows


def launch_shapes(d):
    """{(kernel name, grid size): [duration ns per dispatch]} from the kernel trace."""
    out = defaultdict(list)
    for f in _csvs(d, "kernel_trace.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
                out[(r["Kernel_Name"], grid)].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return out


def counter_table(d):
    """{kernel name: [{counter: value} per dispatch]} (values summed over a counter's instances)."""
    per = defaultdict(lambda: defaultdict(float))
    names = {}
    for f in _csvs(d, "counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                did = r.get("Dispatch_Id") or r.get("Correlation_Id")
                names[did] = r.get("Kernel_Name") or r.get("Kernel-Name")
                per[did][r["Counter_Name"]] += float(r["Counter_Value"])
    out = defaultdict(list)
    for did, cs in per.items():
        out[names[did]].append(dict(cs))
    return out


def counter_values(d):
    """{kernel name: [value per dispatch]} summed over the counter's instances."""
    per = defaultdict(lambda: defaultdict(float))
    names = {}
    for f in _csvs(d, "counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                did = r.get("Dispatch_Id") or r.get("Correlation_Id")
                k = r.get("Kernel_Name") or r.get("Kernel-Name")
                names[did] = k
                per[did][r["Counter_Name"]] += float(r["Counter_Value"])
    out = defaultdict(list)
    for did, cs in per.items():
        for _, v in cs.items():
            out[names[did]].append(v)
    return out


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2501_14534_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


CLOCK_HZ = 2.4e9  # MI355X peak engine clock
SIMDS = 256 * 4  # 256 compute units of 4 SIMDs
FP32_VALU_ISSUE_PER_SIMD_CYCLE = 0.25  # one wave64 FP32 FMA per 4 cycles on a 16-lane SIMD


def _match(values, pattern):
    return {k: v for k, v in values.items() if pattern in k}


def cmd_stats(a):
    rows = kernel_stats(a.dir)
    lines = [f"# rocprofv3 kernel statistics: {a.title}", "", "Command:", "", "```", a.cmd, "```", "",
             "| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for r in rows[: a.top]:
        lines.append(f"| `{r['name'][:90]}` | {r['calls']} | {r['avg_ns'] / 1e3:.2f} | {r['total_ns'] / 1e6:.3f} | "
                     f"{r['pct']:.2f} |")
    shapes = launch_shapes(a.dir)
    if shapes:
        lines += ["", "Per launch shape (grid = total work-items), kernels of libgs only:", "",
                  "| kernel | grid | calls | avg us | min us | max us |", "|---|---|---|---|---|---|"]
        for (name, grid), ds in sorted(shapes.items(), key=lambda kv: -sum(kv[1])):
            if "gs::" not in name:
                continue
            lines.append(f"| `{name[:60]}` | {grid} | {len(ds)} | {statistics.mean(ds) / 1e3:.2f} | "
                         f"{min(ds) / 1e3:.2f} | {max(ds) / 1e3:.2f} |")
    lines.append(f"\nkernel source hash: {kernel_source_hash()}")
    text = "\n".join(lines) + "\n"
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    print(text)


def cmd_counters(a):
    table = counter_table(a.dir)
    rows = [r for k, rs in table.items() if a.kernel in k for r in rs]
    if not rows:
        sys.exit(f"no dispatches of {a.kernel} in {a.dir}")

    def med(name):
        vals = [r[name] for r in rows if name in r]
        return statistics.median(vals) if vals else None

    lds_units = [(r.get("SQ_INSTS_LDS_LOAD_BANDWIDTH", 0.0) + r.get("SQ_INSTS_LDS_STORE_BANDWIDTH", 0.0)) for r in rows]
    # raw issue counters over the kernel's average duration
    irows = [r for k, rs in counter_table(a.issue_dir).items() if a.kernel in k for r in rs]
    durs = [r["avg_ns"] for r in kernel_stats(a.stats_dir) if a.kernel in r["name"]]
    if not irows or not durs:
        sys.exit(f"no issue counters ({len(irows)}) or duration ({len(durs)}) for {a.kernel}")

    def imed(name):
        return statistics.median([r[name] for r in irows])

    cycles = durs[0] * 1e-9 * CLOCK_HZ
    waves, valu, lds = imed("SQ_WAVES"), imed("SQ_INSTS_VALU"), imed("SQ_INSTS_LDS")
    valu_rate = valu / (cycles * SIMDS)
    entry = dict(kernel=a.kernel, workload=a.workload, source_hash=kernel_source_hash(), dispatches=len(rows),
                 waves=waves, valu_insts_per_wave=valu / waves, lds_insts_per_wave=lds / waves,
                 ms_per_launch=durs[0] * 1e-6, valu_insts_per_simd_cycle=valu_rate,
                 valu_issue_frac_fp32=valu_rate / FP32_VALU_ISSUE_PER_SIMD_CYCLE,
                 lds_util=med("LdsUtil"), lds_bank_conflict_per_access=med("LdsBankConflict"),
                 lds_bytes_per_launch=64.0 * statistics.median(lds_units), command=a.cmd,
                 issue_command=a.issue_cmd)
    if a.json:
        d = json.load(open(a.json)) if os.path.exists(a.json) else {}
        d[f"{a.key or a.kernel}@{a.workload}"] = entry
        with open(a.json, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
    text = "\n".join([
        f"# VALU and LDS counters of `{a.kernel}` ({a.workload})", "", "Commands (LDS pass, then raw issue pass):",
        "", "```", a.cmd, a.issue_cmd, "```", "",
        f"Medians over {len(rows)} dispatches; durations from the `--kernel-trace --stats` run of the same "
        f"workload ({entry['ms_per_launch']:.4f} ms per launch), at {CLOCK_HZ / 1e9:.1f} GHz on {SIMDS} SIMDs:", "",
        f"- waves per launch: {waves:.0f}; VALU instructions per wave: {entry['valu_insts_per_wave']:.0f}; "
        f"LDS instructions per wave: {entry['lds_insts_per_wave']:.0f}",
        f"- VALU instructions issued per SIMD per cycle: {valu_rate:.4f}; a wave64 FP32 FMA holds a 16-lane SIMD "
        f"for 4 cycles, so full-rate FP32 issue is {FP32_VALU_ISSUE_PER_SIMD_CYCLE} per SIMD-cycle: "
        f"{entry['valu_issue_frac_fp32']:.3f} of it (above 1 where part of the mix, such as moves, selects and "
        f"compares, issues faster than a full-rate FP32 operation)",
        f"- LdsUtil (share of cycles the LDS serves indexed accesses, per CU): {entry['lds_util']:.2f} %",
        f"- LdsBankConflict (bank-conflict cycles per LDS access cycle): {entry['lds_bank_conflict_per_access']:.4f}",
        f"- LDS bytes per launch (load + store bandwidth counters x 64 B; a broadcast read counts once per "
        f"active lane): {entry['lds_bytes_per_launch']:.4e}",
        f"- kernel source hash: {entry['source_hash']}", ""])
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    print(text)


def cmd_traffic(a):
    fetch = counter_values(a.fetch_dir)
    write = counter_values(a.write_dir)
    copy_f = [v for k, vs in _match(fetch, a.copy_pattern).items() for v in vs]
    copy_w = [v for k, vs in _match(write, a.copy_pattern).items() for v in vs]
    kib = a.copy_bytes / 1024.0
    # the calibration copy is the largest elementwise dispatch of the run
    cf = kib / max(copy_f) if copy_f else None
    cw = kib / max(copy_w) if copy_w else None
    kf = [v for k, vs in _match(fetch, a.kernel).items() for v in vs]
    kw = [v for k, vs in _match(write, a.kernel).items() for v in vs]
    if not kf or not kw or cf is None or cw is None:
        sys.exit(f"missing counters: kernel fetch {len(kf)} write {len(kw)}, copy fetch {len(copy_f)} "
                 f"write {len(copy_w)}")
    f_med, w_med = statistics.median(kf), statistics.median(kw)
    byts = (f_med * cf + w_med * cw) * 1024.0
    entry = dict(kernel=a.kernel, workload=a.workload, source_hash=kernel_source_hash(),
                 fetch_kib_per_launch=f_med, write_kib_per_launch=w_med, copy_scale_fetch=cf, copy_scale_write=cw,
                 hbm_bytes_per_launch=byts, dispatches=len(kf), command=a.cmd)
    if a.json:
        d = json.load(open(a.json)) if os.path.exists(a.json) else {}
        d[f"{a.key or a.kernel}@{a.workload}"] = entry
        with open(a.json, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
    text = "\n".join([
        f"# HBM traffic of `{a.kernel}` ({a.workload})", "", "Commands (FETCH_SIZE run, then WRITE_SIZE run):", "",
        "```", a.cmd, "```", "",
        f"- FETCH_SIZE median over {len(kf)} dispatches: {f_med:.1f} KiB; WRITE_SIZE: {w_med:.1f} KiB",
        f"- calibration copy of {a.copy_bytes} B: FETCH_SIZE scale {cf:.4f}, WRITE_SIZE scale {cw:.4f}",
        f"- HBM bytes per launch: {byts:.4e}", f"- kernel source hash: {entry['source_hash']}", ""])
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    print(text)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--cmd", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--out")
    s.add_argument("--top", type=int, default=25)
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--issue-dir", required=True, help="raw --pmc SQ_INSTS_VALU SQ_INSTS_LDS SQ_WAVES ... run")
    c.add_argument("--issue-cmd", required=True)
    c.add_argument("--stats-dir", required=True, help="--kernel-trace --stats run of the same workload")
    c.add_argument("--kernel", required=True, help="substring of the kernel name, e.g. 'render_fwd_kernel<1, true, 0>'")
    c.add_argument("--key", default=None, help="name under which --json files the entry (default: --kernel)")
    c.add_argument("--workload", required=True)
    c.add_argument("--cmd", required=True)
    c.add_argument("--json")
    c.add_argument("--out")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--kernel", required=True)
    t.add_argument("--key", default=None, help="name under which --json files the entry (default: --kernel)")
    t.add_argument("--workload", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--copy-pattern", default="elementwise")
    t.add_argument("--cmd", required=True)
    t.add_argument("--json")
    t.add_argument("--out")
    a = ap.parse_args(argv)
    {"stats": cmd_stats, "traffic": cmd_traffic, "counters": cmd_counters}[a.what](a)


if __name__ == "__main__":
    main()
