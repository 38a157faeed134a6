"""Short text summaries of rocprofv3 output for the profiles kept with the library.

  python3 -m paper_2607_14025_amd.rocprof_summary stats DB TITLE COMMAND [BENCH_LOG LABEL KERNEL] > summary.md
      kernel table (calls, total and average duration, share) of a --kernel-trace --stats
      results database; with the bench's log, the traced durations of the bench's timed
      launches of KERNEL against the bench's own HIP-event time per launch.

  python3 -m paper_2607_14025_amd.rocprof_summary traffic FETCH_CSV WRITE_CSV BENCH_LOG LABEL KERNEL
          TITLE FETCH_COMMAND WRITE_COMMAND [TRAFFIC_JSON] > summary.md
      HBM bytes per launch of one kernel from two --pmc runs (FETCH_SIZE, then WRITE_SIZE) of
      `bench.py --steps 1 --warmup 0 --copy-calibration`. Each counter is scaled by what it reads
      for the 1 GiB elementwise copy that run starts with. The kernel's last launches are matched
      to the bench's final apply, its profiled headline step, and so to the bench's algorithmic
      bytes for them; the ratio measured / algorithmic goes to TRAFFIC_JSON under
      "WORKLOAD:LABEL", with the source hash bench.py checks.

  python3 -m paper_2607_14025_amd.rocprof_summary sq CSV TITLE COMMAND KERNEL > summary.md
      SQ counters (VALU, SALU, LDS instructions and issue cycles, LDS bank conflicts, wave cycles)
      of one kernel over the bench's final apply, per-dispatch means and their ratios.

  python3 -m paper_2607_14025_amd.rocprof_summary mfma CSV TITLE COMMAND [SIMDS] > summary.md
      MFMA use of the GEMM and net kernels from one --pmc run with SQ_INSTS_VALU_MFMA_MOPS_BF16,
      SQ_INSTS_VALU_MFMA_MOPS_F64, SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE over the bench's
      final apply (the dispatches after the last but one Delta n launch): MFMA FLOPs per dispatch
      (MOPS x 512) and the busy fraction of the matrix units, busy cycles / (active cycles x SIMDS).
      The CSV sums GRBM_GUI_ACTIVE over the XCDs, so it is divided by their count (the
      counter set's own expression takes the largest instance). SIMDS, the XCD count and the
      clock come from the run's agent file (run_agent_info.csv beside CSV), else 1024, 8 and
      2.4 GHz.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_KERNEL = "MulFunctor<double>"
COPY_BYTES = float(1 << 30)
# source file of each kernel class of the per-launch profile (stern_stats)
KERNEL_SOURCES = {"plane_h": "fft.hip", "plane_h32": "fft.hip", "xinv": "fft.hip", "xfwd": "fft.hip",
                  "x32": "fft.hip", "rhs_plane": "fft.hip", "dn_plane": "fft.hip", "pc_reduce": "gemm.hip",
                  "pc_expand": "gemm.hip", "kb_reduce": "gemm.hip", "kb_expand": "gemm.hip",
                  "sum_parts": "gemm.hip", "cg": "cg.hip", "cg32": "cg.hip", "gemm_bf16": "gemm_bf16.hip",
                  "net": "learn.hip"}

# what the bench's algorithmic bytes per launch count, per kernel class
ALGO_NOTE = {"plane_h32": "pencils read and written once, V_loc once",
             "plane_h": "pencils read and written once, V_loc once",
             "gemm_bf16": "the complex FP32 vectors and the projector block moved once each"}


def source_hash(label: str) -> str:
    """sha1 prefix of the source of kernel class `label` ("" if unknown)."""
    f = KERNEL_SOURCES.get(label)
    if f is None:
        return ""
    with open(os.path.join(HERE, "csrc", f), "rb") as fh:
        return hashlib.sha1(fh.read()).hexdigest()[:12]


def short_name(n: str) -> str:
    n = n.replace("stern::(anonymous namespace)::", "").replace("stern::", "")
    n = re.sub(r"\(.*\)$", "", n).replace("void ", "")
    return n


def matches(kernel: str, name: str) -> bool:
    """Whether the trace name `name` is one of the kernels `kernel` lists ("a|b": any of a, b), as
    a substring of its short name; a kernel class of the bench can span several kernels."""
    sn = short_name(name)
    return any(k in sn for k in kernel.split("|"))


def stats(db: str, title: str, cmd: str) -> str:
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    out = [f"# {title}\n", "Command (run from the repository root on one MI355X, with TMPDIR=/tmp):\n",
           f"```\n{cmd}\n```\n", "| kernel | calls | total (us) | average (us) | share |", "|---|---:|---:|---:|---:|"]
    for n, c, t, a, p in rows:
        if p < 0.005:
            continue
        out.append(f"| `{short_name(n)}` | {c} | {t:.0f} | {a:.1f} | {p:.2f}% |")  # the view is in us
    return "\n".join(out) + "\n"


def launch_agreement(db: str, bench_log: str, label: str, kernel: str) -> str:
    """rocprofv3 durations of the launches of `kernel` that the bench timed with HIP events
    against the bench's own HIP-event time per launch. The bench's last apply is the headline
    step with the per-launch profile, so those launches are the kernel's last ones."""
    bench = _bench_line(bench_log)
    k = bench["kernels"][label]
    n = int(k["launches"])
    con = sqlite3.connect(db)
    rows = [(dur, nm) for dur, nm in con.execute("select duration, name from kernels order by start")]
    mine = [dur for dur, nm in rows if matches(kernel, nm)]
    timed = mine[len(mine) - n:]
    avg_us = sum(timed) / len(timed) / 1e3  # durations are in ns
    return (f"Agreement for `{kernel}` ({label}, the kernel the bench's roofline reports): the bench's HIP "
            f"events give {k['ms_per_launch'] * 1e3:.1f} us per launch over the {n} launches of its profiled "
            f"step; this trace gives {avg_us:.1f} us for the same launches "
            f"(ratio {avg_us / (k['ms_per_launch'] * 1e3):.3f}).\n")


def _counter(path: str, counter: str):
    """[(dispatch id, kernel name, value)] of one counter, in dispatch order."""
    return [(d, n, v) for d, n, v, _ in _counter_timed(path, counter)]


def _counter_timed(path: str, counter: str):
    """[(dispatch id, kernel name, value, duration in ns or None)] of one counter, in dispatch order."""
    rows = []
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                t0, t1 = r.get("Start_Timestamp"), r.get("End_Timestamp")
                dur = float(t1) - float(t0) if t0 and t1 else None
                rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"]), dur))
    rows.sort(key=lambda x: x[0])
    return rows


def _bench_line(log: str) -> dict:
    with open(log) as fh:
        for line in fh:
            if line.startswith("{") and '"metric"' in line:
                return json.loads(line)
    raise SystemExit(f"no bench JSON line in {log}")


def traffic(fetch_csv, write_csv, bench_log, label, kernel, title, cmd_f, cmd_w, traffic_json=None) -> str:
    bench = _bench_line(bench_log)
    k = bench["kernels"][label]
    n_launch = int(k["launches"] // bench.get("kernels_steps", bench["steps"]))
    algo = float(k["bytes_per_launch"])
    key = f"{bench['config']['workload']}:{label}"
    res = {}
    for name, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = _counter(path, counter)
        copy = [v for _, n, v in rows if COPY_KERNEL in n]
        if not copy:
            raise SystemExit(f"{path}: no calibration copy kernel ({COPY_KERNEL})")
        scale = COPY_BYTES / (copy[0] * 1024.0)
        mine = [v for _, n, v in rows if matches(kernel, n)]
        if len(mine) < n_launch:
            raise SystemExit(f"{path}: {len(mine)} dispatches of {kernel}, the bench step has {n_launch}")
        last = mine[-n_launch:]
        res[name] = dict(copy_kib=copy[0], scale=scale, kib=sum(last) / len(last),
                         bytes=scale * 1024.0 * sum(last) / len(last), n_all=len(mine))
    measured = res["fetch"]["bytes"] + res["write"]["bytes"]
    ratio = measured / algo
    sha = source_hash(label)
    if traffic_json:
        t = json.load(open(traffic_json)) if os.path.exists(traffic_json) else {}
        t[key] = dict(measured_over_algorithmic=ratio, source_sha1=sha, kernel=kernel, launches_matched=n_launch,
                        algorithmic_bytes_per_launch=algo, measured_bytes_per_launch=measured,
                        read_bytes_per_launch=res["fetch"]["bytes"], write_bytes_per_launch=res["write"]["bytes"])
        with open(traffic_json, "w") as fh:
            json.dump(t, fh, indent=1)
            fh.write("\n")
    f, w = res["fetch"], res["write"]
    # every kernel of the run, for context (all its dispatches, the autotuner's included)
    per = {}
    for key, path, counter in (("r", fetch_csv, "FETCH_SIZE"), ("w", write_csv, "WRITE_SIZE")):
        sc = res["fetch" if key == "r" else "write"]["scale"] * 1024.0
        for _, n, v, dur in _counter_timed(path, counter):
            e = per.setdefault(short_name(n), {"r": [], "w": [], "tr": [], "tw": []})
            e[key].append(v * sc)
            if dur is not None:
                e["t" + key].append(dur)
    table = ["| kernel | dispatches | read MB / dispatch | write MB / dispatch | GB/s past L2 |", "|---|---:|---:|---:|---:|"]
    for n, e in sorted(per.items(), key=lambda kv: -(sum(kv[1]["r"]) + sum(kv[1]["w"]))):
        if not e["r"] or not e["w"] or sum(e["r"]) + sum(e["w"]) < 1e8:
            continue
        rd, wr = sum(e["r"]) / len(e["r"]), sum(e["w"]) / len(e["w"])
        # each counter's bytes over the durations of the run it was taken in
        gbs = ""
        if e["tr"] and e["tw"] and sum(e["tr"]) > 0 and sum(e["tw"]) > 0:
            gbs = f"{sum(e['r']) / sum(e['tr']) + sum(e['w']) / sum(e['tw']):.0f}"
        table.append(f"| `{n[:70]}` | {len(e['r'])} | {rd / 1e6:.1f} | {wr / 1e6:.1f} | {gbs} |")
    return "\n".join([
        f"# {title}\n",
        "Commands (repository root, one MI355X, TMPDIR=/tmp), one counter per run:\n",
        f"```\n{cmd_f}\n{cmd_w}\n```\n",
        f"Calibration: the run starts with one elementwise kernel (`{COPY_KERNEL}`) that reads 1 GiB and writes "
        f"1 GiB. It reads FETCH_SIZE = {f['copy_kib']:.1f} KiB and WRITE_SIZE = {w['copy_kib']:.1f} KiB, so "
        f"bytes = FETCH_SIZE x 1024 x {f['scale']:.4f} and WRITE_SIZE x 1024 x {w['scale']:.4f}.\n",
        f"`{kernel}` ({label}): {f['n_all']} dispatches in the run; the last {n_launch} are the bench's final "
        f"apply, whose launches repeat the timed step's.\n",
        "| per launch (average of those) | bytes |", "|---|---:|",
        f"| FETCH_SIZE {f['kib']:.0f} KiB, calibrated | {f['bytes'] / 1e6:.1f} MB |",
        f"| WRITE_SIZE {w['kib']:.0f} KiB, calibrated | {w['bytes'] / 1e6:.1f} MB |",
        f"| measured total | {measured / 1e6:.1f} MB |",
        f"| algorithmic ({ALGO_NOTE.get(label, 'the bench bytes per launch')}) | {algo / 1e6:.1f} MB |",
        f"| measured / algorithmic | {ratio:.3f} |\n",
        f"Source `paper_2607_14025_amd/csrc/{KERNEL_SOURCES.get(label)}` sha1 prefix at measurement: {sha}\n",
        "All kernels of the run with more than 100 MB of traffic in total (calibrated, per dispatch). The counters "
        "count L2 misses, which the Infinity Cache may serve, so these bytes bound HBM traffic from above. GB/s = "
        "those bytes over the dispatch durations rocprofv3 recorded in the same counter runs (kernels serialised):\n",
    ] + table) + "\n"


MFMA_KERNELS = ("k_reduce_bf16w", "k_expand_bf16s", "k_zgemm_reduce", "k_zgemm_expand", "k_conv3")


def _gpu_agent(csv_path: str):
    """(SIMDs, XCDs, clock in GHz) of the GPU agent of a rocprofv3 run, or None."""
    path = csv_path.replace("counter_collection", "agent_info")
    if path == csv_path or not os.path.exists(path):
        return None
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            if r.get("Agent_Type", "").strip('"') == "GPU":
                return int(r["Simd_Count"]), int(r["Num_Xcc"]), float(r["Max_Engine_Clk_Fcompute"]) / 1e3
    return None


def mfma(csv_path: str, title: str, cmd: str, simds: int = 1024, xcds: int = 8, clock_ghz: float = 2.4) -> str:
    agent = _gpu_agent(csv_path)
    if agent:
        simds, xcds, clock_ghz = agent
    per = {}
    with open(csv_path, newline="") as fh:
        for r in csv.DictReader(fh):
            d = per.setdefault(int(r["Dispatch_Id"]), {"name": short_name(r["Kernel_Name"])})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    order = sorted(per)
    dn = [i for i in order if per[i]["name"].startswith("k_plane_dn")]
    if len(dn) < 2:
        raise SystemExit(f"{csv_path}: fewer than two Delta n dispatches")
    last = [i for i in order if dn[-2] < i <= dn[-1]]
    agg = {}
    for i in last:
        d = per[i]
        if not d["name"].startswith(MFMA_KERNELS):
            continue
        a = agg.setdefault(d["name"], {"n": 0, "bf16": 0.0, "f64": 0.0, "busy": 0.0, "active": 0.0})
        a["n"] += 1
        a["bf16"] += 512.0 * d.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0)
        a["f64"] += 512.0 * d.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0)
        a["busy"] += d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
        a["active"] += d.get("GRBM_GUI_ACTIVE", 0.0) / xcds
    rows = ["| kernel | dispatches | BF16 MFMA GFLOP / dispatch | FP64 MFMA GFLOP / dispatch | matrix units busy | "
            f"MFMA TFLOP/s over the active cycles (at {clock_ghz:g} GHz) |", "|---|---:|---:|---:|---:|---:|"]
    for n, a in sorted(agg.items(), key=lambda kv: -kv[1]["active"]):
        busy = a["busy"] / (a["active"] * simds) if a["active"] > 0 else 0.0
        secs = a["active"] / (clock_ghz * 1e9)
        rate = (a["bf16"] + a["f64"]) / secs / 1e12 if secs > 0 else 0.0
        rows.append(f"| `{n[:60]}` | {a['n']} | {a['bf16'] / a['n'] / 1e9:.2f} | {a['f64'] / a['n'] / 1e9:.2f} | "
                    f"{100 * busy:.1f}% | {rate:.0f} |")
    return "\n".join([
        f"# {title}\n",
        "Command (repository root, one MI355X, TMPDIR=/tmp):\n",
        f"```\n{cmd}\n```\n",
        f"Dispatches of the bench's final apply ({len(last)} in all, between the last two Delta n launches). "
        "FLOPs are the counters' MFMA operations x 512. The busy fraction is the matrix units' busy cycles over "
        f"the kernel's active cycles x {simds} SIMDs, the counter set's own MFMA-utilisation expression; the "
        f"active cycles are GRBM_GUI_ACTIVE / {xcds}, as the CSV sums it over the XCDs. "
        "Peaks: 2.5 PFLOP/s BF16 and 78.6 TFLOP/s FP64 (dense MFMA).\n",
    ] + rows) + "\n"


def sq(csv_path: str, title: str, cmd: str, kernel: str) -> str:
    """SQ counters of one kernel over the bench's final apply (the dispatches after the last but one
    Delta n launch): per-dispatch means and the ratios that say what bounds it."""
    per = {}
    with open(csv_path, newline="") as fh:
        for r in csv.DictReader(fh):
            d = per.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"]})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    order = sorted(per)
    dn = [i for i in order if short_name(per[i]["name"]).startswith("k_plane_dn")]
    if len(dn) < 2:
        raise SystemExit(f"{csv_path}: fewer than two Delta n dispatches")
    mine = [per[i] for i in order if dn[-2] < i <= dn[-1] and matches(kernel, per[i]["name"])]
    if not mine:
        raise SystemExit(f"{csv_path}: no dispatch of {kernel} in the final apply")
    names = sorted(k for k in mine[0] if k != "name")
    mean = {k: sum(d.get(k, 0.0) for d in mine) / len(mine) for k in names}
    rows = ["| counter | mean per dispatch |", "|---|---:|"] + [f"| {k} | {mean[k]:.4g} |" for k in names]
    notes = []
    if mean.get("SQ_ACTIVE_INST_LDS"):
        notes.append(f"LDS bank-conflict cycles per LDS-active cycle: "
                     f"{mean.get('SQ_LDS_BANK_CONFLICT', 0.0) / mean['SQ_ACTIVE_INST_LDS']:.3f}")
    if mean.get("SQ_INSTS_VALU"):
        notes.append(f"SALU / VALU instructions: {mean.get('SQ_INSTS_SALU', 0.0) / mean['SQ_INSTS_VALU']:.3f}; "
                     f"LDS / VALU instructions: {mean.get('SQ_INSTS_LDS', 0.0) / mean['SQ_INSTS_VALU']:.3f}")
    if mean.get("SQ_WAVE_CYCLES"):
        notes.append(f"VALU-issue cycles per wave cycle: "
                     f"{mean.get('SQ_ACTIVE_INST_VALU', 0.0) / mean['SQ_WAVE_CYCLES']:.3f}; LDS-issue cycles per "
                     f"wave cycle: {mean.get('SQ_ACTIVE_INST_LDS', 0.0) / mean['SQ_WAVE_CYCLES']:.3f}")
    return "\n".join([
        f"# {title}\n",
        "Command (repository root, one MI355X, TMPDIR=/tmp):\n",
        f"```\n{cmd}\n```\n",
        f"`{kernel}`: {len(mine)} dispatches in the bench's final apply (between the last two Delta n launches). "
        "SQ counters are summed over the shader engines by rocprofv3; the *_CYCLES counters count in units of "
        "quad-cycles per the counter definitions, and their ratios compare like with like.\n",
    ] + rows + [""] + [f"- {n}" for n in notes]) + "\n"


def main(argv):
    if len(argv) >= 4 and argv[0] == "stats":
        sys.stdout.write(stats(argv[1], argv[2], argv[3]))
        if len(argv) >= 7:  # BENCH_LOG LABEL KERNEL: agreement with the bench's event timing
            sys.stdout.write("\n" + launch_agreement(argv[1], argv[4], argv[5], argv[6]))
    elif len(argv) >= 9 and argv[0] == "traffic":
        sys.stdout.write(traffic(*argv[1:10]))
    elif len(argv) >= 5 and argv[0] == "sq":
        sys.stdout.write(sq(argv[1], argv[2], argv[3], argv[4]))
    elif len(argv) >= 4 and argv[0] == "mfma":
        sys.stdout.write(mfma(argv[1], argv[2], argv[3], *([int(argv[4])] if len(argv) > 4 else [])))
    else:
        sys.stdout.write(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
