"""Workload driver and summariser for rocprofv3 runs of the detection path.

``python -m paper_1611_09704_amd.profiling run --workload ska``
    Generates the SKA-like plane on cuda:0, runs one device copy of a known
    size (the calibration kernel for the FETCH_SIZE / WRITE_SIZE counters),
    then ``--steps`` passes of msd_compute + boxcar_snr.  Meant to be the
    program under ``rocprofv3 --pmc ...`` or ``--kernel-trace --stats``.

``python -m paper_1611_09704_amd.profiling summarize --trace DIR --fetch DIR --write DIR --out profiles``
    Reads the CSV files rocprofv3 wrote and produces the text summaries kept
    under profiles/ (per-kernel durations, and HBM bytes per dispatch scaled
    by what the counters read for the calibration copy).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
COPY_BYTES = 1 << 31          # calibration copy: reads and writes 2 GiB
WORKLOADS = {"ska": None, "ska16": list(range(1, 17)), "dit": "dit", "cluster": "cluster", "dedisp": "dedisp"}
BOXCAR_SOURCES = ("spd_device.h", "spd_kernels.hip", "spd_kernels.h", "spd_internal.h", "spd_stream.hip")
CLUSTER_SOURCES = ("spd_cluster.hip",)
DEDISP_SOURCES = ("spd_dedisp.hip",)
CLUSTER_RADII = (2, 256)     # DM rows, starts
DIT_LEVELS = 4


def kernel_source_sha(files=BOXCAR_SOURCES) -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1611_09704_amd", "csrc")
    for f in files:   # device code
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def run(args):
    import torch

    from paper_1611_09704_amd import binding as B
    from paper_1611_09704_amd import synth
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)                       # calibration dispatch
    torch.cuda.synchronize()
    del src, dst
    if WORKLOADS[args.workload] == "dedisp":
        run_dedisp(args, dev)
        return
    cfg = synth.ska(device=dev, R=args.rows, L=args.cols)
    x = cfg["plane"].x
    dit = WORKLOADS[args.workload] == "dit"
    cluster = WORKLOADS[args.workload] == "cluster"
    W = B.dit_widths(DIT_LEVELS) if dit else (cfg["widths"] if cluster else WORKLOADS[args.workload] or cfg["widths"])
    # the peak-finding workload runs sqrt(N) mode, whose signal-dominated rows flood the list
    p = B.Params(W, cfg["threshold"], "row", "sqrtn" if cluster else cfg["sigma_mode"], cfg["kappa"])
    R, L = x.shape
    nout = L - p.nmax + 1
    stats = torch.empty((R, B.STATS_FIELDS), dtype=torch.float64, device=dev)
    ws = torch.empty(B.workspace_bytes(x, p), dtype=torch.uint8, device=dev)
    po = (nout + 15) // 16 * 16                    # output rows padded as the bench pads them
    snr = torch.empty((R, po), dtype=torch.float32, device=dev)[:, :nout]
    widx = torch.empty((R, po), dtype=torch.uint8, device=dev)[:, :nout]
    cand = B.new_candidates(1 << 23 if cluster else 1 << 21, dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    peaks = B.new_candidates(1 << 20, dev)
    pcount = torch.zeros(1, dtype=torch.int64, device=dev)
    for k in range(args.steps):
        B.msd_compute(x, p, stats=stats, workspace=ws)
        if dit:
            B.boxcar_snr_dit(x, p, DIT_LEVELS, stats, snr=snr, widx=widx, cand=cand, cand_count=count)
        else:
            B.boxcar_snr(x, p, stats, snr=snr, widx=widx, cand=cand, cand_count=count)
        if cluster:
            B.cluster_candidates(snr, cand, count, *CLUSTER_RADII, peaks=peaks, peak_count=pcount)
        torch.cuda.synchronize()
        print("step %d done, %d candidates%s" % (k, int(count.item()),
                                                 ", %d peaks" % int(pcount.item()) if cluster else ""), flush=True)


def run_dedisp(args, dev, n_chan=4096, n_dm=6000):
    """The de-dispersion kernel alone on the benchmark's SKA-like filterbank
    (4,096 channels x 2^20 samples, 6,000 trials one sample apart)."""
    import numpy as np
    import torch

    from paper_1611_09704_amd import binding as B
    from paper_1611_09704_amd import synth
    band = (1550.0, 300.0 / n_chan, 64e-6)
    f_low = band[0] - (n_chan - 1) * band[1]
    dm = np.arange(n_dm) / (4.148808e3 * (1.0 / f_low ** 2 - 1.0 / band[0] ** 2) / band[2])
    fb = synth.filterbank(n_chan, args.cols, seed=1611097060, device=dev)
    plan = B.DedispPlan(n_chan, *band, dm)
    y = torch.empty((n_dm, args.cols - plan.max_delay), dtype=torch.float32, device=dev)
    for k in range(args.steps):
        plan.run(fb, out=y)
        torch.cuda.synchronize()
        print("step %d done" % k, flush=True)


def _csvs(d, suffix):
    return sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))


def _short(name: str, with_args: bool = False) -> str:
    """Kernel name without namespace and signature; ``with_args`` keeps the
    template arguments (dtype, outputs per lane, unit steps, small path)."""
    targs = ""
    if with_args and "<" in name.split("(")[0]:
        targs = "<" + name.split("(")[0].split("<", 1)[1]
    for key in ("batch_boxcar_win_grid_kernel", "batch_boxcar_grid_kernel", "batch_boxcar_kernel", "batch_msd_kernel",
                "batch_finalize_kernel", "boxcar_dit_kernel", "boxcar_stream_fast_kernel", "boxcar_stream_kernel", "boxcar_win_kernel", "boxcar_kernel", "msd_xy_kernel", "msd_x_kernel", "msd_finalize_kernel",
                "select_kernel", "cluster_kernel", "dedisp_u8_wide_kernel", "dedisp_u8_kernel",
                "fill_i64_kernel"):
        if key in name:
            return key + targs
    if "copyBuffer" in name:
        return "calibration_copy"
    return name[:60]


def read_counters(d):
    """{kernel short name: {counter: [value per dispatch]}} from a --pmc run."""
    out = defaultdict(lambda: defaultdict(dict))
    for f in _csvs(d, "counter_collection.csv"):
        for row in csv.DictReader(open(f)):
            k = _short(row["Kernel_Name"])
            disp = row.get("Dispatch_Id") or row.get("Correlation_Id")
            c = row["Counter_Name"]
            out[k][c][disp] = out[k][c].get(disp, 0.0) + float(row["Counter_Value"])
    return {k: {c: list(v.values()) for c, v in cs.items()} for k, cs in out.items()}


def summarize(args):
    sha = kernel_source_sha({"cluster": CLUSTER_SOURCES, "dedisp": DEDISP_SOURCES}.get(args.workload, BOXCAR_SOURCES))
    lines = []
    stats = _csvs(args.trace, "kernel_stats.csv") if args.trace else []
    if stats:
        lines.append("## Kernel durations (rocprofv3 --kernel-trace --stats)\n")
        lines.append("command: `%s`\n" % args.trace_cmd)
        lines.append("| kernel | calls | average ms | total ms | share |")
        lines.append("|---|---|---|---|---|")
        rows = list(csv.DictReader(open(stats[0])))
        total = sum(float(r["TotalDurationNs"]) for r in rows) or 1.0
        for row in rows:
            name = _short(row["Name"], with_args=True)
            if not any(k in name for k in ("boxcar", "msd", "select", "finalize", "fill_i64", "cluster", "dedisp")):
                continue
            lines.append("| %s | %s | %.4f | %.3f | %.2f%% |" % (
                name, row["Calls"], float(row["AverageNs"]) / 1e6, float(row["TotalDurationNs"]) / 1e6,
                100.0 * float(row["TotalDurationNs"]) / total))
        lines.append("")
    traces = _csvs(args.trace, "kernel_trace.csv") if args.trace else []
    if traces:
        groups = defaultdict(list)
        meta = {}
        for row in csv.DictReader(open(traces[0])):
            name = _short(row["Kernel_Name"], with_args=True)
            if not any(k in name for k in ("boxcar", "msd", "select", "finalize", "fill_i64", "cluster", "dedisp")):
                continue
            key = (name, int(row["Grid_Size_X"]))
            groups[key].append((int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e6)
            meta[key] = row.get("Workgroup_Size_X", "")
        lines.append("## Launches by kernel and grid size (rocprofv3 --kernel-trace, same run)\n")
        lines.append("| kernel | grid work-items | work-group | calls | average ms | min ms | max ms |")
        lines.append("|---|---|---|---|---|---|---|")
        for key in sorted(groups, key=lambda k: -sum(groups[k])):
            d = groups[key]
            lines.append("| %s | %d | %s | %d | %.4f | %.4f | %.4f |" % (
                key[0], key[1], meta[key], len(d), sum(d) / len(d), min(d), max(d)))
        lines.append("")
    traffic = {}
    if args.fetch and args.write:
        fc, wc = read_counters(args.fetch), read_counters(args.write)
        copy_f = fc.get("calibration_copy", {}).get("FETCH_SIZE", [])
        copy_w = wc.get("calibration_copy", {}).get("WRITE_SIZE", [])
        cf = max(copy_f) if copy_f else None
        cw = max(copy_w) if copy_w else None
        ff = COPY_BYTES / (cf * 1024.0) if cf else None
        fw = COPY_BYTES / (cw * 1024.0) if cw else None
        lines.append("## HBM traffic per dispatch (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)\n")
        lines.append("commands: `%s` and `%s`\n" % (args.fetch_cmd, args.write_cmd))
        lines.append("Calibration: a device copy of %d bytes read FETCH_SIZE = %s KiB and WRITE_SIZE = %s KiB, "
                     "so counter KiB are scaled by %s (fetch) and %s (write) to bytes.\n" % (
                         COPY_BYTES, cf, cw, "%.4f" % (ff * 1024) if ff else None,
                         "%.4f" % (fw * 1024) if fw else None))
        lines.append("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | read GB | written GB |")
        lines.append("|---|---|---|---|---|---|")
        for k in sorted(set(fc) | set(wc)):
            if not any(s in k for s in ("boxcar", "msd", "select", "cluster", "dedisp")):
                continue
            f = fc.get(k, {}).get("FETCH_SIZE", [])
            w = wc.get(k, {}).get("WRITE_SIZE", [])
            fm = sum(f) / len(f) if f else 0.0
            wm = sum(w) / len(w) if w else 0.0
            rb = fm * ff * 1024 if ff else None
            wb = wm * fw * 1024 if fw else None
            lines.append("| %s | %d | %.0f | %.0f | %s | %s |" % (
                k, len(f), fm, wm, "%.3f" % (rb / 1e9) if rb is not None else "-",
                "%.3f" % (wb / 1e9) if wb is not None else "-"))
            if rb is not None and wb is not None:
                traffic[k] = {"read_bytes": rb, "write_bytes": wb, "hbm_bytes_per_launch": rb + wb}
        lines.append("")
    lines.append("kernel sources sha: %s\n" % sha)
    os.makedirs(args.out, exist_ok=True)
    path = os.path.join(args.out, args.name + ".md")
    with open(path, "w") as fh:
        fh.write("# %s\n\n" % args.title + "\n".join(lines))
    print("wrote", path)
    if traffic and args.workload:
        tpath = os.path.join(args.out, "boxcar_traffic.json")
        try:
            d = json.load(open(tpath))
        except (OSError, ValueError):
            d = {}
        if args.workload == "cluster":
            d["cluster"] = {"kernel_sha": sha, **traffic.get("cluster_kernel", {})}
        elif args.workload == "dedisp":
            d["dedisp"] = {"kernel_sha": sha,
                           **(traffic.get("dedisp_u8_wide_kernel") or traffic.get("dedisp_u8_kernel") or {})}
        else:
            box = (traffic.get("boxcar_dit_kernel") or traffic.get("boxcar_stream_fast_kernel")
                   or traffic.get("boxcar_stream_kernel")
                   or traffic.get("boxcar_win_kernel") or traffic.get("boxcar_kernel") or {})
            d[args.workload] = {"kernel_sha": sha, **box,
                                "msd": traffic.get("msd_xy_kernel") or traffic.get("msd_x_kernel")}
        json.dump(d, open(tpath, "w"), indent=1)
        print("wrote", tpath)


N_CU, N_XCD, N_SIMD = 256, 8, 1024


def counter_summary(args):
    """Clock, LDS and VALU use of each path kernel from --pmc runs of SQ and
    GRBM counters (rocprofv3 reports each counter summed over XCDs and shader
    engines: GRBM_GUI_ACTIVE / 8 is the clock count of one XCD)."""
    lines = ["# %s\n" % args.title]
    for d, cmd in zip(args.dirs, args.cmds or [""] * len(args.dirs)):
        vals = defaultdict(lambda: defaultdict(float))
        span = {}
        for f in _csvs(d, "counter_collection.csv"):
            for row in csv.DictReader(open(f)):
                name = _short(row["Kernel_Name"], with_args=True)
                if not any(k in name for k in ("boxcar", "msd", "cluster", "dedisp")):
                    continue
                key = (name, row.get("Dispatch_Id"))
                vals[key][row["Counter_Name"]] += float(row["Counter_Value"])
                span[key] = (int(row["Start_Timestamp"]), int(row["End_Timestamp"]))
        lines.append("command: `%s`\n" % cmd)
        lines.append("| kernel | ms | counter | total | derived |")
        lines.append("|---|---|---|---|---|")
        for key in sorted(vals):
            c = vals[key]
            ms = (span[key][1] - span[key][0]) / 1e6
            cyc = c.get("GRBM_GUI_ACTIVE", 0.0) / N_XCD
            for n in sorted(c):
                der = ""
                if n == "GRBM_GUI_ACTIVE":
                    der = "clock %.2f GHz" % (cyc / (ms * 1e-3) / 1e9)
                elif cyc and n == "SQ_INSTS_VALU":
                    der = "%.2f VALU instructions per SIMD per 4 clocks (2 = dual-issue peak)" % (
                        c[n] / (N_SIMD * cyc / 4))
                elif cyc and n == "SQ_ACTIVE_INST_VALU2":
                    der = "two VALU issued in %.0f%% of SIMD quad-cycles" % (100 * c[n] / (N_SIMD * cyc / 4))
                elif cyc and n == "SQ_LDS_IDX_ACTIVE":
                    der = "LDS busy %.0f%% of CU clocks" % (100 * c[n] / (N_CU * cyc))
                elif cyc and n == "SQ_LDS_BANK_CONFLICT":
                    der = "bank-conflict stall %.1f%% of CU clocks" % (100 * c[n] / (N_CU * cyc))
                elif cyc and n == "SQ_INSTS_LDS_LOAD_BANDWIDTH":
                    der = "%.0f bytes read from LDS per CU clock" % (c[n] * 64 / (N_CU * cyc))
                lines.append("| %s | %.3f | %s | %.4g | %s |" % (key[0], ms, n, c[n], der))
        lines.append("")
    lines.append("kernel sources sha: %s\n" % kernel_source_sha())
    path = os.path.join(args.out, args.name + ".md")
    with open(path, "w") as fh:
        fh.write("\n".join(lines))
    print("wrote", path)
    if args.workload:
        write_valu_summary(args.workload, args.out, args.dirs)


def workload_evals(workload: str, rows: int = 4096, cols: int = 1 << 20) -> int:
    """(start, width) evaluations of one boxcar launch of a profiled workload."""
    from paper_1611_09704_amd import synth
    if WORKLOADS[workload] == "dit":
        n_ev = 0
        levels = DIT_LEVELS
        nout = cols - 16 * (1 << levels) + 1
        n_ev = nout * 16
        for lv in range(1, levels + 1):      # widths 9..16 of level lv at starts that are multiples of 2^lv
            n_ev += ((nout + (1 << lv) - 1) >> lv) * 8
        return rows * n_ev
    W = WORKLOADS[workload] or synth.SKA_WIDTHS
    return rows * (cols - W[-1] + 1) * len(W)


def write_valu_summary(workload, out, dirs):
    """VALU lane-instructions per (start, width) evaluation and clock of the
    workload's boxcar kernel, from the SQ_INSTS_VALU / GRBM_GUI_ACTIVE runs in
    dirs, into profiles/valu_counters.json (keyed by workload, with the hash of
    the kernel sources the counters were taken on)."""
    tot = defaultdict(lambda: defaultdict(float))
    span = {}
    for d in dirs:
        for f in _csvs(d, "counter_collection.csv"):
            for row in csv.DictReader(open(f)):
                name = _short(row["Kernel_Name"])
                if not name.startswith("boxcar"):
                    continue
                key = (name, row.get("Dispatch_Id"), d)
                tot[key][row["Counter_Name"]] += float(row["Counter_Value"])
                span[key] = (int(row["Start_Timestamp"]), int(row["End_Timestamp"]))
    valu = [(k, c) for k, c in tot.items() if "SQ_INSTS_VALU" in c]
    clk = [(k, c) for k, c in tot.items() if "GRBM_GUI_ACTIVE" in c]
    if not valu:
        return
    k, c = valu[0]
    evals = workload_evals(workload)
    ent = {"kernel_sha": kernel_source_sha(), "kernel": k[0],
           "valu_lane_instr_per_eval": round(c["SQ_INSTS_VALU"] * 64 / evals, 4)}
    if clk:
        kc, cc = clk[0]
        ms = (span[kc][1] - span[kc][0]) / 1e6
        cyc = cc["GRBM_GUI_ACTIVE"] / N_XCD
        ent["clock_ghz"] = round(cyc / (ms * 1e-3) / 1e9, 3)
        if kc[2] == k[2]:
            ent["valu_per_simd_quad_cycle"] = round(c["SQ_INSTS_VALU"] / (N_SIMD * cyc / 4), 3)
    path = os.path.join(out, "valu_counters.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        d = {}
    d[workload] = ent
    json.dump(d, open(path, "w"), indent=1)
    print("wrote", path)


def _busy(intervals):
    """Total length of the union of [start, end) intervals, and the length
    covered by at least two of them."""
    ev = []
    for a, b in intervals:
        ev.append((a, 1))
        ev.append((b, -1))
    ev.sort()
    union = two = 0
    depth, last = 0, None
    for t, d in ev:
        if last is not None:
            if depth >= 1:
                union += t - last
            if depth >= 2:
                two += t - last
        depth += d
        last = t
    return union, two


def overlap_summary(args):
    """Concurrency of a serving run from a rocprofv3 kernel and memory-copy
    trace: the hardware queues used, how long kernels and host-to-device
    copies were in flight, and how much of that time two or more of them ran
    at once (chunks of different beams overlapping on the device)."""
    kern = []
    for f in _csvs(args.trace, "kernel_trace.csv"):
        for row in csv.DictReader(open(f)):
            name = _short(row["Kernel_Name"])
            if not any(k in name for k in ("boxcar", "msd", "select", "fill_i64", "dedisp")):
                continue                  # the path's kernels only (not the workload generator's)
            kern.append((name, int(row["Start_Timestamp"]), int(row["End_Timestamp"]),
                         row.get("Queue_Id", ""), row.get("Stream_Id", "")))
    copies = []
    if kern:
        lo, hi = min(k[1] for k in kern), max(k[2] for k in kern)
        for f in _csvs(args.trace, "memory_copy_trace.csv"):
            for row in csv.DictReader(open(f)):
                a, b = int(row["Start_Timestamp"]), int(row["End_Timestamp"])
                if b >= lo and a <= hi:   # copies while the path ran
                    copies.append((row.get("Direction", row.get("Operation", "")), a, b))
    lines = ["# %s\n" % args.title, "command: `%s`\n" % args.command]
    if not kern:
        lines.append("no kernel trace found")
    else:
        t0 = min(k[1] for k in kern + [(0, c[1], c[2]) for c in copies])
        t1 = max(k[2] for k in kern + [(0, c[1], c[2]) for c in copies])
        ku, k2 = _busy([(k[1], k[2]) for k in kern])
        lines.append("| quantity | value |")
        lines.append("|---|---|")
        lines.append("| traced span | %.1f ms |" % ((t1 - t0) / 1e6))
        lines.append("| kernel dispatches | %d |" % len(kern))
        lines.append("| hardware queues used by kernels | %d (%s) |" % (
            len({k[3] for k in kern}), ", ".join(sorted({k[3] for k in kern}))))
        lines.append("| HIP streams used by kernels | %d |" % len({k[4] for k in kern}))
        lines.append("| time with a kernel running | %.1f ms |" % (ku / 1e6))
        lines.append("| time with two or more kernels running | %.1f ms (%.0f%% of the kernel time) |" % (
            k2 / 1e6, 100.0 * k2 / max(ku, 1)))
        h2d = [(c[1], c[2]) for c in copies if "HOST_TO_DEVICE" in c[0].upper() or "H2D" in c[0].upper()]
        if h2d:
            cu, c2 = _busy(h2d)
            both = _busy([(a, b) for a, b in h2d] + [(k[1], k[2]) for k in kern])
            lines.append("| host-to-device copies | %d, in flight %.1f ms, two or more at once %.1f ms |" % (
                len(h2d), cu / 1e6, c2 / 1e6))
            lines.append("| time with a copy or a kernel in flight | %.1f ms; copies and kernels at once %.1f ms |" % (
                both[0] / 1e6, (cu + ku - both[0]) / 1e6))
        lines.append("")
        lines.append("| kernel | dispatches | total ms |")
        lines.append("|---|---|---|")
        tot = defaultdict(lambda: [0, 0.0])
        for k in kern:
            tot[k[0]][0] += 1
            tot[k[0]][1] += (k[2] - k[1]) / 1e6
        for name, (n, ms) in sorted(tot.items(), key=lambda kv: -kv[1][1]):
            lines.append("| %s | %d | %.3f |" % (name, n, ms))
    lines.append("")
    path = os.path.join(args.out, args.name + ".md")
    with open(path, "w") as fh:
        fh.write("\n".join(lines))
    print("wrote", path)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--workload", default="ska", choices=sorted(WORKLOADS))
    r.add_argument("--steps", type=int, default=2)
    r.add_argument("--rows", type=int, default=4096)
    r.add_argument("--cols", type=int, default=1 << 20)
    s = sub.add_parser("summarize")
    s.add_argument("--trace")
    s.add_argument("--trace-cmd", default="")
    s.add_argument("--fetch")
    s.add_argument("--fetch-cmd", default="")
    s.add_argument("--write")
    s.add_argument("--write-cmd", default="")
    s.add_argument("--workload")
    s.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    s.add_argument("--name", required=True)
    s.add_argument("--title", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--dirs", nargs="+", required=True)
    c.add_argument("--cmds", nargs="*")
    c.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    c.add_argument("--name", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--workload", choices=sorted(WORKLOADS),
                   help="also write the boxcar kernel's VALU per evaluation to valu_counters.json")
    o = sub.add_parser("overlap")
    o.add_argument("--trace", required=True)
    o.add_argument("--command", default="")
    o.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    o.add_argument("--name", required=True)
    o.add_argument("--title", required=True)
    a = ap.parse_args(argv)
    {"run": run, "summarize": summarize, "counters": counter_summary, "overlap": overlap_summary}[a.cmd](a)


if __name__ == "__main__":
    sys.exit(main())
