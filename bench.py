#!/usr/bin/env python3
"""Throughput of the single-pulse detection path on one MI355X.

A step is one pass of the whole path over one synthetic plane already resident
in HBM: msd_compute (per-row mean / sigma, plus sigma of the widest boxcar for
the linear sigma_N correction) then boxcar_snr (every width at every sample,
highest SNR and its width written out, fused SNR threshold into the candidate
list).  The workload is the SKA-like plane: 4,096 DM trials x 2^20 samples
FP32, per-row offsets and scales, 200 pulses, 8 signal-dominated rows, widths
1..16 then 18..256 step 2, threshold 7, AUTO sigma_N (kappa = 1).

Prints one JSON line.  ``value`` is input samples (DM x time) per second over
the K timed steps; ``roofline`` refers to the dominant kernel (boxcar_snr);
``cpu_baseline`` is the FP64 oracle on a sample of the same rows, on this
host's cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "boxcar-SNR GSamples/s (DM×time) & % HBM roofline; p99 chunk latency"
HBM_PEAK_GBS = 8000.0
# FP32 vector lanes: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one add / mul / max
# per lane per clock (no FMA pairing, no packed math in this kernel).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
OPS_PER_EVAL = 3          # boxcar add, SNR multiply, running-max compare per (t, w)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1611_09704_amd", "csrc")
    for f in ("spd_device.h", "spd_kernels.hip", "spd_kernels.h", "spd_internal.h"):   # device code
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(workload: str):
    """HBM bytes per launch from committed rocprofv3 counters, if they were
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "boxcar_traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    e = d.get(workload)
    if not e or e.get("kernel_sha") != kernel_source_sha():
        return None
    return e.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rows", type=int, default=4096)
    ap.add_argument("--cols", type=int, default=1 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--workload", default="ska", choices=["ska", "ska16"],
                    help="ska: widths 1..16,18..256/2 (default); ska16: the same plane with widths 1..16 only")
    ap.add_argument("--form", default="plain", choices=["plain", "batch"],
                    help="plain: the SKA-like plane (default); batch: 48 uneven beams in one persistent, "
                         "graph-replayed launch per step, against per-beam plain launches")
    ap.add_argument("--batch-samples", type=float, default=40e9,
                    help="cap on the batched workload's total samples (the beam draw is re-seeded until it fits)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build runs the path on a single MI355X "
              "(rows and beams are independent, so N GPUs would each take 1/N of the rows); "
              "--gpus %d is not supported" % max(args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1611_09704_amd import binding as B
    from paper_1611_09704_amd import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.form == "batch":
        print(json.dumps(run_batch(args, dev)), flush=True)
        return
    cfg = synth.ska(device=dev, R=args.rows, L=args.cols)
    x = cfg["plane"].x
    R, L = x.shape
    W = cfg["widths"] if args.workload == "ska" else list(range(1, 17))
    p = B.Params(W, cfg["threshold"], "row", cfg["sigma_mode"], cfg["kappa"])
    nout = L - p.nmax + 1
    stats = torch.empty((R, B.STATS_FIELDS), dtype=torch.float64, device=dev)
    ws = torch.empty(B.workspace_bytes(x, p), dtype=torch.uint8, device=dev)
    snr_flat = torch.empty(R * L, dtype=torch.float32, device=dev)
    widx_flat = torch.empty(R * L, dtype=torch.uint8, device=dev)
    cap = 1 << 21
    cand = B.new_candidates(cap, dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    def timed(params, K, Wm):
        """K steps of msd_compute + boxcar_snr after Wm warm-up steps; returns
        wall seconds and the mean duration of each call (HIP events on the
        launch stream)."""
        no = L - params.nmax + 1
        s_out = snr_flat[:R * no].view(R, no)
        w_out = widx_flat[:R * no].view(R, no)

        def one(evs=None):
            if evs: evs[0].record(stream)
            B.msd_compute(x, params, stats=stats, workspace=ws, stream=stream)
            if evs: evs[1].record(stream)
            B.boxcar_snr(x, params, stats, snr=s_out, widx=w_out, cand=cand, cand_count=count, stream=stream)
            if evs: evs[2].record(stream)

        for _ in range(Wm):
            one()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
        t0 = time.perf_counter()
        for k in range(K):
            one(evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        msd_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / K
        box_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / K
        return wall, msd_ms, box_ms

    wall, msd_ms, box_ms = timed(p, args.steps, args.warmup)
    n_cand = int(count.item())
    if n_cand > cap:
        print("warning: %d candidates exceed the list capacity %d" % (n_cand, cap), file=sys.stderr)
    samples = R * L
    value = samples * args.steps / wall / 1e9
    evals = R * nout * len(W)
    box_tops = evals * OPS_PER_EVAL / (box_ms * 1e-3) / 1e12
    box_bytes = R * L * 4 + R * nout * 5
    msd_bytes = R * L * 4
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GSamples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg["name"] + ("" if args.workload == "ska" else " widths 1..16"), "rows": R,
                   "cols": L, "widths": "1..16,18..256/2" if args.workload == "ska" else "1..16",
                   "n_widths": len(W), "threshold": cfg["threshold"], "sigma_mode": "auto", "kappa": 1.0,
                   "scope": "row", "outputs": "snr f32 + width u8 per sample, fused candidate list"},
        "roofline": {"bound": "alu", "achieved": round(box_tops, 3), "peak": round(VALU_PEAK_TOPS, 2),
                     "unit": "TFLOP/s", "frac": round(box_tops / VALU_PEAK_TOPS, 4),
                     "traffic": load_traffic(args.workload), "kernel": "boxcar_kernel",
                     "work_per_launch": "%d (t,w) evaluations x %d FP32 ops" % (evals, OPS_PER_EVAL)},
        "kernels": {
            "msd_compute": {"ms": round(msd_ms, 4), "GB/s": round(msd_bytes / msd_ms / 1e6, 1),
                            "hbm_frac": round(msd_bytes / msd_ms / 1e6 / HBM_PEAK_GBS, 4)},
            "boxcar_snr": {"ms": round(box_ms, 4), "GB/s": round(box_bytes / box_ms / 1e6, 1),
                           "hbm_frac": round(box_bytes / box_ms / 1e6 / HBM_PEAK_GBS, 4),
                           "valu_frac": round(box_tops / VALU_PEAK_TOPS, 4)},
        },
        "n_candidates": n_cand,
        "kernel_sha": kernel_source_sha(),
    }

    if not args.no_secondary and args.workload == "ska":
        # the paper's own measurement setting: widths 1..16 on the same plane
        p16 = B.Params(list(range(1, 17)), cfg["threshold"], "row", "auto", 1.0)
        w16, m16, b16 = timed(p16, args.steps, args.warmup)
        bb16 = R * L * 4 + R * (L - 15) * 5
        out["secondary"] = {
            "workload": cfg["name"] + " widths 1..16", "value": round(samples * args.steps / w16 / 1e9, 3),
            "unit": "GSamples/s", "ms_per_step": round(w16 / args.steps * 1e3, 3),
            "roofline": {"bound": "hbm", "achieved": round(bb16 / b16 / 1e6, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(bb16 / b16 / 1e6 / HBM_PEAK_GBS, 4),
                         "traffic": load_traffic("ska16"), "kernel": "boxcar_kernel"},
            "msd_ms": round(m16, 4), "boxcar_ms": round(b16, 4),
            "msd_hbm_frac": round(msd_bytes / m16 / 1e6 / HBM_PEAK_GBS, 4),
        }

    if not args.no_cpu_baseline:
        import oracle
        cores = len(os.sched_getaffinity(0))
        nrows = max(8, min(64, 2 * cores))
        rows = np.linspace(0, R - 1, nrows).astype(np.int64)
        x64 = x[torch.as_tensor(rows, device=dev)].cpu().double().numpy()
        t0 = time.perf_counter()
        oracle.stream_step(x64, W, sigma_mode="auto", kappa=1.0, nthreads=cores)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(nrows * L / dt / 1e9, 5), "unit": "GSamples/s", "cores": cores,
                               "kind": "oracle",
                               "sample": "%d of %d rows x %d samples, same widths / AUTO sigma_N, FP64, "
                                         "%.1f s wall" % (nrows, R, L, dt)}
    print(json.dumps(out), flush=True)


def run_batch(args, dev):
    """Batched workload: 48 beams, rows from {256..4096}, 2^16..2^21 samples,
    N(0,1), 20 pulses per beam (widths 1..128, SNR 6-30), widths 1..128,
    threshold 7, candidates only.  Times the batched plan (autotuned schedule,
    hipGraph replay) and, on the same beams, per-beam plain launches."""
    import torch

    from paper_1611_09704_amd import binding as B
    from paper_1611_09704_amd import synth
    cfg = synth.batch(device=dev, max_samples=int(args.batch_samples))
    planes = [pl.x for pl in cfg["planes"]]
    W = cfg["widths"]
    p = B.Params(W, cfg["threshold"])
    samples = sum(x.numel() for x in planes)
    evals = sum(x.shape[0] * (x.shape[1] - W[-1] + 1) for x in planes) * len(W)
    cap = 1 << 23
    cand = B.new_candidates(cap, dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    # per-beam plain launches
    stats = [torch.empty((x.shape[0], B.STATS_FIELDS), dtype=torch.float64, device=dev) for x in planes]
    wss = [torch.empty(B.workspace_bytes(x, p), dtype=torch.uint8, device=dev) for x in planes]

    def plain_step():
        n = 0
        for x, st, ws in zip(planes, stats, wss):
            B.msd_compute(x, p, stats=st, workspace=ws, stream=stream)
            B.boxcar_snr(x, p, st, cand=cand, cand_count=count, stream=stream)
        return n

    plain_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain_step()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / args.steps
    # batched plan
    t0 = time.perf_counter()
    os.environ.setdefault("SPD_TUNE_CACHE", os.path.join("/tmp", "spd_bench_schedule_%d.txt" % os.getpid()))
    plan = B.BatchPlan(planes, p, autotune=True)
    t_create = time.perf_counter() - t0
    for _ in range(max(1, args.warmup)):
        plan.run(cand, count, use_graph=True, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.run(cand, count, use_graph=True, stream=stream)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    n_cand = int(count.item())
    info = plan.describe()
    table = plan.tune_table()
    plan.close()
    tops = evals * OPS_PER_EVAL / t_batch / 1e12
    return {
        "metric": METRIC, "value": round(samples / t_batch / 1e9, 3), "unit": "GSamples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t_batch * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": cfg["name"], "beams": len(planes), "samples": samples, "widths": "1..128",
                   "threshold": cfg["threshold"], "sigma_mode": "sqrtn", "outputs": "candidates only",
                   "shapes": cfg["shapes"]},
        "roofline": {"bound": "alu", "achieved": round(tops, 3), "peak": round(VALU_PEAK_TOPS, 2),
                     "unit": "TFLOP/s", "frac": round(tops / VALU_PEAK_TOPS, 4), "traffic": None,
                     "kernel": "whole batched step (msd + finalize + boxcar) from wall time"},
        "plain_per_beam": {"value": round(samples / t_plain / 1e9, 3), "unit": "GSamples/s",
                           "ms_per_step": round(t_plain * 1e3, 3)},
        "speedup_vs_plain": round(t_plain / t_batch, 4),
        "schedule": info, "autotune_table": table, "plan_create_s": round(t_create, 3), "n_candidates": n_cand,
    }


if __name__ == "__main__":
    main()
