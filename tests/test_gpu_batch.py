"""Batched form: many beams of uneven shape in one persistent launch.

Checked against per-beam plain launches of the same ABI, against the FP64
oracle (tests/spd_check.py rules), across hipGraph replays with other work in
between, and at the full batched workload size on sampled rows.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1611_09704_amd import binding as B
from paper_1611_09704_amd import synth
import spd_check as C

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _cands_by_beam(c):
    out = {}
    for x in c:
        out.setdefault(int(x["beam"]), []).append(x)
    return {k: np.array(v, dtype=B.CANDIDATE_DTYPE) for k, v in out.items()}


def _batch_run(plan, cap=1 << 16, graph=False):
    count = torch.zeros(1, dtype=torch.int64, device=DEV)
    while True:
        cand = B.new_candidates(cap, DEV)
        plan.run(cand, count, use_graph=graph)
        n = int(count.item())
        if n <= cap:
            return B.candidates_to_numpy(cand, n)
        cap = n


SHAPES = [(3, 5000), (8, 9001), (17, 20000), (1, 300), (5, 70001), (2, 4096), (11, 12345)]


@pytest.mark.parametrize("widths,mode", [(list(range(1, 33)), "sqrtn"), (synth.SKA_WIDTHS[:40], "auto"),
                                         ([1, 2, 3, 5, 8, 13, 21], "linear")])
def test_batch_matches_plain_and_oracle(widths, mode):
    print("case: batch widths=%d mode=%s" % (len(widths), mode), flush=True)
    cfg = synth.batch(device=DEV, shapes=SHAPES, pulses_per_beam=3, wmax=widths[-1])
    planes = [pl.x for pl in cfg["planes"]]
    p = B.Params(widths, 5.0, "row", mode, 0.5)
    plan = B.BatchPlan(planes, p, autotune=False)
    # the register-window form is the default wherever the width list is made of stepped groups
    assert plan.describe()["window"] == (0 if widths[3] == 5 else 1)
    got = _cands_by_beam(_batch_run(plan))
    for b, x in enumerate(planes):
        plain = B.detect(x, widths, 5.0, sigma_mode=mode, kappa=0.5)
        st_b = plan.stats(b).cpu().numpy()
        st_p = plain["stats"].cpu().numpy()
        # both are within 1e-6 of the oracle (different FP32 block sizes): 2e-6 between them
        sig = st_p[:, 1]
        assert np.all(np.abs(st_b[:, 0] - st_p[:, 0]) <= 2e-6 * sig)
        np.testing.assert_allclose(st_b[:, 1:3], st_p[:, 1:3], rtol=2e-6)
        assert np.all(np.abs(st_b[:, 3] - st_p[:, 3]) <= 2e-6 * sig)
        x64 = x.cpu().double().numpy()
        o = oracle.detect(x64, widths, 5.0, sigma_mode=mode, kappa=0.5)
        C.check_stats(st_b, o["stats"], mode != "sqrtn")
        gb = got.get(b, np.zeros(0, dtype=B.CANDIDATE_DTYPE))
        wr = C.width_rule(x64, widths, o["stats"])
        C.check_candidates(gb, o["cands"], 5.0, lambda r, t: o["snr"][r, t], wr)
        C.check_candidates(gb, {"row": plain["cands"]["row"], "t": plain["cands"]["t"],
                                "snr": plain["cands"]["snr"], "width": plain["cands"]["width"]},
                           5.0, lambda r, t: o["snr"][r, t], wr)
    plan.close()


@pytest.mark.parametrize("form", ["f16", "u8"])
def test_batch_precision_forms(form):
    """FP16 and per-row U8 beams (uneven, mostly unaligned rows) in one plan:
    every beam against the oracle on the values stored, and against plain
    launches of the same beam."""
    print("case: batch form=%s" % form, flush=True)
    widths, thr = list(range(1, 33)), 5.0
    cfg = synth.batch(device=DEV, shapes=SHAPES, pulses_per_beam=3, wmax=widths[-1])
    beams = []
    for pl in cfg["planes"]:
        if form == "f16":
            beams.append((synth.quantize_f16(pl.x), None, None))
        else:
            beams.append(synth.quantize_u8(pl.x, pl.row_sigma))
    p = B.Params(widths, thr, "row", "auto", 1.0)
    plan = B.BatchPlan([b if form == "u8" else b[0] for b in beams], p, autotune=False)
    got = _cands_by_beam(_batch_run(plan))
    for b, (x, sc, z) in enumerate(beams):
        x64 = C.plane_f64(x, sc, z)
        o = oracle.detect(x64, widths, thr, sigma_mode="auto", kappa=1.0)
        C.check_stats(plan.stats(b).cpu().numpy(), o["stats"], True)
        gb = got.get(b, np.zeros(0, dtype=B.CANDIDATE_DTYPE))
        wr = C.width_rule(x64, widths, o["stats"])
        C.check_candidates(gb, o["cands"], thr, lambda r, t: o["snr"][r, t], wr)
        plain = B.detect(x, widths, thr, sigma_mode="auto", kappa=1.0, scale=sc, zero=z)
        C.check_candidates(gb, {"row": plain["cands"]["row"], "t": plain["cands"]["t"],
                                "snr": plain["cands"]["snr"], "width": plain["cands"]["width"]},
                           thr, lambda r, t: o["snr"][r, t], wr)
    plan.close()


def test_batch_graph_replays_match_eager():
    cfg = synth.batch(device=DEV, shapes=SHAPES, pulses_per_beam=4, wmax=64)
    planes = [pl.x for pl in cfg["planes"]]
    p = B.Params(list(range(1, 65)), 5.0)
    plan = B.BatchPlan(planes, p, autotune=False)
    eager = sorted((int(c["beam"]), int(c["row"]), int(c["t"]), float(c["snr"])) for c in _batch_run(plan))
    cap = len(eager) + 16
    cand = B.new_candidates(cap, DEV)
    count = torch.zeros(1, dtype=torch.int64, device=DEV)
    for rep in range(4):
        plan.run(cand, count, use_graph=True)
        torch.cuda.synchronize()
        got = sorted((int(c["beam"]), int(c["row"]), int(c["t"]), float(c["snr"]))
                     for c in B.candidates_to_numpy(cand, int(count.item())))
        assert got == eager, "graph replay %d differs" % rep
        B.detect(planes[rep % len(planes)], [1, 2, 4], 3.0)      # other work between replays
        cand.zero_()
    plan.close()


def test_batch_autotuned_schedule_gives_same_results(tmp_path, monkeypatch):
    monkeypatch.setenv("SPD_TUNE_CACHE", str(tmp_path / "sched.txt"))
    cfg = synth.batch(device=DEV, shapes=SHAPES, pulses_per_beam=3, wmax=32)
    planes = [pl.x for pl in cfg["planes"]]
    p = B.Params(list(range(1, 33)), 5.0)
    base = B.BatchPlan(planes, p, autotune=False)
    tuned = B.BatchPlan(planes, p, autotune=True)
    info = tuned.describe()
    assert info["tuned"] == 1 and info["out_per_lane"] in (4, 8)
    table = tuned.tune_table()
    assert any(r["window"] for r in table) and any(not r["window"] for r in table)
    again = B.BatchPlan(planes, p, autotune=True)
    assert again.describe()["tuned"] == 2                       # from the cache
    ka = sorted((int(c["beam"]), int(c["row"]), int(c["t"]), float(c["snr"])) for c in _batch_run(base))
    kb = sorted((int(c["beam"]), int(c["row"]), int(c["t"]), float(c["snr"])) for c in _batch_run(tuned))
    assert ka == kb
    for pl in (base, tuned, again):
        pl.close()


def test_batch_full_size_sampled_rows():
    """The batched workload (48 beams, rows from {256..4096}, 2^16..2^21
    samples, widths 1..128, threshold 7) at full size, in the schedule the
    benchmark uses; sampled rows of sampled beams checked against the oracle."""
    cfg = synth.batch(device=DEV, max_samples=int(40e9))
    planes = [pl.x for pl in cfg["planes"]]
    W = cfg["widths"]
    print("batch full: %d beams, %.2f G samples" % (len(planes), sum(x.numel() for x in planes) / 1e9), flush=True)
    p = B.Params(W, cfg["threshold"])
    plan = B.BatchPlan(planes, p, autotune=True)
    cands = _cands_by_beam(_batch_run(plan, cap=1 << 22, graph=True))
    rng = np.random.default_rng(5)
    for b in sorted(rng.choice(len(planes), 6, replace=False).tolist()):
        x = planes[b]
        rows = sorted(set([p_.row for p_ in cfg["planes"][b].pulses[:3]] + rng.choice(x.shape[0], 2).tolist()))
        x64 = x[rows].cpu().double().numpy()
        _, ost, osnr, owidx = oracle.stream_step(x64, W)
        C.check_stats(plan.stats(b).cpu().numpy()[rows], ost, False)
        oc = oracle.select(osnr, owidx, W, cfg["threshold"])
        oc["row"] = np.asarray(rows)[oc["row"]]
        gb = cands.get(b, np.zeros(0, dtype=B.CANDIDATE_DTYPE))
        gb = gb[np.isin(gb["row"], rows)]
        C.check_candidates(gb, oc, cfg["threshold"], lambda r, t: osnr[rows.index(r), t],
                           C.width_rule(x64, W, ost, rows=rows))
        print("beam %d rows %s: %d candidates ok" % (b, rows, len(gb)), flush=True)
    plan.close()
    del planes, cfg
    torch.cuda.empty_cache()
