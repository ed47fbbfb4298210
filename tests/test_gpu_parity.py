"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Rules (tests/spd_check.py): per-sample SNR within 1e-4; width equal or the
oracle's SNR at the GPU's width within 1e-4 of the oracle maximum; candidate
sets equal except within 1e-4 of the threshold; mean/sigma to 1e-6 relative.
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


def run_and_check(x, widths, thr, *, scope="row", mode="sqrtn", kappa=1.0, scale=None, zero=None,
                  fused=True, check_cands=True):
    print("case: shape=%s dtype=%s |W|=%d nmax=%d scope=%s mode=%s" % (tuple(x.shape), x.dtype, len(widths),
                                                                        widths[-1], scope, mode), flush=True)
    g = B.detect(x, widths, thr, scope=scope, sigma_mode=mode, kappa=kappa, scale=scale, zero=zero,
                 fused_select=fused)
    torch.cuda.synchronize()
    x64 = C.plane_f64(x, scale, zero)
    o = oracle.detect(x64, widths, thr, scope=scope, sigma_mode=mode, kappa=kappa)
    C.check_stats(g["stats"].cpu().numpy(), o["stats"], mode != "sqrtn")
    worst, nmis = C.check_snr_widx(x64, widths, g["snr"].cpu().numpy(), g["widx"].cpu().numpy(),
                                   o["snr"], o["widx"], o["stats"], scope=scope)
    if check_cands:
        C.check_candidates(g["cands"], o["cands"], thr, lambda r, t: o["snr"][r, t],
                           C.width_rule(x64, widths, o["stats"], scope=scope))
    return g, o, worst, nmis


def test_tiny_plane_parity_and_pulse_recovery():
    cfg = synth.tiny(device=DEV)
    x = cfg["plane"].x
    g, o, worst, nmis = run_and_check(x, cfg["widths"], cfg["threshold"])
    print("tiny: max|dSNR|=%.3g width mismatches=%d candidates=%d" % (worst, nmis, g["n_cands"]))
    for p in cfg["plane"].pulses:            # every injected pulse is detected near its start
        hit = [c for c in g["cands"] if c["row"] == p.row and abs(int(c["t"]) - p.t0) <= p.width]
        assert hit, "pulse %s not detected" % (p,)
        best = max(hit, key=lambda c: c["snr"])
        assert abs(best["snr"] - p.snr) < 4.0


def test_tiny_plane_scope_and_separate_select():
    cfg = synth.tiny(device=DEV, R=16, L=20000)
    x = cfg["plane"].x
    run_and_check(x, cfg["widths"], cfg["threshold"], scope="plane")
    run_and_check(x, cfg["widths"], cfg["threshold"], fused=False)


# select_candidates reads 4,096 columns per work-group, 16 per lane: whole
# chunks and a ragged tail, on aligned and unaligned row strides
@pytest.mark.parametrize("pad", [0, 4, 1])
def test_standalone_select_load_paths(pad):
    W = list(range(1, 33))
    x = synth.make_plane(5, 20031, seed=23, device=DEV, n_pulses=6, pulse_widths=[1, 4, 16, 32],
                         snr_range=(7, 20), t_margin=32).x
    p = B.Params(W, 3.0)                                       # a low threshold: many candidates
    nout = x.shape[1] - 31                                     # 20,000: 4 whole chunks and a tail
    stride = nout + pad
    print("case: select stride=%d" % stride, flush=True)
    stats = B.msd_compute(x, p)
    snr = torch.full((5, stride), -1.0, device=DEV)
    widx = torch.zeros((5, stride), dtype=torch.uint8, device=DEV)
    fused = B.new_candidates(1 << 16, DEV)
    n_fused = torch.zeros(1, dtype=torch.int64, device=DEV)
    B.boxcar_snr(x, p, stats, snr=snr[:, :nout], widx=widx[:, :nout], out_stride=stride, cand=fused,
                 cand_count=n_fused)
    alone = B.new_candidates(1 << 16, DEV)
    n_alone = torch.zeros(1, dtype=torch.int64, device=DEV)
    B.select_candidates(snr[:, :nout], widx[:, :nout], p, t_offset=17, cand=alone, cand_count=n_alone)
    torch.cuda.synchronize()
    nf, na = int(n_fused.item()), int(n_alone.item())
    assert nf == na and 0 < na < (1 << 16)
    key = lambda c: (int(c["row"]), int(c["t"]), int(c["width"]), float(c["snr"]))
    fused_set = {key(c) for c in B.candidates_to_numpy(fused, nf)}
    alone_set = {(r, t - 17, w, v) for r, t, w, v in (key(c) for c in B.candidates_to_numpy(alone, na))}
    assert alone_set == fused_set
    o = oracle.detect(x.cpu().double().numpy(), W, 3.0)
    ok = set(zip(o["cands"]["row"].tolist(), o["cands"]["t"].tolist()))
    got = {(r, t) for r, t, _, _ in alone_set}
    for k in got ^ ok:
        assert abs(o["snr"][k] - 3.0) <= C.TOL_SNR, "candidate mismatch at %s" % (k,)


@pytest.mark.parametrize("mode", ["linear", "auto", "linear_literal"])
def test_sigma_modes_with_signal_dominated_rows(mode):
    cfg = synth.ska(device=DEV, R=12, L=30000, n_pulses=6, n_bright=3)
    x = cfg["plane"].x
    widths = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64]
    run_and_check(x, widths, cfg["threshold"], mode=mode, kappa=1.0)


def test_ska_widths_small_plane():
    cfg = synth.ska(device=DEV, R=10, L=40000, n_pulses=8, n_bright=2)
    g, o, worst, nmis = run_and_check(cfg["plane"].x, cfg["widths"], cfg["threshold"], mode="auto")
    flags = B.stats_flags(g["stats"]).cpu().numpy()
    for r in cfg["plane"].bright_rows:
        assert flags[r] & B.FLAG_LINEAR


@pytest.mark.parametrize("widths", [
    [1, 2, 3, 5, 8, 13, 21, 34],          # irregular gaps: non-unit step counts
    [4, 8, 12, 16, 20],                   # first width > 1, even gaps
    [1, 2, 4, 8, 16, 32, 64, 128],        # geometric
    list(range(1, 17)) + list(range(18, 65, 2)),
    [7],
])
def test_width_lists(widths):
    x = synth.make_plane(5, 9001, seed=7, device=DEV, n_pulses=4, pulse_widths=range(1, 40),
                         snr_range=(8, 30), gap=64, t_margin=widths[-1]).x
    run_and_check(x, widths, 6.0)


# the widest boxcar the library takes (4,096 samples): 21 rows of 256 per statistics
# sub-tile, fewer waves per work-group to fit the LDS, and a boxcar window of 4,607 samples
@pytest.mark.parametrize("mode", ["sqrtn", "auto"])
@pytest.mark.parametrize("widths", [[1 << k for k in range(13)], [4096]])
def test_largest_widest_boxcar(widths, mode):
    x = synth.make_plane(3, 20011, seed=17, device=DEV, n_pulses=3, pulse_widths=[1, 300, 2500],
                         snr_range=(10, 25), gap=4200, t_margin=4096).x
    run_and_check(x, widths, 6.0, mode=mode)


# the widest-boxcar statistics (AUTO, LINEAR) take their own load and edge paths
@pytest.mark.parametrize("mode", ["sqrtn", "auto", "linear"])
def test_ragged_and_edge_shapes(mode):
    rng = np.random.default_rng(3)
    for R, L, W in [(1, 64, list(range(1, 65))), (3, 65, [1, 2, 3]), (2, 1, [1]), (7, 4099, [1, 5, 9]),
                    (1, 300, [300]), (2, 70000, [1, 2, 3, 4, 5, 6, 7]), (3, 5000, list(range(1, 17)))]:
        x = torch.from_numpy(rng.standard_normal((R, L)).astype(np.float32)).to(DEV)
        run_and_check(x, W, 2.5, mode=mode)


@pytest.mark.parametrize("mode", ["sqrtn", "auto", "linear"])
def test_unaligned_views_and_strides(mode):
    base = synth.make_plane(6, 12003, seed=11, device=DEV, n_pulses=3, pulse_widths=[3, 9, 20],
                            snr_range=(10, 20), t_margin=40).x
    run_and_check(base[:, 1:], list(range(1, 33)), 6.0, mode=mode)          # data pointer off by one element
    run_and_check(base[:, 3:11000], [1, 2, 4, 8, 16, 32], 6.0, mode=mode)    # odd stride and length
    run_and_check(base[:, 2:], [1, 3, 5, 7, 9, 11, 13], 6.0, mode=mode)     # Nmax not a multiple of 4


def test_zero_variance_row_and_canary():
    x = torch.randn(4, 5000, device=DEV)
    x[2] = 3.25
    p = B.Params(list(range(1, 17)), 5.0)
    stats = B.msd_compute(x, p)
    nout = 5000 - 15
    pad = 37
    snr = torch.full((4, nout + pad), 123.0, device=DEV)
    widx = torch.full((4, nout + pad), 77, dtype=torch.uint8, device=DEV)
    B.boxcar_snr(x, p, stats, snr=snr[:, :nout], widx=widx[:, :nout], out_stride=nout + pad)
    torch.cuda.synchronize()
    assert int(B.stats_flags(stats)[2]) & B.FLAG_ZERO_VAR
    assert torch.all(snr[2, :nout] == 0) and torch.all(widx[2, :nout] == 0)
    assert torch.all(snr[:, nout:] == 123.0) and torch.all(widx[:, nout:] == 77)


def test_candidate_overflow_reports_total():
    x = synth.make_plane(4, 20000, seed=5, device=DEV).x
    p = B.Params([1, 2, 4], 1.5)
    stats = B.msd_compute(x, p)
    count = torch.zeros(1, dtype=torch.int64, device=DEV)
    small = B.new_candidates(100, DEV)
    B.boxcar_snr(x, p, stats, cand=small, cand_count=count)
    n = int(count.item())
    assert n > 100
    big = B.new_candidates(n, DEV)
    B.boxcar_snr(x, p, stats, cand=big, cand_count=count)
    assert int(count.item()) == n
    all_c = {(int(c["row"]), int(c["t"])) for c in B.candidates_to_numpy(big, n)}
    some = B.candidates_to_numpy(small, 100)
    assert len(some) == 100 and {(int(c["row"]), int(c["t"])) for c in some} <= all_c


def test_determinism():
    cfg = synth.tiny(device=DEV, R=8, L=30000)
    a = B.detect(cfg["plane"].x, cfg["widths"], 4.0)
    b = B.detect(cfg["plane"].x, cfg["widths"], 4.0)
    assert torch.equal(a["snr"], b["snr"]) and torch.equal(a["widx"], b["widx"])
    assert torch.equal(a["stats"], b["stats"])
    ka = sorted((int(c["row"]), int(c["t"]), float(c["snr"])) for c in a["cands"])
    kb = sorted((int(c["row"]), int(c["t"]), float(c["snr"])) for c in b["cands"])
    assert ka == kb


# "+1": the plane viewed from its second column, so no row starts on a
# 4-element boundary and the statistics align their vector loads per row
@pytest.mark.parametrize("form", ["f16", "u8", "f16+1", "u8+1"])
def test_precision_forms_parity(form):
    cfg = synth.tiny(device=DEV, R=16, L=30000)
    x32 = cfg["plane"].x
    if form.startswith("f16"):
        x, scale, zero = synth.quantize_f16(x32), None, None
    else:
        x, scale, zero = synth.quantize_u8(x32, cfg["plane"].row_sigma)
    if form.endswith("+1"):
        x = x[:, 1:]
    run_and_check(x, cfg["widths"], cfg["threshold"], scale=scale, zero=zero)
    if form.endswith("+1"):
        run_and_check(x, cfg["widths"], cfg["threshold"], scale=scale, zero=zero, mode="auto")


@pytest.mark.parametrize("form", ["f16", "u8"])
def test_precision_forms_full_tiny_plane(form):
    """The precision form at its full size: the 64 x 65,536 tiny plane (five
    pulses, widths 1..32, sqrt(N) sigma, threshold 6) stored as FP16 and as
    U8 (20 counts per sigma), every output against the oracle on the stored
    values, and the pulses still recovered."""
    cfg = synth.tiny(device=DEV)
    x32 = cfg["plane"].x
    if form == "f16":
        x, scale, zero = synth.quantize_f16(x32), None, None
    else:
        x, scale, zero = synth.quantize_u8(x32, cfg["plane"].row_sigma)
    g, o, worst, _ = run_and_check(x, cfg["widths"], cfg["threshold"], scale=scale, zero=zero)
    for pu in cfg["plane"].pulses:           # every injected pulse is still detected near its start
        hit = [c for c in g["cands"] if c["row"] == pu.row and abs(int(c["t"]) - pu.t0) <= pu.width]
        assert hit, "pulse %s not detected" % (pu,)


@pytest.mark.parametrize("mode", ["sqrtn", "linear"])
def test_streaming_accumulate_matches_oracle(mode):
    rng = np.random.default_rng(21)
    R, Lc, K = 6, 5000, 4
    W = list(range(1, 33))
    nmax = W[-1]
    full = rng.standard_normal((R, Lc * K)).astype(np.float32) + 3.0
    full[1, Lc - 10:Lc + 12] += 2.5
    xs = torch.from_numpy(full).to(DEV)
    p = B.Params(W, 6.0, sigma_mode=mode)
    state = torch.zeros((R, 6), dtype=torch.float64, device=DEV)
    ostate = None
    for k in range(K):
        lo = 0 if k == 0 else k * Lc - (nmax - 1)
        view = xs[:, lo:(k + 1) * Lc]
        ncb = 0 if k == 0 else nmax - 1
        stats = B.msd_compute(view, p, new_col_begin=ncb, accumulate=k > 0, state=state)
        nout = view.shape[1] - nmax + 1
        snr = torch.empty((R, nout), device=DEV)
        widx = torch.empty((R, nout), dtype=torch.uint8, device=DEV)
        B.boxcar_snr(view, p, stats, snr=snr, widx=widx, t_offset=lo)
        torch.cuda.synchronize()
        v64 = full[:, lo:(k + 1) * Lc].astype(np.float64)
        ostate, ost, osnr, owidx = oracle.stream_step(v64, W, new_col_begin=ncb, state=ostate, sigma_mode=mode)
        np.testing.assert_allclose(state.cpu().numpy()[:, [0, 3]], ostate[:, [0, 3]])
        C.check_stats(stats.cpu().numpy(), ost, mode != "sqrtn")
        C.check_snr_widx(v64, W, snr.cpu().numpy(), widx.cpu().numpy(), osnr, owidx, ost)


def test_ska_full_size_sampled_rows():
    """The 4,096 x 2^20 SKA-like plane at full size, in the launch
    configuration the benchmark times; rows sampled for the oracle (signal-
    dominated rows, pulse rows, random rows)."""
    cfg = synth.ska(device=DEV)
    pl = cfg["plane"]
    x = pl.x
    W = cfg["widths"]
    print("ska full: generated", flush=True)
    g = B.detect(x, W, cfg["threshold"], sigma_mode="auto", kappa=1.0, capacity=1 << 20)
    torch.cuda.synchronize()
    rng = np.random.default_rng(99)
    rows = sorted(set(pl.bright_rows) | {p.row for p in pl.pulses[:8]} |
                  set(rng.choice(x.shape[0], 6, replace=False).tolist()))
    x64 = x[rows].cpu().to(torch.float64).numpy()
    _, ost, osnr, owidx = oracle.stream_step(x64, W, sigma_mode="auto", kappa=1.0)
    gst = g["stats"][rows].cpu().numpy()
    C.check_stats(gst, ost, True)
    worst, nmis = C.check_snr_widx(x64, W, g["snr"][rows].cpu().numpy(), g["widx"][rows].cpu().numpy(),
                                   osnr, owidx, ost, rows=rows)
    print("ska full: rows=%d max|dSNR|=%.3g width mismatches=%d candidates=%d" %
          (len(rows), worst, nmis, g["n_cands"]), flush=True)
    oc = oracle.select(osnr, owidx, W, cfg["threshold"])
    oc["row"] = np.asarray(rows)[oc["row"]]
    rset = set(rows)
    gc = np.array([c for c in g["cands"] if int(c["row"]) in rset], dtype=B.CANDIDATE_DTYPE)
    C.check_candidates(gc, oc, cfg["threshold"], lambda r, t: osnr[rows.index(r), t],
                       C.width_rule(x64, W, ost, rows=rows))
    del g, x
    torch.cuda.empty_cache()


def test_ska_full_size_bench_layout_all_forms():
    """The 4,096 x 2^20 SKA-like plane in exactly the launch configuration the
    benchmark times: msd_compute then boxcar_snr into output rows padded to
    64-byte multiples (the vector-store path), with the fused candidate list,
    for the 136-width list and for widths 1..16 (the streaming form), with the
    plane stored as FP32, FP16 and U8 (per-row zero at the row mean, as the
    benchmark's precision leg stores it); sampled rows against the oracle on
    the stored values, and those rows' candidates against the oracle's."""
    cfg = synth.ska(device=DEV)
    pl = cfg["plane"]
    xs = pl.x
    R, L = xs.shape
    print("ska bench layout: generated", flush=True)
    rng = np.random.default_rng(123)
    rows = sorted(set(pl.bright_rows[:4]) | {p.row for p in pl.pulses[8:14]} |
                  set(rng.choice(R, 4, replace=False).tolist()))
    q, sc, zr = synth.quantize_u8(xs, pl.row_sigma, row_mu=pl.row_mu)
    forms = {"f32": (xs, None, None), "f16": (synth.quantize_f16(xs), None, None), "u8": (q, sc, zr)}
    flat_snr = torch.empty(R * L, dtype=torch.float32, device=DEV)
    flat_widx = torch.empty(R * L, dtype=torch.uint8, device=DEV)
    for name, (x, s_, z_) in forms.items():
        x64 = C.plane_f64(x[rows], None if s_ is None else s_[rows], None if z_ is None else z_[rows])
        for W in (cfg["widths"], list(range(1, 17))):
            p = B.Params(W, cfg["threshold"], "row", "auto", 1.0)
            nout = L - p.nmax + 1
            po = (nout + 15) // 16 * 16
            snr = flat_snr[:R * po].view(R, po)[:, :nout]
            widx = flat_widx[:R * po].view(R, po)[:, :nout]
            cand = B.new_candidates(1 << 21, DEV)
            cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
            stats = B.msd_compute(x, p, scale=s_, zero=z_)
            B.boxcar_snr(x, p, stats, scale=s_, zero=z_, snr=snr, widx=widx, cand=cand, cand_count=cnt)
            torch.cuda.synchronize()
            n = int(cnt.item())
            assert n <= cand.shape[0]
            _, ost, osnr, owidx = oracle.stream_step(x64, W, sigma_mode="auto", kappa=1.0)
            C.check_stats(stats[rows].cpu().numpy(), ost, True)
            worst, nmis = C.check_snr_widx(x64, W, snr[rows].cpu().numpy(), widx[rows].cpu().numpy(), osnr,
                                           owidx, ost, rows=rows)
            oc = oracle.select(osnr, owidx, W, cfg["threshold"])
            oc["row"] = np.asarray(rows)[oc["row"]]
            rset = set(rows)
            gc = np.array([c for c in B.candidates_to_numpy(cand, n) if int(c["row"]) in rset],
                          dtype=B.CANDIDATE_DTYPE)
            C.check_candidates(gc, oc, cfg["threshold"], lambda r, t: osnr[rows.index(r), t],
                               C.width_rule(x64, W, ost, rows=rows))
            print("ska bench layout %s |W|=%d: rows=%d max|dSNR|=%.3g width mismatches=%d candidates=%d" %
                  (name, len(W), len(rows), worst, nmis, n), flush=True)
    del xs, forms, q, flat_snr, flat_widx
    torch.cuda.empty_cache()
