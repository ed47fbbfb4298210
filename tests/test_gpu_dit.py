"""Boxcars combined with decimation in time on the GPU (boxcar_snr_dit)
against the decimated FP64 oracle (oracle.dit_detect), with the parity rules
of tests/spd_check.py, plus:

* the width the GPU reports at t must be one the decimated search evaluates
  at t (its decimation step divides t);
* with no decimated level it is boxcar_snr over 1..16, bit for bit;
* it never beats the exhaustive GPU path over the same width list by more
  than the FP32 budget, and matches it on the coarsest grid.
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


def run_dit(x, levels, thr, mode="sqrtn", scope="row", scale=None, zero=None, stride_pad=0, cap=1 << 18):
    p = B.dit_params(levels, thr, scope, mode, 1.0)
    stats = B.msd_compute(x, p, scale=scale, zero=zero)
    R = x.shape[0]
    nout = x.shape[1] - p.nmax + 1
    stride = nout + stride_pad
    snr = torch.full((R, stride), -5.0, device=DEV)
    widx = torch.full((R, stride), 222, dtype=torch.uint8, device=DEV)
    cand = B.new_candidates(cap, DEV)
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    B.boxcar_snr_dit(x, p, levels, stats, scale=scale, zero=zero, snr=snr[:, :nout], widx=widx[:, :nout],
                     out_stride=stride, cand=cand, cand_count=cnt)
    torch.cuda.synchronize()
    n = int(cnt.item())
    assert n <= cap
    if stride_pad:
        assert torch.all(snr[:, nout:] == -5.0) and torch.all(widx[:, nout:] == 222)
    return p, stats, snr[:, :nout], widx[:, :nout], B.candidates_to_numpy(cand, n)


def check_against_oracle(x, levels, thr, mode="sqrtn", scope="row", scale=None, zero=None, stride_pad=0):
    print("case: dit shape=%s dtype=%s levels=%d mode=%s scope=%s" % (tuple(x.shape), x.dtype, levels, mode, scope),
          flush=True)
    p, stats, snr, widx, cands = run_dit(x, levels, thr, mode, scope, scale, zero, stride_pad)
    x64 = C.plane_f64(x, scale, zero)
    o = oracle.dit_detect(x64, levels, thr, scope=scope, sigma_mode=mode, kappa=1.0)
    C.check_stats(stats.cpu().numpy(), o["stats"], mode != "sqrtn")
    w = np.asarray(o["widths"])
    strides = np.asarray(o["strides"])
    g_snr, g_idx = snr.cpu().numpy(), widx.cpu().numpy().astype(np.int64)
    t = np.arange(g_snr.shape[1])
    assert np.all(t[None, :] % strides[g_idx] == 0), "a reported width is not evaluated at its start"
    worst, nmis = C.check_snr_widx(x64, o["widths"], g_snr, g_idx, o["snr"], o["widx"], o["stats"], scope=scope)
    C.check_candidates(cands, o["cands"], thr, lambda r, tt: o["snr"][r, tt],
                       C.width_rule(x64, o["widths"], o["stats"], scope=scope, strides=o["strides"]))
    print("dit: max|dSNR|=%.3g width mismatches=%d candidates=%d" % (worst, nmis, len(cands)), flush=True)
    return p, snr, widx, cands


@pytest.mark.parametrize("levels", [0, 1, 2, 3, 4])
def test_dit_matches_oracle(levels):
    cfg = synth.make_plane(6, 21011, seed=60 + levels, device=DEV, n_pulses=8,
                           pulse_widths=range(1, (16 << levels) + 1), snr_range=(8, 40), gap=(16 << levels) + 8,
                           t_margin=16 << levels)
    check_against_oracle(cfg.x, levels, 6.0)


def test_dit_sigma_modes_and_signal_dominated_rows():
    cfg = synth.ska(device=DEV, R=8, L=30000, n_pulses=6, n_bright=3)
    check_against_oracle(cfg["plane"].x, 4, 7.0, mode="auto")
    check_against_oracle(cfg["plane"].x, 3, 7.0, mode="linear")


def test_dit_precision_forms_plane_scope_and_padding():
    cfg = synth.tiny(device=DEV, R=8, L=30011)
    x32 = cfg["plane"].x
    check_against_oracle(synth.quantize_f16(x32), 3, 6.0)
    q, s, z = synth.quantize_u8(x32, cfg["plane"].row_sigma)
    check_against_oracle(q, 2, 6.0, scale=s, zero=z)
    check_against_oracle(x32, 2, 6.0, scope="plane", stride_pad=5)


def test_dit_ragged_edges_and_zero_variance():
    rng = np.random.default_rng(71)
    for R, L, lv in [(1, 16, 0), (2, 33, 1), (3, 700, 2), (2, 2300, 4), (1, 256, 4), (2, 4096 + 255, 4)]:
        x = torch.from_numpy(rng.standard_normal((R, L)).astype(np.float32)).to(DEV)
        check_against_oracle(x, lv, 2.5)
    x = torch.randn(3, 9000, device=DEV)
    x[1] = -0.75
    _, _, snr, widx, _ = run_dit(x, 4, 3.0)
    assert torch.all(snr[1] == 0) and torch.all(widx[1] == 0)


def test_dit_level_zero_is_boxcar_snr():
    cfg = synth.make_plane(5, 30001, seed=81, device=DEV, n_pulses=6, pulse_widths=range(1, 17), snr_range=(8, 30),
                           gap=40, t_margin=16)
    x = cfg.x
    p0, stats, snr, widx, cands = run_dit(x, 0, 6.0)
    ref = B.detect(x, list(range(1, 17)), 6.0)
    assert torch.equal(snr, ref["snr"]) and torch.equal(widx, ref["widx"])
    ka = sorted((int(c["row"]), int(c["t"]), int(c["width"]), float(c["snr"])) for c in cands)
    kb = sorted((int(c["row"]), int(c["t"]), int(c["width"]), float(c["snr"])) for c in ref["cands"])
    assert ka == kb


def test_dit_against_exhaustive_gpu():
    cfg = synth.make_plane(4, 40000, seed=91, device=DEV, n_pulses=10, pulse_widths=range(1, 257), snr_range=(8, 40),
                           gap=300, t_margin=256)
    x = cfg.x
    p, stats, snr, widx, _ = run_dit(x, 4, 6.0)
    ex = torch.empty_like(snr)
    exw = torch.empty_like(widx)
    B.boxcar_snr(x, p, stats, snr=ex, widx=exw)
    torch.cuda.synchronize()
    assert torch.all(snr <= ex + 1e-4)
    grid = torch.arange(0, snr.shape[1], 16, device=DEV)
    assert torch.max(torch.abs(snr[:, grid] - ex[:, grid])).item() <= 1e-4
    assert torch.any(snr < ex - 1e-3)                             # windows off the decimated grid are missed


def test_dit_full_size_sampled_rows():
    """The 4,096 x 2^20 SKA-like plane with 4 levels (widths up to 256), in the
    launch configuration the benchmark times; rows sampled for the oracle."""
    cfg = synth.ska(device=DEV)
    pl = cfg["plane"]
    x = pl.x
    print("dit full: generated", flush=True)
    levels = 4
    p, stats, snr, widx, cands = run_dit(x, levels, cfg["threshold"], mode="auto", cap=1 << 21)
    rng = np.random.default_rng(7)
    rows = sorted(set(pl.bright_rows[:3]) | {q.row for q in pl.pulses[:6]} |
                  set(rng.choice(x.shape[0], 4, replace=False).tolist()))
    x64 = x[rows].cpu().double().numpy()
    w, s = oracle.dit_widths(levels)
    _, ost, osnr, owidx = oracle.stream_step(x64, w, sigma_mode="auto", kappa=1.0, strides=s)
    C.check_stats(stats[rows].cpu().numpy(), ost, True)
    worst, nmis = C.check_snr_widx(x64, w, snr[rows].cpu().numpy(), widx[rows].cpu().numpy(), osnr, owidx, ost,
                                   rows=rows)
    print("dit full: rows=%d max|dSNR|=%.3g width mismatches=%d candidates=%d" % (len(rows), worst, nmis,
                                                                                  len(cands)), flush=True)
    del snr, widx, x
    torch.cuda.empty_cache()
