"""The register-window form of the boxcar kernel (8 consecutive starts per
lane, the group's reads held in registers) and, for the lists 1..n with
n <= 16, the streaming form (a wave walks a long run of one row, 4
consecutive starts per lane per block) against the strided form (starts 64
apart per lane, one LDS read per width and start).

All run the same running sums in the same order on the same staged values
and apply the same first-maximiser rule, so SNRs, width indices and the
candidate set must agree bit for bit.  The form is chosen per call (the
default: streaming for 1..n, n <= 16, else register-window where the list
allows it); SPD_BOXCAR_FORM=window forces the register-window tiles and
SPD_BOXCAR_FORM=strided the strided one.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1611_09704_amd import binding as B
from paper_1611_09704_amd import synth
import spd_check as C

pytestmark = pytest.mark.gpu

DEV = "cuda"
SKA = list(range(1, 17)) + list(range(18, 257, 2))


def run_form(form, x, p, stats, stride_pad=0, scale=None, zero=None):
    R = x.shape[0]
    nout = x.shape[1] - p.nmax + 1
    stride = nout + stride_pad
    snr = torch.full((R, stride), -3.0, device=DEV)
    widx = torch.full((R, stride), 250, dtype=torch.uint8, device=DEV)
    cand = B.new_candidates(1 << 18, DEV)
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    old = os.environ.get("SPD_BOXCAR_FORM")
    if form is None:
        os.environ.pop("SPD_BOXCAR_FORM", None)
    else:
        os.environ["SPD_BOXCAR_FORM"] = form
    try:
        B.boxcar_snr(x, p, stats, scale=scale, zero=zero, snr=snr[:, :nout], widx=widx[:, :nout],
                     out_stride=stride, cand=cand, cand_count=cnt)
        torch.cuda.synchronize()
    finally:
        if old is None:
            os.environ.pop("SPD_BOXCAR_FORM", None)
        else:
            os.environ["SPD_BOXCAR_FORM"] = old
    n = int(cnt.item())
    assert n <= cand.shape[0]
    keys = sorted((int(c["row"]), int(c["t"]), int(c["width"]), float(c["snr"]))
                  for c in B.candidates_to_numpy(cand, n))
    return snr, widx, keys


def compare(x, widths, thr, *, mode="sqrtn", scope="row", stride_pad=0, scale=None, zero=None):
    print("case: window vs strided shape=%s dtype=%s |W|=%d nmax=%d mode=%s scope=%s pad=%d" % (
        tuple(x.shape), x.dtype, len(widths), widths[-1], mode, scope, stride_pad), flush=True)
    p = B.Params(widths, thr, scope, mode, 1.0)
    stats = B.msd_compute(x, p, scale=scale, zero=zero)
    b = run_form("strided", x, p, stats, stride_pad, scale, zero)
    nout = x.shape[1] - p.nmax + 1
    for form in ("window", None):
        a = run_form(form, x, p, stats, stride_pad, scale, zero)
        assert torch.equal(a[0], b[0]), "snr differs (%s)" % form
        assert torch.equal(a[1], b[1]), "width indices differ (%s)" % form
        assert a[2] == b[2], "candidate sets differ (%s: %d vs %d)" % (form, len(a[2]), len(b[2]))
        if stride_pad:
            assert torch.all(a[0][:, nout:] == -3.0) and torch.all(a[1][:, nout:] == 250)
    return a


@pytest.mark.parametrize("widths", [list(range(1, 6)), list(range(1, 9)), list(range(1, 13)),
                                    list(range(1, 17)), list(range(1, 33)), SKA, list(range(1, 129)),
                                    list(range(1, 257))])
def test_window_equals_strided(widths):
    cfg = synth.make_plane(7, 9001 + widths[-1], seed=31, device=DEV, n_pulses=5,
                           pulse_widths=range(1, min(widths[-1], 64) + 1), snr_range=(8, 30), gap=64,
                           t_margin=widths[-1])
    a = compare(cfg.x, widths, 6.0)
    assert len(a[2]) > 0


@pytest.mark.parametrize("pad", [1, 3, 8])
def test_window_unaligned_output_rows(pad):
    cfg = synth.ska(device=DEV, R=6, L=20003, n_pulses=4, n_bright=2)
    compare(cfg["plane"].x, SKA, cfg["threshold"], mode="auto", stride_pad=pad)
    compare(cfg["plane"].x, list(range(1, 17)), cfg["threshold"], stride_pad=pad)


def test_window_precision_forms_and_plane_scope():
    cfg = synth.tiny(device=DEV, R=8, L=30011)
    x32 = cfg["plane"].x
    compare(synth.quantize_f16(x32), SKA, 6.0)
    q, s, z = synth.quantize_u8(x32, cfg["plane"].row_sigma)
    compare(q, list(range(1, 17)), 6.0, scale=s, zero=z)
    compare(x32, list(range(1, 33)), 6.0, scope="plane")


def test_window_ragged_edges_and_zero_variance():
    rng = np.random.default_rng(17)
    for R, L, W in [(1, 16, list(range(1, 17))), (2, 513, list(range(1, 9))), (3, 2300, SKA[:24]),
                    (2, 257, SKA), (1, 4096 + 255, SKA)]:
        x = torch.from_numpy(rng.standard_normal((R, L)).astype(np.float32)).to(DEV)
        compare(x, W, 2.5)
    x = torch.randn(3, 6000, device=DEV)
    x[1] = 1.5
    a = compare(x, SKA, 3.0)
    assert torch.all(a[0][1] == 0) and torch.all(a[1][1] == 0)


@pytest.mark.parametrize("L", [15, 16, 17, 511, 527, 528, 8192 + 15, 8192 + 16, 4 * 8192 + 15, 4 * 8192 + 16 + 700,
                               5 * 8192 * 4 + 1234])
@pytest.mark.parametrize("n", [1, 7, 8, 9, 16])
def test_stream_runs_steps_and_row_ends(L, n):
    """Row lengths around the streaming form's step (512 starts), run (8,192)
    and work-group (32,768) boundaries, for every list length class."""
    if L < n:
        pytest.skip("row shorter than the widest boxcar")
    rng = np.random.default_rng(1000 + L + n)
    x = torch.from_numpy(rng.standard_normal((3, L)).astype(np.float32) * 2 + 0.5).to(DEV)
    compare(x, list(range(1, n + 1)), 2.0)


def test_stream_unaligned_plane_rows():
    """Rows that do not start on a 4-element boundary take the checked loads."""
    rng = np.random.default_rng(5)
    base = torch.from_numpy(rng.standard_normal((4, 40001)).astype(np.float32)).to(DEV)
    compare(base[:, 1:], list(range(1, 17)), 2.5)
    compare(base[:, 3:], list(range(1, 9)), 2.5, mode="linear")
    h = synth.quantize_f16(base)
    compare(h[:, 1:], list(range(1, 17)), 2.5)


def test_window_matches_oracle_ska_widths():
    cfg = synth.ska(device=DEV, R=6, L=25000, n_pulses=5, n_bright=2)
    x = cfg["plane"].x
    W, thr = cfg["widths"], cfg["threshold"]
    print("case: window vs oracle", flush=True)
    g = B.detect(x, W, thr, sigma_mode="auto", kappa=1.0)
    torch.cuda.synchronize()
    x64 = x.cpu().double().numpy()
    o = oracle.detect(x64, W, thr, sigma_mode="auto", kappa=1.0)
    C.check_stats(g["stats"].cpu().numpy(), o["stats"], True)
    C.check_snr_widx(x64, W, g["snr"].cpu().numpy(), g["widx"].cpu().numpy(), o["snr"], o["widx"], o["stats"])
    C.check_candidates(g["cands"], o["cands"], thr, lambda r, t: o["snr"][r, t],
                       C.width_rule(x64, W, o["stats"]))
