"""Bounds of every boxcar kernel form.  The per-sample outputs (SNR and width
index) are written into views of larger buffers: columns before and after
each row's outputs and one row after the last hold canary values.  The
forms the width list selects are all run (the streaming form for 1..n, the
register-window tiles for short lists and for stepped groups, the strided
tiles for general lists, the decimated levels), with FP32, FP16 and U8
planes and the degenerate shapes (one row; L = Nmax, one start; L = Nmax + 1;
ragged lengths over several tiles).  The canaries must keep their values and
the outputs and candidates must equal those of the same call into tight
buffers."""
import os

import pytest
import torch

from paper_1611_09704_amd import binding as B
from paper_1611_09704_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"
SKA = list(range(1, 17)) + list(range(18, 257, 2))
SNR_CANARY, IDX_CANARY = -7.25, 201

# (name, width list or decimation levels, forced form or None)
CASES = [
    ("w16", list(range(1, 17)), None),
    ("w16", list(range(1, 17)), "window"),
    ("w16", list(range(1, 17)), "strided"),
    ("w5", list(range(1, 6)), "window"),
    ("ska", SKA, None),
    ("ska", SKA, "strided"),
    ("odd", [1, 3, 5, 7, 9, 11, 13], None),
    ("pow2", [1 << k for k in range(9)], None),
    ("dit2", 2, None),
    ("dit4", 4, None),
]


def _plane(R, L, dtype, seed):
    pl = synth.make_plane(R, L, seed=seed, device=DEV, n_pulses=2 * R if L > 128 else 0,
                          pulse_widths=range(1, 65), snr_range=(8, 30))
    if dtype == "f32":
        return pl.x, None, None
    if dtype == "f16":
        return synth.quantize_f16(pl.x), None, None
    return synth.quantize_u8(pl.x, pl.row_sigma)


def _run(x, spec, form, params, stats, snr, widx, stride, scale, zero):
    cand = B.new_candidates(1 << 16, DEV)
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    old = os.environ.get("SPD_BOXCAR_FORM")
    if form is None:
        os.environ.pop("SPD_BOXCAR_FORM", None)
    else:
        os.environ["SPD_BOXCAR_FORM"] = form
    try:
        if isinstance(spec, int):
            B.boxcar_snr_dit(x, params, spec, stats, scale=scale, zero=zero, snr=snr, widx=widx,
                             out_stride=stride, cand=cand, cand_count=cnt)
        else:
            B.boxcar_snr(x, params, stats, scale=scale, zero=zero, snr=snr, widx=widx, out_stride=stride,
                         cand=cand, cand_count=cnt)
        torch.cuda.synchronize()
    finally:
        if old is None:
            os.environ.pop("SPD_BOXCAR_FORM", None)
        else:
            os.environ["SPD_BOXCAR_FORM"] = old
    n = int(cnt.item())
    assert n <= cand.shape[0]
    return sorted((int(c["row"]), int(c["t"]), int(c["width"]), float(c["snr"]))
                  for c in B.candidates_to_numpy(cand, n))


@pytest.mark.parametrize("dtype", ["f32", "f16", "u8"])
@pytest.mark.parametrize("case", range(len(CASES)), ids=["%s-%s" % (c[0], c[2] or "default") for c in CASES])
def test_outputs_stay_in_bounds(case, dtype):
    name, spec, form = CASES[case]
    params = B.dit_params(spec, 5.0) if isinstance(spec, int) else B.Params(spec, 5.0)
    nmax = params.nmax
    for k, (R, L) in enumerate([(1, nmax), (3, nmax + 1), (1, nmax + 1013), (3, 4 * 8192 + 17)]):
        front, back = (5, 7) if k % 2 else (0, 9)
        print("case: %s form=%s dtype=%s shape=(%d, %d) front=%d" % (name, form, dtype, R, L, front), flush=True)
        x, scale, zero = _plane(R, L, dtype, seed=1000 + 17 * case + k)
        stats = B.msd_compute(x, params, scale=scale, zero=zero)
        nout = L - nmax + 1
        stride = front + nout + back
        snr_full = torch.full((R + 1, stride), SNR_CANARY, device=DEV)
        widx_full = torch.full((R + 1, stride), IDX_CANARY, dtype=torch.uint8, device=DEV)
        keys = _run(x, spec, form, params, stats, snr_full[:R, front:front + nout],
                    widx_full[:R, front:front + nout], stride, scale, zero)
        for t, c in ((snr_full, SNR_CANARY), (widx_full, IDX_CANARY)):
            assert torch.all(t[:R, :front] == c) and torch.all(t[:R, front + nout:] == c), "row canary overwritten"
            assert torch.all(t[R:] == c), "canary after the last row overwritten"
        snr = torch.empty((R, nout), device=DEV)
        widx = torch.empty((R, nout), dtype=torch.uint8, device=DEV)
        ref = _run(x, spec, form, params, stats, snr, widx, nout, scale, zero)
        assert torch.equal(snr_full[:R, front:front + nout], snr)
        assert torch.equal(widx_full[:R, front:front + nout], widx)
        assert keys == ref


@pytest.mark.parametrize("dtype", ["f32", "f16", "u8"])
def test_statistics_stay_in_bounds(dtype):
    """msd_compute writes units x 5 doubles: a canary row after them keeps its
    value (row and plane scope, sqrt(N) and AUTO sigma_N)."""
    x, scale, zero = _plane(5, 20011, dtype, seed=77)
    for scope in ("row", "plane"):
        for mode in ("sqrtn", "auto"):
            p = B.Params(SKA, 6.0, scope, mode, 1.0)
            units = p.n_units(x.shape[0])
            full = torch.full((units + 1, B.STATS_FIELDS), -3.5, dtype=torch.float64, device=DEV)
            B.msd_compute(x, p, scale=scale, zero=zero, stats=full[:units])
            ref = B.msd_compute(x, p, scale=scale, zero=zero)
            torch.cuda.synchronize()
            assert torch.all(full[units:] == -3.5), "statistics written past the last unit"
            assert torch.equal(full[:units], ref)


def _raw_tail_untouched(full, cap, fill):
    return bool(torch.all(full[cap:] == fill).item())


def test_candidate_lists_stay_in_bounds():
    """Every producer of a candidate list (fused threshold of boxcar_snr and of
    the decimated search, select_candidates, cluster_candidates) writes at most
    its capacity: records past it in a larger buffer keep their bytes, and the
    count still reports the total."""
    pl = synth.make_plane(6, 30011, seed=88, device=DEV, n_pulses=12, pulse_widths=range(1, 65), snr_range=(8, 30))
    x = pl.x
    p = B.Params(SKA, 2.5)
    stats = B.msd_compute(x, p)
    nout = x.shape[1] - p.nmax + 1
    snr = torch.empty((6, nout), device=DEV)
    widx = torch.empty((6, nout), dtype=torch.uint8, device=DEV)
    big = B.new_candidates(1 << 20, DEV)
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    B.boxcar_snr(x, p, stats, snr=snr, widx=widx, cand=big, cand_count=cnt)
    torch.cuda.synchronize()
    total = int(cnt.item())
    assert 1000 < total < big.shape[0]
    cap = 97
    for name in ("boxcar", "select", "dit", "cluster"):
        full = torch.full((cap + 64, big.shape[1]), 0xA5, dtype=torch.uint8, device=DEV)
        c = torch.zeros(1, dtype=torch.int64, device=DEV)
        if name == "boxcar":
            B.boxcar_snr(x, p, stats, cand=full[:cap], cand_count=c)
        elif name == "select":
            B.select_candidates(snr, widx, p, cand=full[:cap], cand_count=c)
        elif name == "dit":
            pd = B.dit_params(3, 2.5)
            sd = B.msd_compute(x, pd)
            B.boxcar_snr_dit(x, pd, 3, sd, cand=full[:cap], cand_count=c)
        else:
            B.cluster_candidates(snr, big, cnt, 2, 8, peaks=full[:cap], peak_count=c)
        torch.cuda.synchronize()
        n = int(c.item())
        print("case: %s list capacity %d, count %d" % (name, cap, n), flush=True)
        assert n > cap, name
        if name in ("boxcar", "select"):
            assert n == total, name
        assert _raw_tail_untouched(full, cap, 0xA5), "%s wrote past its capacity" % name


def test_dedisp_output_stays_in_bounds():
    """spd_dedisperse writes n_dm rows of n_samp - max_delay columns: canaries
    before and after each row's outputs and a row after the last keep their
    values, and the outputs equal the same call into a tight buffer."""
    band = (1550.0, 300.0 / 256, 64e-6)
    dm = [0.0, 3.0, 7.5, 12.0, 40.0]
    fb = synth.filterbank(256, 3001, seed=5, device=DEV)
    plan = B.DedispPlan(256, *band, dm)
    n_out = fb.shape[1] - plan.max_delay
    front, back = 3, 5
    full = torch.full((len(dm) + 1, front + n_out + back), -9.0, device=DEV)
    plan.run(fb, out=full[:len(dm), front:])
    ref = plan.run(fb)
    torch.cuda.synchronize()
    assert torch.all(full[:len(dm), :front] == -9.0) and torch.all(full[:len(dm), front + n_out:] == -9.0)
    assert torch.all(full[len(dm):] == -9.0)
    assert torch.equal(full[:len(dm), front:front + n_out], ref)
