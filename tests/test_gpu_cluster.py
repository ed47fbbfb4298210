"""Peak-finding over candidate lists on the GPU (cluster_candidates) against
the oracle's definition (oracle.cluster_peaks).

* On SNR-like planes drawn by the seeded generator (values on a 0.25 grid,
  so ties are common) both sides read the same float32 values, and the peak
  sets must be equal exactly.
* Capacity rules: only min(count, capacity) candidates are read; the peak
  count is the total even when the peak list is too short; candidates off
  the plane are never kept.
* End to end (boxcar SNRs from the GPU against FP64 SNRs from the oracle):
  the sets may differ only where the decision hangs on SNRs that the FP32
  budget cannot order -- a candidate within TOL of the threshold, or another
  sample in its neighbourhood within 2*TOL of it.
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
TOL = C.TOL_SNR


def select(snr_t, thr, cap=1 << 18, t_offset=0):
    p = B.Params([1], thr)
    wbuf = torch.zeros((snr_t.shape[0], snr_t.stride(0)), dtype=torch.uint8, device=DEV)
    widx = wbuf[:, :snr_t.shape[1]]                           # the same row stride as the snr view
    cand = B.new_candidates(cap, DEV)
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    B.select_candidates(snr_t, widx, p, t_offset=t_offset, cand=cand, cand_count=cnt)
    return cand, cnt


def peaks_of(snr_t, cand, cnt, dr, dt, t_offset=0, n_out_cols=None, peak_cap=None):
    pk = B.new_candidates(peak_cap, DEV) if peak_cap is not None else None
    pk, pc = B.cluster_candidates(snr_t, cand, cnt, dr, dt, t_offset=t_offset, n_out_cols=n_out_cols, peaks=pk)
    torch.cuda.synchronize()
    n = int(pc.item())
    recs = B.candidates_to_numpy(pk, n)
    keys = [(int(c["row"]), int(c["t"]) - t_offset) for c in recs]
    assert len(set(keys)) == len(keys), "a peak was written twice"
    return n, recs, set(keys)


def oracle_set(plane, thr, dr, dt):
    o = oracle.cluster_peaks(np.asarray(plane, dtype=np.float64), thr, dr, dt)
    return set(zip(o["row"].tolist(), o["t"].tolist()))


@pytest.mark.parametrize("R,L,pad", [(7, 3000, 0), (1, 1, 0), (3, 5, 2), (2, 63, 1), (2, 65, 0), (40, 777, 3),
                                     (5, 4096 + 17, 0)])
@pytest.mark.parametrize("dr,dt", [(0, 0), (1, 3), (2, 64), (0, 300), (5, 1), (3, 1000), (1, 40), (0, 31), (1, 33),
                                   (4096, 1 << 20)])
def test_peaks_equal_oracle_on_seeded_planes(R, L, pad, dr, dt):
    print("case: cluster plane %dx%d pad=%d radii=(%d,%d)" % (R, L, pad, dr, dt), flush=True)
    plane = synth.snr_plane(R, L, seed=1000 + R * 7 + L, n_bumps=max(1, R * L // 2000), n_plateaus=2)
    thr = 2.0 if L < 100 else 5.0
    buf = torch.full((R, L + pad), 99.0, device=DEV)          # the padding is never read as the plane
    buf[:, :L] = torch.from_numpy(plane).to(DEV)
    view = buf[:, :L]
    cand, cnt = select(view, thr)
    n_c = int(cnt.item())
    assert n_c == int(np.sum(plane >= thr))
    n, recs, got = peaks_of(view, cand, cnt, dr, dt)
    want = oracle_set(plane, thr, dr, dt)
    assert got == want, "only GPU: %s, only oracle: %s" % (sorted(got - want)[:5], sorted(want - got)[:5])
    for c in recs:                                            # whole candidate records are copied
        assert c["width"] == 1 and c["beam"] == 0 and c["snr"] == plane[c["row"], c["t"]]
    if dr == 0 and dt == 0:
        assert n == n_c
    if dr >= R and dt >= L and n_c:                           # the whole plane is every window: one peak
        assert n == 1
    print("cluster: candidates=%d peaks=%d" % (n_c, n), flush=True)


def test_time_offset_and_column_limit():
    plane = synth.snr_plane(6, 5000, seed=77, n_bumps=12)
    x = torch.from_numpy(plane).to(DEV)
    off = 123456789
    cand, cnt = select(x[:, :4000], 5.0, t_offset=off)
    _, _, got = peaks_of(x, cand, cnt, 2, 50, t_offset=off, n_out_cols=4000)
    assert got == oracle_set(plane[:, :4000], 5.0, 2, 50)


def test_capacities_and_off_plane_entries():
    plane = synth.snr_plane(8, 6000, seed=78, n_bumps=20)
    x = torch.from_numpy(plane).to(DEV)
    thr, dr, dt = 5.0, 1, 40
    want = oracle_set(plane, thr, dr, dt)
    assert len(want) > 4
    # a peak list shorter than the number of peaks: the count is the total
    cand, cnt = select(x, thr)
    pk = B.new_candidates(3, DEV)
    pk, pc = B.cluster_candidates(x, cand, cnt, dr, dt, peaks=pk)
    torch.cuda.synchronize()
    assert int(pc.item()) == len(want)
    part = {(int(c["row"]), int(c["t"])) for c in B.candidates_to_numpy(pk, 3)}
    assert len(part) == 3 and part <= want
    # a candidate list that overflowed: only its capacity is read
    cap = int(np.sum(plane >= thr)) // 3
    cand, cnt = select(x, thr, cap=cap)
    assert int(cnt.item()) > cap
    listed = {(int(c["row"]), int(c["t"])) for c in B.candidates_to_numpy(cand, cap)}
    _, _, got = peaks_of(x, cand, cnt, dr, dt)
    assert got == listed & want
    # hand-made list: entries off the plane are skipped, the others decided as usual
    rows, ts = np.nonzero(plane >= thr)
    recs = np.zeros(len(rows) + 5, dtype=B.CANDIDATE_DTYPE)
    recs["row"][:len(rows)], recs["t"][:len(rows)] = rows, ts + 10
    recs["snr"][:len(rows)] = plane[rows, ts]
    recs["row"][len(rows):] = [-1, 8, 0, 3, 7]
    recs["t"][len(rows):] = [20, 20, 9, 6010, 6000 + 10]
    recs["snr"][len(rows):] = 100.0
    cand = torch.from_numpy(recs.view(np.uint8).reshape(len(recs), -1).copy()).to(DEV)
    cnt = torch.tensor([len(recs)], dtype=torch.int64, device=DEV)
    _, _, got = peaks_of(x, cand, cnt, dr, dt, t_offset=10)
    assert got == want


def test_empty_and_radius_zero():
    x = torch.zeros((3, 100), device=DEV)
    cand, cnt = select(x, 1.0)
    n, _, got = peaks_of(x, cand, cnt, 4, 4)
    assert n == 0 and not got
    x = torch.full((3, 100), 2.0, device=DEV)                 # one plateau over the whole plane
    cand, cnt = select(x, 1.0)
    assert int(cnt.item()) == 300
    n, _, got = peaks_of(x, cand, cnt, 0, 0)
    assert n == 300
    n, _, got = peaks_of(x, cand, cnt, 1, 10)
    assert got == {(0, 0)} == oracle_set(np.full((3, 100), 2.0), 1.0, 1, 10)


def robust(so, r, t, thr, dr, dt):
    """True when FP32 rounding of the SNRs (<= TOL each) cannot change the
    decision about (r, t)."""
    v = so[r, t]
    if abs(v - thr) <= TOL:
        return False
    R, L = so.shape
    win = so[max(0, r - dr):min(R, r + dr + 1), max(0, t - dt):min(L, t + dt + 1)]
    return int(np.sum(np.abs(win - v) <= 2 * TOL)) == 1


def compare_end_to_end(got, want, so, thr, dr, dt, rows=None):
    bad = [k for k in got ^ want if (rows is None or k[0] in rows) and robust(so, *k, thr, dr, dt)]
    assert not bad, "robust decisions differ at %s" % bad[:5]


@pytest.mark.parametrize("mode", ["sqrtn", "auto"])
def test_end_to_end_against_oracle(mode):
    cfg = synth.ska(device=DEV, R=12, L=40000, n_pulses=10, n_bright=2)
    x = cfg["plane"].x
    W, thr, dr, dt = cfg["widths"], cfg["threshold"], 2, 256
    print("case: cluster end to end mode=%s" % mode, flush=True)
    p = B.Params(W, thr, "row", mode, 1.0)
    stats = B.msd_compute(x, p)
    nout = x.shape[1] - p.nmax + 1
    snr = torch.empty((x.shape[0], nout), device=DEV)
    cand = B.new_candidates(1 << 20, DEV)
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    B.boxcar_snr(x, p, stats, snr=snr, cand=cand, cand_count=cnt)
    torch.cuda.synchronize()
    n_c = int(cnt.item())
    assert n_c <= cand.shape[0]
    n, _, got = peaks_of(snr, cand, cnt, dr, dt)
    o = oracle.detect(x.cpu().double().numpy(), W, thr, sigma_mode=mode, kappa=1.0)
    want = oracle_set(o["snr"], thr, dr, dt)
    compare_end_to_end(got, want, o["snr"], thr, dr, dt)
    print("cluster e2e: candidates=%d peaks=%d oracle peaks=%d" % (n_c, n, len(want)), flush=True)
    assert n < n_c


def test_full_size_sampled_rows():
    """The 4,096 x 2^20 SKA-like plane in the benchmark's configuration
    (AUTO sigma_N, 136 widths, radii 2 rows x 256 starts); the decisions in
    sampled rows are checked against oracle SNRs of those rows and their
    neighbours."""
    cfg = synth.ska(device=DEV)
    pl = cfg["plane"]
    x = pl.x
    W, thr, dr, dt = cfg["widths"], cfg["threshold"], 2, 256
    print("cluster full: generated", flush=True)
    p = B.Params(W, thr, "row", "auto", 1.0)
    stats = B.msd_compute(x, p)
    nout = x.shape[1] - p.nmax + 1
    snr = torch.empty((x.shape[0], nout), device=DEV)
    cand = B.new_candidates(1 << 22, DEV)
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    B.boxcar_snr(x, p, stats, snr=snr, cand=cand, cand_count=cnt)
    torch.cuda.synchronize()
    n_c = int(cnt.item())
    assert n_c <= cand.shape[0]
    n, recs, got = peaks_of(snr, cand, cnt, dr, dt)
    print("cluster full: candidates=%d peaks=%d" % (n_c, n), flush=True)
    rng = np.random.default_rng(11)
    centre = sorted(set(pl.bright_rows[:2]) | {q.row for q in pl.pulses[:4]} |
                    set(rng.choice(x.shape[0], 2, replace=False).tolist()))
    for r in centre:
        lo, hi = max(0, r - dr), min(x.shape[0], r + dr + 1)
        x64 = x[lo:hi].cpu().double().numpy()
        _, _, so, _ = oracle.stream_step(x64, W, sigma_mode="auto", kappa=1.0)
        sub = oracle.cluster_peaks(so, thr, dr, dt)
        want = {(int(a) + lo, int(b)) for a, b in zip(sub["row"], sub["t"]) if int(a) + lo == r}
        got_r = {k for k in got if k[0] == r}
        shifted = so.copy()
        bad = [k for k in got_r ^ want if robust(shifted, k[0] - lo, k[1], thr, dr, dt)]
        assert not bad, "row %d: robust decisions differ at %s" % (r, bad[:5])
        print("cluster full: row %d peaks=%d oracle=%d" % (r, len(got_r), len(want)), flush=True)
    del snr, x
    torch.cuda.empty_cache()
