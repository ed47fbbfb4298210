"""Pins of the de-dispersion step of the oracle (oracle.dedisp_*), the step
before the detection path: a filterbank of frequency channels x time samples
becomes one series per trial DM by summing every channel shifted by its
dispersion delay.

Pinned to things other than the oracle's own code:

* the cold-plasma delay law at numbers worked by hand: between 1500 and 1200
  MHz, 1/1200^2 - 1/1500^2 is exactly 2.5e-7 MHz^-2, so DM 500 delays the
  lower channel by 4148.808 * 500 * 2.5e-7 = 0.518601 s, which is 8103.14
  samples of 64 us (-> 8103), and DM 250 by 4051.57 (-> 4052); the textbook
  2.1167 ms per unit DM between 1400 MHz and infinite frequency;
* DM 0 is the plain sum over channels;
* a pure-Python brute force over (trial, start, channel) on small inputs;
* a pulse laid exactly along one trial's delay curve adds up in that trial's
  series at its start, and only there;
* linearity, and a shift of the input shifts the output;
* delays grow with DM and towards lower frequencies.
"""
import math

import numpy as np
import pytest

import oracle


def test_delay_law_at_hand_worked_numbers():
    kc = oracle.dedisp_channel_factors(2, 1500.0, 300.0, 64e-6)
    assert kc[0] == 0.0
    assert kc[1] * 64e-6 == pytest.approx(1.037202e-3, rel=1e-12)      # seconds per unit DM
    d = oracle.dedisp_delays([0.0, 1.0, 250.0, 500.0], kc)
    assert d[:, 0].tolist() == [0, 0, 0, 0]
    assert d[:, 1].tolist() == [0, 16, 4052, 8103]                        # 16.206, 4051.57, 8103.14 samples
    # 1400 MHz against infinite frequency: the top channel far above the band
    kc = oracle.dedisp_channel_factors(2, 1e12, 1e12 - 1400.0, 1.0)
    assert kc[1] == pytest.approx(2.1167e-3, rel=1e-4)


def test_delays_monotone_and_halves_round_up():
    kc = oracle.dedisp_channel_factors(256, 1550.0, 300.0 / 256, 64e-6)
    assert np.all(np.diff(kc) > 0)
    dm = np.arange(0, 300, 0.37)
    d = oracle.dedisp_delays(dm, kc)
    assert np.all(np.diff(d, axis=0) >= 0) and np.all(np.diff(d, axis=1) >= 0)
    assert oracle.dedisp_delays([1.0], [2.5]).tolist() == [[3]] and oracle.dedisp_delays([1.0], [2.4999]).tolist() == [[2]]


def brute(fb, dm, kc):
    C, S = fb.shape
    delays = [[math.floor(float(v) * float(k) + 0.5) for k in kc] for v in dm]
    n_out = S - max(max(r) for r in delays)
    out = [[0.0] * n_out for _ in dm]
    for d in range(len(dm)):
        for t in range(n_out):
            out[d][t] = float(sum(int(fb[c, t + delays[d][c]]) for c in range(C)))
    return np.array(out)


@pytest.mark.parametrize("C,S,n_dm,seed", [(1, 50, 3, 1), (5, 120, 4, 2), (16, 300, 7, 3), (33, 700, 5, 4)])
def test_matches_brute_force(C, S, n_dm, seed):
    rng = np.random.default_rng(seed)
    fb = rng.integers(0, 256, (C, S), dtype=np.uint8)
    kc = oracle.dedisp_channel_factors(C, 1500.0, 20.0 / C, 64e-6)   # up to ~1.2 samples per unit DM
    dm = np.sort(rng.uniform(0, 40, n_dm))
    got = oracle.dedisperse(fb, dm, kc)
    assert got.shape[1] == S - int(oracle.dedisp_delays(dm, kc).max())
    assert np.array_equal(got, brute(fb, dm, kc))


def test_dm_zero_is_the_channel_sum():
    rng = np.random.default_rng(5)
    fb = rng.integers(0, 256, (64, 1000), dtype=np.uint8)
    kc = oracle.dedisp_channel_factors(64, 1400.0, 1.0, 1e-4)
    out = oracle.dedisperse(fb, [0.0], kc)
    assert np.array_equal(out[0], fb.sum(axis=0, dtype=np.int64).astype(np.float64))


def test_pulse_along_one_delay_curve():
    C, S = 48, 3000
    kc = oracle.dedisp_channel_factors(C, 1500.0, 5.0, 64e-6)
    dm = np.linspace(0, 60, 25)
    delays = oracle.dedisp_delays(dm, kc)
    assert delays.max() < 1500 and delays[13, -1] > 100
    fb = np.zeros((C, S), dtype=np.uint8)
    t_p = 700
    for c in range(C):
        fb[c, t_p + delays[13, c]] = 5
    out = oracle.dedisperse(fb, dm, kc)
    assert out[13, t_p] == 5 * C
    assert out[13].sum() == 5 * C and np.count_nonzero(out[13]) == 1
    others = np.delete(out, 13, axis=0)
    assert others.max() < 5 * C


def test_linearity_and_shift():
    rng = np.random.default_rng(6)
    C, S = 20, 900
    kc = oracle.dedisp_channel_factors(C, 1300.0, 4.0, 1e-4)
    dm = np.linspace(0, 30, 6)
    a = rng.integers(0, 100, (C, S), dtype=np.uint8)
    b = rng.integers(0, 100, (C, S), dtype=np.uint8)
    oa, ob = oracle.dedisperse(a, dm, kc), oracle.dedisperse(b, dm, kc)
    assert np.array_equal(oracle.dedisperse(a + b, dm, kc), oa + ob)
    s = 37
    shifted = np.concatenate([np.zeros((C, s), dtype=np.uint8), a], axis=1)
    assert np.array_equal(oracle.dedisperse(shifted, dm, kc)[:, s:], oa)
