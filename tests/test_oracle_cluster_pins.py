"""Pins of the candidate peak-finding in the oracle (oracle.cluster_peaks).

Checked against a pure-Python brute force over every pair of samples, and
against properties that hold by construction: radius 0 keeps every
candidate; peaks are candidates; no peak lies in another peak's
neighbourhood; an isolated pulse gives one peak at its maximum; a plateau
keeps its first sample in row-major order; far-apart pulses stay separate.
"""
import itertools

import numpy as np
import pytest

import oracle


def brute(snr, thr, dr, dt):
    R, L = snr.shape
    out = []
    for r, t in itertools.product(range(R), range(L)):
        v = snr[r, t]
        if not v >= thr:
            continue
        ok = True
        for r2, t2 in itertools.product(range(max(0, r - dr), min(R, r + dr + 1)),
                                        range(max(0, t - dt), min(L, t + dt + 1))):
            if (r2, t2) == (r, t):
                continue
            w = snr[r2, t2]
            if w > v or (w == v and (r2, t2) < (r, t)):
                ok = False
                break
        if ok:
            out.append((r, t))
    return out


@pytest.mark.parametrize("dr,dt,seed", [(0, 0, 1), (1, 3, 2), (2, 1, 3), (1, 8, 4), (3, 20, 5)])
def test_matches_brute_force(dr, dt, seed):
    rng = np.random.default_rng(seed)
    snr = np.round(rng.standard_normal((7, 60)) * 2.0, 1)      # rounding makes ties common
    got = oracle.cluster_peaks(snr, 1.0, dr, dt)
    assert list(zip(got["row"].tolist(), got["t"].tolist())) == brute(snr, 1.0, dr, dt)


def test_radius_zero_keeps_every_candidate():
    rng = np.random.default_rng(9)
    snr = rng.standard_normal((5, 300)) * 3
    got = oracle.cluster_peaks(snr, 2.0, 0, 0)
    assert np.array_equal(np.stack([got["row"], got["t"]], 1), np.argwhere(snr >= 2.0))


def test_peaks_are_separated_candidates():
    rng = np.random.default_rng(10)
    snr = rng.standard_normal((12, 2000)) * 2.5
    dr, dt = 2, 30
    got = oracle.cluster_peaks(snr, 3.0, dr, dt)
    pk = list(zip(got["row"].tolist(), got["t"].tolist()))
    assert all(snr[r, t] >= 3.0 for r, t in pk)
    for (a, b), (c, d) in itertools.combinations(pk, 2):
        assert not (abs(a - c) <= dr and abs(b - d) <= dt)
    assert 0 < len(pk) < int(np.sum(snr >= 3.0))


def test_pulse_plateau_and_separation():
    snr = np.zeros((6, 400))
    # a pulse smeared over rows and starts, maximum at (2, 100)
    for r in range(6):
        for t in range(400):
            snr[r, t] = 9.0 - abs(r - 2) - 0.05 * abs(t - 100)
    got = oracle.cluster_peaks(snr, 5.0, 2, 64)
    assert list(zip(got["row"].tolist(), got["t"].tolist()))[0] == (2, 100)
    # a plateau: the first sample in row-major order wins
    flat = np.zeros((4, 50))
    flat[1:3, 10:20] = 7.0
    got = oracle.cluster_peaks(flat, 5.0, 1, 15)
    assert list(zip(got["row"].tolist(), got["t"].tolist())) == [(1, 10)]
    # two pulses farther apart than the radius stay two peaks
    two = np.zeros((3, 500))
    two[1, 100] = 8.0
    two[1, 300] = 9.0
    got = oracle.cluster_peaks(two, 5.0, 1, 150)
    assert list(zip(got["row"].tolist(), got["t"].tolist())) == [(1, 100), (1, 300)]
    got = oracle.cluster_peaks(two, 5.0, 1, 250)
    assert list(zip(got["row"].tolist(), got["t"].tolist())) == [(1, 300)]
