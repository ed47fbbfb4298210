"""Pins of the FP64 oracle against facts fixed outside it.

Each test checks the oracle against something it does not compute itself:
textbook two-pass statistics, exact rational arithmetic, hand-derived closed
forms (tests/golden), the brute-force restatement in oracle/brute.py, exact
invariances of the definition, or statistical laws with fixed seeds.  A
plausible slip in the oracle -- a missing square, a wrong index, mu instead of
w*mu, a wrong sign in Eq. (sd03), '>=' instead of '>' -- fails at least one.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _two_pass(x):
    x = np.asarray(x, dtype=np.float64)
    mu = x.mean()
    return x.size, x.sum(), ((x - mu) ** 2).sum()


# --- Sec. 2.1: Eq. (MSD03) and Eq. (MSD04) -------------------------------------

def test_textbook_example():
    g = json.load(open(os.path.join(GOLD, "textbook_msd.json")))
    n, T, S = oracle.chan_stream(g["x"])
    assert (n, T, S) == (g["n"], g["T"], g["S"])
    assert T / n == g["mean"] and math.sqrt(S / n) == g["sigma"]


def test_stream_matches_two_pass_with_offset():
    rng = np.random.default_rng(1)
    for n in (1, 2, 3, 17, 1000, 65536):
        x = 1.0e3 + 0.25 * rng.standard_normal(n)        # |mu| >> sigma
        n_, T, S = oracle.chan_stream(x)
        m, T2, S2 = _two_pass(x)
        assert n_ == m
        assert T == pytest.approx(T2, rel=1e-13)
        assert S == pytest.approx(S2, rel=1e-10, abs=1e-12)


def test_stream_exact_on_integers():
    """Integers with exact rational two-pass statistics."""
    rng = np.random.default_rng(2)
    x = rng.integers(-50, 50, size=300)
    n = len(x)
    mu = Fraction(int(x.sum()), n)
    S = sum((Fraction(int(v)) - mu) ** 2 for v in x)
    _, T, S_o = oracle.chan_stream(x)
    assert T == int(x.sum())
    assert S_o == pytest.approx(float(S), rel=1e-13)


def test_special_cases():
    assert tuple(oracle.chan_stream([3.5])) == (1.0, 3.5, 0.0)
    n, T, S = oracle.chan_stream([1.0, 4.0])
    assert S == pytest.approx((1.0 - 4.0) ** 2 / 2.0, abs=0)
    assert oracle.chan_stream(np.full(999, 7.25))[2] == 0.0


def test_printed_update_without_square_is_wrong():
    """Eq. (MSD03) as printed (no square) disagrees with two-pass; the squared
    reading used by the oracle agrees.  Guards the reading, not the oracle."""
    rng = np.random.default_rng(3)
    x = 5.0 + rng.standard_normal(4000)
    T = S = 0.0
    for j, v in enumerate(x, start=1):
        T += v
        if j > 1:
            S += (j * v - T) / (j * (j - 1))
    _, _, S_ref = _two_pass(x)
    assert abs(S - S_ref) > 0.5 * S_ref
    assert oracle.chan_stream(x)[2] == pytest.approx(S_ref, rel=1e-10)


def test_merge_any_partition_and_tree():
    rng = np.random.default_rng(4)
    x = -3.0 + 2.0 * rng.standard_normal(5000)
    _, T_ref, S_ref = _two_pass(x)
    for trial in range(20):
        cuts = np.sort(rng.choice(np.arange(1, x.size), size=rng.integers(1, 12), replace=False))
        parts = [oracle.chan_stream(p) for p in np.split(x, cuts)]
        if trial % 3 == 2:                                  # include empty parts
            parts.insert(int(rng.integers(0, len(parts))), np.zeros(3))
        while len(parts) > 1:                               # random adjacent-merge tree
            i = int(rng.integers(0, len(parts) - 1))
            parts[i:i + 2] = [oracle.chan_merge(parts[i], parts[i + 1])]
        n, T, S = parts[0]
        assert n == x.size
        assert T == pytest.approx(T_ref, rel=1e-12)
        assert S == pytest.approx(S_ref, rel=1e-12)


# --- Sec. 2.2-2.4 and Algorithm 1 against brute force -----------------------------

@pytest.mark.parametrize("scope", ["row", "plane"])
@pytest.mark.parametrize("mode", ["sqrtn", "linear", "auto", "linear_literal"])
def test_oracle_matches_brute_force(scope, mode):
    rng = np.random.default_rng(5)
    R, L = 3, 90
    x = rng.standard_normal((R, L)) * np.array([[1.0], [0.6], [2.0]]) + np.array([[0.0], [3.0], [-1.5]])
    x[1, 30:60] += 4.0                                      # a signal-dominated stretch
    x[2, 10:13] += 5.0
    widths = [1, 2, 3, 5, 8, 9, 13]
    thr = 1.5
    o = oracle.detect(x, widths, thr, scope=scope, sigma_mode=mode, kappa=0.05)
    b = brute.detect(x.tolist(), widths, thr, scope=scope, sigma_mode=mode, kappa=0.05)
    for u, st in enumerate(b["stats"]):
        cols = [0, 1, 3] if mode == "sqrtn" else [0, 1, 2, 3]      # sigma_Nmax only when needed
        assert o["stats"][u, cols] == pytest.approx([st[c] for c in cols], rel=1e-11, abs=1e-12)
        assert int(o["stats"][u, 4]) == st[4]
    np.testing.assert_allclose(o["snr"], np.array(b["snr"]), rtol=0, atol=1e-11)
    np.testing.assert_array_equal(o["widx"], np.array(b["widx"]))
    got = list(zip(o["cands"]["row"], o["cands"]["t"], o["cands"]["width"]))
    assert got == [(r, t, w) for r, t, _, w in b["cands"]]


def test_closed_form_pulse_snr_curve():
    """Figure 1 shape: SNR of each width at the pulse start, closed form."""
    g = json.load(open(os.path.join(GOLD, "pulse_closed_form.json")))
    x = np.zeros((1, g["L"]))
    x[0, g["t0"]:g["t0"] + g["wp"]] = g["A"]
    sigma = math.sqrt(g["sigma_squared"])
    curve = []
    for w, num in zip(g["widths"], g["snr_numerators"]):
        _, stats, snr, _ = oracle.stream_step(x, [w])
        assert stats[0, 0] == g["mean"] and stats[0, 1] == pytest.approx(sigma, rel=1e-15)
        assert snr[0, g["t0"]] == pytest.approx(num / (math.sqrt(w) * sigma), rel=1e-14)
        curve.append(snr[0, g["t0"]])
    assert g["widths"][int(np.argmax(curve))] == g["argmax_width"]
    _, _, snr, widx = oracle.stream_step(x, g["widths"])
    assert g["widths"][widx[0, g["t0"]]] == g["argmax_width"]


def test_pulse_recovered_at_its_width_and_snr():
    """A rectangle with true SNR s on N(0,1) noise: best width is the pulse
    width and the SNR there is s within the noise of one boxcar (~1)."""
    rng = np.random.default_rng(6)
    L = 20000
    x = rng.standard_normal((1, L))
    for wp, s in ((1, 30.0), (7, 25.0), (32, 40.0)):
        y = x.copy()
        y[0, 5000:5000 + wp] += s / math.sqrt(wp)
        o = oracle.detect(y, list(range(1, 65)), 6.0)
        t = 5000
        assert abs(o["snr"][0, t] - s) < 4.0
        assert abs((o["widx"][0, t] + 1) - wp) <= max(2, wp // 4)


def test_sqrt_n_law_on_noise():
    """Eq. (sd02): the measured sigma of the Nmax boxcar is sqrt(Nmax)*sigma on
    i.i.d. noise (up to sampling error)."""
    rng = np.random.default_rng(7)
    L = 400000
    x = 2.0 + 3.0 * rng.standard_normal((1, L))
    for nmax in (4, 16, 64):
        _, stats, _, _ = oracle.stream_step(x, list(range(1, nmax + 1)), sigma_mode="linear")
        rho = stats[0, 2] / (math.sqrt(nmax) * stats[0, 1])
        assert abs(rho - 1.0) < 5.0 * math.sqrt(nmax / L)
        y = np.convolve(x[0], np.ones(nmax), mode="valid")
        assert stats[0, 2] == pytest.approx(y.std(), rel=1e-10)


def test_linear_form_identities():
    """Anchored Eq. (sd03): sigma_1 = sigma, sigma_Nmax = measured; so at a single
    width the SNR series is a z-score (population std exactly 1)."""
    rng = np.random.default_rng(8)
    x = rng.standard_normal((1, 3000))
    x[0, 1000:1900] += 3.0
    _, st, snr, _ = oracle.stream_step(x, [1], sigma_mode="linear")
    assert snr.mean() == pytest.approx(0.0, abs=1e-12) and snr.std() == pytest.approx(1.0, rel=1e-12)
    _, st, snr, _ = oracle.stream_step(x, [24], sigma_mode="linear")
    assert snr.std() == pytest.approx(1.0, rel=1e-12)
    # literal reading: sigma at Nmax = sqrt(Nmax)*sigma + sigma_Nmax
    _, st, snr_l, _ = oracle.stream_step(x, [24], sigma_mode="linear_literal")
    mu, sigma, sn = st[0, :3]
    y = np.convolve(x[0], np.ones(24), mode="valid")
    np.testing.assert_allclose(snr_l[0], (y - 24 * mu) / (math.sqrt(24) * sigma + sn), rtol=1e-12)


def test_auto_mode_switches_on_signal_dominated_rows():
    rng = np.random.default_rng(9)
    L = 50000
    x = rng.standard_normal((2, L))
    x[1, 10000:10000 + int(0.3 * L)] += 2.0
    _, st, _, _ = oracle.stream_step(x, list(range(1, 129)), sigma_mode="auto", kappa=1.0)
    assert int(st[0, 4]) & oracle.FLAG_LINEAR == 0 and st[0, 3] == 0.0
    assert int(st[1, 4]) & oracle.FLAG_LINEAR and st[1, 3] > 0.0
    rho = st[1, 2] / (math.sqrt(128) * st[1, 1])
    assert rho > 2.0


def test_affine_invariance_per_row():
    rng = np.random.default_rng(10)
    x = rng.standard_normal((3, 4000))
    x[1, 100:110] += 3.0
    y = x * np.array([[2.5], [0.1], [7.0]]) + np.array([[-40.0], [3.0], [1e3]])
    for mode in ("sqrtn", "linear"):
        a = oracle.detect(x, [1, 2, 4, 8, 16], 5.0, sigma_mode=mode)
        b = oracle.detect(y, [1, 2, 4, 8, 16], 5.0, sigma_mode=mode)
        np.testing.assert_allclose(a["snr"], b["snr"], atol=1e-9)
        assert (a["widx"] == b["widx"]).mean() > 0.999


def test_threshold_is_inclusive():
    rng = np.random.default_rng(11)
    x = rng.standard_normal((2, 500))
    o = oracle.detect(x, [1, 2, 3], 0.0)
    r, t = np.unravel_index(np.argmax(o["snr"]), o["snr"].shape)
    top = o["snr"][r, t]
    c = oracle.select(o["snr"], o["widx"], [1, 2, 3], top)
    assert list(c["row"]) == [r] and list(c["t"]) == [t]
    assert oracle.select(o["snr"], o["widx"], [1, 2, 3], np.nextafter(top, np.inf))["row"].size == 0


def test_sigma_w_vanishing_at_nmax_contributes_zero():
    """Anchored Eq. (sd03) gives sigma_Nmax exactly at w = Nmax; when that is 0
    (a single valid start, or a row whose Nmax-boxcar is constant) the width
    has no noise estimate and contributes SNR 0 whatever the rounding residual
    of sigma_w, while the other widths keep their direct z-scores."""
    rng = np.random.default_rng(31)
    for n in (300, 97, 1024):
        x = rng.standard_normal((1, n))
        _, st, snr, widx = oracle.stream_step(x, [1, n // 2, n], sigma_mode="linear")
        mu, sigma, sn, coef = st[0, :4]
        assert sn == 0.0 and coef == pytest.approx(-math.sqrt(n) * sigma / (n - 1), rel=1e-12)
        direct = [(x[0, 0] - mu) / sigma,
                  (x[0, :n // 2].sum() - n // 2 * mu) / (math.sqrt(n // 2) * sigma + (n // 2 - 1) * coef), 0.0]
        assert snr[0, 0] == pytest.approx(max(direct), rel=1e-12) and widx[0, 0] == int(np.argmax(direct))
    # period 2: every 4-boxcar sums to 0, so sigma_4 = 0 and width 4 never wins
    x = np.tile([1.0, -1.0], 500)[None, :]
    _, st, snr, widx = oracle.stream_step(x, [1, 2, 4], sigma_mode="linear")
    assert st[0, 2] == 0.0
    assert np.all(widx[0] != 2) and np.all(np.abs(snr[0]) <= 1.0 + 1e-12)


def test_zero_variance_unit():
    x = np.vstack([np.full(300, 4.0), np.random.default_rng(12).standard_normal(300)])
    _, st, snr, widx = oracle.stream_step(x, [1, 3, 9])
    assert int(st[0, 4]) & oracle.FLAG_ZERO_VAR
    assert np.all(snr[0] == 0.0) and np.all(widx[0] == 0)
    assert not int(st[1, 4]) & oracle.FLAG_ZERO_VAR


def test_ties_keep_first_width():
    """Exact ties (zero signal over a window) keep the smallest width: strict '>'."""
    x = np.zeros((1, 64))
    x[0, 0] = 1.0
    x[0, 40] = -1.0
    _, st, snr, widx = oracle.stream_step(x, [1, 2, 4])
    # t = 20: every boxcar is 0 - w*mu with mu = 0 -> all SNRs 0, first width wins
    assert st[0, 0] == 0.0 and snr[0, 20] == 0.0 and widx[0, 20] == 0


# --- streaming: chunk + halo + running state --------------------------------------

@pytest.mark.parametrize("mode", ["sqrtn", "linear"])
def test_stream_equals_one_shot_on_prefix(mode):
    """Chunk k of a stream, carried with an (Nmax-1)-column halo and a running
    state, gives what a one-shot run on the whole series up to chunk k gives for
    the window starts that end inside chunk k."""
    rng = np.random.default_rng(13)
    R, Lc, K = 2, 700, 4
    W = [1, 2, 3, 6, 11]
    nmax = W[-1]
    full = rng.standard_normal((R, Lc * K)) + np.array([[0.0], [5.0]])
    full[0, Lc - 3:Lc + 5] += 4.0                        # straddles a boundary
    state = None
    for k in range(K):
        if k == 0:
            view, ncb, toff = full[:, :Lc], 0, 0
        else:
            view, ncb, toff = full[:, k * Lc - (nmax - 1):(k + 1) * Lc], nmax - 1, k * Lc - (nmax - 1)
        state, st, snr, widx = oracle.stream_step(view, W, new_col_begin=ncb, state=state,
                                                  sigma_mode=mode)
        _, st1, snr1, widx1 = oracle.stream_step(full[:, :(k + 1) * Lc], W, sigma_mode=mode)
        np.testing.assert_allclose(st[:, :4], st1[:, :4], rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(snr, snr1[:, toff:toff + snr.shape[1]], rtol=0, atol=1e-10)
        np.testing.assert_array_equal(widx, widx1[:, toff:toff + snr.shape[1]])


def test_auto_switches_exactly_at_one_plus_kappa():
    """AUTO applies the linear form iff rho = sigma_Nmax / (sqrt(Nmax) sigma)
    exceeds 1 + kappa; rho recomputed here by numpy from the definitions."""
    rng = np.random.default_rng(14)
    L, nmax = 40000, 32
    x = rng.standard_normal((2, L))
    x[1, 5000:5000 + int(0.3 * L)] += 1.0
    for r in range(2):
        y = np.convolve(x[r], np.ones(nmax), mode="valid")
        rho = y.std() / (np.sqrt(nmax) * x[r].std())
        for kappa in (0.0, 0.5, rho - 1.0 - 1e-3, rho - 1.0 + 1e-3, 2.0):
            if kappa < 0:
                continue
            _, st, _, _ = oracle.stream_step(x[r:r + 1], list(range(1, nmax + 1)), sigma_mode="auto", kappa=kappa)
            assert bool(int(st[0, 4]) & oracle.FLAG_LINEAR) == (rho > 1.0 + kappa), (r, rho, kappa)
