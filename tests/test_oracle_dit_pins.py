"""Pins of the decimated search in the oracle (boxcars combined with
decimation in time, the direction Sec. 3 gives for wide boxcars).

The oracle evaluates width 2^l*w only at starts that are multiples of 2^l (a
per-width start stride in the exhaustive C loop).  These checks tie that to
things other than the C code itself:

* an explicit decimation in numpy -- the series summed pairwise l times, a
  boxcar of w decimated samples -- must give the same per-start maximum and
  first maximiser (brute force on small planes);
* with every stride 1 the strided loop is the exhaustive one, bit for bit;
* with no decimated level it is the exhaustive search over 1..16;
* the evaluated windows are a subset of the exhaustive ones, so no start can
  score higher, and starts on the coarsest grid score the same;
* a pulse on the grid is recovered at exactly its exhaustive SNR.
"""
import numpy as np
import pytest

import oracle


def _stats(x, widths, mode="sqrtn"):
    _, st, snr, widx = oracle.stream_step(x, widths, sigma_mode=mode)
    return st, snr, widx


def _snr(b, w, st):
    mean, sigma, _, coef, flags = (float(v) for v in st)
    sw = np.sqrt(w) * sigma + (w - 1) * coef
    if int(flags) & oracle.FLAG_ZERO_VAR or not sw > oracle.SW_FLOOR * np.sqrt(w) * sigma:
        return 0.0
    return (b - w * mean) / sw


def _brute_by_decimation(x, levels, base, stats):
    """Per start: the best window among level 0 (widths 1..base on x) and, for
    every level l whose grid holds the start, widths base/2+1..base on the
    series decimated l times; ascending physical width, strict '>'."""
    R, L = x.shape
    nmax = base << levels
    n_out = L - nmax + 1
    snr = np.zeros((R, n_out))
    idx = np.zeros((R, n_out), dtype=np.int64)
    gap = np.zeros((R, n_out))                   # best minus runner-up, for tie-safe width checks
    for r in range(R):
        dec = [x[r]]
        for lv in range(1, levels + 1):
            p = dec[-1]
            n2 = len(p) // 2
            dec.append(p[0:2 * n2:2] + p[1:2 * n2:2])
        for t in range(n_out):
            vals = []
            for w in range(1, base + 1):
                vals.append(_snr(float(np.sum(x[r, t:t + w])), w, stats[r]))
            for lv in range(1, levels + 1):
                for w in range(base // 2 + 1, base + 1):
                    if t % (1 << lv) == 0:
                        tp = t >> lv
                        vals.append(_snr(float(np.sum(dec[lv][tp:tp + w])), w << lv, stats[r]))
                    else:
                        vals.append(-np.inf)
            v = np.array(vals)
            best = -np.inf
            bi = 0
            for i, s in enumerate(v):
                if s > best:
                    best, bi = s, i
            snr[r, t] = best
            idx[r, t] = bi
            srt = np.sort(v[np.isfinite(v)])
            gap[r, t] = srt[-1] - srt[-2] if srt.size > 1 else np.inf
    return snr, idx, gap


def test_widths_and_strides():
    w, s = oracle.dit_widths(4)
    assert w[:16] == list(range(1, 17)) and s[:16] == [1] * 16
    assert w[16:24] == list(range(18, 33, 2)) and s[16:24] == [2] * 8
    assert w[24:32] == list(range(36, 65, 4)) and w[32:40] == list(range(72, 129, 8))
    assert w[40:] == list(range(144, 257, 16)) and s[40:] == [16] * 8
    assert oracle.dit_widths(0) == (list(range(1, 17)), [1] * 16)
    w, s = oracle.dit_widths(2, base=4)
    assert w == [1, 2, 3, 4, 6, 8, 12, 16] and s == [1, 1, 1, 1, 2, 2, 4, 4]


@pytest.mark.parametrize("levels,base,mode", [(2, 8, "sqrtn"), (3, 4, "linear"), (1, 16, "auto")])
def test_matches_explicit_decimation(levels, base, mode):
    rng = np.random.default_rng(40 + levels)
    x = rng.standard_normal((3, 260)) + np.array([[0.0], [2.0], [-1.0]])
    x[1, 100:140] += 3.0                                       # a bright stretch: linear sigma_N on that row
    x[2, 64:64 + (base << levels) // 2] += 1.5
    widths, strides = oracle.dit_widths(levels, base)
    _, st, snr, widx = oracle.stream_step(x, widths, sigma_mode=mode, strides=strides)
    bs, bi, gap = _brute_by_decimation(x, levels, base, st)
    np.testing.assert_allclose(snr, bs, rtol=0, atol=1e-9)
    clear = gap > 1e-9
    assert np.array_equal(widx[clear], bi[clear])


def test_level_zero_is_the_exhaustive_search():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((4, 3000))
    d = oracle.dit_detect(x, 0, 4.0)
    e = oracle.detect(x, list(range(1, 17)), 4.0)
    assert np.array_equal(d["snr"], e["snr"]) and np.array_equal(d["widx"], e["widx"])


def test_unit_strides_are_the_exhaustive_loop():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((3, 2000))
    w, _ = oracle.dit_widths(3)
    a = oracle.stream_step(x, w, sigma_mode="auto")
    b = oracle.stream_step(x, w, sigma_mode="auto", strides=[1] * len(w))
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_subset_bound_and_coarsest_grid():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((4, 5000))
    x[2, 1000:1100] += 1.0
    levels = 3
    w, s = oracle.dit_widths(levels)
    _, _, ex, exw = oracle.stream_step(x, w)
    d = oracle.dit_detect(x, levels, 5.0)
    assert np.all(d["snr"] <= ex + 1e-12)
    grid = np.arange(0, ex.shape[1], 1 << levels)
    assert np.array_equal(d["snr"][:, grid], ex[:, grid]) and np.array_equal(d["widx"][:, grid], exw[:, grid])
    off = np.setdiff1d(np.arange(ex.shape[1]), grid)
    assert np.any(d["snr"][:, off] < ex[:, off])               # the decimated search does miss windows


@pytest.mark.parametrize("lv,w,t0", [(1, 12, 600), (2, 10, 1204), (3, 16, 2000), (4, 9, 3200)])
def test_pulse_on_the_grid_is_found_at_its_exhaustive_snr(lv, w, t0):
    rng = np.random.default_rng(100 + lv)
    L = 8192
    x = rng.standard_normal((1, L))
    width = w << lv
    assert t0 % (1 << lv) == 0
    x[0, t0:t0 + width] += 12.0 / np.sqrt(width)
    widths, strides = oracle.dit_widths(4)
    d = oracle.dit_detect(x, 4, 6.0)
    _, st, ex, _ = oracle.stream_step(x, widths)
    k = widths.index(width)
    direct = oracle.snr_at(x[0], t0, width, st[0])
    assert d["snr"][0, t0] >= direct - 1e-12                    # that window is evaluated at t0
    assert d["snr"][0, t0] <= ex[0, t0] + 1e-12
    lo, hi = max(0, t0 - width), t0 + width
    assert np.max(d["snr"][0, lo:hi]) >= direct - 1e-12 and direct > 8.0
    assert strides[k] == 1 << lv
