"""The parity checker itself (CPU): given the oracle's own candidate list it
passes, and it fails when one field of one candidate is wrong -- in particular
a width that is not the first maximiser and not a near-tie, a width outside the
list, or a width the decimated search does not evaluate at that start."""
import numpy as np
import pytest

import oracle
import spd_check as C


def _case(seed=3, R=4, L=3000, widths=tuple(range(1, 17)), thr=4.0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((R, L))
    x[1, 700:709] += 2.0
    x[2, 1500:1503] += 3.0
    o = oracle.detect(x, list(widths), thr)
    cands = np.zeros(len(o["cands"]["row"]), dtype=[("row", "<i4"), ("width", "<i4"), ("t", "<i8"),
                                                    ("snr", "<f4"), ("beam", "<u4")])
    for f in ("row", "width", "t", "snr"):
        cands[f] = o["cands"][f]
    return x, list(widths), o, cands


def _check(x, widths, o, cands, thr=4.0, **kw):
    return C.check_candidates(cands, o["cands"], thr, lambda r, t: o["snr"][r, t],
                              C.width_rule(x, widths, o["stats"], **kw))


def test_oracle_list_passes():
    x, W, o, c = _case()
    assert len(c) >= 5
    _check(x, W, o, c)


def test_wrong_width_is_caught():
    x, W, o, c = _case()
    i = int(np.argmax(c["snr"]))                   # the brightest candidate: no near-tie across widths
    r, t = int(c["row"][i]), int(c["t"][i])
    bad = next(w for w in W if oracle.snr_at(x[r], t, w, o["stats"][r]) < o["snr"][r, t] - 1e-3)
    c["width"][i] = bad
    with pytest.raises(AssertionError, match="width"):
        _check(x, W, o, c)


def test_width_outside_the_list_is_caught():
    x, W, o, c = _case(widths=(1, 2, 4, 8, 16))
    c["width"][0] = 3
    with pytest.raises(AssertionError, match="not in the list"):
        _check(x, W, o, c)


def test_near_tie_width_is_accepted():
    # integer samples summing to zero, so the mean is exactly 0: at t = 50 the
    # window [3, 1, 1, 1] gives SNR_1 = 3/sigma and SNR_4 = 6/(2 sigma), an exact
    # tie (the oracle reports the first, width 1); width 2 gives 4/(sqrt(2) sigma),
    # 6% lower
    x = np.zeros((1, 200))
    x[0, 50:54] = [3, 1, 1, 1]
    x[0, 150:154] = [-3, -1, -1, -1]
    W = [1, 2, 3, 4]
    o = oracle.detect(x, W, 5.0)
    assert o["stats"][0, 0] == 0.0
    c = np.zeros(len(o["cands"]["row"]), dtype=[("row", "<i4"), ("width", "<i4"), ("t", "<i8"),
                                                ("snr", "<f4"), ("beam", "<u4")])
    for f in ("row", "width", "t", "snr"):
        c[f] = o["cands"][f]
    i = int(np.nonzero(c["t"] == 50)[0][0])
    assert c["width"][i] == 1
    c["width"][i] = 4
    _check(x, W, o, c, thr=5.0)
    c["width"][i] = 2
    with pytest.raises(AssertionError, match="width 2"):
        _check(x, W, o, c, thr=5.0)


def test_dit_width_off_its_grid_is_caught():
    rng = np.random.default_rng(8)
    x = rng.standard_normal((2, 4000))
    x[0, 1000:1040] += 1.5
    o = oracle.dit_detect(x, 2, 4.0)
    c = np.zeros(len(o["cands"]["row"]), dtype=[("row", "<i4"), ("width", "<i4"), ("t", "<i8"),
                                                ("snr", "<f4"), ("beam", "<u4")])
    for f in ("row", "width", "t", "snr"):
        c[f] = o["cands"][f]
    rule = C.width_rule(x, o["widths"], o["stats"], strides=o["strides"])
    C.check_candidates(c, o["cands"], 4.0, lambda r, t: o["snr"][r, t], rule)
    odd = [i for i in range(len(c)) if c["t"][i] % 4 != 0]
    assert odd
    c["width"][odd[0]] = 36                            # 4*9: only at starts divisible by 4
    with pytest.raises(AssertionError, match="not evaluated there|width"):
        C.check_candidates(c, o["cands"], 4.0, lambda r, t: o["snr"][r, t], rule)
