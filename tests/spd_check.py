"""Parity rules between the HIP path and the FP64 oracle (test helper).

* every per-sample SNR within ``tol`` of the oracle's;
* width index equal, or the oracle's SNR at the GPU's width within ``tol`` of
  the oracle's maximum (near-ties may resolve either way);
* candidate sets equal except entries whose oracle SNR is within ``tol`` of
  the threshold, and every listed width equal to the oracle's or a near-tie
  by the rule above (the list's four fields of Sec. 2.4);
* statistics: mean and sigma to 1e-6 relative (sigma_Nmax too when used), the
  same flags.
"""
import numpy as np
import torch

import oracle

TOL_SNR = 1e-4
TOL_STAT = 1e-6


def plane_f64(x: torch.Tensor, scale=None, zero=None) -> np.ndarray:
    """Exactly the values the GPU consumed, as FP64."""
    if x.dtype == torch.uint8:
        return oracle.dequantize_u8(x.cpu().numpy(), scale.cpu().numpy(), zero.cpu().numpy())
    return x.cpu().to(torch.float64).numpy()


def check_stats(gpu_stats: np.ndarray, ora_stats: np.ndarray, need_y: bool):
    g = np.asarray(gpu_stats, dtype=np.float64)
    gflags = g.view(np.int32)[:, 8].copy()
    assert np.all(gflags == ora_stats[:, 4].astype(np.int32)), "flags differ"
    np.testing.assert_allclose(g[:, 0], ora_stats[:, 0], rtol=TOL_STAT, atol=TOL_STAT * np.abs(ora_stats[:, 1]).max())
    np.testing.assert_allclose(g[:, 1], ora_stats[:, 1], rtol=TOL_STAT)
    if need_y:
        np.testing.assert_allclose(g[:, 2], ora_stats[:, 2], rtol=TOL_STAT)
        np.testing.assert_allclose(g[:, 3], ora_stats[:, 3], rtol=TOL_STAT, atol=TOL_STAT * np.abs(ora_stats[:, 1]).max())


def check_snr_widx(x64, widths, snr_g, widx_g, snr_o, widx_o, ora_stats, scope="row", tol=TOL_SNR,
                   rows=None):
    """Element-wise parity of the per-sample outputs; ``rows`` maps output rows
    to plane rows when only a sample of rows is checked."""
    snr_g = np.asarray(snr_g, dtype=np.float64)
    d = np.abs(snr_g - snr_o)
    worst = float(d.max()) if d.size else 0.0
    assert worst <= tol, "max |dSNR| = %g > %g at %s" % (worst, tol, np.unravel_index(np.argmax(d), d.shape))
    mism = np.argwhere(np.asarray(widx_g) != widx_o)
    for r, t in mism:
        pr = rows[r] if rows is not None else r
        u = 0 if scope == "plane" else r
        s = oracle.snr_at(x64[r], t, widths[int(widx_g[r, t])], ora_stats[u])
        assert s >= snr_o[r, t] - tol, "row %d t %d: width %d gives %g < max %g" % (
            pr, t, widths[int(widx_g[r, t])], s, snr_o[r, t])
    return worst, len(mism)


def width_rule(x64, widths, stats, scope="row", rows=None, t_offset=0, strides=None):
    """The oracle's SNR of candidate (row, t) at a given width, in candidate
    coordinates: ``row`` a plane row (``rows`` lists the plane rows that
    ``x64`` holds when only a sample was checked), ``t`` a window start plus
    ``t_offset``.  The width must be one of ``widths`` and, where ``strides``
    (one per width) are given, evaluated at that start."""
    wl = [int(w) for w in widths]
    stride_of = dict(zip(wl, [int(s) for s in strides])) if strides is not None else None

    def snr_w(row, t, width):
        assert width in wl, "candidate (%d, %d): width %d is not in the list" % (row, t, width)
        i = rows.index(row) if rows is not None else row
        tt = t - t_offset
        if stride_of is not None:
            assert tt % stride_of[width] == 0, "candidate (%d, %d): width %d is not evaluated there" % (
                row, t, width)
        return oracle.snr_at(x64[i], tt, width, stats[0 if scope == "plane" else i])
    return snr_w


def check_candidates(cands_g: np.ndarray, cands_o: dict, threshold: float, snr_o_lookup, snr_at_width,
                     tol=TOL_SNR):
    """A candidate list against the oracle's, every field of Sec. 2.4.

    * sets of (row, t) equal except entries whose oracle SNR is within ``tol``
      of the threshold;
    * the SNR of every common entry within ``tol`` of the oracle's;
    * the width of every GPU entry equal to the oracle's, or one whose oracle
      SNR at that start is within ``tol`` of the oracle maximum (a near-tie).
    ``snr_o_lookup(row, t)`` returns the oracle's highest SNR there and
    ``snr_at_width(row, t, width)`` its SNR at one width (``width_rule``)."""
    g = {(int(c["row"]), int(c["t"])): (float(c["snr"]), int(c["width"])) for c in cands_g}
    o = {(int(r), int(t)): (float(s), int(w)) for r, t, s, w in
         zip(cands_o["row"], cands_o["t"], cands_o["snr"], cands_o["width"])}
    assert len(g) == len(cands_g), "duplicate candidates"
    for k in set(g) ^ set(o):
        s = snr_o_lookup(*k)
        assert abs(s - threshold) <= tol, "candidate %s only on one side (oracle snr %g)" % (k, s)
    for k, (gs, gw) in g.items():
        if k in o:
            assert abs(gs - o[k][0]) <= tol, "candidate %s snr %g vs %g" % (k, gs, o[k][0])
            if gw == o[k][1]:
                continue
        smax = snr_o_lookup(*k)
        s = snr_at_width(k[0], k[1], gw)
        assert s >= smax - tol, "candidate %s width %d gives oracle snr %g < max %g" % (k, gw, s, smax)
    return len(g), len(o)
