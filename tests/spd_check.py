"""Parity rules between the HIP path and the FP64 oracle (test helper).

* every per-sample SNR within ``tol`` of the oracle's;
* width index equal, or the oracle's SNR at the GPU's width within ``tol`` of
  the oracle's maximum (near-ties may resolve either way);
* candidate sets equal except entries whose oracle SNR is within ``tol`` of
  the threshold;
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


def check_candidates(cands_g: np.ndarray, cands_o: dict, threshold: float, snr_o_lookup, tol=TOL_SNR,
                     widths=None, width_ok=None):
    """Candidate sets equal except within ``tol`` of the threshold.
    ``snr_o_lookup(row, t)`` returns the oracle's SNR there."""
    g = {(int(c["row"]), int(c["t"])): (float(c["snr"]), int(c["width"])) for c in cands_g}
    o = {(int(r), int(t)): (float(s), int(w)) for r, t, s, w in
         zip(cands_o["row"], cands_o["t"], cands_o["snr"], cands_o["width"])}
    assert len(g) == len(cands_g), "duplicate candidates"
    for k in set(g) ^ set(o):
        s = snr_o_lookup(*k)
        assert abs(s - threshold) <= tol, "candidate %s only on one side (oracle snr %g)" % (k, s)
    for k in set(g) & set(o):
        assert abs(g[k][0] - o[k][0]) <= tol
        if g[k][1] != o[k][1] and width_ok is not None:
            assert width_ok(k, g[k][1]), "candidate %s width %d vs %d" % (k, g[k][1], o[k][1])
    return len(g), len(o)
