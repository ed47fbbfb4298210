"""Brute-force restatement of the detection path for tiny planes.

TEST INFRASTRUCTURE ONLY: a second, independent way to compute what the C
oracle computes, used to pin it.  It avoids every shortcut of the streaming
method on purpose: mean and variance by the textbook two-pass formula, every
boxcar as a separate direct sum, every SNR evaluated, then max and first
argmax taken over the list.  Pure Python loops; keep inputs small.
"""
from __future__ import annotations

import math

SW_FLOOR = 1e-9   # sigma_w counts as positive above SW_FLOOR * sqrt(w) * sigma


def two_pass(values):
    """Population mean and the sum of squared deviations, two passes."""
    n = len(values)
    mu = sum(values) / n
    return mu, sum((v - mu) ** 2 for v in values)


def sigma_widths(widths, sigma, coef):
    """sigma_w = sqrt(w)*sigma + (w-1)*coef (Sec. 2.2, Eq. sd02 / sd03)."""
    return [math.sqrt(w) * sigma + (w - 1) * coef for w in widths]


def unit_stats(rows, widths, sigma_mode="sqrtn", kappa=1.0):
    """(mu, sigma, sigma_Nmax, coef, flags) of the samples in ``rows``."""
    samples = [v for row in rows for v in row]
    mu, ss = two_pass(samples)
    sigma = math.sqrt(ss / len(samples))
    nmax = widths[-1]
    ys = [sum(row[t:t + nmax]) for row in rows for t in range(len(row) - nmax + 1)]
    _, ssy = two_pass(ys)
    sig_n = math.sqrt(ssy / len(ys))
    coef, flags = 0.0, 0
    if sigma == 0.0:
        return mu, sigma, sig_n, 0.0, 1
    if nmax > 1 and sigma_mode != "sqrtn":
        base = math.sqrt(nmax) * sigma
        anchored = (sig_n - base) / (nmax - 1)
        if sigma_mode == "linear":
            coef, flags = anchored, 2
        elif sigma_mode == "linear_literal":
            coef, flags = sig_n / (nmax - 1), 2
        elif sigma_mode == "auto" and sig_n / base > 1.0 + kappa:
            coef, flags = anchored, 2
    return mu, sigma, sig_n, coef, flags


def detect(plane, widths, threshold, scope="row", sigma_mode="sqrtn", kappa=1.0):
    """snr[r][t], widx[r][t] and the candidate list, by exhaustive evaluation."""
    nmax = widths[-1]
    units = [[row] for row in plane] if scope == "row" else [list(plane)]
    stats = [unit_stats(u, widths, sigma_mode, kappa) for u in units]
    snr, widx, cands = [], [], []
    for r, row in enumerate(plane):
        mu, sigma, _, coef, flags = stats[0 if scope == "plane" else r]
        sw = sigma_widths(widths, sigma, coef)
        srow, irow = [], []
        for t in range(len(row) - nmax + 1):
            vals = []
            for i, w in enumerate(widths):
                if flags & 1 or sw[i] <= SW_FLOOR * math.sqrt(w) * sigma:
                    vals.append(0.0)
                else:
                    vals.append((sum(row[t:t + w]) - w * mu) / sw[i])
            best = max(vals)
            bi = vals.index(best)            # first maximiser
            srow.append(best)
            irow.append(bi)
            if best >= threshold:
                cands.append((r, t, best, widths[bi]))
        snr.append(srow)
        widx.append(irow)
    return {"stats": stats, "snr": snr, "widx": widx, "cands": cands}
