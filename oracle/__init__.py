"""FP64 CPU oracle of the single-pulse detection path (arXiv:1611.09704).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product library
never calls it, and it shares no code with the HIP path: the C file next to this
one is compiled with gcc, on its own, into ``libspd_oracle.so``.

The functions follow the paper's steps:

* ``chan_stream`` -- Sec. 2.1, Eq. (MSD03), the serial streaming update;
* ``chan_merge`` -- Sec. 2.1, Eq. (MSD04), the pairwise merge;
* ``stream_step`` / ``detect`` -- Sec. 2.1-2.3 and Algorithm 1: statistics per
  unit, sigma_N from Eq. (sd02) or the linear form Eq. (sd03), the highest SNR
  over the width list and the first width that reaches it;
* ``select`` -- Sec. 2.4, the SNR threshold and the candidate list;
* ``dit_widths`` / ``dit_detect`` -- boxcars combined with decimation in time
  (the direction Sec. 3 names for wide boxcars): the same definition with
  width 2^l*w evaluated only at starts that are multiples of 2^l;
* ``cluster_peaks`` -- peak-finding over the candidates of Sec. 2.4 (a step
  the paper leaves out: its list is unclustered): a candidate is kept iff no
  sample within the DM-row and time radii has a higher SNR, and no sample
  there with the same SNR comes first in row-major order;
* ``dedisp_channel_factors`` / ``dedisp_delays`` / ``dedisperse`` -- the step
  before the path (Sec. 1: detection runs on de-dispersed series): brute-force
  incoherent de-dispersion of a frequency x time filterbank, the sum over
  channels of each channel shifted by its cold-plasma dispersion delay,
  rounded to whole samples.

The readings taken where the paper is silent or garbled are listed in the
header of ``spd_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spd_oracle.c")
_LIB = os.environ.get("SPD_ORACLE_LIB") or os.path.join(_HERE, "libspd_oracle.so")   # override: pin checks
_lock = threading.Lock()
_lib = None

SCOPES = {"row": 0, "plane": 1}
SIGMA_MODES = {"sqrtn": 0, "linear": 1, "auto": 2, "linear_literal": 3}
FLAG_ZERO_VAR = 1
FLAG_LINEAR = 2
# sigma_w counts as positive above SW_FLOOR * sqrt(w) * sigma: the anchored form of
# Eq. (sd03) reaches zero at w = Nmax when sigma_Nmax = 0, where its rounding
# residual can take either sign.
SW_FLOOR = 1e-9


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP over rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.environ.get("SPD_ORACLE_LIB") and (
                    not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            d, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
            lib.oracle_chan_stream.argtypes = [d, i64, d]
            lib.oracle_chan_stream.restype = None
            lib.oracle_chan_merge.argtypes = [d, d, d]
            lib.oracle_chan_merge.restype = None
            lib.oracle_stream_step.argtypes = [d, i64, i64, i64, d, i32, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_double, d, d, d, d, ctypes.c_int]
            lib.oracle_stream_step.restype = ctypes.c_int
            lib.oracle_stream_step_strided.argtypes = [d, i64, i64, i64, d, d, i32, ctypes.c_int, ctypes.c_int,
                                                       ctypes.c_double, d, d, d, d, ctypes.c_int]
            lib.oracle_stream_step_strided.restype = ctypes.c_int
            lib.oracle_select.argtypes = [d, d, i64, i64, d, ctypes.c_double, i64, d, d, d, d, i64]
            lib.oracle_select.restype = i64
            lib.oracle_max_threads.argtypes = []
            lib.oracle_max_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def chan_stream(x) -> np.ndarray:
    """(n, T, S) of a sequence by the streaming update, Eq. (MSD03)."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    out = np.zeros(3)
    _load().oracle_chan_stream(_ptr(x), x.size, _ptr(out))
    return out


def chan_merge(a, b) -> np.ndarray:
    """Merge two (n, T, S) partials with Eq. (MSD04)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    out = np.zeros(3)
    _load().oracle_chan_merge(_ptr(a), _ptr(b), _ptr(out))
    return out


def new_state(n_units: int) -> np.ndarray:
    """Empty running state {n, T, S, n_y, T_y, S_y} per unit."""
    return np.zeros((n_units, 6))


def stream_step(x, widths, *, new_col_begin=0, state=None, scope="row", sigma_mode="sqrtn",
                kappa=1.0, nthreads=None, strides=None):
    """One step over a plane view; returns (state, stats, snr, widx).

    ``stats`` has one row per unit: mean, sigma, sigma_Nmax, linear coefficient,
    flags.  ``snr``/``widx`` have shape (R, L_view - Nmax + 1); ``widx`` indexes
    ``widths``.  ``strides`` (optional, one per width, the first 1) evaluates
    width i only at starts that are multiples of strides[i].
    """
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim != 2:
        raise ValueError("plane must be 2-D")
    R, L = x.shape
    W = np.ascontiguousarray(widths, dtype=np.int32)
    nmax = int(W[-1])
    n_units = 1 if scope == "plane" else R
    if state is None:
        state = new_state(n_units)
    state = np.ascontiguousarray(state, dtype=np.float64).copy()
    if state.shape != (n_units, 6):
        raise ValueError("state shape mismatch")
    stats = np.zeros((n_units, 5))
    n_out = L - nmax + 1
    if n_out < 1:
        raise ValueError("plane shorter than the widest boxcar")
    snr = np.zeros((R, n_out))
    widx = np.zeros((R, n_out), dtype=np.int32)
    if strides is None:
        rc = _load().oracle_stream_step(_ptr(x), R, L, int(new_col_begin), _ptr(W), W.size,
                                        SCOPES[scope], SIGMA_MODES[sigma_mode], float(kappa),
                                        _ptr(state), _ptr(stats), _ptr(snr), _ptr(widx),
                                        int(nthreads or default_threads()))
    else:
        S = np.ascontiguousarray(strides, dtype=np.int32)
        if S.shape != W.shape:
            raise ValueError("one stride per width")
        rc = _load().oracle_stream_step_strided(_ptr(x), R, L, int(new_col_begin), _ptr(W), _ptr(S), W.size,
                                                SCOPES[scope], SIGMA_MODES[sigma_mode], float(kappa),
                                                _ptr(state), _ptr(stats), _ptr(snr), _ptr(widx),
                                                int(nthreads or default_threads()))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return state, stats, snr, widx


def select(snr, widx, widths, threshold, t_offset=0):
    """Candidate list of Sec. 2.4 as a dict of arrays (row-major order)."""
    snr = np.ascontiguousarray(snr, dtype=np.float64)
    widx = np.ascontiguousarray(widx, dtype=np.int32)
    W = np.ascontiguousarray(widths, dtype=np.int32)
    R, n_out = snr.shape
    lib = _load()
    cap = 0
    total = lib.oracle_select(_ptr(snr), _ptr(widx), R, n_out, _ptr(W), float(threshold),
                              int(t_offset), None, None, None, None, cap)
    rows = np.zeros(total, dtype=np.int64)
    ts = np.zeros(total, dtype=np.int64)
    ss = np.zeros(total)
    ws = np.zeros(total, dtype=np.int32)
    lib.oracle_select(_ptr(snr), _ptr(widx), R, n_out, _ptr(W), float(threshold), int(t_offset),
                      _ptr(rows), _ptr(ts), _ptr(ss), _ptr(ws), total)
    return {"row": rows, "t": ts, "snr": ss, "width": ws}


def detect(x, widths, threshold, *, scope="row", sigma_mode="sqrtn", kappa=1.0, nthreads=None):
    """The whole path on one plane, one shot: stats, snr, widx and candidates."""
    _, stats, snr, widx = stream_step(x, widths, scope=scope, sigma_mode=sigma_mode,
                                      kappa=kappa, nthreads=nthreads)
    cands = select(snr, widx, widths, threshold)
    return {"stats": stats, "snr": snr, "widx": widx, "cands": cands}


def dit_widths(levels: int, base: int = 16):
    """Widths and start strides of boxcars combined with decimation in time.

    Level 0 runs widths 1..base on the series itself.  Level l >= 1 runs
    widths base/2+1..base on the series decimated l times (adjacent pairs
    summed each time): physical width 2^l*w at starts that are multiples of
    2^l.  Returned in ascending width order, as (widths, strides)."""
    if base < 2 or base % 2 or levels < 0:
        raise ValueError("base must be even and >= 2, levels >= 0")
    widths = list(range(1, base + 1))
    strides = [1] * base
    for lv in range(1, levels + 1):
        for w in range(base // 2 + 1, base + 1):
            widths.append(w << lv)
            strides.append(1 << lv)
    return widths, strides


def dit_detect(x, levels, threshold, *, base=16, scope="row", sigma_mode="sqrtn", kappa=1.0, nthreads=None):
    """The decimated search on one plane, one shot: for every start the highest
    SNR over the widths evaluated there (first maximiser in ascending width),
    and the candidates.  Statistics are those of the exhaustive path over the
    same width list."""
    widths, strides = dit_widths(levels, base)
    _, stats, snr, widx = stream_step(x, widths, scope=scope, sigma_mode=sigma_mode, kappa=kappa,
                                      nthreads=nthreads, strides=strides)
    cands = select(snr, widx, widths, threshold)
    return {"stats": stats, "snr": snr, "widx": widx, "cands": cands, "widths": widths, "strides": strides}


def cluster_peaks(snr, threshold, dm_radius, t_radius):
    """Peaks among the candidates (snr >= threshold) of a snr plane [rows][starts].

    (r, t) is a peak iff snr[r, t] >= threshold and every other (r', t') with
    |r' - r| <= dm_radius and |t' - t| <= t_radius inside the plane has
    snr[r', t'] < snr[r, t], or an equal SNR and a later row-major position.
    Returns row and t arrays in row-major order."""
    snr = np.asarray(snr, dtype=np.float64)
    R, L = snr.shape
    rows, ts = [], []
    for r, t in np.argwhere(snr >= threshold):
        v = snr[r, t]
        r0, r1 = max(0, r - dm_radius), min(R, r + dm_radius + 1)
        t0, t1 = max(0, t - t_radius), min(L, t + t_radius + 1)
        win = snr[r0:r1, t0:t1]
        if np.any(win > v):
            continue
        rr, tt = np.nonzero(win == v)
        rr, tt = rr + r0, tt + t0
        if np.any((rr < r) | ((rr == r) & (tt < t))):
            continue
        rows.append(int(r))
        ts.append(int(t))
    return {"row": np.array(rows, dtype=np.int64), "t": np.array(ts, dtype=np.int64)}


# Dispersion constant of the cold-plasma delay law, in MHz^2 pc^-1 cm^3 s:
# a signal at frequency f (MHz) through dispersion measure DM (pc cm^-3)
# arrives KDM * DM / f^2 seconds later than at infinite frequency.
KDM = 4.148808e3


def dedisp_channel_factors(n_chan, f_top_mhz, chan_bw_mhz, t_samp_s):
    """k_c, the delay of channel c relative to channel 0 per unit DM, in samples:
    KDM * (1/f_c^2 - 1/f_top^2) / t_samp with f_c = f_top - c * chan_bw
    (channel 0 is the highest frequency).  FP64, evaluated in that order."""
    f = float(f_top_mhz) - np.arange(int(n_chan), dtype=np.float64) * float(chan_bw_mhz)
    ft = float(f_top_mhz)
    return KDM * (1.0 / (f * f) - 1.0 / (ft * ft)) / float(t_samp_s)


def dedisp_delays(dm, kc) -> np.ndarray:
    """Delay of channel c at trial DM d, rounded to the nearest sample (halves
    up): floor(dm[d] * k_c + 0.5), the product and the sum each rounded in
    FP64.  int64 [n_dm][n_chan]."""
    dm = np.asarray(dm, dtype=np.float64)
    kc = np.asarray(kc, dtype=np.float64)
    return np.floor(dm[:, None] * kc[None, :] + 0.5).astype(np.int64)


def dedisperse(fb, dm, kc) -> np.ndarray:
    """De-dispersed series of a filterbank fb [n_chan][n_samp]: for every trial
    d and every t < n_samp - max delay, y[d][t] = sum over channels c of
    fb[c][t + delay[d][c]].  Summed in FP64 (exact for 8-bit samples).
    Returns [n_dm][n_out]."""
    fb = np.asarray(fb)
    delays = dedisp_delays(dm, kc)
    n_out = fb.shape[1] - int(delays.max())
    if n_out <= 0:
        raise ValueError("the series is shorter than the largest delay")
    out = np.zeros((delays.shape[0], n_out), dtype=np.float64)
    for d in range(delays.shape[0]):
        for c in range(fb.shape[0]):
            k = int(delays[d, c])
            out[d] += fb[c, k:k + n_out]
    return out


def dequantize_u8(q, scale, zero) -> np.ndarray:
    """Exact FP64 value of a per-row quantised plane: x = scale_r * (q - zero_r)."""
    q = np.asarray(q, dtype=np.float64)
    s = np.asarray(scale, dtype=np.float64).reshape(-1, 1)
    z = np.asarray(zero, dtype=np.float64).reshape(-1, 1)
    return s * (q - z)


def snr_at(row, t, width, unit_stats):
    """SNR of one boxcar, Sec. 2.3 with sigma_w of Eq. (sd02)/(sd03):
    (sum_{k<w} x[t+k] - w*mean) / (sqrt(w)*sigma + (w-1)*coef); 0 for a
    ZERO_VAR unit or a non-positive sigma_w.  ``unit_stats`` is one row of the
    ``stats`` array returned by ``stream_step``."""
    mean, sigma, _, coef, flags = (float(v) for v in unit_stats)
    sw = np.sqrt(width) * sigma + (width - 1) * coef
    if int(flags) & FLAG_ZERO_VAR or not sw > SW_FLOOR * np.sqrt(width) * sigma:
        return 0.0
    b = float(np.sum(np.asarray(row[t:t + width], dtype=np.float64)))
    return (b - width * mean) / sw
