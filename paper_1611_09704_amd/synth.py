"""Seeded synthetic DM-trial x time planes with injected pulses.

This module only makes input data: it holds none of the detection method's
arithmetic, and both the HIP path's tests and the oracle's tests draw their
inputs from it.  The paper measures on survey data that is not available here
(SKA-like, ~6000 DM trials at 64 us sampling, Sec. 3), so seeded synthetic
planes of the same shape and structure stand in for it:

* rows are DM trials, columns are time samples (time contiguous);
* noise is Gaussian, optionally with a per-row offset and scale;
* a pulse is a rectangle of width ``w`` and "true SNR" ``s``: amplitude
  ``s * sigma_row / sqrt(w)``, so its width-``w`` boxcar rises ``s`` noise
  standard deviations above the mean;
* "signal-dominated" rows carry one long bright block (a fraction of the row
  at a fixed multiple of the row's sigma) -- the case the paper's linear
  approximation of sigma_N is for (Sec. 2.2).

Bulk noise is drawn with torch on the target device (a CUDA tensor on a GPU
box, so even the 17 GB plane is generated in place); every structural choice
(offsets, scales, pulse rows, times, widths, SNRs) is drawn on the host with
NumPy's PCG64 from ``numpy.random.SeedSequence(seed)``, so it is identical on
every device.  Parity checks always feed the oracle the exact bytes the GPU
consumed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

BASE_SEED = 1611097040


@dataclass
class Pulse:
    row: int
    t0: int
    width: int
    snr: float
    amp: float


@dataclass
class Plane:
    x: torch.Tensor                    # [R, L] float32
    row_mu: np.ndarray                 # offset used per row
    row_sigma: np.ndarray              # noise sigma used per row
    pulses: List[Pulse] = field(default_factory=list)
    bright_rows: List[int] = field(default_factory=list)


def _widths_range(a: int, b: int, step: int = 1) -> List[int]:
    return list(range(a, b + 1, step))


def make_plane(R: int, L: int, *, seed: int, device="cpu", n_pulses: int = 0,
               pulse_widths: Sequence[int] = (1,), snr_range: Tuple[float, float] = (8.0, 20.0),
               fixed_widths: bool = False, gap: int = 0, mean_range: Optional[Tuple[float, float]] = None,
               scale_range: Optional[Tuple[float, float]] = None, n_bright: int = 0,
               bright_frac: float = 0.3, bright_amp: float = 2.0, t_margin: int = 0) -> Plane:
    """Gaussian plane with per-row offset/scale, rectangular pulses and bright rows.

    ``fixed_widths`` places exactly one pulse of each width in ``pulse_widths``;
    otherwise widths are drawn uniformly from it.  Pulse starts are uniform in
    [0, L - t_margin - w] and pulses sharing a row keep ``gap`` samples apart.
    """
    ss = np.random.SeedSequence(seed)
    host_ss, dev_ss = ss.spawn(2)
    rng = np.random.Generator(np.random.PCG64(host_ss))
    row_mu = rng.uniform(*mean_range, size=R) if mean_range else np.zeros(R)
    row_sigma = rng.uniform(*scale_range, size=R) if scale_range else np.ones(R)
    row_mu = row_mu.astype(np.float32).astype(np.float64)
    row_sigma = row_sigma.astype(np.float32).astype(np.float64)

    bright = sorted(rng.choice(R, size=n_bright, replace=False).tolist()) if n_bright else []
    bright_set = set(bright)
    free_rows = np.array([r for r in range(R) if r not in bright_set])
    if fixed_widths:
        widths = list(pulse_widths)
        n_pulses = len(widths)
    else:
        widths = rng.choice(np.asarray(pulse_widths), size=n_pulses).tolist() if n_pulses else []
    snrs = rng.uniform(*snr_range, size=n_pulses).tolist()
    if n_pulses <= free_rows.size:
        rows = rng.choice(free_rows, size=n_pulses, replace=False).tolist()
    else:
        rows = rng.choice(free_rows, size=n_pulses, replace=True).tolist()
    pulses: List[Pulse] = []
    taken = {}
    for r, w, s in zip(rows, widths, snrs):
        for _ in range(1000):
            t0 = int(rng.integers(0, L - t_margin - w + 1))
            if all(abs(t0 - o) >= gap + max(w, ow) for o, ow in taken.get(r, [])):
                break
        taken.setdefault(r, []).append((t0, w))
        amp = float(s * row_sigma[r] / np.sqrt(w))
        pulses.append(Pulse(int(r), t0, int(w), float(s), amp))
    bright_starts = [int(rng.integers(0, L - int(bright_frac * L) + 1)) for _ in bright]

    g = torch.Generator(device=device)
    g.manual_seed(int(dev_ss.generate_state(1, dtype=np.uint64)[0] % (2 ** 63)))
    x = torch.randn((R, L), generator=g, device=device, dtype=torch.float32)
    if scale_range:
        x.mul_(torch.as_tensor(row_sigma, dtype=torch.float32, device=device).view(R, 1))
    if mean_range:
        x.add_(torch.as_tensor(row_mu, dtype=torch.float32, device=device).view(R, 1))
    for p in pulses:
        x[p.row, p.t0:p.t0 + p.width] += p.amp
    nb = int(bright_frac * L)
    for r, t0 in zip(bright, bright_starts):
        x[r, t0:t0 + nb] += float(bright_amp * row_sigma[r])
    return Plane(x=x, row_mu=row_mu, row_sigma=row_sigma, pulses=pulses, bright_rows=bright)


# ---------------------------------------------------------------------------
# The workloads.  Each returns the plane plus the detection parameters.
# ---------------------------------------------------------------------------

def tiny(device="cpu", R: int = 64, L: int = 65536, seed: int = BASE_SEED + 0) -> dict:
    """64 DM x 65,536 FP32 N(0,1); pulses of widths 1,3,8,17,32 at SNR 8-20;
    widths 1..32, threshold 6, sigma_N = sqrt(N)*sigma, per-row statistics."""
    pl = make_plane(R, L, seed=seed, device=device, pulse_widths=(1, 3, 8, 17, 32),
                    fixed_widths=True, snr_range=(8.0, 20.0), gap=32, t_margin=31)
    return dict(plane=pl, widths=_widths_range(1, 32), threshold=6.0, sigma_mode="sqrtn",
                scope="row", kappa=1.0, name="tiny-64x65536-f32")


SKA_WIDTHS = _widths_range(1, 16) + _widths_range(18, 256, 2)


def ska(device="cpu", R: int = 4096, L: int = 1 << 20, seed: int = BASE_SEED + 1,
        widths: Optional[Sequence[int]] = None, n_pulses: Optional[int] = None,
        n_bright: Optional[int] = None) -> dict:
    """SKA-like plane: 4,096 DM x 2^20 FP32, per-row offset U(-5,5) and scale
    U(0.5,2), 200 pulses (widths 1-256, SNR 6-50), 8 signal-dominated rows
    (30% of the row at 2 sigma); widths 1..16 then 18..256 step 2; threshold 7;
    the linear sigma_N correction where a row is signal dominated (kappa = 1)."""
    if n_pulses is None:
        n_pulses = max(1, round(200 * R / 4096)) if R < 4096 else 200
    if n_bright is None:
        n_bright = 8 if R >= 64 else min(2, R)
    pl = make_plane(R, L, seed=seed, device=device, n_pulses=n_pulses,
                    pulse_widths=_widths_range(1, 256), snr_range=(6.0, 50.0), gap=256,
                    mean_range=(-5.0, 5.0), scale_range=(0.5, 2.0), n_bright=n_bright,
                    bright_frac=0.3, bright_amp=2.0, t_margin=255)
    return dict(plane=pl, widths=list(widths) if widths is not None else list(SKA_WIDTHS),
                threshold=7.0, sigma_mode="auto", scope="row", kappa=1.0,
                name="ska-%dx%d-f32" % (R, L))


def quantize_f16(x: torch.Tensor) -> torch.Tensor:
    """FP16 storage: round to nearest even."""
    return x.to(torch.float16)


def quantize_u8(x: torch.Tensor, row_sigma, counts_per_sigma: float = 20.0, zero: float = 64.0,
                row_mu=None):
    """Per-row uint8 storage q = clamp(rint(x / s_r) + z_r, 0, 255) with
    s_r = sigma_r / counts_per_sigma and z_r = 64 (noise at ~20 counts, range
    -3.2 to +9.6 sigma); with ``row_mu`` given, z_r = 64 - rint(mu_r / s_r) so
    each row's mean sits at 64 counts.  Returns (q, scale[R] f32, zero[R] f32)."""
    R = x.shape[0]
    s64 = np.asarray(row_sigma, dtype=np.float64) / counts_per_sigma
    scale = torch.as_tensor(s64, dtype=torch.float32, device=x.device)
    z64 = np.full(R, zero)
    if row_mu is not None:
        z64 = zero - np.rint(np.asarray(row_mu, dtype=np.float64) / scale.cpu().double().numpy())
    z = torch.as_tensor(z64, dtype=torch.float32, device=x.device)
    q = torch.round(x / scale.view(R, 1)) + z.view(R, 1)
    q = q.clamp_(0, 255).to(torch.uint8)
    return q, scale, z


# ---------------------------------------------------------------------------
# Batched beams: uneven shapes, one plane per beam.
# ---------------------------------------------------------------------------

BATCH_ROWS = (256, 512, 1024, 2048, 4096)


def batch_shapes(n_beams: int = 48, seed: int = BASE_SEED + 3, max_samples: Optional[int] = None,
                 rows=BATCH_ROWS, log2_len=(16, 21)) -> List[Tuple[int, int]]:
    """Beam shapes: rows from ``rows``, length 2^e with e uniform in ``log2_len``.
    When ``max_samples`` is given, the first sub-seed (counting up from
    ``seed``) whose total fits is used, so the draw is fixed and reproducible."""
    s = seed
    while True:
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(s)))
        shapes = [(int(rng.choice(rows)), int(2 ** rng.integers(log2_len[0], log2_len[1] + 1)))
                  for _ in range(n_beams)]
        if max_samples is None or sum(r * l for r, l in shapes) <= max_samples:
            return shapes
        s += 1000003


def batch(device="cpu", shapes: Optional[List[Tuple[int, int]]] = None, n_beams: int = 48,
          seed: int = BASE_SEED + 3, pulses_per_beam: int = 20, wmax: int = 128,
          max_samples: Optional[int] = None) -> dict:
    """Batched workload: N(0,1) beams, 20 pulses each (widths 1..128, SNR 6-30),
    widths 1..wmax, threshold 7, sigma_N = sqrt(N)*sigma, per-row statistics."""
    if shapes is None:
        shapes = batch_shapes(n_beams, seed, max_samples)
    children = np.random.SeedSequence(seed).spawn(len(shapes))
    planes = []
    for (R, L), child in zip(shapes, children):
        sub = int(child.generate_state(1, dtype=np.uint32)[0])
        planes.append(make_plane(R, L, seed=sub, device=device, n_pulses=pulses_per_beam,
                                 pulse_widths=_widths_range(1, wmax), snr_range=(6.0, 30.0),
                                 gap=wmax, t_margin=wmax - 1))
    return dict(planes=planes, shapes=shapes, widths=_widths_range(1, wmax), threshold=7.0,
                sigma_mode="sqrtn", scope="row", kappa=1.0,
                name="batch-%dbeams" % len(shapes))


# ---------------------------------------------------------------------------
# Streaming chunks for the serving loop.
# ---------------------------------------------------------------------------

def stream_chunks(n_chunks: int, R: int, L_chunk: int, *, seed: int, device="cpu", wmax: int = 256,
                  snr_range=(6.0, 30.0), dtype=torch.float16) -> Tuple[List[torch.Tensor], List[Pulse]]:
    """Consecutive chunks of one beam's time series (N(0,1) noise), with at
    least one pulse per chunk boundary that starts before the boundary and ends
    after it.  Pulse times are global sample indices.  The series is generated
    in float32 and then stored in ``dtype``."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    g = torch.Generator(device=device)
    g.manual_seed(int(rng.integers(0, 2 ** 62)))
    pulses: List[Pulse] = []
    for k in range(1, n_chunks):
        w = int(rng.integers(2, wmax + 1))
        s = float(rng.uniform(*snr_range))
        boundary = k * L_chunk
        t0 = int(rng.integers(boundary - w + 1, boundary))
        pulses.append(Pulse(int(rng.integers(0, R)), t0, w, s, float(s / np.sqrt(w))))
    chunks = []
    for k in range(n_chunks):
        c = torch.randn((R, L_chunk), generator=g, device=device, dtype=torch.float32)
        lo, hi = k * L_chunk, (k + 1) * L_chunk
        for p in pulses:
            a, b = max(p.t0, lo), min(p.t0 + p.width, hi)
            if a < b:
                c[p.row, a - lo:b - lo] += p.amp
        chunks.append(c.to(dtype))
    return chunks, pulses


# ---------------------------------------------------------------------------
# SNR-like planes for the peak-finding step on its own.
# ---------------------------------------------------------------------------

def snr_plane(R: int, L: int, *, seed: int, n_bumps: int = 8, quantum: float = 0.25,
              n_plateaus: int = 2) -> np.ndarray:
    """A float32 [R][L] plane shaped like the SNR output of the boxcar step:
    N(0,1) background, plus ``n_bumps`` clouds that fall off over DM rows and
    starts from a peak of 6..30 (the cloud one bright pulse leaves), plus
    ``n_plateaus`` flat rectangles.  Values are rounded to multiples of
    ``quantum`` so that equal SNRs (ties) are common.  NumPy only."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    x = rng.standard_normal((R, L))
    rr = np.arange(R)[:, None]
    tt = np.arange(L)[None, :]
    for _ in range(n_bumps):
        r0, t0 = int(rng.integers(0, R)), int(rng.integers(0, L))
        peak = float(rng.uniform(6.0, 30.0))
        dr, dt = float(rng.uniform(0.5, 4.0)), float(rng.uniform(2.0, 200.0))
        x += peak * np.exp(-np.abs(rr - r0) / dr - np.abs(tt - t0) / dt)
    for _ in range(n_plateaus):
        r0, t0 = int(rng.integers(0, R)), int(rng.integers(0, L))
        h, w = int(rng.integers(1, 4)), int(rng.integers(1, 40))
        x[r0:r0 + h, t0:t0 + w] = float(rng.uniform(8.0, 12.0))
    if quantum > 0:
        x = np.round(x / quantum) * quantum
    return x.astype(np.float32)


# ---------------------------------------------------------------------------
# Filterbanks (frequency channels x time) for the de-dispersion step.
# ---------------------------------------------------------------------------

def filterbank(C: int, S: int, *, seed: int, device="cpu", mean: float = 96.0, sigma: float = 16.0,
               stride: Optional[int] = None) -> torch.Tensor:
    """uint8 [C][S] noise filterbank (rows padded to ``stride`` bytes, a
    multiple of 4, default the next one up from S): round(mean + sigma * z)
    clamped to 0..255, z ~ N(0, 1) drawn with torch on ``device`` from a seed
    taken from numpy's SeedSequence(seed).  Returns the [C][S] view."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    g = torch.Generator(device=device)
    g.manual_seed(int(rng.integers(0, 2 ** 62)))
    stride = stride or (S + 3) // 4 * 4
    buf = torch.empty((C, stride), dtype=torch.uint8, device=device)
    for c0 in range(0, C, 256):                      # bounded float scratch
        c1 = min(C, c0 + 256)
        z = torch.randn((c1 - c0, S), generator=g, device=device, dtype=torch.float32)
        buf[c0:c1, :S] = torch.clamp(torch.round(mean + sigma * z), 0, 255).to(torch.uint8)
        buf[c0:c1, S:] = 0
    return buf[:, :S]


def inject_along(fb: torch.Tensor, delays_row, t0: int, width: int, amp: int) -> None:
    """Add ``amp`` counts (saturating at 255) to fb[c][t0 + delays_row[c] + k]
    for k < width: a pulse that reaches channel c after the given delay (the
    caller supplies the delay curve)."""
    d = torch.as_tensor(np.asarray(delays_row, dtype=np.int64), device=fb.device)
    cols = t0 + d[:, None] + torch.arange(width, device=fb.device)[None, :]
    rows = torch.arange(fb.shape[0], device=fb.device)[:, None].expand_as(cols)
    v = fb[rows, cols].to(torch.int32) + int(amp)
    fb[rows, cols] = torch.clamp(v, 0, 255).to(torch.uint8)
