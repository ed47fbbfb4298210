"""ctypes binding of libspd (include/spd.h).

Argument marshalling only: every step of the detection path runs in the HIP
kernels of libspd.so.  Torch tensors provide device memory and the current
HIP stream.  If the library is missing, loading raises -- there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import threading
import time
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspd.so")

SPD_F32, SPD_F16, SPD_U8 = 0, 1, 2
SCOPES = {"row": 0, "plane": 1}
SIGMA_MODES = {"sqrtn": 0, "linear": 1, "auto": 2, "linear_literal": 3}
FLAG_ZERO_VAR, FLAG_LINEAR = 1, 2
SERVE_GAP = 1             # spd_server_result.flags: the chunk followed missing chunks
SERVE_RERUN = 2           # spd_server_result.flags: the chunk overflowed and was searched again
STATUS = {0: "SPD_OK", 1: "SPD_E_INVALID", 2: "SPD_E_UNSUPPORTED", 3: "SPD_E_NOMEM",
          4: "SPD_E_DEVICE", 5: "SPD_E_AGAIN"}

CANDIDATE_DTYPE = np.dtype([("row", "<i4"), ("width", "<i4"), ("t", "<i8"), ("snr", "<f4"),
                            ("beam", "<u4")])
STATS_FIELDS = 5          # mean, sigma, sigma_nmax, lin_coef, flags|reserved (as doubles)
STATE_FIELDS = 6          # n, T, S, n_y, T_y, S_y


class SpdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


class SpdPlane(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("row_stride", ctypes.c_int64),
                ("row_scale", ctypes.c_void_p), ("row_zero", ctypes.c_void_p)]


class SpdParams(ctypes.Structure):
    _fields_ = [("widths", ctypes.POINTER(ctypes.c_int32)), ("n_widths", ctypes.c_int32),
                ("threshold", ctypes.c_float), ("scope", ctypes.c_int32), ("sigma_mode", ctypes.c_int32),
                ("auto_kappa", ctypes.c_float), ("reserved0", ctypes.c_int32)]


class SpdBatchInfo(ctypes.Structure):
    _fields_ = [("out_per_lane", ctypes.c_int32), ("waves_per_group", ctypes.c_int32),
                ("groups_per_cu", ctypes.c_int32), ("tiles_per_grab", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("window", ctypes.c_int32), ("msd_items", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("rows", ctypes.c_int64)]


class SpdBand(ctypes.Structure):
    _fields_ = [("n_chan", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("f_top_mhz", ctypes.c_double),
                ("chan_bw_mhz", ctypes.c_double), ("t_samp_s", ctypes.c_double)]


class SpdServerConfig(ctypes.Structure):
    _fields_ = [("n_beams", ctypes.c_int32), ("dtype", ctypes.c_int32), ("n_rows", ctypes.c_int64),
                ("chunk_cols", ctypes.c_int64), ("cand_capacity", ctypes.c_int64),
                ("slots_per_beam", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_int64), ("deadline_s", ctypes.c_double),
                ("overflow_capacity", ctypes.c_int64)]


class SpdServerResult(ctypes.Structure):
    _fields_ = [("beam", ctypes.c_int32), ("status", ctypes.c_int32), ("seq", ctypes.c_int64),
                ("t_offset", ctypes.c_int64), ("n_cands", ctypes.c_int64), ("n_copied", ctypes.c_int64),
                ("submit_s", ctypes.c_double), ("start_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("flags", ctypes.c_int32), ("reserved0", ctypes.c_int32)]


_lock = threading.Lock()
_lib = None


def lib_path() -> str:
    return LIB_PATH


def load():
    """Load libspd.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError("libspd.so not found at %s; build it with "
                              "`python -m paper_1611_09704_amd.build`" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        P = ctypes.POINTER
        lib.spd_abi_version.restype = ctypes.c_int
        lib.spd_last_error.restype = ctypes.c_char_p
        lib.spd_workspace_bytes.argtypes = [P(SpdPlane), P(SpdParams)]
        lib.spd_workspace_bytes.restype = ctypes.c_size_t
        lib.msd_compute.argtypes = [P(SpdPlane), P(SpdParams), i64, i32, vp, vp, vp, ctypes.c_size_t, vp]
        lib.msd_compute.restype = ctypes.c_int
        lib.boxcar_snr.argtypes = [P(SpdPlane), P(SpdParams), vp, vp, vp, i64, i64, vp, i64, vp, vp]
        lib.boxcar_snr.restype = ctypes.c_int
        lib.select_candidates.argtypes = [vp, vp, i64, i64, i64, P(SpdParams), i64, vp, i64, vp, vp]
        lib.select_candidates.restype = ctypes.c_int
        lib.spd_detect.argtypes = [P(SpdPlane), P(SpdParams), vp, vp, vp, i64, i64, vp, i64, vp, vp,
                                   ctypes.c_size_t, i32, vp, vp]
        lib.spd_detect.restype = ctypes.c_int
        lib.spd_detect_static.argtypes = [P(SpdPlane), P(SpdParams), vp, vp, vp, i64, i64, vp, i64, vp, vp]
        lib.spd_detect_static.restype = ctypes.c_int
        lib.boxcar_snr_dit.argtypes = [P(SpdPlane), P(SpdParams), i32, vp, vp, vp, i64, i64, vp, i64, vp, vp]
        lib.cluster_candidates.argtypes = [vp, i64, i64, i64, i64, vp, i64, vp, i32, i32, vp, i64, vp, vp]
        lib.cluster_candidates.restype = ctypes.c_int
        lib.spd_dedisp_plan_create.argtypes = [P(SpdBand), P(ctypes.c_double), i32, P(vp)]
        lib.spd_dedisp_plan_create.restype = ctypes.c_int
        lib.spd_dedisp_plan_destroy.argtypes = [vp]
        lib.spd_dedisp_plan_destroy.restype = None
        lib.spd_dedisp_describe.argtypes = [vp, P(i32), P(i32)]
        lib.spd_dedisp_describe.restype = ctypes.c_int
        lib.spd_dedisp_delays.argtypes = [vp, P(i32)]
        lib.spd_dedisp_delays.restype = ctypes.c_int
        lib.spd_dedisp_delay_table.argtypes = [P(SpdBand), P(ctypes.c_double), i32, P(i32), P(i32)]
        lib.spd_dedisp_delay_table.restype = ctypes.c_int
        lib.spd_dedisperse.argtypes = [vp, P(SpdPlane), vp, i64, vp]
        lib.spd_dedisperse.restype = ctypes.c_int
        lib.boxcar_snr_dit.restype = ctypes.c_int
        lib.spd_batch_plan_create.argtypes = [P(SpdPlane), i32, P(SpdParams), i32, P(vp)]
        lib.spd_batch_plan_create.restype = ctypes.c_int
        lib.spd_batch_run.argtypes = [vp, vp, i64, vp, i32, vp]
        lib.spd_batch_run.restype = ctypes.c_int
        lib.spd_batch_copy_stats.argtypes = [vp, i32, vp, vp]
        lib.spd_batch_copy_stats.restype = ctypes.c_int
        lib.spd_batch_describe.argtypes = [vp, P(SpdBatchInfo)]
        lib.spd_batch_describe.restype = ctypes.c_int
        lib.spd_batch_tune_table.argtypes = [vp, P(SpdBatchInfo), P(ctypes.c_float), i32]
        lib.spd_batch_tune_table.restype = i32
        lib.spd_server_device_bytes.argtypes = [P(SpdServerConfig), P(SpdParams)]
        lib.spd_server_device_bytes.restype = ctypes.c_size_t
        lib.spd_server_create.argtypes = [P(SpdServerConfig), P(SpdParams), P(vp)]
        lib.spd_server_create_dedisp.argtypes = [P(SpdServerConfig), P(SpdParams), vp, P(vp)]
        lib.spd_server_create_dedisp.restype = ctypes.c_int
        lib.spd_server_create.restype = ctypes.c_int
        lib.spd_server_submit.argtypes = [vp, i32, i64, vp, ctypes.c_double]
        lib.spd_server_submit.restype = ctypes.c_int
        lib.spd_server_poll.argtypes = [vp, P(SpdServerResult), vp, i64, i32]
        lib.spd_server_poll.restype = ctypes.c_int
        lib.spd_server_counters.argtypes = [vp, P(i64), P(i64), P(i64)]
        lib.spd_server_counters.restype = ctypes.c_int
        lib.spd_server_destroy.argtypes = [vp]
        lib.spd_server_info.argtypes = [vp, P(i32), P(i32), P(i64)]
        lib.spd_server_info.restype = ctypes.c_int
        lib.spd_server_beam_state_bytes.argtypes = [vp]
        lib.spd_server_beam_state_bytes.restype = ctypes.c_size_t
        lib.spd_server_save_beam.argtypes = [vp, i32, vp, ctypes.c_size_t]
        lib.spd_server_save_beam.restype = ctypes.c_int
        lib.spd_server_load_beam.argtypes = [vp, i32, vp, ctypes.c_size_t]
        lib.spd_server_load_beam.restype = ctypes.c_int
        lib.spd_server_destroy.restype = None
        lib.spd_batch_plan_destroy.argtypes = [vp]
        lib.spd_batch_plan_destroy.restype = None
        _lib = lib
        return lib


def abi_version() -> int:
    return load().spd_abi_version()


def _check(status: int):
    if status != 0:
        raise SpdError(status, load().spd_last_error().decode())


class Params:
    """Width list, threshold and options of one detection (spd_params)."""

    def __init__(self, widths: Sequence[int], threshold: float, scope: str = "row",
                 sigma_mode: str = "sqrtn", kappa: float = 1.0):
        self.widths = [int(w) for w in widths]
        self._w = (ctypes.c_int32 * len(self.widths))(*self.widths)
        self.threshold = float(threshold)
        self.scope = scope
        self.sigma_mode = sigma_mode
        self.kappa = float(kappa)
        self.c = SpdParams(ctypes.cast(self._w, ctypes.POINTER(ctypes.c_int32)), len(self.widths),
                           self.threshold, SCOPES[scope], SIGMA_MODES[sigma_mode], self.kappa, 0)

    @property
    def nmax(self) -> int:
        return self.widths[-1]

    def n_units(self, n_rows: int) -> int:
        return 1 if self.scope == "plane" else n_rows


def _stream(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def plane_struct(x: torch.Tensor, scale: Optional[torch.Tensor] = None,
                 zero: Optional[torch.Tensor] = None) -> SpdPlane:
    """spd_plane view of a 2-D device tensor (rows = DM trials, time contiguous)."""
    if x.dim() != 2 or x.stride(1) != 1:
        raise ValueError("plane must be 2-D with a contiguous time axis")
    if not x.is_cuda:
        raise ValueError("plane must be a device tensor")
    if x.dtype == torch.float32:
        dt = SPD_F32
    elif x.dtype == torch.float16:
        dt = SPD_F16
    elif x.dtype == torch.uint8:
        dt = SPD_U8
        if scale is None or zero is None:
            raise ValueError("uint8 plane needs per-row scale and zero")
    else:
        raise ValueError("unsupported plane dtype %s" % x.dtype)
    return SpdPlane(x.data_ptr(), dt, 0, x.shape[0], x.shape[1], x.stride(0),
                    scale.data_ptr() if scale is not None else None,
                    zero.data_ptr() if zero is not None else None)


def workspace_bytes(x: torch.Tensor, params: Params, scale=None, zero=None) -> int:
    pl = plane_struct(x, scale, zero)
    n = load().spd_workspace_bytes(ctypes.byref(pl), ctypes.byref(params.c))
    if n == 0:
        _check(1)
    return n


def msd_compute(x: torch.Tensor, params: Params, *, scale=None, zero=None, new_col_begin: int = 0,
                accumulate: bool = False, state: Optional[torch.Tensor] = None,
                stats: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                stream=None) -> torch.Tensor:
    """Per-unit statistics (Sec. 2.1-2.2); returns stats as float64 [units, 5]."""
    lib = load()
    pl = plane_struct(x, scale, zero)
    units = params.n_units(x.shape[0])
    if stats is None:
        stats = torch.empty((units, STATS_FIELDS), dtype=torch.float64, device=x.device)
    need = lib.spd_workspace_bytes(ctypes.byref(pl), ctypes.byref(params.c))
    if need == 0:
        _check(1)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    _check(lib.msd_compute(ctypes.byref(pl), ctypes.byref(params.c), int(new_col_begin), int(bool(accumulate)),
                           state.data_ptr() if state is not None else None, stats.data_ptr(),
                           workspace.data_ptr(), workspace.numel() * workspace.element_size(), _stream(stream)))
    return stats


def boxcar_snr(x: torch.Tensor, params: Params, stats: torch.Tensor, *, scale=None, zero=None,
               snr: Optional[torch.Tensor] = None, widx: Optional[torch.Tensor] = None,
               out_stride: Optional[int] = None, t_offset: int = 0, cand: Optional[torch.Tensor] = None,
               cand_count: Optional[torch.Tensor] = None, stream=None) -> None:
    """Boxcar bank, SNR and per-sample max/argmax (Sec. 2.3), optional fused threshold."""
    lib = load()
    pl = plane_struct(x, scale, zero)
    if out_stride is None:
        out_stride = snr.stride(0) if snr is not None else (widx.stride(0) if widx is not None else 0)
    cap = cand.shape[0] if cand is not None else 0
    _check(lib.boxcar_snr(ctypes.byref(pl), ctypes.byref(params.c), stats.data_ptr(),
                          snr.data_ptr() if snr is not None else None,
                          widx.data_ptr() if widx is not None else None, int(out_stride), int(t_offset),
                          cand.data_ptr() if cand is not None else None, int(cap),
                          cand_count.data_ptr() if cand_count is not None else None, _stream(stream)))


DIT_BASE = 16


def dit_widths(levels: int) -> list:
    """Widths of the decimated search: 1..16, then 2^l*(9..16) for l = 1..levels."""
    w = list(range(1, DIT_BASE + 1))
    for lv in range(1, levels + 1):
        w += [k << lv for k in range(DIT_BASE // 2 + 1, DIT_BASE + 1)]
    return w


def dit_params(levels: int, threshold: float, scope: str = "row", sigma_mode: str = "sqrtn",
               kappa: float = 1.0) -> Params:
    return Params(dit_widths(levels), threshold, scope, sigma_mode, kappa)


def boxcar_snr_dit(x: torch.Tensor, params: Params, levels: int, stats: torch.Tensor, *, scale=None, zero=None,
                   snr: Optional[torch.Tensor] = None, widx: Optional[torch.Tensor] = None,
                   out_stride: Optional[int] = None, t_offset: int = 0, cand: Optional[torch.Tensor] = None,
                   cand_count: Optional[torch.Tensor] = None, stream=None) -> None:
    """Boxcars combined with decimation in time (widths from dit_widths)."""
    lib = load()
    pl = plane_struct(x, scale, zero)
    if out_stride is None:
        out_stride = snr.stride(0) if snr is not None else (widx.stride(0) if widx is not None else 0)
    cap = cand.shape[0] if cand is not None else 0
    _check(lib.boxcar_snr_dit(ctypes.byref(pl), ctypes.byref(params.c), int(levels), stats.data_ptr(),
                              snr.data_ptr() if snr is not None else None,
                              widx.data_ptr() if widx is not None else None, int(out_stride), int(t_offset),
                              cand.data_ptr() if cand is not None else None, int(cap),
                              cand_count.data_ptr() if cand_count is not None else None, _stream(stream)))


def select_candidates(snr: torch.Tensor, widx: torch.Tensor, params: Params, *, n_out_cols: Optional[int] = None,
                      t_offset: int = 0, cand: torch.Tensor, cand_count: torch.Tensor, stream=None) -> None:
    """Threshold of Sec. 2.4 over stored snr / width-index arrays."""
    lib = load()
    if snr.dtype != torch.float32 or widx.dtype != torch.uint8 or snr.dim() != 2 or widx.shape != snr.shape:
        raise ValueError("snr (float32) and widx (uint8) must be 2-D arrays of one shape")
    if snr.stride(1) != 1 or widx.stride(1) != 1 or widx.stride(0) != snr.stride(0):
        raise ValueError("snr and widx must share one row stride with unit column stride")
    n_rows = snr.shape[0]
    ncols = snr.shape[1] if n_out_cols is None else int(n_out_cols)
    _check(lib.select_candidates(snr.data_ptr(), widx.data_ptr(), n_rows, ncols, snr.stride(0),
                                 ctypes.byref(params.c), int(t_offset), cand.data_ptr(), cand.shape[0],
                                 cand_count.data_ptr(), _stream(stream)))


def cluster_candidates(snr: torch.Tensor, cand: torch.Tensor, cand_count: torch.Tensor, dm_radius: int,
                       t_radius: int, *, n_out_cols: Optional[int] = None, t_offset: int = 0,
                       peaks: Optional[torch.Tensor] = None, peak_count: Optional[torch.Tensor] = None,
                       stream=None):
    """Peak-finding over a candidate list in (DM row, time) against the snr
    plane it came from: keeps the candidates with no higher SNR within the
    radii (ties go to the first sample in row-major order).  Returns
    (peaks, peak_count); the count is a device int64 and may exceed the
    peak list's capacity (by default that of the candidate list)."""
    lib = load()
    if snr.dtype != torch.float32 or snr.dim() != 2 or snr.stride(1) != 1:
        raise ValueError("snr must be a float32 [rows][stride] view with unit column stride")
    ncols = snr.shape[1] if n_out_cols is None else int(n_out_cols)
    if peaks is None:
        peaks = new_candidates(max(1, cand.shape[0]), snr.device)
    if peak_count is None:
        peak_count = torch.zeros(1, dtype=torch.int64, device=snr.device)
    _check(lib.cluster_candidates(snr.data_ptr(), snr.shape[0], ncols, snr.stride(0), int(t_offset),
                                  cand.data_ptr(), cand.shape[0], cand_count.data_ptr(), int(dm_radius),
                                  int(t_radius), peaks.data_ptr(), peaks.shape[0], peak_count.data_ptr(),
                                  _stream(stream)))
    return peaks, peak_count


_aux_streams = {}


def aux_stream_for(device) -> torch.cuda.Stream:
    """A side stream per device (default priority) for spd_detect's statistics pass."""
    idx = torch.device(device).index
    idx = torch.cuda.current_device() if idx is None else idx
    st = _aux_streams.get(idx)
    if st is None:
        st = _aux_streams[idx] = torch.cuda.Stream(device=idx)
    return st


def spd_detect(x: torch.Tensor, params: Params, *, scale=None, zero=None, stats: Optional[torch.Tensor] = None,
               snr: Optional[torch.Tensor] = None, widx: Optional[torch.Tensor] = None,
               out_stride: Optional[int] = None, t_offset: int = 0, cand: Optional[torch.Tensor] = None,
               cand_count: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
               row_chunks: int = 1, stream=None, aux_stream=None) -> torch.Tensor:
    """The whole path in one call (statistics, boxcars, fused threshold).
    With ``row_chunks`` > 1 and an ``aux_stream`` ("auto": a cached side
    stream of the plane's device) the statistics of later row chunks run
    beside the boxcars of earlier ones; by default both steps run on
    ``stream``.  Returns stats."""
    lib = load()
    pl = plane_struct(x, scale, zero)
    units = params.n_units(x.shape[0])
    if stats is None:
        stats = torch.empty((units, STATS_FIELDS), dtype=torch.float64, device=x.device)
    if workspace is None:
        need = lib.spd_workspace_bytes(ctypes.byref(pl), ctypes.byref(params.c))
        if need == 0:
            _check(1)
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    if out_stride is None:
        out_stride = snr.stride(0) if snr is not None else (widx.stride(0) if widx is not None else 0)
    if isinstance(aux_stream, str):
        aux_stream = aux_stream_for(x.device)
    aux = _stream(aux_stream) if aux_stream is not None else None
    cap = cand.shape[0] if cand is not None else 0
    _check(lib.spd_detect(ctypes.byref(pl), ctypes.byref(params.c), stats.data_ptr(),
                          snr.data_ptr() if snr is not None else None,
                          widx.data_ptr() if widx is not None else None, int(out_stride), int(t_offset),
                          cand.data_ptr() if cand is not None else None, int(cap),
                          cand_count.data_ptr() if cand_count is not None else None,
                          workspace.data_ptr(), workspace.numel() * workspace.element_size(), int(row_chunks),
                          _stream(stream), aux))
    return stats


def spd_detect_static(x: torch.Tensor, params: Params, *, scale=None, zero=None,
                      stats: Optional[torch.Tensor] = None, snr: Optional[torch.Tensor] = None,
                      widx: Optional[torch.Tensor] = None, out_stride: Optional[int] = None, t_offset: int = 0,
                      cand: Optional[torch.Tensor] = None, cand_count: Optional[torch.Tensor] = None,
                      stream=None) -> torch.Tensor:
    """spd_detect with the statistics pass's partials in the library's fixed
    device array: the call itself allocates nothing (pass ``stats`` to keep
    the wrapper from allocating it).  Calls that overlap on one device race.
    Returns stats."""
    lib = load()
    pl = plane_struct(x, scale, zero)
    if stats is None:
        stats = torch.empty((params.n_units(x.shape[0]), STATS_FIELDS), dtype=torch.float64, device=x.device)
    if out_stride is None:
        out_stride = snr.stride(0) if snr is not None else (widx.stride(0) if widx is not None else 0)
    cap = cand.shape[0] if cand is not None else 0
    _check(lib.spd_detect_static(ctypes.byref(pl), ctypes.byref(params.c), stats.data_ptr(),
                                 snr.data_ptr() if snr is not None else None,
                                 widx.data_ptr() if widx is not None else None, int(out_stride), int(t_offset),
                                 cand.data_ptr() if cand is not None else None, int(cap),
                                 cand_count.data_ptr() if cand_count is not None else None, _stream(stream)))
    return stats


def new_candidates(capacity: int, device) -> torch.Tensor:
    return torch.empty((max(1, int(capacity)), CANDIDATE_DTYPE.itemsize), dtype=torch.uint8, device=device)


def candidates_to_numpy(cand: torch.Tensor, count: int) -> np.ndarray:
    n = min(int(count), cand.shape[0])
    raw = cand[:n].cpu().numpy().tobytes()
    return np.frombuffer(raw, dtype=CANDIDATE_DTYPE).copy()


def stats_flags(stats: torch.Tensor) -> torch.Tensor:
    """The uint32 flags word of each spd_row_stats row."""
    return stats.view(torch.int32)[:, 8]


def detect(x: torch.Tensor, widths: Sequence[int], threshold: float, *, scope: str = "row",
           sigma_mode: str = "sqrtn", kappa: float = 1.0, scale=None, zero=None, outputs: bool = True,
           fused_select: bool = True, capacity: int = 1 << 16, stream=None) -> dict:
    """The whole path on one plane: msd_compute, boxcar_snr (+ fused threshold),
    or boxcar_snr then select_candidates.  Grows the candidate list and re-runs
    if it overflows.  Synchronises the stream before returning."""
    params = Params(widths, threshold, scope, sigma_mode, kappa)
    stats = msd_compute(x, params, scale=scale, zero=zero, stream=stream)
    nout = x.shape[1] - params.nmax + 1
    snr = torch.empty((x.shape[0], nout), dtype=torch.float32, device=x.device) if outputs else None
    widx = torch.empty((x.shape[0], nout), dtype=torch.uint8, device=x.device) if outputs else None
    count = torch.zeros(1, dtype=torch.int64, device=x.device)
    while True:
        cand = new_candidates(capacity, x.device)
        if fused_select or not outputs:
            boxcar_snr(x, params, stats, scale=scale, zero=zero, snr=snr, widx=widx, cand=cand,
                       cand_count=count, stream=stream)
        else:
            boxcar_snr(x, params, stats, scale=scale, zero=zero, snr=snr, widx=widx, stream=stream)
            select_candidates(snr, widx, params, cand=cand, cand_count=count, stream=stream)
        n = int(count.item())
        if n <= cand.shape[0]:
            break
        capacity = n
    return {"params": params, "stats": stats, "snr": snr, "widx": widx,
            "cands": candidates_to_numpy(cand, n), "n_cands": n}


def dedisp_delay_table(n_chan: int, f_top_mhz: float, chan_bw_mhz: float, t_samp_s: float, dm):
    """The library's delay table (host only) and largest delay."""
    lib = load()
    band = SpdBand(int(n_chan), 0, float(f_top_mhz), float(chan_bw_mhz), float(t_samp_s))
    dm = np.ascontiguousarray(np.asarray(dm, dtype=np.float64))
    out = np.empty((dm.size, int(n_chan)), dtype=np.int32)
    md = ctypes.c_int32()
    _check(lib.spd_dedisp_delay_table(ctypes.byref(band), dm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      int(dm.size), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      ctypes.byref(md)))
    return out, int(md.value)


class DedispPlan:
    """Brute-force de-dispersion plan (spd_dedisp_*): one band (n_chan
    channels from f_top_mhz down in steps of chan_bw_mhz, sampling t_samp_s)
    and one non-decreasing list of trial DMs."""

    def __init__(self, n_chan: int, f_top_mhz: float, chan_bw_mhz: float, t_samp_s: float, dm):
        lib = load()
        self._lib = lib
        self.band = SpdBand(int(n_chan), 0, float(f_top_mhz), float(chan_bw_mhz), float(t_samp_s))
        self.dm = np.ascontiguousarray(np.asarray(dm, dtype=np.float64))
        self._h = ctypes.c_void_p()
        _check(lib.spd_dedisp_plan_create(ctypes.byref(self.band),
                                          self.dm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          int(self.dm.size), ctypes.byref(self._h)))
        md, sp = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.spd_dedisp_describe(self._h, ctypes.byref(md), ctypes.byref(sp)))
        self.max_delay, self.span16 = int(md.value), int(sp.value)

    @property
    def n_dm(self) -> int:
        return int(self.dm.size)

    def delays(self) -> np.ndarray:
        out = np.empty((self.n_dm, self.band.n_chan), dtype=np.int32)
        _check(self._lib.spd_dedisp_delays(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out

    def run(self, fb: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """De-disperse fb (uint8 [n_chan][n_samp] device tensor, rows 4-byte
        aligned) into out (float32 [n_dm][>= n_samp - max_delay]); returns out
        narrowed to the valid columns."""
        if fb.dtype != torch.uint8 or fb.dim() != 2 or fb.stride(1) != 1 or not fb.is_cuda:
            raise ValueError("fb must be a uint8 device tensor [n_chan][n_samp] with a contiguous time axis")
        n_out = fb.shape[1] - self.max_delay
        if out is None:
            out = torch.empty((self.n_dm, max(n_out, 1)), dtype=torch.float32, device=fb.device)
        if out.dtype != torch.float32 or out.dim() != 2 or out.stride(1) != 1:
            raise ValueError("out must be a float32 [n_dm][>= n_out] view with unit column stride")
        pl = SpdPlane(fb.data_ptr(), SPD_U8, 0, fb.shape[0], fb.shape[1], fb.stride(0), None, None)
        _check(self._lib.spd_dedisperse(self._h, ctypes.byref(pl), out.data_ptr(), out.stride(0), _stream(stream)))
        return out[:, :n_out]

    def close(self):
        if self._h:
            self._lib.spd_dedisp_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """Batched form (spd_batch_*): many beams of uneven shape, one persistent
    launch per pass, optional hipGraph replay.  ``beams`` is a list of 2-D
    device tensors of one dtype (or (tensor, scale, zero) tuples for uint8);
    they must stay alive while the plan exists."""

    def __init__(self, beams, params: Params, autotune: bool = True):
        lib = load()
        self.params = params
        self._beams = [b if isinstance(b, tuple) else (b, None, None) for b in beams]
        arr = (SpdPlane * len(self._beams))(*[plane_struct(x, s, z) for x, s, z in self._beams])
        h = ctypes.c_void_p()
        _check(lib.spd_batch_plan_create(arr, len(self._beams), ctypes.byref(params.c), int(bool(autotune)),
                                         ctypes.byref(h)))
        self._h = h

    def run(self, cand: torch.Tensor, cand_count: torch.Tensor, use_graph: bool = False, stream=None) -> None:
        _check(load().spd_batch_run(self._h, cand.data_ptr(), cand.shape[0], cand_count.data_ptr(),
                                    int(bool(use_graph)), _stream(stream)))

    def stats(self, beam: int, stream=None) -> torch.Tensor:
        x = self._beams[beam][0]
        out = torch.empty((x.shape[0], STATS_FIELDS), dtype=torch.float64, device=x.device)
        _check(load().spd_batch_copy_stats(self._h, int(beam), out.data_ptr(), _stream(stream)))
        return out

    def describe(self) -> dict:
        info = SpdBatchInfo()
        _check(load().spd_batch_describe(self._h, ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in SpdBatchInfo._fields_}

    def tune_table(self) -> list:
        rows = (SpdBatchInfo * 64)()
        ns = (ctypes.c_float * 64)()
        n = load().spd_batch_tune_table(self._h, rows, ns, 64)
        return [{"out_per_lane": rows[i].out_per_lane, "waves_per_group": rows[i].waves_per_group,
                 "groups_per_cu": rows[i].groups_per_cu, "tiles_per_grab": rows[i].tiles_per_grab,
                 "window": rows[i].window,
                 "ns_per_start": round(float(ns[i]), 5)} for i in range(min(n, 64))]

    def close(self):
        if getattr(self, "_h", None):
            load().spd_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def steady_now() -> float:
    """The steady clock the server stamps results with (seconds)."""
    return time.monotonic()


def server_device_bytes(n_beams: int, n_rows: int, chunk_cols: int, params: Params, dtype=torch.float16,
                        cand_capacity: int = 1 << 16, slots_per_beam: int = 2, hbm_budget_bytes: int = 0) -> int:
    """Device bytes a server (no de-dispersion) of this configuration would
    allocate; 0 when the budget cannot hold the beams' state and one buffer."""
    dt = {torch.float32: SPD_F32, torch.float16: SPD_F16}[dtype]
    cfg = SpdServerConfig(n_beams, dt, n_rows, chunk_cols, cand_capacity, slots_per_beam, 0, hbm_budget_bytes)
    return load().spd_server_device_bytes(ctypes.byref(cfg), ctypes.byref(params.c))


class Server:
    """Serving form (spd_server_*): chunk streams from several beams with
    carried halo and running statistics; results are polled as they finish."""

    def __init__(self, n_beams: int, n_rows: int, chunk_cols: int, params: Params, dtype=torch.float16,
                 cand_capacity: int = 1 << 16, slots_per_beam: int = 2, hbm_budget_bytes: int = 0,
                 dedisp: Optional["DedispPlan"] = None, n_streams: int = 0, deadline_s: float = 0.0,
                 overflow_capacity: int = 0):
        """With ``dedisp`` (a DedispPlan, kept alive by the server) the beams
        stream uint8 filterbank chunks [n_chan][chunk_cols], de-dispersed on
        the device in front of the detection stream.  ``hbm_budget_bytes``
        sizes the shared pool of chunk buffers; ``n_streams`` compute streams
        (0: 2) each with a copy stream carry the work; a chunk still on the
        device ``deadline_s`` after admission (0: no deadline) stops the server;
        with ``overflow_capacity`` (> cand_capacity) a chunk past cand_capacity
        is searched again and all its candidates (up to that many) delivered."""
        lib = load()
        if dedisp is not None:
            dtype = torch.uint8
        dt = {torch.float32: SPD_F32, torch.float16: SPD_F16, torch.uint8: SPD_U8}[dtype]
        self.params = params
        self.dedisp = dedisp
        self.dtype = dtype
        self.shape = (int(n_rows), int(chunk_cols))
        self.cfg = SpdServerConfig(n_beams, dt, n_rows, chunk_cols, cand_capacity, slots_per_beam, n_streams,
                                   hbm_budget_bytes, float(deadline_s), int(overflow_capacity))
        self.cap = max(int(cand_capacity), int(overflow_capacity))
        self._buf = np.empty(self.cap, dtype=CANDIDATE_DTYPE)
        self._keep = {}
        h = ctypes.c_void_p()
        if dedisp is None:
            _check(lib.spd_server_create(ctypes.byref(self.cfg), ctypes.byref(params.c), ctypes.byref(h)))
        else:
            _check(lib.spd_server_create_dedisp(ctypes.byref(self.cfg), ctypes.byref(params.c), dedisp._h,
                                                ctypes.byref(h)))
        self._h = h

    def device_bytes(self) -> int:
        return load().spd_server_device_bytes(ctypes.byref(self.cfg), ctypes.byref(self.params.c))

    def submit(self, beam: int, seq: int, chunk: torch.Tensor, arrival_s: float = 0.0) -> None:
        """chunk: a host tensor [n_rows, chunk_cols] of the server's dtype, kept
        alive until its result is polled.  The C call takes a bare pointer, so a
        malformed chunk is refused here, before anything is enqueued."""
        if chunk.is_cuda or not chunk.is_contiguous():
            raise ValueError("chunk must be a contiguous host tensor (pinned for speed)")
        if tuple(chunk.shape) != self.shape or chunk.dtype != self.dtype:
            raise ValueError("chunk must be %s %s, got %s %s" % (self.dtype, list(self.shape), chunk.dtype,
                                                                 list(chunk.shape)))
        _check(load().spd_server_submit(self._h, int(beam), int(seq), chunk.data_ptr(), float(arrival_s)))
        self._keep[(beam, seq)] = chunk      # until polled (a refused submit keeps nothing)

    def poll(self, wait_ms: int = 0):
        """(result dict, candidates array) of one finished chunk, or None."""
        res = SpdServerResult()
        st = load().spd_server_poll(self._h, ctypes.byref(res), self._buf.ctypes.data_as(ctypes.c_void_p),
                                    self.cap, int(wait_ms))
        if st == 5:
            return None
        _check(st)
        self._keep.pop((res.beam, res.seq), None)
        out = {f: getattr(res, f) for f, _ in SpdServerResult._fields_}
        return out, self._buf[:res.n_copied].copy()

    def info(self) -> dict:
        n, q, m = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(load().spd_server_info(self._h, ctypes.byref(n), ctypes.byref(q), ctypes.byref(m)))
        return {"pool_buffers": n.value, "n_streams": q.value, "device_bytes": m.value}

    def counters(self) -> dict:
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(load().spd_server_counters(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"submitted": a.value, "admitted": b.value, "completed": c.value}

    def save_beam(self, beam: int) -> bytes:
        """Checkpoint of one idle beam (spd_server_save_beam)."""
        n = load().spd_server_beam_state_bytes(self._h)
        buf = ctypes.create_string_buffer(n)
        _check(load().spd_server_save_beam(self._h, int(beam), buf, n))
        return buf.raw

    def load_beam(self, beam: int, state: bytes) -> None:
        """Restore one idle beam from save_beam's bytes (spd_server_load_beam)."""
        buf = ctypes.create_string_buffer(state, len(state))
        _check(load().spd_server_load_beam(self._h, int(beam), buf, len(state)))

    def close(self):
        if getattr(self, "_h", None):
            load().spd_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
