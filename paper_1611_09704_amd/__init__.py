"""MI355X-native single-pulse detection (Adamek & Armour, arXiv:1611.09704).

The detection path -- mean/standard deviation, boxcar matched filters with
SNR, and the candidate threshold -- runs in hand-written HIP kernels for gfx950
behind the C ABI declared in ``include/spd.h`` (``libspd.so``).  This package
is the thin Python binding over that library (``msd_compute``, ``boxcar_snr``,
``select_candidates`` and the batched / serving forms) plus the seeded input
generators in ``synth``.  The binding is loaded lazily so that the generators
can be imported on a machine without the library.
"""
from __future__ import annotations

__all__ = ["msd_compute", "boxcar_snr", "select_candidates", "detect", "lib_path"]


def __getattr__(name):
    if name in ("msd_compute", "boxcar_snr", "select_candidates", "detect", "lib_path",
                "workspace_bytes", "Params", "BatchPlan", "Server", "abi_version", "load"):
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
