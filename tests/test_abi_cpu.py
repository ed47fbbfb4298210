"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/spd.h, and rejects bad arguments before touching a GPU
(validation happens before any HIP call, so these run without one)."""
import ctypes
import os
import re

import pytest

from paper_1611_09704_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_1611_09704_amd import build
        build.build()
    return B.load()


def declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M):
            line = src[m.start():src.find("\n", m.start())]
            if line.startswith("typedef") or line.startswith("#"):
                continue
            names.append(m.group(1))
    return sorted(set(names))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert {"msd_compute", "boxcar_snr", "select_candidates", "spd_last_error",
            "spd_abi_version", "spd_workspace_bytes"} <= set(names)
    for n in names:
        assert hasattr(lib, n), "libspd.so does not export %s" % n
    assert lib.spd_abi_version() == 1


FAKE = 0x10000  # never dereferenced: validation rejects first


def _plane(dtype=B.SPD_F32, rows=4, cols=1000, stride=1000, data=FAKE, scale=None, zero=None):
    return B.SpdPlane(data, dtype, 0, rows, cols, stride, scale, zero)


def _err(lib):
    return lib.spd_last_error().decode()


@pytest.mark.parametrize("widths,msg", [([], "n_widths"), ([0, 1], "widths[0]"), ([1, 3, 3], "strictly"),
                                        ([1, 5000], "largest width"), (list(range(1, 258)), "n_widths")])
def test_params_validation(lib, widths, msg):
    p = B.Params(widths or [1], 5.0)
    if not widths:
        p.c.n_widths = 0
    pl = _plane()
    rc = lib.msd_compute(ctypes.byref(pl), ctypes.byref(p.c), 0, 0, None, FAKE, FAKE, 1 << 20, None)
    assert rc == 1 and msg in _err(lib)


def test_plane_validation(lib):
    p = B.Params([1, 2, 4, 8], 5.0)
    cases = [
        (_plane(rows=0), "n_rows"),
        (_plane(cols=1000, stride=999), "row_stride"),
        (_plane(cols=7, stride=7), "shorter"),
        (_plane(dtype=7), "dtype"),
        (_plane(data=0), "data"),
        (_plane(dtype=B.SPD_F32, data=FAKE + 2), "aligned"),
        (_plane(dtype=B.SPD_U8), "row_scale"),
    ]
    for pl, msg in cases:
        rc = lib.boxcar_snr(ctypes.byref(pl), ctypes.byref(p.c), FAKE, FAKE, FAKE, 1000, 0, None, 0, None, None)
        assert rc == 1, msg
        assert msg in _err(lib)


def test_call_validation(lib):
    p = B.Params([1, 2, 4, 8], 5.0)
    pl = _plane()
    assert lib.boxcar_snr(ctypes.byref(pl), ctypes.byref(p.c), FAKE, None, None, 0, 0, None, 0, None, None) == 1
    assert "no output" in _err(lib)
    assert lib.boxcar_snr(ctypes.byref(pl), ctypes.byref(p.c), FAKE, FAKE, None, 10, 0, None, 0, None, None) == 1
    assert "out_stride" in _err(lib)
    assert lib.boxcar_snr(ctypes.byref(pl), ctypes.byref(p.c), None, FAKE, None, 1000, 0, None, 0, None, None) == 1
    assert lib.boxcar_snr(ctypes.byref(pl), ctypes.byref(p.c), FAKE, None, None, 0, 0, FAKE, 10, None, None) == 1
    assert "cand_count" in _err(lib)
    ws = lib.spd_workspace_bytes(ctypes.byref(pl), ctypes.byref(p.c))
    assert ws > 0 and ws % 48 == 0
    assert lib.msd_compute(ctypes.byref(pl), ctypes.byref(p.c), 0, 0, None, FAKE, FAKE, ws - 1, None) == 3
    assert lib.msd_compute(ctypes.byref(pl), ctypes.byref(p.c), 0, 1, None, FAKE, FAKE, ws, None) == 1
    assert "accumulate" in _err(lib)
    assert lib.msd_compute(ctypes.byref(pl), ctypes.byref(p.c), 1001, 0, None, FAKE, FAKE, ws, None) == 1
    assert lib.msd_compute(ctypes.byref(pl), ctypes.byref(p.c), 0, 0, None, FAKE, FAKE + 8, ws, None) == 1
    assert lib.select_candidates(FAKE, FAKE, 4, 100, 50, ctypes.byref(p.c), 0, FAKE, 10, FAKE, None) == 1
    bad = B.Params([1, 2], float("nan"))
    assert lib.select_candidates(FAKE, FAKE, 4, 100, 100, ctypes.byref(bad.c), 0, FAKE, 10, FAKE, None) == 1
    assert "threshold" in _err(lib)


def test_detect_validation(lib):
    p = B.Params([1, 2, 4, 8], 5.0)
    pl = _plane()
    ws = lib.spd_workspace_bytes(ctypes.byref(pl), ctypes.byref(p.c))

    def call(stats=FAKE, snr=FAKE, stride=1000, cand=None, cap=0, count=None, work=FAKE * 16, nbytes=ws, chunks=4,
             stream=FAKE, aux=FAKE + 64, params=p, plane=pl):
        return lib.spd_detect(ctypes.byref(plane), ctypes.byref(params.c), stats, snr, None, stride, 0, cand, cap,
                              count, work, nbytes, chunks, stream, aux)

    for kw, code, msg in [(dict(stats=None), 1, "stats"), (dict(chunks=0), 1, "row_chunks"),
                          (dict(aux=FAKE), 1, "aux_stream"), (dict(nbytes=ws - 1), 3, "workspace"),
                          (dict(work=FAKE + 8), 1, "aligned"), (dict(work=None), 1, "workspace"),
                          (dict(snr=None), 1, "no output"), (dict(stride=10), 1, "out_stride"),
                          (dict(snr=None, cand=FAKE, cap=5), 1, "cand_count"),
                          (dict(plane=_plane(cols=1000, stride=999)), 1, "row_stride"),
                          (dict(params=B.Params([1, 3, 2], 5.0)), 1, "strictly")]:
        assert call(**kw) == code, kw
        assert msg in _err(lib), (kw, _err(lib))


def test_detect_static_validation(lib):
    """The allocation-free spd_detect rejects, before any HIP call, what
    spd_detect rejects, and planes whose block partials exceed its 4 MiB
    device array (87,381 partials of 48 bytes)."""
    p = B.Params([1, 2, 4, 8], 5.0)
    pl = _plane()

    def call(stats=FAKE, snr=FAKE, stride=1000, cand=None, cap=0, count=None, params=p, plane=pl):
        return lib.spd_detect_static(ctypes.byref(plane), ctypes.byref(params.c), stats, snr, None, stride, 0,
                                     cand, cap, count, FAKE)

    for kw, code, msg in [(dict(stats=None), 1, "stats"), (dict(snr=None), 1, "no output"),
                          (dict(stride=10), 1, "out_stride"), (dict(snr=None, cand=FAKE, cap=5), 1, "cand_count"),
                          (dict(plane=_plane(cols=1000, stride=999)), 1, "row_stride"),
                          (dict(params=B.Params([1, 3, 2], 5.0)), 1, "strictly")]:
        assert call(**kw) == code, kw
        assert msg in _err(lib), (kw, _err(lib))
    # 8,192 rows x 2^20 columns: 16 blocks of 65,536 per row, 131,072 partials = 6 MiB
    big = _plane(rows=8192, cols=1 << 20, stride=1 << 20)
    assert lib.spd_workspace_bytes(ctypes.byref(big), ctypes.byref(p.c)) == 8192 * 16 * 48
    assert call(plane=big, stride=1 << 20) == 2
    assert "static scratch" in _err(lib)
    # 4,096 rows x 2^20 (65,536 partials, 3 MiB) passes the size check; with
    # stats missing it still stops on the host
    ok = _plane(rows=4096, cols=1 << 20, stride=1 << 20)
    assert call(plane=ok, stride=1 << 20, stats=None) == 1 and "stats" in _err(lib)


def test_dit_validation(lib):
    import oracle
    for lv in range(5):
        assert B.dit_widths(lv) == oracle.dit_widths(lv)[0]
    pl = _plane(cols=3000, stride=3000)
    p = B.dit_params(2, 6.0)

    def call(params=p, levels=2, stats=FAKE, snr=FAKE, stride=3000):
        return lib.boxcar_snr_dit(ctypes.byref(pl), ctypes.byref(params.c), levels, stats, snr, None, stride, 0,
                                  None, 0, None, None)

    for kw, msg in [(dict(levels=5), "levels"), (dict(levels=-1), "levels"), (dict(levels=3), "widths must"),
                    (dict(params=B.Params(list(range(1, 17)) + [18], 6.0)), "widths must"),
                    (dict(stats=None), "stats"), (dict(snr=None), "no output"), (dict(stride=10), "out_stride")]:
        assert call(**kw) == 1, kw
        assert msg in _err(lib), (kw, _err(lib))


def test_cluster_validation(lib):
    C = B.CANDIDATE_DTYPE.itemsize

    def call(snr=FAKE, rows=4, cols=100, stride=100, cand=FAKE, cap=10, count=FAKE, dr=1, dt=8,
             peaks=FAKE + 4096, pcap=10, pcount=FAKE):
        return lib.cluster_candidates(snr, rows, cols, stride, 0, cand, cap, count, dr, dt, peaks, pcap, pcount, None)

    for kw, msg in [(dict(snr=None), "required"), (dict(count=None), "required"), (dict(peaks=None), "required"),
                    (dict(pcount=None), "required"), (dict(rows=-1), "shape"), (dict(stride=99), "shape"),
                    (dict(cap=-1), "capacities"), (dict(pcap=-2), "capacities"), (dict(dr=-1), "radii"),
                    (dict(dt=(1 << 20) + 1), "radii"), (dict(dr=4097), "radii"),
                    (dict(peaks=FAKE + 9 * C), "overlap"), (dict(peaks=FAKE - 10 * C + 1), "overlap")]:
        assert call(**kw) == 1, kw
        assert msg in _err(lib), (kw, _err(lib))


def test_dedisp_delay_table_and_validation(lib):
    import numpy as np
    import oracle
    for C, band, dm in [(256, (1550.0, 300 / 256, 64e-6), np.arange(40) * 0.5),
                        (4096, (1550.0, 300 / 4096, 64e-6), np.arange(6000) * 0.0689),
                        (7, (400.0, 10.0, 1e-3), [0, 1.5, 1.5, 800.25])]:
        table, md = B.dedisp_delay_table(C, *band, dm)
        want = oracle.dedisp_delays(dm, oracle.dedisp_channel_factors(C, *band))
        assert np.array_equal(table, want) and md == want.max()
    for args, msg in [((0, 1500.0, 1.0, 1e-4, [0.0]), "n_chan"), ((8, -1.0, 1.0, 1e-4, [0.0]), "finite"),
                      ((8, 1500.0, 0.0, 1e-4, [0.0]), "finite"), ((8, 1500.0, 1.0, 0.0, [0.0]), "finite"),
                      ((8, 10.0, 2.0, 1e-4, [0.0]), "lowest channel"), ((8, 1500.0, 1.0, 1e-4, []), "n_dm"),
                      ((8, 1500.0, 1.0, 1e-4, [1.0, 0.5]), "non-decreasing"),
                      ((8, 1500.0, 1.0, 1e-4, [-1.0]), ">= 0"), ((8, 1500.0, 1.0, 1e-4, [float("nan")]), "finite"),
                      ((8, 1500.0, 100.0, 1e-9, [1e9]), "exceeds")]:
        with pytest.raises(B.SpdError) as e:
            B.dedisp_delay_table(*args)
        assert msg in str(e.value), (args, str(e.value))
    assert lib.spd_dedisperse(None, None, None, 0, None) == 1 and "required" in _err(lib)


def test_batch_validation(lib):
    p = B.Params([1, 2, 4, 8], 5.0)
    out = ctypes.c_void_p(123)
    arr = (B.SpdPlane * 2)(_plane(), _plane(dtype=B.SPD_F16))
    assert lib.spd_batch_plan_create(arr, 0, ctypes.byref(p.c), 0, ctypes.byref(out)) == 1
    assert out.value is None and "n_beams" in _err(lib)
    assert lib.spd_batch_plan_create(arr, 2, ctypes.byref(p.c), 0, ctypes.byref(out)) == 1
    assert "dtype differs" in _err(lib)
    bad = (B.SpdPlane * 1)(_plane(cols=5, stride=5))
    assert lib.spd_batch_plan_create(bad, 1, ctypes.byref(p.c), 0, ctypes.byref(out)) == 1
    assert "beam 0" in _err(lib)
    pp = B.Params([1, 2], 5.0, scope="plane")
    assert lib.spd_batch_plan_create(arr, 1, ctypes.byref(pp.c), 0, ctypes.byref(out)) == 2
    assert lib.spd_batch_run(None, FAKE, 1, FAKE, 0, None) == 1
    lib.spd_batch_plan_destroy(None)


def test_server_validation(lib):
    p = B.Params(list(range(1, 17)), 7.0)
    out = ctypes.c_void_p(7)

    def cfg(**kw):
        c = dict(n_beams=2, dtype=B.SPD_F16, n_rows=8, chunk_cols=4096, cand_capacity=100, slots_per_beam=2,
                 n_streams=0, hbm_budget_bytes=0)
        c.update(kw)
        return B.SpdServerConfig(**c)

    for c, code, msg in [(cfg(n_beams=0), 1, "n_beams"), (cfg(dtype=B.SPD_U8), 2, "F32 or F16"),
                         (cfg(chunk_cols=8), 1, "chunk_cols"), (cfg(slots_per_beam=0), 1, "slots_per_beam"),
                         (cfg(cand_capacity=0), 1, "cand_capacity"), (cfg(hbm_budget_bytes=1000), 3, "budget"),
                         (cfg(n_streams=9), 1, "n_streams"), (cfg(hbm_budget_bytes=-1), 1, "budget"),
                         (cfg(deadline_s=-1.0), 1, "deadline_s"), (cfg(deadline_s=float("nan")), 1, "deadline_s"),
                         (cfg(overflow_capacity=-1), 1, "overflow_capacity"),
                         (cfg(overflow_capacity=100), 1, "overflow_capacity")]:
        assert lib.spd_server_create(ctypes.byref(c), ctypes.byref(p.c), ctypes.byref(out)) == code
        assert out.value is None and msg in _err(lib)
    pp = B.Params([1, 2], 5.0, scope="plane")
    assert lib.spd_server_create(ctypes.byref(cfg()), ctypes.byref(pp.c), ctypes.byref(out)) == 2
    need = lib.spd_server_device_bytes(ctypes.byref(cfg()), ctypes.byref(p.c))
    assert need > 2 * 2 * 8 * (4096 + 15) * 2


def test_server_checkpoint_validation(lib):
    """Beam checkpoints: a NULL server has no checkpoint size, and saving or
    restoring without a server or buffer is refused before any device work."""
    assert lib.spd_server_beam_state_bytes(None) == 0
    buf = ctypes.create_string_buffer(64)
    assert lib.spd_server_save_beam(None, 0, buf, 64) == 1
    assert lib.spd_server_load_beam(None, 0, buf, 64) == 1
    assert lib.spd_server_save_beam(ctypes.c_void_p(0), 0, None, 0) == 1


def test_server_pool_sizing(lib):
    """The shared pool of chunk buffers follows the device-memory budget: the
    beams' own state first, then as many buffers as fit, at most
    slots_per_beam per beam, and none (an error) when not even one fits."""
    p = B.Params(list(range(1, 17)), 7.0)

    def need(**kw):
        c = dict(n_beams=4, dtype=B.SPD_F16, n_rows=8, chunk_cols=4096, cand_capacity=100, slots_per_beam=2,
                 n_streams=0, hbm_budget_bytes=0)
        c.update(kw)
        return lib.spd_server_device_bytes(ctypes.byref(B.SpdServerConfig(**c)), ctypes.byref(p.c))

    all2, all1 = need(), need(slots_per_beam=1)
    per_buf = (all2 - all1) // 4
    beams = all1 - 4 * per_buf
    # one buffer: the chunk with its halo (FP16), the staged chunk, 100 candidates and a count,
    # and the statistics the chunk is searched with (5 doubles per row)
    assert per_buf == 8 * (15 + 4096) * 2 + 8 * 4096 * 2 + 100 * 24 + 8 + 8 * 40
    # the overflow list is allocated once, beside the beams' state
    assert need(overflow_capacity=1000) == all2 + 1000 * 24 + 8
    assert beams > 4 * 8 * 15 * 2                               # halos, statistics, workspaces
    for k in range(1, 9):
        assert need(hbm_budget_bytes=beams + k * per_buf + per_buf // 3) == beams + k * per_buf
    assert need(hbm_budget_bytes=beams + 100 * per_buf) == all2     # never more than slots_per_beam each
    assert need(hbm_budget_bytes=beams + per_buf - 1) == 0 and "budget" in _err(lib)
    assert lib.spd_server_submit(None, 0, 0, FAKE, 0.0) == 1
    lib.spd_server_destroy(None)
