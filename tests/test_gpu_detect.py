"""spd_detect: the whole path in one call, with the statistics of later row
chunks on a second stream overlapping the boxcars of earlier ones.

Its statistics, SNRs and width indices must equal, bit for bit, those of
msd_compute followed by boxcar_snr on the same plane (the same kernels run on
the same rows with the same block layout), and its candidate set must be the
same set; one case is also checked against the FP64 oracle directly.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1611_09704_amd import binding as B
from paper_1611_09704_amd import synth
import spd_check as C

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _outputs(x, p):
    R = x.shape[0]
    nout = x.shape[1] - p.nmax + 1
    return (torch.empty((p.n_units(R), B.STATS_FIELDS), dtype=torch.float64, device=DEV),
            torch.full((R, nout), -7.0, device=DEV), torch.full((R, nout), 201, dtype=torch.uint8, device=DEV),
            B.new_candidates(1 << 18, DEV), torch.zeros(1, dtype=torch.int64, device=DEV))


def _cand_keys(cand, count):
    n = int(count.item())
    assert n <= cand.shape[0]
    c = B.candidates_to_numpy(cand, n)
    return sorted((int(a["row"]), int(a["t"]), int(a["width"]), float(a["snr"])) for a in c)


def separate(x, p, scale=None, zero=None):
    st, snr, widx, cand, cnt = _outputs(x, p)
    B.msd_compute(x, p, scale=scale, zero=zero, stats=st)
    B.boxcar_snr(x, p, st, scale=scale, zero=zero, snr=snr, widx=widx, cand=cand, cand_count=cnt)
    torch.cuda.synchronize()
    return st, snr, widx, _cand_keys(cand, cnt)


def pipelined(x, p, chunks, scale=None, zero=None, aux="auto"):
    st, snr, widx, cand, cnt = _outputs(x, p)
    B.spd_detect(x, p, scale=scale, zero=zero, stats=st, snr=snr, widx=widx, cand=cand, cand_count=cnt,
                 row_chunks=chunks, aux_stream=aux)
    torch.cuda.synchronize()
    return st, snr, widx, _cand_keys(cand, cnt)


def assert_same(a, b):
    assert torch.equal(a[0], b[0]), "statistics differ"
    assert torch.equal(a[1], b[1]), "snr differs"
    assert torch.equal(a[2], b[2]), "width indices differ"
    assert a[3] == b[3], "candidate sets differ (%d vs %d)" % (len(a[3]), len(b[3]))


@pytest.mark.parametrize("chunks", [1, 3, 7, 64])
@pytest.mark.parametrize("mode", ["sqrtn", "auto"])
def test_detect_equals_separate_calls(chunks, mode):
    cfg = synth.ska(device=DEV, R=21, L=20011, n_pulses=10, n_bright=3)
    x = cfg["plane"].x
    p = B.Params(cfg["widths"], cfg["threshold"], "row", mode, 1.0)
    print("case: detect R=21 L=20011 chunks=%d mode=%s" % (chunks, mode), flush=True)
    ref = separate(x, p)
    got = pipelined(x, p, chunks)
    assert_same(got, ref)
    assert len(ref[3]) > 0


@pytest.mark.parametrize("form", ["f16", "u8"])
def test_detect_precision_forms(form):
    cfg = synth.tiny(device=DEV, R=16, L=30000)
    x32 = cfg["plane"].x
    if form == "f16":
        x, scale, zero = synth.quantize_f16(x32), None, None
    else:
        x, scale, zero = synth.quantize_u8(x32, cfg["plane"].row_sigma)
    p = B.Params(cfg["widths"], cfg["threshold"])
    print("case: detect %s" % form, flush=True)
    assert_same(pipelined(x, p, 5, scale, zero), separate(x, p, scale, zero))


def test_detect_plane_scope_and_no_aux_stream_run_serially():
    cfg = synth.tiny(device=DEV, R=12, L=20000)
    x = cfg["plane"].x
    pp = B.Params(cfg["widths"], cfg["threshold"], scope="plane")
    print("case: detect plane scope", flush=True)
    assert_same(pipelined(x, pp, 4), separate(x, pp))
    pr = B.Params(cfg["widths"], cfg["threshold"])
    print("case: detect without aux stream", flush=True)
    assert_same(pipelined(x, pr, 4, aux=None), separate(x, pr))


def test_detect_matches_oracle():
    cfg = synth.ska(device=DEV, R=9, L=30000, n_pulses=6, n_bright=2)
    x = cfg["plane"].x
    W, thr = cfg["widths"], cfg["threshold"]
    p = B.Params(W, thr, "row", "auto", 1.0)
    print("case: detect vs oracle", flush=True)
    st, snr, widx, cand, cnt = _outputs(x, p)
    B.spd_detect(x, p, stats=st, snr=snr, widx=widx, cand=cand, cand_count=cnt, row_chunks=4, aux_stream="auto")
    torch.cuda.synchronize()
    x64 = x.cpu().double().numpy()
    o = oracle.detect(x64, W, thr, sigma_mode="auto", kappa=1.0)
    C.check_stats(st.cpu().numpy(), o["stats"], True)
    C.check_snr_widx(x64, W, snr.cpu().numpy(), widx.cpu().numpy(), o["snr"], o["widx"], o["stats"])
    C.check_candidates(B.candidates_to_numpy(cand, int(cnt.item())), o["cands"], thr,
                       lambda r, t: o["snr"][r, t], C.width_rule(x64, W, o["stats"]))


def test_detect_graph_replays():
    """Captured once into a graph (fork onto the statistics stream and join
    back), replayed several times with eager work in between; every replay
    equals the eager result."""
    cfg = synth.tiny(device=DEV, R=24, L=40000)
    x = cfg["plane"].x
    p = B.Params(cfg["widths"], cfg["threshold"])
    ref = separate(x, p)
    st, snr, widx, cand, cnt = _outputs(x, p)
    ws = torch.empty(B.workspace_bytes(x, p), dtype=torch.uint8, device=DEV)
    aux = torch.cuda.Stream()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):               # warm the event cache outside the capture
        B.spd_detect(x, p, stats=st, snr=snr, widx=widx, cand=cand, cand_count=cnt, workspace=ws,
                     row_chunks=6, aux_stream=aux)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    print("case: detect graph capture", flush=True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        B.spd_detect(x, p, stats=st, snr=snr, widx=widx, cand=cand, cand_count=cnt, workspace=ws,
                     row_chunks=6, aux_stream=aux)
    for k in range(3):
        snr.fill_(-1.0)
        widx.fill_(255)
        st.zero_()
        cnt.fill_(-5)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        print("replay %d" % k, flush=True)
        assert_same((st, snr, widx, _cand_keys(cand, cnt)), ref)


def test_detect_full_size_equals_separate_calls():
    """The 4,096 x 2^20 SKA-like plane in the launch configuration the
    benchmark times (16 row chunks): bitwise equal to the separate calls,
    whose own full-size parity with the oracle is checked on sampled rows
    elsewhere."""
    cfg = synth.ska(device=DEV)
    x = cfg["plane"].x
    p = B.Params(cfg["widths"], cfg["threshold"], "row", "auto", 1.0)
    print("case: detect full size", flush=True)
    R, L = x.shape
    nout = L - p.nmax + 1
    snr_a = torch.empty((R, nout), device=DEV)
    widx_a = torch.empty((R, nout), dtype=torch.uint8, device=DEV)
    st_a = torch.empty((R, B.STATS_FIELDS), dtype=torch.float64, device=DEV)
    cand_a, cnt_a = B.new_candidates(1 << 21, DEV), torch.zeros(1, dtype=torch.int64, device=DEV)
    B.msd_compute(x, p, stats=st_a)
    B.boxcar_snr(x, p, st_a, snr=snr_a, widx=widx_a, cand=cand_a, cand_count=cnt_a)
    snr_b = torch.empty_like(snr_a)
    widx_b = torch.empty_like(widx_a)
    st_b = torch.empty_like(st_a)
    cand_b, cnt_b = B.new_candidates(1 << 21, DEV), torch.zeros(1, dtype=torch.int64, device=DEV)
    B.spd_detect(x, p, stats=st_b, snr=snr_b, widx=widx_b, cand=cand_b, cand_count=cnt_b, row_chunks=16,
                 aux_stream="auto")
    torch.cuda.synchronize()
    assert torch.equal(st_a, st_b)
    assert torch.equal(widx_a, widx_b)
    assert torch.equal(snr_a, snr_b)
    ka, kb = _cand_keys(cand_a, cnt_a), _cand_keys(cand_b, cnt_b)
    print("detect full size: %d candidates" % len(ka), flush=True)
    assert ka == kb and len(ka) > 1000
    del snr_a, snr_b, widx_a, widx_b, x
    torch.cuda.empty_cache()
