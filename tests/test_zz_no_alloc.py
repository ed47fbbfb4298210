"""spd_detect_static: the whole path with the statistics pass's block
partials in the library's fixed device array instead of a caller workspace.

Two calls in a row on one device, the second on a smaller plane (so the
array holds the first call's partials when the second starts), must each
give bit for bit the statistics, SNRs and width indices of spd_detect with a
workspace on the same arguments, and the same candidate set.
"""
import pytest
import torch

from paper_1611_09704_amd import binding as B
from paper_1611_09704_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _outputs(x, p):
    R = x.shape[0]
    nout = x.shape[1] - p.nmax + 1
    return (torch.empty((p.n_units(R), B.STATS_FIELDS), dtype=torch.float64, device=DEV),
            torch.full((R, nout), -7.0, device=DEV), torch.full((R, nout), 201, dtype=torch.uint8, device=DEV),
            B.new_candidates(1 << 18, DEV), torch.zeros(1, dtype=torch.int64, device=DEV))


def _keys(cand, count):
    n = int(count.item())
    assert n <= cand.shape[0]
    c = B.candidates_to_numpy(cand, n)
    return sorted((int(a["row"]), int(a["t"]), int(a["width"]), float(a["snr"])) for a in c)


def run(fn, x, p, **kw):
    st, snr, widx, cand, cnt = _outputs(x, p)
    fn(x, p, stats=st, snr=snr, widx=widx, cand=cand, cand_count=cnt, **kw)
    torch.cuda.synchronize()
    return st, snr, widx, _keys(cand, cnt)


def check_same(x, p, **kw):
    ref = run(B.spd_detect, x, p, **kw)
    got = run(B.spd_detect_static, x, p, **kw)
    assert torch.equal(got[0], ref[0]), "statistics differ"
    assert torch.equal(got[1], ref[1]), "snr differs"
    assert torch.equal(got[2], ref[2]), "width indices differ"
    assert got[3] == ref[3], "candidate sets differ (%d vs %d)" % (len(got[3]), len(ref[3]))
    return len(ref[3])


@pytest.mark.parametrize("mode", ["sqrtn", "auto"])
def test_static_scratch_matches_workspace_twice(mode):
    big = synth.ska(device=DEV, R=96, L=1 << 18, n_pulses=20, n_bright=3)
    small = synth.ska(device=DEV, R=21, L=20011, n_pulses=10, n_bright=2, seed=7)
    for cfg in (big, small):
        x = cfg["plane"].x
        p = B.Params(cfg["widths"], cfg["threshold"], "row", mode, 1.0)
        print("case: detect_static R=%d L=%d mode=%s" % (x.shape[0], x.shape[1], mode), flush=True)
        assert check_same(x, p) > 0


def test_static_scratch_plane_scope_and_u8():
    cfg = synth.tiny(device=DEV, R=40, L=70001)
    x32 = cfg["plane"].x
    q, scale, zero = synth.quantize_u8(x32, cfg["plane"].row_sigma)
    p = B.Params(cfg["widths"], cfg["threshold"], "plane", "linear", 1.0)
    print("case: detect_static plane scope R=40 L=70001, then u8 R=40 L=70001", flush=True)
    check_same(x32, p)
    pr = B.Params(cfg["widths"], cfg["threshold"], "row", "sqrtn", 1.0)
    check_same(q, pr, scale=scale, zero=zero)
