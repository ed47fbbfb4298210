"""U8 planes: the statistics pass sums the stored bytes as integers (Sum q,
Sum q^2, and the widest boxcar's integer window sums), so its mean, sigma and
sigma of the widest boxcar match the FP64 oracle on the dequantised plane far
inside the 1e-6 parity bound of the float paths -- to 1e-10 relative, the
oracle's own FP64 summation error at these lengths -- in every sigma mode, in
plane scope, with misaligned rows and when streaming (new_col_begin)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1611_09704_amd import binding as B
from paper_1611_09704_amd import synth

pytestmark = pytest.mark.gpu

TIGHT = 1e-10


def _u8_plane(R, L, seed, pad=0):
    cfg = synth.ska(device="cuda", R=R, L=L, n_pulses=max(1, R // 4), n_bright=min(2, R), seed=seed)
    x = cfg["plane"].x
    q, sc, zr = synth.quantize_u8(x, cfg["plane"].row_sigma, row_mu=cfg["plane"].row_mu)
    if pad:
        big = torch.zeros((R, L + pad), dtype=torch.uint8, device="cuda")
        big[:, pad:] = q
        q = big[:, pad:]
    return q, sc, zr


def _compare(q, sc, zr, W, mode, scope="row", ncb=0):
    p = B.Params(W, 7.0, scope, mode, 1.0)
    st = B.msd_compute(q, p, scale=sc, zero=zr, new_col_begin=ncb)
    torch.cuda.synchronize()
    g = st.cpu().numpy()
    x64 = oracle.dequantize_u8(q.cpu().numpy(), sc.cpu().numpy(), zr.cpu().numpy())
    state, o, _, _ = oracle.stream_step(x64, W, new_col_begin=ncb, scope=scope, sigma_mode=mode)
    np.testing.assert_allclose(g[:, 0], o[:, 0], rtol=TIGHT, atol=TIGHT * np.abs(o[:, 1]).max())
    np.testing.assert_allclose(g[:, 1], o[:, 1], rtol=TIGHT)
    if mode != "sqrtn":
        np.testing.assert_allclose(g[:, 2], o[:, 2], rtol=TIGHT)
        np.testing.assert_allclose(g[:, 3], o[:, 3], rtol=TIGHT, atol=TIGHT * np.abs(o[:, 1]).max())
    np.testing.assert_array_equal(B.stats_flags(st).cpu().numpy(), o[:, 4].astype(np.int64))


@pytest.mark.parametrize("mode", ["sqrtn", "auto", "linear"])
@pytest.mark.parametrize("W", [list(range(1, 17)), synth.SKA_WIDTHS, [1, 2, 3, 5, 7, 11, 13]])
def test_u8_statistics_are_exact_sums(mode, W):
    q, sc, zr = _u8_plane(9, 70001, seed=11)
    print("case: u8 stats mode=%s nmax=%d" % (mode, W[-1]), flush=True)
    _compare(q, sc, zr, W, mode)


def test_u8_statistics_plane_scope_misaligned_and_streaming():
    q, sc, zr = _u8_plane(6, 50003, seed=12, pad=3)          # rows start off 4-byte boundaries
    print("case: u8 stats misaligned rows", flush=True)
    _compare(q, sc, zr, synth.SKA_WIDTHS, "auto")
    _compare(q, sc, zr, list(range(1, 33)), "sqrtn", scope="plane")
    q2, sc2, zr2 = _u8_plane(5, 40000, seed=13)
    print("case: u8 stats new_col_begin", flush=True)
    _compare(q2, sc2, zr2, list(range(1, 65)), "linear", ncb=255)
    _compare(q2, sc2, zr2, list(range(1, 17)), "sqrtn", ncb=4099)


def test_u8_statistics_widest_boxcar_4096():
    """The largest widest boxcar: window sums up to 255 * 4096 and their squares."""
    q, sc, zr = _u8_plane(3, 3 * 65536 + 17, seed=14)
    q[1, : 70000] = 255                                      # saturated stretch
    print("case: u8 stats nmax=4096", flush=True)
    _compare(q, sc, zr, [1, 16, 256, 4096], "linear")
