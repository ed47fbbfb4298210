"""The statistics pass with sigma_Nmax walks runs of consecutive starts with
two windows per lane (own and shifted by Nmax).  These cases drive every
variant of that walk against the FP64 oracle: F32 and F16 rows long enough
for the unchecked steps, rows off 4-byte boundaries (the F16 own window
realigned), odd and even Nmax (the F16 shifted window realigned), plane
scope, streaming with new_col_begin, large offsets against small spreads,
signal-dominated rows and constant rows (exact zero variance)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1611_09704_amd import binding as B
import spd_check as C

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _plane(R, L, seed, dtype, offset=0, mean=0.0, scale=1.0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((R, L + offset)) * scale + mean
    x[min(1, R - 1), L // 3: L // 3 + int(0.3 * L)] += 2.0 * scale     # signal-dominated stretch
    t = torch.from_numpy(x.astype(np.float32)).to(DEV)
    if dtype == "f16":
        t = t.to(torch.float16)
    return t[:, offset:]


def _check(x, W, mode, scope="row", ncb=0):
    p = B.Params(W, 7.0, scope, mode, 1.0)
    st = B.msd_compute(x, p, new_col_begin=ncb)
    torch.cuda.synchronize()
    x64 = C.plane_f64(x)
    _, o, _, _ = oracle.stream_step(x64, W, new_col_begin=ncb, scope=scope, sigma_mode=mode)
    C.check_stats(st.cpu().numpy(), o, True)


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("offset", [0, 1, 3])
@pytest.mark.parametrize("nmax", [16, 255, 256, 1023])
def test_walk_variants_match_oracle(dtype, offset, nmax):
    x = _plane(5, 70001, 31 + nmax + offset, dtype, offset)
    print("case: stats walk %s offset=%d nmax=%d" % (dtype, offset, nmax), flush=True)
    W = sorted(set([1, 2, 3, max(1, nmax // 2), nmax]))
    _check(x, W, "auto")


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_walk_plane_scope_streaming_and_wide(dtype):
    x = _plane(4, 3 * 16384 + 999, 41, dtype, 1)
    print("case: stats walk plane scope / streaming / nmax 4096 %s" % dtype, flush=True)
    _check(x, list(range(1, 65)), "linear", scope="plane")
    _check(x, list(range(1, 33)), "auto", ncb=31)
    _check(x, [1, 64, 4096], "linear")


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_walk_offset_rows_and_constant_rows(dtype):
    # mean 1000 against sigma 1 (F16 stores 1000 +- 4 to 0.5): the shift keeps the sums exact enough
    x = _plane(3, 40000, 51, dtype, 0, mean=1000.0, scale=1.0 if dtype == "f32" else 4.0)
    print("case: stats walk large offset %s" % dtype, flush=True)
    _check(x, list(range(1, 129)), "auto")
    c = torch.full((2, 40000), 3.25, dtype=x.dtype, device=DEV)
    p = B.Params(list(range(1, 33)), 7.0, "row", "auto", 1.0)
    st = B.msd_compute(c, p)
    torch.cuda.synchronize()
    s = st.cpu().numpy()
    assert np.all(s[:, 1] == 0.0) and np.all(s[:, 2] == 0.0)
    assert np.all(B.stats_flags(st).cpu().numpy() & B.FLAG_ZERO_VAR)
