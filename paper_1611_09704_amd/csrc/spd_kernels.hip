// spd_kernels.hip -- one-plane launches of the detection path on gfx950.
//
//   msd_x_kernel / msd_xy_kernel   per-block (n, T, S) partials, Sec. 2.1
//   msd_finalize_kernel            FP64 merge across blocks and sigma_N
//                                  coefficients, Sec. 2.1-2.2
//   boxcar_kernel                  boxcars, SNR, highest SNR and its width,
//                                  fused threshold, Sec. 2.3 / Algorithm 1,
//                                  Sec. 2.4 (starts 64 apart per lane)
//   boxcar_win_kernel              the same with 8 consecutive starts per lane
//                                  and each group's reads held in registers
//   boxcar_dit_kernel              boxcars combined with decimation in time
//                                  (widths 2^l*(9..16) on the decimated series)
// (the streaming form of the lists 1..n, n <= 16, is in spd_stream.hip)
//   select_kernel                  threshold over stored outputs, Sec. 2.4
//
// One work-group per (row, column block) or (row, time tile), numbered so that
// each XCD gets a contiguous range.  The arithmetic lives in spd_device.h.
#include "spd_device.h"
#include "spd_kernels.h"

namespace spd {

template <int DT>
__global__ __launch_bounds__(256) void msd_x_kernel(PlaneArg pl, bool vec, int64_t ncb, int64_t bc,
                                                    int64_t nblk, double* part)
{
    __shared__ MsdScratch sh;
    const uint64_t wg = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t r = (int64_t)(wg / (uint64_t)nblk), b = (int64_t)(wg % (uint64_t)nblk);
    msd_block_x<DT>(pl, vec, r, b, ncb, bc, part + wg * 6, sh);
}

template <int DT>
__global__ __launch_bounds__(256) void msd_xy_kernel(PlaneArg pl, bool vec, int64_t ncb, int64_t bc,
                                                     int64_t nblk, int32_t nmax, int64_t nout, double* part)
{
    __shared__ MsdScratch sh;
    const uint64_t wg = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t r = (int64_t)(wg / (uint64_t)nblk), b = (int64_t)(wg % (uint64_t)nblk);
    msd_block_xy<DT>(pl, vec, r, b, ncb, bc, nmax, nout, part + wg * 6, sh);
}

__global__ __launch_bounds__(256) void msd_finalize_kernel(const double* part, int64_t per_unit,
                                                           int32_t need_y, int32_t accumulate,
                                                           spd_msd_state* state, spd_row_stats* stats,
                                                           int32_t nmax, int32_t mode, double kappa)
{
    __shared__ FinalizeScratch sh;
    const int64_t u = blockIdx.x;
    finalize_unit(part + (size_t)u * per_unit * 6, per_unit, need_y != 0, accumulate != 0,
                  state ? state + u : nullptr, stats + u, nmax, mode, kappa, sh);
}

template <int DT, int X, bool UNIT, int SMALL>
__global__ __launch_bounds__(256) void boxcar_kernel(PlaneArg pl, bool vec, const spd_row_stats* stats,
                                                     BoxcarArgs ba, WidthPlan wp)
{
    extern __shared__ float smem[];
    const uint64_t tile = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t r = (int64_t)(tile / (uint64_t)ba.tiles_per_row);
    const int64_t tt = (int64_t)(tile % (uint64_t)ba.tiles_per_row);
    const spd_row_stats st = stats[ba.scope == SPD_SCOPE_ROW ? r : 0];
    boxcar_tile<DT, X, UNIT, SMALL>(pl, vec, r, tt, st, ba, wp, smem, true);
}

// The group form holds each start's running sum, maximum, group and group-start
// sum plus two groups' windows; capping it at 128 VGPRs keeps 4 waves per SIMD
// without spills (uncapped it takes 132 and drops to 3).
template <int DT, int SMALLN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SMALLN == 0 ? 4 : 1))) void boxcar_win_kernel(PlaneArg pl, bool vec, const spd_row_stats* stats,
                                                         BoxcarArgs ba, WidthPlan wp)
{
    extern __shared__ float smem[];
    const uint64_t tile = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t r = (int64_t)(tile / (uint64_t)ba.tiles_per_row);
    const int64_t tt = (int64_t)(tile % (uint64_t)ba.tiles_per_row);
    const spd_row_stats st = stats[ba.scope == SPD_SCOPE_ROW ? r : 0];
    boxcar_tile_win<DT, SMALLN>(pl, vec, r, tt, st, ba, wp, smem);
}

// Boxcars combined with decimation in time: widths 1..16 at every start, and
// 2^l*(9..16) at starts that are multiples of 2^l, l = 1..levels.
template <int DT>
__global__ __launch_bounds__(256) void boxcar_dit_kernel(PlaneArg pl, bool vec, const spd_row_stats* stats,
                                                         BoxcarArgs ba, WidthPlan wp)
{
    extern __shared__ float smem[];
    const uint64_t tile = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t r = (int64_t)(tile / (uint64_t)ba.tiles_per_row);
    const int64_t tt = (int64_t)(tile % (uint64_t)ba.tiles_per_row);
    const spd_row_stats st = stats[ba.scope == SPD_SCOPE_ROW ? r : 0];
    boxcar_tile_win<DT, kDitBase, true>(pl, vec, r, tt, st, ba, wp, smem);
}

// Sec. 2.4 over stored snr / width-index arrays.  A work-group covers kSelCols
// columns of one row, 16 per lane in dword loads 256 columns apart: every load
// instruction reads 256 consecutive bytes per wave, and sixteen loads per lane
// are in flight (measured faster than four 16-byte loads per lane, even on
// aligned rows).  A wave with no SNR at the threshold stops there; the others
// compact with one ballot per value and one atomic per wave that has
// candidates.
__global__ __launch_bounds__(256) void select_kernel(const float* snr, const uint8_t* widx,
                                                     int64_t ncols, int64_t stride, int64_t chunks,
                                                     SelectArgs sa)
{
    const int lane = threadIdx.x & 63, tid = threadIdx.x;
    const uint64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t r = (int64_t)(blk / (uint64_t)chunks), ch = (int64_t)(blk % (uint64_t)chunks);
    const float* row = snr + r * stride;
    const int64_t p0 = ch * kSelCols + tid;                         // column of v[i] is p0 + 256i
    float v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int64_t t = p0 + 256 * i;
        v[i] = t < ncols ? row[t] : -INFINITY;                     // never at a finite threshold
    }
    float m = v[0];
#pragma unroll
    for (int i = 1; i < 16; ++i) m = fmaxf(m, v[i]);
    if (!__ballot(m >= sa.threshold)) return;                      // the whole wave leaves
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const bool pred = v[i] >= sa.threshold;
        const uint64_t mask = __ballot(pred);
        if (!mask) continue;
        const int cntw = __popcll(mask);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd((unsigned long long*)sa.cand_count, (unsigned long long)cntw);
        base = __shfl(base, 0);
        if (pred) {
            const unsigned long long k = base + (unsigned long long)before;
            if (k < (unsigned long long)sa.cand_capacity) {
                const int64_t t = p0 + 256 * i;
                spd_candidate cd;
                cd.row = (int32_t)r;
                cd.width = sa.width[widx[r * stride + t]];
                cd.t = t + sa.t_offset;
                cd.snr = v[i];
                cd.beam = 0;
                sa.cand[k] = cd;
            }
        }
    }
}

__global__ void fill_i64_kernel(int64_t* p, int64_t n, int64_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <int DT>
static hipError_t launch_msd_dt(const PlaneArg& pl, bool vec, bool with_y, int64_t ncb, int64_t bc,
                                int64_t nblk, int32_t nmax, int64_t nout, double* part, hipStream_t s)
{
    const uint64_t nwg = (uint64_t)pl.n_rows * (uint64_t)nblk;
    if (!with_y) {
        hipLaunchKernelGGL((msd_x_kernel<DT>), dim3(nwg), dim3(256), 0, s, pl, vec, ncb, bc, nblk, part);
    } else {
        hipLaunchKernelGGL((msd_xy_kernel<DT>), dim3(nwg), dim3(256), 0, s, pl, vec, ncb, bc, nblk, nmax, nout,
                           part);
    }
    return hipGetLastError();
}

hipError_t launch_msd(int dtype, const PlaneArg& pl, bool vec, bool with_y, int64_t ncb, int64_t bc,
                      int64_t nblk, int32_t nmax, int64_t nout, double* part, hipStream_t s)
{
    switch (dtype) {
    case SPD_F32: return launch_msd_dt<SPD_F32>(pl, vec, with_y, ncb, bc, nblk, nmax, nout, part, s);
    case SPD_F16: return launch_msd_dt<SPD_F16>(pl, vec, with_y, ncb, bc, nblk, nmax, nout, part, s);
    default: return launch_msd_dt<SPD_U8>(pl, vec, with_y, ncb, bc, nblk, nmax, nout, part, s);
    }
}

hipError_t launch_finalize(const double* part, int64_t n_units, int64_t per_unit, bool need_y,
                           bool accumulate, spd_msd_state* state, spd_row_stats* stats, int32_t nmax,
                           int32_t mode, double kappa, hipStream_t s)
{
    hipLaunchKernelGGL(msd_finalize_kernel, dim3((uint32_t)n_units), dim3(256), 0, s, part, per_unit,
                       (int32_t)need_y, (int32_t)accumulate, state, stats, nmax, mode, kappa);
    return hipGetLastError();
}

size_t boxcar_lds_bytes(int waves, const BoxcarArgs& ba, bool win)
{
    return (size_t)(win ? kWinTableFloats : kTableFloats) * 4 + (size_t)waves * ba.wave_floats * 4;
}

template <int DT>
static hipError_t launch_boxcar_dt(const PlaneArg& pl, bool vec, const spd_row_stats* stats,
                                   const BoxcarArgs& ba, const WidthPlan& wp, int waves, uint64_t ntiles,
                                   hipStream_t s)
{
    const size_t lds = boxcar_lds_bytes(waves, ba, wp.win != 0);   // <= 64 KiB by construction of the plan
    constexpr int X = kOutPerLane;
    if (wp.win == 4)
        return launch_stream(DT, pl, vec, stats, ba, wp, waves, ntiles, s);
    if (wp.win == 3)
        hipLaunchKernelGGL((boxcar_dit_kernel<DT>), dim3(ntiles), dim3(64 * waves), lds, s, pl, vec, stats, ba, wp);
    else if (wp.win == 1)
        hipLaunchKernelGGL((boxcar_win_kernel<DT, 0>), dim3(ntiles), dim3(64 * waves), lds, s, pl, vec, stats, ba, wp);
    else if (wp.win == 2 && wp.n <= 8)
        hipLaunchKernelGGL((boxcar_win_kernel<DT, 8>), dim3(ntiles), dim3(64 * waves), lds, s, pl, vec, stats, ba, wp);
    else if (wp.win == 2)
        hipLaunchKernelGGL((boxcar_win_kernel<DT, 16>), dim3(ntiles), dim3(64 * waves), lds, s, pl, vec, stats, ba,
                           wp);
    else if (wp.unit_counts && wp.n <= 8)
        hipLaunchKernelGGL((boxcar_kernel<DT, X, true, 8>), dim3(ntiles), dim3(64 * waves), lds, s, pl, vec, stats,
                           ba, wp);
    else if (wp.unit_counts && wp.n <= 16)
        hipLaunchKernelGGL((boxcar_kernel<DT, X, true, 16>), dim3(ntiles), dim3(64 * waves), lds, s, pl, vec, stats,
                           ba, wp);
    else if (wp.unit_counts)
        hipLaunchKernelGGL((boxcar_kernel<DT, X, true, 0>), dim3(ntiles), dim3(64 * waves), lds, s, pl, vec, stats,
                           ba, wp);
    else
        hipLaunchKernelGGL((boxcar_kernel<DT, X, false, 0>), dim3(ntiles), dim3(64 * waves), lds, s, pl, vec, stats,
                           ba, wp);
    return hipGetLastError();
}

hipError_t launch_boxcar(int dtype, const PlaneArg& pl, bool vec, const spd_row_stats* stats,
                         const BoxcarArgs& ba, const WidthPlan& wp, int X, int waves, uint64_t ntiles,
                         hipStream_t s)
{
    (void)X;
    switch (dtype) {
    case SPD_F32: return launch_boxcar_dt<SPD_F32>(pl, vec, stats, ba, wp, waves, ntiles, s);
    case SPD_F16: return launch_boxcar_dt<SPD_F16>(pl, vec, stats, ba, wp, waves, ntiles, s);
    default: return launch_boxcar_dt<SPD_U8>(pl, vec, stats, ba, wp, waves, ntiles, s);
    }
}

hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s)
{
    hipLaunchKernelGGL(fill_i64_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_zero_count(int64_t* count, hipStream_t s) { return launch_fill_i64(count, 1, 0, s); }

hipError_t launch_select(const float* snr, const uint8_t* widx, int64_t nrows, int64_t ncols,
                         int64_t stride, const SelectArgs& sa, hipStream_t s)
{
    const int64_t chunks = (ncols + kSelCols - 1) / kSelCols;
    const uint64_t nb = (uint64_t)nrows * (uint64_t)chunks;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(select_kernel, dim3(nb), dim3(256), 0, s, snr, widx, ncols, stride, chunks, sa);
    return hipGetLastError();
}

}  // namespace spd
