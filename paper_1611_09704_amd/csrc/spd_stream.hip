// spd_stream.hip -- the streaming form of the boxcar pass for the width lists
// 1..n, n <= 16 (Sec. 2.3 / Algorithm 1 with the fused threshold of Sec.
// 2.4).  The arithmetic lives in spd_device.h (boxcar_run_fast,
// boxcar_run_short).
//
// Each row's starts are cut into runs of kStreamRun, one wave per run, four
// runs per work-group.  The runs that lie wholly inside their row (every
// start valid, every sample they read inside the row) of planes that allow
// vector loads, with both outputs vector-aligned or none at all, go to
// boxcar_stream_fast_kernel; the rest (each row's last run, or every run of
// other planes) to boxcar_stream_kernel.  The fast kernel exists for the
// lists 1..8 and 1..16; other lists use the checked kernel throughout.
#include <algorithm>

#include "spd_device.h"
#include "spd_kernels.h"

namespace spd {

// Run (row, run0 + segment * waves + w) of work-group (row, segment), wave w.
__device__ __forceinline__ bool stream_run(const BoxcarArgs& ba, int64_t& r, int64_t& t0)
{
    const uint64_t wg = xcd_remap(blockIdx.x, gridDim.x);
    r = (int64_t)(wg / (uint64_t)ba.tiles_per_row);
    const int64_t seg = (int64_t)(wg % (uint64_t)ba.tiles_per_row);
    const int64_t run = ba.run0 + seg * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    t0 = run * kStreamRun;
    return run < ba.run1;
}

template <int DT, int N, bool OUT>
__global__ __launch_bounds__(256) void boxcar_stream_fast_kernel(PlaneArg pl, const spd_row_stats* stats,
                                                                 BoxcarArgs ba, WidthPlan wp)
{
    extern __shared__ float smem[];
    int64_t r, t0;
    if (!stream_run(ba, r, t0)) return;
    const spd_row_stats st = stats[ba.scope == SPD_SCOPE_ROW ? r : 0];
    boxcar_run_fast<DT, N, OUT>(pl, r, t0, st, ba, wp, smem + (size_t)(threadIdx.x >> 6) * 2 * kStreamBuf);
}

template <int DT, int N>
__global__ __launch_bounds__(256) void boxcar_stream_kernel(PlaneArg pl, bool vec, const spd_row_stats* stats,
                                                            BoxcarArgs ba, WidthPlan wp)
{
    extern __shared__ float smem[];
    int64_t r, t0;
    if (!stream_run(ba, r, t0) || t0 >= ba.nout) return;
    const spd_row_stats st = stats[ba.scope == SPD_SCOPE_ROW ? r : 0];
    boxcar_run_short<DT, N>(pl, vec, r, t0, st, ba, wp, smem + (size_t)(threadIdx.x >> 6) * 2 * kStreamBuf);
}

template <int DT, int N>
static hipError_t launch_checked(const PlaneArg& pl, bool vec, const spd_row_stats* stats, const BoxcarArgs& ba,
                                 const WidthPlan& wp, int waves, uint64_t grid, size_t lds, hipStream_t s)
{
    if constexpr (N < 16) {
        if (wp.n != N) return launch_checked<DT, N + 1>(pl, vec, stats, ba, wp, waves, grid, lds, s);
    }
    hipLaunchKernelGGL((boxcar_stream_kernel<DT, N>), dim3(grid), dim3(64 * waves), lds, s, pl, vec, stats, ba, wp);
    return hipGetLastError();
}

template <int DT>
static hipError_t launch_fast(const PlaneArg& pl, const spd_row_stats* stats, const BoxcarArgs& ba,
                              const WidthPlan& wp, bool out, int waves, uint64_t grid, size_t lds, hipStream_t s)
{
    const dim3 g(grid), b(64 * waves);
    if (wp.n == 16 && out)
        hipLaunchKernelGGL((boxcar_stream_fast_kernel<DT, 16, true>), g, b, lds, s, pl, stats, ba, wp);
    else if (wp.n == 16)
        hipLaunchKernelGGL((boxcar_stream_fast_kernel<DT, 16, false>), g, b, lds, s, pl, stats, ba, wp);
    else if (out)
        hipLaunchKernelGGL((boxcar_stream_fast_kernel<DT, 8, true>), g, b, lds, s, pl, stats, ba, wp);
    else
        hipLaunchKernelGGL((boxcar_stream_fast_kernel<DT, 8, false>), g, b, lds, s, pl, stats, ba, wp);
    return hipGetLastError();
}

template <int DT>
static hipError_t launch_stream_dt(const PlaneArg& pl, bool vec, const spd_row_stats* stats, const BoxcarArgs& ba0,
                                   const WidthPlan& wp, int waves, hipStream_t s)
{
    const size_t lds = (size_t)waves * 2 * kStreamBuf * sizeof(float);
    const int64_t runs = (ba0.nout + kStreamRun - 1) / kStreamRun;
    // runs wholly inside the row: every start valid and the 16 samples after the run inside
    int64_t inner = 0;
    const bool both = ba0.snr && ba0.widx && (ba0.out_vec & 1u) && (ba0.out_vec & 4u);
    const bool none = !ba0.snr && !ba0.widx;
    if (vec && (wp.n == 8 || wp.n == 16) && (both || none))
        inner = std::max<int64_t>(0, std::min(ba0.nout / kStreamRun, (pl.n_cols - 16) / kStreamRun));
    BoxcarArgs ba = ba0;
    hipError_t e = hipSuccess;
    if (inner > 0) {
        ba.run0 = 0;
        ba.run1 = inner;
        ba.tiles_per_row = (inner + waves - 1) / waves;
        e = launch_fast<DT>(pl, stats, ba, wp, both, waves, (uint64_t)pl.n_rows * ba.tiles_per_row, lds, s);
        if (e != hipSuccess) return e;
    }
    if (runs > inner) {
        ba.run0 = inner;
        ba.run1 = runs;
        ba.tiles_per_row = (runs - inner + waves - 1) / waves;
        e = launch_checked<DT, 1>(pl, vec, stats, ba, wp, waves, (uint64_t)pl.n_rows * ba.tiles_per_row, lds, s);
    }
    return e;
}

hipError_t launch_stream(int dtype, const PlaneArg& pl, bool vec, const spd_row_stats* stats, const BoxcarArgs& ba,
                         const WidthPlan& wp, int waves, uint64_t ntiles, hipStream_t s)
{
    (void)ntiles;
    if (wp.n < 1 || wp.n > 16) return hipErrorInvalidValue;
    switch (dtype) {
    case SPD_F32: return launch_stream_dt<SPD_F32>(pl, vec, stats, ba, wp, waves, s);
    case SPD_F16: return launch_stream_dt<SPD_F16>(pl, vec, stats, ba, wp, waves, s);
    default: return launch_stream_dt<SPD_U8>(pl, vec, stats, ba, wp, waves, s);
    }
}

}  // namespace spd
