// spd_cluster.hip -- peak-finding over a candidate list in (DM row, time).
//
// Sec. 2.4 keeps every sample above the threshold, so one bright pulse gives
// a cloud of candidates over neighbouring DM trials, starts and widths.  This
// step keeps only the local maxima: a candidate survives iff no SNR in its
// (2*dm_radius+1) x (2*t_radius+1) neighbourhood of the snr plane is higher,
// and no equal SNR there comes earlier in row-major order (so a plateau keeps
// exactly one sample).  Every SNR above a candidate's is itself above the
// threshold, so reading the plane gives the same answer as comparing the
// candidates among themselves.
//
// Each wave takes a contiguous run of the list, 64 entries at a time.  A
// lane per entry first compares it with its nearest neighbours on the row;
// inside a cloud of candidates nearly all lose there.  The rest (local
// maxima along the row) are decided one at a time by the whole wave: the
// own row first, from the 256 starts around the candidate outwards, then the
// other rows of the clipped neighbourhood as one flattened row-major index,
// 64 consecutive elements per pass (a short window packs several rows into
// a pass); four passes make a round, so that four loads per lane are in
// flight, and the wave stops at the first round that finds a beating sample.
// Candidates are sparse next to the plane, so this reads far less than a
// dense max filter over all of it would.

#include <hip/hip_runtime.h>
#include <string.h>

#include "spd_abi_internal.h"
#include "spd_device.h"
#include "spd_kernels.h"

namespace spd {
namespace {

constexpr int kClusterWaves = 4;                 // waves per workgroup
constexpr int kClusterUnroll = 4;                // passes per round
constexpr int kClusterNear = 4;                  // starts each side checked per lane first
constexpr uint32_t kClusterMaxBlocks = 16384;    // grid-stride beyond this

struct ClusterArgs {
    const float* snr;
    int64_t n_rows, n_cols, stride, t_offset;
    const spd_candidate* cand;
    int64_t cand_capacity;
    const int64_t* cand_count;
    int64_t dm_radius, t_radius;
    spd_candidate* peaks;
    int64_t peak_capacity;
    int64_t* peak_count;
};

// Whether any sample of `nrows` window rows other than the candidate's own
// beats v at (r, t): higher, or equal and earlier in row-major order.  The
// rows are row_base, row_base+1, ... passing over row r; columns
// [t0, t0 + W).  Walks the rows x W elements as one flattened index, 64 per
// pass, kClusterUnroll passes per round, and returns after the first round
// in which some lane found a beating sample.
__device__ bool scan_rows(const ClusterArgs& a, float v, int64_t r, int64_t t, int64_t row_base, int64_t nrows,
                          int64_t t0, int64_t W, int lane)
{
    // (row, col) of this lane's element, and a step of 64 elements as rows and columns
    int64_t row, col, step_r, step_c;
    if (W > 64) {
        row = 0; col = lane; step_r = 0; step_c = 64;
    } else {
        const int w = (int)W;
        row = lane / w; col = lane % w; step_r = 64 / w; step_c = 64 % w;
    }
    const int64_t rounds = (nrows * W + 64 * kClusterUnroll - 1) / (64 * kClusterUnroll);
    for (int64_t k = 0; k < rounds; ++k) {
        // lanes past the last row load that row again (in bounds) and ignore
        // the value, so the loads of a round issue back to back
        float s[kClusterUnroll];
        int64_t rr[kClusterUnroll], tt[kClusterUnroll];
        bool in[kClusterUnroll];
#pragma unroll
        for (int u = 0; u < kClusterUnroll; ++u) {
            in[u] = row < nrows;
            const int64_t vr = row_base + (in[u] ? row : nrows - 1);
            rr[u] = vr >= r ? vr + 1 : vr;
            tt[u] = t0 + col;
            s[u] = a.snr[rr[u] * a.stride + tt[u]];
            row += step_r;
            col += step_c;
            if (col >= W) { col -= W; ++row; }
        }
        bool b = false;
#pragma unroll
        for (int u = 0; u < kClusterUnroll; ++u)
            b |= in[u] & ((s[u] > v) | ((s[u] == v) & ((rr[u] < r) | ((rr[u] == r) & (tt[u] < t)))));
        if (__any(b)) return true;
    }
    return false;
}

// Whether any sample of the candidate's own row in [t0, t0 + W) beats v at
// (r, t): higher, or equal at an earlier start.  The row is walked from
// column t - 128 on, wrapping round to t0, so that the first round (256
// starts) is the one centred on t.
__device__ bool scan_own_row(const ClusterArgs& a, float v, int64_t r, int64_t t, int64_t t0, int64_t W, int lane)
{
    constexpr int64_t kHalf = 32 * kClusterUnroll;
    int64_t off = t - t0 - kHalf;
    off = off < 0 ? 0 : off;                        // off < W since t - t0 < W
    const float* row = a.snr + r * a.stride + t0;
    const int64_t rounds = (W + 64 * kClusterUnroll - 1) / (64 * kClusterUnroll);
    for (int64_t k = 0; k < rounds; ++k) {
        float s[kClusterUnroll];
        int64_t cc[kClusterUnroll];
        bool in[kClusterUnroll];
#pragma unroll
        for (int u = 0; u < kClusterUnroll; ++u) {
            const int64_t e = (k * kClusterUnroll + u) * 64 + lane;
            in[u] = e < W;
            int64_t c = (in[u] ? e : 0) + off;
            if (c >= W) c -= W;
            cc[u] = c;
            s[u] = row[c];
        }
        bool b = false;
#pragma unroll
        for (int u = 0; u < kClusterUnroll; ++u)
            b |= in[u] & ((s[u] > v) | ((s[u] == v) & (t0 + cc[u] < t)));
        if (__any(b)) return true;
    }
    return false;
}

__global__ __launch_bounds__(64 * kClusterWaves) void cluster_kernel(ClusterArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * kClusterWaves;
    int64_t n = *a.cand_count;
    if (n > a.cand_capacity) n = a.cand_capacity;
    // Each wave takes a contiguous run of the list, and the runs of one XCD
    // are adjacent: entries appended together lie close together on the
    // plane, so their windows overlap and stay in that XCD's L2.
    const int64_t wave = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kClusterWaves + (threadIdx.x >> 6);
    const int64_t per = (n + nwaves - 1) / nwaves;
    const int64_t i_end = (wave + 1) * per < n ? (wave + 1) * per : n;
    const int64_t i_begin = wave * per;
    if (i_begin >= i_end || a.n_rows == 0 || a.n_cols == 0) return;
    for (int64_t base = i_begin; base < i_end; base += 64) {
        // One candidate per lane first, against its nearest neighbours on
        // the row (kClusterNear each side): inside a cloud of candidates the
        // SNR varies smoothly from one start to the next, so nearly every
        // candidate already loses to an earlier start that is not lower or a
        // later one that is higher.  Indexes and addresses are clamped rather
        // than branched on.
        const int64_t j = base + lane < i_end ? base + lane : i_end - 1;
        const int64_t rl = a.cand[j].row, tl = a.cand[j].t - a.t_offset;
        const bool on = base + lane < i_end && rl >= 0 && rl < a.n_rows && tl >= 0 && tl < a.n_cols;
        const int64_t at = on ? rl * a.stride + tl : 0;
        const float vl = a.snr[at];
        bool lost = false;
#pragma unroll
        for (int d = 1; d <= kClusterNear; ++d) {
            const bool has_l = on && a.t_radius >= d && tl >= d;
            const bool has_r = on && a.t_radius >= d && tl + d < a.n_cols;
            const float left = a.snr[has_l ? at - d : at];
            const float right = a.snr[has_r ? at + d : at];
            lost |= (has_l & (left >= vl)) | (has_r & (right > vl));
        }
        const bool survives = on & !lost;
        uint64_t todo = __ballot(survives);
        // The survivors (local maxima along the row) one at a time with the
        // whole wave: the own row centred on t first, then the other rows.
        while (todo) {
            const int l = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int64_t r = __shfl(rl, l), t = __shfl(tl, l);
            const float v = __shfl(vl, l);
            const int64_t r0 = r - a.dm_radius > 0 ? r - a.dm_radius : 0;
            const int64_t r1 = r + a.dm_radius + 1 < a.n_rows ? r + a.dm_radius + 1 : a.n_rows;
            const int64_t t0 = t - a.t_radius > 0 ? t - a.t_radius : 0;
            const int64_t t1 = t + a.t_radius + 1 < a.n_cols ? t + a.t_radius + 1 : a.n_cols;
            const int64_t W = t1 - t0, H = r1 - r0;
            bool beaten = scan_own_row(a, v, r, t, t0, W, lane);
            if (!beaten && H > 1) beaten = scan_rows(a, v, r, t, r0, H - 1, t0, W, lane);
            if (!beaten && lane == 0) {
                const unsigned long long k = atomicAdd((unsigned long long*)a.peak_count, 1ull);
                if (k < (unsigned long long)a.peak_capacity) a.peaks[k] = a.cand[base + l];
            }
        }
    }
}

}  // namespace
}  // namespace spd

using namespace spd;

extern "C" {

spd_status cluster_candidates(const float* snr, int64_t n_rows, int64_t n_out_cols, int64_t out_stride,
                              int64_t t_offset, const spd_candidate* cand, int64_t cand_capacity,
                              const int64_t* cand_count, int32_t dm_radius, int32_t t_radius,
                              spd_candidate* peaks, int64_t peak_capacity, int64_t* peak_count, void* stream)
{
    clear_error();
    if (!snr || !cand || !cand_count || !peaks || !peak_count)
        return fail(SPD_E_INVALID, "snr, cand, cand_count, peaks and peak_count are required");
    if (n_rows < 0 || n_out_cols < 0 || out_stride < n_out_cols) return fail(SPD_E_INVALID, "bad plane shape");
    if (cand_capacity < 0 || peak_capacity < 0) return fail(SPD_E_INVALID, "capacities must be >= 0");
    if (dm_radius < 0 || dm_radius > SPD_MAX_DM_RADIUS || t_radius < 0 || t_radius > SPD_MAX_T_RADIUS)
        return fail(SPD_E_INVALID, "radii must lie in [0, %d] (rows) and [0, %d] (starts)", SPD_MAX_DM_RADIUS,
                    SPD_MAX_T_RADIUS);
    const uintptr_t c0 = (uintptr_t)cand, c1 = c0 + (uintptr_t)cand_capacity * sizeof(spd_candidate);
    const uintptr_t p0 = (uintptr_t)peaks, p1 = p0 + (uintptr_t)peak_capacity * sizeof(spd_candidate);
    if (c0 < p1 && p0 < c1) return fail(SPD_E_INVALID, "peaks must not overlap the candidate list");
    ClusterArgs a;
    memset(&a, 0, sizeof a);
    a.snr = snr;
    a.n_rows = n_rows;
    a.n_cols = n_out_cols;
    a.stride = out_stride;
    a.t_offset = t_offset;
    a.cand = cand;
    a.cand_capacity = cand_capacity;
    a.cand_count = cand_count;
    a.dm_radius = dm_radius;
    a.t_radius = t_radius;
    a.peaks = peaks;
    a.peak_capacity = peak_capacity;
    a.peak_count = peak_count;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_zero_count(peak_count, s);
    if (e != hipSuccess) return device_status(e, "count reset launch");
    if (cand_capacity == 0) return SPD_OK;
    const int64_t want = (cand_capacity + kClusterWaves - 1) / kClusterWaves;
    const uint32_t blocks = want < (int64_t)kClusterMaxBlocks ? (uint32_t)want : kClusterMaxBlocks;
    hipLaunchKernelGGL(cluster_kernel, dim3(blocks), dim3(64 * kClusterWaves), 0, s, a);
    return device_status(hipGetLastError(), "cluster launch");
}

}  // extern "C"
