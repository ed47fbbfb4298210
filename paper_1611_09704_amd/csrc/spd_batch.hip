// spd_batch.hip -- the detection path over many beams of uneven shape in one
// persistent launch per step (Sec. 2.1-2.4 applied to every beam).
//
// A plan owns the per-beam descriptors, the block partials, the per-row
// statistics and two work-queue counters.  A run is five launches:
//   fill (queue counters)  ->  batch_msd_kernel (persistent; items are
//   (beam, row, column block))  ->  batch_finalize_kernel (one work-group per
//   row of every beam)  ->  fill (candidate count)  ->  batch_boxcar_kernel
//   (persistent; items are (beam, row, time tile), fused threshold,
//   candidates only).
// Persistent work-groups take chunks of consecutive items from an atomic
// counter until it passes the total, so every wave reaches the exit.  The
// five launches can be captured once into a hipGraph and replayed; counters
// are cleared by a fill kernel, never by a memset node.
//
// The autotuner times the boxcar kernel on the plan's own data for a few
// schedules (outputs per lane, waves per work-group, work-groups per CU) and
// caches the winner on disk keyed by device, dtype and width list.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "spd_abi_internal.h"
#include "spd_device.h"
#include "spd_kernels.h"
#include "spd_sched.h"

namespace spd {

constexpr int kMaxBeams = 256;
constexpr int64_t kMsdBlockCols = 32768;
constexpr size_t kBatchLdsReserve = 4096;     // static LDS of the persistent kernels (beam table)

struct BeamDesc {
    PlaneArg pl;
    int64_t msd_start;      // first MSD item of the beam
    int64_t tile_start;     // first boxcar tile of the beam
    int64_t unit_start;     // first row (statistics unit) of the beam
    int64_t nblk;           // MSD column blocks per row
    int64_t tiles_per_row;
    int64_t nout;
    int32_t vec;
    int32_t reserved;
};

// The value of lane 0 as a wave-uniform (scalar) value.
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// beam holding item `it` given ascending starts s[0..n); wave-uniform
__device__ __forceinline__ int find_beam(const int64_t* s, int n, int64_t it)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s[mid] <= it) lo = mid; else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// Next chunk of items for the whole work-group; uniform result.
__device__ __forceinline__ int64_t grab_items(int64_t* queue, int grab, int64_t* slot)
{
    if (threadIdx.x == 0) *slot = (int64_t)atomicAdd((unsigned long long*)queue, (unsigned long long)grab);
    __syncthreads();
    const int64_t g0 = uniform64(*slot);
    __syncthreads();
    return g0;
}

template <int DT, bool WITH_Y>
__global__ __launch_bounds__(256) void batch_msd_kernel(const BeamDesc* beams, int n_beams, int64_t total,
                                                        int64_t* queue, int grab, int32_t nmax, double* part)
{
    __shared__ MsdScratch sh;
    __shared__ int64_t starts[kMaxBeams];
    __shared__ int64_t slot;
    for (int b = threadIdx.x; b < n_beams; b += blockDim.x) starts[b] = beams[b].msd_start;
    __syncthreads();
    for (;;) {
        const int64_t g0 = grab_items(queue, grab, &slot);
        if (g0 >= total) break;
        const int64_t g1 = min(g0 + (int64_t)grab, total);
        for (int64_t it = g0; it < g1; ++it) {
            const int b = find_beam(starts, n_beams, it);
            const BeamDesc d = beams[b];
            const int64_t local = it - d.msd_start;
            const int64_t r = local / d.nblk, blk = local % d.nblk;
            double* out6 = part + it * 6;
            if (WITH_Y)
                msd_block_xy<DT>(d.pl, d.vec != 0, r, blk, 0, kMsdBlockCols, nmax, d.nout, out6, sh);
            else
                msd_block_x<DT>(d.pl, d.vec != 0, r, blk, 0, kMsdBlockCols, out6, sh);
        }
    }
}

__global__ __launch_bounds__(256) void batch_finalize_kernel(const BeamDesc* beams, int n_beams,
                                                             const double* part, spd_row_stats* stats,
                                                             int32_t need_y, int32_t nmax, int32_t mode,
                                                             double kappa)
{
    __shared__ FinalizeScratch sh;
    __shared__ int64_t starts[kMaxBeams];
    for (int b = threadIdx.x; b < n_beams; b += blockDim.x) starts[b] = beams[b].unit_start;
    __syncthreads();
    const int64_t u = blockIdx.x;
    const int b = find_beam(starts, n_beams, u);
    const BeamDesc d = beams[b];
    const int64_t first_item = d.msd_start + (u - d.unit_start) * d.nblk;
    finalize_unit(part + first_item * 6, d.nblk, need_y != 0, false, nullptr, stats + u, nmax, mode, kappa, sh);
}

template <int DT, int X, bool UNIT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(X == 4 ? 5 : (UNIT ? 4 : 3)))) void batch_boxcar_kernel(const BeamDesc* beams, int n_beams, int64_t total,
                                                           int64_t* queue, int grab, const spd_row_stats* stats,
                                                           BoxcarArgs ba, WidthPlan wp)
{
    extern __shared__ float smem[];
    __shared__ int64_t starts[kMaxBeams];
    __shared__ int64_t slot;
    for (int b = threadIdx.x; b < n_beams; b += blockDim.x) starts[b] = beams[b].tile_start;
    __syncthreads();
    int64_t prev_unit = -1;
    for (;;) {
        const int64_t g0 = grab_items(queue, grab, &slot);
        if (g0 >= total) break;
        const int64_t g1 = min(g0 + (int64_t)grab, total);
        for (int64_t it = g0; it < g1; ++it) {
            const int b = find_beam(starts, n_beams, it);
            const BeamDesc d = beams[b];
            const int64_t local = it - d.tile_start;
            const int64_t r = local / d.tiles_per_row, tt = local % d.tiles_per_row;
            BoxcarArgs a = ba;
            a.tiles_per_row = d.tiles_per_row;
            a.nout = d.nout;
            a.beam = (uint32_t)b;
            const int64_t unit = d.unit_start + r;
            const spd_row_stats st = stats[unit];
            boxcar_tile<DT, X, UNIT>(d.pl, d.vec != 0, r, tt, st, a, wp, smem, unit != prev_unit);
            prev_unit = unit;
        }
    }
}

// All tiles of all beams in one ordinary launch: work-group i takes tile i
// (XCD-aware numbering), finds its beam and row, and runs the same tile code.
template <int DT, int X, bool UNIT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(UNIT ? 5 : 1))) void batch_boxcar_grid_kernel(const BeamDesc* beams, int n_beams,
                                                                const spd_row_stats* stats, BoxcarArgs ba,
                                                                WidthPlan wp)
{
    extern __shared__ float smem[];
    __shared__ int64_t starts[kMaxBeams];
    for (int b = threadIdx.x; b < n_beams; b += blockDim.x) starts[b] = beams[b].tile_start;
    __syncthreads();
    const int64_t it = (int64_t)xcd_remap(blockIdx.x, gridDim.x);
    const int b = find_beam(starts, n_beams, it);
    const BeamDesc d = beams[b];
    const int64_t local = it - d.tile_start;
    const int64_t r = local / d.tiles_per_row, tt = local % d.tiles_per_row;
    ba.tiles_per_row = d.tiles_per_row;
    ba.nout = d.nout;
    ba.beam = (uint32_t)b;
    const spd_row_stats st = stats[d.unit_start + r];
    boxcar_tile<DT, X, UNIT>(d.pl, d.vec != 0, r, tt, st, ba, wp, smem, true);
}

// The register-window form of the same grid launch (8 consecutive starts per
// lane; tiles numbered for that form).  Capped at 128 VGPRs like the one-plane
// kernel of the same form.
template <int DT, int SMALLN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SMALLN == 0 ? 4 : 6))) void batch_boxcar_win_grid_kernel(
    const BeamDesc* beams, int n_beams, const spd_row_stats* stats, BoxcarArgs ba, WidthPlan wp)
{
    extern __shared__ float smem[];
    __shared__ int64_t starts[kMaxBeams];
    for (int b = threadIdx.x; b < n_beams; b += blockDim.x) starts[b] = beams[b].tile_start;
    __syncthreads();
    const int64_t it = (int64_t)xcd_remap(blockIdx.x, gridDim.x);
    const int b = find_beam(starts, n_beams, it);
    const BeamDesc d = beams[b];
    const int64_t local = it - d.tile_start;
    const int64_t r = local / d.tiles_per_row, tt = local % d.tiles_per_row;
    ba.tiles_per_row = d.tiles_per_row;
    ba.nout = d.nout;
    ba.beam = (uint32_t)b;
    const spd_row_stats st = stats[d.unit_start + r];
    boxcar_tile_win<DT, SMALLN>(d.pl, d.vec != 0, r, tt, st, ba, wp, smem);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct Schedule {
    int X = kOutPerLane;    // outputs per lane (4 or 8)
    int waves = 4;          // waves per work-group
    int wgs_per_cu = 4;     // persistent work-groups per CU; 0 = one work-group per tile (grid launch)
    int grab = 4;           // tiles per queue grab (persistent only)
    int win = 0;            // 1: register-window form (X = 8 consecutive starts, grid launch only)
};

// Plan slots: 0 strided X = 4, 1 strided X = 8, 2 register-window form.
constexpr int kLayouts = 3;

}  // namespace spd

struct spd_batch_plan {
    int n_beams = 0;
    int dtype = 0;
    int device = 0;
    int cus = 0;
    std::vector<int32_t> widths;
    spd_params params{};
    spd::WidthPlan wp[spd::kLayouts];       // strided X = 4, strided X = 8, register-window form
    spd::BoxcarArgs ba[spd::kLayouts];
    int max_waves[spd::kLayouts] = {1, 1, 1};
    bool has_win = false;
    spd::Schedule sched;
    int tuned = 0;
    float tune_ms = 0.f;
    int64_t msd_items = 0, tiles[spd::kLayouts] = {0, 0, 0}, units = 0;
    std::vector<spd::BeamDesc> host_beams;
    spd::BeamDesc* d_beams[spd::kLayouts] = {nullptr, nullptr, nullptr};   // tile numbering differs per slot
    double* d_part = nullptr;
    spd_row_stats* d_stats = nullptr;
    int64_t* d_counters = nullptr;          // [0] msd queue, [1] boxcar queue, [2] scratch count
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t capture_stream = nullptr;
    spd_candidate* g_cand = nullptr;
    int64_t g_cap = -1;
    int64_t* g_count = nullptr;
    std::vector<std::pair<spd::Schedule, float>> tune_table;   // schedule, ns per output start
};

namespace spd {

static int xi(int X) { return X == 4 ? 0 : 1; }
static int slot(const Schedule& sc) { return sc.win ? 2 : xi(sc.X); }

template <int DT>
static hipError_t enqueue_msd(spd_batch_plan* P, hipStream_t s)
{
    const bool need_y = P->params.sigma_mode != SPD_SIGMA_SQRTN;
    const int nmax = P->widths.back();
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(P->msd_items, (int64_t)P->cus * 8));
    if (need_y)
        hipLaunchKernelGGL((batch_msd_kernel<DT, true>), dim3(grid), dim3(256), 0, s, P->d_beams[1], P->n_beams,
                           P->msd_items, P->d_counters, 2, nmax, P->d_part);
    else
        hipLaunchKernelGGL((batch_msd_kernel<DT, false>), dim3(grid), dim3(256), 0, s, P->d_beams[1], P->n_beams,
                           P->msd_items, P->d_counters, 2, nmax, P->d_part);
    return hipGetLastError();
}

template <int DT, int X>
static hipError_t enqueue_boxcar_x(spd_batch_plan* P, const Schedule& sc, const BoxcarArgs& ba, int64_t total,
                                   hipStream_t s)
{
    const int k = xi(X);
    const size_t lds = boxcar_lds_bytes(sc.waves, P->ba[k]);
    if (sc.wgs_per_cu == 0) {
        if (total <= 0) return hipSuccess;
        if ((uint64_t)total * 64u * (uint64_t)sc.waves > kMaxGridItems) return hipErrorInvalidConfiguration;
        if (P->wp[k].unit_counts)
            hipLaunchKernelGGL((batch_boxcar_grid_kernel<DT, X, true>), dim3((unsigned)total), dim3(64 * sc.waves),
                               lds, s, P->d_beams[k], P->n_beams, P->d_stats, ba, P->wp[k]);
        else
            hipLaunchKernelGGL((batch_boxcar_grid_kernel<DT, X, false>), dim3((unsigned)total), dim3(64 * sc.waves),
                               lds, s, P->d_beams[k], P->n_beams, P->d_stats, ba, P->wp[k]);
        return hipGetLastError();
    }
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(total, (int64_t)P->cus * sc.wgs_per_cu));
    if (P->wp[k].unit_counts)
        hipLaunchKernelGGL((batch_boxcar_kernel<DT, X, true>), dim3(grid), dim3(64 * sc.waves), lds, s,
                           P->d_beams[k], P->n_beams, total, P->d_counters + 1, sc.grab, P->d_stats, ba, P->wp[k]);
    else
        hipLaunchKernelGGL((batch_boxcar_kernel<DT, X, false>), dim3(grid), dim3(64 * sc.waves), lds, s,
                           P->d_beams[k], P->n_beams, total, P->d_counters + 1, sc.grab, P->d_stats, ba, P->wp[k]);
    return hipGetLastError();
}

template <int DT>
static hipError_t enqueue_boxcar_win(spd_batch_plan* P, const Schedule& sc, const BoxcarArgs& ba, int64_t total,
                                     hipStream_t s)
{
    const WidthPlan& wp = P->wp[2];
    const size_t lds = boxcar_lds_bytes(sc.waves, P->ba[2], true);
    if (total <= 0) return hipSuccess;
    if ((uint64_t)total * 64u * (uint64_t)sc.waves > kMaxGridItems) return hipErrorInvalidConfiguration;
    if (wp.win == 1)
        hipLaunchKernelGGL((batch_boxcar_win_grid_kernel<DT, 0>), dim3((unsigned)total), dim3(64 * sc.waves), lds, s,
                           P->d_beams[2], P->n_beams, P->d_stats, ba, wp);
    else if (wp.n <= 8)
        hipLaunchKernelGGL((batch_boxcar_win_grid_kernel<DT, 8>), dim3((unsigned)total), dim3(64 * sc.waves), lds, s,
                           P->d_beams[2], P->n_beams, P->d_stats, ba, wp);
    else
        hipLaunchKernelGGL((batch_boxcar_win_grid_kernel<DT, 16>), dim3((unsigned)total), dim3(64 * sc.waves), lds,
                           s, P->d_beams[2], P->n_beams, P->d_stats, ba, wp);
    return hipGetLastError();
}

template <int DT>
static hipError_t enqueue_boxcar(spd_batch_plan* P, const Schedule& sc, spd_candidate* cand, int64_t cap,
                                 int64_t* count, int64_t limit, hipStream_t s)
{
    const int k = slot(sc);
    BoxcarArgs ba = P->ba[k];
    ba.cand = cand;
    ba.cand_capacity = cap;
    ba.cand_count = count;
    // Each work-group holds sc.waves waves; tiles were numbered for max_waves waves.
    // Renumbering is avoided by requiring sc.waves == max_waves (see tune()).
    const int64_t total = limit >= 0 ? std::min(limit, P->tiles[k]) : P->tiles[k];
    if (sc.win) return enqueue_boxcar_win<DT>(P, sc, ba, total, s);
    return sc.X == 4 ? enqueue_boxcar_x<DT, 4>(P, sc, ba, total, s) : enqueue_boxcar_x<DT, 8>(P, sc, ba, total, s);
}

static hipError_t enqueue_boxcar_dt(spd_batch_plan* P, const Schedule& sc, spd_candidate* cand, int64_t cap,
                                    int64_t* count, int64_t limit, hipStream_t s)
{
    switch (P->dtype) {
    case SPD_F32: return enqueue_boxcar<SPD_F32>(P, sc, cand, cap, count, limit, s);
    case SPD_F16: return enqueue_boxcar<SPD_F16>(P, sc, cand, cap, count, limit, s);
    default: return enqueue_boxcar<SPD_U8>(P, sc, cand, cap, count, limit, s);
    }
}

static hipError_t enqueue_run(spd_batch_plan* P, spd_candidate* cand, int64_t cap, int64_t* count, hipStream_t s)
{
    hipError_t e = launch_fill_i64(P->d_counters, 2, 0, s);
    if (e != hipSuccess) return e;
    switch (P->dtype) {
    case SPD_F32: e = enqueue_msd<SPD_F32>(P, s); break;
    case SPD_F16: e = enqueue_msd<SPD_F16>(P, s); break;
    default: e = enqueue_msd<SPD_U8>(P, s); break;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_finalize_kernel, dim3((unsigned)P->units), dim3(256), 0, s, P->d_beams[1], P->n_beams,
                       P->d_part, P->d_stats, (int32_t)(P->params.sigma_mode != SPD_SIGMA_SQRTN),
                       (int32_t)P->widths.back(), (int32_t)P->params.sigma_mode, (double)P->params.auto_kappa);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_fill_i64(count, 1, 0, s)) != hipSuccess) return e;
    return enqueue_boxcar_dt(P, P->sched, cand, cap, count, -1, s);
}

static std::string tune_cache_path()
{
    const char* env = getenv("SPD_TUNE_CACHE");
    if (env && *env) return env;
    const char* home = getenv("HOME");
    if (!home) return "";
    std::string dir = std::string(home) + "/.cache";
    mkdir(dir.c_str(), 0755);
    dir += "/spd";
    mkdir(dir.c_str(), 0755);
    return dir + "/batch_schedule.txt";
}

static std::string tune_key(const spd_batch_plan* P)
{
    hipDeviceProp_t prop;
    hipGetDeviceProperties(&prop, P->device);
    char buf[256];
    unsigned h = 2166136261u;
    for (int32_t w : P->widths) h = (h ^ (unsigned)w) * 16777619u;
    snprintf(buf, sizeof buf, "v3|%s|cu%d|dt%d|n%zu|nmax%d|w%08x", prop.gcnArchName, P->cus, P->dtype,
             P->widths.size(), P->widths.back(), h);
    return buf;
}

static bool cache_lookup(const std::string& key, Schedule& sc)
{
    const std::string path = tune_cache_path();
    if (path.empty()) return false;
    FILE* f = fopen(path.c_str(), "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char k[300];
        Schedule s;
        if (sscanf(line, "%299s %d %d %d %d %d", k, &s.X, &s.waves, &s.wgs_per_cu, &s.grab, &s.win) == 6 &&
            key == k) {
            sc = s;
            found = true;
        }
    }
    fclose(f);
    return found;
}

static void cache_store(const std::string& key, const Schedule& sc)
{
    static std::mutex mu;
    std::lock_guard<std::mutex> g(mu);
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    FILE* f = fopen(path.c_str(), "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %d %d\n", key.c_str(), sc.X, sc.waves, sc.wgs_per_cu, sc.grab, sc.win);
    fclose(f);
}

}  // namespace spd

using namespace spd;

static spd_status build_beams(spd_batch_plan* P, const spd_plane* beams)
{
    P->host_beams.resize(P->n_beams);
    int64_t msd = 0, units = 0, tiles[kLayouts] = {0, 0, 0};
    const int nmax = P->widths.back();
    for (int b = 0; b < P->n_beams; ++b) {
        const spd_plane& x = beams[b];
        BeamDesc& d = P->host_beams[b];
        memset(&d, 0, sizeof d);
        d.pl = plane_arg(&x);
        d.vec = plane_vec_ok(&x) ? 1 : 0;
        d.msd_start = msd;
        d.unit_start = units;
        d.nblk = (x.n_cols + kMsdBlockCols - 1) / kMsdBlockCols;
        d.nout = x.n_cols - nmax + 1;
        msd += x.n_rows * d.nblk;
        units += x.n_rows;
    }
    P->msd_items = msd;
    P->units = units;
    for (int k = 0; k < kLayouts; ++k) {
        if (k == 2 && !P->has_win) continue;
        const int X = k ? 8 : 4;
        std::vector<BeamDesc> v = P->host_beams;
        int64_t t = 0;
        for (auto& d : v) {
            const int64_t per = (int64_t)P->max_waves[k] * 64 * X;
            d.tiles_per_row = (d.nout + per - 1) / per;
            d.tile_start = t;
            t += d.pl.n_rows * d.tiles_per_row;
        }
        tiles[k] = t;
        hipError_t e = hipMalloc((void**)&P->d_beams[k], sizeof(BeamDesc) * P->n_beams);
        if (e != hipSuccess) return device_status(e, "hipMalloc(beams)");
        e = hipMemcpy(P->d_beams[k], v.data(), sizeof(BeamDesc) * P->n_beams, hipMemcpyHostToDevice);
        if (e != hipSuccess) return device_status(e, "hipMemcpy(beams)");
    }
    for (int k = 0; k < kLayouts; ++k) P->tiles[k] = tiles[k];
    if (P->units > 0x7fffffffLL || P->msd_items > 0x7fffffffLL)
        return fail(SPD_E_UNSUPPORTED, "batch too large");
    return SPD_OK;
}

// Time candidate schedules of the boxcar kernel on the plan's own data (a
// prefix of its tiles) and keep the fastest.  Tiles are numbered for the
// largest waves-per-group that fits, so only schedules with that wave count
// are timed; the free choices are the outputs per lane, the number of
// persistent work-groups per CU and the queue grab size.
static spd_status tune(spd_batch_plan* P, hipStream_t s)
{
    const std::string key = tune_key(P);
    Schedule best;
    best.X = 8;
    best.waves = P->max_waves[1];
    if (cache_lookup(key, best) && (best.X == 4 || best.X == 8) &&
        schedule_usable(best.X, best.win, best.wgs_per_cu, best.grab, P->has_win, P->tiles[slot(best)],
                        P->max_waves[slot(best)], kMaxGridItems)) {
        best.waves = P->max_waves[slot(best)];
        P->sched = best;
        P->tuned = 2;
        return SPD_OK;
    }
    hipError_t e = launch_fill_i64(P->d_counters, 4, 0, s);
    if (e != hipSuccess) return device_status(e, "tune reset");
    switch (P->dtype) {
    case SPD_F32: e = enqueue_msd<SPD_F32>(P, s); break;
    case SPD_F16: e = enqueue_msd<SPD_F16>(P, s); break;
    default: e = enqueue_msd<SPD_U8>(P, s); break;
    }
    if (e != hipSuccess) return device_status(e, "tune msd");
    hipLaunchKernelGGL(batch_finalize_kernel, dim3((unsigned)P->units), dim3(256), 0, s, P->d_beams[1], P->n_beams,
                       P->d_part, P->d_stats, (int32_t)(P->params.sigma_mode != SPD_SIGMA_SQRTN),
                       (int32_t)P->widths.back(), (int32_t)P->params.sigma_mode, (double)P->params.auto_kappa);
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    float best_ms = 1e30f;
    const int Xs[3] = {4, 8, 0};                      // 0: the register-window form (X = 8, grid launch)
    const int wpc[4] = {0, 2, 4, 6};                  // 0: grid launch, one work-group per tile
    const int grabs[2] = {1, 8};
    P->tune_table.clear();
    for (int xv : Xs)
        for (int w : wpc)
            for (int g : grabs) {
                Schedule sc;
                sc.win = xv == 0 ? 1 : 0;
                sc.X = xv == 0 ? 8 : xv;
                if (sc.win && (!P->has_win || w != 0)) continue;
                const int k = slot(sc);
                if (w == 0 && g != 1) continue;
                if (w == 0 && (uint64_t)P->tiles[k] * 64u * (uint64_t)P->max_waves[k] > kMaxGridItems)
                    continue;                             // one launch cannot hold every tile
                sc.waves = P->max_waves[k];
                sc.wgs_per_cu = w;
                sc.grab = g;
                // the same prefix of the work for every schedule: a few waves of
                // persistent work-groups deep
                const int64_t limit = std::min<int64_t>(P->tiles[k], (int64_t)P->cus * 6 * 8 * 6);
                float ms = 0.f;
                for (int rep = 0; rep < 2; ++rep) {
                    launch_fill_i64(P->d_counters + 1, 2, 0, s);
                    hipEventRecord(e0, s);
                    e = enqueue_boxcar_dt(P, sc, nullptr, 0, P->d_counters + 2, limit, s);
                    hipEventRecord(e1, s);
                    if (e != hipSuccess) break;
                    hipEventSynchronize(e1);
                    hipEventElapsedTime(&ms, e0, e1);
                }
                if (e != hipSuccess) break;
                const int64_t starts_done = limit * (int64_t)sc.waves * 64 * sc.X;
                const float per = ms * 1e6f / (float)starts_done;      // ns per output start
                P->tune_table.push_back({sc, per});
                if (per < best_ms) {
                    best_ms = per;
                    best = sc;
                }
            }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) return device_status(e, "tune boxcar");
    P->sched = best;
    P->tuned = 1;
    P->tune_ms = best_ms;
    cache_store(key, best);
    return SPD_OK;
}

extern "C" {

spd_status spd_batch_plan_create(const spd_plane* beams, int32_t n_beams, const spd_params* p, int32_t autotune,
                                 spd_batch_plan** out)
{
    clear_error();
    spd_status st;
    if (!out) return fail(SPD_E_INVALID, "out is NULL");
    *out = nullptr;
    if ((st = check_params(p))) return st;
    if (!beams || n_beams < 1 || n_beams > kMaxBeams)
        return fail(SPD_E_INVALID, "n_beams=%d outside [1, %d]", n_beams, kMaxBeams);
    if (p->scope != SPD_SCOPE_ROW) return fail(SPD_E_UNSUPPORTED, "batched runs use per-row statistics");
    for (int b = 0; b < n_beams; ++b) {
        if ((st = check_plane(&beams[b], p))) return fail(st, "beam %d: %s", b, spd_last_error());
        if (beams[b].dtype != beams[0].dtype) return fail(SPD_E_INVALID, "beam %d: dtype differs from beam 0", b);
    }
    spd_batch_plan* P = new spd_batch_plan();
    P->n_beams = n_beams;
    P->dtype = beams[0].dtype;
    P->widths.assign(p->widths, p->widths + p->n_widths);
    P->params = *p;
    P->params.widths = P->widths.data();
    hipGetDevice(&P->device);
    hipDeviceProp_t prop;
    hipGetDeviceProperties(&prop, P->device);
    P->cus = prop.multiProcessorCount;
    for (int k = 0; k < 2; ++k) {
        memset(&P->ba[k], 0, sizeof P->ba[k]);
        if (!build_width_plan(&P->params, k ? 8 : 4, P->wp[k], P->ba[k], P->max_waves[k], kBatchLdsReserve)) {
            delete P;
            return fail(SPD_E_UNSUPPORTED, "width list does not fit in LDS");
        }
        P->ba[k].scope = SPD_SCOPE_ROW;
        P->ba[k].threshold = p->threshold;
    }
    memset(&P->ba[2], 0, sizeof P->ba[2]);
    if (build_width_plan(&P->params, kWinX, P->wp[2], P->ba[2], P->max_waves[2], kBatchLdsReserve, true) &&
        P->wp[2].win) {
        P->has_win = true;
        P->ba[2].scope = SPD_SCOPE_ROW;
        P->ba[2].threshold = p->threshold;
    }
    // default schedule: the register-window form where the width list allows it, else strided X = 8;
    // one ordinary launch with one work-group per tile
    P->sched.X = 8;
    P->sched.win = P->has_win ? 1 : 0;
    P->sched.waves = P->max_waves[P->has_win ? 2 : 1];
    P->sched.wgs_per_cu = 0;
    P->sched.grab = 1;
    if ((st = build_beams(P, beams))) { spd_batch_plan_destroy(P); return st; }
    if ((uint64_t)P->tiles[slot(P->sched)] * 64u * (uint64_t)P->sched.waves > kMaxGridItems) {
        P->sched.win = 0;                       // too many tiles for one grid launch: persistent queue
        P->sched.waves = P->max_waves[1];
        P->sched.wgs_per_cu = 4;
        P->sched.grab = 4;
    }
    hipError_t e = hipMalloc((void**)&P->d_part, sizeof(double) * 6 * (size_t)P->msd_items);
    if (e == hipSuccess) e = hipMalloc((void**)&P->d_stats, sizeof(spd_row_stats) * (size_t)P->units);
    if (e == hipSuccess) e = hipMalloc((void**)&P->d_counters, sizeof(int64_t) * 4);
    if (e == hipSuccess) e = hipMemset(P->d_counters, 0, sizeof(int64_t) * 4);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) { spd_batch_plan_destroy(P); return device_status(e, "batch plan allocation"); }
    if (autotune) {
        if ((st = tune(P, P->capture_stream))) { spd_batch_plan_destroy(P); return st; }
        hipStreamSynchronize(P->capture_stream);
    }
    *out = P;
    return SPD_OK;
}

spd_status spd_batch_run(spd_batch_plan* P, spd_candidate* cand, int64_t cand_capacity, int64_t* cand_count,
                         int32_t use_graph, void* stream)
{
    clear_error();
    if (!P) return fail(SPD_E_INVALID, "plan is NULL");
    if (!cand_count || cand_capacity < 0 || (cand_capacity > 0 && !cand))
        return fail(SPD_E_INVALID, "candidate list needs cand (when capacity > 0), cand_count and capacity >= 0");
    hipStream_t s = (hipStream_t)stream;
    if (!use_graph) return device_status(enqueue_run(P, cand, cand_capacity, cand_count, s), "batch run");
    if (!P->exec || P->g_cand != cand || P->g_cap != cand_capacity || P->g_count != cand_count) {
        if (P->exec) { hipGraphExecDestroy(P->exec); P->exec = nullptr; }
        if (P->graph) { hipGraphDestroy(P->graph); P->graph = nullptr; }
        hipError_t e = hipStreamBeginCapture(P->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return device_status(e, "hipStreamBeginCapture");
        hipError_t e2 = enqueue_run(P, cand, cand_capacity, cand_count, P->capture_stream);
        e = hipStreamEndCapture(P->capture_stream, &P->graph);
        if (e2 != hipSuccess) return device_status(e2, "batch capture");
        if (e != hipSuccess) return device_status(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return device_status(e, "hipGraphInstantiate");
        P->g_cand = cand;
        P->g_cap = cand_capacity;
        P->g_count = cand_count;
    }
    return device_status(hipGraphLaunch(P->exec, s), "hipGraphLaunch");
}

spd_status spd_batch_stats(const spd_batch_plan* P, int32_t beam, const spd_row_stats** stats)
{
    clear_error();
    if (!P || !stats) return fail(SPD_E_INVALID, "plan and stats are required");
    if (beam < 0 || beam >= P->n_beams) return fail(SPD_E_INVALID, "beam %d out of range", beam);
    *stats = P->d_stats + P->host_beams[beam].unit_start;
    return SPD_OK;
}

spd_status spd_batch_copy_stats(const spd_batch_plan* P, int32_t beam, spd_row_stats* dst, void* stream)
{
    clear_error();
    if (!P || !dst) return fail(SPD_E_INVALID, "plan and dst are required");
    if (beam < 0 || beam >= P->n_beams) return fail(SPD_E_INVALID, "beam %d out of range", beam);
    const size_t n = (size_t)P->host_beams[beam].pl.n_rows;
    return device_status(hipMemcpyAsync(dst, P->d_stats + P->host_beams[beam].unit_start, n * sizeof(spd_row_stats),
                                        hipMemcpyDeviceToDevice, (hipStream_t)stream),
                         "hipMemcpyAsync(stats)");
}

spd_status spd_batch_describe(const spd_batch_plan* P, spd_batch_info* info)
{
    clear_error();
    if (!P || !info) return fail(SPD_E_INVALID, "plan and info are required");
    info->out_per_lane = P->sched.X;
    info->waves_per_group = P->sched.waves;
    info->groups_per_cu = P->sched.wgs_per_cu;
    info->tiles_per_grab = P->sched.grab;
    info->tuned = P->tuned;
    info->window = P->sched.win;
    info->msd_items = P->msd_items;
    info->tiles = P->tiles[slot(P->sched)];
    info->rows = P->units;
    return SPD_OK;
}

int32_t spd_batch_tune_table(const spd_batch_plan* P, spd_batch_info* rows, float* ns_per_start, int32_t cap)
{
    clear_error();
    if (!P) return 0;
    const int32_t n = (int32_t)P->tune_table.size();
    for (int32_t i = 0; i < n && i < cap; ++i) {
        const Schedule& sc = P->tune_table[i].first;
        spd_batch_info& r = rows[i];
        memset(&r, 0, sizeof r);
        r.out_per_lane = sc.X;
        r.waves_per_group = sc.waves;
        r.groups_per_cu = sc.wgs_per_cu;
        r.tiles_per_grab = sc.grab;
        r.window = sc.win;
        ns_per_start[i] = P->tune_table[i].second;
    }
    return n;
}

void spd_batch_plan_destroy(spd_batch_plan* P)
{
    if (!P) return;
    if (P->exec) hipGraphExecDestroy(P->exec);
    if (P->graph) hipGraphDestroy(P->graph);
    if (P->capture_stream) hipStreamDestroy(P->capture_stream);
    for (int k = 0; k < kLayouts; ++k)
        if (P->d_beams[k]) hipFree(P->d_beams[k]);
    if (P->d_part) hipFree(P->d_part);
    if (P->d_stats) hipFree(P->d_stats);
    if (P->d_counters) hipFree(P->d_counters);
    delete P;
}

}  // extern "C"
