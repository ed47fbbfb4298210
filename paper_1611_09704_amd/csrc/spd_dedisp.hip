// spd_dedisp.hip -- brute-force incoherent de-dispersion, the step before the
// detection path (Sec. 1: detection runs on de-dispersed time series).
//
// A filterbank of 8-bit samples x[c][s] (channel 0 the highest frequency)
// becomes one series per trial DM:
//     y[d][t] = sum over c of x[c][t + delay(d, c)],  t < n_samp - max delay,
// with delay(d, c) = floor(dm[d] * k_c + 0.5) and
// k_c = KDM * (1/f_c^2 - 1/f_top^2) / t_samp, the cold-plasma delay law.  The
// sums are of whole 8-bit counts, so they are exact in every form below and
// the output (float) holds them exactly (below 2^24 for the up to 65,536
// channels a plan accepts).
//
// Kernel layout (gfx950).  A work-group owns 16 consecutive trials x 512
// consecutive starts; each of its 4 waves owns 4 trials, and lane l the
// starts t0 + l + 64k (k < 8).  Channels come in chunks of up to 16, staged
// in LDS relative to g = (t0 + delay of the group's first trial) & ~3:
//  * wide layout (dedisp_u8_wide_kernel, the common case): entry e is 16
//    bytes holding x[g + e + 64k], k < 8, as 16-bit fields, so one 16-byte
//    LDS read gives a lane all 8 of its starts for a trial; the next chunk's
//    bytes are loaded into registers while the current one accumulates;
//  * narrow layout (dedisp_u8_kernel, any span of delays): entry e is 4
//    bytes holding x[g + e] and x[g + e + 64]; staging between barriers.
// Either way one 32-bit integer add accumulates two starts as 16-bit fields,
// flushed into 32-bit totals every 256 channels (256 * 255 < 65536).  Lanes
// read consecutive entries, so the reads are free of bank conflicts.  Each
// 4 bytes read from LDS carry two of the definition's additions, and the LDS
// read bandwidth is the binding resource.
//
// The delays are evaluated where they are used, in FP64, with the product and
// the sum rounded separately (no fused multiply-add), the same way the host
// evaluates them for the plan's maximum delay and span.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "spd_abi_internal.h"

namespace spd {
namespace {

constexpr double kKdm = 4.148808e3;          // MHz^2 pc^-1 cm^3 s
constexpr int kDdWaves = 4;
constexpr int kDdDmPerWave = 4;
constexpr int kDdDms = kDdWaves * kDdDmPerWave;   // trials per work-group
constexpr int kDdOut = 512;                       // starts per work-group
constexpr int kDdFlush = 256;                     // channels per 16-bit partial sum
constexpr int kDdMaxChunk = 16;                   // channels per LDS chunk (<= 256 / kDdDms)
constexpr size_t kDdLdsMax = 65536;

struct DedispArgs {
    const uint8_t* fb;
    int64_t stride, n_samp;
    const double* dm;
    const double* kc;
    float* out;
    int64_t out_stride, n_out;
    int32_t n_chan, n_dm, n_dm_tiles, entries, chunk;
    int32_t groups;          // wide layout: groups of 4 entries staged per channel
    int32_t max_delay;
};

// floor(dm * k + 0.5) with the product and the sum each rounded to FP64.
__host__ __device__ inline int32_t dd_delay(double dm, double k)
{
#pragma clang fp contract(off)
    const double p = dm * k;
    return (int32_t)floor(p + 0.5);
}

// Four bytes of a channel row from byte g on (g a multiple of 4); bytes at or
// beyond n_samp read as zero.
__device__ inline uint32_t dd_load4(const uint8_t* row, int64_t g, int64_t n_samp)
{
    if (g + 3 < n_samp) return *(const uint32_t*)(row + g);
    uint32_t v = 0;
    for (int i = 0; i < 4; ++i)
        if (g + i < n_samp) v |= (uint32_t)row[g + i] << (8 * i);
    return v;
}

// The chunk's accumulation: for each staged channel, the wave's 4 trials x
// 4 entries per lane, all 16 reads in flight before the adds.  my_off (lane
// cc < ncc) is channel cc's entry offset, my_dl (lane 4cc + j) trial j's
// delay minus the group's first trial's; both are read as scalars.
__device__ inline void dd_accumulate(const uint32_t* P, int ncc, int32_t my_off, int32_t my_dl, int lane,
                                     uint32_t (&part)[kDdDmPerWave][4])
{
    for (int cc = 0; cc < ncc; ++cc) {
        const int32_t off_c = __builtin_amdgcn_readlane(my_off, cc);
        uint32_t v[kDdDmPerWave][4];
#pragma unroll
        for (int j = 0; j < kDdDmPerWave; ++j) {
            const uint32_t* q = P + off_c + __builtin_amdgcn_readlane(my_dl, cc * kDdDmPerWave + j) + lane;
#pragma unroll
            for (int i = 0; i < 4; ++i) v[j][i] = q[128 * i];
        }
#pragma unroll
        for (int j = 0; j < kDdDmPerWave; ++j) {
#pragma unroll
            for (int i = 0; i < 4; ++i) part[j][i] += v[j][i];
        }
    }
}

// The 16-bit partial sums (fields: starts t and t + 64) into the 32-bit totals.
__device__ inline void dd_flush(uint32_t (&part)[kDdDmPerWave][4], uint32_t (&tot)[kDdDmPerWave][8])
{
#pragma unroll
    for (int j = 0; j < kDdDmPerWave; ++j) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            tot[j][2 * i] += part[j][i] & 0xffffu;
            tot[j][2 * i + 1] += part[j][i] >> 16;
            part[j][i] = 0;
        }
    }
}

__device__ inline void dd_store(const DedispArgs& a, int d0, int wv, int lane, int64_t t0,
                                const uint32_t (&tot)[kDdDmPerWave][8])
{
#pragma unroll
    for (int j = 0; j < kDdDmPerWave; ++j) {
        const int d = d0 + wv * kDdDmPerWave + j;
        if (d >= a.n_dm) continue;
        float* orow = a.out + (int64_t)d * a.out_stride;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t t = t0 + lane + 64 * k;
            if (t < a.n_out) orow[t] = (float)tot[j][k];
        }
    }
}

// Entries 4q..4q+3 of a channel from the bytes A = x[g..g+3], B = x[g+64..g+67].
__device__ inline uint4 dd_pack(uint32_t A, uint32_t B)
{
    uint4 v;
    v.x = (A & 0xffu) | ((B & 0xffu) << 16);
    v.y = ((A >> 8) & 0xffu) | (((B >> 8) & 0xffu) << 16);
    v.z = ((A >> 16) & 0xffu) | (((B >> 16) & 0xffu) << 16);
    v.w = (A >> 24) | ((B >> 24) << 16);
    return v;
}

// Any chunk size and span: delays through LDS, staging between barriers.
__global__ __launch_bounds__(64 * kDdWaves) void dedisp_u8_kernel(DedispArgs a)
{
    extern __shared__ __align__(16) uint32_t dd_smem[];
    uint32_t* P = dd_smem;                                   // [chunk][entries]
    int32_t* dl = (int32_t*)(P + a.chunk * a.entries);       // [chunk][16] delay - first trial's delay
    int32_t* base = dl + a.chunk * kDdDms;                   // [chunk] first trial's delay
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t t0 = (int64_t)(blockIdx.x / (uint32_t)a.n_dm_tiles) * kDdOut;
    const int d0 = (int)(blockIdx.x % (uint32_t)a.n_dm_tiles) * kDdDms;

    uint32_t part[kDdDmPerWave][4] = {};
    uint32_t tot[kDdDmPerWave][8] = {};
    int since = 0;
    const int nq = a.entries / 4;
    for (int c0 = 0; c0 < a.n_chan; c0 += a.chunk) {
        const int ncc = min(a.chunk, a.n_chan - c0);
        __syncthreads();                                     // the previous chunk is consumed
        if (tid < ncc * kDdDms) {
            const int cc = tid / kDdDms, j = tid % kDdDms;
            const double k = a.kc[c0 + cc];
            const int32_t db = dd_delay(a.dm[d0], k);
            dl[tid] = dd_delay(a.dm[min(d0 + j, a.n_dm - 1)], k) - db;
            if (j == 0) base[cc] = db;
        }
        __syncthreads();
        // wave w stages channels w, w + 4, ...; lane l the entries 4q..4q+3, q = l, l + 64, ...
        for (int cc = wv; cc < ncc; cc += kDdWaves) {
            const uint8_t* row = a.fb + (int64_t)(c0 + cc) * a.stride;
            const int64_t g0 = (t0 + base[cc]) & ~(int64_t)3;
            uint32_t* pc = P + cc * a.entries;
            for (int q = lane; q < nq; q += 64)
                *(uint4*)(pc + 4 * q) = dd_pack(dd_load4(row, g0 + 4 * q, a.n_samp),
                                               dd_load4(row, g0 + 4 * q + 64, a.n_samp));
        }
        __syncthreads();
        const int32_t my_dl = (lane >> 2) < ncc ? dl[(lane >> 2) * kDdDms + wv * kDdDmPerWave + (lane & 3)] : 0;
        const int32_t my_off = lane < ncc ? lane * a.entries + (int)((t0 + base[lane]) & 3) : 0;
        dd_accumulate(P, ncc, my_off, my_dl, lane, part);
        since += ncc;
        if (since + a.chunk > kDdFlush || c0 + a.chunk >= a.n_chan) {
            dd_flush(part, tot);
            since = 0;
        }
    }
    dd_store(a, d0, wv, lane, t0, tot);
}

// ---------------------------------------------------------------------------
// Wide layout: entry e of a channel is 16 bytes holding x[g + e + 64k] for
// k < 8 as 16-bit fields (k = 2p, 2p+1 in dword p), so one 16-byte LDS read
// gives a lane all 8 of its starts for a trial, and the 4 dwords add into
// the same partial sums as above.  A channel needs 67 + span entries.
// ---------------------------------------------------------------------------
constexpr int kWideRounds = 2;              // staging items per thread per chunk (prefetching kernel)

// Entries 4m..4m+3 of a channel (dst = entry 4m) from D[k] = x[g + 4m + 64k
// .. +3], k < 8.  Entry 4m + b, dword p, is byte b of D[2p] | byte b of
// D[2p+1] << 16: one v_perm_b32 (selector bytes 0-3 pick from its second
// operand, 4-7 from its first, 0x0c gives zero).  The four 16-byte writes go
// out in the order b = (i + item/4) mod 4, i = 0..3, so that in each write
// instruction 16 consecutive items (lanes) hit 16 different 16-byte bank
// groups instead of four.
__device__ inline void dd_pack_wide(const uint32_t (&D)[8], int item, uint4* dst)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t b = (uint32_t)(i + (item >> 2)) & 3u;
        const uint32_t sel = 0x0c040c00u + b * 0x00010001u;
        dst[b] = make_uint4(__builtin_amdgcn_perm(D[1], D[0], sel), __builtin_amdgcn_perm(D[3], D[2], sel),
                            __builtin_amdgcn_perm(D[5], D[4], sel), __builtin_amdgcn_perm(D[7], D[6], sel));
    }
}

__device__ inline void dd_load_group(const uint8_t* row, int64_t g, int64_t n_samp, bool interior, uint32_t (&D)[8])
{
    if (interior) {
#pragma unroll
        for (int k = 0; k < 8; ++k) D[k] = *(const uint32_t*)(row + g + 64 * k);
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) D[k] = dd_load4(row, g + 64 * k, n_samp);
    }
}

__device__ inline void dd_accumulate_wide(const uint4* P4, int ncc, int32_t my_off, int32_t my_dl, int lane,
                                          uint32_t (&part)[kDdDmPerWave][4])
{
    for (int cc = 0; cc < ncc; ++cc) {
        const int32_t off_c = __builtin_amdgcn_readlane(my_off, cc);
        uint4 v[kDdDmPerWave];
#pragma unroll
        for (int j = 0; j < kDdDmPerWave; ++j)
            v[j] = P4[off_c + __builtin_amdgcn_readlane(my_dl, cc * kDdDmPerWave + j) + lane];
#pragma unroll
        for (int j = 0; j < kDdDmPerWave; ++j) {
            part[j][0] += v[j].x;
            part[j][1] += v[j].y;
            part[j][2] += v[j].z;
            part[j][3] += v[j].w;
        }
    }
}

// Wide layout, next chunk prefetched into registers (16-channel chunks, at
// most 2 * 256 staging groups per chunk).
__global__ __launch_bounds__(64 * kDdWaves) void dedisp_u8_wide_kernel(DedispArgs a)
{
    extern __shared__ __align__(16) uint32_t dd_smem[];
    uint4* P4 = (uint4*)dd_smem;                             // [16][4 * groups]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t t0 = (int64_t)(blockIdx.x / (uint32_t)a.n_dm_tiles) * kDdOut;
    const int d0 = (int)(blockIdx.x % (uint32_t)a.n_dm_tiles) * kDdDms;
    const int G = a.groups, E4 = 4 * a.groups;
    const double dm0 = a.dm[d0];
    const double dmj = a.dm[min(d0 + wv * kDdDmPerWave + (lane & 3), a.n_dm - 1)];
    // every byte this group stages lies inside the rows (the last tiles take the checked loads)
    const bool interior = t0 + a.max_delay + 4 * G + 64 * 8 <= a.n_samp;

    uint32_t D[kWideRounds][8];
    auto fetch = [&](int c0) {
#pragma unroll
        for (int r = 0; r < kWideRounds; ++r) {
            const int item = min(tid + 64 * kDdWaves * r, kDdMaxChunk * G - 1);
            const int cc = item / G, m = item - cc * G;
            const int c = min(c0 + cc, a.n_chan - 1);
            const int64_t g = ((t0 + dd_delay(dm0, a.kc[c])) & ~(int64_t)3) + 4 * m;
            dd_load_group(a.fb + (int64_t)c * a.stride, g, a.n_samp, interior, D[r]);
        }
    };
    auto store = [&](int ncc) {
#pragma unroll
        for (int r = 0; r < kWideRounds; ++r) {
            const int item = tid + 64 * kDdWaves * r;
            const int cc = item / G, m = item - cc * G;
            if (cc < ncc) dd_pack_wide(D[r], item, P4 + cc * E4 + 4 * m);
        }
    };

    uint32_t part[kDdDmPerWave][4] = {};
    uint32_t tot[kDdDmPerWave][8] = {};
    int since = 0;
    fetch(0);
    store(min(kDdMaxChunk, a.n_chan));
    __syncthreads();
    for (int c0 = 0; c0 < a.n_chan; c0 += kDdMaxChunk) {
        const int ncc = min(kDdMaxChunk, a.n_chan - c0);
        const double kd = a.kc[min(c0 + (lane >> 2), a.n_chan - 1)];
        const double ko = a.kc[min(c0 + lane, a.n_chan - 1)];
        const int32_t my_dl = dd_delay(dmj, kd) - dd_delay(dm0, kd);
        const int32_t my_off = lane * E4 + (int)((t0 + dd_delay(dm0, ko)) & 3);
        const bool more = c0 + kDdMaxChunk < a.n_chan;
        if (more) fetch(c0 + kDdMaxChunk);
        dd_accumulate_wide(P4, ncc, my_off, my_dl, lane, part);
        since += ncc;
        if (since + kDdMaxChunk > kDdFlush || !more) {
            dd_flush(part, tot);
            since = 0;
        }
        if (more) {
            __syncthreads();
            store(min(kDdMaxChunk, a.n_chan - c0 - kDdMaxChunk));
            __syncthreads();
        }
    }
    dd_store(a, d0, wv, lane, t0, tot);
}

// SPD_DEDISP_FORM=generic selects the chunk-by-chunk kernel for any plan (the
// two kernels give identical sums).
bool dd_force_generic()
{
    const char* e = getenv("SPD_DEDISP_FORM");
    return e && strcmp(e, "generic") == 0;
}

}  // namespace
}  // namespace spd

using namespace spd;

struct spd_dedisp_plan {
    spd_band band;
    int32_t n_dm;
    std::vector<double> dm, kc;
    double* d_dm = nullptr;
    double* d_kc = nullptr;
    int32_t max_delay = 0, span = 0, entries = 0, chunk = 0, groups = 0;
    int device = 0;
};

extern "C" {

}  // extern "C"

namespace {

// Validation shared by the plan and the host delay table; fills k_c.
spd_status dd_prepare(const spd_band* band, const double* dm, int32_t n_dm, std::vector<double>& kc,
                      int32_t* max_delay)
{
    if (!band || !dm) return fail(SPD_E_INVALID, "band and dm are required");
    const spd_band b = *band;
    if (b.n_chan < 1 || b.n_chan > SPD_MAX_CHANNELS) return fail(SPD_E_INVALID, "n_chan must lie in [1, %d]", SPD_MAX_CHANNELS);
    if (!(b.f_top_mhz > 0.0) || !(b.chan_bw_mhz > 0.0) || !(b.t_samp_s > 0.0) || !isfinite(b.f_top_mhz) ||
        !isfinite(b.chan_bw_mhz) || !isfinite(b.t_samp_s))
        return fail(SPD_E_INVALID, "f_top_mhz, chan_bw_mhz and t_samp_s must be finite and > 0");
    if (!(b.f_top_mhz - (double)(b.n_chan - 1) * b.chan_bw_mhz > 0.0))
        return fail(SPD_E_INVALID, "the lowest channel frequency must be > 0");
    if (n_dm < 1 || n_dm > SPD_MAX_DM_TRIALS) return fail(SPD_E_INVALID, "n_dm must lie in [1, %d]", SPD_MAX_DM_TRIALS);
    for (int32_t d = 0; d < n_dm; ++d) {
        if (!isfinite(dm[d]) || dm[d] < 0.0) return fail(SPD_E_INVALID, "dm[%d] must be finite and >= 0", d);
        if (d && dm[d] < dm[d - 1]) return fail(SPD_E_INVALID, "dm must be non-decreasing (dm[%d] < dm[%d])", d, d - 1);
    }
    kc.resize(b.n_chan);
    for (int32_t c = 0; c < b.n_chan; ++c) {
        const double f = b.f_top_mhz - (double)c * b.chan_bw_mhz, ft = b.f_top_mhz;
        kc[c] = kKdm * (1.0 / (f * f) - 1.0 / (ft * ft)) / b.t_samp_s;
    }
    // the delays grow with the trial and towards the last channel
    const double p = dm[n_dm - 1] * kc[b.n_chan - 1];
    if (!(p < (double)SPD_MAX_DELAY)) return fail(SPD_E_UNSUPPORTED, "largest delay exceeds %d samples", SPD_MAX_DELAY);
    *max_delay = dd_delay(dm[n_dm - 1], kc[b.n_chan - 1]);
    return SPD_OK;
}

}  // namespace

extern "C" {

spd_status spd_dedisp_delay_table(const spd_band* band, const double* dm, int32_t n_dm, int32_t* delays,
                                  int32_t* max_delay)
{
    clear_error();
    std::vector<double> kc;
    int32_t md = 0;
    spd_status st = dd_prepare(band, dm, n_dm, kc, &md);
    if (st) return st;
    if (max_delay) *max_delay = md;
    if (delays)
        for (int32_t d = 0; d < n_dm; ++d)
            for (int32_t c = 0; c < band->n_chan; ++c) delays[(int64_t)d * band->n_chan + c] = dd_delay(dm[d], kc[c]);
    return SPD_OK;
}

spd_status spd_dedisp_plan_create(const spd_band* band, const double* dm, int32_t n_dm, spd_dedisp_plan** plan)
{
    clear_error();
    if (!plan) return fail(SPD_E_INVALID, "plan is required");
    *plan = nullptr;
    std::vector<double> kc;
    int32_t md = 0;
    spd_status st = dd_prepare(band, dm, n_dm, kc, &md);
    if (st) return st;
    spd_dedisp_plan* P = new (std::nothrow) spd_dedisp_plan;
    if (!P) return fail(SPD_E_NOMEM, "host allocation");
    const spd_band b = *band;
    P->band = b;
    P->n_dm = n_dm;
    P->dm.assign(dm, dm + n_dm);
    P->kc = kc;
    P->max_delay = md;
    int32_t span = 0;
    for (int32_t d0 = 0; d0 < n_dm; d0 += kDdDms) {
        const int32_t d1 = d0 + kDdDms - 1 < n_dm - 1 ? d0 + kDdDms - 1 : n_dm - 1;
        for (int32_t c = 0; c < b.n_chan; ++c) {
            const int32_t s = dd_delay(P->dm[d1], P->kc[c]) - dd_delay(P->dm[d0], P->kc[c]);
            span = s > span ? s : span;
        }
    }
    P->span = span;
    // entries per channel: the largest index read is 3 + 63 + 384 + span
    P->entries = (451 + span + 3) & ~3;
    const size_t per_chan = (size_t)P->entries * 4 + kDdDms * 4 + 4;
    P->chunk = 0;
    for (int cc = kDdMaxChunk; cc >= 1; cc >>= 1)
        if ((size_t)cc * per_chan <= kDdLdsMax) { P->chunk = cc; break; }
    // wide layout: the largest entry read is 3 + 63 + span
    P->groups = (67 + span + 3) / 4;
    if (!P->chunk) {
        delete P;
        return fail(SPD_E_UNSUPPORTED, "trials 16 apart differ by %d samples of delay; at most about %d fit the LDS",
                    span, (int)(kDdLdsMax / 4) - 460);
    }
    hipError_t e = hipGetDevice(&P->device);
    if (e == hipSuccess) e = hipMalloc((void**)&P->d_dm, sizeof(double) * n_dm);
    if (e == hipSuccess) e = hipMalloc((void**)&P->d_kc, sizeof(double) * b.n_chan);
    if (e == hipSuccess) e = hipMemcpy(P->d_dm, P->dm.data(), sizeof(double) * n_dm, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(P->d_kc, P->kc.data(), sizeof(double) * b.n_chan, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (P->d_dm) (void)hipFree(P->d_dm);
        if (P->d_kc) (void)hipFree(P->d_kc);
        delete P;
        return device_status(e, "de-dispersion plan tables");
    }
    *plan = P;
    return SPD_OK;
}

}  // extern "C"

namespace spd {

void dedisp_plan_shape(const spd_dedisp_plan* plan, int32_t* n_chan, int32_t* n_dm, int32_t* max_delay, int* device)
{
    *n_chan = plan->band.n_chan;
    *n_dm = plan->n_dm;
    *max_delay = plan->max_delay;
    *device = plan->device;
}

}  // namespace spd

extern "C" {

void spd_dedisp_plan_destroy(spd_dedisp_plan* plan)
{
    if (!plan) return;
    if (plan->d_dm) (void)hipFree(plan->d_dm);
    if (plan->d_kc) (void)hipFree(plan->d_kc);
    delete plan;
}

spd_status spd_dedisp_describe(const spd_dedisp_plan* plan, int32_t* max_delay, int32_t* span16)
{
    clear_error();
    if (!plan) return fail(SPD_E_INVALID, "plan is required");
    if (max_delay) *max_delay = plan->max_delay;
    if (span16) *span16 = plan->span;
    return SPD_OK;
}

spd_status spd_dedisp_delays(const spd_dedisp_plan* plan, int32_t* delays)
{
    clear_error();
    if (!plan || !delays) return fail(SPD_E_INVALID, "plan and delays are required");
    const int32_t C = plan->band.n_chan;
    for (int32_t d = 0; d < plan->n_dm; ++d)
        for (int32_t c = 0; c < C; ++c) delays[(int64_t)d * C + c] = dd_delay(plan->dm[d], plan->kc[c]);
    return SPD_OK;
}

spd_status spd_dedisperse(const spd_dedisp_plan* plan, const spd_plane* fb, float* out, int64_t out_stride,
                          void* stream)
{
    clear_error();
    if (!plan || !fb || !out) return fail(SPD_E_INVALID, "plan, fb and out are required");
    if (!fb->data) return fail(SPD_E_INVALID, "fb->data is NULL");
    if (fb->dtype != SPD_U8) return fail(SPD_E_UNSUPPORTED, "de-dispersion takes 8-bit filterbanks (SPD_U8)");
    if (fb->row_scale || fb->row_zero) return fail(SPD_E_INVALID, "de-dispersion sums raw counts: no scale or zero");
    if (fb->n_rows != plan->band.n_chan) return fail(SPD_E_INVALID, "fb has %lld rows, the plan %d channels",
                                                     (long long)fb->n_rows, plan->band.n_chan);
    if (fb->row_stride < fb->n_cols || fb->row_stride % 4 != 0 || ((uintptr_t)fb->data & 3))
        return fail(SPD_E_INVALID, "fb rows must be 4-byte aligned: data and row_stride (>= n_cols) multiples of 4");
    const int64_t n_out = fb->n_cols - plan->max_delay;
    if (n_out < 1) return fail(SPD_E_INVALID, "n_cols %lld must exceed the largest delay %d", (long long)fb->n_cols,
                               plan->max_delay);
    if (out_stride < n_out) return fail(SPD_E_INVALID, "out_stride < n_out (%lld)", (long long)n_out);
    int dev = 0;
    hipError_t ge = hipGetDevice(&dev);
    if (ge != hipSuccess) return device_status(ge, "hipGetDevice");
    if (dev != plan->device) return fail(SPD_E_INVALID, "the plan was made on device %d, not %d", plan->device, dev);
    const int64_t n_dm_tiles = (plan->n_dm + kDdDms - 1) / kDdDms;
    const int64_t n_t_tiles = (n_out + kDdOut - 1) / kDdOut;
    if ((uint64_t)(n_dm_tiles * n_t_tiles) * 64 * kDdWaves > kMaxGridItems)
        return fail(SPD_E_UNSUPPORTED, "output too large for one launch");
    DedispArgs a;
    memset(&a, 0, sizeof a);
    a.fb = (const uint8_t*)fb->data;
    a.stride = fb->row_stride;
    a.n_samp = fb->n_cols;
    a.dm = plan->d_dm;
    a.kc = plan->d_kc;
    a.out = out;
    a.out_stride = out_stride;
    a.n_out = n_out;
    a.n_chan = plan->band.n_chan;
    a.n_dm = plan->n_dm;
    a.n_dm_tiles = (int32_t)n_dm_tiles;
    a.entries = plan->entries;
    a.chunk = plan->chunk;
    a.groups = plan->groups;
    a.max_delay = plan->max_delay;
    const dim3 grid((uint32_t)(n_dm_tiles * n_t_tiles));
    const size_t wide_lds = (size_t)kDdMaxChunk * plan->groups * 64;
    if (!dd_force_generic() && kDdMaxChunk * plan->groups <= 64 * kDdWaves * kWideRounds && wide_lds <= kDdLdsMax)
        hipLaunchKernelGGL(dedisp_u8_wide_kernel, grid, dim3(64 * kDdWaves), wide_lds, (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL(dedisp_u8_kernel, grid, dim3(64 * kDdWaves),
                           (size_t)plan->chunk * ((size_t)plan->entries * 4 + kDdDms * 4 + 4), (hipStream_t)stream, a);
    return device_status(hipGetLastError(), "de-dispersion launch");
}

}  // extern "C"
