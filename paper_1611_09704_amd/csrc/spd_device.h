// spd_device.h -- device building blocks of the detection path, shared by the
// one-plane kernels (spd_kernels.hip) and the persistent batched kernels
// (spd_batch.hip).  Library-internal.
//
//   msd_block_x / msd_block_xy   per-(row, column block) partials, Sec. 2.1
//   finalize_unit                FP64 merge across blocks, sigma_N, Sec. 2.1-2.2
//   boxcar_tile                  boxcars, SNR, highest SNR and its first width,
//                                fused threshold; Sec. 2.3 / Algorithm 1, Sec. 2.4
//   boxcar_tile_win              the same for width lists of stepped groups,
//                                with each group's LDS reads held in registers
//
// The path is a streaming reduction plus a sliding-window scan: no dense
// contraction, so everything is vector ALU and LDS work.  Loads are coalesced
// along time, the contiguous axis.
#pragma once

#include <type_traits>

#include "spd_internal.h"

namespace spd {

// The dispatcher hands work-group i to XCD (i mod 8).  Renumber so that each
// XCD receives one contiguous range of logical blocks: neighbouring time tiles
// of a row, whose halos overlap, then share an L2.
__device__ __forceinline__ uint64_t xcd_remap(uint64_t bid, uint64_t nb)
{
    const uint64_t nx = 8;
    uint64_t xcd = bid % nx, local = bid / nx;
    uint64_t per = nb / nx, extra = nb % nx;
    uint64_t start = xcd * per + (xcd < extra ? xcd : extra);
    return start + local;
}

// ---------------------------------------------------------------------------
// element loaders (Sec. 2: the plane of de-dispersed time series)
// ---------------------------------------------------------------------------

template <int DT> struct Loader;

template <> struct Loader<SPD_F32> {
    const float* row;
    __device__ Loader(const PlaneArg& p, int64_t r) : row((const float*)p.data + r * p.stride) {}
    __device__ __forceinline__ float at(int64_t c) const { return row[c]; }
    __device__ __forceinline__ float4 vec(int64_t c) const { return *(const float4*)(row + c); }
    __device__ __forceinline__ int mis4() const { return (int)(((uintptr_t)row / sizeof(*row)) & 3); }
};

template <> struct Loader<SPD_F16> {
    const __half* row;
    __device__ Loader(const PlaneArg& p, int64_t r) : row((const __half*)p.data + r * p.stride) {}
    __device__ __forceinline__ float at(int64_t c) const { return __half2float(row[c]); }
    __device__ __forceinline__ float4 vec(int64_t c) const {
        uint2 u = *(const uint2*)(row + c);
        __half2 h0 = *reinterpret_cast<__half2*>(&u.x), h1 = *reinterpret_cast<__half2*>(&u.y);
        float2 a = __half22float2(h0), b = __half22float2(h1);
        return make_float4(a.x, a.y, b.x, b.y);
    }
    __device__ __forceinline__ int mis4() const { return (int)(((uintptr_t)row / sizeof(*row)) & 3); }
};

// x = scale_r * (q - zero_r), evaluated in FP32.
template <> struct Loader<SPD_U8> {
    const uint8_t* row;
    float sc, z;
    __device__ Loader(const PlaneArg& p, int64_t r)
        : row((const uint8_t*)p.data + r * p.stride), sc(p.scale[r]), z(p.zero[r]) {}
    __device__ __forceinline__ float deq(uint32_t q) const { return sc * ((float)q - z); }
    __device__ __forceinline__ float at(int64_t c) const { return deq(row[c]); }
    __device__ __forceinline__ float4 vec(int64_t c) const {
        uint32_t u = *(const uint32_t*)(row + c);
        return make_float4(deq(u & 255u), deq((u >> 8) & 255u), deq((u >> 16) & 255u), deq(u >> 24));
    }
    __device__ __forceinline__ int mis4() const { return (int)((uintptr_t)row & 3); }
};

// Four consecutive samples from column c, all inside the row.  `vec`
// (uniform) says the row start is aligned for vector loads.
template <int DT>
__device__ __forceinline__ float4 load4(const Loader<DT>& ld, int64_t c, bool vec)
{
    if (vec) return ld.vec(c);
    return make_float4(ld.at(c), ld.at(c + 1), ld.at(c + 2), ld.at(c + 3));
}

// Four samples from column c minus `shift`, with zero past the end of the row.
template <int DT>
__device__ __forceinline__ float4 load4_shifted(const Loader<DT>& ld, int64_t c, int64_t ncols, bool vec,
                                                float shift_hi, float shift_lo)
{
    float4 v;
    if (c + 3 < ncols) {
        v = load4<DT>(ld, c, vec);
        v.x = (v.x - shift_hi) - shift_lo;
        v.y = (v.y - shift_hi) - shift_lo;
        v.z = (v.z - shift_hi) - shift_lo;
        v.w = (v.w - shift_hi) - shift_lo;
    } else {
        v.x = c < ncols ? (ld.at(c) - shift_hi) - shift_lo : 0.f;
        v.y = c + 1 < ncols ? (ld.at(c + 1) - shift_hi) - shift_lo : 0.f;
        v.z = c + 2 < ncols ? (ld.at(c + 2) - shift_hi) - shift_lo : 0.f;
        v.w = c + 3 < ncols ? (ld.at(c + 3) - shift_hi) - shift_lo : 0.f;
    }
    return v;
}

// Eq. (sd02)/(sd03): a width contributes SNR 0 unless sigma_w is positive
// beyond rounding, i.e. above 1e-9 * sqrt(w) * sigma.  The anchored linear form
// reaches zero at w = Nmax when sigma_Nmax = 0 (one valid start, or a row whose
// Nmax-boxcar is constant), and its rounding residual there has either sign.
__device__ __forceinline__ bool sigma_w_positive(double sw, double w, double sigma)
{
    return sw > 1e-9 * sqrt(w) * sigma;
}

// ---------------------------------------------------------------------------
// Sec. 2.1: streaming and pairwise mean / deviation in FP32 inside a block
// ---------------------------------------------------------------------------

struct Msd { float n, T, S; };

// Eq. (MSD04): merge the partial of samples 1..m (a) with m+1..m+n (b).
// m/(n(m+n)) * (n/m*T_a - T_b)^2 is evaluated as (n*T_a - m*T_b)^2/(m*n*(m+n)).
__device__ __forceinline__ Msd msd_merge(Msd a, Msd b)
{
    if (a.n == 0.f) return b;
    if (b.n == 0.f) return a;
    float d = b.n * a.T - a.n * b.T;
    Msd o;
    o.n = a.n + b.n;
    o.T = a.T + b.T;
    o.S = a.S + b.S + d * d / (a.n * b.n * o.n);
    return o;
}

// Eq. (MSD03) for one more sample x_j: T_j = T_{j-1} + x_j,
// S_j = S_{j-1} + (j*x_j - T_j)^2 / (j(j-1)).
__device__ __forceinline__ void msd_add1(Msd& s, float x)
{
    s.n += 1.f;
    s.T += x;
    if (s.n > 1.f) {
        float d = s.n * x - s.T;
        s.S += d * d / (s.n * (s.n - 1.f));
    }
}

// Four consecutive samples: Eq. (MSD03) over them with j = 1..4 (constant
// coefficients 1/2, 1/6, 1/12), then Eq. (MSD04) into the running partial.
__device__ __forceinline__ void msd_add4(Msd& s, float a, float b, float c, float d)
{
    float T2 = a + b, e2 = 2.f * b - T2;
    float T3 = T2 + c, e3 = 3.f * c - T3;
    float T4 = T3 + d, e4 = 4.f * d - T4;
    float S4 = e2 * e2 * 0.5f + e3 * e3 * (1.f / 6.f) + e4 * e4 * (1.f / 12.f);
    float dd = 4.f * s.T - s.n * T4;
    float inc = s.n > 0.f ? dd * dd * __builtin_amdgcn_rcpf(s.n * 4.f * (s.n + 4.f)) : 0.f;
    s.S = s.S + S4 + inc;
    s.T += T4;
    s.n += 4.f;
}

// Sixteen samples (any order) as one mini-batch: their sum and the sum of
// squared deviations from their own mean, both from registers, then Eq. (MSD04)
// with the batch as the second part.  About 4 VALU per sample against ~7 for
// Eq. (MSD03) four samples at a time.
__device__ __forceinline__ void msd_add16(Msd& s, const float (&v)[16])
{
    float h[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) h[j] = v[2 * j] + v[2 * j + 1];
    const float T16 = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7]));
    const float m = T16 * 0.0625f;
    float S16 = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const float d = v[j] - m;
        S16 = fmaf(d, d, S16);
    }
    const float dd = 16.f * s.T - s.n * T16;
    const float inc = s.n > 0.f ? dd * dd * __builtin_amdgcn_rcpf(s.n * 16.f * (s.n + 16.f)) : 0.f;
    s.S = s.S + S16 + inc;
    s.T += T16;
    s.n += 16.f;
}

// Samples of a four-sample group that fall inside [lo, hi): the whole group in
// one mini-batch when possible, one sample at a time at the edges.
__device__ __forceinline__ void msd_add4_clipped(Msd& s, float4 v, int64_t c, int64_t lo, int64_t hi)
{
    if (c >= lo && c + 3 < hi) {
        msd_add4(s, v.x, v.y, v.z, v.w);
    } else if (c + 3 >= lo && c < hi) {
        const float vv[4] = {v.x, v.y, v.z, v.w};
        for (int j = 0; j < 4; ++j)
            if (c + j >= lo && c + j < hi) msd_add1(s, vv[j]);
    }
}

__device__ __forceinline__ Msd wave_merge(Msd v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        Msd o{__shfl_xor(v.n, off), __shfl_xor(v.T, off), __shfl_xor(v.S, off)};
        v = (lane & off) ? msd_merge(o, v) : msd_merge(v, o);   // lower lanes first
    }
    return v;
}

// Merge every thread's partial; the result is valid in thread 0 (fixed order:
// lanes, then waves).
__device__ __forceinline__ Msd block_merge(Msd v, Msd* scratch)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_merge(v);
    __syncthreads();
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    Msd acc{0.f, 0.f, 0.f};
    if (threadIdx.x == 0)
        for (int w = 0; w < nw; ++w) acc = msd_merge(acc, scratch[w]);
    return acc;
}

// Shared-memory scratch of the MSD block functions.
struct MsdScratch {
    Msd part[16];
    float shift[16];
    unsigned long long isum[4][16];        // U8: per-wave integer sums; the pilot's closest sample
    double dsum[4][16];                    // per-wave FP64 sums
};

// Shift applied before the FP32 reduction: among the row's first (up to)
// block-size samples, the one closest to their mean (the first such on a
// tie).  Shifted samples -- and the widest-boxcar series built from them --
// then have a mean small against their spread, and a constant row shifts to
// exact zeros.  Any constant gives the same statistics in exact arithmetic; T
// is shifted back in FP64.
template <int DT>
__device__ float pilot_shift(const Loader<DT>& ld, int64_t ncols, MsdScratch& sh)
{
    const int tid = threadIdx.x, nw = blockDim.x >> 6;
    const int64_t n = ncols < (int64_t)blockDim.x ? ncols : (int64_t)blockDim.x;
    const float x = tid < n ? ld.at(tid) : 0.f;
    float v = x;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((tid & 63) == 0) sh.shift[tid >> 6] = v;
    __syncthreads();
    float sum = 0.f;
    for (int w = 0; w < nw; ++w) sum += sh.shift[w];
    const float m = sum / (float)n;
    // key: |x - m| (a non-negative float orders as its bits), then the index
    unsigned long long key = tid < n ? ((unsigned long long)__float_as_uint(fabsf(x - m)) << 32) | (unsigned)tid
                                     : ~0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(key, off);
        key = o < key ? o : key;
    }
    if ((tid & 63) == 0) sh.isum[0][tid >> 6] = key;
    __syncthreads();
    unsigned long long best = sh.isum[0][0];
    for (int w = 1; w < nw; ++w) best = sh.isum[0][w] < best ? sh.isum[0][w] : best;
    __syncthreads();                                    // isum is reused by the caller
    return ld.at((int64_t)(best & 0xffffffffu));
}

// ---------------------------------------------------------------------------
// Sec. 2.1 on U8 planes: exact integer sums in the stored domain
// ---------------------------------------------------------------------------
//
// x = s*(q - z) is affine in the stored byte q, so a block's count, sum and
// sum of squared deviations follow exactly from the integer sums Sum q and
// Sum q^2: T_x = s*(Sum q - n*z) and S_x = s^2*(n*Sum q^2 - (Sum q)^2)/n.
// Four bytes take one v_sad_u8 (their sum) and one v_dot4_u32_u8 (their
// squares' sum); the widest boxcar's values y are integer window sums (exact
// prefix differences), their squares accumulated in 64 bits.

__device__ __forceinline__ void u8_word(uint32_t w, uint32_t& s1, uint32_t& s2)
{
    s1 = __builtin_amdgcn_sad_u8(w, 0u, s1);
    s2 = __builtin_amdgcn_udot4(w, w, s2, false);
}

// Block sums of up to four per-thread 64-bit counters (in a fixed order, so
// every launch gives the same bits); the result is valid in thread 0.
template <int K>
__device__ __forceinline__ void block_isum(unsigned long long (&v)[K], MsdScratch& sh)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) sh.isum[k][wave] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            unsigned long long t = 0;
            for (int w = 0; w < nw; ++w) t += sh.isum[k][w];
            v[k] = t;
        }
}

// (n, T, S) in the x domain from integer sums of n stored values v, where
// x = s*(v - c*z) (c = 1 for samples, Nmax for widest-boxcar values).
__device__ __forceinline__ void u8_partial(double n, unsigned long long sum, unsigned long long sumsq, double s,
                                           double cz, double* out3)
{
    if (n == 0.0) {
        out3[0] = out3[1] = out3[2] = 0.0;
        return;
    }
    const unsigned long long nn = (unsigned long long)n;
    const unsigned __int128 num = (unsigned __int128)nn * sumsq - (unsigned __int128)sum * sum;
    out3[0] = n;
    out3[1] = s * ((double)sum - n * cz);
    out3[2] = s * s * ((double)num / n);
}

// Raw-sample partials of one (row, column block) of a U8 plane: columns
// [lo, hi), lo = max(block start, new_col_begin).
__device__ void msd_block_x_u8(const PlaneArg& pl, bool vec, int64_t r, int64_t b, int64_t ncb, int64_t bc,
                               double* out6, MsdScratch& sh)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const uint8_t* row = (const uint8_t*)pl.data + r * pl.stride;
    const int64_t lo = max(b * bc, ncb), hi = min((b + 1) * bc, pl.n_cols);
    uint32_t s1 = 0, s2 = 0;                            // <= 256 samples per thread: no overflow
    if (lo < hi) {
        if (vec) {                                      // rows start on 4-byte boundaries
            const int64_t a = min(hi, (lo + 3) & ~(int64_t)3), e = max(a, hi & ~(int64_t)3);
            if (tid < a - lo) { const uint32_t q = row[lo + tid]; s1 += q; s2 += q * q; }
            if (tid < hi - e) { const uint32_t q = row[e + tid]; s1 += q; s2 += q * q; }
            const uint32_t* w = (const uint32_t*)(row + a);
            const int64_t nw = (e - a) / 4;
            int64_t i = tid;
            for (; i + 3 * nt < nw; i += 4 * nt) {
                const uint32_t w0 = w[i], w1 = w[i + nt], w2 = w[i + 2 * nt], w3 = w[i + 3 * nt];
                u8_word(w0, s1, s2); u8_word(w1, s1, s2); u8_word(w2, s1, s2); u8_word(w3, s1, s2);
            }
            for (; i < nw; i += nt) u8_word(w[i], s1, s2);
        } else {
            for (int64_t c = lo + tid; c < hi; c += nt) { const uint32_t q = row[c]; s1 += q; s2 += q * q; }
        }
    }
    unsigned long long v[2] = {s1, s2};
    block_isum<2>(v, sh);
    if (tid == 0) {
        u8_partial((double)max(hi - lo, (int64_t)0), v[0], v[1], (double)pl.scale[r], (double)pl.zero[r], out6);
        out6[3] = 0.0; out6[4] = 0.0; out6[5] = 0.0;
    }
}

// Inclusive prefix sum of 32-bit integers across the 64 lanes of a wave
// (DPP row shifts and row broadcasts, as wave_inclusive_scan).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_mov_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, true);
}

__device__ __forceinline__ int wave_inclusive_scan_i(int x)
{
    x += dpp_mov_i<0x111, 0xf>(x);
    x += dpp_mov_i<0x112, 0xf>(x);
    x += dpp_mov_i<0x114, 0xf>(x);
    x += dpp_mov_i<0x118, 0xf>(x);
    x += dpp_mov_i<0x142, 0xa>(x);
    x += dpp_mov_i<0x143, 0xc>(x);
    return x;
}

// Raw-sample partials of one (row, column block): columns [lo, hi) with
// lo = max(block start, new_col_begin).  Writes {n, T, S, 0, 0, 0} to out6.
template <int DT>
__device__ void msd_block_x(const PlaneArg& pl, bool vec, int64_t r, int64_t b, int64_t ncb, int64_t bc,
                            double* out6, MsdScratch& sh)
{
    if constexpr (DT == SPD_U8) {
        msd_block_x_u8(pl, vec, r, b, ncb, bc, out6, sh);
        return;
    }
    const int tid = threadIdx.x, nt = blockDim.x;
    Loader<DT> ld(pl, r);
    const float K = pilot_shift<DT>(ld, pl.n_cols, sh);
    const int64_t lo = max(b * bc, ncb), hi = min((b + 1) * bc, pl.n_cols);
    Msd s{0.f, 0.f, 0.f};
    if (lo < hi) {
        // vector loads need an address that is a multiple of four elements: the
        // columns c with (row offset + c) % 4 == 0, for any data pointer and
        // row stride (the element alignment of the pointer is checked on the host)
        (void)vec;
        const int64_t q = (4 - ld.mis4()) & 3;
        const int64_t a = min(lo + ((q - lo) & 3), hi);
        const int64_t e = max(a, hi - ((hi - q) & 3));
        if (tid < a - lo) msd_add1(s, ld.at(lo + tid) - K);
        if (tid < hi - e) { Msd t{0.f, 0.f, 0.f}; msd_add1(t, ld.at(e + tid) - K); s = msd_merge(s, t); }
        int64_t c = a + 4 * (int64_t)tid;
        const int64_t step = 4 * (int64_t)nt;
        for (; c + 3 * step < e; c += 4 * step) {
            const float4 v0 = ld.vec(c), v1 = ld.vec(c + step);
            const float4 v2 = ld.vec(c + 2 * step), v3 = ld.vec(c + 3 * step);
            const float v[16] = {v0.x - K, v0.y - K, v0.z - K, v0.w - K, v1.x - K, v1.y - K, v1.z - K, v1.w - K,
                                 v2.x - K, v2.y - K, v2.z - K, v2.w - K, v3.x - K, v3.y - K, v3.z - K, v3.w - K};
            msd_add16(s, v);
        }
        for (; c < e; c += step) {
            float4 v = ld.vec(c);
            msd_add4(s, v.x - K, v.y - K, v.z - K, v.w - K);
        }
    }
    Msd t = block_merge(s, sh.part);
    if (tid == 0) {
        out6[0] = t.n;
        out6[1] = (double)t.T + (double)t.n * (double)K;
        out6[2] = t.S;
        out6[3] = 0.0; out6[4] = 0.0; out6[5] = 0.0;
    }
}

// Inclusive prefix sum across the 64 lanes of a wave with DPP row shifts and
// row broadcasts (Hillis-Steele inside each row of 16, then across rows).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, true));
}

__device__ __forceinline__ float wave_inclusive_scan(float x)
{
    x += dpp_mov<0x111, 0xf>(x);   // row_shr:1
    x += dpp_mov<0x112, 0xf>(x);   // row_shr:2
    x += dpp_mov<0x114, 0xf>(x);   // row_shr:4
    x += dpp_mov<0x118, 0xf>(x);   // row_shr:8
    x += dpp_mov<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
    x += dpp_mov<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
    return x;
}

// Orders LDS writes and reads between lanes of one wave.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Sec. 2.1-2.2: raw statistics and the widest boxcar's statistics in one read
// ---------------------------------------------------------------------------
//
// sigma_Nmax of Eq. (sd03) needs the mean and spread of the widest boxcar
// y(t) = sum_{k<nmax} x[t+k] over every start t.  A wave owns a contiguous
// range of the block's columns and walks it in steps of 64*R starts; lane l
// takes the run of R consecutive starts t0 = u + R*l (R = 16, 8 for F32) and
// reads two windows of R samples straight from memory: its own x[t0 ..] and
// the shifted x[t0+nmax ..].  With D_k = x[t0+nmax+k] - x[t0+k] the series
// advances as y(t+1) = y(t) + D_k, so y(t0+k) = y0 + c_k, c_k = D_0 + ... +
// D_{k-1}, and the lane needs y0 = y(t0) only once per run:
//   sum_k y = R*y0 + sum_k c_k,   sum_k y^2 = R*y0^2 + 2*y0*sum_k c_k + sum_k c_k^2.
// y0 of lane l is the y of the step's first start plus the exclusive wave scan
// of the runs' drifts c_R; the next step starts from that plus the whole
// wave's drift (a running FP64 carry), and only the first start of the range
// takes a direct window sum.  Every sample is read twice, the second time
// mostly from cache, with no LDS and no barrier inside the walk.  Samples are
// shifted by K (pilot_shift); the raw sums and the run sums are FP32 over one
// run and FP64 across runs, and the block's S = sum d^2 - (sum d)^2/n is
// formed in FP64.

constexpr int kRun = 16;                // consecutive starts per lane (F16; 8 for F32)
// The U8 walk: longer runs (its per-run fold, a wave scan and 64-bit sums, is
// then paid once per 32 starts), one step per iteration; wave spans are
// multiples of its step.
constexpr int kRunU8 = 32;
constexpr int kRunStepU8 = 64 * kRunU8;

// 4*NDW bytes from `p` with aligned dword loads.  RA (realign): p may sit off a
// 4-byte boundary by sh = p & 3 (the same for every lane of the wave); one more
// dword is read and v_alignbyte shifts the bytes into place.  Each dword read
// holds a byte of the window or of the 4 bytes after it.
template <int NDW, bool RA>
__device__ __forceinline__ void load_window(const uint8_t* p, uint32_t sh, uint32_t (&w)[NDW])
{
    struct __attribute__((aligned(4))) U4 { uint32_t v[4]; };
    const uint32_t* q = (const uint32_t*)(p - (RA ? sh : 0u));
    uint32_t d[NDW + 1];
#pragma unroll
    for (int j = 0; j < NDW; j += 4) {
        const U4 t = *(const U4*)(q + j);
        d[j] = t.v[0]; d[j + 1] = t.v[1]; d[j + 2] = t.v[2]; d[j + 3] = t.v[3];
    }
    if constexpr (RA) {
        d[NDW] = q[NDW];
#pragma unroll
        for (int j = 0; j < NDW; ++j) w[j] = __builtin_amdgcn_alignbyte(d[j + 1], d[j], sh);
    } else {
#pragma unroll
        for (int j = 0; j < NDW; ++j) w[j] = d[j];
    }
}

// Run length of the F32 / F16 walks: 8 for F32, so that a lane's window is 32
// bytes as for F16 (64-byte windows per lane cost F32 about 10% in load rate).
template <int DT> constexpr int run_len() { return DT == SPD_F32 ? 8 : kRun; }

// Sample k of a run's dwords (F32 / F16).
template <int DT, int NDW>
__device__ __forceinline__ float run_at(const uint32_t (&w)[NDW], int k)
{
    if constexpr (DT == SPD_F32) {
        return __uint_as_float(w[k]);
    } else {
        const __half2 h = *reinterpret_cast<const __half2*>(&w[k >> 1]);
        return (k & 1) ? __high2float(h) : __low2float(h);
    }
}

// Sum of a double over the wave (every lane gets the same value).
__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Block sums of K per-thread doubles in a fixed order (lanes, then waves);
// the result is valid in thread 0.
template <int K>
__device__ __forceinline__ void block_dsum(double (&v)[K], MsdScratch& sh)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum_f64(v[k]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) sh.dsum[k][wave] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double t = 0.0;
            for (int w = 0; w < nw; ++w) t += sh.dsum[k][w];
            v[k] = t;
        }
}

// One run's sums, fed start by start: the raw sums of the shifted samples
// that count (xv), and sum c_k, sum c_k^2 over the starts that count (yv);
// c ends as the run's drift c_kRun.
struct RunAcc {
    float s1 = 0.f, s2 = 0.f, c = 0.f, sc = 0.f, qc = 0.f;
    // d = x[t0+k] - K, D = x[t0+nmax+k] - x[t0+k]; S1: also sum d (else the
    // caller sets s1)
    template <bool ALL, bool S1 = true>
    __device__ __forceinline__ void add(float d, float D, bool xv, bool yv)
    {
        const float v = ALL || xv ? d : 0.f;
        if constexpr (S1) s1 += v;
        s2 = fmaf(v, v, s2);
        const float cy = ALL || yv ? c : 0.f;
        sc += cy;
        qc = fmaf(cy, cy, qc);
        c += D;
    }
};

// Folds one step's run sums into the lane's FP64 accumulators {sum x, sum x^2,
// sum y, sum y^2} (shifted); `ny` starts of the run count for y.
__device__ __forceinline__ void step_fold(double (&acc)[4], double& carry, bool with_y, const RunAcc& ra, int ny)
{
    acc[0] += (double)ra.s1;
    acc[1] += (double)ra.s2;
    if (with_y) {                                       // uniform
        const float inc = wave_inclusive_scan(ra.c);
        const double y0 = carry + (double)(inc - ra.c);
        const double dsc = (double)ra.sc;
        acc[2] += fma((double)ny, y0, dsc);
        acc[3] += fma(y0, fma((double)ny, y0, 2.0 * dsc), (double)ra.qc);
        carry += (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(inc), 63));
    }
}

// The walk of one wave's columns [w0, w1) on an F32 / F16 row, one step at a
// time: RAO / RAN say whether the own / shifted windows sit off 4-byte
// boundaries.  (Loading the next step ahead into a second register set was
// slower: the extra registers halve the waves per SIMD.)
template <int DT, bool RAO, bool RAN>
__device__ __forceinline__ void walk_f(const Loader<DT>& ld, float K, int64_t w0, int64_t w1, int64_t xlo,
                                       int64_t yhi, int64_t ncols, int32_t nmax, double (&acc)[4], double& carry)
{
    constexpr int ES = DT == SPD_F32 ? 4 : 2, RUN = run_len<DT>(), STEP = 64 * RUN, NDW = RUN * ES / 4;
    const int lane = threadIdx.x & 63;
    const uint8_t* rowb = (const uint8_t*)ld.row;
    // F16: x - K and x[t+nmax] - x as FMAs by an opaque 1 take the halves as
    // they are (v_fma_mix_f32, one rounding like a convert and a subtract)
    float one = 1.f;
    if constexpr (DT == SPD_F16) asm("s_mov_b32 %0, 1.0" : "=s"(one));
    const uint32_t sho = (uint32_t)((uintptr_t)rowb & 3), shn = (uint32_t)(((uintptr_t)rowb + nmax * ES) & 3);
    for (int64_t u = w0; u < w1; u += STEP) {
        const int64_t t0 = u + RUN * lane;
        RunAcc ra;
        if (u >= xlo && u + STEP <= min(w1, yhi) && u + STEP + nmax + 4 <= ncols) {
            // every start counts and every sample read is inside the row
            uint32_t wo[NDW], wn[NDW];
            load_window<NDW, RAO>(rowb + t0 * ES, sho, wo);
            load_window<NDW, RAN>(rowb + (t0 + nmax) * ES, shn, wn);
            if constexpr (DT == SPD_F16) {
                // the run's sum from the stored halves, two per v_dot2c_f32_f16
                typedef _Float16 h2 __attribute__((ext_vector_type(2)));
                const h2 ones = {(_Float16)1.0f, (_Float16)1.0f};
                float sx = 0.f;
#pragma unroll
                for (int j = 0; j < NDW; ++j) sx = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2, wo[j]), ones, sx, false);
#pragma unroll
                for (int k = 0; k < RUN; ++k) {
                    const float x = run_at<DT, NDW>(wo, k), xn = run_at<DT, NDW>(wn, k);
                    ra.add<true, false>(fmaf(x, one, -K), fmaf(xn, one, -x), true, true);
                }
                ra.s1 = fmaf(-(float)RUN, K, sx);
            } else {
#pragma unroll
                for (int k = 0; k < RUN; ++k) {
                    const float x = run_at<DT, NDW>(wo, k), xn = run_at<DT, NDW>(wn, k);
                    ra.add<true>(x - K, xn - x, true, true);
                }
            }
            step_fold(acc, carry, true, ra, RUN);
        } else {
            const bool with_y = u < yhi;
#pragma unroll 1
            for (int k = 0; k < RUN; ++k) {
                const int64_t c = t0 + k;
                const float x = c < ncols ? ld.at(c) : 0.f;
                const float xn = with_y && c + nmax < ncols ? ld.at(c + nmax) : 0.f;
                ra.add<false>(x - K, xn - x, c >= xlo && c < w1, c < yhi);
            }
            step_fold(acc, carry, with_y, ra, (int)max(min(yhi - t0, (int64_t)RUN), (int64_t)0));
        }
    }
}

// Raw-sample partials of columns [max(block start, new_col_begin), block end)
// and the widest-boxcar partials of starts [block start, min(block end, nout)),
// which give sigma_Nmax of Eq. (sd03).  Writes {n, T, S} of each to out6.
template <int DT>
__device__ void msd_block_xy_f(const PlaneArg& pl, int64_t r, int64_t b, int64_t ncb, int64_t bc, int32_t nmax,
                               int64_t nout, double* out6, MsdScratch& sh)
{
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: scalar walk bounds
    Loader<DT> ld(pl, r);
    const float K = pilot_shift<DT>(ld, pl.n_cols, sh);
    const int64_t ncols = pl.n_cols;
    const int64_t c0 = b * bc, c1 = min(c0 + bc, ncols);
    const int64_t xlo = max(c0, ncb), yhi = min(c1, nout);
    const int64_t w0 = c0 + (int64_t)wave * (bc / nw), w1 = min(w0 + bc / nw, c1);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};              // sum x, sum x^2, sum y, sum y^2 (shifted)
    double carry = 0.0;                                 // y at the next step's first start
    if (w0 < yhi) {
        double s = 0.0;
        for (int64_t c = w0 + lane; c < w0 + nmax; c += 64) s += c < ncols ? (double)(ld.at(c) - K) : 0.0;
        carry = wave_sum_f64(s);
    }
    if constexpr (DT == SPD_F32) {
        walk_f<DT, false, false>(ld, K, w0, w1, xlo, yhi, ncols, nmax, acc, carry);
    } else {
        const uintptr_t a = (uintptr_t)ld.row;
        const bool ro = (a & 3) != 0, rn = ((a + 2 * (uintptr_t)nmax) & 3) != 0;
        if (!ro && !rn) walk_f<DT, false, false>(ld, K, w0, w1, xlo, yhi, ncols, nmax, acc, carry);
        else if (!ro) walk_f<DT, false, true>(ld, K, w0, w1, xlo, yhi, ncols, nmax, acc, carry);
        else if (!rn) walk_f<DT, true, false>(ld, K, w0, w1, xlo, yhi, ncols, nmax, acc, carry);
        else walk_f<DT, true, true>(ld, K, w0, w1, xlo, yhi, ncols, nmax, acc, carry);
    }
    block_dsum<4>(acc, sh);
    if (threadIdx.x == 0) {
        // S = sum d^2 - (sum d)^2 / n without contraction: one value gives S = 0
#pragma clang fp contract(off)
        const double nx = (double)max(c1 - xlo, (int64_t)0), ny = (double)max(yhi - c0, (int64_t)0);
        out6[0] = nx;
        out6[1] = acc[0] + nx * (double)K;
        out6[2] = nx > 0.0 ? fmax(acc[1] - acc[0] * (acc[0] / nx), 0.0) : 0.0;
        out6[3] = ny;
        out6[4] = acc[2] + ny * (double)nmax * (double)K;
        out6[5] = ny > 0.0 ? fmax(acc[3] - acc[2] * (acc[2] / ny), 0.0) : 0.0;
    }
}

// One U8 run's widest-boxcar sums in integers, fed start by start (as RunAcc):
// |c_k| <= 255*k for k <= kRunU8, so c_k^2 and the run's sums (sum of c_k^2 at
// most 255^2 * 11440 < 2^30) fit in int32.
struct RunAccI {
    int c = 0, sc = 0, qc = 0;
    template <bool ALL>
    __device__ __forceinline__ void add(int x, int xn, bool yv)
    {
        if (ALL || yv) {
            sc += c;
            // |c| < 2^23: the full-rate 24-bit multiply-add (the compiler cannot
            // prove the range through the run and would pick v_mul_lo_u32)
            int r;
            asm("v_mad_i32_i24 %0, %1, %1, %2" : "=v"(r) : "v"(c), "v"(qc));
            qc = r;
        }
        c += xn - x;
    }
};

// Folds a U8 run into the lane's y sums: y0 and the carry are at most
// 255*nmax < 2^21; a lane's sum of y over its <= 8 runs of 32 starts (a block
// spans at most 65536 columns, 16384 per wave) stays below 2^31; the sum of y^2
// is 64-bit.
__device__ __forceinline__ void u8_fold(const RunAccI& ra, int ny, uint32_t& sy1, long long& sy2, int& carry)
{
    const int inc = wave_inclusive_scan_i(ra.c);
    const int y0 = carry + (inc - ra.c);
    sy1 += (uint32_t)(ny * y0 + ra.sc);
    sy2 += (long long)y0 * (long long)(ny * y0 + 2 * ra.sc) + (long long)ra.qc;
    carry += __builtin_amdgcn_readlane(inc, 63);
}

// The walk of one wave's columns [w0, w1) on a U8 row.  RAO / RAN: the own /
// shifted windows sit off 4-byte boundaries.  (Taking the shifted window
// across lanes with ds_bpermute instead of a second load was slower.)
template <bool RAO, bool RAN>
__device__ __forceinline__ void walk_u8(const uint8_t* row, int64_t w0, int64_t w1, int64_t xlo, int64_t yhi,
                                        int64_t ncols, int32_t nmax, uint32_t& sx1, uint32_t& sx2, uint32_t& sy1,
                                        long long& sy2, int& carry)
{
    constexpr int SPAN = kRunStepU8, NW = kRunU8 / 4;
    const int lane = threadIdx.x & 63;
    const uint32_t sho = (uint32_t)((uintptr_t)row & 3), shn = (uint32_t)(((uintptr_t)row + nmax) & 3);
    for (int64_t u = w0; u < w1; u += SPAN) {
        const int64_t t0 = u + kRunU8 * lane;
        RunAccI ra;
        if (u >= xlo && u + SPAN <= min(w1, yhi) && u + SPAN + nmax + 4 <= ncols) {
            uint32_t wo[NW], wn[NW];
            load_window<NW, RAO>(row + t0, sho, wo);
            load_window<NW, RAN>(row + t0 + nmax, shn, wn);
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                u8_word(wo[i], sx1, sx2);
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    ra.add<true>((int)((wo[i] >> (8 * k)) & 255u), (int)((wn[i] >> (8 * k)) & 255u), true);
            }
            u8_fold(ra, kRunU8, sy1, sy2, carry);
        } else {
            const bool with_y = u < yhi;
#pragma unroll 1
            for (int k = 0; k < kRunU8; ++k) {
                const int64_t c = t0 + k;
                const uint32_t q = c < ncols ? (uint32_t)row[c] : 0u;
                const uint32_t qn = with_y && c + nmax < ncols ? (uint32_t)row[c + nmax] : 0u;
                if (c >= xlo && c < w1) {
                    sx1 += q;
                    sx2 += q * q;
                }
                ra.add<false>((int)q, (int)qn, c < yhi);
            }
            if (with_y) u8_fold(ra, (int)max(min(yhi - t0, (int64_t)kRunU8), (int64_t)0), sy1, sy2, carry);
        }
    }
}

// The same on a U8 plane, in integers (exact up to the conversion's last
// rounding in u8_partial): byte sums per word (v_sad_u8, v_dot4), the runs'
// c_k sums in int32, the y sums in 64 bits.
__device__ void msd_block_xy_u8(const PlaneArg& pl, int64_t r, int64_t b, int64_t ncb, int64_t bc, int32_t nmax,
                                int64_t nout, double* out6, MsdScratch& sh)
{
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: scalar walk bounds
    const uint8_t* row = (const uint8_t*)pl.data + r * pl.stride;
    const int64_t ncols = pl.n_cols;
    const int64_t c0 = b * bc, c1 = min(c0 + bc, ncols);
    const int64_t xlo = max(c0, ncb), yhi = min(c1, nout);
    const int64_t w0 = c0 + (int64_t)wave * (bc / nw), w1 = min(w0 + bc / nw, c1);
    uint32_t sx1 = 0, sx2 = 0, sy1 = 0;                 // <= 16 runs of 16 bytes per lane (block span <= 65536)
    long long sy2 = 0;
    int carry = 0;
    if (w0 < yhi) {
        int s = 0;
        for (int64_t c = w0 + lane; c < w0 + nmax; c += 64) s += c < ncols ? (int)row[c] : 0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        carry = s;
    }
    const uintptr_t a = (uintptr_t)row;
    const bool ro = (a & 3) != 0, rn = ((a + (uintptr_t)nmax) & 3) != 0;
    if (!ro && !rn) walk_u8<false, false>(row, w0, w1, xlo, yhi, ncols, nmax, sx1, sx2, sy1, sy2, carry);
    else if (!ro) walk_u8<false, true>(row, w0, w1, xlo, yhi, ncols, nmax, sx1, sx2, sy1, sy2, carry);
    else if (!rn) walk_u8<true, false>(row, w0, w1, xlo, yhi, ncols, nmax, sx1, sx2, sy1, sy2, carry);
    else walk_u8<true, true>(row, w0, w1, xlo, yhi, ncols, nmax, sx1, sx2, sy1, sy2, carry);
    unsigned long long acc[4] = {sx1, sx2, sy1, (unsigned long long)sy2};
    block_isum<4>(acc, sh);
    if (threadIdx.x == 0) {
        const double s = (double)pl.scale[r], z = (double)pl.zero[r];
        u8_partial((double)max(c1 - xlo, (int64_t)0), acc[0], acc[1], s, z, out6);
        u8_partial((double)max(yhi - c0, (int64_t)0), acc[2], acc[3], s, (double)nmax * z, out6 + 3);
    }
}

template <int DT>
__device__ void msd_block_xy(const PlaneArg& pl, bool vec, int64_t r, int64_t b, int64_t ncb, int64_t bc,
                             int32_t nmax, int64_t nout, double* out6, MsdScratch& sh)
{
    (void)vec;                                          // windows are realigned per row
    if constexpr (DT == SPD_U8) msd_block_xy_u8(pl, r, b, ncb, bc, nmax, nout, out6, sh);
    else msd_block_xy_f<DT>(pl, r, b, ncb, bc, nmax, nout, out6, sh);
}

// ---------------------------------------------------------------------------
// FP64 merge across blocks (Eq. MSD04) and the sigma_N coefficients
// ---------------------------------------------------------------------------

struct Msd64 { double n, T, S; };

__device__ __forceinline__ Msd64 merge64(Msd64 a, Msd64 b)
{
    if (a.n == 0.0) return b;
    if (b.n == 0.0) return a;
    double d = (b.n / a.n) * a.T - b.T;
    return Msd64{a.n + b.n, a.T + b.T, a.S + b.S + a.n / (b.n * (a.n + b.n)) * d * d};
}

struct FinalizeScratch {
    Msd64 x[256], y[256];
};

// One unit's statistics from its `per_unit` block partials p[per_unit][6]:
// thread j merges a contiguous run in order, then a fixed neighbour tree
// merges the runs (deterministic).  Thread 0 merges the result into the
// running state (when given), then writes mean, sigma, sigma_Nmax and the
// coefficient of Eq. (sd03) for the sigma mode.
__device__ void finalize_unit(const double* p, int64_t per_unit, bool need_y, bool accumulate,
                              spd_msd_state* state, spd_row_stats* stats, int32_t nmax, int32_t mode,
                              double kappa, FinalizeScratch& sh)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int64_t q = (per_unit + nt - 1) / nt;
    Msd64 ax{0, 0, 0}, ay{0, 0, 0};
    for (int64_t i = tid * q; i < min((int64_t)(tid + 1) * q, per_unit); ++i) {
        ax = merge64(ax, Msd64{p[i * 6 + 0], p[i * 6 + 1], p[i * 6 + 2]});
        ay = merge64(ay, Msd64{p[i * 6 + 3], p[i * 6 + 4], p[i * 6 + 5]});
    }
    sh.x[tid] = ax;
    sh.y[tid] = ay;
    __syncthreads();
    for (int h = 1; h < nt; h <<= 1) {                 // merge neighbours: runs stay in order
        if ((tid & (2 * h - 1)) == 0 && tid + h < nt) {
            sh.x[tid] = merge64(sh.x[tid], sh.x[tid + h]);
            sh.y[tid] = merge64(sh.y[tid], sh.y[tid + h]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        Msd64 X = sh.x[0], Y = sh.y[0];
        if (state) {
            const spd_msd_state st = *state;
            if (accumulate) {
                X = merge64(Msd64{st.n, st.T, st.S}, X);
                Y = merge64(Msd64{st.n_y, st.T_y, st.S_y}, Y);
            }
            *state = spd_msd_state{X.n, X.T, X.S, Y.n, Y.T, Y.S};
        }
        spd_row_stats o;
        o.mean = X.n > 0.0 ? X.T / X.n : 0.0;
        o.sigma = X.n > 0.0 ? sqrt(X.S / X.n) : 0.0;
        o.sigma_nmax = (need_y && Y.n > 0.0) ? sqrt(Y.S / Y.n) : 0.0;
        o.lin_coef = 0.0;
        o.flags = 0;
        o.reserved0 = 0;
        if (!(o.sigma > 0.0)) {
            o.flags |= SPD_FLAG_ZERO_VAR;
        } else if (nmax > 1 && mode != SPD_SIGMA_SQRTN) {
            const double base = sqrt((double)nmax) * o.sigma;
            const double anchored = (o.sigma_nmax - base) / (double)(nmax - 1);
            if (mode == SPD_SIGMA_LINEAR) {
                o.lin_coef = anchored; o.flags |= SPD_FLAG_LINEAR;
            } else if (mode == SPD_SIGMA_LINEAR_LITERAL) {
                o.lin_coef = o.sigma_nmax / (double)(nmax - 1); o.flags |= SPD_FLAG_LINEAR;
            } else if (mode == SPD_SIGMA_AUTO && o.sigma_nmax / base > 1.0 + kappa) {
                o.lin_coef = anchored; o.flags |= SPD_FLAG_LINEAR;
            }
        }
        *stats = o;
    }
}

// ---------------------------------------------------------------------------
// Sec. 2.3, Algorithm 1: boxcars, SNR, highest SNR and first width; Sec. 2.4
// ---------------------------------------------------------------------------
//
// One wave owns 64*X consecutive output starts of one row; lane l handles
// starts t = l + 64*i (i < X) so that every LDS read is conflict free.  The
// wave stages x' = x - mean for its window [t_w, t_w + 64X + Nmax - 1) in LDS
// (array 0) plus presummed arrays D_g for other gaps, then walks the width list
// once: B_{w_i} = B_{w_{i-1}} + D_g[t + w_{i-1}], s_i = B_{w_i} * (1/sigma_{w_i}).
// Every boxcar sum is a running sum that starts at t, as in Algorithm 1, so
// its rounding error grows with w only.
//
// The highest SNR and the first width reaching it are found exactly, with the
// bookkeeping of Algorithm 1 (compare, then keep value and width) done once
// per group of 8 widths on the group maximum: the first group whose maximum is
// strictly larger than everything before it holds the first maximiser.  After
// the list is done, that one group is evaluated again from the running sum
// saved at its start (bit-identical operations) and the first width whose SNR
// equals the maximum is taken.

// LDS layout of a work-group: [kTableFloats] tables, then per wave
// ba.wave_floats floats of presummed arrays.
template <int DT, int X, bool UNIT, int SMALL = 0>
__device__ void boxcar_tile(const PlaneArg& pl, bool vec, int64_t r, int64_t tt, const spd_row_stats& st,
                            const BoxcarArgs& ba, const WidthPlan& wp, float* smem, bool setup_tables)
{
    float* coef = smem;                                              // 1/sigma_w; NaN past n
    uint32_t* toff = (uint32_t*)(coef + kMaxWidthsPadded);           // read offsets; 0 past n
    uint32_t* tcg = toff + kMaxWidthsPadded;                         // cnt | gap<<16; 0 past n
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
    float* arrs = smem + kTableFloats + (size_t)wave * ba.wave_floats;
    const int64_t tw = tt * (int64_t)(nwaves * 64 * X) + (int64_t)wave * 64 * X;

    __syncthreads();                                    // the previous tile is done with LDS
    if (setup_tables) {
        const bool zero_var = (st.flags & SPD_FLAG_ZERO_VAR) != 0;
        for (int i = tid; i < kMaxWidthsPadded; i += blockDim.x) {
            if (i < wp.n) {
                const int w = wp.width[i];
                const double sw = sqrt((double)w) * st.sigma + (double)(w - 1) * st.lin_coef;
                coef[i] = (zero_var || !sigma_w_positive(sw, w, st.sigma)) ? 0.f : (float)(1.0 / sw);   // Eq. (sd02)/(sd03)
                toff[i] = wp.off[i];
                tcg[i] = wp.cg[i];
            } else {
                coef[i] = __int_as_float(0x7fc00000);
                toff[i] = 0;
                tcg[i] = 0;
            }
        }
    }
    const float mu_hi = (float)st.mean;
    const float mu_lo = (float)(st.mean - (double)mu_hi);

    // stage x' = x - mean for this wave's window; zero beyond the row
    Loader<DT> ld(pl, r);
    const int np = 64 * X + wp.nmax - 1;
    for (int k = 4 * lane; k < ba.npw; k += 256) {
        const int64_t c = tw + k;
        *(float4*)(arrs + k) = load4_shifted<DT>(ld, c, pl.n_cols, vec, mu_hi, mu_lo);
    }
    __syncthreads();
    for (int a = 1; a < wp.n_arr; ++a) {                // presummed arrays D_g
        const int g = wp.arr_gap[a];
        float* Da = arrs + (size_t)a * ba.npw;
        for (int k = lane; k < ba.npw; k += 64) {
            float s = 0.f;
            if (k + g <= np) {
                s = arrs[k];
                for (int j = 1; j < g; ++j) s += arrs[k + j];
            }
            Da[k] = s;
        }
    }
    __syncthreads();

    const float* lbase = arrs + lane;
    // output start t = tw + lane + 64 i: per-sample outputs and the fused threshold
    auto emit = [&](int i, float m, int idx) {
        const int64_t t = tw + lane + 64 * i;
        const bool valid = t < ba.nout;
        if (valid && ba.snr) ba.snr[r * ba.out_stride + t] = m;
        if (valid && ba.widx) ba.widx[r * ba.out_stride + t] = (uint8_t)idx;
        if (ba.cand) {
            const bool pred = valid && m >= ba.threshold;
            const uint64_t mask = __ballot(pred);
            if (mask) {
                const int cntw = __popcll(mask);
                const int before = __popcll(mask & ((1ull << lane) - 1ull));
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd((unsigned long long*)ba.cand_count, (unsigned long long)cntw);
                base = __shfl(base, 0);
                if (pred) {
                    const unsigned long long k = base + (unsigned long long)before;
                    if (k < (unsigned long long)ba.cand_capacity) {
                        spd_candidate cd;
                        cd.row = (int32_t)r + ba.row0;
                        cd.width = wp.width[idx];
                        cd.t = t + ba.t_offset;
                        cd.snr = m;
                        cd.beam = ba.beam;
                        ba.cand[k] = cd;
                    }
                }
            }
        }
    };
    if constexpr (SMALL > 0) {
        // Short lists (n <= SMALL, one step per width): every SNR of a start
        // stays in registers; the maximum is a max tree and the first width
        // reaching it a reverse select chain.  Entries past n have a NaN
        // coefficient: max ignores them and they never compare equal.
        constexpr int NS = SMALL > 0 ? SMALL : 1;
        float a[NS];
        uint32_t off[NS];
#pragma unroll
        for (int j = 0; j < SMALL; j += 4) {
            const float4 c = *(const float4*)(coef + j);
            a[j] = c.x; a[j + 1] = c.y; a[j + 2] = c.z; a[j + 3] = c.w;
        }
#pragma unroll
        for (int j = 0; j < SMALL; ++j) off[j] = wp.off[j];
#pragma unroll
        for (int i = 0; i < X; ++i) {
            float b = 0.f, sv[NS];
#pragma unroll
            for (int j = 0; j < SMALL; ++j) {
                b = __fadd_rn(b, lbase[off[j] + 64 * i]);
                sv[j] = __fmul_rn(b, a[j]);
            }
            float m = sv[0];
#pragma unroll
            for (int j = 1; j < SMALL; ++j) m = fmaxf(m, sv[j]);
            int idx = wp.n - 1;
#pragma unroll
            for (int j = SMALL - 1; j >= 0; --j) idx = (sv[j] == m) ? j : idx;
            emit(i, m, idx);
        }
    } else {
        float B[X], mx[X], Bg[X];
        int gi[X];
#pragma unroll
        for (int i = 0; i < X; ++i) { B[i] = 0.f; mx[i] = -INFINITY; Bg[i] = 0.f; gi[i] = 0; }

        const int nfull = wp.n / kGroup;
        // Two groups per trip let the carried sums and maxima alternate
        // registers instead of being copied; the general-count form is
        // already register-heavy and stays rolled.
        constexpr int kGroupUnroll = UNIT ? 2 : 1;
#pragma unroll kGroupUnroll
        for (int g = 0; g < nfull; ++g) {
            const int i0 = g * kGroup;
            const float4 a03 = *(const float4*)(coef + i0);
            const float4 a47 = *(const float4*)(coef + i0 + 4);
            const float a[8] = {a03.x, a03.y, a03.z, a03.w, a47.x, a47.y, a47.z, a47.w};
            uint32_t off[8], cg[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) { off[j] = wp.off[i0 + j]; cg[j] = wp.cg[i0 + j]; }
#pragma unroll
            for (int i = 0; i < X; ++i) {
                float b = B[i];
                float s[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    if (UNIT) {
                        b = __fadd_rn(b, lbase[off[j] + 64 * i]);
                    } else {
                        const uint32_t cnt = cg[j] & 0xffffu, gap = cg[j] >> 16;
                        for (uint32_t m = 0; m < cnt; ++m) b = __fadd_rn(b, lbase[off[j] + m * gap + 64 * i]);
                    }
                    s[j] = __fmul_rn(b, a[j]);
                }
                // running maximum folded into the group's max3 tree; c: this group beats all before it
                const float mnew = fmaxf(fmaxf(fmaxf(fmaxf(fmaxf(fmaxf(fmaxf(fmaxf(s[0], s[1]), s[2]), s[3]), s[4]),
                                                           s[5]), s[6]), s[7]), mx[i]);
                const bool c = mnew > mx[i];
                Bg[i] = c ? B[i] : Bg[i];
                gi[i] = c ? g : gi[i];
                mx[i] = mnew;
                B[i] = b;
            }
        }
        const int rem = wp.n - nfull * kGroup;
        if (rem) {                                          // last, partial group
            const int i0 = nfull * kGroup;
#pragma unroll
            for (int i = 0; i < X; ++i) {
                float b = B[i], gm = -INFINITY;
                for (int j = 0; j < rem; ++j) {
                    const uint32_t o = wp.off[i0 + j], cgv = wp.cg[i0 + j];
                    const uint32_t cnt = cgv & 0xffffu, gap = cgv >> 16;
                    for (uint32_t m = 0; m < cnt; ++m) b = __fadd_rn(b, lbase[o + m * gap + 64 * i]);
                    gm = fmaxf(gm, __fmul_rn(b, coef[i0 + j]));
                }
                const bool c = gm > mx[i];
                Bg[i] = c ? B[i] : Bg[i];
                gi[i] = c ? nfull : gi[i];
                mx[i] = c ? gm : mx[i];
                B[i] = b;
            }
        }

        // first width inside the winning group, then outputs and the fused threshold
#pragma unroll
        for (int i = 0; i < X; ++i) {
            const int i0 = gi[i] * kGroup;
            const float4 c03 = *(const float4*)(coef + i0);
            const float4 c47 = *(const float4*)(coef + i0 + 4);
            const float cf[8] = {c03.x, c03.y, c03.z, c03.w, c47.x, c47.y, c47.z, c47.w};
            float b = Bg[i];
            float s[8];
            if (UNIT) {
                const uint4 o03 = *(const uint4*)(toff + i0);
                const uint4 o47 = *(const uint4*)(toff + i0 + 4);
                const uint32_t o[8] = {o03.x, o03.y, o03.z, o03.w, o47.x, o47.y, o47.z, o47.w};
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    b = __fadd_rn(b, lbase[o[j] + 64 * i]);
                    s[j] = __fmul_rn(b, cf[j]);
                }
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const uint32_t o = toff[i0 + j], cgv = tcg[i0 + j];
                    const uint32_t cnt = cgv & 0xffffu, gap = cgv >> 16;
                    for (uint32_t m = 0; m < cnt; ++m) b = __fadd_rn(b, lbase[o + m * gap + 64 * i]);
                    s[j] = __fmul_rn(b, cf[j]);
                }
            }
            int idx = wp.n - 1;                             // reached only if no SNR equals the max (NaN input)
#pragma unroll
            for (int j = 7; j >= 0; --j) idx = (s[j] == mx[i]) ? i0 + j : idx;
            emit(i, mx[i], idx);
        }
    }
}

// The highest SNR and its first width in one max: the key of width index j
// is the double whose high word is the SNR's bit pattern and whose low word is
// N-1-j.  Doubles and floats are both sign-magnitude, so keys order as their
// SNRs do; between equal SNRs the larger low word, i.e. the smaller j, wins
// when the SNR is positive (zero included), and the larger j when it is
// negative.  The maximum key carries the highest SNR exactly in its high word.
// v_max_f64 runs at the FP32 rate; written out so that no canonicalising max
// is inserted for the keys, which are not arithmetic results.
__device__ __forceinline__ double key_max(double a, double b)
{
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// ---------------------------------------------------------------------------
// Sec. 2.3 / Algorithm 1, register-window form
// ---------------------------------------------------------------------------
//
// Lane l of a wave owns the kWinX consecutive starts t = tw + 8l + i (i < 8).
// The wave's window sits in LDS with one pad float after every 8 (rows of 9):
// logical element k of an array is at k + k/8, so lane l's starts begin at
// 9l and a read of one logical offset by the 64 lanes hits distinct banks.
// A group of 8 widths whose boxcar steps read one array at offsets
// o, o+d, ..., o+7d (d = 1 or 2, o a multiple of 8) needs only the 8 + 7d
// values D[8l + o + m], m < 8 + 7d, for all of its 64 (start, width) pairs:
// they are read once into registers, where the pair (i, j) finds
// D[t_i + o + d*j] at m = i + d*j.  The same holds for the list 1..n
// (n <= 16) over x' itself.  Results are those of boxcar_tile: the same
// running sums in the same order, and the same first-maximiser rule.

template <int DT, int SMALLN, bool DIT = false>
__device__ void boxcar_tile_win(const PlaneArg& pl, bool vec, int64_t r, int64_t tt, const spd_row_stats& st,
                                const BoxcarArgs& ba, const WidthPlan& wp, float* smem)
{
    constexpr int X = kWinX;
    float* coef = smem;                                             // 1/sigma_w; NaN past n
    uint32_t* tgb = (uint32_t*)(coef + kMaxWidthsPadded);           // per group: padded offset of its reads
    uint32_t* tgs = tgb + kMaxGroups;                               // per group: step d
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
    float* arrs = smem + kWinTableFloats + (size_t)wave * ba.wave_floats;
    const int64_t tw = tt * (int64_t)(nwaves * 64 * X) + (int64_t)wave * 64 * X;
    const int rows9 = ba.npw / 9;                                   // rows of 8 logical floats per array
    const int nlog = rows9 * 8;

    {
        const bool zero_var = (st.flags & SPD_FLAG_ZERO_VAR) != 0;
        for (int i = tid; i < kMaxWidthsPadded; i += blockDim.x) {
            if (i < wp.n) {
                const int w = wp.width[i];
                const double sw = sqrt((double)w) * st.sigma + (double)(w - 1) * st.lin_coef;
                coef[i] = (zero_var || !sigma_w_positive(sw, w, st.sigma)) ? 0.f : (float)(1.0 / sw);   // Eq. (sd02)/(sd03)
            } else {
                coef[i] = __int_as_float(0x7fc00000);
            }
        }
        for (int g = tid; g < kMaxGroups; g += blockDim.x) {
            tgb[g] = wp.gbase[g];
            tgs[g] = wp.gstep[g];
        }
    }
    const float mu_hi = (float)st.mean;
    const float mu_lo = (float)(st.mean - (double)mu_hi);

    // stage x' = x - mean (array 0); zero beyond the row
    Loader<DT> ld(pl, r);
    if (vec && tw + nlog <= pl.n_cols) {
        // window inside the row (all but the last tiles): four vector loads per
        // lane in flight before any is written; lanes past the window reload
        // its last four samples and skip the write
        for (int k0 = 4 * lane; k0 < nlog; k0 += 1024) {
            float4 v[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) v[m] = ld.vec(tw + min(k0 + 256 * m, nlog - 4));
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int k = k0 + 256 * m;
                if (k < nlog) {
                    float* d = arrs + win_phys(k);                  // k..k+3 share one row of 9
                    d[0] = (v[m].x - mu_hi) - mu_lo;
                    d[1] = (v[m].y - mu_hi) - mu_lo;
                    d[2] = (v[m].z - mu_hi) - mu_lo;
                    d[3] = (v[m].w - mu_hi) - mu_lo;
                }
            }
        }
    } else {
        for (int k = 4 * lane; k < nlog; k += 256) {
            const float4 v = load4_shifted<DT>(ld, tw + k, pl.n_cols, vec, mu_hi, mu_lo);
            float* d = arrs + win_phys(k);
            d[0] = v.x;
            d[1] = v.y;
            d[2] = v.z;
            d[3] = v.w;
        }
    }
    __syncthreads();
    for (int a = 1; a < wp.n_arr; ++a) {                            // presummed arrays D_g
        const int g = wp.arr_gap[a];
        float* Da = arrs + (size_t)a * ba.npw;
        for (int row = lane; row < rows9; row += 64) {
            const float* xr = arrs + 9 * row;                       // logical 8row.., then the next row at 9
            if (g == 2) {
                // the 9 values of a row and the next one's first, read once
                float v[9];
#pragma unroll
                for (int c = 0; c < 8; ++c) v[c] = xr[c];
                v[8] = row + 1 < rows9 ? xr[9] : 0.f;
                const bool last = row + 1 == rows9;                 // its final sum would run past the window
#pragma unroll
                for (int c = 0; c < 8; ++c) Da[9 * row + c] = (last && c == 7) ? 0.f : v[c] + v[c + 1];
            } else {
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int k = 8 * row + c;
                    float s = 0.f;
                    if (k + g <= nlog) {
                        s = arrs[win_phys(k)];
                        for (int j = 1; j < g; ++j) s += arrs[win_phys(k + j)];
                    }
                    Da[9 * row + c] = s;
                }
            }
        }
    }
    __syncthreads();

    // lane base as one opaque register, so the reads below keep small immediate
    // offsets (the paired LDS read encodes at most 255 dwords)
    int lbo = kWinTableFloats + wave * ba.wave_floats + 9 * lane;
    asm volatile("" : "+v"(lbo));
    const float* lb = smem + lbo;
    const int64_t t0 = tw + (int64_t)X * lane;
    float sv[X];
    int iv[X];

    if constexpr (SMALLN > 0) {
        // widths 1..n: every SNR of a start in registers, max tree, reverse select chain
        constexpr int NS = SMALLN > 0 ? SMALLN : 1;
        constexpr int NV = X + NS - 1;
        float v[NV];
#pragma unroll
        for (int m = 0; m < NV; ++m) v[m] = lb[win_phys(m)];
        float a[NS];
#pragma unroll
        for (int j = 0; j < NS; j += 4) {
            const float4 c = *(const float4*)(coef + j);
            a[j] = c.x; a[j + 1] = c.y; a[j + 2] = c.z; a[j + 3] = c.w;
        }
        // the decimated search keeps, per start, the running maximum of FP64 keys
        // (key_max) over its base widths and then over each level's widths
        double mk[DIT ? X : 1];
#pragma unroll
        for (int i = 0; i < X; ++i) {
            if constexpr (DIT) {
                float b = v[i];
                double m = __hiloint2double(__float_as_int(__fmul_rn(b, a[0])), wp.n - 1);
#pragma unroll
                for (int j = 1; j < NS; ++j) {
                    b = __fadd_rn(b, v[i + j]);
                    m = key_max(m, __hiloint2double(__float_as_int(__fmul_rn(b, a[j])), wp.n - 1 - j));
                }
                mk[i] = m;
                continue;
            }
            float b = 0.f, s[NS];
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                b = __fadd_rn(b, v[i + j]);
                s[j] = __fmul_rn(b, a[j]);
            }
            if constexpr (NS == 16) {
                // the half that holds the first maximiser, then a chain over its 8 SNRs
                float mlo = s[0], mhi = s[8];
#pragma unroll
                for (int j = 1; j < 8; ++j) { mlo = fmaxf(mlo, s[j]); mhi = fmaxf(mhi, s[8 + j]); }
                const float m = fmaxf(mlo, mhi);
                const bool hi = !(mlo == m);
                int idx = -1;
#pragma unroll
                for (int j = 7; j >= 0; --j) idx = ((hi ? s[8 + j] : s[j]) == m) ? j : idx;
                sv[i] = m;
                iv[i] = idx < 0 ? wp.n - 1 : idx + (hi ? 8 : 0);    // no match only for NaN input
            } else {
                float m = s[0];
#pragma unroll
                for (int j = 1; j < NS; ++j) m = fmaxf(m, s[j]);
                int idx = wp.n - 1;
#pragma unroll
                for (int j = NS - 1; j >= 0; --j) idx = (s[j] == m) ? j : idx;
                sv[i] = m;
                iv[i] = idx;
            }
        }
        if constexpr (DIT) {
            // Decimated levels: level lv holds x'_lv[k] = x'_{lv-1}[2k] + x'_{lv-1}[2k+1].
            // Lane l evaluates widths 9..16 at its 8/2^lv decimated starts
            // 8l/2^lv + j (level 4: lane l/2, even lanes only), i.e. physical
            // widths 2^lv*(9..16) at starts 8l + 2^lv*j, and merges their keys
            // into those starts' running maxima (the list ascends, so equal
            // positive SNRs keep the narrower width).
            const int levels = (wp.n - kDitBase) / (kDitBase / 2);
            float* lev = arrs + ba.npw;
            auto level = [&](auto lv_c) {
                constexpr int LV = decltype(lv_c)::value;
                constexpr int S = LV < 4 ? (8 >> LV) : 1;              // decimated starts per lane
                float* dst = lev;
                for (int l2 = 1; l2 < LV; ++l2) dst += dit_level_floats(levels, l2);
                const float* src = LV == 1 ? arrs : dst - dit_level_floats(levels, LV - 1);
                const int n = dit_level_len(levels, LV);
                // k = lane + 64 i: every padded index is the lane's plus a multiple of
                // i known at compile time (the pads repeat every 8, 4 or 2 elements),
                // so the unrolled build reads and writes at immediate offsets
                constexpr int NI = (dit_level_len(4, LV) + 63) / 64;
                const float* s0 = src + (LV == 1 ? win_phys(2 * lane) : dit_pad(LV - 1, 2 * lane));
                const float* s1 = src + (LV == 1 ? win_phys(2 * lane + 1) : dit_pad(LV - 1, 2 * lane + 1));
                float* d0 = dst + dit_pad(LV, lane);
                constexpr int SS = LV == 1 ? win_phys(128) : dit_pad(LV - 1, 128);   // source step per i
                constexpr int DS = dit_pad(LV, 64);                                  // destination step per i
#pragma unroll
                for (int i = 0; i < NI; ++i)
                    if (lane + 64 * i < n) d0[DS * i] = __fadd_rn(s0[SS * i], s1[SS * i]);
                wave_sync();
                const int lstride = LV == 1 ? 5 : LV == 2 ? 3 : 1;      // padded offset of lane l's first start
                const float* lbv = dst + (LV < 4 ? lstride * lane : (lane >> 1));
                constexpr int NV = S + kDitBase - 1;
                float v[NV];
#pragma unroll
                for (int m = 0; m < NV; ++m) v[m] = lbv[dit_pad(LV, m)];
                const int c0 = kDitBase + (kDitBase / 2) * (LV - 1);
                const float4 a03 = *(const float4*)(coef + c0);
                const float4 a47 = *(const float4*)(coef + c0 + 4);
                const float a[8] = {a03.x, a03.y, a03.z, a03.w, a47.x, a47.y, a47.z, a47.w};
                const int rank0 = wp.n - 1 - c0;
#pragma unroll
                for (int j = 0; j < S; ++j) {
                    float b = v[j];
#pragma unroll
                    for (int q = 1; q < kDitBase / 2; ++q) b = __fadd_rn(b, v[j + q]);
                    double m = mk[LV < 4 ? (j << LV) : 0];
#pragma unroll
                    for (int q = kDitBase / 2; q < kDitBase; ++q) {
                        b = __fadd_rn(b, v[j + q]);
                        const float sq = __fmul_rn(b, a[q - kDitBase / 2]);
                        m = key_max(m, __hiloint2double(__float_as_int(sq), rank0 - (q - kDitBase / 2)));
                    }
                    if (LV < 4 || (lane & 1) == 0) mk[LV < 4 ? (j << LV) : 0] = m;
                }
            };
            if (levels >= 1) level(std::integral_constant<int, 1>());
            if (levels >= 2) level(std::integral_constant<int, 2>());
            if (levels >= 3) level(std::integral_constant<int, 3>());
            if (levels >= 4) level(std::integral_constant<int, 4>());
#pragma unroll
            for (int i = 0; i < X; ++i) {
                sv[i] = __int_as_float(__double2hiint(mk[i]));
                iv[i] = wp.n - 1 - __double2loint(mk[i]);
            }
        }
    } else {
        float B[X], mx[X], Bg[X];
        int gi[X];
#pragma unroll
        for (int i = 0; i < X; ++i) { B[i] = 0.f; mx[i] = -INFINITY; Bg[i] = 0.f; gi[i] = 0; }
        auto group = [&](auto step_c, int g) {
            constexpr int D = decltype(step_c)::value;
            constexpr int NV = 8 + 7 * D;
            const float* gb = lb + wp.gbase[g];
            float v[NV];
#pragma unroll
            for (int m = 0; m < NV; ++m) v[m] = gb[win_phys(m)];
            const float4 a03 = *(const float4*)(coef + g * kGroup);
            const float4 a47 = *(const float4*)(coef + g * kGroup + 4);
            const float a[8] = {a03.x, a03.y, a03.z, a03.w, a47.x, a47.y, a47.z, a47.w};
#pragma unroll
            for (int i = 0; i < X; ++i) {
                float b = B[i];
                float s[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    b = __fadd_rn(b, v[i + D * j]);
                    s[j] = __fmul_rn(b, a[j]);
                }
                // running maximum folded into the group's max3 tree; c: this group beats all before it
                const float mnew = fmaxf(fmaxf(fmaxf(fmaxf(fmaxf(fmaxf(fmaxf(fmaxf(s[0], s[1]), s[2]), s[3]), s[4]),
                                                           s[5]), s[6]), s[7]), mx[i]);
                const bool c = mnew > mx[i];
                Bg[i] = c ? B[i] : Bg[i];
                gi[i] = c ? g : gi[i];
                mx[i] = mnew;
                B[i] = b;
            }
        };
        const int ng = wp.n / kGroup;                               // n is a multiple of 8 in this form
        // runs of groups with one step; two groups per trip let the carried
        // sums and maxima alternate registers instead of being copied
        for (int g = 0; g < ng;) {
            const int d = wp.gstep[g];
            int g1 = g + 1;
            while (g1 < ng && wp.gstep[g1] == d) ++g1;
            if (d == 1) {
#pragma unroll 2
                for (; g < g1; ++g) group(std::integral_constant<int, 1>(), g);
            } else {
#pragma unroll 2
                for (; g < g1; ++g) group(std::integral_constant<int, 2>(), g);
            }
        }
        // first width inside the winning group, with bit-identical operations.  Both
        // steps' reads sit at immediate offsets of the group base (inside the
        // staged window either way); the lane's step picks the value.
#pragma unroll
        for (int i = 0; i < X; ++i) {
            const int g = gi[i];
            const float* gb = lb + tgb[g];
            const bool two = tgs[g] == 2u;
            const float4 c03 = *(const float4*)(coef + g * kGroup);
            const float4 c47 = *(const float4*)(coef + g * kGroup + 4);
            const float cf[8] = {c03.x, c03.y, c03.z, c03.w, c47.x, c47.y, c47.z, c47.w};
            float b = Bg[i];
            float s[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float d1 = gb[win_phys(i + j)], d2 = gb[win_phys(i + 2 * j)];
                b = __fadd_rn(b, two ? d2 : d1);
                s[j] = __fmul_rn(b, cf[j]);
            }
            int jj = -1;
#pragma unroll
            for (int j = 7; j >= 0; --j) jj = (s[j] == mx[i]) ? j : jj;
            sv[i] = mx[i];
            iv[i] = jj < 0 ? wp.n - 1 : g * kGroup + jj;           // no match only for NaN input
        }
    }

    // fused threshold (Sec. 2.4): a wave with no SNR at the threshold skips it; otherwise one
    // ballot per start index and one atomic per wave with candidates
    const int64_t left = ba.nout - t0;
    const int nvalid = left <= 0 ? 0 : (left >= X ? X : (int)left);
    float mall = sv[0];
#pragma unroll
    for (int i = 1; i < X; ++i) mall = fmaxf(mall, sv[i]);
    if (ba.cand && __ballot(mall >= ba.threshold)) {
#pragma unroll
        for (int i = 0; i < X; ++i) {
            const int64_t t = t0 + i;
            const bool pred = i < nvalid && sv[i] >= ba.threshold;
            const uint64_t mask = __ballot(pred);
            if (mask) {
                const int cntw = __popcll(mask);
                const int before = __popcll(mask & ((1ull << lane) - 1ull));
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd((unsigned long long*)ba.cand_count, (unsigned long long)cntw);
                base = __shfl(base, 0);
                if (pred) {
                    const unsigned long long k = base + (unsigned long long)before;
                    if (k < (unsigned long long)ba.cand_capacity) {
                        spd_candidate cd;
                        cd.row = (int32_t)r + ba.row0;
                        cd.width = wp.width[iv[i]];
                        cd.t = t + ba.t_offset;
                        cd.snr = sv[i];
                        cd.beam = ba.beam;
                        ba.cand[k] = cd;
                    }
                }
            }
        }
    }
    // per-start outputs.  In the grouped form (long width lists, bound by the ALU)
    // rows that allow vector stores take each lane's 8 starts directly, which
    // saves the transpose's work.  Otherwise -- and always for the short lists,
    // whose stores weigh more -- the wave transposes them through its LDS region
    // (done with the window by now) and lane l stores starts tw + l + 64i, so
    // every store instruction covers consecutive addresses; measured faster
    // for those lists even where vector stores are allowed.
    if (!ba.snr && !ba.widx) return;
    const uint32_t need_vec = (ba.snr ? 1u : 0u) | (ba.widx ? 2u : 0u);
    if (SMALLN == 0 && (ba.out_vec & need_vec) == need_vec) {
        if (ba.snr) {
            float* dst = ba.snr + r * ba.out_stride + t0;
            if (nvalid == X) {
                *(float4*)dst = make_float4(sv[0], sv[1], sv[2], sv[3]);
                *(float4*)(dst + 4) = make_float4(sv[4], sv[5], sv[6], sv[7]);
            } else {
#pragma unroll
                for (int i = 0; i < X; ++i)
                    if (i < nvalid) dst[i] = sv[i];
            }
        }
        if (ba.widx) {
            uint8_t* dst = ba.widx + r * ba.out_stride + t0;
            if (nvalid == X) {
                uint2 u;
                u.x = (uint32_t)iv[0] | ((uint32_t)iv[1] << 8) | ((uint32_t)iv[2] << 16) | ((uint32_t)iv[3] << 24);
                u.y = (uint32_t)iv[4] | ((uint32_t)iv[5] << 8) | ((uint32_t)iv[6] << 16) | ((uint32_t)iv[7] << 24);
                *(uint2*)dst = u;
            } else {
#pragma unroll
                for (int i = 0; i < X; ++i)
                    if (i < nvalid) dst[i] = (uint8_t)iv[i];
            }
        }
        return;
    }
    float* xs = arrs;                                               // 64X floats, then 64X bytes
    uint8_t* xb = (uint8_t*)(arrs + 64 * X);
    wave_sync();                                                    // the wave's window reads are done
    *(float4*)(xs + X * lane) = make_float4(sv[0], sv[1], sv[2], sv[3]);
    *(float4*)(xs + X * lane + 4) = make_float4(sv[4], sv[5], sv[6], sv[7]);
    uint2 u;
    u.x = (uint32_t)iv[0] | ((uint32_t)iv[1] << 8) | ((uint32_t)iv[2] << 16) | ((uint32_t)iv[3] << 24);
    u.y = (uint32_t)iv[4] | ((uint32_t)iv[5] << 8) | ((uint32_t)iv[6] << 16) | ((uint32_t)iv[7] << 24);
    *(uint2*)(xb + X * lane) = u;
    wave_sync();
    const int64_t wleft = ba.nout - tw;                             // valid starts of this wave
    const int64_t rowo = r * ba.out_stride + tw + lane;
    float* ds = ba.snr ? ba.snr + rowo : nullptr;                   // one base each, immediate offsets below
    uint8_t* db = ba.widx ? ba.widx + rowo : nullptr;
    if (wleft >= 64 * X) {
#pragma unroll
        for (int i = 0; i < X; ++i) {
            if (ds) ds[64 * i] = xs[lane + 64 * i];
            if (db) db[64 * i] = xb[lane + 64 * i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < X; ++i) {
            if (lane + 64 * i < wleft) {
                if (ds) ds[64 * i] = xs[lane + 64 * i];
                if (db) db[64 * i] = xb[lane + 64 * i];
            }
        }
    }
}


// ---------------------------------------------------------------------------
// Sec. 2.3 / Algorithm 1, streaming form of the short lists 1..n (n <= 16)
// ---------------------------------------------------------------------------
//
// A wave owns a run of kStreamRun consecutive starts of one row and walks it
// in steps of kStreamStep.  Lane l takes the 4 consecutive starts 4l..4l+3 of
// a step (block 0) and 256+4l..256+4l+3 (block 1), so its outputs are one
// 16-byte SNR store and one 4-byte width-index store per block, and a store
// instruction of the wave covers consecutive addresses.  A block needs the
// samples 4l .. 4l+n+2 of its step: five aligned 16-byte LDS reads.
//
// The wave's LDS holds two buffers of kStreamBuf floats: x' = x - mean of one
// step and the first 16 samples of the next.  While a step is evaluated the
// samples of the step after next are in flight from HBM; the step in
// registers is written to the other buffer before the evaluation starts, so
// no work-group barrier is needed and every sample is read from HBM once.
// The coefficients 1/sigma_w are wave-uniform (scalar registers).

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <int DT> struct RawT;
template <> struct RawT<SPD_F32> { using T = f32x4; };
template <> struct RawT<SPD_F16> { using T = u32x2; };
template <> struct RawT<SPD_U8> { using T = uint32_t; };

// Four samples from column c as stored; past the end of the row the value is
// unspecified (those samples only reach windows that start past the last
// valid start).  `vec`: the row allows aligned vector loads at c.
template <int DT>
__device__ __forceinline__ typename RawT<DT>::T raw4(const Loader<DT>& ld, int64_t c, int64_t ncols, bool vec)
{
    using T = typename RawT<DT>::T;
    if (vec && c + 3 < ncols) return *(const T*)(ld.row + c);
    if constexpr (DT == SPD_F32) {
        f32x4 v;
        v.x = c < ncols ? ld.row[c] : 0.f;
        v.y = c + 1 < ncols ? ld.row[c + 1] : 0.f;
        v.z = c + 2 < ncols ? ld.row[c + 2] : 0.f;
        v.w = c + 3 < ncols ? ld.row[c + 3] : 0.f;
        return v;
    } else if constexpr (DT == SPD_F16) {
        const uint16_t* h = (const uint16_t*)ld.row;
        uint32_t e[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) e[k] = c + k < ncols ? (uint32_t)h[c + k] : 0u;
        const u32x2 u = {e[0] | (e[1] << 16), e[2] | (e[3] << 16)};
        return u;
    } else {
        uint32_t u = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) u |= (c + k < ncols ? (uint32_t)ld.row[c + k] : 0u) << (8 * k);
        return u;
    }
}

template <int DT>
__device__ __forceinline__ float4 cvt4(const Loader<DT>& ld, typename RawT<DT>::T u)
{
    if constexpr (DT == SPD_F32) {
        return make_float4(u.x, u.y, u.z, u.w);
    } else if constexpr (DT == SPD_F16) {
        const uint32_t lo = u.x, hi = u.y;
        const float2 a = __half22float2(*reinterpret_cast<const __half2*>(&lo));
        const float2 b = __half22float2(*reinterpret_cast<const __half2*>(&hi));
        return make_float4(a.x, a.y, b.x, b.y);
    } else {
        return make_float4(ld.deq(u & 255u), ld.deq((u >> 8) & 255u), ld.deq((u >> 16) & 255u), ld.deq(u >> 24));
    }
}

__device__ __forceinline__ void put_shifted(float* d, float4 v, float mu_hi, float mu_lo)
{
    *(float4*)d = make_float4((v.x - mu_hi) - mu_lo, (v.y - mu_hi) - mu_lo, (v.z - mu_hi) - mu_lo,
                              (v.w - mu_hi) - mu_lo);
}

// The 4 starts of one block for the list 1..N: their highest SNR and the index
// of the width reaching it (see key_max).  `src` points at the block's first
// start in LDS.
template <int N>
__device__ __forceinline__ void short_block(const float* src, const float (&a)[N], float (&sv)[4], uint32_t& packed)
{
    constexpr int NV = 4 + N - 1;
    constexpr int NR = (NV + 3) / 4;
    float v[4 * NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const float4 f = *(const float4*)(src + 4 * q);
        v[4 * q] = f.x; v[4 * q + 1] = f.y; v[4 * q + 2] = f.z; v[4 * q + 3] = f.w;
    }
    uint32_t ranks = 0;                                     // N-1-j of each start's width, one byte each
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float b = v[i];
        double m = __hiloint2double(__float_as_int(__fmul_rn(b, a[0])), N - 1);
#pragma unroll
        for (int j = 1; j < N; ++j) {
            b = __fadd_rn(b, v[i + j]);
            m = key_max(m, __hiloint2double(__float_as_int(__fmul_rn(b, a[j])), N - 1 - j));
        }
        sv[i] = __int_as_float(__double2hiint(m));
        ranks |= (uint32_t)__double2loint(m) << (8 * i);
    }
    packed = (uint32_t)(N - 1) * 0x01010101u - ranks;      // bytewise, no borrows: every rank <= N-1
}

// One candidate per (start, lane) with snr >= threshold among the lane's
// `cnt` starts beginning at t: one ballot per start index, one atomic per
// wave and start index that has candidates.
__device__ __forceinline__ void emit_block_cands(const BoxcarArgs& ba, const WidthPlan& wp, int64_t r, int64_t t,
                                                 int cnt, const float (&sv)[4], uint32_t packed)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bool pred = i < cnt && sv[i] >= ba.threshold;
        const uint64_t mask = __ballot(pred);
        if (!mask) continue;
        const int cntw = __popcll(mask);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd((unsigned long long*)ba.cand_count, (unsigned long long)cntw);
        base = __shfl(base, 0);
        if (pred) {
            const unsigned long long k = base + (unsigned long long)before;
            if (k < (unsigned long long)ba.cand_capacity) {
                spd_candidate cd;
                cd.row = (int32_t)r + ba.row0;
                cd.width = wp.width[(packed >> (8 * i)) & 255u];
                cd.t = t + i + ba.t_offset;
                cd.snr = sv[i];
                cd.beam = ba.beam;
                ba.cand[k] = cd;
            }
        }
    }
}

// Coefficients 1/sigma_w of widths 1..N (Eq. sd02 / sd03), wave-uniform: lane
// j computes width j+1 in FP64 and the values are read into scalar registers.
template <int N>
__device__ __forceinline__ void short_coefs(const spd_row_stats& st, float (&a)[N])
{
    const int lane = threadIdx.x & 63;
    const bool zero_var = (st.flags & SPD_FLAG_ZERO_VAR) != 0;
    float cf = 0.f;
    if (lane < N) {
        const double w = (double)(lane + 1);
        const double sw = sqrt(w) * st.sigma + (w - 1.0) * st.lin_coef;
        cf = (zero_var || !sigma_w_positive(sw, w, st.sigma)) ? 0.f : (float)(1.0 / sw);
    }
#pragma unroll
    for (int j = 0; j < N; ++j) a[j] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cf), j));
}

// One run of kStreamRun starts at t_begin whose every start is valid and
// every sample it reads (its starts plus the 16 samples after them) lies
// inside a row that allows vector loads.  OUT: both outputs are written with
// 16-byte and 4-byte stores; otherwise candidates only.  Every step is whole,
// so the stores are unconditional and a step's loads are waited for without
// waiting for the previous step's stores.
template <int DT, int N, bool OUT>
__device__ void boxcar_run_fast(const PlaneArg& pl, int64_t r, int64_t t_begin, const spd_row_stats& st,
                                const BoxcarArgs& ba, const WidthPlan& wp, float* buf)
{
    using Raw = typename RawT<DT>::T;
    constexpr int S = kStreamSteps;
    const int lane = threadIdx.x & 63, lo = 4 * lane;
    float a[N];
    short_coefs<N>(st, a);
    const float mu_hi = (float)st.mean;
    const float mu_lo = (float)(st.mean - (double)mu_hi);
    const Loader<DT> ld(pl, r);
    const Raw* rowp = (const Raw*)(ld.row + t_begin) + lane;      // one Raw per 4 samples
    float* so = OUT ? ba.snr + r * ba.out_stride + t_begin + lo : nullptr;
    uint8_t* wo = OUT ? ba.widx + r * ba.out_stride + t_begin + lo : nullptr;

    float* A = buf;
    float* Bv = buf + kStreamBuf;
    {
        const Raw s0 = rowp[0], s1 = rowp[64];
        put_shifted(A + lo, cvt4<DT>(ld, s0), mu_hi, mu_lo);
        put_shifted(A + 256 + lo, cvt4<DT>(ld, s1), mu_hi, mu_lo);
    }
    Raw r0 = rowp[kStreamStep / 4], r1 = rowp[kStreamStep / 4 + 64];
    if (lane < 4) put_shifted(A + kStreamStep + lo, cvt4<DT>(ld, r0), mu_hi, mu_lo);
    wave_sync();
    for (int k = 0; k < S; ++k) {
        if (k + 1 < S) {
            put_shifted(Bv + lo, cvt4<DT>(ld, r0), mu_hi, mu_lo);
            put_shifted(Bv + 256 + lo, cvt4<DT>(ld, r1), mu_hi, mu_lo);
        }
        const Raw* nx = rowp + (k + 2) * (kStreamStep / 4);
        if (k + 2 < S) {                                    // read once: nontemporal
            r0 = __builtin_nontemporal_load(nx);
            r1 = __builtin_nontemporal_load(nx + 64);
        } else if (k + 2 == S && lane < 4) {
            r0 = nx[0];
        }
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) {
            float sv[4];
            uint32_t pk;
            short_block<N>(A + 256 * blk + lo, a, sv, pk);
            const int off = k * kStreamStep + 256 * blk;
            if (ba.cand && __ballot(fmaxf(fmaxf(sv[0], sv[1]), fmaxf(sv[2], sv[3])) >= ba.threshold))
                emit_block_cands(ba, wp, r, t_begin + off + lo, 4, sv, pk);
            if (OUT) {                                                  // written once, never read here
                const f32x4 q = {sv[0], sv[1], sv[2], sv[3]};
                __builtin_nontemporal_store(q, (f32x4*)(so + off));
                __builtin_nontemporal_store(pk, (uint32_t*)(wo + off));
            }
        }
        if (k + 1 < S && lane < 4) put_shifted(Bv + kStreamStep + lo, cvt4<DT>(ld, r0), mu_hi, mu_lo);
        wave_sync();
        float* tmp = A; A = Bv; Bv = tmp;
    }
}

// Starts [t_begin, min(t_begin + kStreamRun, nout)) of row r by one wave, for
// any run: loads checked against the row end and against vector alignment,
// stores per element where a step is partial or the rows do not allow vector
// stores.  buf is the wave's 2*kStreamBuf floats of LDS (16-byte aligned).
template <int DT, int N>
__device__ void boxcar_run_short(const PlaneArg& pl, bool vec, int64_t r, int64_t t_begin, const spd_row_stats& st,
                                 const BoxcarArgs& ba, const WidthPlan& wp, float* buf)
{
    using Raw = typename RawT<DT>::T;
    const int lane = threadIdx.x & 63;
    const int64_t nout = ba.nout;
    const int64_t t_end = min(t_begin + kStreamRun, nout);
    const int steps = (int)((t_end - t_begin + kStreamStep - 1) / kStreamStep);
    float a[N];
    short_coefs<N>(st, a);
    const float mu_hi = (float)st.mean;
    const float mu_lo = (float)(st.mean - (double)mu_hi);
    const Loader<DT> ld(pl, r);
    const int64_t ncols = pl.n_cols;
    const int lo = 4 * lane;
    auto load = [&](int64_t off) -> Raw { return raw4<DT>(ld, t_begin + off, ncols, vec); };

    float* A = buf;
    float* Bv = buf + kStreamBuf;
    {
        const Raw s0 = load(lo), s1 = load(lo + 256);
        put_shifted(A + lo, cvt4<DT>(ld, s0), mu_hi, mu_lo);
        put_shifted(A + 256 + lo, cvt4<DT>(ld, s1), mu_hi, mu_lo);
    }
    Raw r0{}, r1{};
    if (steps > 1) {
        r0 = load(kStreamStep + lo);
        r1 = load(kStreamStep + 256 + lo);
    } else if (lane < 4) {
        r0 = load(kStreamStep + lo);
    }
    if (lane < 4) put_shifted(A + kStreamStep + lo, cvt4<DT>(ld, r0), mu_hi, mu_lo);
    wave_sync();

    float* so = ba.snr ? ba.snr + r * ba.out_stride + t_begin : nullptr;
    uint8_t* wo = ba.widx ? ba.widx + r * ba.out_stride + t_begin : nullptr;
    const bool vs = (ba.out_vec & 1u) != 0, vw = (ba.out_vec & 4u) != 0;
    for (int k = 0; k < steps; ++k) {
        const int ks = k * kStreamStep;
        if (k + 1 < steps) {
            put_shifted(Bv + lo, cvt4<DT>(ld, r0), mu_hi, mu_lo);
            put_shifted(Bv + 256 + lo, cvt4<DT>(ld, r1), mu_hi, mu_lo);
        }
        if (k + 2 < steps) {
            r0 = load(ks + 2 * kStreamStep + lo);
            r1 = load(ks + 2 * kStreamStep + 256 + lo);
        } else if (k + 2 == steps && lane < 4) {
            r0 = load(ks + 2 * kStreamStep + lo);
        }
        const bool whole = t_begin + ks + kStreamStep <= t_end;
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) {
            float sv[4];
            uint32_t pk;
            short_block<N>(A + 256 * blk + lo, a, sv, pk);
            const int off = ks + 256 * blk + lo;
            int cnt = 4;
            if (!whole) {
                const int64_t left = t_end - (t_begin + off);
                cnt = left <= 0 ? 0 : (left >= 4 ? 4 : (int)left);
            }
            if (ba.cand && __ballot(fmaxf(fmaxf(sv[0], sv[1]), fmaxf(sv[2], sv[3])) >= ba.threshold))
                emit_block_cands(ba, wp, r, t_begin + off, cnt, sv, pk);
            if (whole && vs && so) {
                *(float4*)(so + off) = make_float4(sv[0], sv[1], sv[2], sv[3]);
            } else if (so) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (i < cnt) so[off + i] = sv[i];
            }
            if (whole && vw && wo) {
                *(uint32_t*)(wo + off) = pk;
            } else if (wo) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (i < cnt) wo[off + i] = (uint8_t)(pk >> (8 * i));
            }
        }
        if (k + 1 < steps && lane < 4) put_shifted(Bv + kStreamStep + lo, cvt4<DT>(ld, r0), mu_hi, mu_lo);
        wave_sync();
        float* tmp = A; A = Bv; Bv = tmp;
    }
}

}  // namespace spd
