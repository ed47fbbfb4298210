// spd_internal.h -- types shared by the host and device parts of libspd.
// (Library-internal; the public boundary is include/spd.h.)
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "spd.h"

namespace spd {

constexpr int kWave = 64;           // CDNA wavefront
constexpr int kGroup = 8;           // widths evaluated between two argmax bookkeeping steps
constexpr int kMaxArrays = 4;       // presummed LDS arrays per wave (gap sizes)
constexpr int kOutPerLane = 8;      // boxcar outputs per lane (strided by 64)
constexpr int kMaxWidthsPadded = SPD_MAX_WIDTHS + kGroup;
constexpr int kMaxGroups = kMaxWidthsPadded / kGroup;
constexpr int kWinX = 8;           // consecutive starts per lane in the register-window form
constexpr int kSelCols = 4096;     // columns per work-group of the standalone threshold (16 per lane)
constexpr int kWinTableFloats = (kMaxWidthsPadded + 2 * kMaxGroups + 63) / 64 * 64;

// Streaming form of the short lists 1..n (n <= 16): a wave walks a run of
// kStreamSteps steps of kStreamStep consecutive starts of one row; lane l
// takes starts 4l..4l+3 and 256+4l..256+4l+3 of each step.  Its LDS holds two
// buffers of one step's samples plus the next 16.
constexpr int kStreamStep = 512;
constexpr int kStreamSteps = 16;
constexpr int64_t kStreamRun = (int64_t)kStreamStep * kStreamSteps;
constexpr int kStreamBuf = kStreamStep + 16;

// Register-window form: logical element m of a wave's LDS array is stored at
// m + m/8 (one pad float after every 8).
__host__ __device__ constexpr int win_phys(int m) { return m + (m >> 3); }

// Decimated search (boxcars combined with decimation in time): base widths
// 1..kDitBase, then kDitBase/2+1..kDitBase on the series decimated 1..levels
// times.  Level lv of a wave holds dit_level_len(levels, lv) decimated
// samples, padded so that the starts of lane l begin at a conflict-free offset
// (level 1: one pad per 4, level 2: one pad per 2, level >= 3: none).
constexpr int kDitBase = 16;
constexpr int kDitMaxLevels = 4;
__host__ __device__ constexpr int dit_level_len(int levels, int lv)
{
    return (64 * kWinX + (kDitBase - 1) * (1 << levels)) >> lv;
}
__host__ __device__ constexpr int dit_pad(int lv, int k) { return lv == 1 ? k + (k >> 2) : lv == 2 ? k + (k >> 1) : k; }
__host__ __device__ constexpr int dit_level_floats(int levels, int lv)
{
    return (dit_pad(lv, dit_level_len(levels, lv) - 1) + 1 + 3) & ~3;
}
// LDS floats of the boxcar kernel's coefficient and step tables, rounded up so
// the per-wave arrays after them start on a 256-byte boundary.
constexpr int kTableFloats = (3 * kMaxWidthsPadded + 63) / 64 * 64;
constexpr uint64_t kMaxGridItems = 0xffffffffull;   // work-items per launch (1-D grid)

// How each width's boxcar is reached from the previous one:
//   B_{w_i}(t) = B_{w_{i-1}}(t) + sum_{m < cnt_i} D_{g}[t + off_i + m*g]
// where D_g[k] = sum_{j<g} x'[k+j] is a presummed array held in LDS (g = the
// array's gap) and x' = x - mean.  For a list of contiguous or evenly spaced
// widths every cnt_i is 1, so each width costs one LDS read and one add.
struct WidthPlan {
    int32_t n;              // |W|
    int32_t nmax;           // largest width
    int32_t n_groups;       // ceil(n / kGroup); the last group may be partial
    int32_t n_arr;          // presummed arrays in use (array 0 is x' itself, gap 1)
    int32_t arr_gap[kMaxArrays];
    int32_t unit_counts;    // 1 when every cnt_i == 1
    int32_t win;            // register-window form: 0 none, 1 groups of 8, 2 the list 1..n (n <= 16),
                            // 3 the decimated search (1..16, then 2^l*(9..16)),
                            // 4 the list 1..n (n <= 16) in the streaming form
    uint32_t off[kMaxWidthsPadded];    // element offset of the first read: array base + w_{i-1}
    uint32_t cg[kMaxWidthsPadded];     // cnt | (gap << 16)
    int16_t width[kMaxWidthsPadded];   // w_i
    // register-window form, per group of 8 widths: padded LDS offset of the
    // group's first read (array base + o + o/8, o = w_{8g-1}) and its step d
    uint32_t gbase[kMaxGroups];
    uint8_t gstep[kMaxGroups];
};

struct PlaneArg {
    const void* data;
    int64_t n_rows, n_cols, stride;
    const float* scale;     // U8 only
    const float* zero;      // U8 only
};

// Arguments of the boxcar/SNR kernel besides the plane and the width plan.
struct BoxcarArgs {
    int32_t scope;
    int32_t npw;            // floats per presummed array (>= 64X + Nmax - 1, multiple of 4)
    int32_t wave_floats;    // LDS floats per wave: n_arr*npw
    int32_t row0;           // added to the row stored in each candidate (row-chunked launches)
    int64_t tiles_per_row;
    int64_t nout;           // valid starts per row
    float* snr;
    uint8_t* widx;
    int64_t out_stride;
    int64_t t_offset;
    spd_candidate* cand;
    int64_t cand_capacity;
    int64_t* cand_count;
    float threshold;
    uint32_t beam;          // stored in each candidate (batched runs)
    uint32_t out_vec;       // bit 0: snr rows allow 16-byte stores; bit 1: widx rows allow 8-byte stores;
                            // bit 2: widx rows allow 4-byte stores
    uint32_t reserved;
    int64_t run0, run1;     // streaming form: the runs [run0, run1) of every row this launch covers
};

struct SelectArgs {
    int32_t width[SPD_MAX_WIDTHS];
    float threshold;
    int32_t reserved;
    int64_t t_offset;
    spd_candidate* cand;
    int64_t cand_capacity;
    int64_t* cand_count;
};

}  // namespace spd
