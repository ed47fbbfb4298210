// spd_abi_internal.h -- host helpers shared by the ABI translation units.
#pragma once

#include <stdarg.h>

#include "spd_internal.h"

namespace spd {

struct MsdLayout {
    int64_t bc;          // columns per block
    int64_t nblk;        // blocks per row
    size_t ws_bytes;     // partials: n_rows * nblk * 6 doubles
};

spd_status fail(spd_status st, const char* fmt, ...);
void clear_error();
spd_status device_status(hipError_t e, const char* what);
int elem_size(int dtype);
spd_status check_params(const spd_params* p);
spd_status check_plane(const spd_plane* x, const spd_params* p);
PlaneArg plane_arg(const spd_plane* x);
bool plane_vec_ok(const spd_plane* x);
MsdLayout msd_layout(const spd_plane* x);
bool build_width_plan(const spd_params* p, int X, WidthPlan& wp, BoxcarArgs& ba, int& waves,
                      size_t lds_reserve = 0, bool window = false);

struct BoxcarPlan {
    WidthPlan wp;
    BoxcarArgs ba;
    int waves;
};

spd_status check_msd_workspace(const spd_plane* x, const MsdLayout& m, const void* workspace, size_t bytes);
spd_status enqueue_msd(const spd_plane* x, const spd_params* p, int64_t new_col_begin, bool accumulate,
                       spd_msd_state* state, spd_row_stats* stats, double* part, const MsdLayout& m, hipStream_t s);
spd_status plan_boxcar(const spd_plane* x, const spd_params* p, const spd_row_stats* stats, float* snr_out,
                       uint8_t* widx_out, int64_t out_stride, int64_t t_offset, spd_candidate* cand,
                       int64_t cand_capacity, int64_t* cand_count, BoxcarPlan& bp);
spd_status enqueue_boxcar(const spd_plane* x, const spd_row_stats* stats, const BoxcarPlan& bp, int64_t r0,
                          int64_t rows, hipStream_t s);
spd_plane row_slice(const spd_plane* x, int64_t r0, int64_t rows);
spd_status detect_events(hipEvent_t** out);
void dedisp_plan_shape(const spd_dedisp_plan* plan, int32_t* n_chan, int32_t* n_dm, int32_t* max_delay, int* device);

}  // namespace spd
