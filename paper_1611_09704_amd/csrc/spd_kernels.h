// spd_kernels.h -- launch entry points of the gfx950 kernels (library-internal).
#pragma once

#include "spd_internal.h"

namespace spd {

hipError_t launch_msd(int dtype, const PlaneArg& pl, bool vec, bool with_y, int64_t ncb, int64_t bc,
                      int64_t nblk, int32_t nmax, int64_t nout, double* part, hipStream_t s);
hipError_t launch_finalize(const double* part, int64_t n_units, int64_t per_unit, bool need_y,
                           bool accumulate, spd_msd_state* state, spd_row_stats* stats, int32_t nmax,
                           int32_t mode, double kappa, hipStream_t s);
size_t boxcar_lds_bytes(int waves, const BoxcarArgs& ba, bool win = false);
hipError_t launch_boxcar(int dtype, const PlaneArg& pl, bool vec, const spd_row_stats* stats,
                         const BoxcarArgs& ba, const WidthPlan& wp, int X, int waves, uint64_t ntiles,
                         hipStream_t s);
hipError_t launch_stream(int dtype, const PlaneArg& pl, bool vec, const spd_row_stats* stats, const BoxcarArgs& ba,
                         const WidthPlan& wp, int waves, uint64_t ntiles, hipStream_t s);
hipError_t launch_zero_count(int64_t* count, hipStream_t s);
hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s);
hipError_t launch_select(const float* snr, const uint8_t* widx, int64_t nrows, int64_t ncols,
                         int64_t stride, const SelectArgs& sa, hipStream_t s);

}  // namespace spd
