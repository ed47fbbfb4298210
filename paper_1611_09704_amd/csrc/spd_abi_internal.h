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
                      size_t lds_reserve = 0);

}  // namespace spd
