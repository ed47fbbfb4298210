// spd_abi.hip -- host side of the C ABI declared in include/spd.h:
// argument validation (before anything is enqueued), launch planning and
// the thread-local error string.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "spd_abi_internal.h"
#include "spd_kernels.h"

namespace spd {

static thread_local std::string g_err;

spd_status fail(spd_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

void clear_error() { g_err.clear(); }

spd_status device_status(hipError_t e, const char* what)
{
    if (e == hipSuccess) return SPD_OK;
    return fail(SPD_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int elem_size(int dtype) { return dtype == SPD_F32 ? 4 : dtype == SPD_F16 ? 2 : 1; }

spd_status check_params(const spd_params* p)
{
    if (!p) return fail(SPD_E_INVALID, "params is NULL");
    if (!p->widths) return fail(SPD_E_INVALID, "widths is NULL");
    if (p->n_widths < 1 || p->n_widths > SPD_MAX_WIDTHS)
        return fail(SPD_E_INVALID, "n_widths=%d outside [1, %d]", p->n_widths, SPD_MAX_WIDTHS);
    if (p->widths[0] < 1) return fail(SPD_E_INVALID, "widths[0]=%d < 1", p->widths[0]);
    for (int i = 1; i < p->n_widths; ++i)
        if (p->widths[i] <= p->widths[i - 1])
            return fail(SPD_E_INVALID, "widths not strictly increasing at index %d", i);
    if (p->widths[p->n_widths - 1] > SPD_MAX_NMAX)
        return fail(SPD_E_INVALID, "largest width %d > %d", p->widths[p->n_widths - 1], SPD_MAX_NMAX);
    if (!isfinite(p->threshold)) return fail(SPD_E_INVALID, "threshold is not finite");
    if (p->scope != SPD_SCOPE_ROW && p->scope != SPD_SCOPE_PLANE)
        return fail(SPD_E_INVALID, "scope=%d unknown", p->scope);
    if (p->sigma_mode < SPD_SIGMA_SQRTN || p->sigma_mode > SPD_SIGMA_LINEAR_LITERAL)
        return fail(SPD_E_INVALID, "sigma_mode=%d unknown", p->sigma_mode);
    if (p->sigma_mode == SPD_SIGMA_AUTO && !(isfinite(p->auto_kappa) && p->auto_kappa >= 0.f))
        return fail(SPD_E_INVALID, "auto_kappa must be finite and >= 0");
    return SPD_OK;
}

spd_status check_plane(const spd_plane* x, const spd_params* p)
{
    if (!x) return fail(SPD_E_INVALID, "plane is NULL");
    if (!x->data) return fail(SPD_E_INVALID, "plane data is NULL");
    if (x->dtype != SPD_F32 && x->dtype != SPD_F16 && x->dtype != SPD_U8)
        return fail(SPD_E_INVALID, "dtype=%d unknown", x->dtype);
    if (x->n_rows < 1) return fail(SPD_E_INVALID, "n_rows=%lld < 1", (long long)x->n_rows);
    if (x->n_rows > 0x7fffffffLL) return fail(SPD_E_INVALID, "n_rows too large");
    if (x->row_stride < x->n_cols)
        return fail(SPD_E_INVALID, "row_stride=%lld < n_cols=%lld", (long long)x->row_stride,
                    (long long)x->n_cols);
    if (((uintptr_t)x->data) % (uintptr_t)elem_size(x->dtype))
        return fail(SPD_E_INVALID, "data pointer not aligned to its element size");
    if (x->dtype == SPD_U8 && (!x->row_scale || !x->row_zero))
        return fail(SPD_E_INVALID, "U8 plane needs row_scale and row_zero");
    const int nmax = p->widths[p->n_widths - 1];
    if (x->n_cols < nmax)
        return fail(SPD_E_INVALID, "n_cols=%lld shorter than the widest boxcar %d", (long long)x->n_cols, nmax);
    return SPD_OK;
}

PlaneArg plane_arg(const spd_plane* x)
{
    PlaneArg a;
    a.data = x->data;
    a.n_rows = x->n_rows;
    a.n_cols = x->n_cols;
    a.stride = x->row_stride;
    a.scale = x->row_scale;
    a.zero = x->row_zero;
    return a;
}

bool plane_vec_ok(const spd_plane* x)
{
    const uintptr_t need = 4u * (uintptr_t)elem_size(x->dtype);
    return ((uintptr_t)x->data % need) == 0 && (x->row_stride % 4) == 0;
}

MsdLayout msd_layout(const spd_plane* x)
{
    MsdLayout m;
    const int64_t total = x->n_rows * x->n_cols;
    // at least 16384 columns per block, so each of its four waves walks at least
    // 4096 (whole steps of the widest-boxcar pass); at most 16384 blocks
    int64_t bc = 16384;
    while (bc < 65536 && (total + bc - 1) / bc > 16384) bc <<= 1;
    m.bc = bc;
    m.nblk = (x->n_cols + bc - 1) / bc;
    m.ws_bytes = (size_t)x->n_rows * (size_t)m.nblk * 6 * sizeof(double);
    return m;
}

// The register-window form of the boxcar kernel (8 consecutive starts per
// lane): used for the list 1..n with n <= 16, and for lists of whole groups of
// 8 unit-count widths that each step by 1 or 2 through one array from an
// offset that is a multiple of 8.  Leaves wp.win = 0 when neither applies or
// the padded window does not fit.
static void plan_window(const int* W, int n, bool unit, int X, size_t lds_cap, WidthPlan& wp, BoxcarArgs& ba,
                        int& waves)
{
    if (X != kWinX || !unit) return;
    bool contiguous = n <= 16;
    for (int i = 0; i < n && contiguous; ++i) contiguous = W[i] == i + 1;
    int kind = contiguous ? 2 : 0;
    if (!kind && n % kGroup == 0) {
        kind = 1;
        for (int g = 0; g < n / kGroup && kind; ++g) {
            const int i0 = g * kGroup;
            const int o = i0 ? W[i0 - 1] : 0;
            const int d = W[i0] - o;
            if (o % 8 != 0 || (d != 1 && d != 2)) kind = 0;
            for (int j = 1; j < kGroup && kind; ++j)
                if (W[i0 + j] - W[i0 + j - 1] != d) kind = 0;
            int arr = -1;
            for (int a = 0; a < wp.n_arr; ++a)
                if (wp.arr_gap[a] == d) arr = a;
            if (arr < 0) kind = 0;
        }
    }
    if (!kind) return;
    const int nlog = 64 * X + std::max(wp.nmax, kind == 2 ? 16 : 0) + 8;
    const int npp = (nlog + 7) / 8 * 9;
    const int n_arr = kind == 2 ? 1 : wp.n_arr;
    // the region also holds the epilogue's transpose (64X floats + 64X bytes); 16-byte multiple
    const int wave_floats = (std::max(n_arr * npp, 64 * X + 16 * X) + 3) & ~3;
    const size_t per_wave = (size_t)wave_floats * 4;
    const size_t tables = (size_t)kWinTableFloats * 4;
    if (tables + per_wave > lds_cap) return;
    for (int g = 0; g < (kind == 1 ? n / kGroup : 0); ++g) {
        const int i0 = g * kGroup;
        const int o = i0 ? W[i0 - 1] : 0;
        const int d = W[i0] - o;
        int arr = 0;
        for (int a = 0; a < wp.n_arr; ++a)
            if (wp.arr_gap[a] == d) arr = a;
        wp.gbase[g] = (uint32_t)(arr * npp + win_phys(o));
        wp.gstep[g] = (uint8_t)d;
    }
    wp.win = kind;
    wp.n_arr = n_arr;
    ba.npw = npp;
    ba.wave_floats = wave_floats;
    waves = (int)std::min<size_t>(4, (lds_cap - tables) / per_wave);
}

// Presummed LDS arrays and per-width steps for the boxcar kernel.
bool build_width_plan(const spd_params* p, int X, WidthPlan& wp, BoxcarArgs& ba, int& waves, size_t lds_reserve,
                      bool window)
{
    const int n = p->n_widths;
    const int* W = p->widths;
    memset(&wp, 0, sizeof wp);
    wp.n = n;
    wp.nmax = W[n - 1];
    wp.n_groups = (n + kGroup - 1) / kGroup;
    std::map<int, int> freq;
    for (int i = 0; i < n; ++i) {
        const int g = W[i] - (i ? W[i - 1] : 0);
        if (g > 1) freq[g]++;
    }
    std::vector<std::pair<int, int>> cand(freq.begin(), freq.end());
    std::sort(cand.begin(), cand.end(), [](const std::pair<int, int>& a, const std::pair<int, int>& b) {
        return a.second != b.second ? a.second > b.second : a.first < b.first;
    });
    std::vector<int> gaps{1};
    for (auto& c : cand)
        if (c.second >= 2 && c.first <= 16 && (int)gaps.size() < kMaxArrays) gaps.push_back(c.first);

    const int np = 64 * X + wp.nmax - 1;
    const int npw = (np + 3) & ~3;
    const size_t tables = (size_t)kTableFloats * 4;
    const size_t lds_cap = 65536 - lds_reserve;
    for (;;) {
        const size_t per_wave = (size_t)gaps.size() * npw * 4;
        if (tables + per_wave <= lds_cap || gaps.size() == 1) break;
        gaps.pop_back();
    }
    const size_t per_wave = (size_t)gaps.size() * npw * 4;
    if (tables + per_wave > lds_cap) return false;
    waves = (int)std::min<size_t>(4, (lds_cap - tables) / per_wave);
    wp.n_arr = (int)gaps.size();
    for (int a = 0; a < wp.n_arr; ++a) wp.arr_gap[a] = gaps[a];
    bool unit = true;
    for (int i = 0; i < n; ++i) {
        const int prev = i ? W[i - 1] : 0;
        const int g = W[i] - prev;
        int best = 0;
        for (int a = 0; a < wp.n_arr; ++a)
            if (g % gaps[a] == 0 && gaps[a] > gaps[best]) best = a;
        const int cnt = g / gaps[best];
        if (cnt != 1) unit = false;
        wp.off[i] = (uint32_t)(best * npw + prev);
        wp.cg[i] = (uint32_t)cnt | ((uint32_t)gaps[best] << 16);
        wp.width[i] = (int16_t)W[i];
    }
    wp.unit_counts = unit ? 1 : 0;
    ba.npw = npw;
    ba.wave_floats = wp.n_arr * npw;
    wp.win = 0;
    if (window) plan_window(W, n, unit, X, lds_cap, wp, ba, waves);
    return true;
}

spd_status check_msd_workspace(const spd_plane* x, const MsdLayout& m, const void* workspace, size_t bytes)
{
    if (!workspace) return fail(SPD_E_INVALID, "workspace is NULL");
    if (((uintptr_t)workspace) % 256) return fail(SPD_E_INVALID, "workspace not 256-byte aligned");
    if (bytes < m.ws_bytes) return fail(SPD_E_NOMEM, "workspace %zu bytes < %zu needed", bytes, m.ws_bytes);
    if ((uint64_t)x->n_rows * (uint64_t)m.nblk * 256u > kMaxGridItems)
        return fail(SPD_E_UNSUPPORTED, "plane too large for one launch (%lld blocks)",
                    (long long)(x->n_rows * m.nblk));
    return SPD_OK;
}

// Block partials (Sec. 2.1) then the FP64 merge and sigma_N coefficients
// (Sec. 2.1-2.2) of every unit of x, on s.  Arguments already validated.
spd_status enqueue_msd(const spd_plane* x, const spd_params* p, int64_t new_col_begin, bool accumulate,
                       spd_msd_state* state, spd_row_stats* stats, double* part, const MsdLayout& m, hipStream_t s)
{
    const int nmax = p->widths[p->n_widths - 1];
    const int64_t nout = x->n_cols - nmax + 1;
    const bool need_y = p->sigma_mode != SPD_SIGMA_SQRTN;
    hipError_t e = launch_msd(x->dtype, plane_arg(x), plane_vec_ok(x), need_y, new_col_begin, m.bc, m.nblk,
                              nmax, nout, part, s);
    if (e != hipSuccess) return device_status(e, "msd partial launch");
    const bool plane = p->scope == SPD_SCOPE_PLANE;
    const int64_t units = plane ? 1 : x->n_rows;
    const int64_t per_unit = plane ? x->n_rows * m.nblk : m.nblk;
    e = launch_finalize(part, units, per_unit, need_y, accumulate, state, stats, nmax, p->sigma_mode,
                        (double)p->auto_kappa, s);
    return device_status(e, "msd finalize launch");
}

// Validates the boxcar outputs and fills the launch plan for the whole plane.
spd_status plan_boxcar(const spd_plane* x, const spd_params* p, const spd_row_stats* stats, float* snr_out,
                       uint8_t* widx_out, int64_t out_stride, int64_t t_offset, spd_candidate* cand,
                       int64_t cand_capacity, int64_t* cand_count, BoxcarPlan& bp)
{
    if (!stats) return fail(SPD_E_INVALID, "stats is NULL");
    if (!snr_out && !widx_out && !cand) return fail(SPD_E_INVALID, "no output requested");
    const int nmax = p->widths[p->n_widths - 1];
    const int64_t nout = x->n_cols - nmax + 1;
    if ((snr_out || widx_out) && out_stride < nout)
        return fail(SPD_E_INVALID, "out_stride=%lld < %lld outputs per row", (long long)out_stride, (long long)nout);
    if (cand && (!cand_count || cand_capacity < 0))
        return fail(SPD_E_INVALID, "candidate list needs cand_count and capacity >= 0");
    const int X = kOutPerLane;
    memset(&bp.ba, 0, sizeof bp.ba);
    bp.waves = 4;
    const char* form = getenv("SPD_BOXCAR_FORM");          // "strided": never the register-window form
    const bool window = !(form && strcmp(form, "strided") == 0);
    if (!build_width_plan(p, X, bp.wp, bp.ba, bp.waves, 0, window))
        return fail(SPD_E_UNSUPPORTED, "width list does not fit in LDS");
    BoxcarArgs& ba = bp.ba;
    ba.scope = p->scope;
    ba.nout = nout;
    ba.tiles_per_row = (nout + (int64_t)bp.waves * 64 * X - 1) / ((int64_t)bp.waves * 64 * X);
    // the list 1..n (n <= 16): streaming form ("window": the register-window tiles)
    if (bp.wp.win == 2 && !(form && strcmp(form, "window") == 0)) {
        bp.wp.win = 4;
        bp.waves = 4;
        ba.tiles_per_row = (nout + bp.waves * kStreamRun - 1) / (bp.waves * kStreamRun);
    }
    ba.snr = snr_out;
    ba.widx = widx_out;
    ba.out_stride = out_stride;
    ba.t_offset = t_offset;
    ba.cand = cand;
    ba.cand_capacity = cand_capacity;
    ba.cand_count = cand_count;
    ba.threshold = p->threshold;
    ba.out_vec = ((snr_out && (uintptr_t)snr_out % 16 == 0 && out_stride % 4 == 0) ? 1u : 0u) |
                 ((widx_out && (uintptr_t)widx_out % 8 == 0 && out_stride % 8 == 0) ? 2u : 0u) |
                 ((widx_out && (uintptr_t)widx_out % 4 == 0 && out_stride % 4 == 0) ? 4u : 0u);
    const uint64_t ntiles = (uint64_t)x->n_rows * (uint64_t)ba.tiles_per_row;
    if (ntiles * 64u * (uint64_t)bp.waves > kMaxGridItems) return fail(SPD_E_UNSUPPORTED, "plane too large for one launch");
    return SPD_OK;
}

// Boxcar launch over rows [r0, r0 + rows) of the plan's plane; x is that row
// range as its own plane and stats its first unit.
spd_status enqueue_boxcar(const spd_plane* x, const spd_row_stats* stats, const BoxcarPlan& bp, int64_t r0,
                          int64_t rows, hipStream_t s)
{
    BoxcarArgs ba = bp.ba;
    ba.row0 = (int32_t)r0;
    if (ba.snr) ba.snr += r0 * ba.out_stride;
    if (ba.widx) ba.widx += r0 * ba.out_stride;
    const uint64_t ntiles = (uint64_t)rows * (uint64_t)ba.tiles_per_row;
    hipError_t e = launch_boxcar(x->dtype, plane_arg(x), plane_vec_ok(x), stats, ba, bp.wp, kOutPerLane, bp.waves,
                                 ntiles, s);
    return device_status(e, "boxcar launch");
}

// Rows [r0, r0 + rows) of x as a plane of their own.
spd_plane row_slice(const spd_plane* x, int64_t r0, int64_t rows)
{
    spd_plane sub = *x;
    sub.data = (const char*)x->data + (size_t)(r0 * x->row_stride) * (size_t)elem_size(x->dtype);
    sub.n_rows = rows;
    if (x->row_scale) sub.row_scale = x->row_scale + r0;
    if (x->row_zero) sub.row_zero = x->row_zero + r0;
    return sub;
}

// One fork event and one event per chunk, per thread and device, created on
// first use and kept for the life of the thread.  A stream wait binds to the
// record that precedes it, so the events can be recorded again by the next call.
spd_status detect_events(hipEvent_t** out)
{
    struct Events {
        int device = -1;
        std::vector<hipEvent_t> ev;
    };
    static thread_local std::vector<Events> cache;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_status(e, "hipGetDevice");
    for (auto& c : cache)
        if (c.device == dev) { *out = c.ev.data(); return SPD_OK; }
    Events c;
    c.device = dev;
    c.ev.assign(SPD_MAX_ROW_CHUNKS + 1, nullptr);
    for (auto& h : c.ev) {
        if ((e = hipEventCreateWithFlags(&h, hipEventDisableTiming)) != hipSuccess) {
            for (auto& g : c.ev)
                if (g) hipEventDestroy(g);
            return device_status(e, "event create");
        }
    }
    cache.push_back(std::move(c));
    *out = cache.back().ev.data();
    return SPD_OK;
}

// Scratch of spd_detect_static: the statistics pass's block partials, in a
// device array of fixed size instead of a caller workspace.  Each device that
// runs the entry point holds its own copy until the process ends.  In host
// code `scratch` names a host-side stand-in, so kernels only ever receive the
// device address that hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch array, looked up once per
// device (with that device current) and kept.
spd_status static_scratch(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_status(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(SPD_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return device_status(e, "hipGetSymbolAddress(scratch)");
        if (!ptr || ((uintptr_t)ptr) % 256) return fail(SPD_E_DEVICE, "scratch address %p not 256-byte aligned", ptr);
        g_scratch_ptr[dev] = ptr;
    }
    *out = (double*)g_scratch_ptr[dev];
    return SPD_OK;
}

}  // namespace spd

using namespace spd;

extern "C" {

int spd_abi_version(void) { return SPD_ABI_VERSION; }

const char* spd_last_error(void) { return g_err.c_str(); }

size_t spd_workspace_bytes(const spd_plane* x, const spd_params* p)
{
    clear_error();
    if (check_params(p) || check_plane(x, p)) return 0;
    return msd_layout(x).ws_bytes;
}

spd_status msd_compute(const spd_plane* x, const spd_params* p, int64_t new_col_begin, int32_t accumulate,
                       spd_msd_state* state, spd_row_stats* stats, void* workspace, size_t workspace_bytes,
                       void* stream)
{
    clear_error();
    spd_status st;
    if ((st = check_params(p)) || (st = check_plane(x, p))) return st;
    if (!stats) return fail(SPD_E_INVALID, "stats is NULL");
    if (accumulate && !state) return fail(SPD_E_INVALID, "accumulate=1 needs a state");
    if (new_col_begin < 0 || new_col_begin > x->n_cols)
        return fail(SPD_E_INVALID, "new_col_begin=%lld outside [0, n_cols]", (long long)new_col_begin);
    const MsdLayout m = msd_layout(x);
    if ((st = check_msd_workspace(x, m, workspace, workspace_bytes))) return st;
    return enqueue_msd(x, p, new_col_begin, accumulate != 0, state, stats, (double*)workspace, m,
                       (hipStream_t)stream);
}

spd_status boxcar_snr(const spd_plane* x, const spd_params* p, const spd_row_stats* stats, float* snr_out,
                      uint8_t* widx_out, int64_t out_stride, int64_t t_offset, spd_candidate* cand,
                      int64_t cand_capacity, int64_t* cand_count, void* stream)
{
    clear_error();
    spd_status st;
    if ((st = check_params(p)) || (st = check_plane(x, p))) return st;
    BoxcarPlan bp;
    if ((st = plan_boxcar(x, p, stats, snr_out, widx_out, out_stride, t_offset, cand, cand_capacity, cand_count,
                          bp)))
        return st;
    hipStream_t s = (hipStream_t)stream;
    if (cand) {
        hipError_t e = launch_zero_count(cand_count, s);
        if (e != hipSuccess) return device_status(e, "count reset launch");
    }
    return enqueue_boxcar(x, stats, bp, 0, x->n_rows, s);
}

spd_status spd_detect(const spd_plane* x, const spd_params* p, spd_row_stats* stats, float* snr_out,
                      uint8_t* widx_out, int64_t out_stride, int64_t t_offset, spd_candidate* cand,
                      int64_t cand_capacity, int64_t* cand_count, void* workspace, size_t workspace_bytes,
                      int32_t row_chunks, void* stream, void* aux_stream)
{
    clear_error();
    spd_status st;
    if ((st = check_params(p)) || (st = check_plane(x, p))) return st;
    if (!stats) return fail(SPD_E_INVALID, "stats is NULL");
    if (row_chunks < 1) return fail(SPD_E_INVALID, "row_chunks=%d < 1", row_chunks);
    if (aux_stream && aux_stream == stream) return fail(SPD_E_INVALID, "aux_stream must differ from stream");
    const MsdLayout m = msd_layout(x);
    if ((st = check_msd_workspace(x, m, workspace, workspace_bytes))) return st;
    BoxcarPlan bp;
    if ((st = plan_boxcar(x, p, stats, snr_out, widx_out, out_stride, t_offset, cand, cand_capacity, cand_count,
                          bp)))
        return st;
    hipStream_t s = (hipStream_t)stream, a = (hipStream_t)aux_stream;
    double* part = (double*)workspace;
    const int64_t chunks = std::min<int64_t>(std::min<int64_t>(row_chunks, SPD_MAX_ROW_CHUNKS), x->n_rows);
    const bool pipelined = a && chunks > 1 && p->scope == SPD_SCOPE_ROW;
    hipEvent_t* ev = nullptr;
    if (pipelined && (st = detect_events(&ev))) return st;

    hipError_t e;
    if (cand && (e = launch_zero_count(cand_count, s)) != hipSuccess) return device_status(e, "count reset launch");
    if (!pipelined) {
        if ((st = enqueue_msd(x, p, 0, false, nullptr, stats, part, m, s))) return st;
        return enqueue_boxcar(x, stats, bp, 0, x->n_rows, s);
    }
    // fork: the statistics stream starts after everything already on `stream`
    if ((e = hipEventRecord(ev[0], s)) != hipSuccess) return device_status(e, "event record");
    if ((e = hipStreamWaitEvent(a, ev[0], 0)) != hipSuccess) return device_status(e, "stream wait");
    const int64_t per = (x->n_rows + chunks - 1) / chunks;
    int k = 0;
    for (int64_t r0 = 0; r0 < x->n_rows; r0 += per, ++k) {
        const int64_t rc = std::min<int64_t>(per, x->n_rows - r0);
        const spd_plane sub = row_slice(x, r0, rc);
        // the chunk's partials use the whole plane's block layout, so they fit the workspace
        if ((st = enqueue_msd(&sub, p, 0, false, nullptr, stats + r0, part, m, a))) return st;
        if ((e = hipEventRecord(ev[k + 1], a)) != hipSuccess) return device_status(e, "event record");
        if ((e = hipStreamWaitEvent(s, ev[k + 1], 0)) != hipSuccess) return device_status(e, "stream wait");
        if ((st = enqueue_boxcar(&sub, stats + r0, bp, r0, rc, s))) return st;
    }
    return SPD_OK;
}

spd_status spd_detect_static(const spd_plane* x, const spd_params* p, spd_row_stats* stats, float* snr_out,
                             uint8_t* widx_out, int64_t out_stride, int64_t t_offset, spd_candidate* cand,
                             int64_t cand_capacity, int64_t* cand_count, void* stream)
{
    clear_error();
    spd_status st;
    if ((st = check_params(p)) || (st = check_plane(x, p))) return st;
    if (!stats) return fail(SPD_E_INVALID, "stats is NULL");
    const MsdLayout m = msd_layout(x);
    if (m.ws_bytes > kStaticScratchBytes)
        return fail(SPD_E_UNSUPPORTED,
                    "plane needs %zu bytes of block partials, more than the %zu-byte static scratch "
                    "(%lld rows x %lld blocks); use spd_detect with a workspace",
                    m.ws_bytes, kStaticScratchBytes, (long long)x->n_rows, (long long)m.nblk);
    if ((uint64_t)x->n_rows * (uint64_t)m.nblk * 256u > kMaxGridItems)
        return fail(SPD_E_UNSUPPORTED, "plane too large for one launch");
    BoxcarPlan bp;
    if ((st = plan_boxcar(x, p, stats, snr_out, widx_out, out_stride, t_offset, cand, cand_capacity, cand_count,
                          bp)))
        return st;
    double* part = nullptr;
    if ((st = static_scratch(&part))) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (cand && (e = launch_zero_count(cand_count, s)) != hipSuccess) return device_status(e, "count reset launch");
    if ((st = enqueue_msd(x, p, 0, false, nullptr, stats, part, m, s))) return st;
    return enqueue_boxcar(x, stats, bp, 0, x->n_rows, s);
}

spd_status boxcar_snr_dit(const spd_plane* x, const spd_params* p, int32_t levels, const spd_row_stats* stats,
                          float* snr_out, uint8_t* widx_out, int64_t out_stride, int64_t t_offset,
                          spd_candidate* cand, int64_t cand_capacity, int64_t* cand_count, void* stream)
{
    clear_error();
    spd_status st;
    if ((st = check_params(p)) || (st = check_plane(x, p))) return st;
    if (levels < 0 || levels > kDitMaxLevels)
        return fail(SPD_E_INVALID, "levels=%d outside [0, %d]", levels, kDitMaxLevels);
    const int n = kDitBase + (kDitBase / 2) * levels;
    bool ok = p->n_widths == n;
    for (int i = 0; i < n && ok; ++i) {
        const int lv = i < kDitBase ? 0 : 1 + (i - kDitBase) / (kDitBase / 2);
        const int w = i < kDitBase ? i + 1 : (kDitBase / 2 + 1 + (i - kDitBase) % (kDitBase / 2)) << lv;
        ok = p->widths[i] == w;
    }
    if (!ok) return fail(SPD_E_INVALID, "widths must be 1..16, then 2^l*(9..16) for l = 1..levels");
    BoxcarPlan bp;
    if ((st = plan_boxcar(x, p, stats, snr_out, widx_out, out_stride, t_offset, cand, cand_capacity, cand_count,
                          bp)))
        return st;
    // the decimated layout: x' in padded rows of 9, then one region per level
    WidthPlan& wp = bp.wp;
    BoxcarArgs& ba = bp.ba;
    const int X = kWinX;
    const int nlog = 64 * X + wp.nmax + 8;
    const int npw = (nlog + 7) / 8 * 9;
    int wave_floats = npw;
    for (int lv = 1; lv <= levels; ++lv) wave_floats += dit_level_floats(levels, lv);
    wave_floats = (std::max(wave_floats, 64 * X + 16 * X) + 3) & ~3;
    const size_t tables = (size_t)kWinTableFloats * 4;
    if (tables + (size_t)wave_floats * 4 > 65536) return fail(SPD_E_UNSUPPORTED, "decimated window does not fit in LDS");
    wp.win = 3;
    wp.n_arr = 1;
    ba.npw = npw;
    ba.wave_floats = wave_floats;
    bp.waves = (int)std::min<size_t>(4, (65536 - tables) / ((size_t)wave_floats * 4));
    ba.tiles_per_row = (ba.nout + (int64_t)bp.waves * 64 * X - 1) / ((int64_t)bp.waves * 64 * X);
    if ((uint64_t)x->n_rows * (uint64_t)ba.tiles_per_row * 64u * (uint64_t)bp.waves > kMaxGridItems)
        return fail(SPD_E_UNSUPPORTED, "plane too large for one launch");
    hipStream_t s = (hipStream_t)stream;
    if (cand) {
        hipError_t e = launch_zero_count(cand_count, s);
        if (e != hipSuccess) return device_status(e, "count reset launch");
    }
    return enqueue_boxcar(x, stats, bp, 0, x->n_rows, s);
}

spd_status select_candidates(const float* snr, const uint8_t* widx, int64_t n_rows, int64_t n_out_cols,
                             int64_t out_stride, const spd_params* p, int64_t t_offset, spd_candidate* cand,
                             int64_t cand_capacity, int64_t* cand_count, void* stream)
{
    clear_error();
    spd_status st;
    if ((st = check_params(p))) return st;
    if (!snr || !widx) return fail(SPD_E_INVALID, "snr and widx are required");
    if (n_rows < 1 || n_out_cols < 0) return fail(SPD_E_INVALID, "bad shape");
    if (out_stride < n_out_cols) return fail(SPD_E_INVALID, "out_stride < n_out_cols");
    if (!cand || !cand_count || cand_capacity < 0)
        return fail(SPD_E_INVALID, "candidate list needs cand, cand_count and capacity >= 0");
    if ((uint64_t)n_rows * (uint64_t)((n_out_cols + kSelCols - 1) / kSelCols) * 256u > kMaxGridItems)
        return fail(SPD_E_UNSUPPORTED, "output too large for one launch");
    SelectArgs sa;
    memset(&sa, 0, sizeof sa);
    for (int i = 0; i < p->n_widths; ++i) sa.width[i] = p->widths[i];
    sa.threshold = p->threshold;
    sa.t_offset = t_offset;
    sa.cand = cand;
    sa.cand_capacity = cand_capacity;
    sa.cand_count = cand_count;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_zero_count(cand_count, s);
    if (e != hipSuccess) return device_status(e, "count reset launch");
    e = launch_select(snr, widx, n_rows, n_out_cols, out_stride, sa, s);
    return device_status(e, "select launch");
}

}  // extern "C"
