// spd_serve.hip -- real-time serving of the detection path over streams of
// chunks from several beams (Sec. 2.1-2.4 applied chunk by chunk).
//
// Each beam streams consecutive chunks of [n_rows][chunk_cols] new samples.
// The server keeps, per beam and on the device:
//   - the running FP64 statistics (Eq. MSD04 merges each chunk's partials), so
//     mean and sigma cover every sample received so far;
//   - the last Nmax-1 columns of the previous chunk (the halo), placed in front
//     of the next chunk so every boxcar window that ends in the new chunk is
//     evaluated exactly once;
//   - `slots_per_beam` chunk buffers, so the host-to-device copy of chunk k+1
//     overlaps the work on chunk k.
// Requests are admitted as soon as their beam has a free slot and every
// earlier chunk of the beam has been admitted (continuous batching: nothing
// waits for a batch to fill).  Each beam has its own compute stream, so chunks
// of different beams run concurrently on the device while chunks of one beam
// stay in order; copies run on per-beam copy streams, a chunk in row groups
// whose statistics and boxcars start as soon as their rows have arrived.  A
// worker thread admits requests and detects completions; spd_server_poll
// hands finished chunks out.
//
// With a de-dispersion plan in front (spd_server_create_dedisp) a beam streams
// 8-bit filterbank chunks instead.  The server also keeps the beam's last
// max-delay filterbank columns (rounded up to 4 bytes), de-disperses
// [filterbank halo | chunk] into the beam's DM-trial x time plane right
// behind its detection halo, and runs the detection stream on that plane.
// Chunk 0 yields chunk_cols - max_delay new de-dispersed starts, every later
// chunk chunk_cols (global starts k * chunk_cols - max_delay onwards).
#include <hip/hip_runtime.h>

#include <string.h>

#include <chrono>
#include <algorithm>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "spd_abi_internal.h"
#include "spd_kernels.h"

namespace spd {

// A chunk without de-dispersion in front is copied in this many row groups;
// each group's statistics and boxcars start as soon as its rows have arrived
// (rows are independent under per-row statistics), so a chunk's latency is
// close to its copy time plus the work of one group.
constexpr int kServeRowGroups = 4;

static double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct ServeReq {
    int beam = 0;
    int64_t seq = 0;
    const void* host = nullptr;
    double submit_s = 0.0, start_s = 0.0, done_s = 0.0;
    int slot = 0;
};

struct ServeDone {
    spd_server_result res;
    std::vector<spd_candidate> cands;
};

struct ServeBeam {
    std::deque<ServeReq> pending;          // submitted, not admitted
    std::deque<ServeReq> inflight;         // admitted, not complete (in order)
    int64_t next_submit = 0;               // next sequence number accepted
    std::vector<void*> buf;                // [slots] device [n_rows][H + C]
    std::vector<void*> stage;              // [slots] device [n_rows][C], the contiguous copy-in target
    std::vector<void*> fb;                 // [slots] device [n_chan][fb_pitch] filterbank (de-dispersion)
    std::vector<spd_candidate*> d_cand;    // [slots]
    std::vector<int64_t*> d_count;
    std::vector<spd_candidate*> h_cand;    // pinned
    std::vector<int64_t*> h_count;
    std::vector<hipEvent_t> h2d_done;      // [slots][kServeRowGroups]: a row group of the chunk is on the device
    std::vector<hipEvent_t> free_ev, done_ev;
    spd_msd_state* state = nullptr;
    spd_row_stats* stats = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr, copy = nullptr;
};

}  // namespace spd

struct spd_server {
    spd_server_config cfg{};
    std::vector<int32_t> widths;
    spd_params params{};
    int device = 0;
    int esize = 4;                         // bytes per sample of the detection plane
    int in_esize = 4;                      // bytes per sample of a submitted chunk
    int64_t halo = 0;                      // Nmax - 1
    int64_t det_rows = 0;                  // rows of the detection plane (n_rows, or the plan's trials)
    const spd_dedisp_plan* dd = nullptr;   // de-dispersion in front, or none
    int64_t dd_delay = 0;                  // the plan's largest delay (samples)
    int64_t dd_halo = 0;                   // filterbank columns kept: dd_delay rounded up to 4
    int64_t fb_pitch = 0;                  // bytes per filterbank row in a slot
    std::vector<spd::ServeBeam> beams;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<spd::ServeDone> done;
    std::thread worker;
    bool stop = false;
    spd_status fault = SPD_OK;
    std::string fault_msg;
    int64_t n_submitted = 0, n_admitted = 0, n_completed = 0;
};

namespace spd {

// New detection-plane columns chunk `seq` brings, and the global index of the
// first of them.
static int64_t new_cols(const spd_server* S, int64_t seq)
{
    return S->dd && seq == 0 ? S->cfg.chunk_cols - S->dd_delay : S->cfg.chunk_cols;
}

static int64_t first_col(const spd_server* S, int64_t seq)
{
    return S->dd && seq > 0 ? seq * S->cfg.chunk_cols - S->dd_delay : seq * S->cfg.chunk_cols;
}

// Global start of the chunk's first window (the halo's first column after chunk 0).
static int64_t chunk_t_offset(const spd_server* S, int64_t seq)
{
    return seq == 0 ? 0 : first_col(S, seq) - S->halo;
}

static spd_plane view_plane(const spd_server* S, const ServeBeam& b, int slot, int64_t seq)
{
    spd_plane x;
    memset(&x, 0, sizeof x);
    const int64_t pitch = S->halo + S->cfg.chunk_cols;
    const char* base = (const char*)b.buf[slot];
    if (seq == 0) {                                 // first chunk: no halo in front
        x.data = base + S->halo * S->esize;
        x.n_cols = new_cols(S, 0);
    } else {
        x.data = base;
        x.n_cols = pitch;
    }
    x.dtype = S->dd ? SPD_F32 : S->cfg.dtype;
    x.n_rows = S->det_rows;
    x.row_stride = pitch;
    return x;
}

// De-dispersion of one chunk on the beam's compute stream: re-pitch the
// staged bytes behind the filterbank halo, de-disperse into the detection
// plane behind its halo, and hand the last dd_halo filterbank columns on to
// the next slot.  After chunk 0 the view starts dd_halo - dd_delay (< 4)
// columns early so that its rows stay 4-byte aligned; those first outputs
// repeat the previous chunk's last ones exactly (whole-count sums) and land
// on the same columns of the detection halo.
static spd_status dedisperse_chunk(spd_server* S, ServeBeam& b, int slot, int64_t seq)
{
    const int64_t C = S->cfg.chunk_cols, Hf = S->dd_halo, R = S->cfg.n_rows, H = S->halo;
    char* fb = (char*)b.fb[slot];
    hipError_t e = hipMemcpy2DAsync(fb + Hf, (size_t)S->fb_pitch, b.stage[slot], (size_t)C, (size_t)C, (size_t)R,
                                    hipMemcpyDeviceToDevice, b.stream);
    if (e != hipSuccess) return device_status(e, "filterbank re-pitch");
    spd_plane f;
    memset(&f, 0, sizeof f);
    f.dtype = SPD_U8;
    f.n_rows = R;
    f.row_stride = S->fb_pitch;
    f.data = seq == 0 ? fb + Hf : fb;
    f.n_cols = seq == 0 ? C : Hf + C;
    const int64_t lead = seq == 0 ? 0 : Hf - S->dd_delay;
    float* out = (float*)b.buf[slot] + (H - lead);
    spd_status st = spd_dedisperse(S->dd, &f, out, H + C, b.stream);
    if (st) return st;
    e = hipMemcpy2DAsync((char*)b.fb[(slot + 1) % S->cfg.slots_per_beam], (size_t)S->fb_pitch, fb + C,
                         (size_t)S->fb_pitch, (size_t)Hf, (size_t)R, hipMemcpyDeviceToDevice, b.stream);
    return device_status(e, "filterbank halo copy");
}

// Enqueue one admitted chunk: copy in, statistics, boxcar/SNR with the fused
// threshold, halo hand-over to the next slot, candidates back to the host.
static spd_status launch_chunk(spd_server* S, ServeReq& r)
{
    ServeBeam& b = S->beams[r.beam];
    const int slots = S->cfg.slots_per_beam;
    const int slot = (int)(r.seq % slots);
    r.slot = slot;
    const int64_t C = S->cfg.chunk_cols, H = S->halo, R = S->cfg.n_rows, D = S->det_rows;
    const size_t pitch_b = (size_t)(H + C) * S->esize;
    char* base = (char*)b.buf[slot];
    hipError_t e;
    // the slot's previous chunk has handed its halo on and is finished
    if ((e = hipStreamWaitEvent(b.copy, b.free_ev[slot], 0)) != hipSuccess) return device_status(e, "wait free");
    spd_status st;
    const spd_plane x = view_plane(S, b, slot, r.seq);
    if (S->dd) {
        // de-dispersion needs every channel: one contiguous host-to-device copy
        e = hipMemcpyAsync(b.stage[slot], r.host, (size_t)R * C * S->in_esize, hipMemcpyHostToDevice, b.copy);
        if (e != hipSuccess) return device_status(e, "chunk copy-in");
        hipEvent_t h2d = b.h2d_done[(size_t)slot * kServeRowGroups];
        if ((e = hipEventRecord(h2d, b.copy)) != hipSuccess) return device_status(e, "record h2d");
        if ((e = hipStreamWaitEvent(b.stream, h2d, 0)) != hipSuccess) return device_status(e, "wait h2d");
        if ((st = dedisperse_chunk(S, b, slot, r.seq))) return st;
        st = msd_compute(&x, &S->params, r.seq == 0 ? 0 : H, r.seq == 0 ? 0 : 1, b.state, b.stats, b.ws, b.ws_bytes,
                         b.stream);
        if (st) return st;
        st = boxcar_snr(&x, &S->params, b.stats, nullptr, nullptr, 0, chunk_t_offset(S, r.seq), b.d_cand[slot],
                        S->cfg.cand_capacity, b.d_count[slot], b.stream);
        if (st) return st;
    } else {
        // row groups: each is one contiguous host-to-device copy (full link speed), then a
        // pitched device-to-device copy behind the halo columns, its statistics (the whole
        // view's block layout, so the partials fit the workspace) and its boxcars
        const MsdLayout m = msd_layout(&x);
        if ((st = check_msd_workspace(&x, m, b.ws, b.ws_bytes))) return st;
        BoxcarPlan bp;
        if ((st = plan_boxcar(&x, &S->params, b.stats, nullptr, nullptr, 0, chunk_t_offset(S, r.seq), b.d_cand[slot],
                              S->cfg.cand_capacity, b.d_count[slot], bp)))
            return st;
        if ((e = launch_zero_count(b.d_count[slot], b.stream)) != hipSuccess) return device_status(e, "count reset");
        const int64_t per = (R + kServeRowGroups - 1) / kServeRowGroups;
        for (int g = 0; g < kServeRowGroups; ++g) {
            const int64_t r0 = (int64_t)g * per, rows = std::min<int64_t>(per, R - r0);
            if (rows <= 0) break;
            const size_t in_off = (size_t)r0 * (size_t)C * S->in_esize;
            e = hipMemcpyAsync((char*)b.stage[slot] + in_off, (const char*)r.host + in_off,
                               (size_t)rows * (size_t)C * S->in_esize, hipMemcpyHostToDevice, b.copy);
            if (e != hipSuccess) return device_status(e, "chunk copy-in");
            hipEvent_t h2d = b.h2d_done[(size_t)slot * kServeRowGroups + g];
            if ((e = hipEventRecord(h2d, b.copy)) != hipSuccess) return device_status(e, "record h2d");
            if ((e = hipStreamWaitEvent(b.stream, h2d, 0)) != hipSuccess) return device_status(e, "wait h2d");
            e = hipMemcpy2DAsync(base + (size_t)r0 * pitch_b + H * S->esize, pitch_b, (char*)b.stage[slot] + in_off,
                                 (size_t)C * S->esize, (size_t)C * S->esize, (size_t)rows, hipMemcpyDeviceToDevice,
                                 b.stream);
            if (e != hipSuccess) return device_status(e, "chunk re-pitch");
            const spd_plane sub = row_slice(&x, r0, rows);
            if ((st = enqueue_msd(&sub, &S->params, r.seq == 0 ? 0 : H, r.seq != 0, b.state + r0, b.stats + r0,
                                  (double*)b.ws, m, b.stream)))
                return st;
            if ((st = enqueue_boxcar(&sub, b.stats + r0, bp, r0, rows, b.stream))) return st;
        }
    }
    if (H > 0) {                                    // last H columns become the next chunk's halo
        char* next = (char*)b.buf[(slot + 1) % slots];
        e = hipMemcpy2DAsync(next, pitch_b, base + new_cols(S, r.seq) * S->esize, pitch_b, (size_t)H * S->esize,
                             (size_t)D, hipMemcpyDeviceToDevice, b.stream);
        if (e != hipSuccess) return device_status(e, "halo copy");
    }
    if ((e = hipEventRecord(b.free_ev[slot], b.stream)) != hipSuccess) return device_status(e, "record free");
    e = hipMemcpyAsync(b.h_count[slot], b.d_count[slot], sizeof(int64_t), hipMemcpyDeviceToHost, b.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b.h_cand[slot], b.d_cand[slot], sizeof(spd_candidate) * (size_t)S->cfg.cand_capacity,
                           hipMemcpyDeviceToHost, b.stream);
    if (e != hipSuccess) return device_status(e, "candidates copy-out");
    if ((e = hipEventRecord(b.done_ev[slot], b.stream)) != hipSuccess) return device_status(e, "record done");
    return SPD_OK;
}

static void worker_loop(spd_server* S)
{
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (!S->stop) {
        bool progress = false;
        // admission: in order per beam, while the beam has a free slot
        for (size_t bi = 0; bi < S->beams.size() && S->fault == SPD_OK; ++bi) {
            ServeBeam& b = S->beams[bi];
            while (!b.pending.empty() && (int)b.inflight.size() < S->cfg.slots_per_beam) {
                ServeReq r = b.pending.front();
                b.pending.pop_front();
                r.start_s = now_s();
                const spd_status st = launch_chunk(S, r);
                if (st) {
                    S->fault = st;
                    S->fault_msg = spd_last_error();
                    break;
                }
                b.inflight.push_back(r);
                ++S->n_admitted;
                progress = true;
            }
        }
        // completions: the oldest in-flight chunk of each beam
        for (size_t bi = 0; bi < S->beams.size(); ++bi) {
            ServeBeam& b = S->beams[bi];
            while (!b.inflight.empty()) {
                ServeReq& r = b.inflight.front();
                const hipError_t q = hipEventQuery(b.done_ev[r.slot]);
                if (q == hipErrorNotReady) break;
                ServeDone d;
                memset(&d.res, 0, sizeof d.res);
                d.res.beam = r.beam;
                d.res.seq = r.seq;
                d.res.submit_s = r.submit_s;
                d.res.start_s = r.start_s;
                d.res.done_s = now_s();
                d.res.t_offset = chunk_t_offset(S, r.seq);
                if (q != hipSuccess) {
                    d.res.status = SPD_E_DEVICE;
                } else {
                    const int64_t n = *b.h_count[r.slot];
                    d.res.n_cands = n;
                    d.res.status = n > S->cfg.cand_capacity ? SPD_E_NOMEM : SPD_OK;
                    const int64_t k = n < S->cfg.cand_capacity ? n : S->cfg.cand_capacity;
                    d.cands.assign(b.h_cand[r.slot], b.h_cand[r.slot] + k);
                    for (auto& c : d.cands) c.beam = (uint32_t)r.beam;
                }
                S->done.push_back(std::move(d));
                b.inflight.pop_front();
                ++S->n_completed;
                progress = true;
            }
        }
        if (progress) {
            S->cv_done.notify_all();
            continue;
        }
        bool busy = false;
        for (auto& b : S->beams) busy = busy || !b.inflight.empty();
        // poll completions every 50 us while work is on the device; otherwise sleep until a submit
        S->cv_work.wait_for(lk, std::chrono::microseconds(busy ? 50 : 20000));
    }
}

// Workspace of msd_compute for both chunk views: the first chunk (no halo,
// chunk_cols columns) and every later one (halo + chunk_cols columns).
static size_t serve_ws_bytes(int64_t rows, int64_t halo, int64_t cols)
{
    spd_plane x;
    memset(&x, 0, sizeof x);
    x.n_rows = rows;
    x.n_cols = cols;
    const size_t a = msd_layout(&x).ws_bytes;
    x.n_cols = halo + cols;
    const size_t b = msd_layout(&x).ws_bytes;
    return a > b ? a : b;
}

static void free_server(spd_server* S)
{
    for (auto& b : S->beams) {
        if (b.stream) (void)hipStreamSynchronize(b.stream);
        if (b.copy) (void)hipStreamSynchronize(b.copy);
        for (void* p : b.buf) if (p) (void)hipFree(p);
        for (void* p : b.stage) if (p) (void)hipFree(p);
        for (void* p : b.fb) if (p) (void)hipFree(p);
        for (auto* p : b.d_cand) if (p) (void)hipFree(p);
        for (auto* p : b.d_count) if (p) (void)hipFree(p);
        for (auto* p : b.h_cand) if (p) (void)hipHostFree(p);
        for (auto* p : b.h_count) if (p) (void)hipHostFree(p);
        for (auto ev : b.h2d_done) if (ev) (void)hipEventDestroy(ev);
        for (auto ev : b.free_ev) if (ev) (void)hipEventDestroy(ev);
        for (auto ev : b.done_ev) if (ev) (void)hipEventDestroy(ev);
        if (b.state) (void)hipFree(b.state);
        if (b.stats) (void)hipFree(b.stats);
        if (b.ws) (void)hipFree(b.ws);
        if (b.stream) (void)hipStreamDestroy(b.stream);
        if (b.copy) (void)hipStreamDestroy(b.copy);
    }
    delete S;
}

}  // namespace spd

using namespace spd;

extern "C" {

size_t spd_server_device_bytes(const spd_server_config* cfg, const spd_params* p)
{
    clear_error();
    if (!cfg || check_params(p)) return 0;
    const int es = elem_size(cfg->dtype);
    const int64_t H = p->widths[p->n_widths - 1] - 1;
    const size_t ws = serve_ws_bytes(cfg->n_rows, H, cfg->chunk_cols);
    const size_t per_beam = (size_t)cfg->slots_per_beam *
                                ((size_t)cfg->n_rows * (size_t)(H + 2 * cfg->chunk_cols) * es +
                                 (size_t)cfg->cand_capacity * sizeof(spd_candidate) + 256) +
                            (size_t)cfg->n_rows * (sizeof(spd_msd_state) + sizeof(spd_row_stats)) + ws;
    return per_beam * (size_t)cfg->n_beams;
}

}  // extern "C"

namespace spd {

// Device bytes of a server with de-dispersion in front: per slot the staged
// chunk, the filterbank with its halo and the FP32 detection plane.
static size_t dedisp_server_bytes(const spd_server_config* cfg, int64_t H, int64_t n_dm, int64_t fb_pitch)
{
    const size_t ws = serve_ws_bytes(n_dm, H, cfg->chunk_cols);
    const size_t per_beam = (size_t)cfg->slots_per_beam *
                                ((size_t)cfg->n_rows * (size_t)cfg->chunk_cols + (size_t)cfg->n_rows * fb_pitch +
                                 (size_t)n_dm * (size_t)(H + cfg->chunk_cols) * 4 +
                                 (size_t)cfg->cand_capacity * sizeof(spd_candidate) + 256) +
                            (size_t)n_dm * (sizeof(spd_msd_state) + sizeof(spd_row_stats)) + ws;
    return per_beam * (size_t)cfg->n_beams;
}

static spd_status create_server(const spd_server_config* cfg, const spd_params* p, const spd_dedisp_plan* dd,
                                spd_server** out)
{
    spd_status st;
    if (!out) return fail(SPD_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(SPD_E_INVALID, "config is NULL");
    if ((st = check_params(p))) return st;
    if (p->scope != SPD_SCOPE_ROW) return fail(SPD_E_UNSUPPORTED, "serving keeps per-row statistics");
    if (!dd && cfg->dtype != SPD_F32 && cfg->dtype != SPD_F16)
        return fail(SPD_E_UNSUPPORTED, "serving takes F32 or F16 chunks");
    if (cfg->n_beams < 1 || cfg->n_beams > 1024) return fail(SPD_E_INVALID, "n_beams outside [1, 1024]");
    if (cfg->n_rows < 1 || cfg->chunk_cols < 1) return fail(SPD_E_INVALID, "empty chunk shape");
    const int nmax = p->widths[p->n_widths - 1];
    if (cfg->chunk_cols < nmax) return fail(SPD_E_INVALID, "chunk_cols must be >= the widest boxcar");
    if (cfg->slots_per_beam < 1 || cfg->slots_per_beam > 8) return fail(SPD_E_INVALID, "slots_per_beam outside [1, 8]");
    if (cfg->cand_capacity < 1) return fail(SPD_E_INVALID, "cand_capacity must be >= 1");
    int32_t n_chan = 0, n_dm = 0, max_delay = 0;
    int plan_device = 0, device = 0;
    int64_t dd_halo = 0, fb_pitch = 0;
    if (dd) {
        dedisp_plan_shape(dd, &n_chan, &n_dm, &max_delay, &plan_device);
        if (cfg->dtype != SPD_U8) return fail(SPD_E_INVALID, "de-dispersion takes 8-bit filterbank chunks (SPD_U8)");
        if (cfg->n_rows != n_chan) return fail(SPD_E_INVALID, "n_rows %lld != the plan's %d channels",
                                               (long long)cfg->n_rows, n_chan);
        if (nmax < 4) return fail(SPD_E_UNSUPPORTED, "de-dispersion in front needs a widest boxcar of 4 or more");
        if (cfg->chunk_cols <= (int64_t)max_delay + nmax)
            return fail(SPD_E_INVALID, "chunk_cols must exceed the largest delay (%d) plus the widest boxcar", max_delay);
        dd_halo = ((int64_t)max_delay + 3) & ~(int64_t)3;
        fb_pitch = (dd_halo + cfg->chunk_cols + 3) & ~(int64_t)3;
    }
    const size_t need = dd ? dedisp_server_bytes(cfg, nmax - 1, n_dm, fb_pitch) : spd_server_device_bytes(cfg, p);
    if (cfg->hbm_budget_bytes && need > (size_t)cfg->hbm_budget_bytes)
        return fail(SPD_E_NOMEM, "configuration needs %zu device bytes > budget %lld", need,
                    (long long)cfg->hbm_budget_bytes);
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return device_status(e, "hipGetDevice");
    if (dd && plan_device != device)
        return fail(SPD_E_INVALID, "the plan was made on device %d, not %d", plan_device, device);
    spd_server* S = new spd_server();
    S->cfg = *cfg;
    S->widths.assign(p->widths, p->widths + p->n_widths);
    S->params = *p;
    S->params.widths = S->widths.data();
    S->in_esize = elem_size(cfg->dtype);
    S->esize = dd ? 4 : S->in_esize;
    S->halo = nmax - 1;
    S->det_rows = dd ? n_dm : cfg->n_rows;
    S->dd = dd;
    S->dd_delay = max_delay;
    S->dd_halo = dd_halo;
    S->fb_pitch = fb_pitch;
    S->device = device;
    S->beams.resize(cfg->n_beams);
    const int slots = cfg->slots_per_beam;
    const int64_t D = S->det_rows;
    const size_t ws_bytes = serve_ws_bytes(D, S->halo, cfg->chunk_cols);
    for (auto& b : S->beams) {
        b.buf.assign(slots, nullptr);
        b.stage.assign(slots, nullptr);
        b.fb.assign(dd ? slots : 0, nullptr);
        b.d_cand.assign(slots, nullptr);
        b.d_count.assign(slots, nullptr);
        b.h_cand.assign(slots, nullptr);
        b.h_count.assign(slots, nullptr);
        b.h2d_done.assign((size_t)slots * kServeRowGroups, nullptr);
        b.free_ev.assign(slots, nullptr);
        b.done_ev.assign(slots, nullptr);
        const size_t bytes = (size_t)D * (size_t)(S->halo + cfg->chunk_cols) * S->esize;
        for (int s = 0; s < slots && e == hipSuccess; ++s) {
            e = hipMalloc(&b.buf[s], bytes);
            if (e == hipSuccess) e = hipMalloc(&b.stage[s], (size_t)cfg->n_rows * (size_t)cfg->chunk_cols * S->in_esize);
            if (e == hipSuccess && dd) e = hipMalloc(&b.fb[s], (size_t)cfg->n_rows * (size_t)fb_pitch);
            if (e == hipSuccess) e = hipMalloc((void**)&b.d_cand[s], sizeof(spd_candidate) * cfg->cand_capacity);
            if (e == hipSuccess) e = hipMalloc((void**)&b.d_count[s], sizeof(int64_t));
            if (e == hipSuccess) e = hipHostMalloc((void**)&b.h_cand[s], sizeof(spd_candidate) * cfg->cand_capacity, 0);
            if (e == hipSuccess) e = hipHostMalloc((void**)&b.h_count[s], sizeof(int64_t), 0);
            for (int g = 0; g < kServeRowGroups && e == hipSuccess; ++g)
                e = hipEventCreateWithFlags(&b.h2d_done[(size_t)s * kServeRowGroups + g], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&b.free_ev[s], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&b.done_ev[s], hipEventDisableTiming);
        }
        if (e == hipSuccess) e = hipMalloc((void**)&b.state, sizeof(spd_msd_state) * D);
        if (e == hipSuccess) e = hipMemset(b.state, 0, sizeof(spd_msd_state) * D);
        if (e == hipSuccess) e = hipMalloc((void**)&b.stats, sizeof(spd_row_stats) * D);
        b.ws_bytes = ws_bytes;
        if (e == hipSuccess) e = hipMalloc(&b.ws, ws_bytes);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&b.copy, hipStreamNonBlocking);
        if (e != hipSuccess) break;
        for (int s = 0; s < slots && e == hipSuccess; ++s) e = hipEventRecord(b.free_ev[s], b.stream);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_server(S);
        return device_status(e, "server allocation");
    }
    S->worker = std::thread(worker_loop, S);
    *out = S;
    return SPD_OK;
}

}  // namespace spd

extern "C" {

spd_status spd_server_create(const spd_server_config* cfg, const spd_params* p, spd_server** out)
{
    clear_error();
    return create_server(cfg, p, nullptr, out);
}

spd_status spd_server_create_dedisp(const spd_server_config* cfg, const spd_params* p, const spd_dedisp_plan* plan,
                                    spd_server** out)
{
    clear_error();
    if (!plan) return fail(SPD_E_INVALID, "plan is NULL");
    return create_server(cfg, p, plan, out);
}

spd_status spd_server_submit(spd_server* S, int32_t beam, int64_t seq, const void* host_chunk, double arrival_s)
{
    clear_error();
    if (!S || !host_chunk) return fail(SPD_E_INVALID, "server and chunk are required");
    std::lock_guard<std::mutex> g(S->mu);
    if (S->fault) return fail(S->fault, "server stopped after an error: %s", S->fault_msg.c_str());
    if (beam < 0 || beam >= (int)S->beams.size()) return fail(SPD_E_INVALID, "beam %d out of range", beam);
    ServeBeam& b = S->beams[beam];
    if (seq != b.next_submit)
        return fail(SPD_E_INVALID, "beam %d expects chunk %lld next, got %lld", beam, (long long)b.next_submit,
                    (long long)seq);
    ServeReq r;
    r.beam = beam;
    r.seq = seq;
    r.host = host_chunk;
    r.submit_s = arrival_s > 0.0 ? arrival_s : now_s();
    b.pending.push_back(r);
    ++b.next_submit;
    ++S->n_submitted;
    S->cv_work.notify_one();
    return SPD_OK;
}

spd_status spd_server_poll(spd_server* S, spd_server_result* res, spd_candidate* cands, int64_t cap, int32_t wait_ms)
{
    clear_error();
    if (!S || !res || cap < 0 || (cap > 0 && !cands)) return fail(SPD_E_INVALID, "bad poll arguments");
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->done.empty() && wait_ms > 0)
        S->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [S] { return !S->done.empty() || S->fault; });
    if (S->done.empty()) {
        if (S->fault) return fail(S->fault, "server stopped after an error: %s", S->fault_msg.c_str());
        return fail(SPD_E_AGAIN, "no finished chunk");
    }
    ServeDone d = std::move(S->done.front());
    S->done.pop_front();
    lk.unlock();
    *res = d.res;
    const int64_t k = std::min<int64_t>((int64_t)d.cands.size(), cap);
    if (k > 0) memcpy(cands, d.cands.data(), sizeof(spd_candidate) * (size_t)k);
    res->n_copied = k;
    return SPD_OK;
}

spd_status spd_server_counters(spd_server* S, int64_t* submitted, int64_t* admitted, int64_t* completed)
{
    clear_error();
    if (!S) return fail(SPD_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> g(S->mu);
    if (submitted) *submitted = S->n_submitted;
    if (admitted) *admitted = S->n_admitted;
    if (completed) *completed = S->n_completed;
    return SPD_OK;
}

void spd_server_destroy(spd_server* S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    free_server(S);
}

}  // extern "C"
