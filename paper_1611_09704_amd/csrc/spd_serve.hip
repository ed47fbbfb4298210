// spd_serve.hip -- real-time serving of the detection path over streams of
// chunks from several beams (Sec. 2.1-2.4 applied chunk by chunk).
//
// Each beam streams consecutive chunks of [n_rows][chunk_cols] new samples.
// Per beam the server keeps on the device:
//   - the running FP64 statistics (Eq. MSD04 merges each chunk's partials), so
//     mean and sigma cover every sample received so far;
//   - the last Nmax-1 columns of its previous chunk (the halo), put in front of
//     the next chunk so every boxcar window that ends in the new chunk is
//     evaluated exactly once.
// Chunk buffers come from one pool shared by all beams.  Its size follows the
// device-memory budget: what the per-beam state takes is set aside and the
// rest is cut into buffers (at most slots_per_beam per beam, all of them when
// there is no budget).  A request is admitted, in arrival order across beams
// and in chunk order within a beam, as soon as a buffer is free and its beam
// has fewer than slots_per_beam chunks on the device; the buffer goes back to
// the pool when the chunk's candidates are on the host (continuous batching:
// nothing waits for a batch to fill).  The device work runs on a small pool of
// streams (n_streams compute streams and as many copy streams, so the server
// occupies 2*n_streams hardware queues): chunks of different beams overlap,
// and an event per beam keeps each beam's chunks in order.  A chunk is copied
// in row groups whose statistics and boxcars start as soon as their rows have
// arrived.  A worker thread admits requests and detects completions;
// spd_server_poll hands finished chunks out.
//
// With a de-dispersion plan in front (spd_server_create_dedisp) a beam streams
// 8-bit filterbank chunks instead.  The server also keeps the beam's last
// max-delay filterbank columns (rounded up to 4 bytes), de-disperses
// [filterbank halo | chunk] into the chunk buffer's DM-trial x time plane
// right behind its detection halo, and runs the detection steps on that plane.
// Chunk 0 yields chunk_cols - max_delay new de-dispersed starts, every later
// chunk chunk_cols (global starts k * chunk_cols - max_delay onwards).
#include <hip/hip_runtime.h>

#include <string.h>

#include <chrono>
#include <algorithm>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "spd_abi_internal.h"
#include "spd_admit.h"
#include "spd_kernels.h"

namespace spd {

// A chunk without de-dispersion in front is copied in this many row groups;
// each group's statistics and boxcars start as soon as its rows have arrived
// (rows are independent under per-row statistics), so a chunk's latency is
// close to its copy time plus the work of one group.
constexpr int kServeRowGroups = 4;
constexpr int kServeMaxStreams = 8;

static double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct ServeReq {
    int beam = 0;
    int64_t seq = 0;
    bool fresh = true;                     // no previous chunk to take the halo from (chunk 0, or after a gap)
    const void* host = nullptr;
    double submit_s = 0.0, start_s = 0.0, done_s = 0.0;
    int buf = 0;                           // pool buffer while admitted
};

struct ServeDone {
    spd_server_result res;
    std::vector<spd_candidate> cands;
};

// One chunk buffer of the pool.
struct ServeBuf {
    void* plane = nullptr;                 // device [det_rows][H + C]: halo, then the chunk's columns
    void* stage = nullptr;                 // device [n_rows][C], the contiguous copy-in target
    void* fb = nullptr;                    // device [n_chan][fb_pitch] filterbank (de-dispersion)
    spd_row_stats* stats = nullptr;        // device [det_rows]: the statistics this chunk was searched with
    spd_candidate* d_cand = nullptr;
    int64_t* d_count = nullptr;
    spd_candidate* h_cand = nullptr;       // pinned
    int64_t* h_count = nullptr;
    hipEvent_t h2d[kServeRowGroups] = {};  // a row group of the chunk is on the device
    hipEvent_t done = nullptr;             // count and candidates are on the host
};

struct ServeBeam {
    std::deque<ServeReq> inflight;         // admitted, not complete (in order)
    int64_t next_submit = 0;               // next sequence number accepted
    void* halo = nullptr;                  // device [det_rows][H]: last columns of the previous chunk
    void* fb_halo = nullptr;               // device [n_chan][dd_halo]: last filterbank columns (de-dispersion)
    hipEvent_t ready = nullptr;            // the beam's previous chunk has left its state and halos
    spd_msd_state* state = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
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
    int64_t fb_pitch = 0;                  // bytes per filterbank row in a buffer
    int n_streams = 2;
    hipStream_t compute[spd::kServeMaxStreams] = {}, copy[spd::kServeMaxStreams] = {};
    int64_t launches = 0;                  // chunks launched (picks the stream pair)
    std::vector<spd::ServeBeam> beams;
    std::vector<spd::ServeBuf> pool;
    std::vector<int> free_bufs;
    // the overflow list (overflow_capacity > 0): a chunk past cand_capacity is searched again into it
    spd_candidate* ovf_d_cand = nullptr;
    int64_t* ovf_d_count = nullptr;
    spd_candidate* ovf_h_cand = nullptr;   // pinned
    int64_t* ovf_h_count = nullptr;
    hipStream_t ovf_stream = nullptr;
    std::deque<spd::ServeReq> pending;     // submitted, not admitted, in arrival order
    size_t device_bytes = 0;
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

// New detection-plane columns a chunk brings, and the global index of the
// first of them.  A fresh chunk (chunk 0, or the first after a gap) has no
// previous chunk in front: with de-dispersion it yields chunk_cols - max_delay
// starts from its own first sample on.
static int64_t new_cols(const spd_server* S, bool fresh)
{
    return S->dd && fresh ? S->cfg.chunk_cols - S->dd_delay : S->cfg.chunk_cols;
}

static int64_t first_col(const spd_server* S, int64_t seq, bool fresh)
{
    return S->dd && !fresh ? seq * S->cfg.chunk_cols - S->dd_delay : seq * S->cfg.chunk_cols;
}

// Global start of the chunk's first window (the halo's first column when the
// previous chunk is in front).
static int64_t chunk_t_offset(const spd_server* S, int64_t seq, bool fresh)
{
    return fresh ? first_col(S, seq, fresh) : first_col(S, seq, fresh) - S->halo;
}

static spd_plane view_plane(const spd_server* S, const ServeBuf& pb, bool fresh)
{
    spd_plane x;
    memset(&x, 0, sizeof x);
    const int64_t pitch = S->halo + S->cfg.chunk_cols;
    const char* base = (const char*)pb.plane;
    if (fresh) {                                    // no halo in front
        x.data = base + S->halo * S->esize;
        x.n_cols = new_cols(S, true);
    } else {
        x.data = base;
        x.n_cols = pitch;
    }
    x.dtype = S->dd ? SPD_F32 : S->cfg.dtype;
    x.n_rows = S->det_rows;
    x.row_stride = pitch;
    return x;
}

// De-dispersion of one chunk on compute stream cs: the beam's filterbank
// halo in front (after chunk 0), the staged bytes re-pitched behind it, the
// de-dispersion into the detection plane behind its halo, and the last dd_halo
// filterbank columns kept for the beam's next chunk.  After chunk 0 the view
// starts dd_halo - dd_delay (< 4) columns early so that its rows stay 4-byte
// aligned; those first outputs repeat the previous chunk's last ones exactly
// (whole-count sums) and land on the same columns of the detection halo.
static spd_status dedisperse_chunk(spd_server* S, ServeBeam& b, ServeBuf& pb, bool fresh, hipStream_t cs)
{
    const int64_t C = S->cfg.chunk_cols, Hf = S->dd_halo, R = S->cfg.n_rows, H = S->halo;
    char* fb = (char*)pb.fb;
    hipError_t e;
    if (!fresh && Hf > 0) {
        e = hipMemcpy2DAsync(fb, (size_t)S->fb_pitch, b.fb_halo, (size_t)Hf, (size_t)Hf, (size_t)R,
                             hipMemcpyDeviceToDevice, cs);
        if (e != hipSuccess) return device_status(e, "filterbank halo in");
    }
    e = hipMemcpy2DAsync(fb + Hf, (size_t)S->fb_pitch, pb.stage, (size_t)C, (size_t)C, (size_t)R,
                         hipMemcpyDeviceToDevice, cs);
    if (e != hipSuccess) return device_status(e, "filterbank re-pitch");
    spd_plane f;
    memset(&f, 0, sizeof f);
    f.dtype = SPD_U8;
    f.n_rows = R;
    f.row_stride = S->fb_pitch;
    f.data = fresh ? fb + Hf : fb;
    f.n_cols = fresh ? C : Hf + C;
    const int64_t lead = fresh ? 0 : Hf - S->dd_delay;
    float* out = (float*)pb.plane + (H - lead);
    spd_status st = spd_dedisperse(S->dd, &f, out, H + C, cs);
    if (st) return st;
    if (Hf > 0) {
        e = hipMemcpy2DAsync(b.fb_halo, (size_t)Hf, fb + C, (size_t)S->fb_pitch, (size_t)Hf, (size_t)R,
                             hipMemcpyDeviceToDevice, cs);
        if (e != hipSuccess) return device_status(e, "filterbank halo out");
    }
    return SPD_OK;
}

// Enqueue one admitted chunk in its pool buffer on the next stream pair: copy
// in, statistics, boxcar/SNR with the fused threshold, the beam's halo, and
// the candidates back to the host.
static spd_status launch_chunk(spd_server* S, ServeReq& r)
{
    ServeBeam& b = S->beams[r.beam];
    ServeBuf& pb = S->pool[r.buf];
    const int q = (int)(S->launches++ % S->n_streams);
    hipStream_t cs = S->compute[q], ps = S->copy[q];
    const int64_t C = S->cfg.chunk_cols, H = S->halo, R = S->cfg.n_rows, D = S->det_rows;
    const size_t pitch_b = (size_t)(H + C) * S->esize;
    char* base = (char*)pb.plane;
    hipError_t e;
    spd_status st;
    // in order within the beam: its previous chunk has left the state and halos
    if ((e = hipStreamWaitEvent(cs, b.ready, 0)) != hipSuccess) return device_status(e, "wait beam");
    if (!r.fresh && H > 0) {
        e = hipMemcpy2DAsync(base, pitch_b, b.halo, (size_t)H * S->esize, (size_t)H * S->esize, (size_t)D,
                             hipMemcpyDeviceToDevice, cs);
        if (e != hipSuccess) return device_status(e, "halo in");
    }
    const spd_plane x = view_plane(S, pb, r.fresh);
    if (S->dd) {
        // de-dispersion needs every channel: one contiguous host-to-device copy
        e = hipMemcpyAsync(pb.stage, r.host, (size_t)R * C * S->in_esize, hipMemcpyHostToDevice, ps);
        if (e != hipSuccess) return device_status(e, "chunk copy-in");
        if ((e = hipEventRecord(pb.h2d[0], ps)) != hipSuccess) return device_status(e, "record h2d");
        if ((e = hipStreamWaitEvent(cs, pb.h2d[0], 0)) != hipSuccess) return device_status(e, "wait h2d");
        if ((st = dedisperse_chunk(S, b, pb, r.fresh, cs))) return st;
        st = msd_compute(&x, &S->params, r.fresh ? 0 : H, r.seq == 0 ? 0 : 1, b.state, pb.stats, b.ws, b.ws_bytes,
                         cs);
        if (st) return st;
        st = boxcar_snr(&x, &S->params, pb.stats, nullptr, nullptr, 0, chunk_t_offset(S, r.seq, r.fresh), pb.d_cand,
                        S->cfg.cand_capacity, pb.d_count, cs);
        if (st) return st;
    } else {
        // row groups: each is one contiguous host-to-device copy (full link speed), then a
        // pitched device-to-device copy behind the halo columns, its statistics (the whole
        // view's block layout, so the partials fit the workspace) and its boxcars
        const MsdLayout m = msd_layout(&x);
        if ((st = check_msd_workspace(&x, m, b.ws, b.ws_bytes))) return st;
        BoxcarPlan bp;
        if ((st = plan_boxcar(&x, &S->params, pb.stats, nullptr, nullptr, 0, chunk_t_offset(S, r.seq, r.fresh), pb.d_cand,
                              S->cfg.cand_capacity, pb.d_count, bp)))
            return st;
        if ((e = launch_zero_count(pb.d_count, cs)) != hipSuccess) return device_status(e, "count reset");
        const int64_t per = (R + kServeRowGroups - 1) / kServeRowGroups;
        for (int g = 0; g < kServeRowGroups; ++g) {
            const int64_t r0 = (int64_t)g * per, rows = std::min<int64_t>(per, R - r0);
            if (rows <= 0) break;
            const size_t in_off = (size_t)r0 * (size_t)C * S->in_esize;
            e = hipMemcpyAsync((char*)pb.stage + in_off, (const char*)r.host + in_off,
                               (size_t)rows * (size_t)C * S->in_esize, hipMemcpyHostToDevice, ps);
            if (e != hipSuccess) return device_status(e, "chunk copy-in");
            if ((e = hipEventRecord(pb.h2d[g], ps)) != hipSuccess) return device_status(e, "record h2d");
            if ((e = hipStreamWaitEvent(cs, pb.h2d[g], 0)) != hipSuccess) return device_status(e, "wait h2d");
            e = hipMemcpy2DAsync(base + (size_t)r0 * pitch_b + H * S->esize, pitch_b, (char*)pb.stage + in_off,
                                 (size_t)C * S->esize, (size_t)C * S->esize, (size_t)rows, hipMemcpyDeviceToDevice, cs);
            if (e != hipSuccess) return device_status(e, "chunk re-pitch");
            const spd_plane sub = row_slice(&x, r0, rows);
            if ((st = enqueue_msd(&sub, &S->params, r.fresh ? 0 : H, r.seq != 0, b.state + r0, pb.stats + r0,
                                  (double*)b.ws, m, cs)))
                return st;
            if ((st = enqueue_boxcar(&sub, pb.stats + r0, bp, r0, rows, cs))) return st;
        }
    }
    if (H > 0) {                                    // the last H columns become the beam's halo
        e = hipMemcpy2DAsync(b.halo, (size_t)H * S->esize, base + new_cols(S, r.fresh) * S->esize, pitch_b,
                             (size_t)H * S->esize, (size_t)D, hipMemcpyDeviceToDevice, cs);
        if (e != hipSuccess) return device_status(e, "halo out");
    }
    if ((e = hipEventRecord(b.ready, cs)) != hipSuccess) return device_status(e, "record beam");
    e = hipMemcpyAsync(pb.h_count, pb.d_count, sizeof(int64_t), hipMemcpyDeviceToHost, cs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(pb.h_cand, pb.d_cand, sizeof(spd_candidate) * (size_t)S->cfg.cand_capacity,
                           hipMemcpyDeviceToHost, cs);
    if (e != hipSuccess) return device_status(e, "candidates copy-out");
    if ((e = hipEventRecord(pb.done, cs)) != hipSuccess) return device_status(e, "record done");
    return SPD_OK;
}

// A chunk that found more than cand_capacity candidates, searched again into
// the overflow list: its buffer still holds the plane it was searched on and
// the statistics it was searched with (the beam's later chunks have buffers
// of their own), so the rerun gives the same candidates.  Blocks the calling
// thread until the list and its count are on the host.
static spd_status rerun_chunk(spd_server* S, const ServeReq& r)
{
    const ServeBuf& pb = S->pool[r.buf];
    const spd_plane x = view_plane(S, pb, r.fresh);
    hipStream_t s = S->ovf_stream;
    hipError_t e = launch_zero_count(S->ovf_d_count, s);
    if (e != hipSuccess) return device_status(e, "overflow count reset");
    spd_status st = boxcar_snr(&x, &S->params, pb.stats, nullptr, nullptr, 0, chunk_t_offset(S, r.seq, r.fresh),
                               S->ovf_d_cand, S->cfg.overflow_capacity, S->ovf_d_count, s);
    if (st) return st;
    e = hipMemcpyAsync(S->ovf_h_count, S->ovf_d_count, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(S->ovf_h_cand, S->ovf_d_cand, sizeof(spd_candidate) * (size_t)S->cfg.overflow_capacity,
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? SPD_OK : device_status(e, "overflow rerun");
}

static void worker_loop(spd_server* S)
{
    (void)hipSetDevice(S->device);
    std::vector<char> blocked(S->beams.size());
    std::vector<int> on_device(S->beams.size());
    std::unique_lock<std::mutex> lk(S->mu);
    while (!S->stop) {
        bool progress = false;
        // admission: arrival order across beams, chunk order within a beam, while a
        // pool buffer is free and the beam has fewer than slots_per_beam chunks in flight
        if (S->fault == SPD_OK) {
            for (size_t bi = 0; bi < S->beams.size(); ++bi) on_device[bi] = (int)S->beams[bi].inflight.size();
            const int n = admit_pending(S->pending, S->free_bufs, on_device, S->cfg.slots_per_beam, blocked,
                                        [S](ServeReq& r, int buf) {
                                            r.buf = buf;
                                            r.start_s = now_s();
                                            const spd_status st = launch_chunk(S, r);
                                            if (st) {
                                                S->fault = st;
                                                S->fault_msg = spd_last_error();
                                                return false;
                                            }
                                            S->beams[r.beam].inflight.push_back(r);
                                            ++S->n_admitted;
                                            return true;
                                        });
            progress = progress || n > 0;
        }
        // completions: the oldest in-flight chunk of each beam; its buffer returns to the pool
        for (size_t bi = 0; bi < S->beams.size(); ++bi) {
            ServeBeam& b = S->beams[bi];
            while (!b.inflight.empty()) {
                ServeReq& r = b.inflight.front();
                const ServeBuf& pb = S->pool[r.buf];
                const hipError_t q = hipEventQuery(pb.done);
                if (q == hipErrorNotReady) {
                    if (S->fault == SPD_OK && overdue(now_s(), r.start_s, S->cfg.deadline_s)) {
                        // the work cannot be withdrawn from the device: stop admitting and report it
                        S->fault = SPD_E_DEVICE;
                        S->fault_msg = "chunk " + std::to_string((long long)r.seq) + " of beam " +
                                       std::to_string(r.beam) + " still running " +
                                       std::to_string(now_s() - r.start_s) + " s after admission (deadline " +
                                       std::to_string(S->cfg.deadline_s) + " s)";
                        S->cv_done.notify_all();
                    }
                    break;
                }
                ServeDone d;
                memset(&d.res, 0, sizeof d.res);
                d.res.beam = r.beam;
                d.res.seq = r.seq;
                d.res.flags = r.fresh && r.seq > 0 ? SPD_SERVE_GAP : 0;
                d.res.submit_s = r.submit_s;
                d.res.start_s = r.start_s;
                d.res.done_s = now_s();
                d.res.t_offset = chunk_t_offset(S, r.seq, r.fresh);
                if (q != hipSuccess) {
                    d.res.status = SPD_E_DEVICE;
                } else {
                    const int64_t n = *pb.h_count;
                    d.res.n_cands = n;
                    d.res.status = n > S->cfg.cand_capacity ? SPD_E_NOMEM : SPD_OK;
                    if (n > S->cfg.cand_capacity && S->cfg.overflow_capacity > 0) {
                        // only this thread touches the in-flight lists, the buffer and the
                        // overflow list: submit and poll go on during the rerun
                        lk.unlock();
                        const spd_status rs = rerun_chunk(S, r);
                        lk.lock();
                        if (rs == SPD_OK) {
                            const int64_t n2 = *S->ovf_h_count;
                            const int64_t k = std::min<int64_t>(n2, S->cfg.overflow_capacity);
                            d.res.n_cands = n2;
                            d.res.status = n2 > S->cfg.overflow_capacity ? SPD_E_NOMEM : SPD_OK;
                            d.res.flags |= SPD_SERVE_RERUN;
                            d.cands.assign(S->ovf_h_cand, S->ovf_h_cand + k);
                        } else {
                            d.res.status = rs;
                        }
                    }
                    if (!(d.res.flags & SPD_SERVE_RERUN)) {
                        const int64_t k = n < S->cfg.cand_capacity ? n : S->cfg.cand_capacity;
                        d.cands.assign(pb.h_cand, pb.h_cand + k);
                    }
                    for (auto& c : d.cands) c.beam = (uint32_t)r.beam;
                }
                S->free_bufs.push_back(r.buf);
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

// Device bytes of a server: what each beam keeps (running statistics, the
// statistics workspace, the halos) and what one pool buffer holds (the chunk
// with its halo, the staged copy, the filterbank, the candidate list), and
// the number of pool buffers the budget allows.
struct ServeSizes {
    size_t per_beam = 0, per_buf = 0;
    size_t fixed = 0;                    // every beam's state plus the overflow list
    int64_t buffers = 0;                 // 0: the budget does not hold the beams' state and one buffer
    size_t total = 0;
};

static ServeSizes serve_sizes(const spd_server_config* cfg, int64_t H, int64_t det_rows, int det_esize,
                              int64_t dd_halo, int64_t fb_pitch, bool dd)
{
    ServeSizes z;
    const int in_es = elem_size(cfg->dtype);
    z.per_beam = (size_t)det_rows * sizeof(spd_msd_state) +
                 serve_ws_bytes(det_rows, H, cfg->chunk_cols) + (size_t)det_rows * (size_t)H * det_esize +
                 (dd ? (size_t)cfg->n_rows * (size_t)dd_halo : 0);
    z.per_buf = (size_t)det_rows * (size_t)(H + cfg->chunk_cols) * det_esize +
                (size_t)cfg->n_rows * (size_t)cfg->chunk_cols * in_es +
                (dd ? (size_t)cfg->n_rows * (size_t)fb_pitch : 0) +
                (size_t)cfg->cand_capacity * sizeof(spd_candidate) + sizeof(int64_t) +
                (size_t)det_rows * sizeof(spd_row_stats);
    const int64_t most = (int64_t)cfg->n_beams * cfg->slots_per_beam;
    // the beams' own state and the overflow list come first
    const size_t beams = z.per_beam * (size_t)cfg->n_beams +
                         (cfg->overflow_capacity > 0 ? (size_t)cfg->overflow_capacity * sizeof(spd_candidate) +
                                                               sizeof(int64_t)
                                                     : 0);
    if (cfg->hbm_budget_bytes <= 0) {
        z.buffers = most;
    } else if ((size_t)cfg->hbm_budget_bytes > beams) {
        z.buffers = std::min<int64_t>(most, (int64_t)(((size_t)cfg->hbm_budget_bytes - beams) / z.per_buf));
    }
    z.fixed = beams;
    z.total = beams + (size_t)z.buffers * z.per_buf;
    return z;
}

static void free_server(spd_server* S)
{
    for (int q = 0; q < S->n_streams; ++q) {
        if (S->compute[q]) (void)hipStreamSynchronize(S->compute[q]);
        if (S->copy[q]) (void)hipStreamSynchronize(S->copy[q]);
    }
    if (S->ovf_stream) (void)hipStreamSynchronize(S->ovf_stream);
    for (auto& pb : S->pool) {
        if (pb.plane) (void)hipFree(pb.plane);
        if (pb.stats) (void)hipFree(pb.stats);
        if (pb.stage) (void)hipFree(pb.stage);
        if (pb.fb) (void)hipFree(pb.fb);
        if (pb.d_cand) (void)hipFree(pb.d_cand);
        if (pb.d_count) (void)hipFree(pb.d_count);
        if (pb.h_cand) (void)hipHostFree(pb.h_cand);
        if (pb.h_count) (void)hipHostFree(pb.h_count);
        for (auto ev : pb.h2d) if (ev) (void)hipEventDestroy(ev);
        if (pb.done) (void)hipEventDestroy(pb.done);
    }
    for (auto& b : S->beams) {
        if (b.halo) (void)hipFree(b.halo);
        if (b.fb_halo) (void)hipFree(b.fb_halo);
        if (b.ready) (void)hipEventDestroy(b.ready);
        if (b.state) (void)hipFree(b.state);
        if (b.ws) (void)hipFree(b.ws);
    }
    if (S->ovf_d_cand) (void)hipFree(S->ovf_d_cand);
    if (S->ovf_d_count) (void)hipFree(S->ovf_d_count);
    if (S->ovf_h_cand) (void)hipHostFree(S->ovf_h_cand);
    if (S->ovf_h_count) (void)hipHostFree(S->ovf_h_count);
    for (int q = 0; q < S->n_streams; ++q) {
        if (S->compute[q]) (void)hipStreamDestroy(S->compute[q]);
        if (S->copy[q]) (void)hipStreamDestroy(S->copy[q]);
    }
    if (S->ovf_stream) (void)hipStreamDestroy(S->ovf_stream);
    delete S;
}

}  // namespace spd

using namespace spd;

extern "C" {

size_t spd_server_device_bytes(const spd_server_config* cfg, const spd_params* p)
{
    clear_error();
    if (!cfg || check_params(p)) return 0;
    if (cfg->n_beams < 1 || cfg->slots_per_beam < 1) return 0;
    const int64_t H = p->widths[p->n_widths - 1] - 1;
    const ServeSizes z = serve_sizes(cfg, H, cfg->n_rows, elem_size(cfg->dtype), 0, 0, false);
    if (z.buffers < 1) {
        fail(SPD_E_NOMEM, "budget %lld bytes < %zu for the beams' state and one chunk buffer",
             (long long)cfg->hbm_budget_bytes, z.fixed + z.per_buf);
        return 0;
    }
    return z.total;
}

}  // extern "C"

namespace spd {

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
    if (cfg->n_streams < 0 || cfg->n_streams > kServeMaxStreams)
        return fail(SPD_E_INVALID, "n_streams outside [0, %d]", kServeMaxStreams);
    if (cfg->hbm_budget_bytes < 0) return fail(SPD_E_INVALID, "hbm_budget_bytes < 0");
    if (!(cfg->deadline_s >= 0.0) || cfg->deadline_s > 1e9) return fail(SPD_E_INVALID, "deadline_s must be in [0, 1e9]");
    if (cfg->overflow_capacity != 0 &&
        (cfg->overflow_capacity <= cfg->cand_capacity || cfg->overflow_capacity > ((int64_t)1 << 31)))
        return fail(SPD_E_INVALID, "overflow_capacity must be 0 or in (cand_capacity, 2^31]");
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
    const int64_t det_rows = dd ? n_dm : cfg->n_rows;
    const int esize = dd ? 4 : elem_size(cfg->dtype);
    const ServeSizes z = serve_sizes(cfg, nmax - 1, det_rows, esize, dd_halo, fb_pitch, dd != nullptr);
    if (z.buffers < 1)
        return fail(SPD_E_NOMEM, "budget %lld bytes < %zu for the beams' state and one chunk buffer",
                    (long long)cfg->hbm_budget_bytes, z.fixed + z.per_buf);
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
    S->esize = esize;
    S->halo = nmax - 1;
    S->det_rows = det_rows;
    S->dd = dd;
    S->dd_delay = max_delay;
    S->dd_halo = dd_halo;
    S->fb_pitch = fb_pitch;
    S->device = device;
    S->n_streams = cfg->n_streams ? cfg->n_streams : 2;
    S->device_bytes = z.total;
    S->beams.resize(cfg->n_beams);
    S->pool.resize((size_t)z.buffers);
    const int64_t D = det_rows, H = S->halo;
    const size_t ws_bytes = serve_ws_bytes(D, H, cfg->chunk_cols);
    for (int q = 0; q < S->n_streams && e == hipSuccess; ++q) {
        e = hipStreamCreateWithFlags(&S->compute[q], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->copy[q], hipStreamNonBlocking);
    }
    for (auto& pb : S->pool) {
        if (e != hipSuccess) break;
        e = hipMalloc(&pb.plane, (size_t)D * (size_t)(H + cfg->chunk_cols) * esize);
        if (e == hipSuccess) e = hipMalloc(&pb.stage, (size_t)cfg->n_rows * (size_t)cfg->chunk_cols * S->in_esize);
        if (e == hipSuccess && dd) e = hipMalloc(&pb.fb, (size_t)cfg->n_rows * (size_t)fb_pitch);
        if (e == hipSuccess) e = hipMalloc((void**)&pb.stats, sizeof(spd_row_stats) * D);
        if (e == hipSuccess) e = hipMalloc((void**)&pb.d_cand, sizeof(spd_candidate) * cfg->cand_capacity);
        if (e == hipSuccess) e = hipMalloc((void**)&pb.d_count, sizeof(int64_t));
        if (e == hipSuccess) e = hipHostMalloc((void**)&pb.h_cand, sizeof(spd_candidate) * cfg->cand_capacity, 0);
        if (e == hipSuccess) e = hipHostMalloc((void**)&pb.h_count, sizeof(int64_t), 0);
        for (int g = 0; g < kServeRowGroups && e == hipSuccess; ++g)
            e = hipEventCreateWithFlags(&pb.h2d[g], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&pb.done, hipEventDisableTiming);
    }
    for (auto& b : S->beams) {
        if (e != hipSuccess) break;
        if (H > 0) e = hipMalloc(&b.halo, (size_t)D * (size_t)H * esize);
        if (e == hipSuccess && dd && dd_halo > 0) e = hipMalloc(&b.fb_halo, (size_t)cfg->n_rows * (size_t)dd_halo);
        if (e == hipSuccess) e = hipMalloc((void**)&b.state, sizeof(spd_msd_state) * D);
        if (e == hipSuccess) e = hipMemset(b.state, 0, sizeof(spd_msd_state) * D);
        b.ws_bytes = ws_bytes;
        if (e == hipSuccess) e = hipMalloc(&b.ws, ws_bytes);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b.ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(b.ready, S->compute[0]);
    }
    if (e == hipSuccess && cfg->overflow_capacity > 0) {
        e = hipMalloc((void**)&S->ovf_d_cand, sizeof(spd_candidate) * (size_t)cfg->overflow_capacity);
        if (e == hipSuccess) e = hipMalloc((void**)&S->ovf_d_count, sizeof(int64_t));
        if (e == hipSuccess)
            e = hipHostMalloc((void**)&S->ovf_h_cand, sizeof(spd_candidate) * (size_t)cfg->overflow_capacity, 0);
        if (e == hipSuccess) e = hipHostMalloc((void**)&S->ovf_h_count, sizeof(int64_t), 0);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->ovf_stream, hipStreamNonBlocking);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_server(S);
        return device_status(e, "server allocation");
    }
    for (int i = (int)S->pool.size() - 1; i >= 0; --i) S->free_bufs.push_back(i);
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
    if (seq < b.next_submit)
        return fail(SPD_E_INVALID, "beam %d expects chunk %lld or later, got %lld", beam, (long long)b.next_submit,
                    (long long)seq);
    ServeReq r;
    r.beam = beam;
    r.seq = seq;
    r.fresh = seq == 0 || seq != b.next_submit;            // chunk 0, or chunks before it are missing
    r.host = host_chunk;
    r.submit_s = arrival_s > 0.0 ? arrival_s : now_s();
    S->pending.push_back(r);
    b.next_submit = seq + 1;
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

spd_status spd_server_info(spd_server* S, int32_t* pool_buffers, int32_t* n_streams, int64_t* device_bytes)
{
    clear_error();
    if (!S) return fail(SPD_E_INVALID, "server is NULL");
    if (pool_buffers) *pool_buffers = (int32_t)S->pool.size();
    if (n_streams) *n_streams = S->n_streams;
    if (device_bytes) *device_bytes = (int64_t)S->device_bytes;
    return SPD_OK;
}

}  // extern "C"

namespace spd {

// A beam checkpoint: this header, then the running statistics [det_rows], the
// detection halo [det_rows][H] and the filterbank halo [n_rows][dd_halo].
struct BeamCheckpoint {
    uint32_t magic;                        // 'SPDB'
    uint32_t version;
    uint64_t config;                       // fingerprint of the server configuration
    int64_t next_seq;
    int64_t rows, halo_bytes, fb_halo_bytes;
};
constexpr uint32_t kCheckpointMagic = 0x42445053u;

static uint64_t fnv(uint64_t h, const void* p, size_t n)
{
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 0x100000001b3ull;
    return h;
}

// Everything a beam's state depends on: the geometry of its planes and the
// detection parameters.
static uint64_t config_fingerprint(const spd_server* S)
{
    uint64_t h = 0xcbf29ce484222325ull;
    const int64_t geo[] = {S->cfg.n_rows, S->cfg.chunk_cols, S->det_rows, S->halo, S->dd_halo, S->dd_delay,
                           (int64_t)S->esize, (int64_t)S->in_esize, (int64_t)S->cfg.dtype};
    h = fnv(h, geo, sizeof(geo));
    h = fnv(h, S->widths.data(), sizeof(int32_t) * S->widths.size());
    const int32_t modes[] = {(int32_t)S->params.scope, (int32_t)S->params.sigma_mode};
    h = fnv(h, modes, sizeof(modes));
    h = fnv(h, &S->params.threshold, sizeof(S->params.threshold));
    h = fnv(h, &S->params.auto_kappa, sizeof(S->params.auto_kappa));
    return h;
}

static size_t halo_bytes(const spd_server* S) { return (size_t)S->det_rows * (size_t)S->halo * (size_t)S->esize; }
static size_t fb_halo_bytes(const spd_server* S)
{
    return S->dd ? (size_t)S->cfg.n_rows * (size_t)S->dd_halo : 0;
}
static size_t checkpoint_bytes(const spd_server* S)
{
    return sizeof(BeamCheckpoint) + sizeof(spd_msd_state) * (size_t)S->det_rows + halo_bytes(S) + fb_halo_bytes(S);
}

// Called with S->mu held: no request of the beam waits or runs.
static bool beam_idle(const spd_server* S, int beam)
{
    if (!S->beams[beam].inflight.empty()) return false;
    for (const ServeReq& r : S->pending)
        if (r.beam == beam) return false;
    return true;
}

}  // namespace spd

extern "C" {

size_t spd_server_beam_state_bytes(const spd_server* S)
{
    return S ? spd::checkpoint_bytes(S) : 0;
}

spd_status spd_server_save_beam(spd_server* S, int32_t beam, void* buf, size_t bytes)
{
    using namespace spd;
    clear_error();
    if (!S || !buf) return fail(SPD_E_INVALID, "server and buffer are required");
    if (beam < 0 || beam >= (int)S->beams.size()) return fail(SPD_E_INVALID, "beam %d out of range", beam);
    const size_t need = checkpoint_bytes(S);
    if (bytes < need) return fail(SPD_E_INVALID, "checkpoint needs %zu bytes, got %zu", need, bytes);
    std::lock_guard<std::mutex> g(S->mu);
    if (S->fault) return fail(S->fault, "server stopped after an error: %s", S->fault_msg.c_str());
    if (!beam_idle(S, beam)) return fail(SPD_E_AGAIN, "beam %d has chunks pending or in flight", beam);
    ServeBeam& b = S->beams[beam];
    hipError_t e = hipSetDevice(S->device);
    unsigned char* out = (unsigned char*)buf + sizeof(BeamCheckpoint);
    if (e == hipSuccess) e = hipMemcpy(out, b.state, sizeof(spd_msd_state) * (size_t)S->det_rows, hipMemcpyDeviceToHost);
    out += sizeof(spd_msd_state) * (size_t)S->det_rows;
    if (e == hipSuccess && halo_bytes(S)) e = hipMemcpy(out, b.halo, halo_bytes(S), hipMemcpyDeviceToHost);
    out += halo_bytes(S);
    if (e == hipSuccess && fb_halo_bytes(S)) e = hipMemcpy(out, b.fb_halo, fb_halo_bytes(S), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_status(e, "checkpoint copy");
    BeamCheckpoint h{kCheckpointMagic, 1u, config_fingerprint(S), b.next_submit, S->det_rows,
                     (int64_t)halo_bytes(S), (int64_t)fb_halo_bytes(S)};
    memcpy(buf, &h, sizeof(h));
    return SPD_OK;
}

spd_status spd_server_load_beam(spd_server* S, int32_t beam, const void* buf, size_t bytes)
{
    using namespace spd;
    clear_error();
    if (!S || !buf) return fail(SPD_E_INVALID, "server and buffer are required");
    if (beam < 0 || beam >= (int)S->beams.size()) return fail(SPD_E_INVALID, "beam %d out of range", beam);
    const size_t need = checkpoint_bytes(S);
    if (bytes != need) return fail(SPD_E_INVALID, "a checkpoint of this server is %zu bytes, got %zu", need, bytes);
    BeamCheckpoint h;
    memcpy(&h, buf, sizeof(h));
    if (h.magic != kCheckpointMagic || h.version != 1u) return fail(SPD_E_INVALID, "not a beam checkpoint");
    if (h.config != config_fingerprint(S) || h.rows != S->det_rows || h.halo_bytes != (int64_t)halo_bytes(S) ||
        h.fb_halo_bytes != (int64_t)fb_halo_bytes(S))
        return fail(SPD_E_INVALID, "checkpoint of a server with another configuration");
    if (h.next_seq < 0) return fail(SPD_E_INVALID, "bad chunk number in checkpoint");
    std::lock_guard<std::mutex> g(S->mu);
    if (S->fault) return fail(S->fault, "server stopped after an error: %s", S->fault_msg.c_str());
    if (!beam_idle(S, beam)) return fail(SPD_E_AGAIN, "beam %d has chunks pending or in flight", beam);
    ServeBeam& b = S->beams[beam];
    hipError_t e = hipSetDevice(S->device);
    const unsigned char* in = (const unsigned char*)buf + sizeof(BeamCheckpoint);
    if (e == hipSuccess) e = hipMemcpy(b.state, in, sizeof(spd_msd_state) * (size_t)S->det_rows, hipMemcpyHostToDevice);
    in += sizeof(spd_msd_state) * (size_t)S->det_rows;
    if (e == hipSuccess && halo_bytes(S)) e = hipMemcpy(b.halo, in, halo_bytes(S), hipMemcpyHostToDevice);
    in += halo_bytes(S);
    if (e == hipSuccess && fb_halo_bytes(S)) e = hipMemcpy(b.fb_halo, in, fb_halo_bytes(S), hipMemcpyHostToDevice);
    if (e != hipSuccess) return device_status(e, "checkpoint copy");
    b.next_submit = h.next_seq;
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
