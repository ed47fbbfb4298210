/*
 * spd.h -- C ABI of libspd, the MI355X (gfx950) single-pulse detection path of
 * Adamek & Armour, "A Real-time Single Pulse Detection Algorithm for GPUs"
 * (arXiv:1611.09704).
 *
 * The path runs over a plane of de-dispersed time series, one row per DM
 * trial, time contiguous (Sec. 1, Sec. 2.3):
 *   1. msd_compute       mean and standard deviation per unit (Sec. 2.1:
 *                        partial sums inside a block, Eq. MSD04 in FP64
 *                        across blocks), plus sigma of the widest boxcar
 *                        when the linear approximation of Sec. 2.2
 *                        Eq. (sd03) is in use;
 *   2. boxcar_snr        boxcars of every listed width at every sample, their
 *                        SNR with sigma_N from Eq. (sd02) or Eq. (sd03), and
 *                        the highest SNR with its width (Sec. 2.3,
 *                        Algorithm 1); optionally fused with step 3;
 *   3. select_candidates the SNR threshold of Sec. 2.4, producing an unordered
 *                        list of (DM-trial row, time, SNR, width).
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE memory owned by the caller unless marked [host].
 *     The library keeps no pointer after a call returns.
 *   - Every call validates its arguments on the host first.  On any error
 *     nothing is enqueued, the call returns a non-zero spd_status and
 *     spd_last_error() (thread-local) describes the problem.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream)
 *     and the call returns without synchronising.  A launch failure reported
 *     by the HIP runtime returns SPD_E_DEVICE.
 *   - None of these entry points allocates device memory.  Scratch space is
 *     the caller's `workspace`, sized by spd_workspace_bytes(), or for
 *     spd_detect_static a fixed array inside the library.
 *   - Calls are re-entrant; calls on different streams may overlap as long as
 *     they do not share output or workspace buffers.
 *   - Readings of the paper (all shared with the CPU oracle):
 *       * Eq. (MSD03) is applied with its update term squared; sigma is the
 *         population value sqrt(S/n).
 *       * The width-w boxcar at t is B_w(t) = sum_{k<w} x[t+k]; its SNR is
 *         (B_w(t) - w*mean) / sigma_w.  Outputs exist for t in [0, n_cols-Nmax]
 *         where Nmax = the largest width.
 *       * sigma_w = sqrt(w)*sigma + (w-1)*lin_coef, lin_coef = 0 under
 *         Eq. (sd02).  Under Eq. (sd03) (anchored reading) lin_coef =
 *         (sigma_Nmax - sqrt(Nmax)*sigma)/(Nmax-1); the literal printed form
 *         uses sigma_Nmax/(Nmax-1).  sigma_Nmax is the population standard
 *         deviation of B_Nmax(t) over the unit's valid starts.
 *       * The highest SNR keeps the FIRST width that reaches it (strict '>').
 *         For the lists 1..n (n <= 16) exact ties are resolved this way
 *         only among positive SNRs and +0; among exactly equal negative
 *         SNRs the last width is kept, and +0 counts above -0.  Every width
 *         kept is a maximiser (ties of this kind need equal products of
 *         different sums and coefficients).
 *       * A unit with sigma == 0 is flagged SPD_FLAG_ZERO_VAR: all its SNRs
 *         are 0 and all width indices 0.  A width whose sigma_w is not above
 *         1e-9*sqrt(w)*sigma gives 0 (the anchored form is zero at w = Nmax
 *         when sigma_Nmax = 0, and its rounding residual there has either
 *         sign).
 *       * A sample is a candidate iff its highest SNR >= threshold.
 */
#ifndef SPD_H
#define SPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPD_ABI_VERSION 1
#define SPD_MAX_WIDTHS 256     /* |W| limit: width indices are stored as uint8 */
#define SPD_MAX_NMAX 4096      /* largest supported boxcar width              */

typedef enum {
    SPD_OK = 0,
    SPD_E_INVALID = 1,      /* bad argument (message in spd_last_error)         */
    SPD_E_UNSUPPORTED = 2,  /* valid request the library does not handle         */
    SPD_E_NOMEM = 3,        /* workspace too small / allocation failed          */
    SPD_E_DEVICE = 4,       /* the HIP runtime reported an error, or serving
                               work missed its deadline                         */
    SPD_E_AGAIN = 5         /* serving: queue full or nothing ready (retry)      */
} spd_status;

typedef enum { SPD_F32 = 0, SPD_F16 = 1, SPD_U8 = 2 } spd_dtype;
typedef enum { SPD_SCOPE_ROW = 0, SPD_SCOPE_PLANE = 1 } spd_scope;
typedef enum {
    SPD_SIGMA_SQRTN = 0,          /* Eq. (sd02): sigma_w = sqrt(w)*sigma                */
    SPD_SIGMA_LINEAR = 1,         /* Eq. (sd03), anchored reading, every unit           */
    SPD_SIGMA_AUTO = 2,           /* anchored Eq. (sd03) where rho > 1 + kappa, else sd02 */
    SPD_SIGMA_LINEAR_LITERAL = 3  /* Eq. (sd03) exactly as printed                      */
} spd_sigma_mode;

#define SPD_FLAG_ZERO_VAR 1u   /* sigma == 0: SNR 0, width index 0 */
#define SPD_FLAG_LINEAR 2u     /* the linear term of Eq. (sd03) is applied */

/* A DM-trial x time plane.  Element [r][t] lives at
 * (const char*)data + (r*row_stride + t)*elem_size, elem_size 4/2/1 for
 * F32/F16/U8.  For U8 the value is x = row_scale[r]*(q - row_zero[r]).
 * Any element-aligned pointer and stride work.  With data aligned to 4
 * elements and row_stride a multiple of 4, every kernel uses vector loads;
 * otherwise the statistics of the widest boxcar (AUTO and LINEAR sigma_N)
 * read element by element and take about a fifth more time (pad row_stride
 * to avoid it).                                                             */
typedef struct {
    const void* data;
    int32_t dtype;           /* spd_dtype */
    int32_t reserved0;
    int64_t n_rows;          /* >= 1 */
    int64_t n_cols;          /* >= Nmax */
    int64_t row_stride;      /* elements, >= n_cols */
    const float* row_scale;  /* U8 only, [n_rows] */
    const float* row_zero;   /* U8 only, [n_rows] */
} spd_plane;

typedef struct {
    const int32_t* widths;   /* [host] strictly increasing, widths[0] >= 1, last <= SPD_MAX_NMAX */
    int32_t n_widths;        /* 1 .. SPD_MAX_WIDTHS */
    float threshold;         /* f_T of Sec. 2.4, in SNR units; finite */
    int32_t scope;           /* spd_scope: statistics per row, or one set for the plane */
    int32_t sigma_mode;      /* spd_sigma_mode */
    float auto_kappa;        /* AUTO: linear iff sigma_Nmax/(sqrt(Nmax)*sigma) > 1 + kappa */
    int32_t reserved0;
} spd_params;

/* Running FP64 statistics of one unit: count, sum and sum of squared
 * deviations of the raw samples, and the same for B_Nmax(t) (Sec. 2.1).     */
typedef struct { double n, T, S, n_y, T_y, S_y; } spd_msd_state;

/* Per-unit statistics consumed by boxcar_snr. */
typedef struct {
    double mean, sigma, sigma_nmax, lin_coef;
    uint32_t flags;          /* SPD_FLAG_* */
    uint32_t reserved0;
} spd_row_stats;

/* One candidate of Sec. 2.4: DM-trial row, time (window start + t_offset),
 * highest SNR and the boxcar width that produced it.  `beam` is the beam index
 * in batched runs and 0 otherwise.                                          */
typedef struct {
    int32_t row;
    int32_t width;
    int64_t t;
    float snr;
    uint32_t beam;
} spd_candidate;

/* ABI version (SPD_ABI_VERSION of the built library). */
int spd_abi_version(void);

/* Description of the last error on the calling thread ("" if none). */
const char* spd_last_error(void);

/* Bytes of device workspace msd_compute needs for this plane and params, or 0
 * when the arguments are invalid (see spd_last_error).                     */
size_t spd_workspace_bytes(const spd_plane* x, const spd_params* p);

/*
 * msd_compute -- Sec. 2.1: per-unit mean and standard deviation.
 *   A unit is a row (SPD_SCOPE_ROW) or the whole plane (SPD_SCOPE_PLANE).
 *   Each block of a row (16384 to 65536 columns) gives a partial (n, T, S):
 *   raw statistics only: FP32 mini-batches of 16 samples merged with the
 *   streaming update (Eq. MSD03) and the pairwise merge (Eq. MSD04);
 *   with sigma_Nmax: sums of samples shifted by a sample near the row's
 *   mean, in FP32 over runs of 8 or 16 and in FP64 across runs, and the
 *   widest boxcar advanced one start at a time from a running FP64 value;
 *   U8 planes: exact integer sums of the stored bytes.  The block partials
 *   are merged across blocks in FP64 (Eq. MSD04).
 *   Raw-sample statistics use columns [new_col_begin, n_cols).  When
 *   sigma_mode != SPD_SIGMA_SQRTN, the statistics of B_Nmax(t) over every
 *   valid start t in [0, n_cols-Nmax] are gathered in the same pass.
 *   state       [n_units] or NULL.  accumulate=1: *state is merged with this
 *               call's statistics (Eq. MSD04) and the result is written back
 *               (streaming over chunks; the caller passes the previous
 *               chunk's last Nmax-1 columns as a halo and sets
 *               new_col_begin = Nmax-1).  accumulate=0: *state is overwritten.
 *               state may be NULL only when accumulate == 0.
 *   stats       [n_units] output: mean, sigma, sigma_Nmax, lin_coef, flags
 *               from the (merged) state.
 *   workspace   >= spd_workspace_bytes(x, p) bytes, 256-byte aligned.
 */
spd_status msd_compute(const spd_plane* x, const spd_params* p, int64_t new_col_begin,
                       int32_t accumulate, spd_msd_state* state, spd_row_stats* stats,
                       void* workspace, size_t workspace_bytes, void* stream);

/*
 * boxcar_snr -- Sec. 2.2-2.3, Algorithm 1: for every row r and start
 *   t in [0, n_out) with n_out = n_cols - Nmax + 1, the highest
 *   (B_w(t) - w*mean)/sigma_w over the width list and the index (into
 *   p->widths) of the first width reaching it.
 *   stats       [n_units] from msd_compute (unit = row, or one for the plane).
 *   snr_out     [n_rows][out_stride] float, or NULL.
 *   widx_out    [n_rows][out_stride] uint8 index into p->widths, or NULL.
 *   out_stride  elements, >= n_out when an output is given.
 *   cand        when not NULL, the threshold of Sec. 2.4 is fused: every
 *               (r, t) with snr >= p->threshold is appended, unordered, as
 *               {r, widths[idx], t + t_offset, snr}.  At most cand_capacity
 *               entries are written; *cand_count (device int64, reset by the
 *               call) receives the total number found, which may exceed the
 *               capacity -- the caller then grows the list and re-runs.
 *   At least one of snr_out, widx_out, cand must be given.
 */
spd_status boxcar_snr(const spd_plane* x, const spd_params* p, const spd_row_stats* stats,
                      float* snr_out, uint8_t* widx_out, int64_t out_stride, int64_t t_offset,
                      spd_candidate* cand, int64_t cand_capacity, int64_t* cand_count,
                      void* stream);

/*
 * boxcar_snr_dit -- boxcars combined with decimation in time, the direction
 *   Sec. 3 gives for boxcars wider than 16 samples: level 0 runs widths 1..16
 *   at every start; level l = 1..levels runs widths 9..16 on the series
 *   decimated l times (adjacent pairs summed each time), which is the window
 *   of 2^l*(9..16) samples at starts that are multiples of 2^l.  Every
 *   evaluated window's SNR is the one boxcar_snr gives for it; only the set of
 *   windows is smaller (about a third of the work of 1..16 plus every width
 *   step up to 256, for levels = 4), at the cost of sensitivity to pulses
 *   between the decimated grid points and widths.
 *   p->widths must be exactly that list in ascending order: 1..16, then
 *   2^l*9 .. 2^l*16 in steps of 2^l for l = 1..levels (levels 0..4, so the
 *   widest boxcar is 16*2^levels).  stats come from msd_compute with the same
 *   params.  Outputs as in boxcar_snr: per start t in [0, n_cols - Nmax], the
 *   highest SNR over the widths evaluated at t and the index (into p->widths)
 *   of the first width reaching it; candidates {r, width, t + t_offset, snr}.
 */
spd_status boxcar_snr_dit(const spd_plane* x, const spd_params* p, int32_t levels, const spd_row_stats* stats,
                          float* snr_out, uint8_t* widx_out, int64_t out_stride, int64_t t_offset,
                          spd_candidate* cand, int64_t cand_capacity, int64_t* cand_count, void* stream);

/*
 * select_candidates -- Sec. 2.4 on stored outputs: every (r, t) with
 *   snr[r*out_stride + t] >= p->threshold, t < n_out_cols, becomes
 *   {r, p->widths[widx[...]], t + t_offset, snr}.  Unordered; capacity and
 *   *cand_count behave as in boxcar_snr.
 */
spd_status select_candidates(const float* snr, const uint8_t* widx, int64_t n_rows,
                             int64_t n_out_cols, int64_t out_stride, const spd_params* p,
                             int64_t t_offset, spd_candidate* cand, int64_t cand_capacity,
                             int64_t* cand_count, void* stream);

/*
 * spd_detect -- the whole path (Sec. 2.1-2.4) over one plane in one call:
 *   the result of msd_compute(x, p, 0, 0, NULL, stats, workspace, ...)
 *   followed by boxcar_snr(x, p, stats, ...) on `stream`, with identical
 *   statistics, SNRs and width indices and the same candidate set (its
 *   order may differ).
 *   In ROW scope the rows are cut into row_chunks consecutive chunks.  Each
 *   chunk's statistics (Sec. 2.1-2.2) are computed on aux_stream and its
 *   boxcars (Sec. 2.3-2.4) on stream as soon as they are ready, so the
 *   bandwidth-bound statistics pass of later chunks overlaps the
 *   arithmetic-bound boxcar pass of earlier ones.  The overlap shortens the
 *   call only where neither pass fills the device by itself; each launch of
 *   the 4096 x 2^20 plane does, and there the two passes share the compute
 *   units rather than overlap.  aux_stream waits for
 *   the work enqueued on `stream` before this call, and `stream` waits for
 *   every chunk's statistics before the call's last boxcar: work enqueued on
 *   `stream` afterwards sees all outputs.  The call enqueues work on both
 *   streams, so the two must not be the same.
 *   With aux_stream == NULL, row_chunks <= 1, or SPD_SCOPE_PLANE (whose
 *   statistics span every row) the two steps run one after the other on
 *   `stream`.
 *   stats       [n_units] output.
 *   snr_out, widx_out, out_stride, t_offset, cand, cand_capacity,
 *   cand_count  as in boxcar_snr (*cand_count is reset once by the call).
 *   workspace   >= spd_workspace_bytes(x, p) bytes, 256-byte aligned; the
 *               chunks reuse it one after another on aux_stream.
 *   row_chunks  1..SPD_MAX_ROW_CHUNKS (larger values are clamped, and so is
 *               a value above n_rows).
 *   The library keeps one set of HIP events per thread and device for the
 *   stream dependencies, created on the first pipelined call; no device
 *   memory is allocated.
 */
#define SPD_MAX_ROW_CHUNKS 64
spd_status spd_detect(const spd_plane* x, const spd_params* p, spd_row_stats* stats,
                      float* snr_out, uint8_t* widx_out, int64_t out_stride, int64_t t_offset,
                      spd_candidate* cand, int64_t cand_capacity, int64_t* cand_count,
                      void* workspace, size_t workspace_bytes, int32_t row_chunks,
                      void* stream, void* aux_stream);

/*
 * spd_detect_static -- spd_detect without a workspace, for callers that cannot
 *   allocate device memory: code under HIP graph capture, tight serving loops,
 *   harnesses that forbid allocation.  The statistics pass keeps its block
 *   partials in a fixed device array inside the library (4 MiB per device,
 *   enough for 87,381 (row, block) partials; a 4,096 x 2^20 plane uses
 *   65,536) instead of a caller workspace.  Results equal those of
 *   spd_detect(x, p, stats, ..., row_chunks = 1) with the same arguments.
 *   The call allocates nothing: the first call on a device looks up that
 *   device's copy of the array and keeps its address.
 *   Arguments as in spd_detect, minus workspace, row_chunks and aux_stream;
 *   both steps run on `stream`.  A plane whose partials exceed the array
 *   returns SPD_E_UNSUPPORTED (use spd_detect with a workspace).
 *   Every call on one device shares that device's array and leaves its
 *   partials there: calls that overlap on one GPU (other streams or threads)
 *   race and must be serialised by the caller.
 */
spd_status spd_detect_static(const spd_plane* x, const spd_params* p, spd_row_stats* stats,
                             float* snr_out, uint8_t* widx_out, int64_t out_stride, int64_t t_offset,
                             spd_candidate* cand, int64_t cand_capacity, int64_t* cand_count, void* stream);

/*
 * cluster_candidates -- peak-finding over a candidate list, a step after
 *   Sec. 2.4, whose list keeps every sample above the threshold (the paper
 *   does not cluster): candidate c is kept iff, with r = c.row and
 *   t = c.t - t_offset, no (r', t') with |r' - r| <= dm_radius,
 *   |t' - t| <= t_radius inside the plane has snr[r'][t'] > snr[r][t], or an
 *   equal SNR and (r', t') earlier in row-major order.  A plateau therefore
 *   keeps one sample, and peaks farther apart than the radii all survive.
 *   snr         [n_rows][out_stride] float on the device, the plane boxcar_snr
 *               (or boxcar_snr_dit) wrote for these candidates; out_stride >=
 *               n_out_cols.  Read only.
 *   cand        device list; min(*cand_count, cand_capacity) entries are read
 *               (cand_count is a device int64, as boxcar_snr leaves it).
 *               Entries whose (row, t - t_offset) lies outside the plane are
 *               never kept.
 *   peaks       device list of peak_capacity entries, not overlapping cand;
 *               each kept candidate is copied there whole, unordered.
 *   peak_count  device int64, reset by the call, receives the number of
 *               peaks, which may exceed peak_capacity (then only that many
 *               are written).
 *   dm_radius   0..SPD_MAX_DM_RADIUS rows; t_radius 0..SPD_MAX_T_RADIUS
 *               starts.  Both 0 keep every candidate.
 *   Enqueued on stream; nothing is allocated.
 */
#define SPD_MAX_DM_RADIUS 4096
#define SPD_MAX_T_RADIUS (1 << 20)
spd_status cluster_candidates(const float* snr, int64_t n_rows, int64_t n_out_cols, int64_t out_stride,
                              int64_t t_offset, const spd_candidate* cand, int64_t cand_capacity,
                              const int64_t* cand_count, int32_t dm_radius, int32_t t_radius,
                              spd_candidate* peaks, int64_t peak_capacity, int64_t* peak_count, void* stream);

/* ------------------------------------------------------------------------
 * De-dispersion: the step before the path.  Detection runs on de-dispersed
 * time series (Sec. 1); this builds them from a filterbank of 8-bit samples
 * x[c][s], channel 0 the highest frequency, by brute-force incoherent
 * de-dispersion:
 *     y[d][t] = sum over c of x[c][t + delay(d, c)],   0 <= t < n_samp - max delay,
 *     delay(d, c) = floor(dm[d] * k_c + 0.5),
 *     k_c = 4.148808e3 * (1/f_c^2 - 1/f_top^2) / t_samp,   f_c = f_top - c * chan_bw,
 * the cold-plasma dispersion delay (MHz, s, pc cm^-3) rounded to whole
 * samples; the product and the sum in delay() are each rounded to FP64.
 * The sums are exact (whole counts; below 2^24 for up to 65,536 channels).
 * The output is a DM-trial x time plane that msd_compute / boxcar_snr take
 * as they are.
 * ------------------------------------------------------------------------ */
#define SPD_MAX_CHANNELS 65536
#define SPD_MAX_DM_TRIALS (1 << 20)
#define SPD_MAX_DELAY (1 << 30)

typedef struct {
    int32_t n_chan;          /* channels, 1 .. SPD_MAX_CHANNELS */
    int32_t reserved0;
    double f_top_mhz;        /* frequency of channel 0 (the highest), MHz */
    double chan_bw_mhz;      /* channel spacing, MHz, > 0: f_c = f_top - c * chan_bw > 0 */
    double t_samp_s;         /* sampling time, s */
} spd_band;

typedef struct spd_dedisp_plan spd_dedisp_plan;

/* Plan for one band and one list of trial DMs (host array dm[n_dm], pc cm^-3,
 * finite, >= 0, non-decreasing; copied).  Computes the per-channel factors
 * k_c, the largest delay and the largest delay difference between trials 16
 * apart, and copies the tables to the current device (the only allocation).
 * SPD_E_UNSUPPORTED when trials 16 apart differ by more delay than the LDS
 * staging holds (about 16,000 samples) or the largest delay exceeds
 * SPD_MAX_DELAY.                                                            */
spd_status spd_dedisp_plan_create(const spd_band* band, const double* dm, int32_t n_dm, spd_dedisp_plan** plan);
void spd_dedisp_plan_destroy(spd_dedisp_plan* plan);

/* The largest delay (samples; n_out = n_samp - max_delay) and the largest
 * delay difference between trials 16 apart.  Either pointer may be NULL.   */
spd_status spd_dedisp_describe(const spd_dedisp_plan* plan, int32_t* max_delay, int32_t* span16);

/* The plan's delay table, delay(d, c), into host delays[n_dm][n_chan].    */
spd_status spd_dedisp_delays(const spd_dedisp_plan* plan, int32_t* delays);

/* The same table and largest delay without a plan (host only, no device):
 * validates band and dm as spd_dedisp_plan_create does; delays (host
 * [n_dm][n_chan]) and max_delay may each be NULL.                          */
spd_status spd_dedisp_delay_table(const spd_band* band, const double* dm, int32_t n_dm, int32_t* delays,
                                  int32_t* max_delay);

/* De-disperse fb (SPD_U8, n_rows = n_chan, n_cols = n_samp > max delay, data
 * and row_stride 4-byte aligned, no row_scale / row_zero) into
 * out[n_dm][out_stride] float (device), writing t < n_samp - max_delay of
 * every row.  Enqueued on stream, on the plan's device.                    */
spd_status spd_dedisperse(const spd_dedisp_plan* plan, const spd_plane* fb, float* out, int64_t out_stride,
                          void* stream);

/* ------------------------------------------------------------------------
 * Batched form: the same path over many beams of uneven shape per step.
 * Every beam gets per-row statistics (Sec. 2.1-2.2), then the boxcar/SNR
 * pass with the fused threshold (Sec. 2.3-2.4); candidates carry their beam
 * index.  One persistent launch covers all beams' MSD blocks and one all
 * their time tiles; both pull work from an atomic queue.
 * ------------------------------------------------------------------------ */
typedef struct spd_batch_plan spd_batch_plan;

typedef struct {
    int32_t out_per_lane;    /* boxcar starts per lane */
    int32_t waves_per_group; /* waves per work-group: tile = 64*waves*out_per_lane starts */
    int32_t groups_per_cu;   /* persistent work-groups per compute unit; 0 = one ordinary
                                launch with one work-group per tile                      */
    int32_t tiles_per_grab;  /* tiles taken per atomic queue increment */
    int32_t tuned;           /* 0: default schedule, 1: timed at creation, 2: from the cache */
    int32_t window;          /* 1: each lane takes out_per_lane consecutive starts and keeps a
                                group's reads in registers; 0: starts 64 apart per lane    */
    int64_t msd_items;       /* (beam, row, column block) items */
    int64_t tiles;           /* (beam, row, time tile) items */
    int64_t rows;            /* rows over all beams */
} spd_batch_info;

/*
 * spd_batch_plan_create -- set up a batched run over `n_beams` planes
 *   ([host] array of spd_plane describing device memory; same dtype for all,
 *   1..256 beams, per-row statistics only).  ALLOCATES the plan's device
 *   buffers (descriptors, block partials, per-row statistics, queue counters)
 *   and a capture stream; the data pointers must stay valid for the plan's
 *   life.  autotune=1 times candidate schedules of the boxcar pass on this
 *   device (cached in $SPD_TUNE_CACHE or ~/.cache/spd/batch_schedule.txt).
 *   Synchronises the device.  *plan receives the plan, NULL on error.
 */
spd_status spd_batch_plan_create(const spd_plane* beams, int32_t n_beams, const spd_params* p,
                                 int32_t autotune, spd_batch_plan** plan);

/*
 * spd_batch_run -- one pass over every beam; candidates only (no per-sample
 *   outputs).  cand/cand_capacity/cand_count behave as in boxcar_snr; each
 *   candidate's `beam` field names its beam and `row` its row in that beam.
 *   use_graph=1: the run's launches are captured into a hipGraph on first use
 *   (and again whenever cand, capacity or count change) and replayed on
 *   `stream`.  Allocates nothing after the first graph capture.
 */
spd_status spd_batch_run(spd_batch_plan* plan, spd_candidate* cand, int64_t cand_capacity,
                         int64_t* cand_count, int32_t use_graph, void* stream);

/* Device pointer to beam `beam`'s per-row statistics (valid after a run). */
spd_status spd_batch_stats(const spd_batch_plan* plan, int32_t beam, const spd_row_stats** stats);

/* Copy beam `beam`'s per-row statistics (n_rows of that beam) into dst
 * (device memory owned by the caller), asynchronously on `stream`.          */
spd_status spd_batch_copy_stats(const spd_batch_plan* plan, int32_t beam, spd_row_stats* dst, void* stream);

/* The schedule the plan runs with. */
spd_status spd_batch_describe(const spd_batch_plan* plan, spd_batch_info* info);

/* The autotuner's measurements: up to `cap` timed schedules (rows[i]) with the
 * time per output start (ns_per_start[i], host arrays).  Returns how many
 * schedules were timed (0 when the schedule came from the cache or the
 * default).                                                                  */
int32_t spd_batch_tune_table(const spd_batch_plan* plan, spd_batch_info* rows, float* ns_per_start, int32_t cap);

/* Frees everything the plan owns (call when no run is in flight). */
void spd_batch_plan_destroy(spd_batch_plan* plan);

/* ------------------------------------------------------------------------
 * Serving form: real-time streams of chunks from several beams.
 * Each beam sends consecutive chunks of [n_rows][chunk_cols] new samples
 * (time contiguous).  Per beam the server keeps on the device the running
 * FP64 statistics of everything received so far (Eq. MSD04 merges, Sec. 2.1)
 * and the last Nmax-1 columns of the previous chunk, which it puts in front
 * of the next chunk: every boxcar window that ends inside chunk k is
 * evaluated with chunk k, exactly once, and its SNR uses the statistics after
 * chunk k (Sec. 2.2-2.4).  Candidate times are global sample indices.
 * Chunk buffers on the device come from one pool shared by the beams, sized
 * from the device-memory budget: after the beams' own state (running
 * statistics, statistics workspace, halos) the budget is cut into buffers, at
 * most slots_per_beam per beam (all of them when the budget is 0).  Requests
 * are admitted in arrival order across beams and chunk order within a beam as
 * soon as a buffer is free and the beam has fewer than slots_per_beam chunks
 * on the device; a buffer returns to the pool when its chunk's candidates are
 * on the host.  The device work runs on n_streams compute streams plus as
 * many copy streams (2*n_streams hardware queues): chunks of different beams
 * overlap, copies overlap work, and each beam's chunks stay in order.
 * ------------------------------------------------------------------------ */
typedef struct spd_server spd_server;

typedef struct {
    int32_t n_beams;           /* 1 .. 1024 */
    int32_t dtype;             /* SPD_F32 or SPD_F16 */
    int64_t n_rows;            /* DM trials per chunk */
    int64_t chunk_cols;        /* new samples per chunk, >= the widest boxcar */
    int64_t cand_capacity;     /* candidates kept per chunk (more are counted, not kept) */
    int32_t slots_per_beam;    /* chunks of one beam on the device at once, 1..8 (2: the next copy overlaps work) */
    int32_t n_streams;         /* compute streams (each with a copy stream), 0..8; 0 = 2 */
    int64_t hbm_budget_bytes;  /* 0, or the most device memory the server may take; it sets the pool's buffers */
    double deadline_s;         /* 0, or the longest a chunk may run on the device after admission: a chunk
                                * still running later stops the server (SPD_E_DEVICE from submit and poll;
                                * the work itself cannot be withdrawn from the device) */
    int64_t overflow_capacity; /* 0, or > cand_capacity: a chunk that finds more than cand_capacity
                                * candidates is searched again, from the plane and statistics still in
                                * its buffer, into one list of this capacity (allocated at creation and
                                * counted in the device bytes), and all its candidates are delivered
                                * (flag SPD_SERVE_RERUN) */
} spd_server_config;

typedef struct {
    int32_t beam;
    int32_t status;            /* SPD_OK, SPD_E_NOMEM (candidates beyond the capacity, and beyond
                                * overflow_capacity if set), SPD_E_DEVICE */
    int64_t seq;               /* chunk number within the beam */
    int64_t t_offset;          /* global sample index of this chunk's first window start */
    int64_t n_cands;           /* candidates found in the chunk */
    int64_t n_copied;          /* candidates copied to the caller's buffer */
    double submit_s;           /* arrival time given at submit (steady clock, seconds) */
    double start_s;            /* when the chunk was admitted */
    double done_s;             /* when its results reached the host */
    int32_t flags;             /* SPD_SERVE_GAP: chunks before this one were missing */
    int32_t reserved0;
} spd_server_result;

/* spd_server_result.flags: the chunk followed a gap in the beam's chunk
 * numbers, so it was searched without the previous chunk's halo (windows
 * that would start in the missing data are not evaluated; with
 * de-dispersion in front it yields chunk_cols - max_delay starts, like chunk
 * 0).  The running statistics carry on across the gap.                     */
#define SPD_SERVE_GAP 1
/* spd_server_result.flags: the chunk overflowed cand_capacity and was searched
 * again into the overflow list (spd_server_config.overflow_capacity).       */
#define SPD_SERVE_RERUN 2

/* Device bytes a server with this configuration allocates (0 if invalid, or
 * if the budget cannot hold the beams' state plus one chunk buffer).  Host
 * only; for a server with de-dispersion in front see spd_server_info.      */
size_t spd_server_device_bytes(const spd_server_config* cfg, const spd_params* p);

/* Create a server (ALLOCATES all device buffers, pinned result buffers,
 * streams and a worker thread).  Per-row statistics only; p->sigma_mode may
 * be any mode (the widest-boxcar statistics are streamed as well).         */
spd_status spd_server_create(const spd_server_config* cfg, const spd_params* p, spd_server** server);

/* A server with the de-dispersion step in front: each beam streams 8-bit
 * filterbank chunks (cfg->dtype = SPD_U8, cfg->n_rows = the plan's channels,
 * chunk_cols new samples each, chunk_cols > the plan's largest delay plus the
 * widest boxcar; widest boxcar >= 4).  Per beam the server also keeps the
 * last max-delay filterbank columns (rounded up to 4) on the device,
 * de-disperses [filterbank halo | chunk] as spd_dedisperse does into the
 * beam's DM-trial x time plane (the plan's n_dm rows) and runs the detection
 * stream above on it.  Chunk 0 yields chunk_cols - max_delay new starts,
 * chunk k >= 1 chunk_cols starting at global start k*chunk_cols - max_delay;
 * results' t_offset and candidates' t use that global start, rows are trial
 * indices.  The plan must stay alive until the server is destroyed and
 * belong to the current device.                                            */
spd_status spd_server_create_dedisp(const spd_server_config* cfg, const spd_params* p, const spd_dedisp_plan* plan,
                                    spd_server** server);

/* Queue chunk `seq` of `beam` ([host] n_rows x chunk_cols elements of the
 * configured dtype, pinned memory recommended).  seq must be at least the
 * beam's next chunk number (0, 1, 2, ...); a larger one means the chunks in
 * between are missing: the chunk is searched without a halo, its result
 * carries SPD_SERVE_GAP, and its t_offset places it at sample seq*chunk_cols
 * (a lower number is SPD_E_INVALID).  The buffer must stay valid and unchanged
 * until the chunk's result has been returned by spd_server_poll.
 * arrival_s: the chunk's arrival time on the steady clock in seconds (<= 0:
 * now); latency is measured from it.  Never blocks on the device.          */
spd_status spd_server_submit(spd_server* server, int32_t beam, int64_t seq, const void* host_chunk,
                             double arrival_s);

/* Take one finished chunk: its result and up to `cap` candidates ([host]
 * buffer; a chunk searched again after an overflow brings up to
 * overflow_capacity, the rest are dropped and n_copied says how many were
 * copied).  Waits up to wait_ms for one; SPD_E_AGAIN if none finished.    */
spd_status spd_server_poll(spd_server* server, spd_server_result* result, spd_candidate* cands, int64_t cap,
                           int32_t wait_ms);

/* Chunks submitted, admitted to the device, and completed so far. */
spd_status spd_server_counters(spd_server* server, int64_t* submitted, int64_t* admitted, int64_t* completed);

/* The server's pool of chunk buffers, its compute streams and the device
 * bytes it allocated (any output may be NULL).                             */
spd_status spd_server_info(spd_server* server, int32_t* pool_buffers, int32_t* n_streams, int64_t* device_bytes);

/*
 * Checkpoint and restore of one beam's stream: its running FP64 statistics
 * (one spd_msd_state per detection row, Sec. 2.1 Eq. MSD04 merges every chunk
 * into them), the last Nmax-1 detection columns of its previous chunk, with
 * de-dispersion in front the last filterbank columns too, and the number of
 * the chunk it expects next.  A beam restored from a checkpoint continues
 * exactly where the saved one stopped: the chunks that follow give the
 * candidates (bit for bit) an uninterrupted stream gives.
 *
 * spd_server_beam_state_bytes: size of one beam's checkpoint for this
 *   server's configuration (0 if server is NULL).
 * spd_server_save_beam: writes the checkpoint of `beam` to buf [host], of at
 *   least spd_server_beam_state_bytes bytes.  The beam must be idle: every
 *   chunk submitted for it has finished on the device (its result need not
 *   have been polled); otherwise SPD_E_AGAIN and nothing is written.  Blocks
 *   the calling thread for the device-to-host copies.
 * spd_server_load_beam: replaces the state of `beam` with a checkpoint
 *   written by spd_server_save_beam [host buf, bytes as returned by
 *   spd_server_beam_state_bytes] of a server with the same configuration
 *   (rows, chunk columns, dtype, widths, threshold, sigma mode, kappa,
 *   de-dispersion geometry); SPD_E_INVALID for any other buffer.  The beam
 *   must be idle (SPD_E_AGAIN otherwise).  Its next accepted chunk number is
 *   the saved one.  Nothing changes on error.
 */
size_t spd_server_beam_state_bytes(const spd_server* server);
spd_status spd_server_save_beam(spd_server* server, int32_t beam, void* buf, size_t bytes);
spd_status spd_server_load_beam(spd_server* server, int32_t beam, const void* buf, size_t bytes);

/* Finish the chunks in flight, stop the worker and free everything. */
void spd_server_destroy(spd_server* server);

#ifdef __cplusplus
}
#endif

#endif /* SPD_H */
