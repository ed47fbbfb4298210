/*
 * spd_oracle.c -- plain FP64 CPU oracle for the single-pulse detection path of
 * Adamek & Armour, "A Real-time Single Pulse Detection Algorithm for GPUs"
 * (arXiv:1611.09704).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file: it exists so that tests, the smoke check and the CPU-baseline leg
 * of the benchmark can check the HIP implementation against an obviously
 * correct, slow, double-precision restatement of the method.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * What it computes, in the paper's order:
 *   1. mean and standard deviation of every unit (a DM row, or the whole plane)
 *      with the streaming update of Sec. 2.1 Eq. (MSD03) and the pairwise merge
 *      of Eq. (MSD04);
 *   2. optionally the measured standard deviation of the Nmax-sample boxcar
 *      series, needed by the linear approximation of Sec. 2.2 Eq. (sd03);
 *   3. for every output sample, the boxcar sums of every width in the list,
 *      their SNR against sigma_N from Eq. (sd02) or Eq. (sd03), and the highest
 *      SNR with the first width that reaches it (Sec. 2.3, Algorithm 1);
 *   4. the candidate list of Sec. 2.4: every sample whose SNR is at or above
 *      the threshold.
 *
 * Readings of the paper that this file commits to (each one also applies to
 * the GPU path):
 *   - Eq. (MSD03) is printed without a square on the update term; S must carry
 *     the units of x^2, so the term is squared (as in Chan et al. 1983).  T is
 *     updated before S because the S update uses T_{1,j}.  A one-sample
 *     sequence has T = x_1, S = 0.
 *   - sigma = sqrt(S/n) (population normalisation, as printed after MSD03).
 *   - Eq. (MSD04) is used as printed; a part with n = 0 is the identity.
 *   - The boxcar of width w starting at t is B_w(t) = sum_{k<w} x[t+k]; its
 *     SNR is (B_w - w*mu) / sigma_w (Algorithm 1 prints B - mu, which is only
 *     unbiased for w = 1).  Outputs exist for t in [0, L - Nmax], where every
 *     width fits.
 *   - The running maximum uses strict '>' starting from the first width, so
 *     ties keep the smallest width (Algorithm 1).
 *   - Eq. (sd03), anchored reading: sigma_w = sqrt(w)*sigma
 *       + (w-1)*(sigma_Nmax - sqrt(Nmax)*sigma)/(Nmax-1), which returns sigma at
 *     w = 1 and the measured sigma_Nmax at w = Nmax.  The literal printed form
 *     sigma_w = sqrt(w)*sigma + (w-1)*sigma_Nmax/(Nmax-1) is kept as a separate
 *     mode.  sigma_Nmax is the population standard deviation of
 *     y(t) = B_Nmax(t) over the valid starts of the unit.
 *   - AUTO mode applies the anchored linear form to a unit iff
 *     rho = sigma_Nmax / (sqrt(Nmax)*sigma) > 1 + kappa.
 *   - A unit with sigma == 0 is flagged ZERO_VAR: every SNR is 0 and the width
 *     index is 0.  A width whose sigma_w is not positive contributes SNR 0;
 *     "positive" means above SW_FLOOR * sqrt(w) * sigma, since the anchored form
 *     reaches zero at w = Nmax when sigma_Nmax = 0 (one valid start, or a row
 *     whose Nmax-boxcar is constant) and its rounding residual there can take
 *     either sign.
 *   - Threshold (Sec. 2.4): a sample is a candidate iff SNR >= f_T.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { SCOPE_ROW = 0, SCOPE_PLANE = 1 };
enum { SIG_SQRTN = 0, SIG_LINEAR = 1, SIG_AUTO = 2, SIG_LINEAR_LITERAL = 3 };
enum { FLAG_ZERO_VAR = 1, FLAG_LINEAR = 2 };
#define SW_FLOOR 1e-9

/* Sec. 2.1 Eq. (MSD03): serial streaming update over x[0..n).
 * T_j = T_{j-1} + x_j ;  S_j = S_{j-1} + (j*x_j - T_j)^2 / (j*(j-1)).       */
void oracle_chan_stream(const double* x, int64_t n, double* out3)
{
    double T = 0.0, S = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double j = (double)(i + 1);
        T += x[i];
        if (i > 0) {
            double d = j * x[i] - T;
            S += d * d / (j * (j - 1.0));
        }
    }
    out3[0] = (double)n;
    out3[1] = T;
    out3[2] = S;
}

/* Sec. 2.1 Eq. (MSD04): combine the (T, S) of samples 1..m and m+1..m+n.
 * S = S_a + S_b + m/(n(m+n)) * (n/m * T_a - T_b)^2 ;  T = T_a + T_b.       */
void oracle_chan_merge(const double* a3, const double* b3, double* out3)
{
    double m = a3[0], n = b3[0];
    if (m == 0.0) { out3[0] = b3[0]; out3[1] = b3[1]; out3[2] = b3[2]; return; }
    if (n == 0.0) { out3[0] = a3[0]; out3[1] = a3[1]; out3[2] = a3[2]; return; }
    double d = (n / m) * a3[1] - b3[1];
    double S = a3[2] + b3[2] + m / (n * (m + n)) * d * d;
    out3[0] = m + n;
    out3[1] = a3[1] + b3[1];
    out3[2] = S;
}

/* B_Nmax(t) for every valid start of one row: the series whose standard
 * deviation is sigma_Nmax in Eq. (sd03).  Each value is a direct sum.        */
static void nmax_series(const double* row, int64_t n_out, int nmax, double* y)
{
    for (int64_t t = 0; t < n_out; ++t) {
        double b = 0.0;
        for (int k = 0; k < nmax; ++k) b += row[t + k];
        y[t] = b;
    }
}

/* Coefficient of the linear term in Eq. (sd03) for one unit, and its flags. */
static void unit_coefficients(const double* st6, int sigma_mode, double kappa, int nmax,
                              double* stats5)
{
    double n = st6[0], T = st6[1], S = st6[2];
    double mu = n > 0.0 ? T / n : 0.0;
    double sigma = n > 0.0 ? sqrt(S / n) : 0.0;
    double sig_nmax = st6[3] > 0.0 ? sqrt(st6[5] / st6[3]) : 0.0;
    double coef = 0.0;
    uint32_t flags = 0;
    if (!(sigma > 0.0)) {
        flags |= FLAG_ZERO_VAR;
    } else if (nmax > 1 && sigma_mode != SIG_SQRTN) {
        double base = sqrt((double)nmax) * sigma;
        if (sigma_mode == SIG_LINEAR) {
            coef = (sig_nmax - base) / (double)(nmax - 1);
            flags |= FLAG_LINEAR;
        } else if (sigma_mode == SIG_LINEAR_LITERAL) {
            coef = sig_nmax / (double)(nmax - 1);
            flags |= FLAG_LINEAR;
        } else if (sigma_mode == SIG_AUTO) {
            double rho = sig_nmax / base;
            if (rho > 1.0 + kappa) {
                coef = (sig_nmax - base) / (double)(nmax - 1);
                flags |= FLAG_LINEAR;
            }
        }
    }
    stats5[0] = mu;
    stats5[1] = sigma;
    stats5[2] = sig_nmax;
    stats5[3] = coef;
    stats5[4] = (double)flags;
}

/* Sec. 2.3 Algorithm 1 for one row: for each start t the boxcar sum grows one
 * sample at a time; at every width in W the SNR is formed and compared with
 * the best so far (strict '>').                                             */
/* One row of step 3.  stride[i] (NULL: all 1) restricts width W[i] to starts
 * that are multiples of stride[i]; the running sum still passes through it.  */
static void detect_row(const double* row, int64_t n_out, const int32_t* W, const int32_t* stride, int nW,
                       const double* stats5, double* snr, int32_t* widx)
{
    double mu = stats5[0], sigma = stats5[1], coef = stats5[3];
    int zero_var = ((uint32_t)stats5[4] & FLAG_ZERO_VAR) != 0;
    double* sig_w = (double*)malloc(sizeof(double) * (size_t)nW);
    for (int i = 0; i < nW; ++i)
        sig_w[i] = sqrt((double)W[i]) * sigma + (double)(W[i] - 1) * coef;   /* Eq. sd02 / sd03 */
    for (int64_t t = 0; t < n_out; ++t) {
        if (zero_var) { snr[t] = 0.0; widx[t] = 0; continue; }
        double B = 0.0, best = -INFINITY;
        int k = 0, bi = 0;
        for (int i = 0; i < nW; ++i) {
            while (k < W[i]) { B += row[t + k]; ++k; }
            if (stride && t % stride[i] != 0) continue;
            double s = sig_w[i] > SW_FLOOR * sqrt((double)W[i]) * sigma ? (B - (double)W[i] * mu) / sig_w[i] : 0.0;
            if (s > best) { best = s; bi = i; }
        }
        snr[t] = best;
        widx[t] = bi;
    }
    free(sig_w);
}

/*
 * One step of the path over a plane view x[R][L_view] (row-major, time
 * contiguous).  The per-unit running state st6 = {n, T, S, n_y, T_y, S_y} is
 * merged (Eq. MSD04) with the statistics of this view:
 *   - raw-sample statistics over columns [new_col_begin, L_view) only (earlier
 *     columns are a halo already counted by a previous step);
 *   - Nmax-boxcar statistics over every valid start of the view, when the
 *     sigma mode needs sigma_Nmax.
 * Then mu, sigma and the Eq. (sd03) coefficient come from the merged state, and
 * snr/widx are written for starts [0, L_view - Nmax].  A one-shot detection is
 * a single step with a zeroed state and new_col_begin = 0.
 * Returns 0, or -1 for an argument error.
 */
int oracle_stream_step_strided(const double* x, int64_t R, int64_t L_view, int64_t new_col_begin,
                               const int32_t* W, const int32_t* stride, int32_t nW, int scope, int sigma_mode,
                               double kappa, double* state, double* stats, double* snr, int32_t* widx,
                               int nthreads);

int oracle_stream_step(const double* x, int64_t R, int64_t L_view, int64_t new_col_begin,
                       const int32_t* W, int32_t nW, int scope, int sigma_mode, double kappa,
                       double* state, double* stats, double* snr, int32_t* widx, int nthreads)
{
    return oracle_stream_step_strided(x, R, L_view, new_col_begin, W, NULL, nW, scope, sigma_mode, kappa, state,
                                      stats, snr, widx, nthreads);
}

/*
 * The same step where width W[i] is evaluated only at starts t that are
 * multiples of stride[i] (stride NULL: every start).  This is the search of
 * boxcars combined with decimation in time, the direction Sec. 3 names for
 * wide boxcars: decimating the series by 2 (summing adjacent pairs) l times
 * and running a boxcar of w decimated samples gives exactly the window of
 * w*2^l samples that starts at a multiple of 2^l, so the decimated search is
 * this exhaustive definition restricted to those (start, width) pairs.
 * Statistics are unchanged (sigma_Nmax uses every start of the widest width).
 */
int oracle_stream_step_strided(const double* x, int64_t R, int64_t L_view, int64_t new_col_begin,
                               const int32_t* W, const int32_t* stride, int32_t nW, int scope, int sigma_mode,
                               double kappa, double* state, double* stats, double* snr, int32_t* widx,
                               int nthreads)
{
    if (R < 1 || nW < 1 || L_view < 1 || new_col_begin < 0 || new_col_begin > L_view) return -1;
    for (int i = 0; i < nW; ++i)
        if (W[i] < 1 || (i > 0 && W[i] <= W[i - 1]) || (stride && stride[i] < 1)) return -1;
    if (stride && stride[0] != 1) return -1;       /* every start keeps at least the first width */
    int nmax = W[nW - 1];
    if (nmax > L_view) return -1;
    int64_t n_out = L_view - nmax + 1;
    int need_y = (sigma_mode != SIG_SQRTN);
    int64_t n_units = (scope == SCOPE_PLANE) ? 1 : R;
    if (nthreads < 1) nthreads = 1;

    /* per-row partials of this step, combined into the units below */
    double* part = (double*)calloc((size_t)R * 6, sizeof(double));
    #pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t r = 0; r < R; ++r) {
        const double* row = x + r * L_view;
        oracle_chan_stream(row + new_col_begin, L_view - new_col_begin, part + r * 6);
        if (need_y) {
            double* y = (double*)malloc(sizeof(double) * (size_t)n_out);
            nmax_series(row, n_out, nmax, y);
            oracle_chan_stream(y, n_out, part + r * 6 + 3);
            free(y);
        }
    }
    /* combine: a ROW unit is its own row; the PLANE unit takes rows in order */
    for (int64_t u = 0; u < n_units; ++u) {
        double* st = state + u * 6;
        int64_t r0 = (scope == SCOPE_PLANE) ? 0 : u;
        int64_t r1 = (scope == SCOPE_PLANE) ? R : u + 1;
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t r = r0; r < r1; ++r) {
            oracle_chan_merge(acc, part + r * 6, acc);
            oracle_chan_merge(acc + 3, part + r * 6 + 3, acc + 3);
        }
        oracle_chan_merge(st, acc, st);
        oracle_chan_merge(st + 3, acc + 3, st + 3);
        unit_coefficients(st, sigma_mode, kappa, nmax, stats + u * 5);
    }
    free(part);

    #pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t r = 0; r < R; ++r) {
        int64_t u = (scope == SCOPE_PLANE) ? 0 : r;
        detect_row(x + r * L_view, n_out, W, stride, nW, stats + u * 5, snr + r * n_out, widx + r * n_out);
    }
    return 0;
}

/* Sec. 2.4: keep every (row, t) whose highest SNR is >= f_T.  Emits the row
 * (DM-trial index), t + t_offset, the SNR and the boxcar width, in row-major
 * order; writes at most cap entries and returns the total found.            */
int64_t oracle_select(const double* snr, const int32_t* widx, int64_t R, int64_t n_out,
                      const int32_t* W, double f_T, int64_t t_offset,
                      int64_t* rows, int64_t* ts, double* snrs, int32_t* widths, int64_t cap)
{
    int64_t cnt = 0;
    for (int64_t r = 0; r < R; ++r)
        for (int64_t t = 0; t < n_out; ++t) {
            double s = snr[r * n_out + t];
            if (s >= f_T) {
                if (cnt < cap) {
                    rows[cnt] = r;
                    ts[cnt] = t + t_offset;
                    snrs[cnt] = s;
                    widths[cnt] = W[widx[r * n_out + t]];
                }
                ++cnt;
            }
        }
    return cnt;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
