/* Drives the C oracle (oracle/spd_oracle.c) over every scope, sigma mode and
 * edge shape with exactly sized heap buffers, for a build with the address
 * and undefined-behaviour sanitizers (tests/test_host_sanitizers.py).  Exits
 * non-zero on a failed check; the sanitizers abort on a bad access. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_stream_step(const double* x, int64_t R, int64_t L_view, int64_t new_col_begin, const int32_t* W,
                       int32_t nW, int scope, int sigma_mode, double kappa, double* state, double* stats,
                       double* snr, int32_t* widx, int nthreads);
int oracle_stream_step_strided(const double* x, int64_t R, int64_t L_view, int64_t new_col_begin,
                               const int32_t* W, const int32_t* stride, int32_t nW, int scope, int sigma_mode,
                               double kappa, double* state, double* stats, double* snr, int32_t* widx,
                               int nthreads);
int64_t oracle_select(const double* snr, const int32_t* widx, int64_t R, int64_t n_out, const int32_t* W,
                      double f_T, int64_t t_offset, int64_t* rows, int64_t* ts, double* snrs, int32_t* widths,
                      int64_t cap);
void oracle_chan_stream(const double* x, int64_t n, double* out3);
void oracle_chan_merge(const double* a3, const double* b3, double* out3);

static int fails = 0;
#define CHECK(c, msg)                                                   \
    do {                                                                \
        if (!(c)) {                                                     \
            printf("FAIL line %d: %s\n", __LINE__, msg);                \
            ++fails;                                                    \
        }                                                               \
    } while (0)

static uint64_t lcg = 88172645463325252ull;
static double unif(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}
static double gauss(void)
{
    double u = unif(), v = unif();
    return sqrt(-2.0 * log(u + 1e-300)) * cos(6.283185307179586 * v);
}

static void run_case(int64_t R, int64_t L, const int32_t* W, const int32_t* stride, int nW, int scope, int mode,
                     int64_t ncb)
{
    const int64_t nmax = W[nW - 1], n_out = L - nmax + 1, units = scope ? 1 : R;
    double* x = malloc(sizeof(double) * (size_t)(R * L));
    double* state = calloc((size_t)units * 6, sizeof(double));
    double* stats = malloc(sizeof(double) * (size_t)units * 5);
    double* snr = malloc(sizeof(double) * (size_t)(R * n_out));
    int32_t* widx = malloc(sizeof(int32_t) * (size_t)(R * n_out));
    for (int64_t i = 0; i < R * L; ++i) x[i] = 3.0 + gauss();
    if (R > 1)
        for (int64_t t = 0; t < L; ++t) x[L + t] = 0.5;                   /* a constant row */
    int rc = oracle_stream_step_strided(x, R, L, 0, W, stride, nW, scope, mode, 1.0, state, stats, snr, widx, 2);
    CHECK(rc == 0, "step");
    /* a second step over the same view with only its last columns new */
    rc = oracle_stream_step_strided(x, R, L, ncb, W, stride, nW, scope, mode, 1.0, state, stats, snr, widx, 2);
    CHECK(rc == 0, "accumulating step");
    for (int64_t i = 0; i < R * n_out; ++i) {
        CHECK(isfinite(snr[i]), "finite snr");
        CHECK(widx[i] >= 0 && widx[i] < nW, "width index in range");
        if (stride) CHECK((i % n_out) % stride[widx[i]] == 0, "width evaluated at its start");
    }
    const int64_t cap = 3;
    int64_t* rows = malloc(sizeof(int64_t) * cap);
    int64_t* ts = malloc(sizeof(int64_t) * cap);
    double* snrs = malloc(sizeof(double) * cap);
    int32_t* widths = malloc(sizeof(int32_t) * cap);
    const int64_t total = oracle_select(snr, widx, R, n_out, W, -1e300, 7, rows, ts, snrs, widths, cap);
    CHECK(total == R * n_out, "select counts every sample at -inf threshold");
    CHECK(ts[0] == 7, "select t_offset");
    free(rows); free(ts); free(snrs); free(widths);
    free(x); free(state); free(stats); free(snr); free(widx);
}

int main(void)
{
    const int32_t w16[16] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16};
    const int32_t odd[5] = {1, 3, 8, 21, 64};
    const int32_t dw[12] = {1, 2, 3, 4, 5, 6, 7, 8, 18, 20, 36, 40};
    const int32_t ds[12] = {1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 4, 4};
    for (int scope = 0; scope < 2; ++scope)
        for (int mode = 0; mode < 4; ++mode) {
            run_case(3, 1000, w16, NULL, 16, scope, mode, 900);
            run_case(1, 16, w16, NULL, 16, scope, mode, 16);                /* one start, no new column */
            run_case(2, 17, w16, NULL, 16, scope, mode, 0);
            run_case(3, 777, odd, NULL, 5, scope, mode, 700);
            run_case(2, 64, odd, NULL, 5, scope, mode, 1);
            run_case(3, 513, dw, ds, 12, scope, mode, 500);
        }
    /* argument errors */
    double x[8] = {0}, st[6] = {0}, s5[5], o[8];
    int32_t wi[8];
    const int32_t bad[2] = {2, 2}, big[1] = {9}, st2[2] = {2, 1}, w12[2] = {1, 2};
    CHECK(oracle_stream_step(x, 1, 8, 0, bad, 2, 0, 0, 1.0, st, s5, o, wi, 1) == -1, "non-increasing widths");
    CHECK(oracle_stream_step(x, 1, 8, 0, big, 1, 0, 0, 1.0, st, s5, o, wi, 1) == -1, "Nmax > L");
    CHECK(oracle_stream_step(x, 1, 8, 9, w12, 2, 0, 0, 1.0, st, s5, o, wi, 1) == -1, "new_col_begin > L");
    CHECK(oracle_stream_step_strided(x, 1, 8, 0, w12, st2, 2, 0, 0, 1.0, st, s5, o, wi, 1) == -1, "stride[0] != 1");
    /* merges with empty parts are the identity */
    double a[3], e[3] = {0, 0, 0}, m[3];
    const double v[4] = {1.0, 2.0, 4.0, 8.0};
    oracle_chan_stream(v, 4, a);
    oracle_chan_merge(a, e, m);
    CHECK(m[0] == a[0] && m[1] == a[1] && m[2] == a[2], "merge with empty part");
    oracle_chan_merge(e, a, m);
    CHECK(m[0] == a[0] && m[1] == a[1] && m[2] == a[2], "empty part merged with");
    if (fails) return 1;
    printf("ok\n");
    return 0;
}
