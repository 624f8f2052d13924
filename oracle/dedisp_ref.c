/*
 * Plain C oracle for brute-force incoherent dedispersion.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests and by the benchmark's
 * CPU-baseline leg through ctypes; the product library never links it.
 * It shares no code with the HIP library.
 *
 * The operator (the paper names dedispersion as a pipeline module in its
 * Introduction and gives no formula; this is the standard brute-force
 * definition):
 *   DM_i    = lo + i*step,            i < round((hi - lo)/step)
 *   s[d][c] = floor(K*DM_d*(1/f_c^2 - 1/f_ref^2)/(tsamp*ds) + 1/2),
 *             K = 4.148808e3 s MHz^2 pc^-1 cm^3, f_ref = max_c f_c
 *   x_r[c][t'] = sum_{k<ds} x[c][ds*t' + k],  t' < floor(nsamp/ds)
 *   out_r[d][t] = sum_c w_c * x_r[c][t + s[d][c]],
 *             t < nout_r = floor(nsamp/ds) - max_{d,c} s[d][c]
 * Ranges are concatenated in plan order, each DM-major.
 *
 * Integer input is summed in int32 (callers must keep 255*nchans*ds below
 * 2^31, which every entry point checks); float input is summed in double.
 * Loops run over DM rows in parallel with OpenMP; nothing else is blocked
 * or reordered.
 *
 * Every entry point returns 0 on success and a negative value on bad
 * arguments.  Ranges are passed as nranges x 4 doubles: lo, hi, step, ds.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double K_DM = 4.148808e3;

static int64_t range_ndms(const double *rg)
{
    return (int64_t)floor((rg[1] - rg[0]) / rg[2] + 0.5);
}

static double freq_ref(const double *freqs, int32_t nchans)
{
    double m = freqs[0];
    for (int32_t c = 1; c < nchans; ++c)
        if (freqs[c] > m)
            m = freqs[c];
    return m;
}

/* s[d][c] for one range, row-major [ndms][nchans]. */
static void range_shifts(const double *freqs, int32_t nchans, double tsamp,
                         const double *rg, int32_t *s)
{
    const double fr = freq_ref(freqs, nchans);
    const int64_t nd = range_ndms(rg);
    const int ds = (int)rg[3];
    for (int64_t i = 0; i < nd; ++i) {
        const double dm = rg[0] + (double)i * rg[2];
        for (int32_t c = 0; c < nchans; ++c) {
            const double delta = 1.0 / (freqs[c] * freqs[c]) - 1.0 / (fr * fr);
            const double x = K_DM * dm * delta / (tsamp * ds);
            s[i * nchans + c] = (int32_t)floor(x + 0.5);
        }
    }
}

static int32_t max_of(const int32_t *s, int64_t n)
{
    int32_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (s[i] > m)
            m = s[i];
    return m;
}

static int check_common(int32_t nchans, int64_t nsamp, double tsamp,
                        const double *freqs, const double *ranges,
                        int32_t nranges)
{
    if (!freqs || !ranges || nchans <= 0 || nsamp <= 0 || nranges <= 0 ||
        !(tsamp > 0.0))
        return -1;
    for (int32_t r = 0; r < nranges; ++r) {
        const double *rg = ranges + 4 * r;
        if (!(rg[2] > 0.0) || rg[3] < 1.0 || range_ndms(rg) <= 0)
            return -1;
    }
    return 0;
}

/* Number of DMs and valid output samples of every range. */
int oracle_plan_sizes(const double *freqs, int32_t nchans, double tsamp,
                      int64_t nsamp, const double *ranges, int32_t nranges,
                      int32_t *ndms, int64_t *nout)
{
    if (check_common(nchans, nsamp, tsamp, freqs, ranges, nranges))
        return -1;
    for (int32_t r = 0; r < nranges; ++r) {
        const double *rg = ranges + 4 * r;
        const int64_t nd = range_ndms(rg);
        int32_t *s = (int32_t *)malloc(sizeof(int32_t) * nd * nchans);
        if (!s)
            return -2;
        range_shifts(freqs, nchans, tsamp, rg, s);
        ndms[r] = (int32_t)nd;
        nout[r] = nsamp / (int64_t)rg[3] - max_of(s, nd * nchans);
        free(s);
    }
    return 0;
}

/* Shift table of one range into s (ndms x nchans int32). */
int oracle_range_shifts(const double *freqs, int32_t nchans, double tsamp,
                        const double *range, int32_t *s)
{
    if (!freqs || !range || !s || nchans <= 0 || !(tsamp > 0.0))
        return -1;
    range_shifts(freqs, nchans, tsamp, range, s);
    return 0;
}

/*
 * Rows [d_begin, d_end) of one range of the uint8 forward into out
 * ((d_end - d_begin) x nout_r int32).
 */
int oracle_dedisperse_u8_rows(const uint8_t *x, int32_t nchans, int64_t nsamp,
                              const double *freqs, double tsamp,
                              const double *range, int32_t d_begin,
                              int32_t d_end, int32_t *out, int32_t nthreads)
{
    if (!x || !out || check_common(nchans, nsamp, tsamp, freqs, range, 1))
        return -1;
    const int ds = (int)range[3];
    if (255.0 * nchans * ds >= 2147483648.0)
        return -3;
    const int64_t nd = range_ndms(range);
    if (d_begin < 0 || d_end > nd || d_begin >= d_end)
        return -1;
    int32_t *s = (int32_t *)malloc(sizeof(int32_t) * nd * nchans);
    if (!s)
        return -2;
    range_shifts(freqs, nchans, tsamp, range, s);
    const int64_t nbin = nsamp / ds;
    const int64_t nout = nbin - max_of(s, nd * nchans);
    if (nout <= 0) {
        free(s);
        return -4;
    }
    /* Binned input (sum of ds adjacent samples). */
    int32_t *xr = NULL;
    if (ds > 1) {
        xr = (int32_t *)malloc(sizeof(int32_t) * nchans * nbin);
        if (!xr) {
            free(s);
            return -2;
        }
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int32_t c = 0; c < nchans; ++c)
            for (int64_t t = 0; t < nbin; ++t) {
                int32_t v = 0;
                for (int k = 0; k < ds; ++k)
                    v += x[(int64_t)c * nsamp + t * ds + k];
                xr[(int64_t)c * nbin + t] = v;
            }
    }
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int32_t d = d_begin; d < d_end; ++d) {
        int32_t *acc = out + (int64_t)(d - d_begin) * nout;
        memset(acc, 0, sizeof(int32_t) * nout);
        for (int32_t c = 0; c < nchans; ++c) {
            const int64_t sh = s[(int64_t)d * nchans + c];
            if (ds == 1) {
                const uint8_t *row = x + (int64_t)c * nsamp + sh;
                for (int64_t t = 0; t < nout; ++t)
                    acc[t] += row[t];
            } else {
                const int32_t *row = xr + (int64_t)c * nbin + sh;
                for (int64_t t = 0; t < nout; ++t)
                    acc[t] += row[t];
            }
        }
    }
    free(xr);
    free(s);
    return 0;
}

/* Whole uint8 forward, ranges concatenated, into out (capacity in elements). */
int oracle_dedisperse_u8(const uint8_t *x, int32_t nchans, int64_t nsamp,
                         const double *freqs, double tsamp,
                         const double *ranges, int32_t nranges, int32_t *out,
                         int64_t capacity, int32_t nthreads)
{
    if (check_common(nchans, nsamp, tsamp, freqs, ranges, nranges) || !out)
        return -1;
    int64_t off = 0;
    for (int32_t r = 0; r < nranges; ++r) {
        int32_t nd;
        int64_t nout;
        int rc = oracle_plan_sizes(freqs, nchans, tsamp, nsamp, ranges + 4 * r,
                                   1, &nd, &nout);
        if (rc)
            return rc;
        if (nout <= 0)
            return -4;
        if (off + (int64_t)nd * nout > capacity)
            return -5;
        rc = oracle_dedisperse_u8_rows(x, nchans, nsamp, freqs, tsamp,
                                       ranges + 4 * r, 0, nd, out + off,
                                       nthreads);
        if (rc)
            return rc;
        off += (int64_t)nd * nout;
    }
    return 0;
}

/*
 * Float forward with per-channel weights (NULL means all ones), summed in
 * double, ranges concatenated into out (double, capacity in elements).
 */
int oracle_dedisperse_f32(const float *x, int32_t nchans, int64_t nsamp,
                          const double *freqs, double tsamp,
                          const double *ranges, int32_t nranges,
                          const float *weights, double *out, int64_t capacity,
                          int32_t nthreads)
{
    if (!x || !out || check_common(nchans, nsamp, tsamp, freqs, ranges, nranges))
        return -1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#endif
    int64_t off = 0;
    for (int32_t r = 0; r < nranges; ++r) {
        const double *rg = ranges + 4 * r;
        const int ds = (int)rg[3];
        const int64_t nd = range_ndms(rg);
        int32_t *s = (int32_t *)malloc(sizeof(int32_t) * nd * nchans);
        if (!s)
            return -2;
        range_shifts(freqs, nchans, tsamp, rg, s);
        const int64_t nbin = nsamp / ds;
        const int64_t nout = nbin - max_of(s, nd * nchans);
        if (nout <= 0) {
            free(s);
            return -4;
        }
        if (off + nd * nout > capacity) {
            free(s);
            return -5;
        }
        double *xr = (double *)malloc(sizeof(double) * nchans * nbin);
        if (!xr) {
            free(s);
            return -2;
        }
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int32_t c = 0; c < nchans; ++c) {
            const double w = weights ? (double)weights[c] : 1.0;
            for (int64_t t = 0; t < nbin; ++t) {
                double v = 0.0;
                for (int k = 0; k < ds; ++k)
                    v += (double)x[(int64_t)c * nsamp + t * ds + k];
                xr[(int64_t)c * nbin + t] = w * v;
            }
        }
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
        for (int64_t d = 0; d < nd; ++d) {
            double *acc = out + off + d * nout;
            for (int64_t t = 0; t < nout; ++t)
                acc[t] = 0.0;
            for (int32_t c = 0; c < nchans; ++c) {
                const double *row = xr + (int64_t)c * nbin + s[d * nchans + c];
                for (int64_t t = 0; t < nout; ++t)
                    acc[t] += row[t];
            }
        }
        free(xr);
        free(s);
        off += nd * nout;
    }
    return 0;
}

/* Threads OpenMP would use for a parallel region (for reporting). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Adjoint of the float forward (transpose of x -> out for fixed weights, and
 * the derivative in the weights), in double:
 *   G_r[c][tau] = sum_{d in r, 0 <= tau - s[d][c] < nout_r} g_r[d][tau - s[d][c]]
 *   dX[c][ds*tau + k] = w_c * sum_r G_r[c][tau]           (k < ds)
 *   dw[c] = sum_r sum_tau x_r[c][tau] * G_r[c][tau]
 * g is the concatenated per-range output gradient (double).  dX is
 * [nchans][nsamp] double (may be NULL), dw [nchans] double (may be NULL).
 * OpenMP runs over channels.
 */
int oracle_adjoint_f32(const float *x, int32_t nchans, int64_t nsamp,
                       const double *freqs, double tsamp, const double *ranges,
                       int32_t nranges, const float *weights, const double *g,
                       double *dX, double *dw, int32_t nthreads)
{
    if (!x || !g || check_common(nchans, nsamp, tsamp, freqs, ranges, nranges))
        return -1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#endif
    if (dX)
        memset(dX, 0, sizeof(double) * nchans * nsamp);
    if (dw)
        memset(dw, 0, sizeof(double) * nchans);
    int64_t off = 0;
    for (int32_t r = 0; r < nranges; ++r) {
        const double *rg = ranges + 4 * r;
        const int ds = (int)rg[3];
        const int64_t nd = range_ndms(rg);
        int32_t *s = (int32_t *)malloc(sizeof(int32_t) * nd * nchans);
        if (!s)
            return -2;
        range_shifts(freqs, nchans, tsamp, rg, s);
        const int64_t nbin = nsamp / ds;
        const int64_t nout = nbin - max_of(s, nd * nchans);
        if (nout <= 0) {
            free(s);
            return -4;
        }
        int err = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
        for (int32_t c = 0; c < nchans; ++c) {
            double *G = (double *)calloc((size_t)nbin, sizeof(double));
            if (!G) {
                err = 1;
                continue;
            }
            for (int64_t d = 0; d < nd; ++d) {
                const double *gr = g + off + d * nout;
                const int64_t sh = s[d * nchans + c];
                for (int64_t t = 0; t < nout; ++t)
                    G[t + sh] += gr[t];
            }
            const double w = weights ? (double)weights[c] : 1.0;
            double acc = 0.0;
            for (int64_t tau = 0; tau < nbin; ++tau) {
                double xs = 0.0;
                for (int k = 0; k < ds; ++k) {
                    const int64_t t = tau * ds + k;
                    xs += (double)x[(int64_t)c * nsamp + t];
                    if (dX)
                        dX[(int64_t)c * nsamp + t] += w * G[tau];
                }
                acc += xs * G[tau];
            }
            if (dw)
                dw[c] += acc;
            free(G);
        }
        free(s);
        if (err)
            return -2;
        off += nd * nout;
    }
    return 0;
}
