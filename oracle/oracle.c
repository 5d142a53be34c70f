/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the SPOTLIGHT
 * single-pulse search hot path (brute-force incoherent dedispersion followed by
 * the boxcar single-pulse search and peak filtering).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load
 * this file; only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or constant with the HIP
 * library: every quantity (delay table, moments, thresholds, peak filter) is
 * recomputed here from its definition.
 *
 * Floating point: IEEE binary64, compiled with -ffp-contract=off (no fused
 * multiply-add), so every expression rounds exactly as written.
 *
 * Paper sections followed:
 *   - cold-plasma delay, Eq. (1) of the dedispersion section: delay of channel
 *     frequency f relative to the highest frequency of the band, dispersion
 *     constant 4.1488064239e3 MHz^2 pc^-1 cm^3 s;
 *   - brute-force incoherent dedispersion (dedispersion section): every trial DM
 *     row is the sum over channels of the channel shifted by its delay;
 *   - single-pulse search (single pulse search section): boxcar matched filters
 *     of several trial widths applied to every DM row, candidates kept above a
 *     threshold in units of sigma;
 *   - peak filtering (same section): in the DM-time plane, only the highest-S/N
 *     point of each window survives, with a 3x3 stencil and an 11x11 stencil;
 *   - candidate optimisation (candidate optimisation section): DBSCAN in the
 *     DM-time plane, clusters of at least 5 points, the highest-S/N member kept,
 *     then S/N, DM and width thresholds and the anti-coincidence filter.
 * Readings where the paper is silent (reference frequency, rounding of delays,
 * normaliser, window anchors, NMS key, DBSCAN units) are the ones listed in the
 * design notes of the repository; each is restated at the function below.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_DISPERSION_CONSTANT 4148.8064239 /* MHz^2 pc^-1 cm^3 s, Eq. (1) */

/* Threads the oracle's parallel loops use. */
int32_t orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the threads of the oracle's parallel loops (n >= 1). */
void orc_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Eq. (1): integer delay table                                               */
/* ------------------------------------------------------------------------ */
/*
 * f_c = fch1 + c*foff; the reference frequency is the highest channel centre.
 * delay[d][c] = round-half-away( ((D*DM_d) * (1/f_c^2 - 1/f_ref^2)) / tsamp ).
 * Returns the number of entries whose unrounded value lies within 1e-9 of a
 * half-integer (a rounding tie that a different evaluation order could flip).
 */
int64_t orc_delay_table(int32_t nch, double fch1, double foff, double tsamp,
                        int32_t ndm, const double *dms, int64_t *out)
{
    double fref = fch1;
    for (int32_t c = 0; c < nch; ++c) {
        double f = fch1 + (double)c * foff;
        if (f > fref) fref = f;
    }
    int64_t ties = 0;
    for (int32_t d = 0; d < ndm; ++d) {
        for (int32_t c = 0; c < nch; ++c) {
            double f = fch1 + (double)c * foff;
            double v = ((ORC_DISPERSION_CONSTANT * dms[d]) *
                        ((1.0 / (f * f)) - (1.0 / (fref * fref)))) / tsamp;
            double frac = v - floor(v);
            if (fabs(frac - 0.5) < 1e-9) ++ties;
            out[(int64_t)d * nch + c] = (int64_t)llround(v);
        }
    }
    return ties;
}

/* ------------------------------------------------------------------------ */
/* Brute-force dedispersion                                                    */
/* ------------------------------------------------------------------------ */
/*
 * X[d][t] = sum_c x[c][t + delay[d][c]]   for t in [0, n_dd).
 * x is channel-major uint8 with row pitch `pitch` bytes; the caller guarantees
 * t + delay < n_in for every term.
 */
void orc_dedisperse(const uint8_t *x, int64_t pitch, int32_t nch,
                    const int64_t *delay, int32_t ndm, int32_t n_dd, int64_t *X)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t d = 0; d < ndm; ++d) {
        int64_t *row = X + (int64_t)d * n_dd;
        for (int32_t t = 0; t < n_dd; ++t) row[t] = 0;
        for (int32_t c = 0; c < nch; ++c) {
            const uint8_t *src = x + (int64_t)c * pitch + delay[(int64_t)d * nch + c];
            for (int32_t t = 0; t < n_dd; ++t) row[t] += src[t];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Moments of each DM row over segments of the owned samples                 */
/* ------------------------------------------------------------------------ */
/*
 * Segment k covers t in [k*L, min((k+1)*L, n_out)); nseg = ceil(n_out / L).
 * n, S1 = sum X, S2 = sum X^2 as exact integers.
 */
void orc_moments(const int64_t *X, int32_t ndm, int32_t n_dd, int32_t n_out,
                 int32_t L, int64_t *n, int64_t *S1, int64_t *S2)
{
    int32_t nseg = (n_out + L - 1) / L;
#pragma omp parallel for schedule(static)
    for (int32_t d = 0; d < ndm; ++d) {
        for (int32_t k = 0; k < nseg; ++k) {
            int32_t lo = k * L, hi = (k + 1) * L;
            if (hi > n_out) hi = n_out;
            int64_t s1 = 0, s2 = 0;
            for (int32_t t = lo; t < hi; ++t) {
                int64_t v = X[(int64_t)d * n_dd + t];
                s1 += v;
                s2 += v * v;
            }
            n[(int64_t)d * nseg + k] = hi - lo;
            S1[(int64_t)d * nseg + k] = s1;
            S2[(int64_t)d * nseg + k] = s2;
        }
    }
}

/*
 * Mean and standard deviation from exact moments:
 *   V = n*S2 - S1^2 (exact, 128-bit), mu = S1/n, sigma = sqrt(V)/n.
 * sigma = 0 when V = 0 (a constant row has no hits).
 */
void orc_mu_sigma(int64_t n, int64_t S1, int64_t S2, double *mu, double *sigma)
{
    __int128 V = (__int128)n * (__int128)S2 - (__int128)S1 * (__int128)S1;
    *mu = (double)S1 / (double)n;
    *sigma = (V > 0) ? sqrt((double)V) / (double)n : 0.0;
}

/* S/N of a boxcar sum B of width w against a row mean mu and sigma. */
double orc_snr(int64_t B, int32_t w, double mu, double sigma)
{
    return ((double)B - (double)w * mu) / (sigma * sqrt((double)w));
}

/* ------------------------------------------------------------------------ */
/* Boxcar search with threshold and best width                               */
/* ------------------------------------------------------------------------ */
/*
 * For every DM row d and owned sample t in [0, n_out):
 *   B_w = X[d][t] + ... + X[d][t+w-1]  (window anchored at t),
 *   snr_w = orc_snr(B_w, w, mu, sigma) with mu, sigma of t's segment,
 *   hit if some snr_w >= theta; the reported width maximises snr_w over the
 *   widths in ascending order, an equal value keeping the smaller width.
 * Output in (d, t) order.  If out_* is NULL only the count is returned; the
 * caller calls again with buffers of that size.
 */
int64_t orc_search(const int64_t *X, int32_t ndm, int32_t n_dd, int32_t n_out,
                   int32_t L, const int32_t *widths, int32_t nw, double theta,
                   int32_t *out_d, int32_t *out_t, int32_t *out_w,
                   int64_t *out_B, double *out_snr)
{
    int32_t nseg = (n_out + L - 1) / L;
    int64_t *per_row = (int64_t *)calloc((size_t)ndm + 1, sizeof(int64_t));
    double *mu = (double *)malloc(sizeof(double) * (size_t)ndm * nseg);
    double *sg = (double *)malloc(sizeof(double) * (size_t)ndm * nseg);
    int64_t *n = (int64_t *)malloc(sizeof(int64_t) * (size_t)ndm * nseg);
    int64_t *s1 = (int64_t *)malloc(sizeof(int64_t) * (size_t)ndm * nseg);
    int64_t *s2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)ndm * nseg);
    orc_moments(X, ndm, n_dd, n_out, L, n, s1, s2);
    for (int64_t i = 0; i < (int64_t)ndm * nseg; ++i)
        orc_mu_sigma(n[i], s1[i], s2[i], &mu[i], &sg[i]);

    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            if (!out_d) break;
            int64_t acc = 0;
            for (int32_t d = 0; d <= ndm; ++d) {
                int64_t c = per_row[d];
                per_row[d] = acc;
                acc += c;
            }
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int32_t d = 0; d < ndm; ++d) {
            const int64_t *row = X + (int64_t)d * n_dd;
            int64_t count = 0, pos = pass ? per_row[d] : 0;
            for (int32_t t = 0; t < n_out; ++t) {
                int32_t k = t / L;
                double m = mu[(int64_t)d * nseg + k], s = sg[(int64_t)d * nseg + k];
                if (!(s > 0.0)) continue;
                int found = 0;
                int32_t bw = 0;
                int64_t bB = 0;
                double bs = 0.0;
                for (int32_t j = 0; j < nw; ++j) {
                    int32_t w = widths[j];
                    int64_t B = 0;
                    for (int32_t i = 0; i < w; ++i) B += row[t + i];
                    double snr = orc_snr(B, w, m, s);
                    if (snr >= theta && (!found || snr > bs)) {
                        found = 1;
                        bw = w;
                        bB = B;
                        bs = snr;
                    }
                }
                if (!found) continue;
                if (pass == 0) {
                    ++count;
                } else {
                    out_d[pos] = d;
                    out_t[pos] = t;
                    out_w[pos] = bw;
                    out_B[pos] = bB;
                    out_snr[pos] = bs;
                    ++pos;
                }
            }
            if (pass == 0) per_row[d] = count;
        }
    }
    int64_t total = 0;
    if (out_d) {
        total = per_row[ndm];
    } else {
        for (int32_t d = 0; d < ndm; ++d) total += per_row[d];
    }
    free(per_row);
    free(mu);
    free(sg);
    free(n);
    free(s1);
    free(s2);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Peak filter (non-maximum suppression in the DM-time index plane)           */
/* ------------------------------------------------------------------------ */
/*
 * Point q beats point p when (snr_q, -d_q, -t_q) > (snr_p, -d_p, -t_p)
 * lexicographically.  Among the points with alive_in != 0, p survives iff no
 * other such q with |d_q - d_p| <= rd and |t_q - t_p| <= rt beats it.
 * Points must be unique in (d, t), with 0 <= d < ndm and 0 <= t < ntime.
 * Uses a dense (d, t) -> index map; writes alive_out (0/1).
 */
static int orc_beats(double sq, int32_t dq, int32_t tq, double sp, int32_t dp, int32_t tp)
{
    if (sq != sp) return sq > sp;
    if (dq != dp) return dq < dp;
    return tq < tp;
}

int32_t orc_nms(const int32_t *d, const int32_t *t, const double *snr, int64_t n,
                int32_t ndm, int32_t ntime, int32_t rd, int32_t rt,
                const uint8_t *alive_in, uint8_t *alive_out)
{
    int32_t *map = (int32_t *)malloc(sizeof(int32_t) * (size_t)ndm * ntime);
    if (!map) return -1;
    for (int64_t i = 0; i < (int64_t)ndm * ntime; ++i) map[i] = -1;
    for (int64_t i = 0; i < n; ++i)
        if (alive_in[i]) map[(int64_t)d[i] * ntime + t[i]] = (int32_t)i;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        if (!alive_in[i]) {
            alive_out[i] = 0;
            continue;
        }
        int keep = 1;
        for (int32_t dd = -rd; dd <= rd && keep; ++dd) {
            int32_t dq = d[i] + dd;
            if (dq < 0 || dq >= ndm) continue;
            for (int32_t dt = -rt; dt <= rt; ++dt) {
                int32_t tq = t[i] + dt;
                if (tq < 0 || tq >= ntime || (dd == 0 && dt == 0)) continue;
                int32_t q = map[(int64_t)dq * ntime + tq];
                if (q >= 0 && orc_beats(snr[q], dq, tq, snr[i], d[i], t[i])) {
                    keep = 0;
                    break;
                }
            }
        }
        alive_out[i] = (uint8_t)keep;
    }
    free(map);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* DBSCAN (Ester et al. 1996) as used by the candidate optimisation stage     */
/* ------------------------------------------------------------------------ */
/*
 * Points (x_i, y_i); q is a neighbour of p iff (x_p-x_q)^2 + (y_p-y_q)^2 <= eps^2
 * (p is its own neighbour).  Core iff |N(p)| >= min_pts.  Clusters are the
 * connected components of core points under the neighbour relation, numbered
 * 0, 1, ... in order of their lowest-index core point.  A non-core point with
 * at least one core neighbour joins the lowest-numbered cluster among them;
 * other points are noise (label -1).  O(n^2) on purpose.
 */
int32_t orc_dbscan(const double *x, const double *y, int64_t n, double eps,
                   int32_t min_pts, int32_t *label)
{
    double e2 = eps * eps;
    uint8_t *core = (uint8_t *)calloc((size_t)(n ? n : 1), 1);
    int64_t *stack = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    for (int64_t p = 0; p < n; ++p) {
        int64_t cnt = 0;
        for (int64_t q = 0; q < n; ++q) {
            double dx = x[p] - x[q], dy = y[p] - y[q];
            if (dx * dx + dy * dy <= e2) ++cnt;
        }
        core[p] = cnt >= min_pts;
        label[p] = -1;
    }
    int32_t ncl = 0;
    for (int64_t p = 0; p < n; ++p) {
        if (!core[p] || label[p] >= 0) continue;
        int64_t top = 0;
        stack[top++] = p;
        label[p] = ncl;
        while (top) {
            int64_t a = stack[--top];
            for (int64_t q = 0; q < n; ++q) {
                if (!core[q] || label[q] >= 0) continue;
                double dx = x[a] - x[q], dy = y[a] - y[q];
                if (dx * dx + dy * dy <= e2) {
                    label[q] = ncl;
                    stack[top++] = q;
                }
            }
        }
        ++ncl;
    }
    for (int64_t p = 0; p < n; ++p) {
        if (core[p]) continue;
        int32_t best = -1;
        for (int64_t q = 0; q < n; ++q) {
            if (!core[q]) continue;
            double dx = x[p] - x[q], dy = y[p] - y[q];
            if (dx * dx + dy * dy <= e2 && (best < 0 || label[q] < best)) best = label[q];
        }
        label[p] = best;
    }
    free(core);
    free(stack);
    return ncl;
}
