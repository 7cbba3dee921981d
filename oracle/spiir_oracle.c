/*
 * FP64 CPU oracle for the SPIIR filter-bank hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU path is checked against.  It shares no code, header, table or helper with
 * the HIP library; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  Every argument and every operation is double
 * precision; callers promote float32 inputs and complex64 coefficients exactly.
 *
 * Complex values are interleaved (re, im) pairs.
 *
 * Readings of the paper taken here (Section II.B.1, Eq. zk and the text before
 * it, which describes the SPIIR output as the summation of the responses of all
 * first-order IIR filters):
 *   - every filter keeps its own state: y_k[n] = a_k y_k[n-1] + b_k x[n-d_k], and
 *     the template output is z_t[n] = sum over the template's filters of y_k[n]
 *     (Eq. zk written with the template sum fed back would couple all filters
 *     into one high-order filter, which contradicts the summed-response text);
 *   - the delay shifts the input only: with the undelayed filter
 *     w[j] = a w[j-1] + b x[j], Eq. zk's term for filter k is w[n - d_k];
 *   - delays are integer sample counts, zero state and zero input before the
 *     stream starts;
 *   - the sum runs over the template's F_t filters in ascending index order.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define SPO_OK 0
#define SPO_EINVAL 1

/* Number of threads the parallel loops below use. */
int spo_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of threads of the parallel loops (n >= 1). */
void spo_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Filtering: Eq. zk (Section II.B.1) as a sum of parallel first-order       */
/* complex IIR filters.                                                      */
/* ------------------------------------------------------------------------ */

/* Input sample at stream position j of detector det.  Positions before the
 * current block come from the history (the hist_len samples immediately
 * preceding x), and before that the stream is zero. */
static double input_at(const double *x, int64_t n, const double *hist, int64_t hist_len,
                       int64_t det, int64_t j)
{
    if (j >= 0)
        return x[det * n + j];
    if (hist != NULL && j >= -hist_len)
        return hist[det * hist_len + hist_len + j];
    return 0.0;
}

/*
 * z[det][t][i] (complex128) for i in [0, n): output of every template for a
 * block of n input samples per detector.
 *   offsets[T+1]   CSR: template t owns filters offsets[t] .. offsets[t+1]-1
 *   a, b [F]       complex feedback / feedforward coefficients
 *   d [F]          integer delays (samples)
 *   x [D][n]       real input block
 *   hist [D][hist_len] or NULL: the samples just before the block (streaming)
 *   state [D][F] complex128 or NULL: y_k at the sample before the block on
 *                  entry, overwritten with y_k at the block's last sample.
 *                  NULL means zero initial state and no state returned.
 * A block split into consecutive calls that carry state and history gives
 * bit-identical output to one call over the whole stream.
 */
int spo_filter(int32_t n_templates, const int32_t *offsets, const double *a, const double *b,
               const int32_t *d, int32_t n_det, int64_t n, const double *x,
               int64_t hist_len, const double *hist, double *state, double *z)
{
    if (n_templates < 0 || n_det < 0 || n < 0)
        return SPO_EINVAL;
    for (int32_t t = 0; t < n_templates; ++t)
        if (offsets[t + 1] < offsets[t])
            return SPO_EINVAL;
    const int64_t n_filters = offsets[n_templates];
    for (int64_t k = 0; k < n_filters; ++k)
        if (d[k] < 0 || (hist != NULL && d[k] > hist_len))
            return SPO_EINVAL;

    const int64_t jobs = (int64_t)n_det * n_templates;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t job = 0; job < jobs; ++job) {
        const int64_t det = job / n_templates;
        const int64_t t = job % n_templates;
        double *zt = z + 2 * (det * n_templates + t) * n;
        memset(zt, 0, sizeof(double) * 2 * (size_t)n);
        for (int64_t k = offsets[t]; k < offsets[t + 1]; ++k) {
            const double ar = a[2 * k], ai = a[2 * k + 1];
            const double br = b[2 * k], bi = b[2 * k + 1];
            double yr = 0.0, yi = 0.0;
            if (state != NULL) {
                yr = state[2 * (det * n_filters + k)];
                yi = state[2 * (det * n_filters + k) + 1];
            }
            for (int64_t i = 0; i < n; ++i) {
                const double xv = input_at(x, n, hist, hist_len, det, i - d[k]);
                /* y <- a*y + b*x, complex a, b, y and real x */
                const double nr = ar * yr - ai * yi + br * xv;
                const double ni = ar * yi + ai * yr + bi * xv;
                yr = nr;
                yi = ni;
                zt[2 * i] += yr;
                zt[2 * i + 1] += yi;
            }
            if (state != NULL) {
                state[2 * (det * n_filters + k)] = yr;
                state[2 * (det * n_filters + k) + 1] = yi;
            }
        }
    }
    return SPO_OK;
}

/* ------------------------------------------------------------------------ */
/* Peaks: the absolute SNR rho = |z| (Section II.C.1, under Eq. null_def) and */
/* at most one candidate per template per window (Section II.C.1, trigger    */
/* selection; the paper's window is one second).                             */
/* ------------------------------------------------------------------------ */

/*
 * For each row r of z (complex128 [rows][n]) and each window w of `window`
 * samples (the last window may be shorter): the largest |z|, the index in the
 * window where it occurs (lowest index among equal |z|^2), and the relative gap
 * (p1 - p2)/p1 between the largest and the second-largest |z| in the window
 * (0 for a window of one sample).  |z| is compared through |z|^2.
 */
int spo_peaks(int64_t rows, int64_t n, int64_t window, const double *z, double *peak,
              int32_t *argmax, double *margin)
{
    if (rows < 0 || n < 0 || window <= 0)
        return SPO_EINVAL;
    const int64_t n_win = (n + window - 1) / window;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < rows; ++r) {
        const double *zr = z + 2 * r * n;
        for (int64_t w = 0; w < n_win; ++w) {
            const int64_t lo = w * window;
            const int64_t hi = lo + window < n ? lo + window : n;
            double p1 = -1.0, p2 = -1.0;
            int64_t i1 = -1;
            for (int64_t i = lo; i < hi; ++i) {
                const double p = zr[2 * i] * zr[2 * i] + zr[2 * i + 1] * zr[2 * i + 1];
                if (p > p1) {
                    p2 = p1;
                    p1 = p;
                    i1 = i;
                } else if (p > p2) {
                    p2 = p;
                }
            }
            const double a1 = sqrt(p1);
            peak[r * n_win + w] = a1;
            argmax[r * n_win + w] = (int32_t)(i1 - lo);
            if (margin != NULL)
                margin[r * n_win + w] = (p2 < 0.0 || a1 == 0.0) ? 0.0 : (a1 - sqrt(p2)) / a1;
        }
    }
    return SPO_OK;
}

/* ------------------------------------------------------------------------ */
/* Gradients.                                                                */
/* Complex convention: for a real loss L and complex parameter c the         */
/* gradient is dL/dRe(c) + i dL/dIm(c).                                      */
/* ------------------------------------------------------------------------ */

/*
 * Gradient of a real loss L with respect to a_k and b_k, given
 * gz[det][t][i] = dL/dRe z_t[i] + i dL/dIm z_t[i] for the output of spo_filter
 * run from zero state and zero history on x[D][n].
 *
 * Forward-mode sensitivities: y_k is holomorphic in a_k and b_k, so
 *   eta_k[i] = dy_k[i]/db_k follows eta[i] = a eta[i-1] + x[i-d]
 *   xi_k[i]  = dy_k[i]/da_k follows xi[i]  = a xi[i-1]  + y[i-1]
 * and grad_b_k = sum_i gz_t[i] conj(eta_k[i]), grad_a_k = sum_i gz_t[i] conj(xi_k[i])
 * (summed over detectors).  This runs forward in time and is independent of
 * any reverse-time adjoint.
 *   grad_a, grad_b: complex128 [F], overwritten.
 */
int spo_grad(int32_t n_templates, const int32_t *offsets, const double *a, const double *b,
             const int32_t *d, int32_t n_det, int64_t n, const double *x, const double *gz,
             double *grad_a, double *grad_b)
{
    if (n_templates < 0 || n_det < 0 || n < 0)
        return SPO_EINVAL;
    const int64_t n_filters = offsets[n_templates];
    for (int64_t k = 0; k < n_filters; ++k)
        if (d[k] < 0)
            return SPO_EINVAL;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t t = 0; t < n_templates; ++t) {
        for (int64_t k = offsets[t]; k < offsets[t + 1]; ++k) {
            const double ar = a[2 * k], ai = a[2 * k + 1];
            const double br = b[2 * k], bi = b[2 * k + 1];
            double gar = 0.0, gai = 0.0, gbr = 0.0, gbi = 0.0;
            for (int64_t det = 0; det < n_det; ++det) {
                const double *g = gz + 2 * (det * n_templates + t) * n;
                double yr = 0.0, yi = 0.0;     /* y[i-1] */
                double er = 0.0, ei = 0.0;     /* eta[i-1] */
                double sr = 0.0, si = 0.0;     /* xi[i-1] */
                for (int64_t i = 0; i < n; ++i) {
                    const double xv = input_at(x, n, NULL, 0, det, i - d[k]);
                    /* xi[i] = a xi[i-1] + y[i-1] (uses y before its update) */
                    const double nsr = ar * sr - ai * si + yr;
                    const double nsi = ar * si + ai * sr + yi;
                    /* eta[i] = a eta[i-1] + x[i-d] */
                    const double ner = ar * er - ai * ei + xv;
                    const double nei = ar * ei + ai * er;
                    /* y[i] = a y[i-1] + b x[i-d] */
                    const double nyr = ar * yr - ai * yi + br * xv;
                    const double nyi = ar * yi + ai * yr + bi * xv;
                    sr = nsr; si = nsi; er = ner; ei = nei; yr = nyr; yi = nyi;
                    const double gr = g[2 * i], gi = g[2 * i + 1];
                    /* g * conj(xi), g * conj(eta) */
                    gar += gr * sr + gi * si;
                    gai += gi * sr - gr * si;
                    gbr += gr * er + gi * ei;
                    gbi += gi * er - gr * ei;
                }
            }
            grad_a[2 * k] = gar;
            grad_a[2 * k + 1] = gai;
            grad_b[2 * k] = gbr;
            grad_b[2 * k + 1] = gbi;
        }
    }
    return SPO_OK;
}

/*
 * Overlap loss and its gradient in closed form (Eq. overlap, Section II.B.1).
 *
 * u_t[m] = sum_k b_k a_k^(m-d_k) [m >= d_k] is the summed impulse response of
 * template t over m in [0, n) (the closed form of the SPIIR response, Section
 * II.B.1), target g_t[m] is given, and
 *   c = sum_m conj(g[m]) u[m],  O = |c| / (||u|| ||g||)      (mode 0)
 *                               O = Re(c) / (||u|| ||g||)    (mode 1)
 * The loss is L = scale * sum_t (1 - O_t).  With
 *   ubar[m] = dL/dRe u[m] + i dL/dIm u[m]
 * and u holomorphic in a_k, b_k:
 *   grad_b_k = sum_m ubar[m] conj(a_k^(m-d_k))
 *   grad_a_k = sum_m ubar[m] conj(b_k (m-d_k) a_k^(m-d_k-1))
 * Outputs: overlap[T] (O_t), grad_a, grad_b complex128 [F].  Powers are formed
 * by repeated multiplication in double precision.
 */
int spo_overlap_grad(int32_t n_templates, const int32_t *offsets, const double *a,
                     const double *b, const int32_t *d, int64_t n, const double *target,
                     int32_t mode, double scale, double *overlap, double *grad_a,
                     double *grad_b)
{
    if (n_templates < 0 || n < 0 || (mode != 0 && mode != 1))
        return SPO_EINVAL;
    int status = SPO_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t t = 0; t < n_templates; ++t) {
        double *u = (double *)calloc(2 * (size_t)(n > 0 ? n : 1), sizeof(double));
        double *ub = (double *)calloc(2 * (size_t)(n > 0 ? n : 1), sizeof(double));
        if (u == NULL || ub == NULL) {
            free(u);
            free(ub);
#pragma omp atomic write
            status = SPO_EINVAL;
            continue;
        }
        const double *g = target + 2 * (int64_t)t * n;
        /* impulse response: closed form sum of b a^(m-d) */
        for (int64_t k = offsets[t]; k < offsets[t + 1]; ++k) {
            const double ar = a[2 * k], ai = a[2 * k + 1];
            double pr = b[2 * k], pi = b[2 * k + 1]; /* b a^0 */
            for (int64_t m = d[k]; m < n; ++m) {
                u[2 * m] += pr;
                u[2 * m + 1] += pi;
                const double qr = pr * ar - pi * ai;
                const double qi = pr * ai + pi * ar;
                pr = qr;
                pi = qi;
            }
        }
        double cr = 0.0, ci = 0.0, uu = 0.0, gg = 0.0;
        for (int64_t m = 0; m < n; ++m) {
            const double gr = g[2 * m], gi = g[2 * m + 1];
            const double ur = u[2 * m], ui = u[2 * m + 1];
            cr += gr * ur + gi * ui;   /* conj(g) u */
            ci += gr * ui - gi * ur;
            uu += ur * ur + ui * ui;
            gg += gr * gr + gi * gi;
        }
        const double nu = sqrt(uu), ng = sqrt(gg), ac = hypot(cr, ci);
        double o;
        /* 2 dO/dconj(u[m]) = alpha * g[m] - beta * u[m] */
        double alr, ali, beta;
        if (mode == 0) {
            o = ac / (nu * ng);
            alr = cr / (ac * nu * ng);
            ali = ci / (ac * nu * ng);
            beta = ac / (uu * nu * ng);
        } else {
            o = cr / (nu * ng);
            alr = 1.0 / (nu * ng);
            ali = 0.0;
            beta = cr / (uu * nu * ng);
        }
        overlap[t] = o;
        for (int64_t m = 0; m < n; ++m) {
            const double gr = g[2 * m], gi = g[2 * m + 1];
            /* ubar = -scale * (alpha g - beta u) */
            ub[2 * m] = -scale * ((alr * gr - ali * gi) - beta * u[2 * m]);
            ub[2 * m + 1] = -scale * ((alr * gi + ali * gr) - beta * u[2 * m + 1]);
        }
        for (int64_t k = offsets[t]; k < offsets[t + 1]; ++k) {
            const double ar = a[2 * k], ai = a[2 * k + 1];
            const double br = b[2 * k], bi = b[2 * k + 1];
            double gbr = 0.0, gbi = 0.0, gar = 0.0, gai = 0.0;
            double pr = 1.0, pi = 0.0;   /* a^(m-d) */
            double qr = 0.0, qi = 0.0;   /* (m-d) a^(m-d-1) */
            for (int64_t m = d[k]; m < n; ++m) {
                const double vr = ub[2 * m], vi = ub[2 * m + 1];
                /* ubar * conj(p) */
                gbr += vr * pr + vi * pi;
                gbi += vi * pr - vr * pi;
                /* ubar * conj(b q) */
                const double sr = br * qr - bi * qi, si = br * qi + bi * qr;
                gar += vr * sr + vi * si;
                gai += vi * sr - vr * si;
                /* next: q' = (j+1) a^j = a q + p, p' = a p  (j = m - d) */
                const double nqr = ar * qr - ai * qi + pr;
                const double nqi = ar * qi + ai * qr + pi;
                const double npr = ar * pr - ai * pi;
                const double npi = ar * pi + ai * pr;
                qr = nqr; qi = nqi; pr = npr; pi = npi;
            }
            grad_a[2 * k] = gar;
            grad_a[2 * k + 1] = gai;
            grad_b[2 * k] = gbr;
            grad_b[2 * k + 1] = gbi;
        }
        free(u);
        free(ub);
    }
    return status;
}

/* ------------------------------------------------------------------------ */
/* Noise power and trigger selection (Section II.C.1).                       */
/* ------------------------------------------------------------------------ */

/*
 * E|z_t[n]|^2 for stationary white input of unit variance: with
 * z_t[n] = sum_k sum_m b_k a_k^m x[n-d_k-m],
 *   E|z_t|^2 = sum_{k,l} b_k conj(b_l) sum_{m,m' : d_k+m = d_l+m'} a_k^m conj(a_l)^{m'}
 *            = sum_{k,l} b_k conj(b_l) conj(a_l)^(d_k-d_l) / (1 - a_k conj(a_l))   (d_k >= d_l)
 * and the conjugate of the (l,k) term when d_k < d_l.  power[T] (real).
 */
int spo_noise_power(int32_t n_templates, const int32_t *offsets, const double *a, const double *b,
                    const int32_t *d, double *power)
{
    if (n_templates < 0)
        return SPO_EINVAL;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t t = 0; t < n_templates; ++t) {
        double acc = 0.0;
        for (int64_t k = offsets[t]; k < offsets[t + 1]; ++k) {
            for (int64_t l = offsets[t]; l < offsets[t + 1]; ++l) {
                /* term(k,l) = b_k conj(b_l) conj(a_l)^(d_k-d_l) / (1 - a_k conj(a_l)) for d_k >= d_l;
                   only the real part of the double sum survives (it is Hermitian) */
                int64_t p = k, q = l;
                if (d[k] < d[l]) { p = l; q = k; }   /* conj(term(l,k)) has the same real part */
                const double apr = a[2 * p], api = a[2 * p + 1];
                const double aqr = a[2 * q], aqi = -a[2 * q + 1];          /* conj(a_q) */
                /* num = b_p conj(b_q) conj(a_q)^(d_p - d_q), the power by repeated squaring */
                double nr = b[2 * p] * b[2 * q] + b[2 * p + 1] * b[2 * q + 1];
                double ni = b[2 * p + 1] * b[2 * q] - b[2 * p] * b[2 * q + 1];
                double sr = aqr, si = aqi;
                for (int32_t e = d[p] - d[q]; e > 0; e >>= 1) {
                    if (e & 1) {
                        const double tr = nr * sr - ni * si;
                        const double ti = nr * si + ni * sr;
                        nr = tr;
                        ni = ti;
                    }
                    const double qr = sr * sr - si * si;
                    const double qi = 2.0 * sr * si;
                    sr = qr;
                    si = qi;
                }
                /* den = 1 - a_p conj(a_q) */
                const double dr = 1.0 - (apr * aqr - api * aqi);
                const double di = -(apr * aqi + api * aqr);
                const double den2 = dr * dr + di * di;
                acc += (nr * dr + ni * di) / den2;   /* Re(num / den) */
            }
        }
        power[t] = acc;
    }
    return SPO_OK;
}

/* ------------------------------------------------------------------------ */
/* Signal-consistency statistic (Section II.C.1): the correlation function   */
/* of a template with itself.                                                */
/* ------------------------------------------------------------------------ */

/* (re, im) of p^e for integer e >= 0, by repeated squaring. */
static void cpow_int(double pr, double pi, int64_t e, double *rr, double *ri)
{
    double ar = 1.0, ai = 0.0, sr = pr, si = pi;
    for (; e > 0; e >>= 1) {
        if (e & 1) {
            const double tr = ar * sr - ai * si;
            ai = ar * si + ai * sr;
            ar = tr;
        }
        const double qr = sr * sr - si * si;
        si = 2.0 * sr * si;
        sr = qr;
    }
    *rr = ar;
    *ri = ai;
}

/*
 * R_t[j] = sum_m u_t[m+j] conj(u_t[m]) for j = 0..nj, where u_t is the template's
 * response to a unit impulse, u_t[m] = sum_k b_k a_k^(m-d_k) [m >= d_k].  The sum
 * over m is geometric for every pair of filters (k, l):
 *   sum over m >= max(d_l, d_k - j) of a_k^(m+j-d_k) conj(a_l)^(m-d_l)
 *     = a_k^(d_l+j-d_k) / (1 - a_k conj(a_l))          if d_l + j >= d_k,
 *     = conj(a_l)^(d_k-j-d_l) / (1 - a_k conj(a_l))    otherwise,
 * times b_k conj(b_l).  R_t[-j] = conj(R_t[j]); R_t[0] = E|z_t|^2 for unit white input.
 * R: [T][nj+1] complex.
 */
int spo_autocorr(int32_t n_templates, const int32_t *offsets, const double *a, const double *b,
                 const int32_t *d, int32_t nj, double *R)
{
    if (n_templates < 0 || nj < 0)
        return SPO_EINVAL;
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int32_t t = 0; t < n_templates; ++t) {
        for (int32_t j = 0; j <= nj; ++j) {
            double accr = 0.0, acci = 0.0;
            for (int64_t k = offsets[t]; k < offsets[t + 1]; ++k) {
                const double akr = a[2 * k], aki = a[2 * k + 1];
                for (int64_t l = offsets[t]; l < offsets[t + 1]; ++l) {
                    const double alr = a[2 * l], ali = -a[2 * l + 1];      /* conj(a_l) */
                    double pr, pi;
                    const int64_t e = (int64_t)d[l] + j - d[k];
                    if (e >= 0)
                        cpow_int(akr, aki, e, &pr, &pi);
                    else
                        cpow_int(alr, ali, -e, &pr, &pi);
                    /* num = b_k conj(b_l) * power */
                    const double gr = b[2 * k] * b[2 * l] + b[2 * k + 1] * b[2 * l + 1];
                    const double gi = b[2 * k + 1] * b[2 * l] - b[2 * k] * b[2 * l + 1];
                    const double nr = gr * pr - gi * pi;
                    const double ni = gr * pi + gi * pr;
                    /* den = 1 - a_k conj(a_l) */
                    const double dr = 1.0 - (akr * alr - aki * ali);
                    const double di = -(akr * ali + aki * alr);
                    const double den2 = dr * dr + di * di;
                    accr += (nr * dr + ni * di) / den2;
                    acci += (ni * dr - nr * di) / den2;
                }
            }
            R[2 * ((int64_t)t * (nj + 1) + j)] = accr;
            R[2 * ((int64_t)t * (nj + 1) + j) + 1] = acci;
        }
    }
    return SPO_OK;
}
