/*
 * stt_oracle_ext.c -- oracle for the additions around the template search:
 * top-K selection, the bilinear smooth SNR and its gradient with respect to a
 * template's control points, and the gradient-ascent refinement of a template.
 *
 * TEST INFRASTRUCTURE ONLY (same rules as stt_oracle.c): plain single-threaded
 * FP64 C, no code shared with the HIP library.
 *
 * None of this is in the paper except as motivation: the paper follows up its
 * loudest candidates with a deeper search (Sec. V) and keeps the maximum
 * statistic per spectrogram. The definitions below are the readings this
 * project takes; each function states it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Top-K: the K best of n scores ordered by score descending, then index     */
/* ascending; NaN ranks as -infinity (never above a number). Writes K        */
/* indices (K <= n). Plain definition: sort everything, keep the first K.    */
/* ------------------------------------------------------------------------ */
static const double *g_z; /* qsort has no context argument */

static double rank_value(double v) { return isnan(v) ? -INFINITY : v; }

static int cmp_desc(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    double x = rank_value(g_z[i]), y = rank_value(g_z[j]);
    if (x > y) return -1;
    if (x < y) return 1;
    return (i > j) - (i < j);
}

int orc_topk(const double *z, int64_t n, int32_t K, int64_t *idx)
{
    if (K < 0 || K > n) return -1;
    int64_t *all = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) all[i] = i;
    g_z = z;
    qsort(all, (size_t)n, sizeof(int64_t), cmp_desc);
    memcpy(idx, all, sizeof(int64_t) * (size_t)K);
    free(all);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Bilinear smooth SNR of a template (reading; the paper scores only pixel   */
/* sets). Parameters theta = (tau0, tau2, phi0, phi1, phi2, dtau_ms): start  */
/* and end time in columns, three control frequencies in rows (continuous),  */
/* delay in milliseconds. With K samples xi_k = k/(K-1):                     */
/*   t_k = tau0 + xi_k (tau2 - tau0)          (Eq. 6 with t_mid midway)      */
/*   f_k = (1-xi)^2 phi0 + 2 xi (1-xi) phi1 + xi^2 phi2                      */
/*   u_k = clamp(t_k, 0, T-1),  v_k = clamp(f_k - 1/2, 0, F-1)               */
/* (row r's centre sits at r + 1/2, where a rasterised template puts it), and */
/*   z~ = (1/sqrt K) sum_k  bilinear(G)(u_k, v_k),                           */
/*   G(t, r) = Re[exp(2 pi i f(r) dtau) Y(t,r) / sigma(t,r)]   (Eq. 8 term). */
/* The cell of (u, v) is i = min(floor u, T-2), r = min(floor v, F-2) with    */
/* fractions a = u - i, b = v - r in [0, 1]. The gradient is the exact        */
/* derivative of this piecewise-bilinear function where it is differentiable; */
/* a coordinate clamped at a boundary contributes zero.                      */
/* Map: Y interleaved (re, im) doubles, sigma doubles, element (t,r) at      */
/* t*ld + r; requires T >= 2 and F >= 2.                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    const double *Y;
    const double *sigma;
    int32_t T, F;
    int64_t ld;
    int32_t fq4_lo, dfq4;
} orc_map2;

/* G and dG/d(dtau seconds) at a grid node */
static void node(const orc_map2 *m, int64_t t, int64_t r, double dtau_s, double *g, double *gd)
{
    int64_t e = t * m->ld + r;
    double sg = m->sigma[e];
    double pr = m->Y[2 * e] / sg, pim = m->Y[2 * e + 1] / sg;
    double f = (m->fq4_lo + (double)r * m->dfq4) / 16.0;
    double ph = 2.0 * M_PI * f * dtau_s;
    double c = cos(ph), s = sin(ph);
    *g = c * pr - s * pim;                  /* Re[e^{i ph} p] */
    *gd = -2.0 * M_PI * f * (s * pr + c * pim); /* d/d dtau of it: Re[i 2 pi f e^{i ph} p] */
}

double orc_smooth(const orc_map2 *m, const double *theta, int32_t K, double *grad)
{
    const double tau0 = theta[0], tau2 = theta[1];
    const double dtau_s = theta[5] * 1e-3;
    double z = 0.0, gr[6] = {0, 0, 0, 0, 0, 0};
    for (int32_t k = 0; k < K; ++k) {
        const double xi = K > 1 ? (double)k / (double)(K - 1) : 0.0;
        const double b0 = (1 - xi) * (1 - xi), b1 = 2 * xi * (1 - xi), b2 = xi * xi;
        const double t = tau0 + xi * (tau2 - tau0);
        const double f = b0 * theta[2] + b1 * theta[3] + b2 * theta[4];
        double u = t, v = f - 0.5;
        int ut = 1, vt = 1; /* 0 when the coordinate is clamped */
        if (u < 0) { u = 0; ut = 0; }
        if (u > m->T - 1) { u = m->T - 1; ut = 0; }
        if (v < 0) { v = 0; vt = 0; }
        if (v > m->F - 1) { v = m->F - 1; vt = 0; }
        int64_t i = (int64_t)floor(u), r = (int64_t)floor(v);
        if (i > m->T - 2) i = m->T - 2;
        if (r > m->F - 2) r = m->F - 2;
        const double a = u - (double)i, b = v - (double)r;
        double g00, g10, g01, g11, d00, d10, d01, d11;
        node(m, i, r, dtau_s, &g00, &d00);
        node(m, i + 1, r, dtau_s, &g10, &d10);
        node(m, i, r + 1, dtau_s, &g01, &d01);
        node(m, i + 1, r + 1, dtau_s, &g11, &d11);
        z += (1 - a) * (1 - b) * g00 + a * (1 - b) * g10 + (1 - a) * b * g01 + a * b * g11;
        const double du = ut ? (1 - b) * (g10 - g00) + b * (g11 - g01) : 0.0;
        const double dv = vt ? (1 - a) * (g01 - g00) + a * (g11 - g10) : 0.0;
        gr[0] += (1 - xi) * du;
        gr[1] += xi * du;
        gr[2] += b0 * dv;
        gr[3] += b1 * dv;
        gr[4] += b2 * dv;
        gr[5] += ((1 - a) * (1 - b) * d00 + a * (1 - b) * d10 + (1 - a) * b * d01 + a * b * d11) * 1e-3;
    }
    const double s = 1.0 / sqrt((double)K);
    if (grad)
        for (int q = 0; q < 6; ++q) grad[q] = gr[q] * s;
    return z * s;
}

/* ------------------------------------------------------------------------ */
/* Refinement by projected gradient ascent (reading; a follow-up step in the */
/* spirit of the paper's deeper search of its loudest candidates, Sec. V).   */
/* For s = 0 .. steps-1 with fraction w = s/(steps-1):                       */
/*   eta_px = px0 + w (px1 - px0),  eta_ms = ms0 + w (ms1 - ms0)             */
/*   g = grad z~(theta); the five position parameters move by eta_px along   */
/*   g_pos/|g_pos|, the delay by eta_ms along sign(g_dtau);                  */
/*   then theta is projected: tau in [0, T-1] with tau2 - tau0 >= L-1 (both   */
/*   moved apart about their midpoint, then shifted inside), phi in          */
/*   [0, F - 2^-9], |dtau_ms| <= dtau_max_ms.                                */
/* The best (largest z~) of the starting point and every iterate is kept:    */
/* theta is overwritten with it and its z~ returned.                         */
/* ------------------------------------------------------------------------ */
static void project(double *th, int32_t T, int32_t F, int32_t L, double dmax_ms)
{
    double a = th[0], b = th[1];
    if (b - a < L - 1) {
        const double mid = 0.5 * (a + b);
        a = mid - 0.5 * (L - 1);
        b = mid + 0.5 * (L - 1);
    }
    if (a < 0) { b -= a; a = 0; }
    if (b > T - 1) { a -= b - (T - 1); b = T - 1; }
    if (a < 0) a = 0;
    th[0] = a;
    th[1] = b;
    const double fmax = (double)F - 1.0 / 512.0;
    for (int q = 2; q < 5; ++q) {
        if (th[q] < 0) th[q] = 0;
        if (th[q] > fmax) th[q] = fmax;
    }
    if (th[5] > dmax_ms) th[5] = dmax_ms;
    if (th[5] < -dmax_ms) th[5] = -dmax_ms;
}

/* The same ascent with every iterate recorded: trace (may be NULL) receives
 * (steps + 1) rows of 7 doubles, row s = (theta_s[0..5], z~(theta_s)) where
 * theta_0 is the projected start and theta_{s+1} follows ascent step s. */
double orc_refine_trace(const orc_map2 *m, double *theta, int32_t K, int32_t steps, int32_t L, double dmax_ms,
                        const double *sched /* px0, px1, ms0, ms1 */, double *trace)
{
    double th[6], best[6], g[6];
    memcpy(th, theta, sizeof th);
    project(th, m->T, m->F, L, dmax_ms);
    memcpy(best, th, sizeof th);
    double zbest = orc_smooth(m, th, K, g);
    if (trace) {
        memcpy(trace, th, sizeof th);
        trace[6] = zbest;
    }
    for (int32_t s = 0; s < steps; ++s) {
        const double w = steps > 1 ? (double)s / (double)(steps - 1) : 0.0;
        const double epx = sched[0] + w * (sched[1] - sched[0]);
        const double ems = sched[2] + w * (sched[3] - sched[2]);
        double n2 = 0;
        for (int q = 0; q < 5; ++q) n2 += g[q] * g[q];
        if (n2 > 0) {
            const double inv = 1.0 / sqrt(n2);
            for (int q = 0; q < 5; ++q) th[q] += epx * g[q] * inv;
        }
        if (g[5] > 0) th[5] += ems;
        else if (g[5] < 0) th[5] -= ems;
        project(th, m->T, m->F, L, dmax_ms);
        const double z = orc_smooth(m, th, K, g);
        if (trace) {
            memcpy(trace + 7 * (s + 1), th, sizeof th);
            trace[7 * (s + 1) + 6] = z;
        }
        if (z > zbest) {
            zbest = z;
            memcpy(best, th, sizeof th);
        }
    }
    memcpy(theta, best, sizeof best);
    return zbest;
}

double orc_refine(const orc_map2 *m, double *theta, int32_t K, int32_t steps, int32_t L, double dmax_ms,
                  const double *sched /* px0, px1, ms0, ms1 */)
{
    return orc_refine_trace(m, theta, K, steps, L, dmax_ms, sched, NULL);
}

/* ------------------------------------------------------------------------ */
/* Back to a plain template: times rounded half up (then widened to L        */
/* pixels inside the map if rounding shortened it), control frequencies     */
/* floor(phi * 256) kept inside the band, delay rounded to the nearest       */
/* 2^-28 s and clipped to +-dtau_max units.                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t t0, t2;
    uint32_t f0, f1, f2;
    int32_t dtau;
} orc_track2;

void orc_theta_to_track(const double *th, int32_t T, int32_t F, int32_t L, int32_t dtau_max, orc_track2 *out)
{
    int32_t t0 = (int32_t)floor(th[0] + 0.5), t2 = (int32_t)floor(th[1] + 0.5);
    if (t0 < 0) t0 = 0;
    if (t2 > T - 1) t2 = T - 1;
    if (t2 - t0 < L - 1) {
        t2 = t0 + L - 1;
        if (t2 > T - 1) { t0 -= t2 - (T - 1); t2 = T - 1; }
    }
    out->t0 = t0;
    out->t2 = t2;
    uint32_t *f[3] = {&out->f0, &out->f1, &out->f2};
    for (int q = 0; q < 3; ++q) {
        double v = floor(th[2 + q] * 256.0);
        if (v < 0) v = 0;
        if (v > (double)F * 256 - 1) v = (double)F * 256 - 1;
        *f[q] = (uint32_t)v;
    }
    double d = floor(th[5] * 1e-3 * 268435456.0 + 0.5);
    if (d > dtau_max) d = dtau_max;
    if (d < -dtau_max) d = -dtau_max;
    out->dtau = (int32_t)d;
}
