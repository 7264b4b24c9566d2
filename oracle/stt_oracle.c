/*
 * stt_oracle.c -- CPU reference ("oracle") for the all-sky seedless-clustering
 * track search of Thrane & Coughlin, "Seedless clustering in all-sky searches
 * for gravitational-wave transients" (arXiv:1401.8060).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this file:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
 * It shares no code, header, table or helper with the HIP library; both sides
 * read the same input bytes and nothing else.
 *
 * Plain, slow, single-threaded, FP64.  Each function states the passage of the
 * paper it writes out, or the reading taken where the paper is silent.
 *
 * Fixed-point conventions (readings; the paper fixes none of them):
 *   - time column t in [0, T), frequency row r in [0, F); pixel (t, r) of a
 *     map sits at element t*ld + r (time-major, frequency contiguous);
 *   - row r has frequency (fq4_lo + r*dfq4) / 16 Hz;
 *   - a template's control frequencies f0, f1, f2 are in units of 1/256 row;
 *   - its time delay dtau is in units of 2^-28 s, so the phase f*dtau is an
 *     exact integer count of 2^-32 turns.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_FBITS 8 /* control frequencies carry 8 fractional bits */

typedef struct {
    int32_t t0, t2;       /* first and last time column, t0 < t2 */
    uint32_t f0, f1, f2;  /* control frequencies, 1/256-row units */
    int32_t dtau;         /* time delay, units of 2^-28 s */
} orc_track;

/* ------------------------------------------------------------------------ */
/* Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel     */
/* random numbers: as easy as 1, 2, 3", SC'11).  The paper draws each       */
/* template from six random numbers plus a random delay (Sec. III, around   */
/* Eq. 6 and before Eq. 8); a counter-based generator makes track j a pure  */
/* function of (seed, stream, j), so runs with different seeds or disjoint  */
/* index ranges combine by a max exactly as the paper's Sec. V recommends.  */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { /* the key is bumped by the Weyl constants between rounds */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Template draw.  Reading of Sec. III (templates persist at least t_min;   */
/* Eq. 6 with three control points; a delay uniform in +-dtau_max before    */
/* Eq. 8): the time extent (t_start, t_end) is uniform over all pairs with  */
/* at least L pixels, t_mid is the midpoint so time is linear in xi, the    */
/* three control frequencies are uniform on [0, F), and the delay is        */
/* uniform on the integers [-D, D] (D = dtau_max in 2^-28 s units).         */
/* ------------------------------------------------------------------------ */

/* number of (t_start, t_end) pairs with t_end - t_start + 1 >= L */
int64_t orc_npairs(int32_t T, int32_t L)
{
    if (L < 2 || T < L) return 0;
    int64_t npos = (int64_t)T - L + 1;
    return npos * (npos + 1) / 2;
}

static uint64_t isqrt_u64(uint64_t x)
{
    /* largest s with s*s <= x, by bisection */
    uint64_t lo = 0, hi = 4294967296ull; /* hi*hi > any x < 2^64 */
    while (hi - lo > 1) {
        uint64_t mid = lo + (hi - lo) / 2;
        if ((unsigned __int128)mid * mid <= x) lo = mid; else hi = mid;
    }
    return lo;
}

/* pair number k in [0, P) -> (t_start, t_end); pairs ordered by t_end, then t_start */
void orc_unrank(uint64_t k, int32_t L, int32_t *t0, int32_t *t2)
{
    uint64_t s = isqrt_u64(8 * k + 1);
    uint64_t e = (s - 1) / 2;            /* e*(e+1)/2 <= k < (e+1)*(e+2)/2 */
    uint64_t a = k - e * (e + 1) / 2;    /* 0 <= a <= e */
    *t0 = (int32_t)a;
    *t2 = (int32_t)(e + (uint64_t)L - 1);
}

/* floor(u * m / 2^64) for a 64-bit uniform u and a multiplier m */
static uint64_t scale_u64(uint64_t u, uint64_t m)
{
    return (uint64_t)(((unsigned __int128)u * m) >> 64);
}

int orc_draw(uint64_t seed, uint32_t stream, uint64_t j, int32_t T, int32_t F, int32_t L,
             int32_t D, orc_track *tr)
{
    int64_t P = orc_npairs(T, L);
    if (P <= 0 || F < 1 || D < 0) return -1;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x0[4], x1[4];
    uint32_t c0[4] = {(uint32_t)j, (uint32_t)(j >> 32), stream, 0u};
    uint32_t c1[4] = {(uint32_t)j, (uint32_t)(j >> 32), stream, 1u};
    orc_philox4x32_10(c0, key, x0);
    orc_philox4x32_10(c1, key, x1);
    uint64_t u = ((uint64_t)x0[0] << 32) | x0[1];
    orc_unrank(scale_u64(u, (uint64_t)P), L, &tr->t0, &tr->t2);
    uint64_t frange = (uint64_t)F << ORC_FBITS;
    tr->f0 = (uint32_t)(((uint64_t)x0[2] * frange) >> 32);
    tr->f1 = (uint32_t)(((uint64_t)x0[3] * frange) >> 32);
    tr->f2 = (uint32_t)(((uint64_t)x1[0] * frange) >> 32);
    uint64_t u2 = ((uint64_t)x1[1] << 32) | x1[2];
    tr->dtau = (int32_t)(-(int64_t)D + (int64_t)scale_u64(u2, 2 * (uint64_t)D + 1));
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Rasterisation of Eq. 6.  With t_mid at the midpoint, column t0+k sits at */
/* xi = k/(t2-t0); the template occupies one pixel per column, the row      */
/* being the floor of the curve's frequency there, computed exactly:        */
/*   row = floor( ((1-xi)^2 f0 + 2(1-xi) xi f1 + xi^2 f2) / 256 )           */
/* with xi = k/Dt, i.e. numerator and denominator multiplied by Dt^2.       */
/* Writes N = t2-t0+1 rows; returns N or -1.                                */
/* ------------------------------------------------------------------------ */
int orc_rows(const orc_track *tr, int32_t F, int32_t *rows)
{
    int64_t Dt = (int64_t)tr->t2 - tr->t0;
    if (Dt < 1) return -1;
    uint64_t lim = (uint64_t)F << ORC_FBITS;
    if (tr->f0 >= lim || tr->f1 >= lim || tr->f2 >= lim) return -1;
    uint64_t den = (uint64_t)(Dt * Dt) << ORC_FBITS;
    for (int64_t k = 0; k <= Dt; ++k) {
        uint64_t a = (uint64_t)(Dt - k), b = (uint64_t)k;
        uint64_t num = a * a * tr->f0 + 2 * a * b * tr->f1 + b * b * tr->f2;
        rows[k] = (int32_t)(num / den);
    }
    return (int)(Dt + 1);
}

/* ------------------------------------------------------------------------ */
/* Phase factor of Eq. 8: exp(2 pi i f dtau) at the row's frequency f.      */
/* f dtau = (fq4/16 Hz)(dtau 2^-28 s) = fq4*dtau * 2^-32 turns; only the    */
/* fractional part matters, so the phase is the product's low 32 bits, read */
/* as a signed count of 2^-32 turns in [-1/2, 1/2).                         */
/* ------------------------------------------------------------------------ */
double orc_phase_turns(int64_t fq4, int32_t dtau)
{
    uint32_t w = (uint32_t)((uint64_t)(fq4 * (int64_t)dtau));
    return (double)(int32_t)w / 4294967296.0;
}

/* ------------------------------------------------------------------------ */
/* The statistic, Eq. 8: SNR_tot = (1/N) sum over the template's pixels of  */
/* Re[exp(2 pi i f dtau) p(t;f)], with the complex SNR p = Y/sigma (the     */
/* appendix's rho = Y/sigma with Y kept complex, Eq. 7).  norm = 1 gives    */
/* the paper's 1/N; norm = 0 gives 1/sqrt(N), which makes the noise-only    */
/* statistic standard normal (the reading used for the search default).    */
/* The sum is compensated (Neumaier) so that it is exact to FP64 rounding.  */
/* Y is interleaved (re, im) doubles; map element (t, r) at t*ld + r.       */
/* ------------------------------------------------------------------------ */
typedef struct {
    const double *Y;     /* [T][ld][2] */
    const double *sigma; /* [T][ld]    */
    int32_t T, F;
    int64_t ld;
    int32_t fq4_lo, dfq4;
} orc_map;

static int check_track(const orc_map *m, const orc_track *tr)
{
    if (tr->t0 < 0 || tr->t2 >= m->T || tr->t2 <= tr->t0) return -1;
    uint64_t lim = (uint64_t)m->F << ORC_FBITS;
    if (tr->f0 >= lim || tr->f1 >= lim || tr->f2 >= lim) return -1;
    return 0;
}

double orc_score(const orc_map *m, const orc_track *tr, int32_t norm)
{
    if (check_track(m, tr) != 0) return NAN;
    int32_t N = tr->t2 - tr->t0 + 1;
    int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    orc_rows(tr, m->F, rows);
    double s = 0.0, c = 0.0;
    for (int32_t k = 0; k < N; ++k) {
        int64_t t = tr->t0 + k, r = rows[k];
        int64_t e = t * m->ld + r;
        double sg = m->sigma[e];
        double p_re = m->Y[2 * e] / sg, p_im = m->Y[2 * e + 1] / sg;
        double turns = orc_phase_turns((int64_t)m->fq4_lo + r * m->dfq4, tr->dtau);
        double phi = 2.0 * M_PI * turns;
        double term = cos(phi) * p_re - sin(phi) * p_im; /* Re[e^{i phi} p] */
        double nt = s + term;
        if (fabs(s) >= fabs(term)) c += (s - nt) + term; else c += (term - nt) + s;
        s = nt;
    }
    free(rows);
    double S = s + c;
    return norm == 1 ? S / (double)N : S / sqrt((double)N);
}

/* score tracks j = first .. first+n-1 drawn by orc_draw */
int orc_score_gen(const orc_map *m, uint64_t seed, uint32_t stream, int32_t L, int32_t D,
                  uint64_t first, int64_t n, int32_t norm, double *z)
{
    for (int64_t i = 0; i < n; ++i) {
        orc_track tr;
        if (orc_draw(seed, stream, first + (uint64_t)i, m->T, m->F, L, D, &tr) != 0) return -1;
        z[i] = orc_score(m, &tr, norm);
    }
    return 0;
}

/* score tracks j = idx[i] drawn by orc_draw (a sample of a larger run) */
int orc_score_gen_idx(const orc_map *m, uint64_t seed, uint32_t stream, int32_t L, int32_t D,
                      const uint64_t *idx, int64_t n, int32_t norm, double *z)
{
    for (int64_t i = 0; i < n; ++i) {
        orc_track tr;
        if (orc_draw(seed, stream, idx[i], m->T, m->F, L, D, &tr) != 0) return -1;
        z[i] = orc_score(m, &tr, norm);
    }
    return 0;
}

int orc_score_list(const orc_map *m, const orc_track *tr, int64_t n, int32_t norm, double *z)
{
    for (int64_t i = 0; i < n; ++i) z[i] = orc_score(m, &tr[i], norm);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Templates with a free t_mid (Eq. 6 with all six random numbers). The     */
/* time coordinate is itself a quadratic Bezier, t(xi) = (1-xi)^2 t0 +      */
/* 2 xi (1-xi) t1 + xi^2 t2 with an integer t1 in [t0, t2] (so t(xi) is     */
/* monotone); drawn from the last unused word of the template's second      */
/* Philox block: t1 = t0 + floor(x * (t2 - t0 + 1) / 2^32). The template    */
/* still takes one pixel per column: at column t, xi(t) is the root in      */
/* [0, 1] of a xi^2 + b xi + c = 0 with a = t0 - 2 t1 + t2, b = 2 (t1 - t0),  */
/* c = t0 - t, and the row is floor(f(xi)/256) with f the frequency Bezier  */
/* (1/256-row units). For a = 0 (t1 at the midpoint) this is the rasteriser */
/* above. For a != 0, eliminating xi^2 with the quadratic gives             */
/*   f(xi) / 256 = (U + V sqrt(D)) / W,  D = b^2 - 4 a c,                    */
/*   V = a B - C b,  U = 2 a (a f0 - C c) - b V,  W = 512 a^2,               */
/* B = 2 (f1 - f0), C = f0 - 2 f1 + f2 -- all integers -- and the floor is    */
/* decided exactly in 128-bit integers: r <= (U + V sqrt D)/W  iff           */
/* V sqrt(D) >= r W - U, compared by signs and then squares.                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t t0, t1, t2;
    uint32_t f0, f1, f2;
    int32_t dtau;
} orc_track_tm;

int orc_draw_tm(uint64_t seed, uint32_t stream, uint64_t j, int32_t T, int32_t F, int32_t L, int32_t D,
                orc_track_tm *tr)
{
    orc_track b;
    if (orc_draw(seed, stream, j, T, F, L, D, &b) != 0) return -1;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t c1[4] = {(uint32_t)j, (uint32_t)(j >> 32), stream, 1u}, x1[4];
    orc_philox4x32_10(c1, key, x1);
    tr->t0 = b.t0;
    tr->t2 = b.t2;
    tr->t1 = b.t0 + (int32_t)(((uint64_t)x1[3] * (uint64_t)(b.t2 - b.t0 + 1)) >> 32);
    tr->f0 = b.f0;
    tr->f1 = b.f1;
    tr->f2 = b.f2;
    tr->dtau = b.dtau;
    return 0;
}

/* sign of V sqrt(D) - X (D >= 0), exactly */
static int cmp_vsqrtd(int64_t V, int64_t D, int64_t X)
{
    if (D == 0 || V == 0) return (X < 0) - (X > 0);
    if (V > 0 && X <= 0) return 1;
    if (V < 0 && X >= 0) return -1;
    unsigned __int128 av = (unsigned __int128)(V > 0 ? V : -V), ax = (unsigned __int128)(X > 0 ? X : -X);
    unsigned __int128 l = av * av * (unsigned __int128)D, r = ax * ax;
    int c = (l > r) - (l < r); /* |V| sqrt D vs |X| */
    return V > 0 ? c : -c;
}

int orc_rows_tm(const orc_track_tm *tr, int32_t F, int32_t *rows)
{
    int64_t Dt = (int64_t)tr->t2 - tr->t0;
    if (Dt < 1 || tr->t1 < tr->t0 || tr->t1 > tr->t2) return -1;
    uint64_t lim = (uint64_t)F << ORC_FBITS;
    if (tr->f0 >= lim || tr->f1 >= lim || tr->f2 >= lim) return -1;
    int64_t a = (int64_t)tr->t0 - 2 * (int64_t)tr->t1 + tr->t2, b = 2 * ((int64_t)tr->t1 - tr->t0);
    if (a == 0) {
        orc_track q = {tr->t0, tr->t2, tr->f0, tr->f1, tr->f2, tr->dtau};
        return orc_rows(&q, F, rows);
    }
    int64_t f0 = tr->f0, B = 2 * ((int64_t)tr->f1 - f0), C = f0 - 2 * (int64_t)tr->f1 + (int64_t)tr->f2;
    int64_t V = a * B - C * b, W = 512 * a * a;
    for (int64_t k = 0; k <= Dt; ++k) {
        int64_t c = -k; /* t0 - t */
        int64_t D = b * b - 4 * a * c, U = 2 * a * (a * f0 - C * c) - b * V;
        /* largest r in [0, F) with U + V sqrt(D) - r W >= 0; the value lies in [0, F) */
        int32_t lo = 0, hi = F - 1;
        while (lo < hi) {
            int32_t mid = lo + (hi - lo + 1) / 2;
            if (cmp_vsqrtd(V, D, (int64_t)mid * W - U) >= 0) lo = mid; else hi = mid - 1;
        }
        rows[k] = lo;
    }
    return (int)(Dt + 1);
}

/* Eq. 8 of a free-t_mid template (FP64, Neumaier), as orc_score */
double orc_score_tm(const orc_map *m, const orc_track_tm *tr, int32_t norm)
{
    if (tr->t0 < 0 || tr->t2 >= m->T || tr->t2 <= tr->t0) return NAN;
    int32_t N = tr->t2 - tr->t0 + 1;
    int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (orc_rows_tm(tr, m->F, rows) < 0) { free(rows); return NAN; }
    double s = 0.0, c = 0.0;
    for (int32_t k = 0; k < N; ++k) {
        int64_t t = tr->t0 + k, r = rows[k];
        int64_t e = t * m->ld + r;
        double sg = m->sigma[e];
        double p_re = m->Y[2 * e] / sg, p_im = m->Y[2 * e + 1] / sg;
        double phi = 2.0 * M_PI * orc_phase_turns((int64_t)m->fq4_lo + r * m->dfq4, tr->dtau);
        double term = cos(phi) * p_re - sin(phi) * p_im;
        double nt = s + term;
        if (fabs(s) >= fabs(term)) c += (s - nt) + term; else c += (term - nt) + s;
        s = nt;
    }
    free(rows);
    double S = s + c;
    return norm == 1 ? S / (double)N : S / sqrt((double)N);
}

int orc_score_tm_gen_idx(const orc_map *m, uint64_t seed, uint32_t stream, int32_t L, int32_t D,
                         const uint64_t *idx, int64_t n, int32_t norm, double *z)
{
    for (int64_t i = 0; i < n; ++i) {
        orc_track_tm tr;
        if (orc_draw_tm(seed, stream, idx[i], m->T, m->F, L, D, &tr) != 0) return -1;
        z[i] = orc_score_tm(m, &tr, norm);
    }
    return 0;
}

int orc_score_tm_list(const orc_map *m, const orc_track_tm *tr, int64_t n, int32_t norm, double *z)
{
    for (int64_t i = 0; i < n; ++i) z[i] = orc_score_tm(m, &tr[i], norm);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Delay-maximised statistic: the reading of "phase-maximised" that takes,   */
/* per template, the maximum of Eq. 8 over a grid of delays instead of one   */
/* drawn delay. The template's geometry (t0, t2, f0, f1, f2) is kept and its */
/* own delay replaced by dtau_m = d0 + m * step for m = 0 .. n_tau - 1;      */
/* z_max = max_m z(dtau_m), ties to the lowest m. An invalid template gives  */
/* NaN and m = -1. Plain definition: score each delay with orc_score.        */
/* ------------------------------------------------------------------------ */
int orc_score_maxdelay(const orc_map *m, const orc_track *tr, int32_t d0, int32_t step, int32_t n_tau,
                       int32_t norm, double *z_max, int32_t *m_max)
{
    double best = NAN;
    int32_t bm = -1;
    if (n_tau < 1) return -1;
    for (int32_t k = 0; k < n_tau; ++k) {
        int64_t d = (int64_t)d0 + (int64_t)k * step;
        if (d < -(int64_t)1073741823 || d > (int64_t)1073741823) return -1;
        orc_track t = *tr;
        t.dtau = (int32_t)d;
        double z = orc_score(m, &t, norm);
        if (isnan(z)) { best = NAN; bm = -1; break; }
        if (bm < 0 || z > best) { best = z; bm = k; }
    }
    *z_max = best;
    *m_max = bm;
    return 0;
}

int orc_score_maxdelay_gen_idx(const orc_map *m, uint64_t seed, uint32_t stream, int32_t L, int32_t D,
                               const uint64_t *idx, int64_t n, int32_t d0, int32_t step, int32_t n_tau,
                               int32_t norm, double *z, int32_t *mm)
{
    for (int64_t i = 0; i < n; ++i) {
        orc_track tr;
        if (orc_draw(seed, stream, idx[i], m->T, m->F, L, D, &tr) != 0) return -1;
        if (orc_score_maxdelay(m, &tr, d0, step, n_tau, norm, &z[i], &mm[i]) != 0) return -1;
    }
    return 0;
}

int orc_score_maxdelay_list(const orc_map *m, const orc_track *tr, int64_t n, int32_t d0, int32_t step,
                            int32_t n_tau, int32_t norm, double *z, int32_t *mm)
{
    for (int64_t i = 0; i < n; ++i)
        if (orc_score_maxdelay(m, &tr[i], d0, step, n_tau, norm, &z[i], &mm[i]) != 0) return -1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The most significant cluster (Sec. III before Eq. 5; Sec. V keeps the    */
/* maximum per spectrogram).  Reading: ties go to the lowest index and NaN  */
/* never wins.  Returns -1 when there is no finite-or-infinite candidate.   */
/* ------------------------------------------------------------------------ */
int64_t orc_argmax(const double *z, int64_t n)
{
    int64_t best = -1;
    for (int64_t i = 0; i < n; ++i) {
        if (isnan(z[i])) continue;
        if (best < 0 || z[i] > z[best]) best = i;
    }
    return best;
}
