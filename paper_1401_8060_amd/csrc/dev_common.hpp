// dev_common.hpp -- arithmetic shared by the libstt kernels (gfx950).
//
// Everything here is __host__ __device__ so that the host-side unit tests can
// exercise the exact same integer code the kernels run (generator, unranking,
// DDA rasteriser, phase) against the independent CPU reference.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stt {

#define STT_HD __host__ __device__ __forceinline__

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter-based, so track j
// is a pure function of (seed, stream, j) -- any index range can be scored on
// any device in any order and runs merge by a max (paper, Sec. V).
// ----------------------------------------------------------------------------
STT_HD uint32_t mulhi32(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }

// floor(a * b / 2^64), exact, from four 32x32 -> 64 products.
STT_HD uint64_t mulhi64(uint64_t a, uint64_t b)
{
    const uint64_t al = (uint32_t)a, ah = a >> 32, bl = (uint32_t)b, bh = b >> 32;
    const uint64_t p0 = al * bl, p1 = al * bh, p2 = ah * bl, p3 = ah * bh;
    const uint64_t mid = (p0 >> 32) + (uint32_t)p1 + (uint32_t)p2;
    return p3 + (p1 >> 32) + (p2 >> 32) + (mid >> 32);
}

struct u32x4 { uint32_t x, y, z, w; };

STT_HD u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        // each 32 x 32 -> 64-bit product in one multiply: both halves at once
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = u32x4{(uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0};
    }
    return c;
}

// A template: columns t0..t2, control frequencies in 1/256-row units, delay in
// 2^-28 s units. Same layout as stt_track in the public header.
struct Trk {
    int32_t t0, t2;
    uint32_t f0, f1, f2;
    int32_t dtau;
};

// Parameters of the random template law, precomputed on the host.
struct GenP {
    uint32_t key0, key1;  // Philox key = seed
    uint32_t stream;      // counter word 2
    uint32_t npairs;      // number of (t0, t2) pairs with >= L pixels
    int32_t L;            // minimum pixels
    uint32_t frange;      // F << 8
    int32_t dmax;         // minus the lowest delay: D - center (2^-28 s units)
    uint32_t dspan;       // 2*dmax + 1
};

// Pair number k -> (t0, t2): pairs ordered by t2 then t0, i.e. k = e(e+1)/2 + a
// with t2 = e + L - 1, t0 = a, 0 <= a <= e. The float square root is within
// one of the exact integer square root for k < 2^26; two exact integer
// comparisons fix it.
STT_HD void unrank_pair(uint32_t k, int32_t L, int32_t &t0, int32_t &t2)
{
    uint32_t e = (uint32_t)((sqrtf(8.0f * (float)k + 1.0f) - 1.0f) * 0.5f);
    if ((uint64_t)e * (e + 1) / 2 > k) --e;
    if ((uint64_t)(e + 1) * (e + 2) / 2 <= k) ++e;
    t0 = (int32_t)(k - e * (e + 1) / 2);
    t2 = (int32_t)e + L - 1;
}

STT_HD u32x4 philox_block(const GenP &g, uint64_t j, uint32_t b)
{
    return philox4x32_10(u32x4{(uint32_t)j, (uint32_t)(j >> 32), g.stream, b}, g.key0, g.key1);
}

// Time extent only (block 0): what the binning pass needs.
STT_HD void draw_extent(const GenP &g, uint64_t j, int32_t &t0, int32_t &t2)
{
    const u32x4 x = philox_block(g, j, 0);
    const uint64_t u = ((uint64_t)x.x << 32) | x.y;
    unrank_pair((uint32_t)mulhi64(u, g.npairs), g.L, t0, t2);
}

STT_HD Trk draw_track(const GenP &g, uint64_t j)
{
    const u32x4 x0 = philox_block(g, j, 0);
    const u32x4 x1 = philox_block(g, j, 1);
    Trk t;
    const uint64_t u = ((uint64_t)x0.x << 32) | x0.y;
    unrank_pair((uint32_t)mulhi64(u, g.npairs), g.L, t.t0, t.t2);
    t.f0 = mulhi32(x0.z, g.frange);
    t.f1 = mulhi32(x0.w, g.frange);
    t.f2 = mulhi32(x1.x, g.frange);
    const uint64_t u2 = ((uint64_t)x1.y << 32) | x1.z;
    t.dtau = (int32_t)((int64_t)mulhi64(u2, g.dspan) - g.dmax);
    return t;
}

// ----------------------------------------------------------------------------
// Templates with a free t_mid (Eq. 6 with its six random numbers): the time
// coordinate is a quadratic Bezier too, with an integer t1 in [t0, t2] drawn
// from the last word of the second Philox block. Other fields as draw_track.
// ----------------------------------------------------------------------------
struct TrkTm {
    int32_t t0, t1, t2;
    uint32_t f0, f1, f2;
    int32_t dtau;
};

STT_HD TrkTm draw_track_tm(const GenP &g, uint64_t j)
{
    const Trk b = draw_track(g, j);
    const u32x4 x1 = philox_block(g, j, 1);
    TrkTm t;
    t.t0 = b.t0;
    t.t2 = b.t2;
    t.t1 = b.t0 + (int32_t)mulhi32(x1.w, (uint32_t)(b.t2 - b.t0 + 1));
    t.f0 = b.f0;
    t.f1 = b.f1;
    t.f2 = b.f2;
    t.dtau = b.dtau;
    return t;
}

// Row of a free-t_mid template at column t0 + dt. With a = t0 - 2 t1 + t2,
// b = 2 (t1 - t0), the column's xi is the root in [0, 1] of
// a xi^2 + b xi - dt = 0 and the row is floor(f(xi) / 256). For a != 0,
// eliminating xi^2 gives f/256 = (U + V sqrt(D)) / W with the integers
// D = b^2 + 4 a dt, V = a B - C b, U = U0 + U1 dt (U0 = 2 a^2 f0 - b V,
// U1 = 2 a C), W = 512 a^2 (B = 2 (f1 - f0), C = f0 - 2 f1 + f2).
// FP64 evaluates xi = 2 dt / (b + sqrt(D)) (no cancellation) and
// f = f0 + xi (B + C xi), within about 2^-33 row of the truth; a value within
// 1e-6 of an integer (end columns, perfect squares) is settled exactly by the
// sign of V sqrt(D) - (r W - U), from signs and 128-bit squares. For a = 0 (t1
// at the midpoint) xi = dt / Dt and the row is the plain rasteriser's.
// Hardware square root and reciprocal, each within 1 ulp; the host build (tests) uses the
// correctly rounded operations, or moves them by one ulp when STT_HOST_ULP_PERTURB is set.
#if defined(STT_HOST_ULP_PERTURB)
float stt_host_perturb(float);
#endif
STT_HD float sqrt_1ulp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#elif defined(STT_HOST_ULP_PERTURB)
    return stt_host_perturb(std::sqrt(x));
#else
    return std::sqrt(x);
#endif
}
STT_HD float rcp_1ulp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#elif defined(STT_HOST_ULP_PERTURB)
    return stt_host_perturb(1.0f / x);
#else
    return 1.0f / x;
#endif
}

// x * y for |x|, |y| < 2^23 (one full-rate 24-bit multiply on the device)
STT_HD int32_t mul_i24(int32_t x, int32_t y)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __mul24(x, y);
#else
    return x * y;
#endif
}

// Row state of a free-t_mid template. Column t0 + dt has time parameter xi, the root in [0, 1]
// of a xi^2 + b xi = dt (a = t0 - 2 t1 + t2, b = 2 (t1 - t0) >= 0), taken in the stable form
// xi = 2 dt / (b + sqrt(D)) with D = b^2 + 4 a dt, and row floor(f(xi) / 256),
// f = f0 + B xi + C xi^2 (B = 2 (f1 - f0), C = f0 - 2 f1 + f2).
struct RowTm {
    int32_t t0, t1, t2;
    uint32_t f0, f1, f2;
    int32_t bb, a4;        // b^2 and 4 a: D = bb + a4 dt, exact in 32 bits for T <= 2896
    float bf, fs, Bs, Cs;  // b, f0/256, B/256, C/256
    float tol;             // bound on |y32 - f(xi)/256| over the template, in rows
    float hw;              // |fract(y32) - 1/2| < hw certifies tol < fract(y32) < 1 - tol
};

STT_HD RowTm row_tm_init(const TrkTm &t)
{
    RowTm k;
    k.t0 = t.t0; k.t1 = t.t1; k.t2 = t.t2;
    k.f0 = t.f0; k.f1 = t.f1; k.f2 = t.f2;
    const int32_t a = t.t0 - 2 * t.t1 + t.t2, b = 2 * (t.t1 - t.t0);
    const int64_t B = 2 * ((int64_t)t.f1 - t.f0), C = (int64_t)t.f0 - 2 * (int64_t)t.f1 + t.f2;
    k.bb = b * b;
    k.a4 = 4 * a;
    k.bf = (float)b;
    k.fs = (float)t.f0 * (1.0f / 256.0f);
    k.Bs = (float)B * (1.0f / 256.0f);
    k.Cs = (float)C * (1.0f / 256.0f);
    // Error of the FP32 pass, to first order in u = 2^-24. B/256, C/256 and f0/256 are exact
    // (|B|, |C| < 2^24 for F <= 32767). With each of sqrt and rcp within 1 ulp (2u relative),
    // (float)D, sqrt, b + s (b, sqrt(D) >= 0: no cancellation), rcp and * 2dt leave
    // xi32 = xi (1 + e), |e| <= 6.5u. Then g32 = fl(xi32 C' + B') = (g + C' xi e)(1 + e1) and
    // y32 = fl(xi32 g32 + f0') = (xi32 g32 + f0')(1 + e2) (primes: / 256, g = B' + C' xi), so
    //   y32 - y = xi e f'(xi) + xi g e1 + y e2 + O(u^2),   f'(xi) = B' + 2 C' xi.
    // f' is linear in xi, so |f'| <= max(|B'|, |B' + 2C'|) on [0, 1]; y and f0' + xi g = y lie in
    // [0, M'] (M' = max(f0, f1, f2) / 256: y is a convex combination of the control values), so
    // |xi g| <= M' and
    //   |y32 - y| <= 6.5u max(|B'|, |B' + 2C'|) + 2u M'.
    // The window is 1.25 times that, plus 2^-20 for the second-order terms.
    const double u = 1.0 / 16777216.0;
    const double d0 = std::fabs((double)B) / 256.0, d1 = std::fabs((double)(B + 2 * C)) / 256.0;
    const double M = (double)std::max(t.f0, std::max(t.f1, t.f2)) / 256.0;
    k.tol = (float)(1.25 * (6.5 * u * std::max(d0, d1) + 2.0 * u * M) + 1.0 / 1048576.0);
    // fr - 1/2 is exact for fr >= 1/4 and within 2^-26 below (its result lies in (-1/2, -1/4]),
    // so hw = 1/2 - tol - 2^-26, rounded towards zero, keeps the certified fractions inside
    // (tol, 1 - tol).
    const double hw = 0.5 - (double)k.tol - 1.0 / 67108864.0;
    k.hw = (float)hw;
    if ((double)k.hw > hw) k.hw = nextafterf(k.hw, 0.0f);
    return k;
}

// sign of V sqrt(D) - X for D >= 0, exactly
STT_HD int cmp_vsqrtd(int64_t V, int64_t D, int64_t X)
{
    if (D == 0 || V == 0) return (X < 0) - (X > 0);
    if (V > 0 && X <= 0) return 1;
    if (V < 0 && X >= 0) return -1;
    const unsigned __int128 av = (unsigned __int128)(V > 0 ? V : -V), ax = (unsigned __int128)(X > 0 ? X : -X);
    const unsigned __int128 l = av * av * (unsigned __int128)(uint64_t)D, r = ax * ax;
    const int c = (l > r) - (l < r);
    return V > 0 ? c : -c;
}

// Linear time (a = 0: an exact int64 quotient) and values within 1e-6 of a row boundary (the
// 128-bit decision): rare, so out of line.
__host__ __device__ __attribute__((noinline)) int32_t row_tm_decide(const RowTm &k, int32_t dt, int32_t D, double y)
{
    const int64_t a = (int64_t)k.t0 - 2 * (int64_t)k.t1 + k.t2, b = 2 * ((int64_t)k.t1 - k.t0);
    const int64_t f0 = k.f0, B = 2 * ((int64_t)k.f1 - f0), C = f0 - 2 * (int64_t)k.f1 + k.f2;
    if (a == 0) {  // linear time: num(dt) / Q exactly (num < 2^48)
        const int64_t Dt = (int64_t)k.t2 - k.t0;
        const int64_t num = Dt * Dt * f0 + 2 * Dt * ((int64_t)k.f1 - f0) * dt + C * (int64_t)dt * dt;
        return (int32_t)(num / ((Dt * Dt) << 8));
    }
    const int64_t V = a * B - C * b, U0 = 2 * a * a * f0 - b * V, U1 = 2 * a * C, W = 512 * a * a;
    const int64_t ri = (int64_t)floor(y + 0.5);  // the nearest integer: the floor is ri or ri - 1
    return (int32_t)(cmp_vsqrtd(V, D, ri * W - (U0 + U1 * dt)) >= 0 ? ri : ri - 1);
}

// The row where the FP32 pass is too close to a boundary to decide (or undefined: b = 0 at
// dt = 0). FP64 refines the FP32 root: sqrt(D) by one Newton step from s32 (D - s32^2 is exact
// in FP64), 1 / (b + sqrt(D)) by one Newton step from the 1-ulp reciprocal; xi's relative error
// stays below 1e-13, so |y - f/256| < 3e-8 rows for F <= 32767 and a value farther than 1e-6
// from a boundary is decided here. Within 1e-6 the floor is the nearest integer r0 or r0 - 1:
// with xi = (sqrt(D) - b)/(2a), f/256 = (V sqrt(D) + U0 + U1 dt) / W (V = aB - Cb,
// U0 = 2a^2 f0 - bV, U1 = 2aC, W = 512 a^2 > 0), and the sign of V sqrt(D) - (r0 W - U0 - U1 dt),
// taken exactly in 128-bit integers by row_tm_decide, settles it. That call (and linear time)
// stays out of line: inlined, its 128-bit temporaries would raise the scorers' register count.
STT_HD int32_t row_tm_exact(const RowTm &k, int32_t dt, int32_t D, float s32)
{
    if (k.t0 - 2 * k.t1 + k.t2 == 0) return row_tm_decide(k, dt, D, 0.0);
    if (dt == 0) return (int32_t)(k.f0 >> 8);
    const double s0 = (double)s32;
    const double s = D == 0 ? 0.0 : fma(fma(-s0, s0, (double)D), 0.5 * (double)rcp_1ulp(s32), s0);
    const double den = (double)(2 * (k.t1 - k.t0)) + s;
    const double r0 = (double)rcp_1ulp((float)den);
    const double xi = (double)(2 * dt) * fma(r0, fma(-den, r0, 1.0), r0);
    const double B = 2.0 * ((double)k.f1 - (double)k.f0), C = (double)k.f0 - 2.0 * (double)k.f1 + (double)k.f2;
    const double y = fma(xi, fma(xi, C, B), (double)k.f0) * (1.0 / 256.0);
    const double r = floor(y);
    if (y - r > 1e-6 && y - r < 1.0 - 1e-6) return (int32_t)r;
    return row_tm_decide(k, dt, D, y);
}

// Row of column t0 + dt (0 <= dt <= t2 - t0) by the FP32 pass: the floor of y32, and in `ok`
// whether it stands, i.e. y32 lies farther than tol from a row boundary (the FP32 error is below
// tol, so the exact value is on the same side). A row that does not stand may be off by one and
// lie outside [0, F).
// The pass from D = b^2 + 4 a dt and dt2 = 2 dt (as a float, exact) given by the caller.
STT_HD int32_t row_tm_fp32_d(const RowTm &k, int32_t D, float dt2, bool &ok)
{
    const float s32 = sqrt_1ulp((float)D);
    const float xi = dt2 * rcp_1ulp(k.bf + s32);
    const float y = fmaf(xi, fmaf(xi, k.Cs, k.Bs), k.fs);
    // A value that stands lies above tol > 0 (the exact value is >= 0), where truncation is the
    // floor and the fraction y - floor(y) is exact.
#if defined(__HIP_DEVICE_COMPILE__)
    const float fr = __builtin_amdgcn_fractf(y);
#else
    const float fr = y - floorf(y);
#endif
    ok = fabsf(fr - 0.5f) < k.hw;
    return (int32_t)y;
}

STT_HD int32_t row_tm_fp32(const RowTm &k, int32_t dt, bool &ok)
{
    return row_tm_fp32_d(k, k.bb + mul_i24(k.a4, dt), (float)(2 * dt), ok);
}

// The row where the FP32 pass does not stand: its square root again (the same bits), then the
// exact path.
STT_HD int32_t row_tm_fallback(const RowTm &k, int32_t dt)
{
    const int32_t D = k.bb + mul_i24(k.a4, dt);
    return row_tm_exact(k, dt, D, sqrt_1ulp((float)D));
}

STT_HD int32_t row_tm(const RowTm &k, int32_t dt)
{
    bool ok;
    const int32_t r = row_tm_fp32(k, dt, ok);
    return ok ? r : row_tm_fallback(k, dt);
}

// ----------------------------------------------------------------------------
// Exact rasteriser of Eq. 6 as a second-order DDA.
// With Dt = t2 - t0 and k = 0..Dt, row(k) = floor(num(k) / Q) where
//   num(k) = (Dt-k)^2 f0 + 2 (Dt-k) k f1 + k^2 f2 = A + B k + C k^2,
//   A = Dt^2 f0, B = 2 Dt (f1 - f0), C = f0 - 2 f1 + f2, Q = Dt^2 * 256.
// num(k+1) - num(k) = B + C (2k + 1) =: Delta_k and Delta_{k+1} - Delta_k = 2C.
// The state keeps num(k) = row*Q + rem and Delta_k = dq*Q + dr with
// 0 <= rem, dr < Q (floor division), so one step is two carry-propagating
// adds of 32-bit quantities. Q < 2^31 for Dt <= 2895 keeps every sum < 2^32.
// ----------------------------------------------------------------------------
struct Dda {
    int32_t row;
    uint32_t rem;
    int32_t dq;
    uint32_t dr;
    int32_t ddq;
    uint32_t ddr;
    uint32_t Q;
};

STT_HD void floor_divmod(int64_t a, uint32_t q, int32_t &quo, uint32_t &rem)
{
    int64_t d = a / (int64_t)q;
    int64_t r = a - d * (int64_t)q;
    if (r < 0) { r += q; --d; }
    quo = (int32_t)d;
    rem = (uint32_t)r;
}

// State at an arbitrary integer k0 (k0 < 0 "rewinds" before the first column).
// The recurrence is exact for every integer k, so stepping from k0 reaches the
// exact rows at k = 0..Dt; rows at k < 0 or k > Dt are meaningless (and may
// leave [0, F)), which callers mask. row and dq are kept modulo 2^32 (the true
// values at negative k may not fit 32 bits), which is exact for the valid k.
STT_HD Dda dda_init_at(const Trk &t, int32_t k0)
{
    Dda s;
    const int64_t Dt = t.t2 - t.t0;
    const uint32_t Q = (uint32_t)(Dt * Dt) << 8;
    s.Q = Q;
    const int64_t A = Dt * Dt * (int64_t)t.f0;
    const int64_t C = (int64_t)t.f0 - 2 * (int64_t)t.f1 + (int64_t)t.f2;
    const int64_t B = 2 * Dt * ((int64_t)t.f1 - (int64_t)t.f0);
    const int64_t k = k0;
    const int64_t num = A + B * k + C * k * k;
    const int64_t del = B + C * (2 * k + 1);
    int64_t q = num / (int64_t)Q, r = num - q * (int64_t)Q;
    if (r < 0) { r += Q; --q; }
    s.row = (int32_t)(uint32_t)(uint64_t)q;
    s.rem = (uint32_t)r;
    q = del / (int64_t)Q;
    r = del - q * (int64_t)Q;
    if (r < 0) { r += Q; --q; }
    s.dq = (int32_t)(uint32_t)(uint64_t)q;
    s.dr = (uint32_t)r;
    floor_divmod(2 * C, Q, s.ddq, s.ddr);
    return s;
}

STT_HD Dda dda_init(const Trk &t)
{
    Dda s;
    const uint32_t Dt = (uint32_t)(t.t2 - t.t0);
    const uint32_t D2 = Dt * Dt;
    s.Q = D2 << 8;
    s.row = (int32_t)(t.f0 >> 8);
    s.rem = D2 * (t.f0 & 255u);
    const int64_t C = (int64_t)t.f0 - 2 * (int64_t)t.f1 + (int64_t)t.f2;
    const int64_t B = 2 * (int64_t)Dt * ((int64_t)t.f1 - (int64_t)t.f0);
    floor_divmod(B + C, s.Q, s.dq, s.dr);
    floor_divmod(2 * C, s.Q, s.ddq, s.ddr);
    return s;
}

STT_HD void dda_step(Dda &s)
{
    uint32_t r = s.rem + s.dr;
    const bool c1 = r >= s.Q;
    s.rem = c1 ? r - s.Q : r;
    s.row = (int32_t)((uint32_t)s.row + (uint32_t)s.dq + (c1 ? 1u : 0u));  // modulo 2^32
    uint32_t d = s.dr + s.ddr;
    const bool c2 = d >= s.Q;
    s.dr = c2 ? d - s.Q : d;
    s.dq = (int32_t)((uint32_t)s.dq + (uint32_t)s.ddq + (c2 ? 1u : 0u));
}

// The same walk in FP64, for the scorers' inner loops. It carries the
// centred numerator c(k) = num(k) - Q/2 + 1/2 (Q = 256 Dt^2 is even, so c is
// an integer plus a half, |c| < 2^52: exact in FP64, and the two adds per step
// are exact). Write num = a*Q + b with 0 <= b < Q < 2^31: c/Q = a - 1/2 +
// (b + 1/2)/Q lies inside (a - 1/2, a + 1/2), at least 1/(2Q) > 2^-32 from
// either end, while the product with the rounded 1/Q is off by at most 2^-37
// (relative 2^-52 on a value below 2^15). So one FMA, fma(c, 1/Q, 3*2^51),
// rounds to exactly 3*2^51 + a, an integer on the unit grid of [2^52, 2^53)
// whose low 32 bits are the row a = floor(num/Q). Rows of invalid k (k < 0 or
// k > Dt) are meaningless and must be masked by the caller.
struct DdaF {
    double num;   // c(k) = num(k) - Q/2 + 1/2
    double del;   // num(k+1) - num(k)
    double dd;    // 2C
    double invq;  // 1/Q rounded to nearest
};

STT_HD DdaF ddaf_init_at(const Trk &t, int32_t k0)
{
    DdaF s;
    const int64_t Dt = t.t2 - t.t0;
    const int64_t Q = (Dt * Dt) << 8;
    const int64_t A = Dt * Dt * (int64_t)t.f0;
    const int64_t C = (int64_t)t.f0 - 2 * (int64_t)t.f1 + (int64_t)t.f2;
    const int64_t B = 2 * Dt * ((int64_t)t.f1 - (int64_t)t.f0);
    const int64_t k = k0;
    s.num = (double)(A + B * k + C * k * k - (Q >> 1)) + 0.5;
    s.del = (double)(B + C * (2 * k + 1));
    s.dd = (double)(2 * C);
    s.invq = 1.0 / (double)Q;
    return s;
}

STT_HD int32_t ddaf_row(const DdaF &s)
{
    const double y = fma(s.num, s.invq, 6755399441055744.0);  // 3 * 2^51
    uint64_t u;
    __builtin_memcpy(&u, &y, sizeof u);
    return (int32_t)(uint32_t)u;
}

STT_HD void ddaf_step(DdaF &s)
{
    s.num += s.del;
    s.del += s.dd;
}

// ----------------------------------------------------------------------------
// Phase factor of Eq. 8. f dtau = (fq4/16 Hz)(dtau 2^-28 s) = fq4*dtau 2^-32
// turns, so the phase is the 32-bit wrap of fq4*dtau: exact. Per track,
// fq4(row) = fq4_lo + row*dfq4, hence phase(row) = pa + row*pb (mod 2^32).
// ----------------------------------------------------------------------------
STT_HD uint32_t phase_a(int32_t fq4_lo, int32_t dtau) { return (uint32_t)fq4_lo * (uint32_t)dtau; }
STT_HD uint32_t phase_b(int32_t dfq4, int32_t dtau) { return (uint32_t)dfq4 * (uint32_t)dtau; }

// The phase of row `row` as FP32 turns in [1, 2) -- the hardware sine and
// cosine take turns and reduce them exactly (measured on gfx950: the same
// error on [1, 2) as on [0, 1)). The exact 32-bit phase plus half a unit of
// the result is cut to its top 23 bits and spliced under the exponent of 1.0:
// rounded to 23 fractional bits, at most 2^-24 turn off. One funnel shift.
STT_HD float phase_turns(uint32_t pa, uint32_t pb, int32_t row)
{
    const uint32_t ph = pa + (uint32_t)row * pb + 256u;
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_bit_cast(float, __builtin_amdgcn_alignbit(0x7Fu, ph, 9u));  // (0x7F:ph) >> 9
#else
    return __builtin_bit_cast(float, (0x7Fu << 23) | (ph >> 9));
#endif
}

// Re[exp(2 pi i ph/2^32) (pr + i pi)]. The half-turn bit h = [ph in [1/4,3/4)
// turn] is split off exactly in integers, leaving |angle| <= pi/2 where the
// polynomials (near-minimax, from gen_sincos_coeffs.py) are accurate to about
// 1.5e-7; exp(i pi h) = (-1)^h flips the sign of the result.
STT_HD float rot_re(uint32_t ph, float pr, float pim)
{
    const uint32_t u = ph + 0x40000000u;
    const uint32_t h = u & 0x80000000u;
    const int32_t r = (int32_t)(ph - h);  // in [-2^30, 2^30): a quarter turn each side
    const float x = (float)r * 1.4629180792671596e-9f;  // 2 pi / 2^32
    const float s = x * x;
    float ps = 2.634815473e-06f;
    ps = fmaf(ps, s, -1.982276153e-04f);
    ps = fmaf(ps, s, 8.333242498e-03f);
    ps = fmaf(ps, s, -1.666666567e-01f);
    const float sn = fmaf(x * s, ps, x);
    float pc = -2.629789719e-07f;
    pc = fmaf(pc, s, 2.477459748e-05f);
    pc = fmaf(pc, s, -1.388865174e-03f);
    pc = fmaf(pc, s, 4.166666046e-02f);
    pc = fmaf(pc, s, -5.000000000e-01f);
    const float cs = fmaf(s, pc, 1.0f);
    const float v = fmaf(cs, pr, -sn * pim);
    return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v) ^ h);
}

// ----------------------------------------------------------------------------
// Best-key encoding (see the public header): order-preserving bits of the FP32
// score in the high word, 0xFFFFFFFF - j in the low word.
// ----------------------------------------------------------------------------
STT_HD uint64_t key_encode(float z, uint32_t j)
{
    if (z != z) z = -__builtin_huge_valf();
    if (z == 0.0f) z = 0.0f;
    const uint32_t b = __builtin_bit_cast(uint32_t, z);
    const uint32_t o = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ((uint64_t)o << 32) | (uint64_t)(0xFFFFFFFFu - j);
}

}  // namespace stt
