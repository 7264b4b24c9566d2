// Cross-power map formation on gfx950: the step before the template search that turns two
// detectors' strain into the complex SNR maps it scores (Sec. II, Eq. 7, and the formalism
// appendix), with time slides of one detector for background maps (Sec. IV-V).
//
//   k_col_fft     one workgroup per column: M Hann-weighted samples (columns overlap by half),
//                 a length-M/2 complex FFT in LDS over the even/odd sample pairs, then the
//                 real-FFT split for the kept bins only; s~ = dt * DFT.
//   k_psd         P'(t; f): mean of (2 / Nrm) |s~|^2 over the columns 2 .. nb+1 away.
//   k_form_maps   per (t, f) and per slide: Y = (2 / Nrm) conj(s~_I) s~_J(t + shift) and
//                 sigma = sqrt(P'_I P'_J(t + shift) / 2), written to the caller's maps.
//
// Twiddles e^{-2 pi i j / M} (j < M/2) and the window sin^2(pi n / M) come from a table the
// host fills in FP64 and rounds once to FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stt {

constexpr int kFftThreads = 256;
constexpr int kMaxFftM = 8192;     // samples per column; the complex FFT has M/2 points in LDS
constexpr int kSlidesPerLaunch = 16;

struct SlideArgs {
    float2 *Y[kSlidesPerLaunch];
    float *sigma[kSlidesPerLaunch];
    int32_t shift[kSlidesPerLaunch];  // in [0, T)
    int32_t n;
};

// x: strain (8-byte aligned); tab: M/2 twiddles (float2) followed by M window values (float);
// spec: [T][F] complex64. Grid: T workgroups of kFftThreads lanes, N = M/2 float2 of LDS.
__global__ __launch_bounds__(kFftThreads) void k_col_fft(const float *__restrict__ x, int M, int lg, int k_lo, int F,
                                                         float dt, const float2 *__restrict__ tab,
                                                         float2 *__restrict__ spec)
{
    extern __shared__ float2 z[];
    const int N = M >> 1;
    const float2 *tw = tab;
    const float2 *win2 = reinterpret_cast<const float2 *>(tab + N);  // window pairs (w[2i], w[2i+1])
    const int t = blockIdx.x;
    const float2 *seg = reinterpret_cast<const float2 *>(x + (int64_t)t * N);
    // even/odd sample pairs as one complex sequence, stored in bit-reversed order
    for (int i = threadIdx.x; i < N; i += kFftThreads) {
        const float2 v = seg[i], w = win2[i];
        const unsigned r = __builtin_bitreverse32((unsigned)i) >> (32 - lg);
        z[r] = make_float2(v.x * w.x, v.y * w.y);
    }
    __syncthreads();
    // radix-2 decimation in time: stage s joins blocks of 2^s into blocks of 2^(s+1)
    for (int s = 0; s < lg; ++s) {
        const int half = 1 << s;
        const int tstep = M >> (s + 1);  // e^{-2 pi i p / 2^(s+1)} = tw[p * M / 2^(s+1)]
        for (int b = threadIdx.x; b < (N >> 1); b += kFftThreads) {
            const int p = b & (half - 1);
            const int i0 = ((b >> s) << (s + 1)) + p;
            const int i1 = i0 + half;
            const float2 w = tw[p * tstep];
            const float2 a = z[i0], c = z[i1];
            const float cr = w.x * c.x - w.y * c.y, ci = w.x * c.y + w.y * c.x;
            z[i0] = make_float2(a.x + cr, a.y + ci);
            z[i1] = make_float2(a.x - cr, a.y - ci);
        }
        __syncthreads();
    }
    // X[k] = E[k] + e^{-2 pi i k / M} O[k] with E = (Z[k] + conj Z[N-k]) / 2 (even samples) and
    // O = (Z[k] - conj Z[N-k]) / 2i (odd samples); only the kept bins k_lo .. k_lo+F-1 (< N)
    for (int f = threadIdx.x; f < F; f += kFftThreads) {
        const int k = k_lo + f;
        const float2 a = z[k], b = z[(N - k) & (N - 1)];
        const float er = 0.5f * (a.x + b.x), ei = 0.5f * (a.y - b.y);
        const float orr = 0.5f * (a.y + b.y), oi = -0.5f * (a.x - b.x);
        const float2 w = tw[k];
        const float xr = er + (w.x * orr - w.y * oi), xi = ei + (w.x * oi + w.y * orr);
        spec[(int64_t)t * F + f] = make_float2(xr * dt, xi * dt);
    }
}

// P'(t; f) = scale * mean |spec(t', f)|^2 over 2 <= |t' - t| <= nb + 1 inside [0, T).
// Grid: (ceil(F / 256), T); every column has a neighbour (T >= 4, checked by the host).
__global__ __launch_bounds__(256) void k_psd(const float2 *__restrict__ spec, int T, int F, int nb, float scale,
                                             float *__restrict__ psd)
{
    const int f = blockIdx.x * 256 + threadIdx.x;
    const int t = blockIdx.y;
    if (f >= F) return;
    float acc = 0.f;
    int cnt = 0;
    for (int u = t - nb - 1; u <= t + nb + 1; ++u) {
        if (u < 0 || u >= T || (u - t <= 1 && t - u <= 1)) continue;
        const float2 v = spec[(int64_t)u * F + f];
        acc += v.x * v.x + v.y * v.y;
        ++cnt;
    }
    psd[(int64_t)t * F + f] = scale * acc / (float)cnt;
}

// One launch writes up to kSlidesPerLaunch slide maps. Lanes run along frequency, P bins each
// (P = 2 when F and ld are even and the buffers 16-byte aligned: one 16-byte and one 8-byte store
// per lane per slide), so every store is a coalesced row segment. Workgroups go round-robin to the
// 8 XCDs; the remap gives each XCD a contiguous run of columns t, so the J columns t + shift that
// its slides read stay in its own L2 instead of crossing to the MALL once per slide.
// Grid: 1-D, ceil(nbx * T / 8) * 8 workgroups of 256 lanes, nbx = ceil(F / (256 P)).
template <int P>
__global__ __launch_bounds__(256) void k_form_maps(const float2 *__restrict__ si, const float *__restrict__ pi,
                                                   const float2 *__restrict__ sj, const float *__restrict__ pj,
                                                   int T, int F, float scale, int64_t ld, SlideArgs a)
{
    const int nbx = (F + 256 * P - 1) / (256 * P);
    const int64_t nblk = (int64_t)nbx * T;
    const int64_t per = (nblk + 7) / 8;
    const int64_t L = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (L >= nblk) return;
    const int t = (int)(L / nbx);
    const int f = P * ((int)(L % nbx) * 256 + (int)threadIdx.x);
    if (f >= F) return;
    typedef float fv __attribute__((ext_vector_type(2 * P)));  // P complex values
    typedef float pv __attribute__((ext_vector_type(P)));      // P powers
    const fv u = *reinterpret_cast<const fv *>(si + (int64_t)t * F + f);
    const pv pu = *reinterpret_cast<const pv *>(pi + (int64_t)t * F + f);
    for (int k = 0; k < a.n; ++k) {
        int tj = t + a.shift[k];
        if (tj >= T) tj -= T;
        const fv v = *reinterpret_cast<const fv *>(sj + (int64_t)tj * F + f);
        const pv pq = *reinterpret_cast<const pv *>(pj + (int64_t)tj * F + f);
        fv y;
        pv sg;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const float ur = u[2 * q], ui = u[2 * q + 1], vr = v[2 * q], vi = v[2 * q + 1];
            y[2 * q] = scale * (ur * vr + ui * vi);
            y[2 * q + 1] = scale * (ur * vi - ui * vr);
            sg[q] = sqrtf(0.5f * pu[q] * pq[q]);
        }
        *reinterpret_cast<fv *>(a.Y[k] + (int64_t)t * ld + f) = y;
        *reinterpret_cast<pv *>(a.sigma[k] + (int64_t)t * ld + f) = sg;
    }
}

}  // namespace stt
