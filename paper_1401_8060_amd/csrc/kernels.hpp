// kernels.hpp -- the libstt device kernels for gfx950 (wave64, 160 KB LDS per CU).
//
// Hot path of the template search (paper Sec. III, Eq. 6 and Eq. 8):
//   k_make_tracks   materialise templates (Philox4x32-10 + exact unranking)
//   k_bin_count     \  counting sort of templates by (start, end) column bucket,
//   k_bin_scan       | so that a workgroup's templates cover nearly the same
//   k_bin_group      | columns and its lanes stay busy through a time sweep;
//   k_bin_fine      /  scattered in two passes, to groups of buckets, then buckets
//   k_fold_polar    p = Y/sigma of every pixel in polar form (|p|, arg p in
//                   2^-32 turn), the layout the scorers stage: one cosine per term
//   k_score_slab    time-slab scorer: the workgroup copies slabs of consecutive
//                   columns of the folded map into LDS (LDS DMA, double-buffered)
//                   and every lane gathers its templates' pixels there
//   k_score_direct  one lane per template, pixels gathered straight from the
//                   map in global memory (small calls, very wide maps)
//   k_reduce_keys   max of the slab scorer's per-workgroup best keys
//   k_argmax        max/argmax of an existing score array
// Reductions use the packed 64-bit key (score bits, ~index), so results do not
// depend on scheduling: wave shuffles, then across the workgroup through LDS
// (slab scorers) or one 64-bit atomic max per wave (small kernels).
#pragma once

#include <hip/hip_fp16.h>

#include "dev_common.hpp"

namespace stt {

struct MapP {
    const float2 *Y;   // [T][ld] complex64 (FP32 map) -- or __half2 p (FP16 map)
    const float *sig;  // [T][ld] sigma (FP32 map only)
    int32_t T, F;
    int64_t ld;
    int32_t fq4_lo, dfq4;
    float scale;       // FP16 map: p = stored * scale (a power of two)
};

// Map element formats: the caller's (Y, sigma) FP32 map; the caller's FP16 map
// (one 32-bit word per pixel: arg p in 2^-16 turn in the low half, |p| * 2^-e
// as binary16 in the high half); p = Y/sigma folded into complex64 by k_fold_p
// (read by the smooth statistic); p folded into polar form by k_fold_polar
// (read by every scorer of Eq. 8 on an FP32 map): |p| as FP32 and arg p as a
// 32-bit fraction of a turn, 8 bytes per pixel; and the FP16 map's words copied
// into the folded layout (read by every scorer on an FP16 map), 4 bytes per
// pixel. Folded maps pad columns to whole 1 KB pieces (128 or 256 pixels) so
// that slabs can be copied into LDS by 1 KB LDS-DMA instructions.
enum : int { kMapF32 = 0, kMapP16 = 1, kMapPF = 2, kMapPol = 3, kMapPolH = 4 };
constexpr int kDmaBytes = 1024;  // bytes one wave moves per LDS-DMA instruction (64 lanes x 16 B)

// Element type of a map format in registers and LDS.
template <int MAPT> struct ElemOf { using type = float2; };
template <> struct ElemOf<kMapPolH> { using type = uint32_t; };
template <int MAPT> using elem_t = typename ElemOf<MAPT>::type;
template <int MAPT> constexpr int kDmaPix = kDmaBytes / (int)sizeof(elem_t<MAPT>);  // pixels per 1 KB piece

// binary16 bits of the high half of a word, as FP32 (exact)
__device__ __forceinline__ float half_hi(uint32_t w)
{
    return __half2float(__ushort_as_half((unsigned short)(w >> 16)));
}

// The complex SNR p = Y/sigma of pixel element e (Eq. 7 with the appendix's rho = Y/sigma).
// FP16 map: |p| 2^e exp(2 pi i arg) evaluated in FP64 and rounded once per component.
template <int MAPT>
__device__ __forceinline__ float2 load_p(const MapP &m, int64_t e)
{
    if constexpr (MAPT == kMapP16) {
        const uint32_t w = reinterpret_cast<const uint32_t *>(m.Y)[e];
        const double mag = (double)half_hi(w) * (double)m.scale;
        double sn, cs;
        sincospi((double)(w & 0xFFFFu) * (1.0 / 32768.0), &sn, &cs);
        return make_float2((float)(mag * cs), (float)(mag * sn));
    } else if constexpr (MAPT == kMapPF || MAPT == kMapPol) {
        return m.Y[e];  // (a polar map's element is returned as stored)
    } else {
        const float2 y = m.Y[e];
        const float w = 1.0f / m.sig[e];
        return make_float2(y.x * w, y.y * w);
    }
}

// One element of a map as its scorers hold it: a word of a folded FP16 map, p otherwise.
template <int MAPT>
__device__ __forceinline__ elem_t<MAPT> load_e(const MapP &m, int64_t e)
{
    if constexpr (MAPT == kMapPolH) return reinterpret_cast<const uint32_t *>(m.Y)[e];
    else return load_p<MAPT>(m, e);
}

// p of every pixel into a complex64 map with column stride ld_out (pixels
// F..ld_out-1 of a column are zero): Y/sigma of an FP32 map, or the exact FP32
// value of an FP16 map's entry. The same expression as load_p's, so scores do
// not depend on whether the map was folded first.
template <int MAPT>
__global__ __launch_bounds__(256) void k_fold_p(MapP m, float2 *out, int64_t ld_out)
{
    const int64_t n = (int64_t)m.T * ld_out;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t t = i / ld_out, r = i - t * ld_out;
        out[i] = r < m.F ? load_p<MAPT>(m, t * m.ld + r) : make_float2(0.0f, 0.0f);
    }
}

// arg (x + iy) as a 32-bit fraction of a turn, from FP32 components. The first
// octant's angle atan(a), a = min(|x|, |y|) / max(|x|, |y|), is reduced to
// |t| <= tan(pi/8) (atan(a) = pi/4 + atan((a - 1)/(a + 1)) above), evaluated as
// atan(t)/(2 pi) = t P(t^2) in FP32 (coefficients from gen_atan_coeffs.py) and
// rounded to 2^-32 turn; the octant and quadrant are then undone in integers
// (eighths of a turn are exact). The polynomial in FP32 is within 41 units of
// 2^-32 turn; with the FP32 division and reduction about 100 units (2.3e-8
// turn) in all -- well below the 2^-24-turn rounding of the phase each term
// takes before its cosine. arg 0 = 0 (its magnitude is 0 then).
__device__ __forceinline__ uint32_t arg_turns(float x, float y)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const bool swap = ay > ax;  // the angle from the nearer axis is atan(min/max)
    const float num = swap ? ax : ay, den = swap ? ay : ax;
    const float a = den > 0.0f ? num / den : 0.0f;
    const bool hi = a > 0.41421356f;
    const float t = hi ? (a - 1.0f) / (a + 1.0f) : a;
    const float s = t * t;
    float q = -9.602202103e-03f;
    q = fmaf(q, s, 1.682715677e-02f);
    q = fmaf(q, s, -2.266363613e-02f);
    q = fmaf(q, s, 3.182814270e-02f);
    q = fmaf(q, s, -5.305160582e-02f);
    q = fmaf(q, s, 1.591549367e-01f);
    const int32_t f = (int32_t)rintf(t * q * 4294967296.0f);  // |t q| <= 1/16 turn
    uint32_t u = (uint32_t)((hi ? (1 << 29) : 0) + f);        // first-octant angle
    if (swap) u = (1u << 30) - u;                               // first quadrant
    if (x < 0.0f) u = (1u << 31) - u;                           // second quadrant
    if (y < 0.0f) u = 0u - u;                                   // lower half, modulo one turn
    return u;
}

// Polar form of p: (|p| rounded to FP32, arg p in 2^-32 turn as the bits of the second word).
// The FP32 components square exactly in FP64, so |p|^2 = x^2 + y^2 is rounded once, its square
// root once more and the result once to FP32.
__device__ __forceinline__ float2 polar_of(float2 p)
{
    const double x = p.x, y = p.y;
    const float mag = (float)sqrt(fma(x, x, y * y));
    return make_float2(mag, __uint_as_float(arg_turns(p.x, p.y)));
}

constexpr int kFoldRows = 4;  // rows per thread of the fold kernels: all their loads in flight at once

// Column t, rows r0 + 256 i + threadIdx.x (i < kFoldRows) of a fold: every load first, then the
// polar forms and stores (pixels F .. ld_out-1 zero).
template <int MAPT>
__device__ __forceinline__ void fold_rows(const MapP &m, int64_t t, int64_t r0, float2 *out, int64_t ld_out)
{
    float2 p[kFoldRows];
#pragma unroll
    for (int i = 0; i < kFoldRows; ++i) {
        const int64_t r = r0 + i * 256 + threadIdx.x;
        p[i] = r < m.F ? load_p<MAPT>(m, t * m.ld + r) : make_float2(0.0f, 0.0f);
    }
#pragma unroll
    for (int i = 0; i < kFoldRows; ++i) {
        const int64_t r = r0 + i * 256 + threadIdx.x;
        if (r < ld_out) out[t * ld_out + r] = r < m.F ? polar_of(p[i]) : make_float2(0.0f, 0.0f);
    }
}

// The same rows of an FP16 map: its words as they are.
__device__ __forceinline__ void fold_words_rows(const MapP &m, int64_t t, int64_t r0, uint32_t *out, int64_t ld_out)
{
    const uint32_t *w = reinterpret_cast<const uint32_t *>(m.Y);
    uint32_t v[kFoldRows];
#pragma unroll
    for (int i = 0; i < kFoldRows; ++i) {
        const int64_t r = r0 + i * 256 + threadIdx.x;
        v[i] = r < m.F ? w[t * m.ld + r] : 0u;
    }
#pragma unroll
    for (int i = 0; i < kFoldRows; ++i) {
        const int64_t r = r0 + i * 256 + threadIdx.x;
        if (r < ld_out) out[t * ld_out + r] = v[i];
    }
}

// p of every pixel in polar form into a map with column stride ld_out (pixels F..ld_out-1 of a
// column are zero): from Y/sigma of an FP32 map, or from the exact FP32 values of an FP16 map's
// entries (load_p's expression). Grid: column blockIdx.x, y strides over its rows.
template <int MAPT>
__global__ __launch_bounds__(256) void k_fold_polar(MapP m, float2 *out, int64_t ld_out)
{
    for (int64_t r0 = (int64_t)blockIdx.y * 256 * kFoldRows; r0 < ld_out; r0 += (int64_t)gridDim.y * 256 * kFoldRows)
        fold_rows<MAPT>(m, blockIdx.x, r0, out, ld_out);
}

// The words of an FP16 map into the folded layout (column stride ld_out, pixels F..ld_out-1 zero).
// Grid: column blockIdx.x, y strides over its rows.
__global__ __launch_bounds__(256) void k_fold_words(MapP m, uint32_t *out, int64_t ld_out)
{
    for (int64_t r0 = (int64_t)blockIdx.y * 256 * kFoldRows; r0 < ld_out; r0 += (int64_t)gridDim.y * 256 * kFoldRows)
        fold_words_rows(m, blockIdx.x, r0, out, ld_out);
}

// One fold of a batch: map src into dst (column stride ld_out); its columns are col0 .. col0 +
// T - 1 of the batch's column run (col0 ascending over the maps).
struct FoldJob {
    MapP src;
    void *dst;
    int64_t ld_out;
    uint32_t col0;
};

// Every map of a batch in one launch: blockIdx.x runs over the batch's columns, each workgroup
// finds its map once by bisection of col0 (jobs[n_jobs].col0 = the total), y strides over rows.
// FP32 maps fold to polar form (k_fold_polar), FP16 maps copy their words (k_fold_words).
template <int MAPT>
__global__ __launch_bounds__(256) void k_fold_batch(const FoldJob *jobs, int n_jobs)
{
    const uint32_t col = blockIdx.x;
    int lo = 0, hi = n_jobs;  // jobs[lo].col0 <= col < jobs[hi].col0
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (jobs[mid].col0 <= col) lo = mid; else hi = mid;
    }
    const FoldJob &j = jobs[lo];
    const int64_t t = (int64_t)(col - j.col0);
    for (int64_t r0 = (int64_t)blockIdx.y * 256 * kFoldRows; r0 < j.ld_out; r0 += (int64_t)gridDim.y * 256 * kFoldRows) {
        if constexpr (MAPT == kMapP16)
            fold_words_rows(j.src, t, r0, (uint32_t *)j.dst, j.ld_out);
        else
            fold_rows<MAPT>(j.src, t, r0, (float2 *)j.dst, j.ld_out);
    }
}

constexpr int kMaxDt = 2895;  // Dt * Dt * 256 < 2^31
// FP32 partial sums are flushed into the FP64 total after every column c with
// c % kFlush == kFlush - 1: a fixed grid of absolute columns, so a template's
// arithmetic does not depend on which workgroup or scorer handles it.
constexpr int kFlush = 16;
constexpr int kWG = 256;      // threads per workgroup of the scorers

__device__ __forceinline__ bool track_ok(const Trk &t, const MapP &m)
{
    const uint32_t frange = (uint32_t)m.F << 8;
    return t.t0 >= 0 && t.t2 < m.T && t.t2 > t.t0 && t.t2 - t.t0 <= kMaxDt && t.f0 < frange &&
           t.f1 < frange && t.f2 < frange;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

// Wave-wide min/max, returned as a wave-uniform (scalar) value so that loop
// bounds and addresses derived from it stay off the vector ALU.
__device__ __forceinline__ int wave_min_i32(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off));
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int wave_max_i32(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ void merge_key(uint64_t *best, uint64_t key)
{
    key = wave_max_u64(key);
    if (best && (threadIdx.x & 63) == 0 && key) atomicMax((unsigned long long *)best, (unsigned long long)key);
}

// z of a template from its FP64 sum S of terms in units of `scale` (2^e of an FP16 map, else 1).
__device__ __forceinline__ float finish(double S, int32_t N, int32_t norm, float scale)
{
    S *= (double)scale;
    return (float)(norm == 1 ? S / (double)N : S / sqrt((double)N));
}

// Phase constants of one template: its Eq. 8 phase at row r is pa + r*pb in
// units of 2^-32 turn, exact with 32-bit wrap-around.
struct PhaseK {
    uint32_t pa, pb;
};

__device__ __forceinline__ PhaseK phase_k(const MapP &m, int32_t dtau)
{
    return PhaseK{phase_a(m.fq4_lo, dtau), phase_b(m.dfq4, dtau)};
}

// part + Re[exp(2 pi i phase(row)) p], the template's Eq. 8 term at this row.
// HW: the exact 32-bit phase rounded once to FP32 turns (phase_turns) feeds
// the hardware sine and cosine, which take turns; measured on gfx950 over 2^22
// phases spanning a turn: at most 1.25e-7 absolute error, rms 3.5e-8, no bias.
// The two products are added to the running sum by fused multiply-adds.
// HW = false: the polynomial of rot_re (about 1.5e-7 absolute).
template <bool HW>
__device__ __forceinline__ float add_term(float part, const PhaseK &k, int32_t row, float2 p)
{
    if constexpr (HW) {
        const float x = phase_turns(k.pa, k.pb, row);
        part = fmaf(__builtin_amdgcn_cosf(x), p.x, part);
        return fmaf(-__builtin_amdgcn_sinf(x), p.y, part);
    } else {
        return part + rot_re(k.pa + (uint32_t)row * k.pb, p.x, p.y);
    }
}

// The same term from the polar form (|p|, arg p): Re[exp(2 pi i phase) p] = |p| cos(2 pi (phase +
// arg p)). The two phases add exactly in 32-bit turns, so one cosine and one fused multiply-add
// replace the sine, the cosine and the two products of the Cartesian form. HW: the hardware cosine
// of the sum rounded once to FP32 turns; HW = false: the polynomial of rot_re.
// Polar elements: (|p|, arg p) of an FP32 map's fold, or an FP16 map's word (|p| 2^-e and arg p
// in 2^-16 turn, which shifted left by 16 is the same 32-bit fraction of a turn, exactly).
__device__ __forceinline__ float pol_mag(float2 v) { return v.x; }
__device__ __forceinline__ uint32_t pol_arg(float2 v) { return __float_as_uint(v.y); }
__device__ __forceinline__ float pol_mag(uint32_t w) { return half_hi(w); }
__device__ __forceinline__ uint32_t pol_arg(uint32_t w) { return w << 16; }

template <bool HW, typename E>
__device__ __forceinline__ float add_term_pol(float part, const PhaseK &k, int32_t row, E v)
{
    const uint32_t arg = pol_arg(v);
    if constexpr (HW) {
        const float x = phase_turns(k.pa + arg, k.pb, row);
        return fmaf(__builtin_amdgcn_cosf(x), pol_mag(v), part);
    } else {
        return part + rot_re(k.pa + arg + (uint32_t)row * k.pb, pol_mag(v), 0.0f);
    }
}

// The Eq. 8 term of one pixel element of map format MAPT (polar or Cartesian).
template <bool HW, int MAPT>
__device__ __forceinline__ float add_term_m(float part, const PhaseK &k, int32_t row, elem_t<MAPT> v)
{
    if constexpr (MAPT == kMapPol || MAPT == kMapPolH) return add_term_pol<HW>(part, k, row, v);
    else return add_term<HW>(part, k, row, v);
}

// A fill kernel rather than a memset node, so that captured graphs replay it faithfully.
__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- generation

__global__ __launch_bounds__(256) void k_make_tracks(GenP g, uint64_t first, int64_t n, Trk *out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = draw_track(g, first + (uint64_t)i);
}

// ---------------------------------------------------------------- direct scorer

template <bool EXPL, bool HW, int MAPT>
__global__ __launch_bounds__(kWG) void k_score_direct(MapP m, GenP g, const Trk *tr, uint64_t first, int64_t n,
                                                      int32_t norm, float *snr, uint64_t *best)
{
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    uint64_t key = 0;
    if (i < n) {
        const Trk t = EXPL ? tr[i] : draw_track(g, first + (uint64_t)i);
        float z = __builtin_nanf("");
        if (!EXPL || track_ok(t, m)) {
            DdaF s = ddaf_init_at(t, 0);
            const PhaseK pk = phase_k(m, t.dtau);
            const int32_t N = t.t2 - t.t0 + 1;
            int64_t base = (int64_t)t.t0 * m.ld;
            double acc = 0.0;
            float part = 0.0f;
            for (int32_t k = 0; k < N; ++k) {
                const int32_t row = ddaf_row(s);
                const elem_t<MAPT> p = load_e<MAPT>(m, base + row);
                part = add_term_m<HW, MAPT>(part, pk, row, p);
                if (((t.t0 + k) & (kFlush - 1)) == kFlush - 1) { acc += part; part = 0.0f; }
                ddaf_step(s);
                base += m.ld;
            }
            z = finish(acc + part, N, norm, m.scale);
        }
        if (snr) snr[i] = z;
        key = key_encode(z, (uint32_t)(first + (uint64_t)i));
    }
    merge_key(best, key);
}

// One wave per template, for calls too small to fill the chip with one lane
// per template. The template's columns fall into flush groups of kFlush
// aligned columns; lane l takes groups l, l + 64, ... and computes each
// group's FP32 partial with the same operations, in the same order, as the
// sequential walk of k_score_direct. The FP64 sum over groups then runs in
// column order (read lane by lane), so the score is bit-identical to the other
// scorers'. Four waves (templates) per workgroup.
constexpr int kWaveGroups = (STT_MAX_T + kFlush - 1) / kFlush + 1;  // groups a template can touch
constexpr int kWaveRounds = (kWaveGroups + 63) / 64;

template <bool EXPL, bool HW, int MAPT>
__global__ __launch_bounds__(256) void k_score_wave(MapP m, GenP g, const Trk *tr, uint64_t first, int64_t n,
                                                    int32_t norm, float *snr, uint64_t *best)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);  // wave-uniform
    uint64_t key = 0;
    if (i < n) {
        const Trk t = EXPL ? tr[i] : draw_track(g, first + (uint64_t)i);
        float z = __builtin_nanf("");
        if (!EXPL || track_ok(t, m)) {
            const PhaseK pk = phase_k(m, t.dtau);
            const int gfirst = t.t0 / kFlush, glast = t.t2 / kFlush;
            float gp[kWaveRounds];
#pragma unroll
            for (int r = 0; r < kWaveRounds; ++r) {
                gp[r] = 0.0f;
                const int gi = gfirst + r * 64 + lane;
                if (gi > glast) continue;
                const int ca = max(t.t0, gi * kFlush), cb = min(t.t2, gi * kFlush + kFlush - 1);
                DdaF s = ddaf_init_at(t, ca - t.t0);
                int64_t base = (int64_t)ca * m.ld;
                float part = 0.0f;
                for (int c = ca; c <= cb; ++c) {
                    const int32_t row = ddaf_row(s);
                    part = add_term_m<HW, MAPT>(part, pk, row, load_e<MAPT>(m, base + row));
                    ddaf_step(s);
                    base += m.ld;
                }
                gp[r] = part;
            }
            // The sequential walk adds each group's partial to acc, in order: at the group's flush
            // column, or (the last group, when t2 is not a flush column) as finish(acc + part);
            // a flushed last group leaves part = 0 for that final addition.
            const int ng = glast - gfirst + 1;
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < kWaveRounds; ++r) {
                const int cnt = min(64, ng - r * 64);
                for (int l = 0; l < cnt; ++l)
                    acc += __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, gp[r]), l));
            }
            if ((t.t2 & (kFlush - 1)) == kFlush - 1) acc = acc + 0.0f;
            z = finish(acc, t.t2 - t.t0 + 1, norm, m.scale);
        }
        if (lane == 0 && snr) snr[i] = z;
        key = key_encode(z, (uint32_t)(first + (uint64_t)i));
    }
    merge_key(best, key);
}

// ---------------------------------------------------------------- argmax of an array

__global__ __launch_bounds__(256) void k_argmax(const float *z, int64_t n, uint64_t first, uint64_t *best)
{
    uint64_t key = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const uint64_t k = key_encode(z[i], (uint32_t)(first + (uint64_t)i));
        key = k > key ? k : key;
    }
    merge_key(best, key);
}

// ---------------------------------------------------------------- binning by time extent
// Bucket of a template: b0 = t0 >> wb, b2 = t2 >> wb (b0 <= b2), nb buckets
// per axis. Buckets are numbered longest extent first: with e = nb - 1 -
// (b2 - b0) (0 for the longest), bucket = e (e + 1) / 2 + b0, b0 <= e. Blocks
// of binned templates are dispatched in that order, so the longest-running
// blocks start first and the launch ends on short ones. Invalid given
// templates go to bucket 0 (they are skipped when scored).
//
// The sort: count, scans, two scatters. Buckets form groups of 2^kGroupShift
// consecutive ones. The count (one workgroup per chunk of kBinChunk templates)
// draws each template's bucket once and keeps it (2 bytes, in the space the
// binned order fills last), adds its chunk's bucket histogram to the totals
// and writes the chunk's count per group. The scans give every bucket its
// start, every group its region and every chunk its run in each group. The
// first scatter moves each index, with its bucket within the group, to its
// chunk's run in its group's region (no cursor atomics: the place of every run
// is known). The second takes each group's region in chunks of kFineChunk and
// moves each index to its bucket, the runs reserved by atomics on the bucket
// cursors. Each scatter workgroup first orders its chunk by key in LDS, then
// stores it run by run: consecutive lanes write consecutive addresses, so a
// store instruction touches one or two cache lines (a single scatter into all
// buckets would store about one index per bucket per workgroup: one cache
// line per lane).

constexpr int kBinPerThread = 32;                 // templates per thread of the count (256 lanes)
constexpr int kBinChunk = 256 * kBinPerThread;    // templates per sort chunk: count, first scatter
constexpr int kFineChunk = 4096;                  // templates per chunk of the second scatter
constexpr int kScatterWG = 512;                   // lanes of a scatter workgroup
constexpr int kMaxBins = 128 * 129 / 2;           // at most 128 buckets per axis
constexpr int kGroupShift = 6;                    // buckets per group: 64
constexpr int kGroupMask = (1 << kGroupShift) - 1;
constexpr int kMaxGroups = (kMaxBins + kGroupMask) >> kGroupShift;
constexpr int kGroupSlots = kMaxGroups + 1 + (kMaxGroups & 1 ? 0 : 1);  // groups + 1 entries, an even count
static_assert(kMaxGroups << kGroupShift == kMaxBins, "bucket tables are whole groups");
static_assert(kMaxGroups <= 3 * 64, "one wave scans the group table");

// The slot of item in a table of ascending starts: start[k] <= item < start[k + 1], 0 <= k < n.
__device__ __forceinline__ int find_slot(const uint32_t *start, int n, uint32_t item)
{
    int lo = 0, hi = n;  // start[lo] <= item < start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= item) lo = mid; else hi = mid;
    }
    return lo;
}

// Exclusive prefix sums by one wave (the caller's lanes 0..63) of val(0 .. cnt-1),
// cnt <= 192: out[k] = val(0) + ... + val(k-1), out[cnt] = the total.
template <typename F>
__device__ __forceinline__ void wave_prefix(F val, int cnt, uint32_t *out)
{
    const int lane = threadIdx.x & 63;
    uint32_t v[3], s = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int k = 3 * lane + j;
        v[j] = k < cnt ? val(k) : 0u;
        s += v[j];
    }
    uint32_t incl = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    uint32_t run = incl - s;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int k = 3 * lane + j;
        if (k < cnt) out[k] = run;
        run += v[j];
    }
    if (lane == 63) out[cnt] = incl;
}

template <bool EXPL>
__device__ __forceinline__ uint32_t bin_of(const GenP &g, const Trk *tr, const MapP &m, uint64_t first, int64_t i,
                                           int wb)
{
    int32_t t0, t2;
    if (EXPL) {
        const Trk t = tr[i];
        if (!track_ok(t, m)) return 0;
        t0 = t.t0;
        t2 = t.t2;
    } else {
        draw_extent(g, first + (uint64_t)i, t0, t2);
    }
    const uint32_t b0 = (uint32_t)t0 >> wb, b2 = (uint32_t)t2 >> wb;
    const uint32_t e = ((uint32_t)(m.T - 1) >> wb) - (b2 - b0);
    return e * (e + 1) / 2 + b0;
}

// The count's step for one chunk, after its histogram hist[0 .. nbins-1] is
// complete in LDS: totals[b] += hist[b], and ccnt[k * stride] = the chunk's
// templates in group k (a thread per group; thread k starts its sum at bucket
// k mod 64 of the group, so the lanes of a wave read 64 different banks).
__device__ __forceinline__ void count_out(const uint32_t *hist, int nbins, uint32_t *totals, uint32_t *ccnt,
                                          size_t stride)
{
    for (int b = threadIdx.x; b < nbins; b += 256)
        if (hist[b]) atomicAdd(&totals[b], hist[b]);
    const int ngroups = (nbins + kGroupMask) >> kGroupShift;
    for (int k = threadIdx.x; k < ngroups; k += 256) {
        const int b0 = k << kGroupShift, nb = min(1 << kGroupShift, nbins - b0);
        uint32_t v = 0;
#pragma unroll 8
        for (int i = 0; i <= kGroupMask; ++i) {
            const int j = (i + k) & kGroupMask;
            if (j < nb) v += hist[b0 + j];
        }
        ccnt[(size_t)k * stride] = v;
    }
}

// Count: bins[i] = the bucket of template i; count_out for workgroup (chunk) c
// at ccnt + c with stride gridDim.x (row k of ccnt: group k's count per chunk).
template <bool EXPL>
__global__ __launch_bounds__(256) void k_bin_count(MapP m, GenP g, const Trk *tr, uint64_t first, int64_t n, int wb,
                                                   int nbins, uint32_t *totals, uint16_t *bins, uint32_t *ccnt)
{
    __shared__ uint32_t hist[kMaxBins];
    for (int b = threadIdx.x; b < nbins; b += 256) hist[b] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kBinChunk;
    for (int q = 0; q < kBinPerThread; ++q) {
        const int64_t i = base + q * 256 + threadIdx.x;
        if (i < n) {
            const uint32_t b = bin_of<EXPL>(g, tr, m, first, i, wb);
            bins[i] = (uint16_t)b;
            atomicAdd(&hist[b], 1u);
        }
    }
    __syncthreads();
    count_out(hist, nbins, totals, ccnt + blockIdx.x, gridDim.x);
}

// The bucket scan of one call or map by NT threads (nbins <= kMaxBins):
// cursor[b] = base + the templates in buckets before b; gstart[k] = cursor of
// group k's first bucket, gstart[ngroups] = base + all; fitem[k] = the first
// second-scatter chunk of group k, fitem[ngroups] = their count.
template <int NT>
__device__ __forceinline__ void scan_buckets(const uint32_t *totals, int nbins, uint32_t base, uint32_t *cursor,
                                             uint32_t *gstart, uint32_t *fitem)
{
    constexpr int kPer = (kMaxBins + NT - 1) / NT;
    __shared__ uint32_t wsum[NT / 64];
    __shared__ uint32_t gs[kGroupSlots];
    const int per = (nbins + NT - 1) / NT;
    const int lo = threadIdx.x * per;
    uint32_t v[kPer], s = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int b = lo + j;
        v[j] = j < per && b < nbins ? totals[b] : 0u;
        s += v[j];
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t incl = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    uint32_t run = base + incl - s;
    for (int w = 0; w < wv; ++w) run += wsum[w];
    const int ngroups = (nbins + kGroupMask) >> kGroupShift;
    if (threadIdx.x == NT - 1) gs[ngroups] = run + s;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int b = lo + j;
        if (j < per && b < nbins) {
            if (!(b & kGroupMask)) gs[b >> kGroupShift] = run;
            cursor[b] = run;
            run += v[j];
        }
    }
    __syncthreads();
    if ((int)threadIdx.x <= ngroups) gstart[threadIdx.x] = gs[threadIdx.x];
    if (threadIdx.x < 64)
        wave_prefix([&](int k) { return (gs[k + 1] - gs[k] + (uint32_t)kFineChunk - 1) / (uint32_t)kFineChunk; }, ngroups,
                    fitem);
}

// Exclusive scan, in place, of row[0 .. len-1] by one workgroup of 256 threads.
__device__ __forceinline__ void scan_row(uint32_t *row, int len)
{
    __shared__ uint32_t wsum[4];
    uint32_t carry = 0;
    for (int t0 = 0; t0 < len; t0 += 1024) {
        const int lo = t0 + 4 * (int)threadIdx.x;
        uint32_t v[4], s = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[j] = lo + j < len ? row[lo + j] : 0u;
            s += v[j];
        }
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        uint32_t incl = s;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off);
            if (lane >= off) incl += y;
        }
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        uint32_t run = carry + incl - s;
        for (int w = 0; w < wv; ++w) run += wsum[w];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (lo + j < len) {
                row[lo + j] = run;
                run += v[j];
            }
        carry += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
}

// The scans of one call: workgroup 0 scans the buckets (scan_buckets), and
// workgroup k + 1 scans row k of ccnt (nchunks long), which becomes the offset
// of each chunk's run within group k's region.
__global__ __launch_bounds__(256) void k_bin_scan(const uint32_t *totals, int nbins, uint32_t *cursor, uint32_t *gstart,
                                                  uint32_t *fitem, uint32_t *ccnt, int nchunks)
{
    if (blockIdx.x == 0)
        scan_buckets<256>(totals, nbins, 0u, cursor, gstart, fitem);
    else
        scan_row(ccnt + (size_t)(blockIdx.x - 1) * nchunks, nchunks);
}

// The common steps of both scatters, for one chunk of count <= NT * PER
// templates: element q of a thread (present when q*NT + threadIdx.x < count)
// has value kv[q] < 2^16 whose key is kv[q] >> shift (< nkeys <= kMaxGroups).
// Ranks the elements within their keys (kv[q] gets its rank in the high half),
// sets lst[k] = the first position of key k in the chunk ordered by key, and
// cnt[k] = start(k, c) for each key k present c times: the global start of the
// chunk's run of key k. Called by all NT threads; cnt is read back only after
// a later barrier.
template <int PER, typename StartF, int NT>
__device__ __forceinline__ void rank_chunk(uint32_t *cnt, uint32_t *lst, int nkeys, int count, uint32_t (&kv)[PER],
                                           int shift, StartF start)
{
    for (int b = threadIdx.x; b < nkeys; b += NT) cnt[b] = 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q)
        if (q * NT + (int)threadIdx.x < count) kv[q] |= atomicAdd(&cnt[kv[q] >> shift], 1u) << 16;
    __syncthreads();
    if (threadIdx.x < 64) wave_prefix([&](int k) { return cnt[k]; }, nkeys, lst);
    __syncthreads();
    static_assert(kMaxGroups <= 256, "one key per thread");
    if ((int)threadIdx.x < nkeys) {
        const uint32_t c = cnt[threadIdx.x];
        if (c) cnt[threadIdx.x] = start((int)threadIdx.x, c);
    }
}

// LDS of a first-scatter workgroup: the chunk ordered by group, each entry
// (position in the chunk << 16) | bucket.
struct GroupLds {
    uint32_t cnt[kGroupSlots];
    uint32_t lst[kGroupSlots];
    uint32_t sval[kBinChunk];
};

// LDS of a second-scatter workgroup: the chunk ordered by bucket (index and
// bucket within the group).
struct FineLds {
    uint32_t cnt[kGroupSlots];
    uint32_t lst[kGroupSlots];
    uint32_t sidx[kFineChunk];
    uint8_t skey[kFineChunk];
};

// First scatter of chunk c: templates base + j (j < count), buckets bins[base
// + j], to tmp at gstart[k] + crun[k * stride] (group k's region, this chunk's
// run in it) in the order of their ranks; the bucket within the group to tsub
// at the same position.
template <int NT>
__device__ __forceinline__ void group_chunk(GroupLds &L, int ngroups, int64_t base, int count, const uint16_t *bins,
                                            const uint32_t *gstart, const uint32_t *crun, size_t stride, uint32_t *tmp,
                                            uint8_t *tsub)
{
    constexpr int PER = kBinChunk / NT;
    uint32_t kv[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = q * NT + threadIdx.x;
        kv[q] = j < count ? bins[base + j] : 0u;
    }
    auto st = [&](int k, uint32_t) { return gstart[k] + crun[(size_t)k * stride]; };
    rank_chunk<PER, decltype(st), NT>(L.cnt, L.lst, ngroups, count, kv, kGroupShift, st);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = q * NT + threadIdx.x;
        if (j < count) {
            const uint32_t b = kv[q] & 0xffffu;
            L.sval[L.lst[b >> kGroupShift] + (kv[q] >> 16)] = ((uint32_t)j << 16) | b;
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < count; p += NT) {
        const uint32_t v = L.sval[p], b = v & 0xffffu, k = b >> kGroupShift;
        const uint32_t at = L.cnt[k] + ((uint32_t)p - L.lst[k]);
        tmp[at] = (uint32_t)(base + (v >> 16));
        tsub[at] = (uint8_t)(b & kGroupMask);
    }
}

// Second scatter of one chunk: entries src[j] (index) and ssub[j] (bucket
// within the group), j < count, to order at their bucket's cursor cur[sub].
template <int NT>
__device__ __forceinline__ void fine_chunk(FineLds &L, int nkeys, int count, const uint32_t *src, const uint8_t *ssub,
                                           uint32_t *cur, uint32_t *order)
{
    constexpr int PER = kFineChunk / NT;
    uint32_t idx[PER], kv[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = q * NT + threadIdx.x;
        idx[q] = j < count ? src[j] : 0u;
        kv[q] = j < count ? ssub[j] : 0u;
    }
    auto st = [&](int k, uint32_t c) { return atomicAdd(&cur[k], c); };
    rank_chunk<PER, decltype(st), NT>(L.cnt, L.lst, nkeys, count, kv, 0, st);
#pragma unroll
    for (int q = 0; q < PER; ++q)
        if (q * NT + (int)threadIdx.x < count) {
            const uint32_t k = kv[q] & 0xffffu, p = L.lst[k] + (kv[q] >> 16);
            L.sidx[p] = idx[q];
            L.skey[p] = (uint8_t)k;
        }
    __syncthreads();
    for (int p = threadIdx.x; p < count; p += NT) {
        const uint32_t k = L.skey[p];
        order[L.cnt[k] + ((uint32_t)p - L.lst[k])] = L.sidx[p];
    }
}

// First scatter: workgroup c takes the chunk of templates c * kBinChunk .. of
// the call (ccnt as scanned by k_bin_scan, row stride gridDim.x).
__global__ __launch_bounds__(kScatterWG) void k_bin_group(int64_t n, int ngroups, const uint16_t *bins, const uint32_t *gstart,
                                                   const uint32_t *ccnt, uint32_t *tmp, uint8_t *tsub)
{
    __shared__ GroupLds L;
    const int64_t base = (int64_t)blockIdx.x * kBinChunk;
    group_chunk<kScatterWG>(L, ngroups, base, (int)min<int64_t>(kBinChunk, n - base), bins, gstart, ccnt + blockIdx.x, gridDim.x,
                tmp, tsub);
}

// Second scatter: workgroup w takes chunk w - fitem[k] (of kFineChunk) of group
// k's region of tmp (fitem[k] <= w < fitem[k + 1]) to the group's buckets;
// workgroups from fitem[ngroups] on have nothing to do.
__global__ __launch_bounds__(kScatterWG) void k_bin_fine(int nbins, const uint32_t *gstart, const uint32_t *fitem,
                                                  uint32_t *cursor, const uint32_t *tmp, const uint8_t *tsub,
                                                  uint32_t *order)
{
    __shared__ FineLds L;
    const int ngroups = (nbins + kGroupMask) >> kGroupShift;
    const uint32_t w = blockIdx.x;
    if (w >= fitem[ngroups]) return;
    const int k = find_slot(fitem, ngroups, w);
    const uint32_t e0 = gstart[k] + (w - fitem[k]) * (uint32_t)kFineChunk;
    const int b0 = k << kGroupShift;
    fine_chunk<kScatterWG>(L, min(1 << kGroupShift, nbins - b0), (int)min<uint32_t>(kFineChunk, gstart[k + 1] - e0), tmp + e0,
               tsub + e0, cursor + b0, order);
}

// One LDS-DMA copy of 16 bytes per lane: lane i's 16 bytes at src land at
// lds_dst + 16 i (lds_dst wave-uniform). Written as inline assembly so that the
// compiler does not tie it to the LDS reads of the other slab buffer: its
// wait-count pass cannot tell the two buffers apart and would stall each
// wave's first read of a slab until its prefetch of the next slab had landed.
// The caller waits for the copies itself (a full s_waitcnt and a barrier
// before a buffer is read). A copy the compiler does not count can only make
// its own memory waits stricter (vector memory counters drain in order).
__device__ __forceinline__ void lds_dma_16(const float2 *src, float2 *lds_dst)
{
    const uint32_t m0 = __builtin_amdgcn_readfirstlane(
        (uint32_t)(uintptr_t)(__attribute__((address_space(3))) float2 *)lds_dst);
    asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" : : "v"(src), "s"(m0) : "memory", "m0");
}

// ---------------------------------------------------------------- time-slab scorer
// One workgroup = WG lanes x TPT templates taken consecutively from the binned
// order; wave w owns the 64*TPT consecutive entries starting at w*64*TPT, so a
// wave's templates start and end in nearly the same columns. The workgroup
// sweeps the union of its waves' column ranges in slabs of S columns: all lanes
// stage a slab (F rows x S columns of p = Y/sigma, 8 B per pixel) into LDS with
// coalesced loads, then each wave walks its own column range through the slab.
// Every template's DDA is started at its wave's first column (rewound when the
// template starts later), so all lanes step together: no divergent branches in
// the inner loop, the pixels outside a template are masked by a select and
// their LDS address clamped into the column. Per-template partial sums are FP32
// between flush columns and FP64 across them.

// Walk columns ca..cb of the current slab (column c0 at slab[0]) for the TPT
// templates of this lane. MASK = false is the wave's core, where every
// template of the wave covers every column: no select and no clamp.
template <int TPT, bool MASK, bool HW, int MAPT>
__device__ __forceinline__ void walk(int ca, int cb, int c0, const elem_t<MAPT> *slab, int ldc, const int32_t (&t0)[TPT],
                                     const uint32_t (&span)[TPT], const PhaseK (&pk)[TPT], DdaF (&st)[TPT],
                                     float (&part)[TPT], double (&acc)[TPT])
{
    // segments end at the flush columns (c = 15 mod 16), so the inner loop has no flush test
    for (int c = ca; c <= cb;) {
        const int ce = min(cb, c | (kFlush - 1));
        for (; c <= ce; ++c) {
            const elem_t<MAPT> *col = slab + (c - c0) * ldc;
#pragma unroll
            for (int q = 0; q < TPT; ++q) {
                const int32_t row = ddaf_row(st[q]);
                if (MASK) {
                    const bool act = (uint32_t)c - (uint32_t)t0[q] <= span[q];
                    const float v = add_term_m<HW, MAPT>(part[q], pk[q], row, col[act ? row : 0]);
                    part[q] = act ? v : part[q];
                } else {
                    part[q] = add_term_m<HW, MAPT>(part[q], pk[q], row, col[row]);
                }
                ddaf_step(st[q]);
            }
        }
        if ((ce & (kFlush - 1)) == kFlush - 1) {  // wave-uniform
#pragma unroll
            for (int q = 0; q < TPT; ++q) {
                acc[q] += part[q];
                part[q] = 0.0f;
            }
        }
    }
}

// Walk of one aligned slab of SC columns c0 .. c0 + SC - 1 (c0 a multiple of
// SC, SC a divisor of kFlush) at slab[0 .. SC*ldc): straight-line code, SC
// columns x TPT templates. MASK = false when every template of the wave covers
// every column of the slab.
template <int SC, int TPT, bool MASK, bool HW, int SM>
__device__ __forceinline__ void walk_slab(int c0, const elem_t<SM> *slab, int ldc, const int32_t (&t0)[TPT],
                                          const uint32_t (&span)[TPT], const PhaseK (&pk)[TPT], DdaF (&st)[TPT],
                                          float (&part)[TPT])
{
#pragma unroll
    for (int j = 0; j < SC; ++j) {
        const elem_t<SM> *col = slab + j * ldc;
#pragma unroll
        for (int q = 0; q < TPT; ++q) {
            const int32_t row = ddaf_row(st[q]);
            if (MASK) {
                const bool act = (uint32_t)(c0 + j) - (uint32_t)t0[q] <= span[q];
                const float v = add_term_m<HW, SM>(part[q], pk[q], row, col[act ? row : 0]);
                part[q] = act ? v : part[q];
            } else {
                part[q] = add_term_m<HW, SM>(part[q], pk[q], row, col[row]);
            }
            ddaf_step(st[q]);
        }
    }
}

// One block of WG*TPT consecutive entries of `order` (block index b): the
// whole slab sweep for those templates. slab is the dynamic LDS, bnd two LDS
// ints. Callable repeatedly by a persistent workgroup. Templates are drawn
// (tr == NULL) or read from tr and validated.
// SC > 0: a folded map (kMapPol: 8 bytes per pixel, kMapPolH: 4 bytes; columns
// padded to whole 1 KB pieces) is staged with LDS DMA into two slab buffers of
// SC columns (double buffering: slab k+1 streams in while slab k is walked).
// Slabs are aligned to multiples of SC on the absolute column grid, so the FP32
// partial sums are flushed between slabs and a slab is one straight-line
// walk_slab; each wave starts its rows at its first aligned column (columns
// before a template's start and after its end are masked, so the extra columns
// change nothing). SC = 0: the lanes stage S columns through registers into one
// buffer (unfolded formats are converted to Cartesian p on the way; a folded
// map is copied as it is) and walk them column by column.
template <int WG, int TPT, bool HW, int MAPT, int SC>
__device__ __forceinline__ uint64_t score_block(const MapP &m, const GenP &g, const Trk *tr, const uint32_t *order,
                                                uint64_t first, int64_t n, int64_t b, int S, int32_t norm, float *snr,
                                                float2 *slab_raw, int *bnd, uint64_t *kred)
{
    // element format of the slab: the map's own for the folded formats, p in Cartesian form otherwise
    constexpr int SM = (MAPT == kMapPol || MAPT == kMapPolH) ? MAPT : kMapPF;
    using E = elem_t<SM>;
    __syncthreads();  // LDS of a previous block is no longer read
    if (threadIdx.x == 0) { bnd[0] = 0x7fffffff; bnd[1] = -1; }

    const int lane = threadIdx.x & 63;
    const int64_t wbase = b * (WG * TPT) + (int64_t)(threadIdx.x >> 6) * (64 * TPT);
    const bool expl = tr != nullptr;
    Trk tk[TPT];
    int32_t t0[TPT];
    uint32_t span[TPT], idx[TPT];
    PhaseK pk[TPT];
    bool ok[TPT], live[TPT];
    int lo = 0x7fffffff, hi = -1;        // union of this wave's templates
    int clo = -1, chi = 0x7fffffff;      // intersection (the core)
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
        const int64_t e = wbase + q * 64 + lane;
        live[q] = e < n;
        idx[q] = live[q] ? order[e] : 0u;
        Trk t = expl ? tr[idx[q]] : draw_track(g, first + idx[q]);
        ok[q] = live[q] && (!expl || track_ok(t, m));
        if (!ok[q]) t = Trk{0, 1, 0u, 0u, 0u, 0};  // never active: (c - t0) > span below
        tk[q] = t;
        t0[q] = ok[q] ? t.t0 : 0x7fffffff;
        span[q] = ok[q] ? (uint32_t)(t.t2 - t.t0) : 0u;
        pk[q] = phase_k(m, t.dtau);
        if (ok[q]) {
            lo = min(lo, t.t0);
            hi = max(hi, t.t2);
            clo = max(clo, t.t0);
            chi = min(chi, t.t2);
        } else {
            clo = 0x7fffffff;  // a lane without a template: no unmasked core for this wave
            chi = -1;
        }
    }
    lo = wave_min_i32(lo);
    hi = wave_max_i32(hi);
    clo = wave_max_i32(clo);
    chi = wave_min_i32(chi);
    if (clo > chi) {  // empty core: everything goes through the masked walk
        clo = hi + 1;
        chi = hi;
    }
    DdaF st[TPT];
    float part[TPT];
    double acc[TPT];
    // the rows start at the wave's first column (aligned down to a slab boundary when slabs are)
    const int start = lo == 0x7fffffff ? 0 : (SC > 0 ? lo & ~(SC - 1) : lo);
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
        st[q] = ddaf_init_at(tk[q], start - tk[q].t0);
        part[q] = 0.0f;
        acc[q] = 0.0;
    }
    __syncthreads();
    if (lane == 0) {
        atomicMin(&bnd[0], lo);
        atomicMax(&bnd[1], hi);
    }
    __syncthreads();
    const int c_first = __builtin_amdgcn_readfirstlane(bnd[0]), c_last = __builtin_amdgcn_readfirstlane(bnd[1]);
    const int F = m.F;

    if constexpr (SC > 0) {
        static_assert(kFlush % SC == 0, "slabs must tile the flush grid");
        // m.ld is a whole number of 1 KB pieces and the columns are contiguous, so
        // the slab of columns c0.. is one run of pieces, piece ch at byte offset
        // 1024 ch in the map and in the buffer (counted below in 8-byte units).
        const int ldc = (int)m.ld;
        const int col8 = ldc * (int)sizeof(E) / 8, per_col = col8 / (kDmaBytes / 8);
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        auto issue = [&](int c0, int bsel) {
            const int nchunk = min(SC, c_last - c0 + 1) * per_col;
            const float2 *src = m.Y + (int64_t)c0 * col8 + lane * 2;
            float2 *dst = slab_raw + (size_t)bsel * SC * col8;
            for (int ch = wave; ch < nchunk; ch += WG / 64)
                lds_dma_16(src + ch * (kDmaBytes / 8), dst + ch * (kDmaBytes / 8));
        };
        const int a_first = c_first & ~(SC - 1);
        // this wave's slabs: from its aligned first column to its last; the core slabs lie in [clo, chi]
        const int w_lo = start, w_hi = hi;
        if (c_first <= c_last) issue(a_first, 0);
        int k = 0;
        for (int c0 = a_first; c0 <= c_last; c0 += SC, ++k) {
            __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of slab k have landed
            __syncthreads();                // so have everyone's, and slab k-1 is no longer read
            if (c0 + SC <= c_last) issue(c0 + SC, (k + 1) & 1);
            if (c0 < w_lo || c0 > w_hi) continue;  // wave-uniform
            const E *cur = reinterpret_cast<const E *>(slab_raw + (size_t)(k & 1) * SC * col8);
            if (c0 >= clo && c0 + SC - 1 <= chi)
                walk_slab<SC, TPT, false, HW, SM>(c0, cur, ldc, t0, span, pk, st, part);
            else
                walk_slab<SC, TPT, true, HW, SM>(c0, cur, ldc, t0, span, pk, st, part);
            if (((c0 + SC) & (kFlush - 1)) == 0) {  // wave-uniform: the slab ends a flush group
#pragma unroll
                for (int q = 0; q < TPT; ++q) {
                    acc[q] += part[q];
                    part[q] = 0.0f;
                }
            }
        }
    } else {
        E *slab = reinterpret_cast<E *>(slab_raw);
        // staging walk: element e = tid + i*WG of the slab is (column e / F, row e % F)
        const int dcol = WG / F, drow = WG % F;
        const int col0 = threadIdx.x / F, row0 = threadIdx.x % F;
        for (int c0 = c_first; c0 <= c_last; c0 += S) {
            const int ncol = min(S, c_last - c0 + 1);
            __syncthreads();  // the previous slab has been consumed
            {
                int col = col0, r = row0;
                const int64_t base = (int64_t)c0 * m.ld;
#pragma unroll 4
                for (int e = threadIdx.x; e < ncol * F; e += WG) {
                    slab[col * F + r] = load_e<MAPT>(m, base + (int64_t)col * m.ld + r);
                    r += drow;
                    col += dcol;
                    if (r >= F) { r -= F; ++col; }
                }
            }
            __syncthreads();
            const int ca = max(c0, lo), cb = min(c0 + ncol - 1, hi);  // this wave's columns in the slab
            walk<TPT, true, HW, SM>(ca, min(cb, clo - 1), c0, slab, F, t0, span, pk, st, part, acc);
            walk<TPT, false, HW, SM>(max(ca, clo), min(cb, chi), c0, slab, F, t0, span, pk, st, part, acc);
            walk<TPT, true, HW, SM>(max(ca, chi + 1), cb, c0, slab, F, t0, span, pk, st, part, acc);
        }
    }

    uint64_t key = 0;
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
        if (!live[q]) continue;
        const float z = ok[q] ? finish(acc[q] + part[q], (int32_t)span[q] + 1, norm, m.scale) : __builtin_nanf("");
        if (snr) snr[idx[q]] = z;
        const uint64_t k = key_encode(z, (uint32_t)(first + idx[q]));
        key = k > key ? k : key;
    }
    // the block's best key: waves by shuffles, then across waves through LDS
    key = wave_max_u64(key);
    if (lane == 0) kred[threadIdx.x >> 6] = key;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < WG / 64; ++w) key = kred[w] > key ? kred[w] : key;
    return key;  // valid in thread 0
}

// One block of binned templates per workgroup. Each workgroup stores its best
// key in its own slot of wg_keys (no atomics: many same-address atomics from
// every wave serialise across the chip); k_reduce_keys folds the slots.
// At least 4 waves per SIMD (at most 128 VGPRs), so that two workgroups of 512 lanes, or four of
// 256, can share a CU when their slabs fit its LDS.
constexpr int kSlabWavesPerSimd = 4;

template <int WG, int TPT, bool HW, int MAPT, int SC>
__global__ __launch_bounds__(WG, kSlabWavesPerSimd) void k_score_slab(MapP m, GenP g, const Trk *tr,
                                                                      const uint32_t *order, uint64_t first,
                                                                      int64_t n, int S, int32_t norm, float *snr,
                                                                      uint64_t *wg_keys)
{
    extern __shared__ float2 slab[];
    __shared__ int bnd[2];
    __shared__ uint64_t kred[WG / 64];
    const uint64_t key = score_block<WG, TPT, HW, MAPT, SC>(m, g, tr, order, first, n, (int64_t)blockIdx.x, S, norm,
                                                            snr, slab, bnd, kred);
    if (threadIdx.x == 0) wg_keys[blockIdx.x] = key;
}

// Max of n keys into *best (max-merged with what it holds), in one workgroup.
__global__ __launch_bounds__(1024) void k_reduce_keys(const uint64_t *keys, int64_t n, uint64_t *best)
{
    __shared__ uint64_t kred[16];
    uint64_t key = 0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) key = keys[i] > key ? keys[i] : key;
    key = wave_max_u64(key);
    if ((threadIdx.x & 63) == 0) kred[threadIdx.x >> 6] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 16; ++w) key = kred[w] > key ? kred[w] : key;
        if (key) atomicMax((unsigned long long *)best, (unsigned long long)key);
    }
}

// ---------------------------------------------------------------- templates with a free t_mid
// A free-t_mid template's rows have no recurrence: each column's row is an
// independent root (row_tm). Both scorers below walk a template's columns on
// the flush grid of the plain scorers (FP32 partial sums per group of kFlush
// aligned columns, FP64 across groups in column order), so they give the same
// bits: k_score_tm_slab (binned templates, LDS slabs, like k_score_md_slab) for
// generated templates, k_score_tm (one wave per template, lanes over groups,
// like k_score_wave) for small calls and given lists.

__device__ __forceinline__ bool track_tm_ok(const TrkTm &t, const MapP &m)
{
    const uint32_t lim = (uint32_t)m.F << 8;
    return t.t0 >= 0 && t.t0 < t.t2 && t.t2 < m.T && t.t1 >= t.t0 && t.t1 <= t.t2 && t.f0 < lim && t.f1 < lim &&
           t.f2 < lim;
}

__global__ __launch_bounds__(256) void k_make_tracks_tm(GenP g, uint64_t first, int64_t n, TrkTm *out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = draw_track_tm(g, first + (uint64_t)i);
}

template <bool EXPL, bool HW, int MAPT>
__global__ __launch_bounds__(256) void k_score_tm(MapP m, GenP g, const TrkTm *tr, uint64_t first, int64_t n,
                                                  int32_t norm, float *snr, uint64_t *best)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);  // wave-uniform
    uint64_t key = 0;
    if (i < n) {
        const TrkTm t = EXPL ? tr[i] : draw_track_tm(g, first + (uint64_t)i);
        float z = __builtin_nanf("");
        if (!EXPL || track_tm_ok(t, m)) {
            const RowTm k = row_tm_init(t);
            const PhaseK pk = phase_k(m, t.dtau);
            const int gfirst = t.t0 / kFlush, glast = t.t2 / kFlush;
            float gp[kWaveRounds];
#pragma unroll
            for (int r = 0; r < kWaveRounds; ++r) {
                gp[r] = 0.0f;
                const int gi = gfirst + r * 64 + lane;
                if (gi > glast) continue;
                const int ca = max(t.t0, gi * kFlush), cb = min(t.t2, gi * kFlush + kFlush - 1);
                float part = 0.0f;
                for (int c = ca; c <= cb; ++c) {
                    const int32_t row = row_tm(k, c - t.t0);
                    part = add_term_m<HW, MAPT>(part, pk, row, load_e<MAPT>(m, (int64_t)c * m.ld + row));
                }
                gp[r] = part;
            }
            const int ng = glast - gfirst + 1;
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < kWaveRounds; ++r) {
                const int cnt = min(64, ng - r * 64);
                for (int l = 0; l < cnt; ++l)
                    acc += __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, gp[r]), l));
            }
            if ((t.t2 & (kFlush - 1)) == kFlush - 1) acc = acc + 0.0f;
            z = finish(acc, t.t2 - t.t0 + 1, norm, m.scale);
        }
        if (lane == 0 && snr) snr[i] = z;
        key = key_encode(z, (uint32_t)(first + (uint64_t)i));
    }
    merge_key(best, key);
}

// Column walk of the free-t_mid slab scorer (as walk, with an independent row per column). The
// FP32 pass takes every template's row of the column, with D = b^2 + 4 a dt and 2 dt carried from
// column to column by one add each; where it does not stand for some lane (about one template
// pixel in a thousand on the search band), the whole wave takes one uniform branch in which those
// lanes settle their rows exactly. A lane outside its template's columns works on column t0 + 1
// (valid for every template) and drops the term.
// Column walk of the free-t_mid slab scorer (as walk, with an independent row per column). The
// FP32 pass takes every template's row of the column, with D = b^2 + 4 a dt and 2 dt carried from
// column to column by one add each (Dc, dt2c: their values at column ca, advanced past cb on
// return, so that the wave's walks over consecutive column ranges carry them through); where it
// does not stand for some lane (about one template pixel in a thousand on the search band), the
// whole wave takes one uniform branch in which those lanes settle their rows exactly. A lane
// outside its template's columns works on column t0 + 1 (valid for every template) and drops the
// term.
template <int TPT, bool MASK, bool HW, typename E>
__device__ __forceinline__ void walk_tm(int ca, int cb, int c0, const E *slab, int ldc, const int32_t (&t0)[TPT],
                                        const uint32_t (&span)[TPT], const RowTm (&rk)[TPT],
                                        const PhaseK (&pk)[TPT], int32_t (&Dc)[TPT], float (&dt2c)[TPT],
                                        float (&part)[TPT], double (&acc)[TPT])
{
    for (int c = ca; c <= cb;) {
        const int ce = min(cb, c | (kFlush - 1));
        for (; c <= ce; ++c) {
            int32_t row[TPT];
            bool act[TPT], ok[TPT];
            bool redo = false;
#pragma unroll
            for (int q = 0; q < TPT; ++q) {
                act[q] = !MASK || (uint32_t)(c - t0[q]) <= span[q];
                const int32_t D = act[q] ? Dc[q] : rk[q].bb + rk[q].a4;
                row[q] = row_tm_fp32_d(rk[q], D, act[q] ? dt2c[q] : 2.0f, ok[q]);
                ok[q] = ok[q] || !act[q];
                redo = redo || !ok[q];
                Dc[q] = (int32_t)((uint32_t)Dc[q] + (uint32_t)rk[q].a4);
                dt2c[q] += 2.0f;
            }
            if (__builtin_amdgcn_ballot_w64(redo)) {  // wave-uniform
                // the column through readfirstlane: no induction variables for this rare branch
                // are kept up to date in the loop
                const int cu = __builtin_amdgcn_readfirstlane(c);
#pragma unroll
                for (int q = 0; q < TPT; ++q)
                    if (!ok[q]) row[q] = row_tm_fallback(rk[q], cu - t0[q]);
            }
            const E *col = slab + (c - c0) * ldc;
#pragma unroll
            for (int q = 0; q < TPT; ++q) {
                const int32_t r = MASK && !act[q] ? 0 : row[q];
                const float v = add_term_pol<HW>(part[q], pk[q], r, col[r]);
                part[q] = act[q] ? v : part[q];
            }
        }
        if ((ce & (kFlush - 1)) == kFlush - 1) {  // wave-uniform
#pragma unroll
            for (int q = 0; q < TPT; ++q) {
                acc[q] += part[q];
                part[q] = 0.0f;
            }
        }
    }
}

// With one template per lane the scorer fits 64 VGPRs, so that 8 waves share each SIMD (two
// workgroups of 1024 lanes per CU with 80 KB of slabs each): the more waves, the more of the
// latency of the root's square root and reciprocal and of the LDS gathers is hidden.
template <int WG, int TPT, bool HW, int MAPT>
__global__ __launch_bounds__(WG, TPT == 1 ? 8 : 1) void k_score_tm_slab(MapP m, GenP g, const uint32_t *order,
                                                                         uint64_t first, int64_t n, int S, int32_t norm,
                                                                         float *snr, uint64_t *wg_keys)
{
    extern __shared__ float2 slab[];
    __shared__ int bnd[2];
    __shared__ uint64_t kred[WG / 64];
    if (threadIdx.x == 0) { bnd[0] = 0x7fffffff; bnd[1] = -1; }
    const int lane = threadIdx.x & 63;
    const int64_t wbase = (int64_t)blockIdx.x * (WG * TPT) + (int64_t)(threadIdx.x >> 6) * (64 * TPT);
    int32_t t0[TPT];
    uint32_t span[TPT], idx[TPT];
    bool live[TPT];
    RowTm rk[TPT];
    PhaseK pk[TPT];
    int lo = 0x7fffffff, hi = -1, clo = -1, chi = 0x7fffffff;
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
        const int64_t e = wbase + q * 64 + lane;
        live[q] = e < n;
        idx[q] = live[q] ? order[e] : 0u;
        TrkTm t = draw_track_tm(g, first + idx[q]);
        if (!live[q]) t = TrkTm{0, 0, 1, 0u, 0u, 0u, 0};  // never active: (c - t0) > span below
        rk[q] = row_tm_init(t);
        pk[q] = phase_k(m, t.dtau);
        t0[q] = live[q] ? t.t0 : 0x7fffffff;
        span[q] = live[q] ? (uint32_t)(t.t2 - t.t0) : 0u;
        if (live[q]) {
            lo = min(lo, t.t0);
            hi = max(hi, t.t2);
            clo = max(clo, t.t0);
            chi = min(chi, t.t2);
        } else {
            clo = 0x7fffffff;
            chi = -1;
        }
    }
    lo = wave_min_i32(lo);
    hi = wave_max_i32(hi);
    clo = wave_max_i32(clo);
    chi = wave_min_i32(chi);
    if (clo > chi) { clo = hi + 1; chi = hi; }
    float part[TPT];
    double acc[TPT];
    // D and 2 dt at the wave's first column; the walks then carry them column by column. Modulo
    // 2^32: a lane that holds no template (t0 = INT_MAX) only ever takes the masked walk.
    int32_t Dc[TPT];
    float dt2c[TPT];
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
        part[q] = 0.0f;
        acc[q] = 0.0;
        const uint32_t dt = (uint32_t)lo - (uint32_t)t0[q];
        Dc[q] = (int32_t)((uint32_t)rk[q].bb + (uint32_t)rk[q].a4 * dt);
        dt2c[q] = 2.0f * (float)(int32_t)dt;
    }
    __syncthreads();
    if (lane == 0) {
        atomicMin(&bnd[0], lo);
        atomicMax(&bnd[1], hi);
    }
    __syncthreads();
    const int c_first = __builtin_amdgcn_readfirstlane(bnd[0]), c_last = __builtin_amdgcn_readfirstlane(bnd[1]);
    using E = elem_t<MAPT>;
    const int ldc = (int)m.ld;
    const int col8 = ldc * (int)sizeof(E) / 8, per_col = col8 / (kDmaBytes / 8);  // 8-byte units per column
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    auto issue = [&](int c0, int bsel) {
        const int nchunk = min(S, c_last - c0 + 1) * per_col;
        const float2 *src = m.Y + (int64_t)c0 * col8 + lane * 2;
        float2 *dst = slab + (size_t)bsel * S * col8;
        for (int ch = wave; ch < nchunk; ch += WG / 64)
            lds_dma_16(src + ch * (kDmaBytes / 8), dst + ch * (kDmaBytes / 8));
    };
    if (c_first <= c_last) issue(c_first, 0);
    int kk = 0;
    for (int c0 = c_first; c0 <= c_last; c0 += S, ++kk) {
        __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of slab kk have landed
        __syncthreads();                // so have everyone's, and slab kk-1 is no longer read
        if (c0 + S <= c_last) issue(c0 + S, (kk + 1) & 1);
        const E *cur = reinterpret_cast<const E *>(slab + (size_t)(kk & 1) * S * col8);
        const int ncol = min(S, c_last - c0 + 1);
        const int ca = max(c0, lo), cb = min(c0 + ncol - 1, hi);
        walk_tm<TPT, true, HW>(ca, min(cb, clo - 1), c0, cur, ldc, t0, span, rk, pk, Dc, dt2c, part, acc);
        walk_tm<TPT, false, HW>(max(ca, clo), min(cb, chi), c0, cur, ldc, t0, span, rk, pk, Dc, dt2c, part, acc);
        walk_tm<TPT, true, HW>(max(ca, chi + 1), cb, c0, cur, ldc, t0, span, rk, pk, Dc, dt2c, part, acc);
    }
    uint64_t key = 0;
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
        if (!live[q]) continue;
        const float z = finish(acc[q] + part[q], (int32_t)span[q] + 1, norm, m.scale);
        if (snr) snr[idx[q]] = z;
        const uint64_t k = key_encode(z, (uint32_t)(first + idx[q]));
        key = k > key ? k : key;
    }
    key = wave_max_u64(key);
    if (lane == 0) kred[threadIdx.x >> 6] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < WG / 64; ++w) key = kred[w] > key ? kred[w] : key;
        wg_keys[blockIdx.x] = key;
    }
}

// ---------------------------------------------------------------- delay-maximised scoring
// The maximum of Eq. 8 over a grid of delays per template (a reading of
// "phase-maximised"): the template keeps its geometry and its own delay is
// replaced by dtau_m = d0 + m * step. A launch handles kMD consecutive delays
// m0 .. m0 + cnt - 1 of the grid for every template: the row walk and the
// pixel gather are shared, each delay has its own (wave-uniform) phase
// constants and accumulators, on the same flush grid as the other scorers.
// The running maximum and its index live in snr / tidx between launches.
constexpr int kMD = 8;

// The grid is uniform, so at row r the phase of delay k of a launch is
// phase_0(r) + k * dphase(r) (32-bit, exact). The map is in polar form, so the
// term of delay k is |p| cos(theta_k) with theta_k = 2 pi (phase_k + arg p):
// the first delay's term is the plain scorer's (add_term_pol, the same bits),
// and each further (cos, sin) theta_k is the previous one rotated by
// exp(2 pi i dphase(r)), one complex multiply (at most kMD - 1 = 7 in a row, a
// few 1e-7 relative).
struct DelayGrid {
    PhaseK k0;       // phase constants of the launch's first delay
    PhaseK dk;       // phase constants of the grid step
    int32_t m0, cnt;
};

__device__ __forceinline__ DelayGrid delay_grid(const MapP &m, int32_t d0, int32_t step, int32_t m0, int32_t cnt)
{
    DelayGrid dg;
    dg.m0 = m0;
    dg.cnt = cnt;
    const int32_t d = (int32_t)((uint32_t)d0 + (uint32_t)m0 * (uint32_t)step);  // in range (checked by the host)
    dg.k0 = phase_k(m, d);
    dg.dk = phase_k(m, step);
    return dg;
}

// Adds the template's Eq. 8 terms at `row` for all kMD delays of the launch.
template <bool HW, bool MASK, typename E>
__device__ __forceinline__ void add_terms_md(float (&part)[kMD], const DelayGrid &dg, int32_t row, E pp, bool act)
{
    const float v0 = add_term_pol<HW>(part[0], dg.k0, row, pp);
    part[0] = !MASK || act ? v0 : part[0];
    const uint32_t arg = pol_arg(pp);
    const float mag = pol_mag(pp);
    float c, s, cr, sr;
    if constexpr (HW) {
        const float x0 = phase_turns(dg.k0.pa + arg, dg.k0.pb, row), xr = phase_turns(dg.dk.pa, dg.dk.pb, row);
        c = __builtin_amdgcn_cosf(x0);
        s = __builtin_amdgcn_sinf(x0);
        cr = __builtin_amdgcn_cosf(xr);
        sr = __builtin_amdgcn_sinf(xr);
    } else {
        const uint32_t ph0 = dg.k0.pa + arg + (uint32_t)row * dg.k0.pb, phr = dg.dk.pa + (uint32_t)row * dg.dk.pb;
        c = rot_re(ph0, 1.0f, 0.0f);
        s = rot_re(ph0 - 0x40000000u, 1.0f, 0.0f);  // cos(x - pi/2) = sin x
        cr = rot_re(phr, 1.0f, 0.0f);
        sr = rot_re(phr - 0x40000000u, 1.0f, 0.0f);
    }
#pragma unroll
    for (int k = 1; k < kMD; ++k) {
        const float cn = fmaf(c, cr, -s * sr), sn = fmaf(s, cr, c * sr);
        c = cn;
        s = sn;
        const float v = fmaf(c, mag, part[k]);
        part[k] = !MASK || act ? v : part[k];
    }
}

// The best of this launch's delays for one template, merged with the running
// maximum of earlier launches (strictly greater wins, so ties keep the lowest
// index). A NaN score (from NaN map data) makes the result NaN with index -1.
__device__ __forceinline__ void merge_delays(const double (&acc)[kMD], const float (&part)[kMD], int32_t N,
                                             int32_t norm, float scale, const DelayGrid &dg, bool ok, float &z,
                                             int32_t &mi)
{
    z = __builtin_nanf("");
    mi = -1;
    if (!ok) return;
    bool nan = false;
#pragma unroll
    for (int k = 0; k < kMD; ++k) {
        if (k >= dg.cnt) break;
        const float v = finish(acc[k] + part[k], N, norm, scale);
        if (v != v) nan = true;
        else if (mi < 0 || v > z) { z = v; mi = dg.m0 + k; }
    }
    if (nan) { z = __builtin_nanf(""); mi = -1; }
}

__device__ __forceinline__ void merge_running(float &z, int32_t &mi, float zp, int32_t mp, bool first_launch)
{
    if (first_launch) return;
    if (zp != zp || mp < 0 || z != z) { z = __builtin_nanf(""); mi = -1; return; }
    if (!(z > zp)) { z = zp; mi = mp; }
}

// One lane per template, direct gathers (small calls, maps too wide for LDS).
template <bool EXPL, bool HW, int MAPT>
__global__ __launch_bounds__(kWG) void k_score_md_direct(MapP m, GenP g, const Trk *tr, uint64_t first, int64_t n,
                                                         int32_t norm, int32_t d0, int32_t step, int32_t m0,
                                                         int32_t cnt, int32_t last, float *snr, int32_t *tidx,
                                                         uint64_t *best)
{
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    const DelayGrid dg = delay_grid(m, d0, step, m0, cnt);
    uint64_t key = 0;
    if (i < n) {
        const Trk t = EXPL ? tr[i] : draw_track(g, first + (uint64_t)i);
        const bool ok = !EXPL || track_ok(t, m);
        double acc[kMD];
        float part[kMD];
#pragma unroll
        for (int k = 0; k < kMD; ++k) { acc[k] = 0.0; part[k] = 0.0f; }
        const int32_t N = t.t2 - t.t0 + 1;
        if (ok) {
            DdaF s = ddaf_init_at(t, 0);
            int64_t base = (int64_t)t.t0 * m.ld;
            for (int32_t k = 0; k < N; ++k) {
                const int32_t row = ddaf_row(s);
                const elem_t<MAPT> p = load_e<MAPT>(m, base + row);
                add_terms_md<HW, false>(part, dg, row, p, true);
                if (((t.t0 + k) & (kFlush - 1)) == kFlush - 1) {
#pragma unroll
                    for (int q = 0; q < kMD; ++q) { acc[q] += part[q]; part[q] = 0.0f; }
                }
                ddaf_step(s);
                base += m.ld;
            }
        }
        float z;
        int32_t mi;
        merge_delays(acc, part, N, norm, m.scale, dg, ok, z, mi);
        merge_running(z, mi, m0 ? snr[i] : 0.0f, m0 ? tidx[i] : 0, m0 == 0);
        snr[i] = z;
        tidx[i] = mi;
        if (last) key = key_encode(z, (uint32_t)(first + (uint64_t)i));
    }
    if (last) merge_key(best, key);
}

// Column walk of the delay-maximised slab scorer (as walk, with kMD delays).
template <int TPT, bool MASK, bool HW, typename E>
__device__ __forceinline__ void walk_md(int ca, int cb, int c0, const E *slab, int ldc,
                                        const int32_t (&t0)[TPT], const uint32_t (&span)[TPT], const DelayGrid &dg,
                                        DdaF (&st)[TPT], float (&part)[TPT][kMD], double (&acc)[TPT][kMD])
{
    for (int c = ca; c <= cb;) {
        const int ce = min(cb, c | (kFlush - 1));
        for (; c <= ce; ++c) {
            const E *col = slab + (c - c0) * ldc;
#pragma unroll
            for (int q = 0; q < TPT; ++q) {
                const int32_t row = ddaf_row(st[q]);
                const bool act = !MASK || (uint32_t)c - (uint32_t)t0[q] <= span[q];
                const E p = col[act ? row : 0];
                add_terms_md<HW, MASK>(part[q], dg, row, p, act);
                ddaf_step(st[q]);
            }
        }
        if ((ce & (kFlush - 1)) == kFlush - 1) {  // wave-uniform
#pragma unroll
            for (int q = 0; q < TPT; ++q)
#pragma unroll
                for (int k = 0; k < kMD; ++k) { acc[q][k] += part[q][k]; part[q][k] = 0.0f; }
        }
    }
}

// Slab scorer of the delay grid: the folded map streamed into LDS by DMA as in
// score_block, WG lanes x TPT binned templates per workgroup; on the last launch
// each workgroup stores its best key in wg_keys[blockIdx.x].
template <int WG, int TPT, bool EXPL, bool HW, int MAPT>
__global__ __launch_bounds__(WG) void k_score_md_slab(MapP m, GenP g, const Trk *tr, const uint32_t *order,
                                                      uint64_t first, int64_t n, int S, int32_t norm, int32_t d0,
                                                      int32_t step, int32_t m0, int32_t cnt, int32_t last, float *snr,
                                                      int32_t *tidx, uint64_t *wg_keys)
{
    extern __shared__ float2 slab[];
    __shared__ int bnd[2];
    __shared__ uint64_t kred[WG / 64];
    if (threadIdx.x == 0) { bnd[0] = 0x7fffffff; bnd[1] = -1; }
    const DelayGrid dg = delay_grid(m, d0, step, m0, cnt);
    const int lane = threadIdx.x & 63;
    const int64_t wbase = (int64_t)blockIdx.x * (WG * TPT) + (int64_t)(threadIdx.x >> 6) * (64 * TPT);
    Trk tk[TPT];
    int32_t t0[TPT];
    uint32_t span[TPT], idx[TPT];
    bool ok[TPT], live[TPT];
    int lo = 0x7fffffff, hi = -1, clo = -1, chi = 0x7fffffff;
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
        const int64_t e = wbase + q * 64 + lane;
        live[q] = e < n;
        idx[q] = live[q] ? order[e] : 0u;
        Trk t = EXPL ? tr[idx[q]] : draw_track(g, first + idx[q]);
        ok[q] = live[q] && (!EXPL || track_ok(t, m));
        if (!ok[q]) t = Trk{0, 1, 0u, 0u, 0u, 0};
        tk[q] = t;
        t0[q] = ok[q] ? t.t0 : 0x7fffffff;
        span[q] = ok[q] ? (uint32_t)(t.t2 - t.t0) : 0u;
        if (ok[q]) {
            lo = min(lo, t.t0);
            hi = max(hi, t.t2);
            clo = max(clo, t.t0);
            chi = min(chi, t.t2);
        } else {
            clo = 0x7fffffff;
            chi = -1;
        }
    }
    lo = wave_min_i32(lo);
    hi = wave_max_i32(hi);
    clo = wave_max_i32(clo);
    chi = wave_min_i32(chi);
    if (clo > chi) { clo = hi + 1; chi = hi; }
    DdaF st[TPT];
    float part[TPT][kMD];
    double acc[TPT][kMD];
    const int start = lo == 0x7fffffff ? 0 : lo;
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
        st[q] = ddaf_init_at(tk[q], start - tk[q].t0);
#pragma unroll
        for (int k = 0; k < kMD; ++k) { part[q][k] = 0.0f; acc[q][k] = 0.0; }
    }
    __syncthreads();
    if (lane == 0) {
        atomicMin(&bnd[0], lo);
        atomicMax(&bnd[1], hi);
    }
    __syncthreads();
    const int c_first = __builtin_amdgcn_readfirstlane(bnd[0]), c_last = __builtin_amdgcn_readfirstlane(bnd[1]);
    using E = elem_t<MAPT>;
    const int ldc = (int)m.ld;
    const int col8 = ldc * (int)sizeof(E) / 8, per_col = col8 / (kDmaBytes / 8);  // 8-byte units per column
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    auto issue = [&](int c0, int bsel) {
        const int nchunk = min(S, c_last - c0 + 1) * per_col;
        const float2 *src = m.Y + (int64_t)c0 * col8 + lane * 2;
        float2 *dst = slab + (size_t)bsel * S * col8;
        for (int ch = wave; ch < nchunk; ch += WG / 64)
            lds_dma_16(src + ch * (kDmaBytes / 8), dst + ch * (kDmaBytes / 8));
    };
    if (c_first <= c_last) issue(c_first, 0);
    int kk = 0;
    for (int c0 = c_first; c0 <= c_last; c0 += S, ++kk) {
        __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of slab kk have landed
        __syncthreads();                // so have everyone's, and slab kk-1 is no longer read
        if (c0 + S <= c_last) issue(c0 + S, (kk + 1) & 1);
        const E *cur = reinterpret_cast<const E *>(slab + (size_t)(kk & 1) * S * col8);
        const int ncol = min(S, c_last - c0 + 1);
        const int ca = max(c0, lo), cb = min(c0 + ncol - 1, hi);
        walk_md<TPT, true, HW>(ca, min(cb, clo - 1), c0, cur, ldc, t0, span, dg, st, part, acc);
        walk_md<TPT, false, HW>(max(ca, clo), min(cb, chi), c0, cur, ldc, t0, span, dg, st, part, acc);
        walk_md<TPT, true, HW>(max(ca, chi + 1), cb, c0, cur, ldc, t0, span, dg, st, part, acc);
    }
    uint64_t key = 0;
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
        if (!live[q]) continue;
        float z;
        int32_t mi;
        merge_delays(acc[q], part[q], (int32_t)span[q] + 1, norm, m.scale, dg, ok[q], z, mi);
        merge_running(z, mi, m0 ? snr[idx[q]] : 0.0f, m0 ? tidx[idx[q]] : 0, m0 == 0);
        snr[idx[q]] = z;
        tidx[idx[q]] = mi;
        const uint64_t k = key_encode(z, (uint32_t)(first + idx[q]));
        key = k > key ? k : key;
    }
    if (!last) return;  // uniform: every workgroup of a launch has the same flag
    key = wave_max_u64(key);
    if (lane == 0) kred[threadIdx.x >> 6] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < WG / 64; ++w) key = kred[w] > key ? kred[w] : key;
        wg_keys[blockIdx.x] = key;
    }
}

// ---------------------------------------------------------------- batches of maps
// A batch scores n_m generated templates on each map m (the paper's n_ts
// time-shifted background maps, Sec. V). Map m's templates are binned within
// the map; its blocks of WG*TPT binned templates are the work items
// [item0[m], item0[m+1]). One persistent launch: each workgroup takes the
// next item from an atomic queue until the queue is empty, so maps of uneven
// length share the machine without a tail per map.

struct BatchMap {
    MapP m;
    GenP g;
    int64_t n;          // templates on this map
    uint64_t order0;    // offset of this map's binned order in the shared order array
    uint64_t bin0;      // offset of this map's bucket counters
    int32_t wb, nbins;  // bucket shift and count of this map
    int32_t S;          // slab columns
    int32_t chunk0;     // first sort chunk of this map
    uint64_t cc0;       // offset of this map's counts per group and sort chunk
    float *snr;         // optional per-template output
};

__global__ __launch_bounds__(256) void k_bin_count_batch(const BatchMap *maps, int n_maps, const uint32_t *chunk_start,
                                                         uint32_t *totals, uint16_t *bins, uint32_t *ccnt)
{
    __shared__ uint32_t hist[kMaxBins];
    const int mi = find_slot(chunk_start, n_maps, blockIdx.x);
    const BatchMap &d = maps[mi];
    for (int b = threadIdx.x; b < d.nbins; b += 256) hist[b] = 0;
    __syncthreads();
    const uint32_t c = blockIdx.x - chunk_start[mi];
    const int64_t base = (int64_t)c * kBinChunk;
    for (int q = 0; q < kBinPerThread; ++q) {
        const int64_t i = base + q * 256 + threadIdx.x;
        if (i < d.n) {
            const uint32_t b = bin_of<false>(d.g, nullptr, d.m, 0, i, d.wb);
            bins[d.order0 + i] = (uint16_t)b;
            atomicAdd(&hist[b], 1u);
        }
    }
    __syncthreads();
    count_out(hist, d.nbins, totals + d.bin0, ccnt + d.cc0 + c, chunk_start[mi + 1] - chunk_start[mi]);
}

// The scans of a batch, 1 + max_groups workgroups per map: the first scans the
// map's buckets, offset by its order0 (tables at gstart/fitem + map index *
// kGroupSlots); workgroup k + 1 scans row k of the map's chunk counts.
__global__ __launch_bounds__(256) void k_bin_scan_batch(const BatchMap *maps, const uint32_t *chunk_start,
                                                        int max_groups, const uint32_t *totals, uint32_t *cursor,
                                                        uint32_t *gstart, uint32_t *fitem, uint32_t *ccnt)
{
    const int mi = blockIdx.x / (max_groups + 1), k = (int)(blockIdx.x % (max_groups + 1)) - 1;
    const BatchMap &d = maps[mi];
    if (k < 0) {
        const size_t t0 = (size_t)mi * kGroupSlots;
        scan_buckets<256>(totals + d.bin0, d.nbins, (uint32_t)d.order0, cursor + d.bin0, gstart + t0, fitem + t0);
    } else if (k < (d.nbins + kGroupMask) >> kGroupShift) {
        const uint32_t nc = chunk_start[mi + 1] - chunk_start[mi];
        scan_row(ccnt + d.cc0 + (size_t)k * nc, (int)nc);
    }
}

// The scatters of k_bin_group and k_bin_fine, each workgroup on one map's
// templates: sort chunks in map order (chunk_start), and for the second,
// fine_start[mi] = the map's first workgroup (it has its second-scatter chunk
// count plus its group count of them, an upper bound of its chunks of group
// regions).
__global__ __launch_bounds__(kScatterWG) void k_bin_group_batch(const BatchMap *maps, int n_maps, const uint32_t *chunk_start,
                                                         const uint16_t *bins, const uint32_t *gstart,
                                                         const uint32_t *ccnt, uint32_t *tmp, uint8_t *tsub)
{
    __shared__ GroupLds L;
    const int mi = find_slot(chunk_start, n_maps, blockIdx.x);
    const BatchMap &d = maps[mi];
    const uint32_t c = blockIdx.x - chunk_start[mi];
    const int64_t base = (int64_t)c * kBinChunk;
    group_chunk<kScatterWG>(L, (d.nbins + kGroupMask) >> kGroupShift, base, (int)min<int64_t>(kBinChunk, d.n - base),
                bins + d.order0, gstart + (size_t)mi * kGroupSlots, ccnt + d.cc0 + c,
                chunk_start[mi + 1] - chunk_start[mi], tmp, tsub);
}

__global__ __launch_bounds__(kScatterWG) void k_bin_fine_batch(const BatchMap *maps, int n_maps, const uint32_t *fine_start,
                                                        const uint32_t *gstart, const uint32_t *fitem, uint32_t *cursor,
                                                        const uint32_t *tmp, const uint8_t *tsub, uint32_t *order)
{
    __shared__ FineLds L;
    const int mi = find_slot(fine_start, n_maps, blockIdx.x);
    const BatchMap &d = maps[mi];
    const int ngroups = (d.nbins + kGroupMask) >> kGroupShift;
    const uint32_t *fi = fitem + (size_t)mi * kGroupSlots;
    const uint32_t *gs = gstart + (size_t)mi * kGroupSlots;
    const uint32_t w = blockIdx.x - fine_start[mi];
    if (w >= fi[ngroups]) return;
    const int k = find_slot(fi, ngroups, w);
    const uint32_t e0 = gs[k] + (w - fi[k]) * (uint32_t)kFineChunk;
    const int b0 = k << kGroupShift;
    fine_chunk<kScatterWG>(L, min(1 << kGroupShift, d.nbins - b0), (int)min<uint32_t>(kFineChunk, gs[k + 1] - e0), tmp + e0,
               tsub + e0, cursor + d.bin0 + b0, order);
}

template <int WG, int TPT, bool HW, int MAPT, int SC>
__global__ __launch_bounds__(WG, kSlabWavesPerSimd) void k_score_batch(const BatchMap *maps, int n_maps,
                                                                       const uint32_t *item_start, uint32_t *queue,
                                                                       const uint32_t *order, int32_t norm,
                                                                       uint64_t *best)
{
    extern __shared__ float2 slab[];
    __shared__ int bnd[2];
    __shared__ uint64_t kred[WG / 64];
    __shared__ uint32_t item_s;
    const uint32_t total = item_start[n_maps];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) item_s = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t item = item_s;
        if (item >= total) break;  // every workgroup reaches this: the queue only grows
        const int mi = find_slot(item_start, n_maps, item);
        const BatchMap d = maps[mi];
        const uint64_t key = score_block<WG, TPT, HW, MAPT, SC>(d.m, d.g, nullptr, order + d.order0, 0, d.n,
                                                                   (int64_t)(item - item_start[mi]), d.S, norm,
                                                                   d.snr, slab, bnd, kred);
        // one atomic per item, spread over the maps' keys
        if (threadIdx.x == 0 && key) atomicMax((unsigned long long *)(best + mi), (unsigned long long)key);
    }
}

// ---------------------------------------------------------------- FP16 map packing
// p = Y/sigma in FP32 (correctly rounded division). Its magnitude in FP64 (the
// FP32 components square exactly: one rounding of the sum, one of the square
// root) times 2^-e is rounded to binary16, round to nearest even straight from
// FP64; its argument atan2 / (2 pi) to the nearest 2^-16 turn (ties to even),
// modulo one turn. Word = argument | binary16 bits << 16. k_absmax_p finds the
// largest magnitude first (its FP64 bits: non-negative doubles order as
// integers).

__device__ __forceinline__ double p_mag64(float x, float y)
{
    const double dx = x, dy = y;
    return sqrt(fma(dx, dx, dy * dy));
}

// binary16 bits of a non-negative double below 65520, rounded to nearest, ties to even
__device__ __forceinline__ uint32_t f64_to_f16_rne(double d)
{
    const uint64_t b = (uint64_t)__double_as_longlong(d);
    if (b == 0) return 0;
    const int ex = (int)((b >> 52) & 0x7FF) - 1023;
    const uint64_t sig = (b & 0xFFFFFFFFFFFFFull) | (1ull << 52);  // d = sig * 2^(ex - 52)
    // normal results keep 11 significant bits (shift 42); subnormal ones count units of 2^-24
    const int shift = ex >= -14 ? 42 : 28 - ex;
    if (shift >= 64) return 0;  // below 2^-36: rounds to zero
    uint64_t q = sig >> shift;
    const uint64_t rem = sig & ((1ull << shift) - 1), half = 1ull << (shift - 1);
    if (rem > half || (rem == half && (q & 1))) ++q;
    // a normal q in [2^10, 2^11]: exponent field plus fraction; the carry of q = 2^11 moves the exponent
    return ex >= -14 ? (uint32_t)(((uint32_t)(ex + 15) << 10) + (uint32_t)q - 1024u) : (uint32_t)q;
}

__global__ __launch_bounds__(256) void k_absmax_p(MapP m, unsigned long long *amax_bits)
{
    double mx = 0.0;
    const int64_t n = (int64_t)m.T * m.F;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t t = i / m.F, r = i - t * m.F;
        const int64_t e = t * m.ld + r;
        const float2 y = m.Y[e];
        const float sg = m.sig[e];
        mx = fmax(mx, p_mag64(y.x / sg, y.y / sg));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) atomicMax(amax_bits, (unsigned long long)__double_as_longlong(mx));
}

__global__ __launch_bounds__(256) void k_pack_p16(MapP m, double inv_scale, uint32_t *out, int64_t out_ld)
{
    const int64_t n = (int64_t)m.T * m.F;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t t = i / m.F, r = i - t * m.F;
        const int64_t e = t * m.ld + r;
        const float2 y = m.Y[e];
        const float sg = m.sig[e];
        const float px = y.x / sg, py = y.y / sg;
        const uint32_t mag = f64_to_f16_rne(p_mag64(px, py) * inv_scale);
        const double turns = atan2((double)py, (double)px) * 0.15915494309189535;  // 1 / (2 pi), rounded
        const uint32_t arg = (uint32_t)(int64_t)rint(turns * 65536.0) & 0xFFFFu;
        out[t * out_ld + r] = arg | (mag << 16);
    }
}

// ---------------------------------------------------------------- top-K
// Radix select over the 64-bit keys (score bits, ~index) -- all distinct, so
// the K-th largest key is a threshold that admits exactly K elements. Eight
// passes of 8 bits, each a histogram of the keys that share the digits fixed
// so far, with the choice of the next digit made on the device; then the K
// keys at or above the threshold are gathered and sorted in one workgroup.

struct TopkState {
    uint64_t prefix;     // digits fixed so far
    uint64_t mask;       // which bits of prefix are fixed
    uint32_t remaining;  // how many of the K still lie in the undecided bucket
    uint32_t count;      // gather cursor
    uint32_t hist[256];
};

__global__ __launch_bounds__(256) void k_topk_init(TopkState *st, uint32_t K)
{
    if (threadIdx.x == 0) {
        st->prefix = 0;
        st->mask = 0;
        st->remaining = K;
        st->count = 0;
    }
    st->hist[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void k_topk_hist(const float *z, int64_t n, uint64_t first, TopkState *st, int shift)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t prefix = st->prefix, mask = st->mask;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const uint64_t k = key_encode(z[i], (uint32_t)(first + (uint64_t)i));
        if ((k & mask) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&st->hist[threadIdx.x], h[threadIdx.x]);
}

// One workgroup: choose the digit holding the remaining-th largest key, then clear the histogram.
__global__ __launch_bounds__(256) void k_topk_pick(TopkState *st, int shift)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = st->hist[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t need = st->remaining, above = 0;
        int d = 255;
        for (; d > 0; --d) {
            if (above + h[d] >= need) break;
            above += h[d];
        }
        st->prefix |= (uint64_t)d << shift;
        st->mask |= (uint64_t)0xFF << shift;
        st->remaining = need - above;
    }
    st->hist[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void k_topk_gather(const float *z, int64_t n, uint64_t first, TopkState *st,
                                                     uint64_t *cand, uint32_t K)
{
    const uint64_t thr = st->prefix;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const uint64_t k = key_encode(z[i], (uint32_t)(first + (uint64_t)i));
        if (k >= thr) {
            const uint32_t pos = atomicAdd(&st->count, 1u);
            if (pos < K) cand[pos] = k;  // exactly K keys pass (all keys are distinct); the bound is a guard
        }
    }
}

// Sort the K gathered keys descending (bitonic, in LDS) and write (index, score).
__global__ __launch_bounds__(1024) void k_topk_sort(const uint64_t *cand, int K, int P, int64_t *idx, float *val)
{
    extern __shared__ uint64_t kk[];  // P = power of two >= K
    for (int i = threadIdx.x; i < P; i += 1024) kk[i] = i < K ? cand[i] : 0;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P; i += 1024) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool desc = (i & size) == 0;
                    const uint64_t a = kk[i], b = kk[j];
                    if (desc ? a < b : a > b) { kk[i] = b; kk[j] = a; }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < K; i += 1024) {
        const uint64_t k = kk[i];
        const uint32_t o = (uint32_t)(k >> 32);
        const uint32_t b = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
        if (idx) idx[i] = (int64_t)(0xFFFFFFFFu - (uint32_t)k);
        if (val) val[i] = __uint_as_float(b);
    }
}

// ---------------------------------------------------------------- FP64 re-score
// One wave per template: lanes stride over its columns; each pixel's row is
// the exact floor of Eq. 6 by 64-bit integer division, the phase the exact
// 2^-32-turn integer, the term and the sum in FP64 (fixed-order wave
// reduction, so the result is deterministic).

template <bool EXPL>
__global__ __launch_bounds__(256) void k_rescore_f64(MapP m, GenP g, const Trk *tr, int64_t ntr, uint64_t first,
                                                     const int64_t *idx, int32_t K, int32_t norm, double *out)
{
    const int w = (int)(((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= K) return;
    const int64_t j = idx[w];
    Trk t;
    bool ok;
    if (EXPL) {
        ok = j >= (int64_t)first && j - (int64_t)first < ntr;
        t = tr[ok ? j - (int64_t)first : 0];
        ok = ok && track_ok(t, m);
    } else {
        ok = j >= 0 && j < ((int64_t)1 << 32);
        t = draw_track(g, (uint64_t)j);
    }
    double s = 0.0;
    int32_t N = 1;
    if (ok) {
        const int64_t Dt = t.t2 - t.t0;
        N = (int32_t)Dt + 1;
        const uint64_t Q = (uint64_t)(Dt * Dt) << 8;
        for (int64_t k = lane; k <= Dt; k += 64) {
            const uint64_t a = (uint64_t)(Dt - k), b = (uint64_t)k;
            const uint64_t num = a * a * t.f0 + 2 * a * b * t.f1 + b * b * t.f2;
            const int64_t row = (int64_t)(num / Q);
            const int64_t e = (t.t0 + k) * m.ld + row;
            const double sg = m.sig[e];
            const double pr = (double)m.Y[e].x / sg, pim = (double)m.Y[e].y / sg;
            const uint32_t ph = (uint32_t)((int64_t)(m.fq4_lo + row * m.dfq4) * (int64_t)t.dtau);
            double sn, cs;
            sincos(6.283185307179586 * ((double)(int32_t)ph * 2.3283064365386963e-10), &sn, &cs);
            s += cs * pr - sn * pim;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) out[w] = ok ? (norm == 1 ? s / N : s / sqrt((double)N)) : __builtin_nan("");
}

// ---------------------------------------------------------------- smooth SNR and its gradient
// theta = (tau0, tau2, phi0, phi1, phi2, dtau_ms) per template, K samples
// xi_k = k/(K-1); sample (u, v) = (clamp(t_k, 0, T-1), clamp(f_k - 1/2, 0, F-1)),
// bilinear interpolation of G(t, r) = Re[exp(2 pi i f(r) dtau) p(t, r)] and
// of its dtau-derivative; z~ = K^-1/2 sum. One wave per template, lanes over
// samples; sums in FP64, reduced in a fixed order (deterministic).

template <int MAPT>
__device__ __forceinline__ void smooth_node(const MapP &m, int64_t t, int64_t r, double dtau_s, float &g, float &gd)
{
    const float2 p = load_p<MAPT>(m, t * m.ld + r);
    const double f_hz = (double)(m.fq4_lo + r * m.dfq4) * 0.0625;
    double turns = f_hz * dtau_s;
    turns -= floor(turns);
    const float x = (float)turns;
    const float c = __builtin_amdgcn_cosf(x), s = __builtin_amdgcn_sinf(x);
    g = c * p.x - s * p.y;
    gd = -6.283185307179586f * (float)f_hz * (s * p.x + c * p.y);
}

// One workgroup of kSmoothWG lanes per template (lanes over the K samples):
// the bilinear gathers miss L2, so several waves per template keep more of
// them in flight than one wave could.
constexpr int kSmoothWG = 256;

// The smooth statistic of one template at th[0..5] (readable by every lane)
// and, with grad_out, its gradient; all kSmoothWG lanes of the workgroup call
// it. Lane k sums samples k, k + kSmoothWG, ...; waves reduce by shuffles and
// thread 0 adds the waves in order, so the result does not depend on timing.
// Results (z, grad_out[0..5]) are valid in thread 0.
template <int MAPT>
__device__ __forceinline__ void smooth_block(const MapP &m, const float *th, int K, double (*red)[7], float &z_out,
                                             float *grad_out)
{
    const int lane = threadIdx.x & 63;
    const double tau0 = th[0], tau2 = th[1], ph0 = th[2], ph1 = th[3], ph2 = th[4];
    const double dtau_s = (double)th[5] * 1e-3;
    double z = 0, g0 = 0, g1 = 0, g2 = 0, g3 = 0, g4 = 0, g5 = 0;
    for (int k = threadIdx.x; k < K; k += kSmoothWG) {
        const double xi = K > 1 ? (double)k / (double)(K - 1) : 0.0;
        const double b0 = (1 - xi) * (1 - xi), b1 = 2 * xi * (1 - xi), b2 = xi * xi;
        const double u0 = tau0 + xi * (tau2 - tau0), v0 = b0 * ph0 + b1 * ph1 + b2 * ph2 - 0.5;
        // clamp into the map (fmax/fmin also send a NaN coordinate to the lower edge)
        const double u = fmin(fmax(u0, 0.0), (double)(m.T - 1)), v = fmin(fmax(v0, 0.0), (double)(m.F - 1));
        const bool ut = u0 >= 0.0 && u0 <= (double)(m.T - 1), vt = v0 >= 0.0 && v0 <= (double)(m.F - 1);
        int64_t i = (int64_t)floor(u), r = (int64_t)floor(v);
        if (i > m.T - 2) i = m.T - 2;
        if (r > m.F - 2) r = m.F - 2;
        const double a = u - (double)i, b = v - (double)r;
        float G00, G10, G01, G11, D00, D10, D01, D11;
        smooth_node<MAPT>(m, i, r, dtau_s, G00, D00);
        smooth_node<MAPT>(m, i + 1, r, dtau_s, G10, D10);
        smooth_node<MAPT>(m, i, r + 1, dtau_s, G01, D01);
        smooth_node<MAPT>(m, i + 1, r + 1, dtau_s, G11, D11);
        z += (1 - a) * (1 - b) * G00 + a * (1 - b) * G10 + (1 - a) * b * G01 + a * b * G11;
        const double du = ut ? (1 - b) * (G10 - G00) + b * (G11 - G01) : 0.0;
        const double dv = vt ? (1 - a) * (G01 - G00) + a * (G11 - G10) : 0.0;
        g0 += (1 - xi) * du;
        g1 += xi * du;
        g2 += b0 * dv;
        g3 += b1 * dv;
        g4 += b2 * dv;
        g5 += ((1 - a) * (1 - b) * D00 + a * (1 - b) * D10 + (1 - a) * b * D01 + a * b * D11) * 1e-3;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        z += __shfl_xor(z, off);
        g0 += __shfl_xor(g0, off);
        g1 += __shfl_xor(g1, off);
        g2 += __shfl_xor(g2, off);
        g3 += __shfl_xor(g3, off);
        g4 += __shfl_xor(g4, off);
        g5 += __shfl_xor(g5, off);
    }
    if (lane == 0) {
        double *r = red[threadIdx.x >> 6];
        r[0] = z, r[1] = g0, r[2] = g1, r[3] = g2, r[4] = g3, r[5] = g4, r[6] = g5;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < kSmoothWG / 64; ++v) {
            z += red[v][0], g0 += red[v][1], g1 += red[v][2], g2 += red[v][3];
            g3 += red[v][4], g4 += red[v][5], g5 += red[v][6];
        }
        const double sc = K > 0 ? 1.0 / sqrt((double)K) : 0.0;
        z_out = (float)(z * sc);
        if (grad_out) {
            grad_out[0] = (float)(g0 * sc);
            grad_out[1] = (float)(g1 * sc);
            grad_out[2] = (float)(g2 * sc);
            grad_out[3] = (float)(g3 * sc);
            grad_out[4] = (float)(g4 * sc);
            grad_out[5] = (float)(g5 * sc);
        }
    }
}

template <int MAPT>
__global__ __launch_bounds__(kSmoothWG) void k_smooth_grad(MapP m, const float *theta, const int32_t *Ks, int32_t n,
                                                           float *z_out, float *grad_out)
{
    __shared__ double red[kSmoothWG / 64][7];
    const int w = blockIdx.x;
    if (w >= n) return;  // whole workgroup
    float z;
    smooth_block<MAPT>(m, theta + (int64_t)w * 6, Ks[w], red, z, grad_out ? grad_out + (int64_t)w * 6 : nullptr);
    if (threadIdx.x == 0) z_out[w] = z;
}

// ---------------------------------------------------------------- refinement helpers

__global__ __launch_bounds__(256) void k_tracks_at(GenP g, const int64_t *idx, int64_t n, Trk *out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = draw_track(g, (uint64_t)idx[i]);
}

// A plain template's parameters as a smooth-SNR point: times as columns,
// control frequencies in rows, delay in ms; K = its pixel count.
__global__ __launch_bounds__(256) void k_track_to_theta(const Trk *tr, int64_t n, float *theta, int32_t *Ks)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const Trk t = tr[i];
    float *th = theta + i * 6;
    th[0] = (float)t.t0;
    th[1] = (float)t.t2;
    th[2] = (float)t.f0 * (1.0f / 256.0f);
    th[3] = (float)t.f1 * (1.0f / 256.0f);
    th[4] = (float)t.f2 * (1.0f / 256.0f);
    th[5] = (float)((double)t.dtau * (1e3 / 268435456.0));
    Ks[i] = t.t2 - t.t0 + 1;
}

struct RefineP {
    int32_t T, F, L;
    double dmax_ms;
    double px0, px1, ms0, ms1;
    int32_t steps;
};

__device__ __forceinline__ void project_theta(double *th, const RefineP &p)
{
    double a = th[0], b = th[1];
    if (b - a < p.L - 1) {
        const double mid = 0.5 * (a + b);
        a = mid - 0.5 * (p.L - 1);
        b = mid + 0.5 * (p.L - 1);
    }
    if (a < 0) { b -= a; a = 0; }
    if (b > p.T - 1) { a -= b - (p.T - 1); b = p.T - 1; }
    if (a < 0) a = 0;
    th[0] = a;
    th[1] = b;
    const double fhi = (double)p.F - 1.0 / 512.0;
    for (int q = 2; q < 5; ++q) th[q] = fmin(fhi, fmax(0.0, th[q]));
    th[5] = fmin(p.dmax_ms, fmax(-p.dmax_ms, th[5]));
}

// Ascent step s of a template at th (FP32 parameters, updated in place) with
// gradient g: the five positions move by eta_px * g / |g|, the delay by
// eta_ms * sign(g), with the step sizes falling linearly over the steps; then
// projection onto the feasible set.
__device__ __forceinline__ void refine_move(float *th, const float *g, int32_t s, const RefineP &p)
{
    const double w = p.steps > 1 ? (double)s / (double)(p.steps - 1) : 0.0;
    const double epx = p.px0 + w * (p.px1 - p.px0), ems = p.ms0 + w * (p.ms1 - p.ms0);
    double t[6];
    for (int q = 0; q < 6; ++q) t[q] = th[q];
    double n2 = 0;
    for (int q = 0; q < 5; ++q) n2 += (double)g[q] * g[q];
    if (n2 > 0) {
        const double inv = 1.0 / sqrt(n2);
        for (int q = 0; q < 5; ++q) t[q] += epx * g[q] * inv;
    }
    if (g[5] > 0) t[5] += ems;
    else if (g[5] < 0) t[5] -= ems;
    project_theta(t, p);
    for (int q = 0; q < 6; ++q) th[q] = (float)t[q];
}

// The whole refinement of one template in one workgroup: project the start,
// then for s = 0..steps evaluate the smooth statistic and its gradient at the
// current point, keep the point if it is the best so far (s = 0 starts the
// best), and, while s < steps, take ascent step s. theta holds the start on
// entry and the best point on exit; best_z receives its smooth statistic.
template <int MAPT>
__global__ __launch_bounds__(kSmoothWG) void k_refine(MapP m, float *theta, const int32_t *Ks, int32_t n,
                                                      float *best_z, RefineP p)
{
    __shared__ double red[kSmoothWG / 64][7];
    __shared__ float cur[6];
    const int w = blockIdx.x;
    if (w >= n) return;  // whole workgroup
    float *th_io = theta + (int64_t)w * 6;
    if (threadIdx.x == 0) {
        double t[6];
        for (int q = 0; q < 6; ++q) t[q] = th_io[q];
        project_theta(t, p);
        for (int q = 0; q < 6; ++q) cur[q] = (float)t[q];
    }
    __syncthreads();
    const int K = Ks[w];
    float best[6], bz = 0.0f, z, g[6];
    for (int32_t s = 0; s <= p.steps; ++s) {
        smooth_block<MAPT>(m, cur, K, red, z, g);
        if (threadIdx.x == 0) {
            if (s == 0 || z > bz) {
                bz = z;
                for (int q = 0; q < 6; ++q) best[q] = cur[q];
            }
            if (s < p.steps) refine_move(cur, g, s, p);
        }
        __syncthreads();  // the new point is visible; red may be reused
    }
    if (threadIdx.x == 0) {
        for (int q = 0; q < 6; ++q) th_io[q] = best[q];
        best_z[w] = bz;
    }
}

// Back to a plain template (times half up, widened to L pixels; frequencies
// floor(256 phi) inside the band; delay to the nearest 2^-28 s, clipped).
__global__ __launch_bounds__(256) void k_theta_to_track(const float *theta, int64_t n, int32_t T, int32_t F, int32_t L,
                                                        int32_t dtau_max, Trk *out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float *th = theta + i * 6;
    // rounded and clamped in FP64 before converting, so any input stays inside the map
    int32_t t0 = (int32_t)fmin(fmax(floor((double)th[0] + 0.5), 0.0), (double)(T - 1));
    int32_t t2 = (int32_t)fmin(fmax(floor((double)th[1] + 0.5), 0.0), (double)(T - 1));
    if (t2 - t0 < L - 1) {
        t2 = t0 + L - 1;
        if (t2 > T - 1) { t0 -= t2 - (T - 1); t2 = T - 1; }
    }
    Trk t;
    t.t0 = t0;
    t.t2 = t2;
    uint32_t f[3];
    for (int q = 0; q < 3; ++q) {
        double v = floor((double)th[2 + q] * 256.0);
        v = fmin(fmax(v, 0.0), (double)F * 256 - 1);
        f[q] = (uint32_t)v;
    }
    t.f0 = f[0];
    t.f1 = f[1];
    t.f2 = f[2];
    double d = floor((double)th[5] * 1e-3 * 268435456.0 + 0.5);
    d = fmin(fmax(d, -(double)dtau_max), (double)dtau_max);
    t.dtau = (int32_t)d;
    out[i] = t;
}

}  // namespace stt
