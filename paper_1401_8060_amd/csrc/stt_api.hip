// stt_api.hip -- host side of libstt: contexts, argument validation, scratch,
// launch configuration and the extern "C" entry points declared in stt.h.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "stt.h"
#include "kernels.hpp"
#include "mapform.hpp"
#include "signif.hpp"

using namespace stt;

struct Rec {
    size_t base;  // first of the call's six events in the pool
    bool used[3];
};

struct stt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    void *aux = nullptr;  // top-K state and candidates
    size_t aux_bytes = 0;
    void *pbuf = nullptr;  // folded p = Y/sigma maps for LDS-DMA staging
    size_t pbuf_bytes = 0;
    void *mdbuf = nullptr;  // running maxima of delay-grid scoring when the caller keeps none
    size_t mdbuf_bytes = 0;
    bool dma = true;       // fold + double-buffered LDS-DMA staging where a column fits
    int path = 0;  // 0 auto, 1 direct, 2 slab
    int lds_bytes = 160 * 1024;  // slab budget per workgroup
    int slab_wg = 1024;          // slab scorer shape: lanes per workgroup
    int slab_tpt = 4;            //                    templates per lane
    bool hw_trig = true;         // hardware sine/cosine (measured max error 1.3e-7) or the polynomial
    // Timing: every call takes six events from a pool (start/end of the scoring
    // kernel, of the binning kernels and of the whole call); queries sum them.
    bool timing = false;
    std::vector<hipEvent_t> pool;
    size_t next = 0;         // first free event of the pool
    size_t last = 0;         // first event of the last call
    bool used[3] = {false, false, false};
    // events that the next launch_ev records from its own dispatch (its start, its end)
    hipEvent_t kev_start = nullptr, kev_stop = nullptr;
    std::vector<Rec> recs;   // calls since the last total query
    // Batches: descriptor tables on the device, and the captured graph of the
    // last batch (replayed while the arguments stay the same).
    bool use_graph = true;
    hipStream_t cap_stream = nullptr;
    void *bdev = nullptr;
    size_t bdev_bytes = 0;
    std::vector<uint8_t> bkey;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int n_cu = 0;
    // map formation: FFT twiddles and window of the current column length
    void *fft_tab = nullptr;
    int fft_M = 0;
};

namespace {

stt_status fail(stt_ctx *c, stt_status s, const char *fmt, ...)
    __attribute__((format(printf, 3, 4)));

stt_status fail(stt_ctx *c, stt_status s, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

#define STT_HIP(c, call)                                                                      \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail((c), STT_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

stt_status ensure_scratch(stt_ctx *c, size_t bytes)
{
    if (bytes <= c->scratch_bytes) return STT_OK;
    if (c->scratch) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return fail(c, STT_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
        (void)hipFree(c->scratch);
        c->scratch = nullptr;
        c->scratch_bytes = 0;
    }
    size_t want = std::max(bytes, (size_t)1 << 20);
    if (hipMalloc(&c->scratch, want) != hipSuccess) {
        (void)hipGetLastError();
        c->scratch = nullptr;
        return fail(c, STT_ENOMEM, "cannot allocate %zu bytes of scratch", want);
    }
    c->scratch_bytes = want;
    return STT_OK;
}

stt_status ensure_aux(stt_ctx *c, size_t bytes)
{
    if (bytes <= c->aux_bytes) return STT_OK;
    if (c->aux) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return fail(c, STT_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
        (void)hipFree(c->aux);
        c->aux = nullptr;
        c->aux_bytes = 0;
    }
    if (hipMalloc(&c->aux, bytes) != hipSuccess) {
        (void)hipGetLastError();
        c->aux = nullptr;
        return fail(c, STT_ENOMEM, "cannot allocate %zu bytes", bytes);
    }
    c->aux_bytes = bytes;
    return STT_OK;
}

stt_status ensure_pbuf(stt_ctx *c, size_t bytes)
{
    if (bytes <= c->pbuf_bytes) return STT_OK;
    if (c->pbuf) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return fail(c, STT_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
        (void)hipFree(c->pbuf);
        c->pbuf = nullptr;
        c->pbuf_bytes = 0;
    }
    if (hipMalloc(&c->pbuf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, STT_ENOMEM, "cannot allocate %zu bytes for the folded map", bytes);
    }
    c->pbuf_bytes = bytes;
    return STT_OK;
}

stt_status ensure_mdbuf(stt_ctx *c, size_t bytes)
{
    if (bytes <= c->mdbuf_bytes) return STT_OK;
    if (c->mdbuf) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return fail(c, STT_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
        (void)hipFree(c->mdbuf);
        c->mdbuf = nullptr;
        c->mdbuf_bytes = 0;
    }
    if (hipMalloc(&c->mdbuf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, STT_ENOMEM, "cannot allocate %zu bytes of delay-grid maxima", bytes);
    }
    c->mdbuf_bytes = bytes;
    return STT_OK;
}

// Column stride of a folded map and the slab depth that two buffers of it allow.
// Bytes per pixel of the folded map the scorers read: 8 for an FP32 map (polar FP32 pair), 4 for
// an FP16 map (its words).
int fold_esize(int dtype) { return dtype == STT_P16 ? 4 : 8; }
int64_t fold_ld(int F, int esize = 8)
{
    const int64_t per = kDmaBytes / esize;  // pixels per 1 KB piece
    return ((int64_t)F + per - 1) / per * per;
}
int dma_slab_cols(int lds_bytes, int64_t ldc, int esize = 8)
{
    return (int)std::min<int64_t>(64, (lds_bytes - 256) / (2 * ldc * esize));
}
int dma_slab_cols(const stt_ctx *c, int64_t ldc, int esize = 8) { return dma_slab_cols(c->lds_bytes, ldc, esize); }

stt_status check_map(stt_ctx *c, const stt_map *m)
{
    if (!m) return fail(c, STT_EINVAL, "map is NULL");
    if (m->dtype != STT_C64F32 && m->dtype != STT_P16)
        return fail(c, STT_EINVAL, "map dtype %d unknown", m->dtype);
    if (m->dtype == STT_P16 && m->sigma) return fail(c, STT_EINVAL, "an FP16 map has no sigma array (pass NULL)");
    if (m->dtype == STT_P16 && (m->scale_exp < -126 || m->scale_exp > 127))
        return fail(c, STT_ERANGE, "scale_exp=%d outside [-126, 127]", m->scale_exp);
    if (m->T < 2 || m->T > STT_MAX_T) return fail(c, STT_ERANGE, "T=%d outside [2, %d]", m->T, STT_MAX_T);
    if (m->F < 1 || m->F > STT_MAX_F) return fail(c, STT_ERANGE, "F=%d outside [1, %d]", m->F, STT_MAX_F);
    if (m->ld < m->F) return fail(c, STT_EINVAL, "ld=%lld < F=%d", (long long)m->ld, m->F);
    if (!m->Y || (m->dtype == STT_C64F32 && !m->sigma)) return fail(c, STT_EINVAL, "map Y or sigma is NULL");
    const int64_t fmax = std::llabs((int64_t)m->fq4_lo) + (int64_t)(m->F - 1) * std::llabs((int64_t)m->dfq4);
    if (fmax >= ((int64_t)1 << 31)) return fail(c, STT_ERANGE, "row frequencies overflow 32 bits");
    return STT_OK;
}

stt_status make_genp(stt_ctx *c, const stt_gen *g, int32_t T, int32_t F, GenP &p)
{
    if (!g) return fail(c, STT_EINVAL, "gen is NULL");
    if (T < 2 || T > STT_MAX_T) return fail(c, STT_ERANGE, "T=%d outside [2, %d]", T, STT_MAX_T);
    if (F < 1 || F > STT_MAX_F) return fail(c, STT_ERANGE, "F=%d outside [1, %d]", F, STT_MAX_F);
    if (g->min_len < 2 || g->min_len > T) return fail(c, STT_ERANGE, "min_len=%d outside [2, T=%d]", g->min_len, T);
    if (g->dtau_max < 0 || g->dtau_max >= (1 << 30)) return fail(c, STT_ERANGE, "dtau_max=%d outside [0, 2^30)", g->dtau_max);
    if (std::llabs((int64_t)g->dtau_center) + g->dtau_max >= ((int64_t)1 << 30))
        return fail(c, STT_ERANGE, "delay patch [%d - %d, %d + %d] leaves (-2^30, 2^30)", g->dtau_center, g->dtau_max,
                    g->dtau_center, g->dtau_max);
    const int64_t npos = (int64_t)T - g->min_len + 1;
    p.key0 = (uint32_t)g->seed;
    p.key1 = (uint32_t)(g->seed >> 32);
    p.stream = g->stream;
    p.npairs = (uint32_t)(npos * (npos + 1) / 2);
    p.L = g->min_len;
    p.frange = (uint32_t)F << 8;
    p.dmax = g->dtau_max - g->dtau_center;  // the draw subtracts this: delays on [center - D, center + D]
    p.dspan = 2u * (uint32_t)g->dtau_max + 1u;
    return STT_OK;
}

stt_status check_range(stt_ctx *c, int64_t first, int64_t n)
{
    if (first < 0 || n < 0) return fail(c, STT_EINVAL, "first=%lld, n=%lld must be >= 0", (long long)first, (long long)n);
    if (first + n > ((int64_t)1 << 32)) return fail(c, STT_ERANGE, "track indices must stay below 2^32");
    return STT_OK;
}

MapP to_mapp(const stt_map *m)
{
    MapP p;
    p.Y = (const float2 *)m->Y;
    p.sig = (const float *)m->sigma;
    p.T = m->T;
    p.F = m->F;
    p.ld = m->ld;
    p.fq4_lo = m->fq4_lo;
    p.dfq4 = m->dfq4;
    p.scale = m->dtype == STT_P16 ? std::ldexp(1.0f, m->scale_exp) : 1.0f;
    return p;
}

// Reserve six events for this call (growing the pool when needed).
stt_status ev_begin(stt_ctx *c)
{
    for (bool &u : c->used) u = false;
    c->kev_start = c->kev_stop = nullptr;
    if (!c->timing) return STT_OK;
    while (c->pool.size() < c->next + 6) {
        hipEvent_t e;
        STT_HIP(c, hipEventCreate(&e));
        c->pool.push_back(e);
    }
    c->last = c->next;
    c->next += 6;
    return STT_OK;
}

void ev_record(stt_ctx *c, int i)
{
    if (c->timing) (void)hipEventRecord(c->pool[c->last + i], c->stream);
}

// Events i (start) and j (end) of this call, -1 for none, taken by the next launch_ev from its
// kernel's own dispatch. (hipEventRecord enqueues a marker, which waits for the stream to drain:
// about 6 us between two kernels.)
void ev_attach(stt_ctx *c, int i, int j)
{
    c->kev_start = c->timing && i >= 0 ? c->pool[c->last + i] : nullptr;
    c->kev_stop = c->timing && j >= 0 ? c->pool[c->last + j] : nullptr;
}

// A kernel launch on the context's stream that records the attached events, if any.
template <typename K, typename... A>
void launch_ev(stt_ctx *c, K kern, dim3 grid, dim3 block, size_t shm, A... args)
{
    hipExtLaunchKernelGGL(kern, grid, block, (uint32_t)shm, c->stream, c->kev_start, c->kev_stop, 0u, args...);
    c->kev_start = c->kev_stop = nullptr;
}

void ev_end(stt_ctx *c)
{
    if (!c->timing) return;
    Rec r;
    r.base = c->last;
    for (int i = 0; i < 3; ++i) r.used[i] = c->used[i];
    c->recs.push_back(r);
}

// Bucket width 2^wb of the time-extent sort: the narrowest that keeps at most
// 128 buckets per axis and, on average, at least one wave's worth (256) of
// templates per (start, end) bucket -- narrow buckets make a wave's templates
// start and end together, so more of its columns need no mask.
int bucket_shift(int T, int64_t n)
{
    int wb = 0;
    for (;; ++wb) {
        const int64_t nb = ((T - 1) >> wb) + 1;
        if (nb > 128) continue;
        if (nb <= 1 || n / (nb * (nb + 1) / 2) >= 256) break;
    }
    return wb;
}

template <int WG, int TPT, bool HW, int MAPT, int SC>
stt_status launch_slab_t(stt_ctx *c, const MapP &m, const GenP &g, const Trk *tr, const uint32_t *order,
                         int64_t first, int64_t n, int S, size_t shm, int32_t norm, float *snr, uint64_t *wg_keys)
{
    auto kern = k_score_slab<WG, TPT, HW, MAPT, SC>;
    if (shm > 64 * 1024)
        STT_HIP(c, hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    const unsigned grid = (unsigned)((n + WG * TPT - 1) / (WG * TPT));
    launch_ev(c, kern, dim3(grid), dim3(WG), shm, m, g, tr, order, (uint64_t)first, n, S, norm, snr, wg_keys);
    STT_HIP(c, hipGetLastError());
    return STT_OK;
}

// The (workgroup size, templates per lane) shapes compiled into the library.
static const int kShapes[][2] = {{1024, 4}, {512, 4}, {256, 4}, {1024, 2}, {512, 2}};

template <bool HW, int MAPT, int SC>
stt_status launch_slab_h(stt_ctx *c, int wg, int tpt, const MapP &m, const GenP &g, const Trk *tr,
                         const uint32_t *order, int64_t first, int64_t n, int S, size_t shm, int32_t norm, float *snr,
                         uint64_t *wg_keys)
{
#define STT_SLAB_CASE(W, P)                                                                                     \
    if (wg == W && tpt == P)                                                                                    \
        return launch_slab_t<W, P, HW, MAPT, SC>(c, m, g, tr, order, first, n, S, shm, norm, snr, wg_keys);
    STT_SLAB_CASE(1024, 4)
    STT_SLAB_CASE(512, 4)
    STT_SLAB_CASE(256, 4)
    STT_SLAB_CASE(1024, 2)
    STT_SLAB_CASE(512, 2)
#undef STT_SLAB_CASE
    return fail(c, STT_EUNSUPPORTED, "no slab scorer compiled for workgroup %d x %d templates", wg, tpt);
}

template <int MAPT, int SC>
stt_status launch_slab_sc(stt_ctx *c, int wg, int tpt, const MapP &m, const GenP &g, const Trk *tr,
                          const uint32_t *order, int64_t first, int64_t n, int S, size_t shm, int32_t norm, float *snr,
                          uint64_t *wg_keys)
{
    if (c->hw_trig)
        return launch_slab_h<true, MAPT, SC>(c, wg, tpt, m, g, tr, order, first, n, S, shm, norm, snr, wg_keys);
    return launch_slab_h<false, MAPT, SC>(c, wg, tpt, m, g, tr, order, first, n, S, shm, norm, snr, wg_keys);
}

// The widest aligned slab (a power of two dividing the 16-column flush grid) not wider than
// `cols`, the columns two buffers fit; 0 below 2 (then the slabs stage through registers).
int aligned_slab(int cols)
{
    int sc = 16;
    while (sc > cols) sc >>= 1;
    return sc >= 2 ? sc : 0;
}

// sc > 0: LDS-DMA slabs of sc aligned columns (sc in 2, 4, 8, 16); sc = 0: register staging of
// S columns. Templates are drawn (tr == NULL) or given.
template <int MAPT>
stt_status launch_slab(stt_ctx *c, int sc, int wg, int tpt, const MapP &m, const GenP &g, const Trk *tr,
                       const uint32_t *order, int64_t first, int64_t n, int S, size_t shm, int32_t norm, float *snr,
                       uint64_t *wg_keys)
{
    switch (sc) {
    case 0: return launch_slab_sc<MAPT, 0>(c, wg, tpt, m, g, tr, order, first, n, S, shm, norm, snr, wg_keys);
    case 2: return launch_slab_sc<MAPT, 2>(c, wg, tpt, m, g, tr, order, first, n, S, shm, norm, snr, wg_keys);
    case 4: return launch_slab_sc<MAPT, 4>(c, wg, tpt, m, g, tr, order, first, n, S, shm, norm, snr, wg_keys);
    case 8: return launch_slab_sc<MAPT, 8>(c, wg, tpt, m, g, tr, order, first, n, S, shm, norm, snr, wg_keys);
    case 16: return launch_slab_sc<MAPT, 16>(c, wg, tpt, m, g, tr, order, first, n, S, shm, norm, snr, wg_keys);
    default: return fail(c, STT_EUNSUPPORTED, "no slab scorer for %d-column slabs", sc);
    }
}

template <bool EXPL, bool HW, int MAPT>
void launch_direct(stt_ctx *c, bool per_wave, const MapP &m, const GenP &g, const Trk *tr, int64_t first, int64_t n,
                   int32_t norm, float *snr, uint64_t *best)
{
    if (per_wave) {
        hipLaunchKernelGGL((k_score_wave<EXPL, HW, MAPT>), dim3((unsigned)((n + 3) / 4)), dim3(256), 0, c->stream, m,
                           g, tr, (uint64_t)first, n, norm, snr, best);
        return;
    }
    const unsigned grid = (unsigned)((n + kWG - 1) / kWG);
    hipLaunchKernelGGL((k_score_direct<EXPL, HW, MAPT>), dim3(grid), dim3(kWG), 0, c->stream, m, g, tr,
                       (uint64_t)first, n, norm, snr, best);
}

// Work memory handed to a scoring call instead of the context's own (which grows
// on demand): the binning scratch and the folded map, both big enough for the
// call (checked by the caller).
struct FixedBufs {
    void *scratch;  // bucket tables, binned order, per-workgroup keys
    void *pbuf;     // folded map
};

// The map folded for the scorers into the context's folded-map buffer, or into fb's: an FP32 map
// as p in polar form (k_fold_polar, kMapPol), an FP16 map as its words in padded columns
// (k_fold_words, kMapPolH). Every scorer of Eq. 8 reads this copy; mf is its view (column stride
// fold_ld(F, element size)).
stt_status fold_polar(stt_ctx *c, const stt_map *map, const FixedBufs *fb, MapP &mf);
size_t folded_bytes(const stt_map *map);

// Scratch of a scoring call of n templates: bucket totals and cursors, the
// group starts and second-scatter chunk table, the binned order (padded to an
// even count; the count pass keeps each template's bucket there until the
// last scatter), one best-key slot per scorer workgroup (each takes at least
// 1024 templates, whatever the shape), the group regions of the first scatter
// (4 B index per template), the counts per group and sort chunk, then the
// bucket within the group of each entry of the group regions (1 B).
constexpr size_t score_scratch_bytes(int64_t n)
{
    const size_t n_order = ((size_t)n + 1) & ~(size_t)1;
    const size_t n_chunks = ((size_t)n + kBinChunk - 1) / kBinChunk;
    return sizeof(uint32_t) * (2 * (size_t)kMaxBins + 2 * (size_t)kGroupSlots + 2 * n_order + kMaxGroups * n_chunks) +
           n_order + sizeof(uint64_t) * (size_t)((n + 1023) / 1024);
}

}  // namespace

// ---------------------------------------------------------------- fixed scratch of stt_score_noalloc
// One static device array per GPU, for callers that cannot allocate: the
// folded map in its first kNaMapBytes, then the binning scratch of up to
// kNaMaxTracks templates. In host code `scratch` only names the symbol; its
// device address comes from hipGetSymbolAddress, taken once per device (with
// that device current) by stt_create and kept in g_na_ptr.
constexpr size_t kNaMapBytes = (size_t)32 << 20;
constexpr int64_t kNaMaxTracks = (int64_t)1 << 22;
constexpr size_t kNaScratchBytes = score_scratch_bytes(kNaMaxTracks);
constexpr size_t kNaBytes = kNaMapBytes + kNaScratchBytes;
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

constexpr int kNaMaxDevices = 64;
void *g_na_ptr[kNaMaxDevices] = {};
std::mutex g_na_mu;

// Device address of this device's copy of `scratch` (device current); false when it is unavailable.
bool na_init(int device)
{
    if (device < 0 || device >= kNaMaxDevices) return false;
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (g_na_ptr[device]) return true;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return false;
    }
    g_na_ptr[device] = p;
    return true;
}

void *na_ptr(int device)
{
    if (device < 0 || device >= kNaMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_na_mu);
    return g_na_ptr[device];
}

bool slab_shape_ok(int wg, int tpt)
{
    for (const auto &s : kShapes)
        if (s[0] == wg && s[1] == tpt) return true;
    return false;
}

// Counting sort of templates first .. first+n-1 by time-extent bucket into the
// context's scratch (timed as the binning stage): returns the binned order and
// the per-workgroup key slots that follow it.
template <bool EXPL>
stt_status bin_templates(stt_ctx *c, const MapP &m, const GenP &g, const Trk *tr, int64_t first, int64_t n,
                         const FixedBufs *fb, uint32_t *&order, uint64_t *&wg_keys)
{
    const int wb = bucket_shift(m.T, n);
    const int nb = ((m.T - 1) >> wb) + 1;
    const int nbins = nb * (nb + 1) / 2;
    const size_t n_order = ((size_t)n + 1) & ~(size_t)1;  // keeps the key slots 8-byte aligned
    if (!fb) {
        stt_status s = ensure_scratch(c, score_scratch_bytes(n));
        if (s != STT_OK) return s;
    }
    const int ngroups = (nbins + (1 << kGroupShift) - 1) >> kGroupShift;
    uint32_t *totals = (uint32_t *)(fb ? fb->scratch : c->scratch);
    uint32_t *cursor = totals + kMaxBins;
    const unsigned bgrid = (unsigned)((n + kBinChunk - 1) / kBinChunk);
    uint32_t *gstart = cursor + kMaxBins;
    uint32_t *fitem = gstart + kGroupSlots;
    order = fitem + kGroupSlots;
    wg_keys = (uint64_t *)(order + n_order);
    uint32_t *tmp = (uint32_t *)(wg_keys + (n + 1023) / 1024);
    uint32_t *ccnt = tmp + n_order;  // [group][chunk], ngroups rows of bgrid
    uint8_t *tsub = (uint8_t *)(ccnt + (size_t)kMaxGroups * bgrid);
    uint16_t *bins = (uint16_t *)order;
    ev_attach(c, 2, -1);
    launch_ev(c, k_fill_u32, dim3((nbins + 255) / 256), dim3(256), 0, totals, (int64_t)nbins, 0u);
    hipLaunchKernelGGL(k_bin_count<EXPL>, dim3(bgrid), dim3(256), 0, c->stream, m, g, tr, (uint64_t)first, n, wb,
                       nbins, totals, bins, ccnt);
    hipLaunchKernelGGL(k_bin_scan, dim3(1 + (unsigned)ngroups), dim3(256), 0, c->stream, (const uint32_t *)totals, nbins,
                       cursor, gstart, fitem, ccnt, (int)bgrid);
    hipLaunchKernelGGL(k_bin_group, dim3(bgrid), dim3(kScatterWG), 0, c->stream, n, ngroups, (const uint16_t *)bins,
                       (const uint32_t *)gstart, (const uint32_t *)ccnt, tmp, tsub);
    // a group of c templates has ceil(c / kFineChunk) chunks: at most ceil(n / kFineChunk) + ngroups in all
    ev_attach(c, -1, 3);
    launch_ev(c, k_bin_fine, dim3((unsigned)((n + kFineChunk - 1) / kFineChunk) + (unsigned)ngroups), dim3(kScatterWG), 0,
              nbins, (const uint32_t *)gstart, (const uint32_t *)fitem, cursor, (const uint32_t *)tmp,
              (const uint8_t *)tsub, order);
    STT_HIP(c, hipGetLastError());
    c->used[1] = true;
    return STT_OK;
}

// The scorers of one call on the folded map m (format MAPT: kMapPol or kMapPolH).
template <bool EXPL, int MAPT>
stt_status score_folded(stt_ctx *c, const MapP &m, const GenP &g, const Trk *tr, int64_t first, int64_t n,
                        int32_t norm, float *snr, uint64_t *best, const FixedBufs *fb, bool slab, bool per_wave)
{
    constexpr int esize = (int)sizeof(elem_t<MAPT>);
    stt_status s;
    if (!slab) {
        ev_record(c, 0);
        if (c->hw_trig)
            launch_direct<EXPL, true, MAPT>(c, per_wave, m, g, tr, first, n, norm, snr, best);
        else
            launch_direct<EXPL, false, MAPT>(c, per_wave, m, g, tr, first, n, norm, snr, best);
        STT_HIP(c, hipGetLastError());
        ev_record(c, 1);
        ev_record(c, 5);
        c->used[0] = true;
        return STT_OK;
    }
    uint32_t *order = nullptr;
    uint64_t *wg_keys = nullptr;
    if ((s = bin_templates<EXPL>(c, m, g, tr, first, n, fb, order, wg_keys)) != STT_OK) return s;
    const int64_t ldc = m.ld;
    const int sc = c->dma ? aligned_slab(dma_slab_cols(c, ldc, esize)) : 0;
    if (sc > 0) {
        // aligned slabs of the folded map streamed into LDS with double-buffered DMA
        const size_t shm = 2 * (size_t)esize * (size_t)sc * ldc;
        ev_attach(c, 0, 1);
        s = launch_slab<MAPT>(c, sc, c->slab_wg, c->slab_tpt, m, g, tr, order, first, n, sc, shm, norm, snr, wg_keys);
    } else {
        // one slab buffer, staged through registers (maps too wide for two DMA slabs)
        const int S = std::min<int>(std::min<int>(64, (c->lds_bytes - 256) / (esize * m.F)), m.T);
        const size_t shm = (size_t)esize * (size_t)S * m.F;
        ev_attach(c, 0, 1);
        s = launch_slab<MAPT>(c, 0, c->slab_wg, c->slab_tpt, m, g, tr, order, first, n, S, shm, norm, snr, wg_keys);
    }
    if (s != STT_OK) return s;
    c->used[0] = true;
    if (best) {
        const int64_t n_wg = (n + (int64_t)c->slab_wg * c->slab_tpt - 1) / ((int64_t)c->slab_wg * c->slab_tpt);
        ev_attach(c, -1, 5);
        launch_ev(c, k_reduce_keys, dim3(1), dim3(1024), 0, (const uint64_t *)wg_keys, n_wg, best);
        STT_HIP(c, hipGetLastError());
    } else {
        ev_record(c, 5);
    }
    return STT_OK;
}

template <bool EXPL>
stt_status score_impl(stt_ctx *c, const stt_map *map, const GenP &g, const Trk *tr, int64_t first, int64_t n,
                      int32_t norm, float *snr, uint64_t *best, const FixedBufs *fb = nullptr)
{
    const int F = map->F, esize = fold_esize(map->dtype);
    // the slab plus the kernel's few static LDS words must fit the 160 KB of a CU
    bool slab = (c->lds_bytes - 256) / (esize * F) >= 1;
    if (c->path == 1 || c->path == 3) slab = false;
    if (c->path == 0 && n < 4096) slab = false;
    // without slabs: one wave per template for calls too small to fill the chip lane by lane
    const bool per_wave = c->path == 3 || (c->path == 0 && n < 65536);
    if (c->path == 2 && !slab)
        return fail(c, STT_EUNSUPPORTED, "F=%d too wide for an LDS slab of %d bytes", F, c->lds_bytes);

    stt_status s = ev_begin(c);
    if (s != STT_OK) return s;
    ev_attach(c, 4, -1);  // taken by the fold's launch
    MapP m;
    if ((s = fold_polar(c, map, fb, m)) != STT_OK) return s;
    // score_folded records event 5 at the end of its last kernel
    s = map->dtype == STT_P16 ? score_folded<EXPL, kMapPolH>(c, m, g, tr, first, n, norm, snr, best, fb, slab, per_wave)
                              : score_folded<EXPL, kMapPol>(c, m, g, tr, first, n, norm, snr, best, fb, slab, per_wave);
    if (s != STT_OK) return s;
    c->used[2] = true;
    ev_end(c);
    return STT_OK;
}

// Bytes of the folded copy of a map.
size_t folded_bytes(const stt_map *map)
{
    const int esize = fold_esize(map->dtype);
    return (size_t)esize * (size_t)map->T * (size_t)fold_ld(map->F, esize);
}

stt_status fold_polar(stt_ctx *c, const stt_map *map, const FixedBufs *fb, MapP &mf)
{
    const MapP m = to_mapp(map);
    const int esize = fold_esize(map->dtype);
    const int64_t ldc = fold_ld(m.F, esize);
    if (!fb) {
        const stt_status s = ensure_pbuf(c, folded_bytes(map));
        if (s != STT_OK) return s;
    }
    void *pbuf = fb ? fb->pbuf : c->pbuf;
    const dim3 fg((unsigned)m.T, (unsigned)((ldc + 256 * kFoldRows - 1) / (256 * kFoldRows)));  // one column per x, rows over y
    if (map->dtype == STT_P16)
        launch_ev(c, k_fold_words, fg, dim3(256), 0, m, (uint32_t *)pbuf, (int64_t)ldc);
    else
        launch_ev(c, k_fold_polar<kMapF32>, fg, dim3(256), 0, m, (float2 *)pbuf, (int64_t)ldc);
    STT_HIP(c, hipGetLastError());
    mf = m;  // an FP16 map keeps its scale 2^e
    mf.Y = (const float2 *)pbuf;
    mf.sig = nullptr;
    mf.ld = ldc;
    return STT_OK;
}

// The delay grid in launches of kMD delays. Slabs (binned templates, folded map,
// LDS-DMA) from 4096 templates on when two slabs of a column fit; otherwise one
// lane per template with direct gathers. Both give bit-identical results.
template <bool EXPL, int MAPT>
stt_status maxdelay_folded(stt_ctx *c, const MapP &mf, const GenP &g, const Trk *tr, int64_t first, int64_t n,
                           int32_t d0, int32_t step, int32_t n_tau, int32_t norm, float *snr, int32_t *tidx,
                           uint64_t *best, bool slab, int lds)
{
    // 1024 lanes x 1 template, at most 80 KB of slabs (measured on the search map: 512 x 2, 1024 x 2,
    // 256 x 4 and smaller slabs were 15-75 % slower; one template per lane leaves room for more waves)
    constexpr int kMdWG = 1024, kMdTPT = 1;
    constexpr int esize = (int)sizeof(elem_t<MAPT>);
    const int64_t ldc = mf.ld;
    const int n_launch = (n_tau + kMD - 1) / kMD;
    stt_status s;
    if (!slab) {
        ev_record(c, 0);
        const unsigned grid = (unsigned)((n + kWG - 1) / kWG);
        for (int l = 0; l < n_launch; ++l) {
            const int32_t m0 = l * kMD, cnt = std::min(kMD, n_tau - m0), last = l == n_launch - 1;
            if (c->hw_trig)
                hipLaunchKernelGGL((k_score_md_direct<EXPL, true, MAPT>), dim3(grid), dim3(kWG), 0, c->stream, mf, g,
                                   tr, (uint64_t)first, n, norm, d0, step, m0, cnt, last, snr, tidx, best);
            else
                hipLaunchKernelGGL((k_score_md_direct<EXPL, false, MAPT>), dim3(grid), dim3(kWG), 0, c->stream, mf,
                                   g, tr, (uint64_t)first, n, norm, d0, step, m0, cnt, last, snr, tidx, best);
        }
        STT_HIP(c, hipGetLastError());
        ev_record(c, 1);
        c->used[0] = true;
        return STT_OK;
    }
    uint32_t *order = nullptr;
    uint64_t *wg_keys = nullptr;
    if ((s = bin_templates<EXPL>(c, mf, g, tr, first, n, nullptr, order, wg_keys)) != STT_OK) return s;
    const int S = std::min(dma_slab_cols(lds, ldc, esize), mf.T);
    const size_t shm = 2 * (size_t)esize * (size_t)S * ldc;
    const unsigned grid = (unsigned)((n + kMdWG * kMdTPT - 1) / (kMdWG * kMdTPT));
    auto kh = k_score_md_slab<kMdWG, kMdTPT, EXPL, true, MAPT>;
    auto kp = k_score_md_slab<kMdWG, kMdTPT, EXPL, false, MAPT>;
    auto kern = c->hw_trig ? kh : kp;
    if (shm > 64 * 1024)
        STT_HIP(c, hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    ev_record(c, 0);
    for (int l = 0; l < n_launch; ++l) {
        const int32_t m0 = l * kMD, cnt = std::min(kMD, n_tau - m0), last = l == n_launch - 1;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kMdWG), shm, c->stream, mf, g, tr, (const uint32_t *)order,
                           (uint64_t)first, n, S, norm, d0, step, m0, cnt, last, snr, tidx, wg_keys);
    }
    STT_HIP(c, hipGetLastError());
    ev_record(c, 1);
    c->used[0] = true;
    if (best) {
        hipLaunchKernelGGL(k_reduce_keys, dim3(1), dim3(1024), 0, c->stream, (const uint64_t *)wg_keys, (int64_t)grid,
                           best);
        STT_HIP(c, hipGetLastError());
    }
    return STT_OK;
}

template <bool EXPL>
stt_status maxdelay_impl(stt_ctx *c, const stt_map *map, const GenP &g, const Trk *tr, int64_t first, int64_t n,
                         int32_t d0, int32_t step, int32_t n_tau, int32_t norm, float *snr, int32_t *tidx,
                         uint64_t *best)
{
    const int lds = std::min(c->lds_bytes, 80 * 1024);
    const int esize = fold_esize(map->dtype);
    const int64_t ldc = fold_ld(map->F, esize);
    bool slab = c->dma && dma_slab_cols(lds, ldc, esize) >= 1 && c->path != 1 && c->path != 3 &&
                (c->path == 2 || n >= 4096);
    if (c->path == 2 && !slab)
        return fail(c, STT_EUNSUPPORTED, "F=%d too wide for two LDS slabs of %d bytes", map->F, lds);
    stt_status s;
    if (!snr || !tidx) {
        if ((s = ensure_mdbuf(c, (sizeof(float) + sizeof(int32_t)) * (size_t)n)) != STT_OK) return s;
        if (!snr) snr = (float *)c->mdbuf;
        if (!tidx) tidx = (int32_t *)((float *)c->mdbuf + n);
    }
    if ((s = ev_begin(c)) != STT_OK) return s;
    ev_record(c, 4);
    MapP mf;
    if ((s = fold_polar(c, map, nullptr, mf)) != STT_OK) return s;
    s = map->dtype == STT_P16
            ? maxdelay_folded<EXPL, kMapPolH>(c, mf, g, tr, first, n, d0, step, n_tau, norm, snr, tidx, best, slab, lds)
            : maxdelay_folded<EXPL, kMapPol>(c, mf, g, tr, first, n, d0, step, n_tau, norm, snr, tidx, best, slab, lds);
    if (s != STT_OK) return s;
    ev_record(c, 5);
    c->used[2] = true;
    ev_end(c);
    return STT_OK;
}

// The free-t_mid scorers of one call on the folded map mf (format MAPT).
template <int MAPT>
stt_status score_tm_folded(stt_ctx *c, const MapP &mf, const GenP &g, const TrkTm *tr, int64_t first, int64_t n,
                           int32_t norm, float *snr_dev, uint64_t *best_key_dev, bool slab, int lds)
{
    constexpr int kTmWG = 1024, kTmTPT = 1;
    constexpr int esize = (int)sizeof(elem_t<MAPT>);
    stt_status s;
    if (slab) {
        uint32_t *order = nullptr;
        uint64_t *wg_keys = nullptr;
        if ((s = bin_templates<false>(c, mf, g, nullptr, first, n, nullptr, order, wg_keys)) != STT_OK) return s;
        const int S = std::min(dma_slab_cols(lds, mf.ld, esize), mf.T);
        const size_t shm = 2 * (size_t)esize * (size_t)S * mf.ld;
        const unsigned grid = (unsigned)((n + kTmWG * kTmTPT - 1) / (kTmWG * kTmTPT));
        auto kern = c->hw_trig ? k_score_tm_slab<kTmWG, kTmTPT, true, MAPT> : k_score_tm_slab<kTmWG, kTmTPT, false, MAPT>;
        if (shm > 64 * 1024)
            STT_HIP(c, hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
        ev_record(c, 0);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kTmWG), shm, c->stream, mf, g, (const uint32_t *)order,
                           (uint64_t)first, n, S, norm, snr_dev, wg_keys);
        STT_HIP(c, hipGetLastError());
        ev_record(c, 1);
        c->used[0] = true;
        if (best_key_dev) {
            hipLaunchKernelGGL(k_reduce_keys, dim3(1), dim3(1024), 0, c->stream, (const uint64_t *)wg_keys,
                               (int64_t)grid, best_key_dev);
            STT_HIP(c, hipGetLastError());
        }
        return STT_OK;
    }
    const dim3 grid((unsigned)((n + 3) / 4)), block(256);
    ev_record(c, 0);
#define STT_TM_LAUNCH(E, H)                                                                                     \
    hipLaunchKernelGGL((k_score_tm<E, H, MAPT>), grid, block, 0, c->stream, mf, g, tr, (uint64_t)first, n, norm, \
                       snr_dev, best_key_dev)
    if (tr) {
        if (c->hw_trig) STT_TM_LAUNCH(true, true); else STT_TM_LAUNCH(true, false);
    } else {
        if (c->hw_trig) STT_TM_LAUNCH(false, true); else STT_TM_LAUNCH(false, false);
    }
#undef STT_TM_LAUNCH
    STT_HIP(c, hipGetLastError());
    ev_record(c, 1);
    c->used[0] = true;
    return STT_OK;
}

// Twiddles e^{-2 pi i j / M} (j < M/2) then the periodic Hann window sin^2(pi n / M) (n < M),
// evaluated in FP64 and rounded once; rewritten (after the stream drains) when M changes.
stt_status ensure_fft_tab(stt_ctx *c, int M)
{
    if (c->fft_tab && c->fft_M == M) return STT_OK;
    const int N = M / 2;
    std::vector<float> h((size_t)2 * N + M);
    for (int j = 0; j < N; ++j) {
        const double a = 2.0 * M_PI * (double)j / (double)M;
        h[2 * j] = (float)std::cos(a);
        h[2 * j + 1] = (float)-std::sin(a);
    }
    for (int n = 0; n < M; ++n) {
        const double v = std::sin(M_PI * (double)n / (double)M);
        h[(size_t)2 * N + n] = (float)(v * v);
    }
    if (!c->fft_tab) {
        const size_t most = sizeof(float) * (size_t)2 * kMaxFftM;  // room for the largest M
        if (hipMalloc(&c->fft_tab, most) != hipSuccess) {
            (void)hipGetLastError();
            c->fft_tab = nullptr;
            return fail(c, STT_ENOMEM, "cannot allocate the FFT table");
        }
    }
    STT_HIP(c, hipStreamSynchronize(c->stream));  // earlier transforms may still read the old table
    STT_HIP(c, hipMemcpy(c->fft_tab, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice));
    c->fft_M = M;
    return STT_OK;
}

stt_status check_spectro(stt_ctx *c, const stt_spectro *p)
{
    if (!p) return fail(c, STT_EINVAL, "null spectrogram parameters");
    if (!(p->fs > 0) || !std::isfinite(p->fs)) return fail(c, STT_EINVAL, "fs must be positive");
    if (p->M < 8 || p->M > kMaxFftM || (p->M & (p->M - 1)))
        return fail(c, STT_ERANGE, "M=%d: need a power of two in [8, %d]", p->M, kMaxFftM);
    if (p->k_lo < 0 || p->F < 1 || (int64_t)p->k_lo + p->F > p->M / 2)
        return fail(c, STT_ERANGE, "bins [%d, %d) outside [0, M/2)", p->k_lo, p->k_lo + p->F);
    if (p->nb < 1) return fail(c, STT_EINVAL, "nb=%d: need >= 1", p->nb);
    return STT_OK;
}

// 2 / Nrm with Nrm = M dt 3/8 (the Hann window's mean square)
float cross_scale(const stt_spectro *p) { return (float)(2.0 / ((double)p->M / p->fs * 0.375)); }

}  // namespace

extern "C" {

const char *stt_strerror(stt_status s)
{
    switch (s) {
    case STT_OK: return "ok";
    case STT_EINVAL: return "invalid argument";
    case STT_ERANGE: return "size out of supported range";
    case STT_ENOMEM: return "out of device memory";
    case STT_EHIP: return "HIP runtime error";
    case STT_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char *stt_last_error(const stt_ctx *c) { return c ? c->err.c_str() : "no context"; }

stt_status stt_create(int device, void *hip_stream, stt_ctx **out)
{
    if (!out) return STT_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return STT_EHIP;
    if (hipSetDevice(device) != hipSuccess) return STT_EHIP;
    stt_ctx *c = new stt_ctx;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    // the fixed scratch of stt_score_noalloc on this device (that call fails cleanly without it)
    (void)na_init(device);
    *out = c;
    return STT_OK;
}

stt_status stt_destroy(stt_ctx *c)
{
    if (!c) return STT_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->scratch) (void)hipFree(c->scratch);
    if (c->aux) (void)hipFree(c->aux);
    if (c->pbuf) (void)hipFree(c->pbuf);
    if (c->mdbuf) (void)hipFree(c->mdbuf);
    if (c->bdev) (void)hipFree(c->bdev);
    if (c->fft_tab) (void)hipFree(c->fft_tab);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (auto &e : c->pool) (void)hipEventDestroy(e);
    delete c;
    return STT_OK;
}

stt_status stt_set_stream(stt_ctx *c, void *hip_stream)
{
    if (!c) return STT_EINVAL;
    c->stream = (hipStream_t)hip_stream;
    return STT_OK;
}

stt_status stt_sync(stt_ctx *c)
{
    if (!c) return STT_EINVAL;
    STT_HIP(c, hipStreamSynchronize(c->stream));
    return STT_OK;
}

stt_status stt_reserve(stt_ctx *c, int64_t max_tracks)
{
    if (!c || max_tracks < 0) return fail(c, STT_EINVAL, "bad reserve request");
    return ensure_scratch(c, score_scratch_bytes(max_tracks));
}

stt_status stt_set_timing(stt_ctx *c, int32_t on)
{
    if (!c) return STT_EINVAL;
    c->timing = on != 0;
    c->recs.clear();
    c->next = c->last = 0;
    return STT_OK;
}

static const int kEvPair[3] = {0, 2, 4};  // start event of each stage within a call's six

stt_status stt_kernel_ms(stt_ctx *c, int32_t which, float *ms)
{
    if (!c || !ms || which < 0 || which > 2) return fail(c, STT_EINVAL, "bad timing query");
    if (!c->timing || c->recs.empty() || !c->recs.back().used[which])
        return fail(c, STT_EINVAL, "no timed stage %d in the last call", which);
    STT_HIP(c, hipStreamSynchronize(c->stream));
    const size_t a = c->recs.back().base + kEvPair[which];
    STT_HIP(c, hipEventElapsedTime(ms, c->pool[a], c->pool[a + 1]));
    return STT_OK;
}

stt_status stt_kernel_ms_total(stt_ctx *c, int32_t which, double *total_ms, int32_t *count)
{
    if (!c || !total_ms || !count || which < 0 || which > 2) return fail(c, STT_EINVAL, "bad timing query");
    if (!c->timing) return fail(c, STT_EINVAL, "timing is off");
    STT_HIP(c, hipStreamSynchronize(c->stream));
    double tot = 0.0;
    int32_t n = 0;
    for (const auto &r : c->recs) {
        if (!r.used[which]) continue;
        float ms = 0.0f;
        const size_t a = r.base + kEvPair[which];
        STT_HIP(c, hipEventElapsedTime(&ms, c->pool[a], c->pool[a + 1]));
        tot += ms;
        ++n;
    }
    *total_ms = tot;
    *count = n;
    c->recs.clear();
    c->next = c->last = 0;
    return STT_OK;
}

// Internal knob used by tests and tuning: 0 auto, 1 direct gathers, 2 LDS slabs.
stt_status stt_set_path(stt_ctx *c, int32_t path, int32_t lds_bytes)
{
    if (!c || path < 0 || path > 3) return STT_EINVAL;
    if (lds_bytes != 0 && (lds_bytes < 1024 || lds_bytes > 160 * 1024))
        return fail(c, STT_ERANGE, "lds_bytes=%d outside [1024, 163840]", lds_bytes);
    c->path = path;
    if (lds_bytes) c->lds_bytes = lds_bytes;
    return STT_OK;
}

stt_status stt_set_slab_shape(stt_ctx *c, int32_t wg, int32_t tpt)
{
    if (!c) return STT_EINVAL;
    if (!slab_shape_ok(wg, tpt)) return fail(c, STT_EUNSUPPORTED, "no slab scorer for %d x %d", wg, tpt);
    c->slab_wg = wg;
    c->slab_tpt = tpt;
    return STT_OK;
}

stt_status stt_set_staging(stt_ctx *c, int32_t dma)
{
    if (!c || dma < 0 || dma > 1) return STT_EINVAL;
    c->dma = dma == 1;
    return STT_OK;
}

stt_status stt_set_trig(stt_ctx *c, int32_t hw)
{
    if (!c || hw < 0 || hw > 1) return STT_EINVAL;
    c->hw_trig = hw == 1;
    return STT_OK;
}

stt_status stt_make_tracks(stt_ctx *c, const stt_gen *gen, int32_t T, int32_t F, int64_t first, int64_t n,
                           stt_track *out_dev)
{
    if (!c) return STT_EINVAL;
    GenP g;
    stt_status s = make_genp(c, gen, T, F, g);
    if (s != STT_OK) return s;
    if ((s = check_range(c, first, n)) != STT_OK) return s;
    if (n == 0) return STT_OK;
    if (!out_dev) return fail(c, STT_EINVAL, "out_dev is NULL");
    STT_HIP(c, hipSetDevice(c->device));
    const unsigned grid = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_make_tracks, dim3(grid), dim3(256), 0, c->stream, g, (uint64_t)first, n, (Trk *)out_dev);
    STT_HIP(c, hipGetLastError());
    return STT_OK;
}

stt_status stt_score(stt_ctx *c, const stt_map *map, const stt_gen *gen, const stt_track *tracks_dev, int64_t first,
                     int64_t n, int32_t norm, float *snr_dev, uint64_t *best_key_dev)
{
    if (!c) return STT_EINVAL;
    stt_status s = check_map(c, map);
    if (s != STT_OK) return s;
    if ((s = check_range(c, first, n)) != STT_OK) return s;
    if (norm != STT_NORM_SQRT_N && norm != STT_NORM_N) return fail(c, STT_EINVAL, "norm=%d", norm);
    GenP g{};
    if (!tracks_dev) {
        if ((s = make_genp(c, gen, map->T, map->F, g)) != STT_OK) return s;
    }
    if (n == 0) return STT_OK;
    STT_HIP(c, hipSetDevice(c->device));
    if (tracks_dev)
        return score_impl<true>(c, map, g, (const Trk *)tracks_dev, first, n, norm, snr_dev, best_key_dev);
    return score_impl<false>(c, map, g, nullptr, first, n, norm, snr_dev, best_key_dev);
}

stt_status stt_score_noalloc(stt_ctx *c, const stt_map *map, const stt_gen *gen, const stt_track *tracks_dev,
                             int64_t first, int64_t n, int32_t norm, float *snr_dev, uint64_t *best_key_dev)
{
    if (!c) return STT_EINVAL;
    stt_status s = check_map(c, map);
    if (s != STT_OK) return s;
    if ((s = check_range(c, first, n)) != STT_OK) return s;
    if (norm != STT_NORM_SQRT_N && norm != STT_NORM_N) return fail(c, STT_EINVAL, "norm=%d", norm);
    if (n > kNaMaxTracks)
        return fail(c, STT_ERANGE, "n=%lld exceeds the %lld templates of the fixed scratch", (long long)n,
                    (long long)kNaMaxTracks);
    const size_t map_bytes = folded_bytes(map);
    if (map_bytes > kNaMapBytes)
        return fail(c, STT_ERANGE, "the folded %dx%d map needs %zu bytes; the fixed scratch holds %zu", map->T,
                    map->F, map_bytes, kNaMapBytes);
    GenP g{};
    if (!tracks_dev) {
        if ((s = make_genp(c, gen, map->T, map->F, g)) != STT_OK) return s;
    }
    if (n == 0) return STT_OK;
    STT_HIP(c, hipSetDevice(c->device));
    void *base = na_ptr(c->device);
    if (!base) return fail(c, STT_EHIP, "no fixed scratch on device %d (hipGetSymbolAddress failed)", c->device);
    const FixedBufs fb{(unsigned char *)base + kNaMapBytes, base};
    // no timing events either: the event pool grows by allocation
    const bool timing = c->timing;
    c->timing = false;
    if (tracks_dev)
        s = score_impl<true>(c, map, g, (const Trk *)tracks_dev, first, n, norm, snr_dev, best_key_dev, &fb);
    else
        s = score_impl<false>(c, map, g, nullptr, first, n, norm, snr_dev, best_key_dev, &fb);
    c->timing = timing;
    return s;
}

stt_status stt_score_maxdelay(stt_ctx *c, const stt_map *map, const stt_gen *gen, const stt_track *tracks_dev,
                              int64_t first, int64_t n, int32_t dtau0, int32_t dtau_step, int32_t n_tau, int32_t norm,
                              float *snr_dev, int32_t *tau_idx_dev, uint64_t *best_key_dev)
{
    if (!c) return STT_EINVAL;
    stt_status s = check_map(c, map);
    if (s != STT_OK) return s;
    if ((s = check_range(c, first, n)) != STT_OK) return s;
    if (norm != STT_NORM_SQRT_N && norm != STT_NORM_N) return fail(c, STT_EINVAL, "norm=%d", norm);
    if (n_tau < 1 || n_tau > 65536) return fail(c, STT_ERANGE, "n_tau=%d outside [1, 65536]", n_tau);
    const int64_t dlast = (int64_t)dtau0 + (int64_t)(n_tau - 1) * dtau_step;
    const int64_t dlim = ((int64_t)1 << 30) - 1;
    if (dtau0 < -dlim || dtau0 > dlim || dlast < -dlim || dlast > dlim)
        return fail(c, STT_ERANGE, "delay grid %d + m*%d (m < %d) leaves (-2^30, 2^30)", dtau0, dtau_step, n_tau);
    GenP g{};
    if (!tracks_dev) {
        if ((s = make_genp(c, gen, map->T, map->F, g)) != STT_OK) return s;
    }
    if (n == 0) return STT_OK;
    STT_HIP(c, hipSetDevice(c->device));
    const Trk *tr = (const Trk *)tracks_dev;
    if (tracks_dev)
        return maxdelay_impl<true>(c, map, g, tr, first, n, dtau0, dtau_step, n_tau, norm, snr_dev, tau_idx_dev,
                                   best_key_dev);
    return maxdelay_impl<false>(c, map, g, nullptr, first, n, dtau0, dtau_step, n_tau, norm, snr_dev, tau_idx_dev,
                                best_key_dev);
}

stt_status stt_make_tracks_tm(stt_ctx *c, const stt_gen *gen, int32_t T, int32_t F, int64_t first, int64_t n,
                              stt_track_tm *out_dev)
{
    if (!c) return STT_EINVAL;
    stt_status s = check_range(c, first, n);
    if (s != STT_OK) return s;
    GenP g;
    if ((s = make_genp(c, gen, T, F, g)) != STT_OK) return s;
    if (n == 0) return STT_OK;
    if (!out_dev) return fail(c, STT_EINVAL, "out_dev is NULL");
    STT_HIP(c, hipSetDevice(c->device));
    hipLaunchKernelGGL(k_make_tracks_tm, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, g,
                       (uint64_t)first, n, (TrkTm *)out_dev);
    STT_HIP(c, hipGetLastError());
    return STT_OK;
}

stt_status stt_score_tm(stt_ctx *c, const stt_map *map, const stt_gen *gen, const stt_track_tm *tracks_dev,
                        int64_t first, int64_t n, int32_t norm, float *snr_dev, uint64_t *best_key_dev)
{
    if (!c) return STT_EINVAL;
    stt_status s = check_map(c, map);
    if (s != STT_OK) return s;
    if ((s = check_range(c, first, n)) != STT_OK) return s;
    if (norm != STT_NORM_SQRT_N && norm != STT_NORM_N) return fail(c, STT_EINVAL, "norm=%d", norm);
    GenP g{};
    if (!tracks_dev) {
        if ((s = make_genp(c, gen, map->T, map->F, g)) != STT_OK) return s;
    }
    if (n == 0) return STT_OK;
    STT_HIP(c, hipSetDevice(c->device));
    // generated templates: binned by time extent (a free t_mid keeps it) and scored from LDS slabs
    // (1024 lanes x 1 template, at most 80 KB of slabs) when a column fits; otherwise one wave each
    const int lds = std::min(c->lds_bytes, 80 * 1024);
    const int esize = fold_esize(map->dtype);
    const int64_t ldc = fold_ld(map->F, esize);
    const bool slab = !tracks_dev && c->dma && dma_slab_cols(lds, ldc, esize) >= 1 && c->path != 1 && c->path != 3 &&
                      (c->path == 2 || n >= 4096);
    if ((s = ev_begin(c)) != STT_OK) return s;
    ev_record(c, 4);
    MapP mf;
    if ((s = fold_polar(c, map, nullptr, mf)) != STT_OK) return s;
    s = map->dtype == STT_P16
            ? score_tm_folded<kMapPolH>(c, mf, g, (const TrkTm *)tracks_dev, first, n, norm, snr_dev, best_key_dev,
                                        slab, lds)
            : score_tm_folded<kMapPol>(c, mf, g, (const TrkTm *)tracks_dev, first, n, norm, snr_dev, best_key_dev,
                                       slab, lds);
    if (s != STT_OK) return s;
    ev_record(c, 5);
    c->used[2] = true;
    ev_end(c);
    return STT_OK;
}

stt_status stt_argmax(stt_ctx *c, const float *snr_dev, int64_t n, int64_t first, uint64_t *best_key_dev)
{
    if (!c) return STT_EINVAL;
    stt_status s = check_range(c, first, n);
    if (s != STT_OK) return s;
    if (n == 0) return STT_OK;
    if (!snr_dev || !best_key_dev) return fail(c, STT_EINVAL, "snr_dev and best_key_dev must be non-NULL");
    STT_HIP(c, hipSetDevice(c->device));
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_argmax, dim3((unsigned)blocks), dim3(256), 0, c->stream, snr_dev, n, (uint64_t)first,
                       best_key_dev);
    STT_HIP(c, hipGetLastError());
    return STT_OK;
}

stt_status stt_map_pack_p16(stt_ctx *c, const stt_map *map, void *out_dev, int64_t out_ld, int32_t *scale_exp)
{
    if (!c) return STT_EINVAL;
    stt_status s = check_map(c, map);
    if (s != STT_OK) return s;
    if (map->dtype != STT_C64F32) return fail(c, STT_EINVAL, "stt_map_pack_p16 packs an FP32 (Y, sigma) map");
    if (!out_dev || !scale_exp) return fail(c, STT_EINVAL, "out_dev and scale_exp must be non-NULL");
    if (out_ld < map->F) return fail(c, STT_EINVAL, "out_ld=%lld < F=%d", (long long)out_ld, map->F);
    STT_HIP(c, hipSetDevice(c->device));
    if ((s = ensure_aux(c, sizeof(TopkState))) != STT_OK) return s;
    unsigned long long *amax = (unsigned long long *)c->aux;
    const MapP m = to_mapp(map);
    const int64_t n = (int64_t)map->T * map->F;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, c->stream, (uint32_t *)amax, (int64_t)2, 0u);
    hipLaunchKernelGGL(k_absmax_p, dim3(grid), dim3(256), 0, c->stream, m, amax);
    STT_HIP(c, hipGetLastError());
    unsigned long long bits = 0;
    STT_HIP(c, hipMemcpyAsync(&bits, amax, sizeof bits, hipMemcpyDeviceToHost, c->stream));
    STT_HIP(c, hipStreamSynchronize(c->stream));
    double amaxd;
    std::memcpy(&amaxd, &bits, sizeof amaxd);
    if (!std::isfinite(amaxd)) return fail(c, STT_EINVAL, "map holds a non-finite Y/sigma");
    // e = ceil(log2(max |p|)) - 15, exactly: with max = fr 2^k, fr in [1/2, 1), the ceiling is k
    // unless fr = 1/2 (a power of two, its own ceiling k - 1)
    int e = 0;
    if (amaxd > 0.0) {
        int k = 0;
        const double fr = std::frexp(amaxd, &k);
        e = (fr > 0.5 ? k : k - 1) - 15;
    }
    hipLaunchKernelGGL(k_pack_p16, dim3(grid), dim3(256), 0, c->stream, m, std::ldexp(1.0, -e), (uint32_t *)out_dev,
                       out_ld);
    STT_HIP(c, hipGetLastError());
    *scale_exp = e;
    return STT_OK;
}

stt_status stt_topk(stt_ctx *c, const float *snr_dev, int64_t n, int64_t first, int32_t K, int64_t *idx_dev,
                    float *val_dev)
{
    if (!c) return STT_EINVAL;
    stt_status s = check_range(c, first, n);
    if (s != STT_OK) return s;
    if (K < 0 || K > n || K > 8192) return fail(c, STT_ERANGE, "K=%d must be in [0, min(n, 8192)]", K);
    if (K == 0) return STT_OK;
    if (!snr_dev || (!idx_dev && !val_dev)) return fail(c, STT_EINVAL, "snr_dev and an output must be non-NULL");
    STT_HIP(c, hipSetDevice(c->device));
    const size_t st_bytes = (sizeof(TopkState) + 255) & ~(size_t)255;
    if ((s = ensure_aux(c, st_bytes + sizeof(uint64_t) * (size_t)K)) != STT_OK) return s;
    TopkState *st = (TopkState *)c->aux;
    uint64_t *cand = (uint64_t *)((char *)c->aux + st_bytes);
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_topk_init, dim3(1), dim3(256), 0, c->stream, st, (uint32_t)K);
    for (int shift = 56; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_topk_hist, dim3(grid), dim3(256), 0, c->stream, snr_dev, n, (uint64_t)first, st, shift);
        hipLaunchKernelGGL(k_topk_pick, dim3(1), dim3(256), 0, c->stream, st, shift);
    }
    hipLaunchKernelGGL(k_topk_gather, dim3(grid), dim3(256), 0, c->stream, snr_dev, n, (uint64_t)first, st, cand,
                       (uint32_t)K);
    int P = 1;
    while (P < K) P <<= 1;
    hipLaunchKernelGGL(k_topk_sort, dim3(1), dim3(1024), sizeof(uint64_t) * P, c->stream, (const uint64_t *)cand, K,
                       P, idx_dev, val_dev);
    STT_HIP(c, hipGetLastError());
    return STT_OK;
}

stt_status stt_rescore_f64(stt_ctx *c, const stt_map *map, const stt_gen *gen, const stt_track *tracks_dev,
                           int64_t n_tracks, int64_t first, const int64_t *idx_dev, int32_t K, int32_t norm,
                           double *z_dev)
{
    if (!c) return STT_EINVAL;
    stt_status s = check_map(c, map);
    if (s != STT_OK) return s;
    if (map->dtype != STT_C64F32) return fail(c, STT_EINVAL, "the FP64 re-score reads an FP32 (Y, sigma) map");
    if (norm != STT_NORM_SQRT_N && norm != STT_NORM_N) return fail(c, STT_EINVAL, "norm=%d", norm);
    if (K < 0) return fail(c, STT_EINVAL, "K=%d", K);
    if (first < 0) return fail(c, STT_EINVAL, "first=%lld", (long long)first);
    if (tracks_dev && n_tracks < 0) return fail(c, STT_EINVAL, "n_tracks=%lld", (long long)n_tracks);
    GenP g{};
    if (!tracks_dev && (s = make_genp(c, gen, map->T, map->F, g)) != STT_OK) return s;
    if (K == 0) return STT_OK;
    if (!idx_dev || !z_dev) return fail(c, STT_EINVAL, "idx_dev and z_dev must be non-NULL");
    STT_HIP(c, hipSetDevice(c->device));
    const MapP m = to_mapp(map);
    const unsigned grid = (unsigned)(((int64_t)K * 64 + 255) / 256);
    if (tracks_dev)
        hipLaunchKernelGGL(k_rescore_f64<true>, dim3(grid), dim3(256), 0, c->stream, m, g, (const Trk *)tracks_dev,
                           n_tracks, (uint64_t)first, idx_dev, K, norm, z_dev);
    else
        hipLaunchKernelGGL(k_rescore_f64<false>, dim3(grid), dim3(256), 0, c->stream, m, g, (const Trk *)nullptr,
                           (int64_t)0, (uint64_t)first, idx_dev, K, norm, z_dev);
    STT_HIP(c, hipGetLastError());
    return STT_OK;
}

// ----------------------------------------------------------------------------- batches

stt_status stt_significance(stt_ctx *c, const uint64_t *bg_keys_dev, int64_t n_bg, const uint64_t *fg_keys_dev,
                            int64_t n_fg, double alpha, int64_t *n_louder_dev, float *fap_dev, float *z_alpha_dev)
{
    if (!c) return STT_EINVAL;
    if (n_bg < 1) return fail(c, STT_EINVAL, "need at least one background map");
    if (n_fg < 0) return fail(c, STT_EINVAL, "n_fg=%lld", (long long)n_fg);
    if (!bg_keys_dev) return fail(c, STT_EINVAL, "null background keys");
    if (n_fg > 0 && !fg_keys_dev && (n_louder_dev || fap_dev)) return fail(c, STT_EINVAL, "null foreground keys");
    if (n_bg > ((int64_t)1 << 38) || n_fg > ((int64_t)1 << 38))
        return fail(c, STT_ERANGE, "more than 2^38 keys");  // keeps the 1-D grids below 2^31 workgroups
    int32_t m = 0;
    if (z_alpha_dev) {
        if (!(alpha > 0.0 && alpha <= 1.0)) return fail(c, STT_EINVAL, "alpha must be in (0, 1]");
        const double mm = std::max(1.0, std::ceil(alpha * (double)n_bg));
        if (mm > 8192) return fail(c, STT_ERANGE, "ceil(alpha n_bg) = %.0f exceeds 8192", mm);
        m = (int32_t)mm;
    }
    STT_HIP(c, hipSetDevice(c->device));
    stt_status s;
    if (n_fg > 0 && (n_louder_dev || fap_dev)) {
        hipLaunchKernelGGL(k_count_louder, dim3((unsigned)((n_fg + 255) / 256)), dim3(256), 0, c->stream, bg_keys_dev,
                           n_bg, fg_keys_dev, n_fg, n_louder_dev, fap_dev, (double)n_bg);
        STT_HIP(c, hipGetLastError());
    }
    if (z_alpha_dev) {
        // the m-th largest background score: decode the keys, select the top m, keep the last
        if ((s = ensure_mdbuf(c, sizeof(float) * ((size_t)n_bg + (size_t)m))) != STT_OK) return s;
        float *scores = (float *)c->mdbuf;
        float *top = scores + n_bg;
        hipLaunchKernelGGL(k_key_scores, dim3((unsigned)((n_bg + 255) / 256)), dim3(256), 0, c->stream, bg_keys_dev,
                           n_bg, scores);
        STT_HIP(c, hipGetLastError());
        if ((s = stt_topk(c, scores, n_bg, 0, m, nullptr, top)) != STT_OK) return s;
        STT_HIP(c, hipMemcpyAsync(z_alpha_dev, top + (m - 1), sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    }
    return STT_OK;
}

stt_status stt_follow_up(stt_ctx *c, const stt_map *maps_host, int32_t n_maps, uint64_t *keys_dev, const stt_gen *gen,
                         int64_t n_deep, int32_t k, int32_t norm, int32_t *chosen_host, int32_t *n_chosen)
{
    if (!c) return STT_EINVAL;
    if (n_chosen) *n_chosen = 0;
    if (n_maps < 1 || !maps_host || !keys_dev) return fail(c, STT_EINVAL, "need at least one map and its key");
    if (k < 1) return fail(c, STT_EINVAL, "k=%d must be >= 1", k);
    if (!gen) return fail(c, STT_EINVAL, "gen is NULL");
    if (norm != STT_NORM_SQRT_N && norm != STT_NORM_N) return fail(c, STT_EINVAL, "norm=%d", norm);
    stt_status s;
    if ((s = check_range(c, 0, n_deep)) != STT_OK) return s;
    if ((uint64_t)gen->stream + (uint64_t)(n_maps - 1) > 0xFFFFFFFFull)
        return fail(c, STT_ERANGE, "Philox streams gen->stream + m overflow 32 bits");
    for (int32_t m = 0; m < n_maps; ++m) {
        if ((s = check_map(c, &maps_host[m])) != STT_OK) return s;
        GenP g;
        if ((s = make_genp(c, gen, maps_host[m].T, maps_host[m].F, g)) != STT_OK) return s;
    }
    STT_HIP(c, hipSetDevice(c->device));
    // rank of map m = the number of maps at least as loud, itself included (as stt_significance counts)
    if ((s = ensure_aux(c, sizeof(int64_t) * (size_t)n_maps)) != STT_OK) return s;
    int64_t *rank_dev = (int64_t *)c->aux;
    hipLaunchKernelGGL(k_count_louder, dim3((unsigned)((n_maps + 255) / 256)), dim3(256), 0, c->stream,
                       (const uint64_t *)keys_dev, (int64_t)n_maps, (const uint64_t *)keys_dev, (int64_t)n_maps,
                       rank_dev, (float *)nullptr, 1.0);
    STT_HIP(c, hipGetLastError());
    std::vector<int64_t> rank((size_t)n_maps);
    STT_HIP(c, hipMemcpyAsync(rank.data(), rank_dev, sizeof(int64_t) * (size_t)n_maps, hipMemcpyDeviceToHost,
                              c->stream));
    STT_HIP(c, hipStreamSynchronize(c->stream));
    int32_t done = 0;
    for (int32_t m = 0; m < n_maps; ++m) {
        if (rank[(size_t)m] > k) continue;
        if (n_deep > 0) {
            stt_gen gm = *gen;
            gm.stream = gen->stream + (uint32_t)m;
            if ((s = stt_score(c, &maps_host[m], &gm, nullptr, 0, n_deep, norm, nullptr, keys_dev + m)) != STT_OK)
                return s;
        }
        if (chosen_host) chosen_host[done] = m;
        ++done;
        if (n_chosen) *n_chosen = done;
    }
    return STT_OK;
}

stt_status stt_spectra(stt_ctx *c, const stt_spectro *p, const float *strain_dev, int64_t n_samples, int32_t T,
                       float *spec_dev, float *psd_dev)
{
    if (!c) return STT_EINVAL;
    stt_status s = check_spectro(c, p);
    if (s != STT_OK) return s;
    if (!strain_dev || !spec_dev || !psd_dev) return fail(c, STT_EINVAL, "null buffer");
    if (((uintptr_t)strain_dev & 7) || ((uintptr_t)spec_dev & 7) || ((uintptr_t)psd_dev & 3))
        return fail(c, STT_EINVAL, "strain and spec must be 8-byte aligned, psd 4-byte aligned");
    if (T < 4 || T > 65535) return fail(c, STT_ERANGE, "T=%d: need 4 <= T <= 65535", T);
    if (n_samples < 0 || (int64_t)(T + 1) * (p->M / 2) > n_samples)
        return fail(c, STT_ERANGE, "%d columns of %d samples need %lld samples, have %lld", T, p->M,
                    (long long)(T + 1) * (p->M / 2), (long long)n_samples);
    STT_HIP(c, hipSetDevice(c->device));
    if ((s = ensure_fft_tab(c, p->M)) != STT_OK) return s;
    if ((s = ev_begin(c)) != STT_OK) return s;
    const int N = p->M / 2;
    int lg = 0;
    while ((1 << lg) < N) ++lg;
    ev_record(c, 4);
    hipLaunchKernelGGL(k_col_fft, dim3(T), dim3(kFftThreads), sizeof(float2) * N, c->stream, strain_dev, p->M, lg,
                       p->k_lo, p->F, (float)(1.0 / p->fs), (const float2 *)c->fft_tab, (float2 *)spec_dev);
    STT_HIP(c, hipGetLastError());
    hipLaunchKernelGGL(k_psd, dim3((p->F + 255) / 256, T), dim3(256), 0, c->stream, (const float2 *)spec_dev, T, p->F,
                       p->nb, cross_scale(p), psd_dev);
    STT_HIP(c, hipGetLastError());
    ev_record(c, 5);
    c->used[2] = true;
    ev_end(c);
    return STT_OK;
}

stt_status stt_form_maps(stt_ctx *c, const stt_spectro *p, int32_t T, const float *spec_i_dev, const float *psd_i_dev,
                         const float *spec_j_dev, const float *psd_j_dev, int32_t n_slides, const int32_t *shifts,
                         int64_t ld, float *const *Y_dev, float *const *sigma_dev)
{
    if (!c) return STT_EINVAL;
    stt_status s = check_spectro(c, p);
    if (s != STT_OK) return s;
    if (!spec_i_dev || !psd_i_dev || !spec_j_dev || !psd_j_dev) return fail(c, STT_EINVAL, "null spectrum");
    if (((uintptr_t)spec_i_dev & 7) || ((uintptr_t)spec_j_dev & 7)) return fail(c, STT_EINVAL, "spectra must be 8-byte aligned");
    if (T < 4 || T > 65535) return fail(c, STT_ERANGE, "T=%d: need 4 <= T <= 65535", T);
    if (n_slides < 0) return fail(c, STT_EINVAL, "n_slides=%d", n_slides);
    if (ld < p->F) return fail(c, STT_EINVAL, "ld=%lld < F=%d", (long long)ld, p->F);
    if (n_slides == 0) return STT_OK;
    if (!shifts || !Y_dev || !sigma_dev) return fail(c, STT_EINVAL, "null slide table");
    for (int k = 0; k < n_slides; ++k) {
        if (!Y_dev[k] || !sigma_dev[k]) return fail(c, STT_EINVAL, "slide %d: null output", k);
        if (((uintptr_t)Y_dev[k] & 7) || ((uintptr_t)sigma_dev[k] & 3))
            return fail(c, STT_EINVAL, "slide %d: misaligned output", k);
    }
    // two bins per lane where every row segment stays 16-byte aligned
    bool pair = (p->F % 2 == 0) && (ld % 2 == 0) && !((uintptr_t)spec_i_dev & 15) && !((uintptr_t)spec_j_dev & 15) &&
                !((uintptr_t)psd_i_dev & 7) && !((uintptr_t)psd_j_dev & 7);
    for (int k = 0; k < n_slides && pair; ++k)
        pair = !((uintptr_t)Y_dev[k] & 15) && !((uintptr_t)sigma_dev[k] & 7);
    const int per_lane = pair ? 2 : 1;
    const int64_t nblk = (int64_t)((p->F + 256 * per_lane - 1) / (256 * per_lane)) * T;
    const dim3 grid((unsigned)((nblk + 7) / 8 * 8));
    STT_HIP(c, hipSetDevice(c->device));
    if ((s = ev_begin(c)) != STT_OK) return s;
    ev_record(c, 4);
    ev_record(c, 0);
    for (int k0 = 0; k0 < n_slides; k0 += kSlidesPerLaunch) {
        SlideArgs a{};
        a.n = std::min(kSlidesPerLaunch, n_slides - k0);
        for (int k = 0; k < a.n; ++k) {
            a.Y[k] = (float2 *)Y_dev[k0 + k];
            a.sigma[k] = sigma_dev[k0 + k];
            const int64_t sh = shifts[k0 + k] % T;
            a.shift[k] = (int32_t)(sh < 0 ? sh + T : sh);
        }
        if (pair)
            hipLaunchKernelGGL(k_form_maps<2>, grid, dim3(256), 0, c->stream, (const float2 *)spec_i_dev, psd_i_dev,
                               (const float2 *)spec_j_dev, psd_j_dev, T, p->F, cross_scale(p), ld, a);
        else
            hipLaunchKernelGGL(k_form_maps<1>, grid, dim3(256), 0, c->stream, (const float2 *)spec_i_dev, psd_i_dev,
                               (const float2 *)spec_j_dev, psd_j_dev, T, p->F, cross_scale(p), ld, a);
        STT_HIP(c, hipGetLastError());
    }
    ev_record(c, 1);
    ev_record(c, 5);
    c->used[0] = true;
    c->used[2] = true;
    ev_end(c);
    return STT_OK;
}

}  // extern "C"

namespace {

template <int WG, int TPT, bool HW, int MAPT, int SC>
stt_status launch_batch_t(stt_ctx *c, hipStream_t st, const BatchMap *maps, int n_maps, const uint32_t *item_start,
                          uint32_t total_items, uint32_t *queue, const uint32_t *order, int32_t norm, uint64_t *best,
                          size_t shm)
{
    auto kern = k_score_batch<WG, TPT, HW, MAPT, SC>;
    if (shm > 64 * 1024)
        STT_HIP(c, hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    int per_cu = 0;
    STT_HIP(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, WG, shm));
    if (per_cu < 1) return fail(c, STT_EUNSUPPORTED, "batch scorer %dx%d does not fit with %zu B of LDS", WG, TPT, shm);
    const unsigned grid = (unsigned)std::min<int64_t>((int64_t)per_cu * c->n_cu, total_items);
    if (grid == 0) return STT_OK;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(WG), shm, st, maps, n_maps, item_start, queue, order, norm, best);
    STT_HIP(c, hipGetLastError());
    return STT_OK;
}

template <bool HW, int MAPT, int SC>
stt_status launch_batch_h(stt_ctx *c, hipStream_t st, const BatchMap *maps, int n_maps, const uint32_t *item_start,
                          uint32_t total_items, uint32_t *queue, const uint32_t *order, int32_t norm, uint64_t *best,
                          size_t shm)
{
#define STT_BATCH_CASE(W, P)                                                                                        \
    if (c->slab_wg == W && c->slab_tpt == P)                                                                        \
        return launch_batch_t<W, P, HW, MAPT, SC>(c, st, maps, n_maps, item_start, total_items, queue, order, norm, \
                                                  best, shm);
    STT_BATCH_CASE(1024, 4)
    STT_BATCH_CASE(512, 4)
    STT_BATCH_CASE(256, 4)
    STT_BATCH_CASE(1024, 2)
    STT_BATCH_CASE(512, 2)
#undef STT_BATCH_CASE
    return fail(c, STT_EUNSUPPORTED, "no batch scorer for %dx%d", c->slab_wg, c->slab_tpt);
}

template <typename T>
void key_add(std::vector<uint8_t> &k, const T &v)
{
    const uint8_t *b = (const uint8_t *)&v;
    k.insert(k.end(), b, b + sizeof(T));
}

}  // namespace

extern "C" {

stt_status stt_set_graph(stt_ctx *c, int32_t on)
{
    if (!c || on < 0 || on > 1) return STT_EINVAL;
    c->use_graph = on == 1;
    return STT_OK;
}

stt_status stt_score_batch(stt_ctx *c, const stt_map *maps_host, int32_t n_maps, const stt_gen *gen,
                           const int64_t *n_trk_host, int32_t norm, uint64_t *best_key_per_map_dev,
                           float *const *snr_dev_host)
{
    if (!c) return STT_EINVAL;
    if (n_maps < 0 || n_maps > 65536) return fail(c, STT_ERANGE, "n_maps=%d outside [0, 65536]", n_maps);
    if (n_maps == 0) return STT_OK;
    if (!maps_host || !n_trk_host || !gen) return fail(c, STT_EINVAL, "maps, gen and n_trk must be non-NULL");
    if (!best_key_per_map_dev) return fail(c, STT_EINVAL, "best_key_per_map_dev must be non-NULL");
    if (norm != STT_NORM_SQRT_N && norm != STT_NORM_N) return fail(c, STT_EINVAL, "norm=%d", norm);
    const int dtype = maps_host[0].dtype;
    const int esize = fold_esize(dtype);
    std::vector<BatchMap> bm(n_maps);
    std::vector<uint32_t> chunk_start(n_maps + 1), item_start(n_maps + 1), fine_start(n_maps + 1);
    const int per_item = c->slab_wg * c->slab_tpt;
    uint64_t norder = 0, nchunks = 0, nitems = 0, nfine = 0;
    size_t ncc = 0;     // counts per group and sort chunk, all maps
    int max_groups = 1;  // most groups of any map
    size_t shm = 0;
    bool dma_ok = c->dma;  // every map's column fits two DMA slabs
    uint64_t fold_px = 0, fold_cols = 0;
    std::vector<uint64_t> fold_off(n_maps, 0), fold_col(n_maps, 0);
    int64_t max_ldc = 0;
    for (int i = 0; i < n_maps; ++i) {
        const stt_map *mp = &maps_host[i];
        stt_status s = check_map(c, mp);
        if (s != STT_OK) return fail(c, s, "map %d: %s", i, c->err.c_str());
        if (mp->dtype != dtype) return fail(c, STT_EINVAL, "all maps of a batch share one dtype");
        const int64_t n = n_trk_host[i];
        if (n < 0 || n > ((int64_t)1 << 32)) return fail(c, STT_ERANGE, "map %d: n_trk=%lld", i, (long long)n);
        stt_gen g = *gen;
        g.stream = gen->stream + (uint32_t)i;
        BatchMap &d = bm[i];
        if ((s = make_genp(c, &g, mp->T, mp->F, d.g)) != STT_OK) return fail(c, s, "map %d: %s", i, c->err.c_str());
        d.m = to_mapp(mp);
        d.n = n;
        d.order0 = norder;
        d.bin0 = (uint64_t)i * kMaxBins;
        d.wb = bucket_shift(mp->T, n);
        const int nb = ((mp->T - 1) >> d.wb) + 1;
        d.nbins = nb * (nb + 1) / 2;
        d.S = std::min(std::min<int>(64, (c->lds_bytes - 256) / (esize * mp->F)), mp->T);
        if (d.S < 1) return fail(c, STT_EUNSUPPORTED, "map %d: F=%d too wide for the LDS slab", i, mp->F);
        {
            const int64_t ldc = fold_ld(mp->F, esize);
            dma_ok = dma_ok && aligned_slab(dma_slab_cols(c, ldc, esize)) >= 2;
            fold_off[i] = fold_px;
            fold_px += (uint64_t)mp->T * (uint64_t)ldc;
            fold_col[i] = fold_cols;
            fold_cols += (uint64_t)mp->T;
        }
        d.snr = snr_dev_host ? snr_dev_host[i] : nullptr;
        chunk_start[i] = (uint32_t)nchunks;
        fine_start[i] = (uint32_t)nfine;
        item_start[i] = (uint32_t)nitems;
        d.chunk0 = (int32_t)nchunks;
        norder += (uint64_t)n;
        nchunks += (uint64_t)((n + kBinChunk - 1) / kBinChunk);
        {
            const int ng = (d.nbins + kGroupMask) >> kGroupShift;
            nfine += (uint64_t)((n + kFineChunk - 1) / kFineChunk) + (uint64_t)ng;
            d.cc0 = ncc;
            ncc += (size_t)ng * (size_t)((n + kBinChunk - 1) / kBinChunk);
            max_groups = std::max(max_groups, ng);
        }
        nitems += (uint64_t)((n + per_item - 1) / per_item);
        if (norder >= ((uint64_t)1 << 32) || nitems >= ((uint64_t)1 << 31))
            return fail(c, STT_ERANGE, "a batch holds fewer than 2^32 templates");
    }
    chunk_start[n_maps] = (uint32_t)nchunks;
    fine_start[n_maps] = (uint32_t)nfine;
    item_start[n_maps] = (uint32_t)nitems;
    STT_HIP(c, hipSetDevice(c->device));
    // every map is scored from its polar fold (one launch folds them all); slabs stream in by DMA
    // when every map's column fits two of them, else through registers
    std::vector<MapP> orig(n_maps);
    for (int i = 0; i < n_maps; ++i) orig[i] = bm[i].m;
    {
        stt_status sf = ensure_pbuf(c, (size_t)esize * (size_t)fold_px);
        if (sf != STT_OK) return sf;
    }
    std::vector<FoldJob> jobs(n_maps + 1);
    shm = 0;
    // one aligned slab width for the whole batch: the narrowest any map's columns allow
    int sc_all = 16;
    if (dma_ok)
        for (int i = 0; i < n_maps; ++i)
            sc_all = std::min(sc_all, aligned_slab(dma_slab_cols(c, fold_ld(bm[i].m.F, esize), esize)));
    for (int i = 0; i < n_maps; ++i) {
        BatchMap &d = bm[i];
        const int64_t ldc = fold_ld(d.m.F, esize);
        void *dst = (char *)c->pbuf + (size_t)esize * fold_off[i];
        jobs[i] = FoldJob{orig[i], dst, ldc, (uint32_t)fold_col[i]};
        max_ldc = std::max(max_ldc, ldc);
        d.m.Y = (const float2 *)dst;  // an FP16 map keeps its scale 2^e
        d.m.sig = nullptr;
        d.m.ld = ldc;
        if (dma_ok) {
            d.S = sc_all;
            shm = std::max(shm, 2 * (size_t)esize * (size_t)d.S * (size_t)ldc);
        } else {
            shm = std::max(shm, (size_t)esize * (size_t)d.S * (size_t)d.m.F);
        }
    }
    jobs[n_maps] = FoldJob{MapP{}, nullptr, 0, (uint32_t)fold_cols};
    if (!c->n_cu) STT_HIP(c, hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device));

    // scratch: [totals | cursor | queue | order (first the buckets of the count) | group starts | second-
    // scatter chunk tables | group regions | counts per group and sort chunk | buckets within the group]
    const size_t nb_all = (size_t)n_maps * kMaxBins;
    const size_t ng_all = (size_t)n_maps * kGroupSlots;
    const size_t need = sizeof(uint32_t) * (2 * nb_all + 64 + 2 * norder + 2 * ng_all + ncc) + norder;
    stt_status s = ensure_scratch(c, need);
    if (s != STT_OK) return s;
    uint32_t *totals = (uint32_t *)c->scratch;
    uint32_t *cursor = totals + nb_all;
    uint32_t *queue = cursor + nb_all;
    uint32_t *order = queue + 64;
    uint32_t *gstart = order + norder;
    uint32_t *fitem = gstart + ng_all;
    uint32_t *tmp = fitem + ng_all;
    uint32_t *ccnt = tmp + norder;
    uint8_t *tsub = (uint8_t *)(ccnt + ncc);
    uint16_t *bins = (uint16_t *)order;

    // the argument key: a repeat of the last batch replays its graph
    std::vector<uint8_t> key;
    key_add(key, n_maps);
    key_add(key, norm);
    key_add(key, best_key_per_map_dev);
    key_add(key, c->scratch);
    key_add(key, c->slab_wg);
    key_add(key, c->slab_tpt);
    key_add(key, c->lds_bytes);
    key_add(key, c->hw_trig);
    key_add(key, dma_ok);
    key_add(key, sc_all);
    key_add(key, c->pbuf);
    for (const auto &d : bm) key_add(key, d);
    for (const auto &o : orig) key_add(key, o);
    const bool same = c->use_graph && c->gexec && key == c->bkey;

    if (!same) {
        // descriptor tables to the device (synchronous: they must outlive the call)
        const size_t tbl = sizeof(BatchMap) * n_maps + sizeof(FoldJob) * (n_maps + 1) + sizeof(uint32_t) * 3 * (n_maps + 1);
        if (tbl > c->bdev_bytes) {
            STT_HIP(c, hipStreamSynchronize(c->stream));
            if (c->bdev) (void)hipFree(c->bdev);
            c->bdev = nullptr;
            c->bdev_bytes = 0;
            if (hipMalloc(&c->bdev, tbl) != hipSuccess) {
                (void)hipGetLastError();
                return fail(c, STT_ENOMEM, "cannot allocate %zu bytes of batch tables", tbl);
            }
            c->bdev_bytes = tbl;
        }
        STT_HIP(c, hipStreamSynchronize(c->stream));  // the previous batch may still read the tables
        BatchMap *dmaps = (BatchMap *)c->bdev;
        FoldJob *djobs = (FoldJob *)(dmaps + n_maps);
        uint32_t *dchunk = (uint32_t *)(djobs + (n_maps + 1));
        uint32_t *ditem = dchunk + (n_maps + 1);
        uint32_t *dfine = ditem + (n_maps + 1);
        STT_HIP(c, hipMemcpy(dmaps, bm.data(), sizeof(BatchMap) * n_maps, hipMemcpyHostToDevice));
        STT_HIP(c, hipMemcpy(djobs, jobs.data(), sizeof(FoldJob) * (n_maps + 1), hipMemcpyHostToDevice));
        STT_HIP(c, hipMemcpy(dchunk, chunk_start.data(), sizeof(uint32_t) * (n_maps + 1), hipMemcpyHostToDevice));
        STT_HIP(c, hipMemcpy(ditem, item_start.data(), sizeof(uint32_t) * (n_maps + 1), hipMemcpyHostToDevice));
        STT_HIP(c, hipMemcpy(dfine, fine_start.data(), sizeof(uint32_t) * (n_maps + 1), hipMemcpyHostToDevice));
        if (c->gexec) { (void)hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
        if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
        c->bkey.clear();

        auto enqueue = [&](hipStream_t st) -> stt_status {
            const bool timed = st == c->stream;  // events only outside graph capture
            if (timed) ev_record(c, 2);
            {
                const dim3 fg((unsigned)fold_cols, (unsigned)((max_ldc + 256 * kFoldRows - 1) / (256 * kFoldRows)));  // columns over x, rows over y
                if (dtype == STT_P16)
                    hipLaunchKernelGGL(k_fold_batch<kMapP16>, dim3(fg), dim3(256), 0, st, (const FoldJob *)djobs,
                                       n_maps);
                else
                    hipLaunchKernelGGL(k_fold_batch<kMapF32>, dim3(fg), dim3(256), 0, st, (const FoldJob *)djobs,
                                       n_maps);
            }
            hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((nb_all + 64 + 255) / 256)), dim3(256), 0, st, totals,
                               (int64_t)(nb_all), 0u);
            hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, queue, (int64_t)1, 0u);
            if (nchunks) {
                hipLaunchKernelGGL(k_bin_count_batch, dim3((unsigned)nchunks), dim3(256), 0, st,
                                   (const BatchMap *)dmaps, n_maps, (const uint32_t *)dchunk, totals, bins, ccnt);
                hipLaunchKernelGGL(k_bin_scan_batch, dim3((unsigned)(max_groups + 1) * (unsigned)n_maps), dim3(256), 0,
                                   st, (const BatchMap *)dmaps, (const uint32_t *)dchunk, max_groups,
                                   (const uint32_t *)totals, cursor, gstart, fitem, ccnt);
                hipLaunchKernelGGL(k_bin_group_batch, dim3((unsigned)nchunks), dim3(kScatterWG), 0, st,
                                   (const BatchMap *)dmaps, n_maps, (const uint32_t *)dchunk, (const uint16_t *)bins,
                                   (const uint32_t *)gstart, (const uint32_t *)ccnt, tmp, tsub);
                hipLaunchKernelGGL(k_bin_fine_batch, dim3((unsigned)nfine), dim3(kScatterWG), 0, st,
                                   (const BatchMap *)dmaps, n_maps, (const uint32_t *)dfine,
                                   (const uint32_t *)gstart, (const uint32_t *)fitem, cursor, (const uint32_t *)tmp,
                                   (const uint8_t *)tsub, order);
            }
            STT_HIP(c, hipGetLastError());
            if (timed) {
                ev_record(c, 3);
                ev_record(c, 0);
                c->used[0] = c->used[1] = true;
            }
            stt_status r;
            const uint32_t ni = (uint32_t)nitems;
            const int sc = dma_ok ? sc_all : 0;
#define STT_BATCH_SC(MT, SCV)                                                                                  \
    r = c->hw_trig ? launch_batch_h<true, MT, SCV>(c, st, dmaps, n_maps, ditem, ni, queue, order, norm,        \
                                                   best_key_per_map_dev, shm)                                 \
                   : launch_batch_h<false, MT, SCV>(c, st, dmaps, n_maps, ditem, ni, queue, order, norm,       \
                                                    best_key_per_map_dev, shm)
#define STT_BATCH_MT(MT)                                                                                       \
    switch (sc) {                                                                                              \
    case 0: STT_BATCH_SC(MT, 0); break;                                                                        \
    case 2: STT_BATCH_SC(MT, 2); break;                                                                        \
    case 4: STT_BATCH_SC(MT, 4); break;                                                                        \
    case 8: STT_BATCH_SC(MT, 8); break;                                                                        \
    case 16: STT_BATCH_SC(MT, 16); break;                                                                      \
    default: r = fail(c, STT_EUNSUPPORTED, "no batch scorer for %d-column slabs", sc);                        \
    }
            if (dtype == STT_P16) { STT_BATCH_MT(kMapPolH) } else { STT_BATCH_MT(kMapPol) }
#undef STT_BATCH_MT
#undef STT_BATCH_SC
            if (timed) ev_record(c, 1);
            return r;
        };

        if (!c->use_graph) {
            if ((s = ev_begin(c)) != STT_OK) return s;
            ev_record(c, 4);
            s = enqueue(c->stream);
            ev_record(c, 5);
            c->used[2] = true;
            ev_end(c);
            return s;
        }
        if (!c->cap_stream) STT_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        STT_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
        s = enqueue(c->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        if (s != STT_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return fail(c, STT_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        c->graph = g;
        STT_HIP(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
        c->bkey = key;
    }
    if ((s = ev_begin(c)) != STT_OK) return s;
    ev_record(c, 4);
    STT_HIP(c, hipGraphLaunch(c->gexec, c->stream));
    ev_record(c, 5);
    c->used[2] = true;  // a replayed graph is timed as a whole
    ev_end(c);
    return STT_OK;
}

// ----------------------------------------------------------------------------- differentiation

stt_status stt_tracks_at(stt_ctx *c, const stt_gen *gen, int32_t T, int32_t F, const int64_t *idx_dev, int64_t n,
                         stt_track *out_dev)
{
    if (!c) return STT_EINVAL;
    GenP g;
    stt_status s = make_genp(c, gen, T, F, g);
    if (s != STT_OK) return s;
    if (n < 0) return fail(c, STT_EINVAL, "n=%lld", (long long)n);
    if (n == 0) return STT_OK;
    if (!idx_dev || !out_dev) return fail(c, STT_EINVAL, "idx_dev and out_dev must be non-NULL");
    STT_HIP(c, hipSetDevice(c->device));
    hipLaunchKernelGGL(k_tracks_at, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, g, idx_dev, n,
                       (Trk *)out_dev);
    STT_HIP(c, hipGetLastError());
    return STT_OK;
}

stt_status stt_tracks_to_theta(stt_ctx *c, const stt_track *tracks_dev, int64_t n, float *theta_dev, int32_t *K_dev)
{
    if (!c) return STT_EINVAL;
    if (n < 0) return fail(c, STT_EINVAL, "n=%lld", (long long)n);
    if (n == 0) return STT_OK;
    if (!tracks_dev || !theta_dev || !K_dev) return fail(c, STT_EINVAL, "NULL buffer");
    STT_HIP(c, hipSetDevice(c->device));
    hipLaunchKernelGGL(k_track_to_theta, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                       (const Trk *)tracks_dev, n, theta_dev, K_dev);
    STT_HIP(c, hipGetLastError());
    return STT_OK;
}

}  // extern "C"

namespace {

stt_status smooth_launch(stt_ctx *c, const stt_map *map, const float *theta, const int32_t *K, int32_t n, float *z,
                         float *grad, hipStream_t st)
{
    const MapP m = to_mapp(map);
    const unsigned grid = (unsigned)n;  // one workgroup per template
    if (map->dtype == STT_P16)
        hipLaunchKernelGGL(k_smooth_grad<kMapP16>, dim3(grid), dim3(kSmoothWG), 0, st, m, theta, K, n, z, grad);
    else
        hipLaunchKernelGGL(k_smooth_grad<kMapF32>, dim3(grid), dim3(kSmoothWG), 0, st, m, theta, K, n, z, grad);
    STT_HIP(c, hipGetLastError());
    return STT_OK;
}

stt_status check_smooth(stt_ctx *c, const stt_map *map, const float *theta, const int32_t *K, int32_t n, float *z)
{
    stt_status s = check_map(c, map);
    if (s != STT_OK) return s;
    if (map->F < 2) return fail(c, STT_ERANGE, "the smooth statistic needs F >= 2");
    if (n < 0) return fail(c, STT_EINVAL, "n=%d", n);
    if (n > 0 && (!theta || !K || !z)) return fail(c, STT_EINVAL, "NULL buffer");
    return STT_OK;
}

}  // namespace

extern "C" {

stt_status stt_smooth(stt_ctx *c, const stt_map *map, const float *theta_dev, const int32_t *K_dev, int32_t n,
                      float *z_dev)
{
    if (!c) return STT_EINVAL;
    stt_status s = check_smooth(c, map, theta_dev, K_dev, n, z_dev);
    if (s != STT_OK || n == 0) return s;
    STT_HIP(c, hipSetDevice(c->device));
    return smooth_launch(c, map, theta_dev, K_dev, n, z_dev, nullptr, c->stream);
}

stt_status stt_grad(stt_ctx *c, const stt_map *map, const float *theta_dev, const int32_t *K_dev, int32_t n,
                    float *z_dev, float *grad_dev)
{
    if (!c) return STT_EINVAL;
    stt_status s = check_smooth(c, map, theta_dev, K_dev, n, z_dev);
    if (s != STT_OK || n == 0) return s;
    if (!grad_dev) return fail(c, STT_EINVAL, "grad_dev is NULL");
    STT_HIP(c, hipSetDevice(c->device));
    return smooth_launch(c, map, theta_dev, K_dev, n, z_dev, grad_dev, c->stream);
}

stt_status stt_refine(stt_ctx *c, const stt_map *map, int32_t min_len, int32_t dtau_max, float *theta_dev,
                      const int32_t *K_dev, int32_t n, int32_t steps, const float *sched_host, float *z_smooth_dev,
                      stt_track *plain_dev, float *z_plain_dev, int32_t norm)
{
    if (!c) return STT_EINVAL;
    stt_status s = check_smooth(c, map, theta_dev, K_dev, n, z_smooth_dev);
    if (s != STT_OK) return s;
    if (steps < 0 || steps > 100000) return fail(c, STT_ERANGE, "steps=%d", steps);
    if (min_len < 2 || min_len > map->T) return fail(c, STT_ERANGE, "min_len=%d outside [2, T]", min_len);
    if (dtau_max < 0 || dtau_max >= (1 << 30)) return fail(c, STT_ERANGE, "dtau_max=%d", dtau_max);
    if (norm != STT_NORM_SQRT_N && norm != STT_NORM_N) return fail(c, STT_EINVAL, "norm=%d", norm);
    if (z_plain_dev && !plain_dev) return fail(c, STT_EINVAL, "z_plain_dev needs plain_dev");
    if (n == 0) return STT_OK;
    STT_HIP(c, hipSetDevice(c->device));
    RefineP p;
    p.T = map->T;
    p.F = map->F;
    p.L = min_len;
    p.dmax_ms = (double)dtau_max * (1e3 / 268435456.0);
    p.px0 = sched_host ? sched_host[0] : 1.0;
    p.px1 = sched_host ? sched_host[1] : 0.02;
    p.ms0 = sched_host ? sched_host[2] : 0.5;
    p.ms1 = sched_host ? sched_host[3] : 0.01;
    p.steps = steps;
    const MapP m = to_mapp(map);
    // The steps gather p = Y/sigma from the folded copy the scorers use (bit-identical to forming
    // it at each gather: one division per pixel instead of one per gather, 8 bytes instead of 12).
    const int64_t ldc = fold_ld(m.F);
    if ((s = ensure_pbuf(c, sizeof(float2) * (size_t)m.T * (size_t)ldc)) != STT_OK) return s;
    // timing: the refinement kernel is this call's stage 0 (the plain re-score below records its own)
    if ((s = ev_begin(c)) != STT_OK) return s;
    ev_record(c, 4);
    const unsigned fg = (unsigned)std::min<int64_t>(((int64_t)m.T * ldc + 255) / 256, 4096);
    if (map->dtype == STT_P16)
        hipLaunchKernelGGL(k_fold_p<kMapP16>, dim3(fg), dim3(256), 0, c->stream, m, (float2 *)c->pbuf, ldc);
    else
        hipLaunchKernelGGL(k_fold_p<kMapF32>, dim3(fg), dim3(256), 0, c->stream, m, (float2 *)c->pbuf, ldc);
    MapP mf = m;
    mf.Y = (const float2 *)c->pbuf;
    mf.sig = nullptr;
    mf.ld = ldc;
    ev_record(c, 0);
    hipLaunchKernelGGL(k_refine<kMapPF>, dim3((unsigned)n), dim3(kSmoothWG), 0, c->stream, mf, theta_dev, K_dev, n,
                       z_smooth_dev, p);
    STT_HIP(c, hipGetLastError());
    ev_record(c, 1);
    ev_record(c, 5);
    c->used[0] = true;
    c->used[2] = true;
    ev_end(c);
    if (plain_dev) {
        hipLaunchKernelGGL(k_theta_to_track, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                           (const float *)theta_dev, (int64_t)n,
                           map->T, map->F, min_len, dtau_max, (Trk *)plain_dev);
        STT_HIP(c, hipGetLastError());
        if (z_plain_dev) {
            const int old = c->path;
            c->path = 0;  // automatic: a short explicit list takes one wave per template
            s = stt_score(c, map, nullptr, plain_dev, 0, n, norm, z_plain_dev, nullptr);
            c->path = old;
            if (s != STT_OK) return s;
        }
    }
    return STT_OK;
}

// ----------------------------------------------------------------------------- autotuning

}  // extern "C"

namespace {

struct TuneChoice {
    int wg, tpt, lds;
    double ms;
};

std::string gpu_arch(const stt_ctx *c)
{
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) arch = prop.gcnArchName;
    return arch.substr(0, arch.find(':'));
}

int log2_floor(int64_t v)
{
    int b = 0;
    while (((int64_t)1 << (b + 1)) <= v) ++b;
    return b;
}

// Generation of the scorers' inner loop: part of every cache key, so that choices timed on an
// earlier loop are searched again. "pol2": polar folded map, one cosine per pixel, slab scorers
// held to 128 VGPRs (4 waves per SIMD).
constexpr const char *kCoreTag = "pol2";

// maps of similar duration (power-of-two bucket) and call size share a choice
std::string tune_key(const stt_ctx *c, const stt_map *m, int64_t n)
{
    char buf[192];
    snprintf(buf, sizeof buf, "%s/%s/F=%d/dtype=%d/T=2^%d/n=2^%d/trig=%d", gpu_arch(c).c_str(), kCoreTag, m->F,
             m->dtype, log2_floor(m->T), log2_floor(n), c->hw_trig ? 1 : 0);
    return buf;
}

std::string tune_key_batch(const stt_ctx *c, int F, int dtype, int T, int n_maps, int64_t n_total)
{
    char buf[224];
    snprintf(buf, sizeof buf, "%s/%s/batch/F=%d/dtype=%d/T=2^%d/maps=2^%d/n=2^%d/trig=%d", gpu_arch(c).c_str(),
             kCoreTag, F, dtype, log2_floor(T), log2_floor(n_maps), log2_floor(n_total), c->hw_trig ? 1 : 0);
    return buf;
}

// Times `call` (which must leave a timed scoring stage) for every compiled
// shape and LDS budget that fits columns of F pixels: `reps` timed runs after
// one warm-up, mean of the scoring kernel's HIP-event time. The context's
// shape, budget, timing and graph settings and the caller's pending timing
// records are restored afterwards.
stt_status tune_search(stt_ctx *c, int F, int reps, const std::function<stt_status()> &call, TuneChoice &best)
{
    const int old_path = c->path, old_wg = c->slab_wg, old_tpt = c->slab_tpt, old_lds = c->lds_bytes;
    const bool old_timing = c->timing, old_graph = c->use_graph;
    std::vector<Rec> saved;
    saved.swap(c->recs);
    const size_t saved_next = c->next;
    c->timing = true;
    c->use_graph = false;
    c->recs.clear();
    c->next = saved_next;  // tuning events come after any the caller has not read yet
    static const int ldss[] = {160 * 1024, 112 * 1024, 80 * 1024, 48 * 1024};
    stt_status s = STT_OK;
    for (const auto &sh : kShapes) {
        for (int lds : ldss) {
            if ((lds - 256) / (8 * F) < 1) continue;
            c->path = 2;
            c->slab_wg = sh[0];
            c->slab_tpt = sh[1];
            c->lds_bytes = lds;
            double tot = 0;
            int cnt = 0;
            for (int rep = 0; rep <= reps && s == STT_OK; ++rep) {
                if ((s = call()) != STT_OK) break;
                float ms = 0;
                if ((s = stt_kernel_ms(c, 0, &ms)) != STT_OK) break;
                if (rep > 0) { tot += ms; ++cnt; }  // the first run warms up
            }
            c->recs.clear();
            c->next = saved_next;
            if (s != STT_OK) break;
            if (cnt && tot / cnt < best.ms) best = TuneChoice{sh[0], sh[1], lds, tot / cnt};
        }
        if (s != STT_OK) break;
    }
    c->path = old_path;
    c->slab_wg = old_wg;
    c->slab_tpt = old_tpt;
    c->lds_bytes = old_lds;
    c->timing = old_timing;
    c->use_graph = old_graph;
    c->recs.swap(saved);
    c->next = saved_next;
    if (s != STT_OK) return s;
    if (best.wg == 0) return fail(c, STT_EUNSUPPORTED, "no slab configuration fits F=%d", F);
    return STT_OK;
}

stt_status apply_choice(stt_ctx *c, const std::string &key, const TuneChoice &best, int32_t *choice_out)
{
    if (!slab_shape_ok(best.wg, best.tpt) || best.lds < 1024 || best.lds > 160 * 1024)
        return fail(c, STT_EINVAL, "cache entry for %s is not a valid configuration", key.c_str());
    c->slab_wg = best.wg;
    c->slab_tpt = best.tpt;
    c->lds_bytes = best.lds;
    if (choice_out) {
        choice_out[0] = best.wg;
        choice_out[1] = best.tpt;
        choice_out[2] = best.lds;
    }
    return STT_OK;
}

// The cache file holds one line per key:  "<key>": {"wg": W, "tpt": P, "lds": B, "ms": T}
bool cache_lookup(const char *path, const std::string &key, TuneChoice &out)
{
    if (!path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    const std::string pat = "\"" + key + "\":";
    while (fgets(line, sizeof line, f)) {
        const char *p = strstr(line, pat.c_str());
        if (!p) continue;
        TuneChoice t;
        if (sscanf(p + pat.size(), " {\"wg\": %d, \"tpt\": %d, \"lds\": %d, \"ms\": %lf}", &t.wg, &t.tpt, &t.lds,
                   &t.ms) == 4) {
            out = t;
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, const TuneChoice &t)
{
    if (!path) return;
    std::vector<std::string> lines;
    if (FILE *f = fopen(path, "r")) {
        char line[512];
        const std::string pat = "\"" + key + "\":";
        while (fgets(line, sizeof line, f)) {
            std::string l(line);
            while (!l.empty() && (l.back() == '\n' || l.back() == ',')) l.pop_back();
            // keep the other entries only: braces (also "{}" of an empty cache) are written anew
            const size_t q = l.find_first_not_of(" \t");
            if (q == std::string::npos || l[q] != '"' || l.find(pat) != std::string::npos) continue;
            lines.push_back(l);
        }
        fclose(f);
    }
    char buf[512];
    snprintf(buf, sizeof buf, "  \"%s\": {\"wg\": %d, \"tpt\": %d, \"lds\": %d, \"ms\": %.6f}", key.c_str(), t.wg,
             t.tpt, t.lds, t.ms);
    lines.push_back(buf);
    const std::string tmp = std::string(path) + ".tmp";
    if (FILE *f = fopen(tmp.c_str(), "w")) {
        fprintf(f, "{\n");
        for (size_t i = 0; i < lines.size(); ++i) fprintf(f, "%s%s\n", lines[i].c_str(), i + 1 < lines.size() ? "," : "");
        fprintf(f, "}\n");
        fclose(f);
        rename(tmp.c_str(), path);
    }
}

}  // namespace

extern "C" {

stt_status stt_autotune(stt_ctx *c, const stt_map *map, const stt_gen *gen, int64_t n, const char *cache_path,
                        int32_t *choice_out)
{
    if (!c) return STT_EINVAL;
    stt_status s = check_map(c, map);
    if (s != STT_OK) return s;
    if (n < 1 || n > ((int64_t)1 << 32)) return fail(c, STT_ERANGE, "n=%lld", (long long)n);
    GenP gp;
    if ((s = make_genp(c, gen, map->T, map->F, gp)) != STT_OK) return s;
    const std::string key = tune_key(c, map, n);
    TuneChoice best{0, 0, 0, 1e30};
    if (!cache_lookup(cache_path, key, best)) {
        s = tune_search(c, map->F, 3, [&] { return stt_score(c, map, gen, nullptr, 0, n, STT_NORM_SQRT_N, nullptr, nullptr); },
                        best);
        if (s != STT_OK) return s;
        cache_store(cache_path, key, best);
    }
    return apply_choice(c, key, best, choice_out);
}

stt_status stt_autotune_batch(stt_ctx *c, const stt_map *maps_host, int32_t n_maps, const stt_gen *gen,
                              const int64_t *n_trk_host, const char *cache_path, int32_t *choice_out)
{
    if (!c) return STT_EINVAL;
    if (n_maps < 1 || n_maps > 65536) return fail(c, STT_ERANGE, "n_maps=%d outside [1, 65536]", n_maps);
    if (!maps_host || !gen || !n_trk_host) return fail(c, STT_EINVAL, "maps, gen and n_trk must be non-NULL");
    int Fmax = 0, Tmax = 0;
    int64_t ntot = 0;
    for (int i = 0; i < n_maps; ++i) {
        stt_status s = check_map(c, &maps_host[i]);
        if (s != STT_OK) return s;
        if (n_trk_host[i] < 0) return fail(c, STT_ERANGE, "n_trk[%d] < 0", i);
        Fmax = std::max(Fmax, maps_host[i].F);
        Tmax = std::max(Tmax, maps_host[i].T);
        ntot += n_trk_host[i];
    }
    if (ntot < 1) return fail(c, STT_ERANGE, "no templates to time");
    const std::string key = tune_key_batch(c, Fmax, maps_host[0].dtype, Tmax, n_maps, ntot);
    TuneChoice best{0, 0, 0, 1e30};
    if (!cache_lookup(cache_path, key, best)) {
        void *keys = nullptr;
        STT_HIP(c, hipSetDevice(c->device));
        if (hipMalloc(&keys, sizeof(uint64_t) * (size_t)n_maps) != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, STT_ENOMEM, "cannot allocate the tuner's %d keys", n_maps);
        }
        stt_status s = tune_search(c, Fmax, 2, [&] {
            return stt_score_batch(c, maps_host, n_maps, gen, n_trk_host, STT_NORM_SQRT_N, (uint64_t *)keys, nullptr);
        }, best);
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(keys);
        if (s != STT_OK) return s;
        cache_store(cache_path, key, best);
    }
    return apply_choice(c, key, best, choice_out);
}

uint64_t stt_key_encode(float z, uint32_t j) { return key_encode(z, j); }

void stt_key_decode(uint64_t key, float *z, uint32_t *j)
{
    const uint32_t o = (uint32_t)(key >> 32);
    const uint32_t b = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
    if (z) std::memcpy(z, &b, sizeof b);
    if (j) *j = 0xFFFFFFFFu - (uint32_t)key;
}

}  // extern "C"
