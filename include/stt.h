/*
 * stt.h -- C ABI of libstt, an MI355X (gfx950) implementation of the template
 * search of "all-sky stochtrack" (Thrane & Coughlin, arXiv:1401.8060): very
 * many random quadratic-Bezier tracks are scored on a complex cross-power
 * ft-map with the random-phase-factor statistic of Eq. 8 and reduced by
 * max/argmax (Sec. III; Sec. V records the maximum per spectrogram).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Ownership: every bulk buffer is caller-owned DEVICE memory (for example
 *    a torch tensor's data pointer). The library never frees it and touches it
 *    only in work it enqueues. Host-side arguments (structs, small arrays
 *    marked "host") are read before the call returns.
 *  - Streams: work is enqueued asynchronously on the context's stream and is
 *    ordered after earlier work on that stream. Results are valid once the
 *    stream has been synchronised (stt_sync, or the caller's own sync).
 *  - Errors: argument, shape and range errors are detected on the host before
 *    anything is enqueued and returned as a negative stt_status; nothing is
 *    written then. HIP launch failures return STT_EHIP. Device-side faults
 *    surface at the next synchronisation. stt_last_error() gives a message.
 *  - Threads: a context is not thread-safe; use one context per host thread.
 *  - Map layout: pixel (t, r) -- time column t in [0, T), frequency row r in
 *    [0, F) -- sits at element t*ld + r (time-major, frequency contiguous).
 *    Row r has frequency (fq4_lo + r*dfq4)/16 Hz.
 *  - Template (track) format, a reading of Eq. 6 with t_mid at the midpoint:
 *    the track covers columns t0..t2 (N = t2-t0+1 pixels, one per column).
 *    Column t0+k takes row floor(B(k/(t2-t0))/256) where B is the quadratic
 *    Bezier through the control frequencies f0, f1, f2 given in 1/256-row
 *    units; the floor is exact (integer arithmetic). dtau is the template's
 *    time delay (Eq. 8) in units of 2^-28 s.
 *  - Statistic (Eq. 8, with the complex SNR p = Y/sigma of Eq. 7 and the
 *    appendix): S = sum over the N pixels of Re[exp(2 pi i f dtau) Y/sigma];
 *    z = S/sqrt(N) (STT_NORM_SQRT_N, standard normal on noise) or S/N
 *    (STT_NORM_N, the paper's literal 1/N). The scorers evaluate each term
 *    as |p| cos(2 pi (f dtau + arg p)) from a polar copy of p (one cosine
 *    per pixel), in FP32 with FP64 sums every 16 columns; scores agree with
 *    the FP64 definition to 1e-5 max(1, |z|).
 *  - Best key: a 64-bit word (ordered bits of the FP32 score << 32) |
 *    (0xFFFFFFFF - j) where j is the track index. A larger key is a higher
 *    score, then a lower index. NaN scores count as -inf, -0 as +0. Every
 *    real key is > 0, so a buffer initialised to 0 means "empty"; entry points
 *    that take best_key_dev max-merge into it (never overwrite), which is the
 *    paper's Sec. V combination of runs by their maximum.
 */
#ifndef STT_H
#define STT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t stt_status;
#define STT_OK 0
#define STT_EINVAL (-1)      /* bad argument: null pointer, bad enum, bad shape */
#define STT_ERANGE (-2)      /* size outside the supported range */
#define STT_ENOMEM (-3)      /* device allocation of internal scratch failed */
#define STT_EHIP (-4)        /* a HIP runtime call failed */
#define STT_EUNSUPPORTED (-5) /* valid request this build does not support */

#define STT_NORM_SQRT_N 0
#define STT_NORM_N 1

#define STT_C64F32 0 /* Y: complex64 (re, im float32 interleaved); sigma: float32 */
#define STT_P16 1    /* Y: the complex SNR p = Y/sigma in FP16 polar form, one 32-bit word per pixel: arg p in
                        units of 2^-16 turn in the low half, |p| * 2^-scale_exp as binary16 in the high half;
                        sigma: NULL (see stt_map_pack_p16) */

#define STT_FBITS 8        /* fractional bits of control frequencies */
#define STT_MAX_T 2896     /* largest map duration (columns) */
#define STT_MAX_F 32767    /* largest map bandwidth (rows) */

typedef struct {
    int32_t t0, t2;       /* first and last column, 0 <= t0 < t2 < T */
    uint32_t f0, f1, f2;  /* control frequencies, 1/256-row units, < F*256 */
    int32_t dtau;         /* time delay, units of 2^-28 s */
} stt_track;

/* A template with a free t_mid (Eq. 6 with all six random numbers): the time
 * coordinate is a quadratic Bezier with control points t0, t1, t2 (integer
 * columns, t0 <= t1 <= t2); other fields as stt_track. 28 bytes. */
typedef struct {
    int32_t t0, t1, t2;
    uint32_t f0, f1, f2;
    int32_t dtau;
} stt_track_tm;

typedef struct {
    uint64_t seed;     /* Philox4x32-10 key (low word, high word) */
    uint32_t stream;   /* Philox counter word 2: an independent sequence per map */
    int32_t min_len;   /* L: minimum pixels per track (the paper's t_min), >= 2 */
    int32_t dtau_max;  /* delays are uniform on [dtau_center - dtau_max, dtau_center + dtau_max], 2^-28 s
                          units; 0 = one fixed delay (the targeted search of Eq. 5) */
    int32_t dtau_center; /* 0 for the all-sky (isotropic) prior; otherwise the centre of a sky patch's delay
                            band (Sec. VI: a patch of sky instead of the isotropic prior; a band of directions
                            about the baseline gives uniform delays on its interval). |center| + max < 2^30 */
} stt_gen;

typedef struct {
    int32_t T, F;         /* columns, rows */
    int64_t ld;           /* elements between columns, ld >= F */
    int32_t dtype;        /* STT_C64F32 or STT_P16 */
    int32_t scale_exp;    /* STT_P16 only: |p| = stored magnitude * 2^scale_exp */
    const void *Y;        /* device: [T][ld] complex64, or 32-bit polar words for STT_P16 */
    const void *sigma;    /* device: [T][ld] float32 sigma (STT_C64F32); NULL for STT_P16 */
    int32_t fq4_lo;       /* frequency of row 0 in 1/16 Hz (1600 = 100 Hz) */
    int32_t dfq4;         /* row spacing in 1/16 Hz (16 = 1 Hz) */
} stt_map;

typedef struct stt_ctx stt_ctx;

/* Lifecycle. stt_create binds the context to HIP device `device` and to the
 * stream `hip_stream` (a hipStream_t; NULL = the device's null stream), which
 * the context borrows and never destroys. The context owns only its internal
 * scratch memory. Returns STT_EHIP if the device cannot be selected. */
stt_status stt_create(int device, void *hip_stream, stt_ctx **out);
stt_status stt_destroy(stt_ctx *ctx);
stt_status stt_set_stream(stt_ctx *ctx, void *hip_stream);
stt_status stt_sync(stt_ctx *ctx);
const char *stt_strerror(stt_status s);
const char *stt_last_error(const stt_ctx *ctx);

/* Pre-size internal scratch for calls of up to max_tracks tracks, so that
 * later calls of that size allocate nothing. */
stt_status stt_reserve(stt_ctx *ctx, int64_t max_tracks);

/* Kernel timing. When on, the context records HIP events around its stages
 * on its stream: `which` = 0 scoring kernel, 1 binning kernels, 2 whole call.
 * stt_kernel_ms gives the last call's stage time; stt_kernel_ms_total sums the
 * stage over every call since timing was switched on or last totalled (and
 * forgets them). Both synchronise the stream. stt_set_timing resets. */
stt_status stt_set_timing(stt_ctx *ctx, int32_t on);
stt_status stt_kernel_ms(stt_ctx *ctx, int32_t which, float *ms);
stt_status stt_kernel_ms_total(stt_ctx *ctx, int32_t which, double *total_ms, int32_t *count);

/* Scorer selection, for tests and tuning: path 0 = automatic (LDS time slabs
 * from 4096 templates on when a column fits; otherwise one wave per template
 * below 65536 templates, else one lane per template), 1 = one lane per
 * template, direct gathers from global memory, 2 = LDS time slabs
 * (STT_EUNSUPPORTED when one column of the map does not fit lds_bytes), 3 =
 * one wave per template, direct gathers. All paths give bit-identical scores.
 * lds_bytes (0 = keep) is the slab budget per workgroup, in [1024, 163840];
 * default 163840. */
stt_status stt_set_path(stt_ctx *ctx, int32_t path, int32_t lds_bytes);

/* Shape of the LDS-slab scorer: wg lanes per workgroup and tpt templates per
 * lane; STT_EUNSUPPORTED for a shape not compiled in (1024x4, 512x4, 256x4,
 * 1024x2, 512x2). Default 1024x4. */
stt_status stt_set_slab_shape(stt_ctx *ctx, int32_t wg, int32_t tpt);

/* Slab staging. Every scoring call first folds the map into a context-owned
 * copy with columns padded to whole 1 KB pieces: an FP32 map as p = Y/sigma in
 * polar form (|p| as float32, arg p as a 32-bit fraction of a turn, 8 bytes per
 * pixel), an FP16 map as its own 4-byte words. dma = 1 (default) streams slabs
 * of it into two LDS buffers with direct global-to-LDS copies, overlapping the
 * next slab with the current one; dma = 0 stages through registers into one
 * buffer. Scores are identical. */
stt_status stt_set_staging(stt_ctx *ctx, int32_t dma);

/* Phase-factor evaluation: hw = 1 (default) the hardware sine/cosine
 * instructions (argument in turns; measured on gfx950 at most 1.3e-7 from the
 * true values over a full turn); hw = 0 a polynomial accurate to 1.5e-7. */
stt_status stt_set_trig(stt_ctx *ctx, int32_t hw);

/* Template generation (Sec. III: each template from six random numbers plus
 * a random delay, before Eq. 8). Writes out_dev[i] = track j = first + i for
 * i in [0, n): Philox4x32-10 with key = seed, counter = (j, stream, b) for
 * blocks b = 0, 1; the time extent is uniform over the pairs (t0, t2) with
 * t2 - t0 + 1 >= min_len, the control frequencies are uniform on [0, F) and
 * the delay uniform on the integers [dtau_center - dtau_max, dtau_center +
 * dtau_max] (the same random word whatever the centre, so a patch moves every
 * delay by exactly dtau_center). Requires 2 <= min_len <= T <= STT_MAX_T,
 * 1 <= F <= STT_MAX_F, 0 <= dtau_max, |dtau_center| + dtau_max < 2^30,
 * first + n <= 2^32. n = 0 is a no-op. */
stt_status stt_make_tracks(stt_ctx *ctx, const stt_gen *gen, int32_t T, int32_t F, int64_t first,
                           int64_t n, stt_track *out_dev);

/* Score tracks on one map (Eq. 8) and reduce them (Sec. III, Sec. V).
 * Tracks are either generated (tracks_dev == NULL: j = first + i drawn as by
 * stt_make_tracks with `gen`) or given (tracks_dev[i] has index j = first + i;
 * `gen` may then be NULL). For i in [0, n): if snr_dev is non-NULL,
 * snr_dev[i] = z_j (FP32); if best_key_dev is non-NULL, *best_key_dev is
 * max-merged with the best key over the n tracks. Given tracks are validated
 * on the device: an out-of-range track scores NaN (never wins). Requires
 * first + n <= 2^32 and a valid map (T, F within range, ld >= F). */
stt_status stt_score(stt_ctx *ctx, const stt_map *map, const stt_gen *gen, const stt_track *tracks_dev,
                     int64_t first, int64_t n, int32_t norm, float *snr_dev, uint64_t *best_key_dev);

/* stt_score without allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). Arguments, results and errors as stt_score; the scores are the
 * same bits. The binning scratch and the folded map live in one static
 * device array per GPU (about 71.7 MB, held from library load until the
 * process ends; its address is taken by stt_create), so this call makes no
 * allocation, records no timing events, and limits the call to
 * n <= 4194304 templates and maps whose folded copy (T x F rounded up to a
 * multiple of 128, 8 bytes per pixel) fits 32 MiB -- STT_ERANGE otherwise,
 * before anything is enqueued. Every call on one GPU shares that array and
 * leaves its contents behind; calls that overlap on one GPU (other streams,
 * other contexts, other host threads) race and must be serialised by the
 * caller. STT_EHIP if the array's address could not be taken on this device. */
stt_status stt_score_noalloc(stt_ctx *ctx, const stt_map *map, const stt_gen *gen, const stt_track *tracks_dev,
                             int64_t first, int64_t n, int32_t norm, float *snr_dev, uint64_t *best_key_dev);

/* Free-t_mid templates (an addition: the paper's six random numbers, with t_mid
 * free instead of at the midpoint). Generation as stt_make_tracks, plus
 * t1 = t0 + floor(x * (t2 - t0 + 1) / 2^32) from the last word x of the second
 * Philox block. Scoring as stt_score (Eq. 8, one pixel per column): at column
 * t the row is floor(f(xi)/256), xi the root in [0, 1] of t(xi) = t, computed
 * exactly (an FP32 evaluation inside a certified error window, else FP64
 * Newton refinement of the root, else an exact 128-bit integer decision).
 * Generated templates (from 4096 on, when two slabs of a column fit 80 KB) are
 * binned by time extent and scored from LDS slabs; given lists and small
 * calls take one wave per template. Both give the same bits. */
stt_status stt_make_tracks_tm(stt_ctx *ctx, const stt_gen *gen, int32_t T, int32_t F, int64_t first, int64_t n,
                              stt_track_tm *out_dev);
stt_status stt_score_tm(stt_ctx *ctx, const stt_map *map, const stt_gen *gen, const stt_track_tm *tracks_dev,
                        int64_t first, int64_t n, int32_t norm, float *snr_dev, uint64_t *best_key_dev);

/* Delay-maximised scores: the reading of "phase-maximised" (Sec. III, Eq. 8)
 * that maximises the statistic over the delay per template instead of drawing
 * one. Track j (generated or given, as in stt_score) keeps its time extent and
 * control frequencies; its own delay is replaced by each of the grid delays
 * dtau_m = dtau0 + m * dtau_step (2^-28 s units), m = 0 .. n_tau - 1. For i in
 * [0, n): snr_dev[i] = max_m z_j(dtau_m) (FP32; ties keep the lowest m) and
 * tau_idx_dev[i] = that m; an invalid given track (or NaN map data) gives NaN
 * and -1. Either output may be NULL (the context then keeps its own). The
 * key of (max, j) is max-merged into *best_key_dev (may be NULL). Requires
 * 1 <= n_tau <= 65536 and every grid delay in (-2^30, 2^30). The row walk and
 * the pixel gathers are shared by the delays (8 per kernel launch). */
stt_status stt_score_maxdelay(stt_ctx *ctx, const stt_map *map, const stt_gen *gen, const stt_track *tracks_dev,
                              int64_t first, int64_t n, int32_t dtau0, int32_t dtau_step, int32_t n_tau, int32_t norm,
                              float *snr_dev, int32_t *tau_idx_dev, uint64_t *best_key_dev);

/* ---- Significance of per-map maxima (the step after the search) ----
 *
 * The search keeps the best key of every map (Sec. V records the maximum per
 * spectrogram); over background maps (time slides) these give the maximum's
 * distribution in noise. For each foreground key i < n_fg:
 *   n_louder_dev[i] = number of background keys at least as loud (int64),
 *   fap_dev[i] = n_louder_dev[i] / n_bg (FP32), the false-alarm probability;
 * and *z_alpha_dev = the ceil(alpha n_bg)-th largest background score (at least
 * the largest one), so that a foreground maximum strictly above it has FAP <
 * alpha (Sec. IV detects at FAP < 0.1 %). Loudness compares the keys' FP32
 * scores; an empty key (0) is quieter than any score and counts as -inf in the
 * threshold. Keys are 8-byte device arrays as written by the scorers. Any of
 * the three outputs may be NULL (z_alpha needs 0 < alpha <= 1 and
 * ceil(alpha n_bg) <= 8192); 1 <= n_bg <= 2^38, n_fg <= 2^38. Exact counts: n_fg * n_bg
 * comparisons. */
stt_status stt_significance(stt_ctx *ctx, const uint64_t *bg_keys_dev, int64_t n_bg, const uint64_t *fg_keys_dev,
                            int64_t n_fg, double alpha, int64_t *n_louder_dev, float *fap_dev, float *z_alpha_dev);

/* Follow-up of the loudest maps (Sec. V: the ~10 loudest events are searched
 * again, deeper and with a new seed, and runs combine by their maximum).
 * keys_dev[m] (device, n_maps 8-byte keys as the scorers write them) holds map
 * m's best key. Map m's rank is the number of maps at least as loud, itself
 * included (counted on the device as stt_significance counts). Every map of
 * rank <= k (k >= 1; ties at the k-th place can leave maps out) is scored
 * again with templates j = 0 .. n_deep-1 drawn from `gen` with Philox stream
 * gen->stream + m (use a seed the first search did not, or it repeats its
 * templates), and that search's best key is max-merged into keys_dev[m].
 * chosen_host (host, room for n_maps, may be NULL) receives the searched
 * maps' indices in increasing order and *n_chosen (host, may be NULL) their
 * number. The maps (host array of n_maps descriptors) are validated first;
 * the call then synchronises the stream once to read the ranks back. */
stt_status stt_follow_up(stt_ctx *ctx, const stt_map *maps_host, int32_t n_maps, uint64_t *keys_dev,
                         const stt_gen *gen, int64_t n_deep, int32_t k, int32_t norm, int32_t *chosen_host,
                         int32_t *n_chosen);

/* ---- Map formation: the complex SNR maps the search scores, from strain ----
 *
 * Two detectors' strain streams I and J become cross-power maps (Y, sigma) in
 * the layout above (Sec. II, Eq. 7, and the formalism appendix), with the
 * segmenting of Sec. IV (columns of M samples overlapping by half, each
 * weighted by the periodic Hann window w[n] = sin^2(pi n / M)):
 *   s~(t; k) = dt sum_n w[n] s[t M/2 + n] e^{-2 pi i k n / M}   (dt = 1/fs)
 *   Nrm = M dt 3/8   (DFT normalisation with the window's mean square)
 *   P'(t; k) = mean of (2/Nrm) |s~(t'; k)|^2 over 2 <= |t' - t| <= nb + 1
 *              (the neighbouring columns that share no samples with t)
 *   Y = (2/Nrm) conj(s~_I(t; k)) s~_J(t'; k),  sigma = sqrt(P'_I(t) P'_J(t') / 2)
 * with t' = (t + shift) mod T for a time slide of J by `shift` columns (0:
 * zero lag). This is the appendix's estimator with the direction filter set to
 * 1: the direction enters through Eq. 8's phase factor. Y / sigma is then twice
 * the paper's lambda s~_I^* s~_J, with unit-variance real and imaginary parts
 * in Gaussian noise. Row r = k - k_lo has frequency (k_lo + r) fs / M Hz, so a
 * map from these entry points scores with fq4_lo = 16 k_lo fs / M and
 * dfq4 = 16 fs / M (integers when fs / M is a multiple of 1/16 Hz).
 * Computed in FP32: scale strain so that |s~|^2 stays a normal FP32 number
 * (the maps' Y / sigma does not depend on a scale of either stream). */
typedef struct {
    double fs;      /* sample rate, Hz (> 0) */
    int32_t M;      /* samples per column: a power of two in [8, 8192]; columns start every M/2 samples */
    int32_t k_lo;   /* first frequency bin kept */
    int32_t F;      /* bins kept, k_lo .. k_lo + F - 1, all < M/2 */
    int32_t nb;     /* neighbour columns per side in P' (>= 1) */
} stt_spectro;

/* Column spectra and P' of one detector. strain_dev: n_samples FP32 samples,
 * 8-byte aligned; columns t = 0 .. T-1 cover samples [t M/2, t M/2 + M), so
 * (T + 1) M / 2 <= n_samples; 4 <= T <= 65535. Outputs (caller-owned):
 * spec_dev [T][F] complex64 (interleaved FP32, 8-byte aligned) = s~, and
 * psd_dev [T][F] FP32 = P'. */
stt_status stt_spectra(stt_ctx *ctx, const stt_spectro *p, const float *strain_dev, int64_t n_samples, int32_t T,
                       float *spec_dev, float *psd_dev);

/* Time-slide maps from two detectors' stt_spectra outputs (same p and T).
 * For k < n_slides: map k pairs column t of I with column (t + shifts[k]) mod T
 * of J (shifts: host array, any integers) and writes Y into Y_dev[k] and sigma
 * into sigma_dev[k] (host arrays of caller-owned device pointers; each map is
 * [T][ld], ld >= F, Y complex64 8-byte aligned, sigma FP32). Shifts of at
 * least 2 columns decorrelate a transient shorter than the shift. */
stt_status stt_form_maps(stt_ctx *ctx, const stt_spectro *p, int32_t T, const float *spec_i_dev,
                         const float *psd_i_dev, const float *spec_j_dev, const float *psd_j_dev, int32_t n_slides,
                         const int32_t *shifts, int64_t ld, float *const *Y_dev, float *const *sigma_dev);

/* Max/argmax over an existing score array (Sec. III keeps the template with
 * the largest statistic; Sec. V records that maximum per spectrogram and
 * combines runs by their maximum): *best_key_dev is max-merged with the best
 * key over snr_dev[0..n), the index of element i being first + i. Ties go to
 * the lowest index, NaN never wins (the key format above). */
stt_status stt_argmax(stt_ctx *ctx, const float *snr_dev, int64_t n, int64_t first,
                      uint64_t *best_key_dev);

/* FP16 storage of a map (a precision addition; the paper states no
 * precision). Packs an STT_C64F32 map into out_dev, [T][out_ld] 32-bit words
 * (4 bytes per pixel, caller-owned, out_ld >= F), each the complex SNR
 * p = Y/sigma (formed in FP32 with a correctly rounded division) in polar
 * form: the magnitude |p| (FP64) scaled by 2^-e and rounded to binary16 to
 * nearest even in the high half, e = ceil(log2(max |p|)) - 15 keeping every
 * scaled magnitude at most 2^15; the argument atan2(Im p, Re p) as a fraction
 * of a turn rounded to the nearest multiple of 2^-16 (ties to even, modulo one
 * turn) in the low half. |p| keeps 11 significant bits and arg p is within
 * pi 2^-16 rad, so |stored - p| <= (2^-11 + pi 2^-16) |p|: the precision of
 * binary16 (re, im) pairs, in a form whose phase adds to Eq. 8's exactly (the
 * scorers take one cosine per pixel). Writes e to *scale_exp (host).
 * Synchronises the stream (the exponent is read back); STT_EINVAL if the map
 * holds a non-finite value. The packed map is used as stt_map{dtype =
 * STT_P16, Y = out_dev, sigma = NULL, scale_exp = e, ld = out_ld}. */
stt_status stt_map_pack_p16(stt_ctx *ctx, const stt_map *map, void *out_dev, int64_t out_ld, int32_t *scale_exp);

/* The K best scores of snr_dev[0..n) (Sec. V's follow-up of the loudest
 * candidates), ordered by score descending then index ascending; NaN ranks
 * lowest. Element i has index first + i. Writes idx_dev[0..K) (int64) and/or
 * val_dev[0..K) (float; either may be NULL, not both). Device-resident: a
 * radix select over the 64-bit (score, ~index) keys, no host round trip.
 * Requires 0 <= K <= min(n, 8192). */
stt_status stt_topk(stt_ctx *ctx, const float *snr_dev, int64_t n, int64_t first, int32_t K, int64_t *idx_dev,
                    float *val_dev);

/* FP64 re-score of K tracks (Eq. 8) from an FP32 (STT_C64F32) map: z_dev[i]
 * (double) for track j = idx_dev[i], drawn from `gen` (tracks_dev == NULL) or
 * read at tracks_dev[j - first] from a list of n_tracks. Rows and phases are
 * exact integers, terms and sums FP64; an invalid track, or j outside the
 * list (or outside [0, 2^32) for drawn tracks), gives NaN. */
stt_status stt_rescore_f64(stt_ctx *ctx, const stt_map *map, const stt_gen *gen, const stt_track *tracks_dev,
                           int64_t n_tracks, int64_t first, const int64_t *idx_dev, int32_t K, int32_t norm,
                           double *z_dev);

/* Batch of maps (the paper's n_ts time-shifted background maps, Sec. V; one
 * recorded maximum per spectrogram). Map m (maps_host[m], host array; all of
 * one dtype, each its own T, F, ld) is scored with n_trk_host[m] templates
 * j = 0 .. n_trk-1 drawn from `gen` with Philox stream gen->stream + m.
 * best_key_per_map_dev[m] is max-merged with map m's best key (indices are
 * per map); if snr_dev_host (host array of n_maps device pointers, entries
 * may be NULL) is given, snr_dev_host[m][j] receives the scores. All maps are
 * binned and scored by one persistent launch whose workgroups take (map,
 * block) items from a device queue. With graphs on (default) the whole call
 * is captured in a HIP graph, replayed while every argument stays the same.
 * Any change of arguments re-uploads the descriptor tables (synchronising the
 * stream) and re-captures. Requires sum n_trk < 2^32. */
stt_status stt_score_batch(stt_ctx *ctx, const stt_map *maps_host, int32_t n_maps, const stt_gen *gen,
                           const int64_t *n_trk_host, int32_t norm, uint64_t *best_key_per_map_dev,
                           float *const *snr_dev_host);

/* Graph capture of batches on (1, default) or off (0: direct launches). */
stt_status stt_set_graph(stt_ctx *ctx, int32_t on);

/* Autotuner of the slab scorer: times every compiled workgroup shape with LDS
 * slab budgets of 160, 112, 80 and 48 KB on `n` templates from `gen` on this
 * map (one warm-up and three timed calls each, HIP events, kernel time only),
 * applies the fastest to the context (stt_set_slab_shape, stt_set_path's
 * lds_bytes) and writes it as choice_out[3] = {wg, tpt, lds_bytes} (host,
 * may be NULL). With cache_path (a JSON file, may be NULL) the choice is
 * looked up first under a key of (GPU architecture, generation tag of the
 * scorers' inner loop, F, dtype, power-of-two buckets of T and n, trig mode)
 * and stored after a search. Synchronises. */
stt_status stt_autotune(stt_ctx *ctx, const stt_map *map, const stt_gen *gen, int64_t n, const char *cache_path,
                        int32_t *choice_out);

/* Autotuner of the batch scorer: the same search, timing the persistent batch
 * launch of stt_score_batch itself on these maps (direct launches, one warm-up
 * and two timed batches per candidate, kernel time only), since the best shape
 * of a queue of many uneven maps differs from a single map's. Arguments as in
 * stt_score_batch; cache key (GPU architecture, generation tag, "batch", largest F, dtype,
 * power-of-two buckets of the longest T, of n_maps and of the total template
 * count, trig mode). Uses a temporary device buffer of n_maps keys. Applies and
 * returns the choice as stt_autotune does. Synchronises. */
stt_status stt_autotune_batch(stt_ctx *ctx, const stt_map *maps_host, int32_t n_maps, const stt_gen *gen,
                              const int64_t *n_trk_host, const char *cache_path, int32_t *choice_out);

/* ---- differentiation (an addition; the paper scores only pixel sets) ----
 * theta_dev: [n][6] float32 per template, (tau0, tau2, phi0, phi1, phi2,
 * dtau_ms): start and end time in columns, control frequencies in rows
 * (continuous), delay in milliseconds. K_dev: [n] int32 sample counts (K = the
 * seed template's N). The smooth statistic z~ interpolates
 * G(t, r) = Re[exp(2 pi i f(r) dtau) p(t, r)] (the Eq. 8 term) bilinearly at
 * K points along the Eq. 6 curve, u = clamp(t, 0, T-1), v = clamp(f - 1/2,
 * 0, F-1), and divides the sum by sqrt(K); a clamped coordinate has zero
 * derivative. Requires F >= 2. */

/* Templates j = idx_dev[i] (device int64) drawn as by stt_make_tracks. */
stt_status stt_tracks_at(stt_ctx *ctx, const stt_gen *gen, int32_t T, int32_t F, const int64_t *idx_dev, int64_t n,
                         stt_track *out_dev);

/* theta and K of plain templates: (t0, t2, f0/256, f1/256, f2/256, dtau 2^-28 s in ms), K = N. */
stt_status stt_tracks_to_theta(stt_ctx *ctx, const stt_track *tracks_dev, int64_t n, float *theta_dev,
                               int32_t *K_dev);

/* Forward: z_dev[i] = z~(theta_i). */
stt_status stt_smooth(stt_ctx *ctx, const stt_map *map, const float *theta_dev, const int32_t *K_dev, int32_t n,
                      float *z_dev);

/* Forward and hand-written backward: z_dev[i] = z~(theta_i) and grad_dev[i][q] = dz~/dtheta_q. */
stt_status stt_grad(stt_ctx *ctx, const stt_map *map, const float *theta_dev, const int32_t *K_dev, int32_t n,
                    float *z_dev, float *grad_dev);

/* Projected gradient ascent of z~ for every template (Sec. V's deeper
 * follow-up of the loudest candidates, here as a local refinement): `steps`
 * iterations; the five positions move by eta_px along g/|g|, the delay by
 * eta_ms along sign(g), eta falling linearly over the steps from sched_host =
 * {px0, px1, ms0, ms1} (host; NULL = {1, 0.02, 0.5, 0.01}); after each step
 * theta is projected onto 0 <= tau <= T-1, tau2 - tau0 >= min_len - 1,
 * 0 <= phi < F, |dtau| <= dtau_max (2^-28 s units). On return theta_dev holds
 * each template's best iterate (the projected start included) and
 * z_smooth_dev its z~. If plain_dev is given the best iterates are rounded to
 * plain templates (times half up and widened to min_len, frequencies
 * floor(256 phi) inside the band, delay to the nearest unit); if also
 * z_plain_dev, those are scored with the plain statistic (norm). One
 * workgroup per template runs all its steps in a single launch. */
stt_status stt_refine(stt_ctx *ctx, const stt_map *map, int32_t min_len, int32_t dtau_max, float *theta_dev,
                      const int32_t *K_dev, int32_t n, int32_t steps, const float *sched_host, float *z_smooth_dev,
                      stt_track *plain_dev, float *z_plain_dev, int32_t norm);

/* Host helpers for the key format (no device work). */
uint64_t stt_key_encode(float z, uint32_t j);
void stt_key_decode(uint64_t key, float *z, uint32_t *j);

#ifdef __cplusplus
}
#endif

#endif /* STT_H */
