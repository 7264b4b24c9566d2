// Significance of per-map maxima (the step after the search): Sec. V records each map's
// maximum statistic; background maps (time slides) give its distribution in noise, and a map
// is significant at false-alarm probability FAP < alpha (Sec. IV: 0.1 %).
//
//   k_count_louder  for each query key, the number of reference keys at least as loud,
//                   compared on the keys' high words (the order-preserving image of the FP32
//                   score; an empty key, 0, is quieter than every score)
//   k_key_scores    the FP32 score of each key (empty keys as -inf), for the threshold's select
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stt {

constexpr int kLouderTile = 4096;  // reference high words staged in LDS per pass (16 KB)

// Grid: ceil(n_q / 256) workgroups of 256 lanes, one query per lane.
__global__ __launch_bounds__(256) void k_count_louder(const uint64_t *__restrict__ ref, int64_t n_ref,
                                                      const uint64_t *__restrict__ q, int64_t n_q,
                                                      int64_t *__restrict__ count, float *__restrict__ fap,
                                                      double n_div)
{
    __shared__ __attribute__((aligned(16))) uint32_t tile[kLouderTile];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const uint32_t hq = i < n_q ? (uint32_t)(q[i] >> 32) : 0u;
    int64_t c = 0;
    for (int64_t r0 = 0; r0 < n_ref; r0 += kLouderTile) {
        const int m = (int)(n_ref - r0 < kLouderTile ? n_ref - r0 : kLouderTile);
        __syncthreads();
        for (int k = threadIdx.x; k < m; k += 256) tile[k] = (uint32_t)(ref[r0 + k] >> 32);
        __syncthreads();
        int cc = 0;
        const int m4 = m & ~3;
        for (int k = 0; k < m4; k += 4) {  // one broadcast 16-byte LDS read per four references
            const uint4 v = *reinterpret_cast<const uint4 *>(tile + k);
            cc += (v.x >= hq) + (v.y >= hq) + (v.z >= hq) + (v.w >= hq);
        }
        for (int k = m4; k < m; ++k) cc += tile[k] >= hq;
        c += cc;
    }
    if (i < n_q) {
        if (count) count[i] = c;
        if (fap) fap[i] = (float)((double)c / n_div);
    }
}

__global__ __launch_bounds__(256) void k_key_scores(const uint64_t *__restrict__ keys, int64_t n,
                                                    float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint32_t hi = (uint32_t)(keys[i] >> 32);
    const uint32_t bits = (hi & 0x80000000u) ? (hi ^ 0x80000000u) : ~hi;  // undo the order-preserving map
    out[i] = hi == 0u ? -__builtin_inff() : __builtin_bit_cast(float, bits);
}

}  // namespace stt
