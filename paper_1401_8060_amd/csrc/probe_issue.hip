// probe_issue.hip -- vector-ALU issue rates of the instructions in the scorers'
// inner loops, and the memory-side ceilings the scorers are measured against
// (streaming reads served by HBM or by the MALL, LDS reads at random rows and
// conflict-free), measured on the device (gfx950).
//
// Each probe kernel runs, in every lane, eight independent chains of one
// instruction (register operands only, no memory), unrolled four times, so the
// SIMDs are limited by issue rather than by latency. The rate reported is
// lane-instructions per shader clock per compute unit:
//   threads x iterations x 32 / (kernel seconds x shader clock x CUs).
// The shader clock is measured inside the same launch: the first wave reads
// the cycle counter and the constant-rate wall counter at its start and end.
// These rates feed the issue model of the scorers' instruction mix (bench.py).
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

enum Op : int {
    kFmaF32 = 0,
    kFmaF64,
    kAddF64,
    kMadU64,
    kLshlAdd,
    kAlignbit,
    kAddU32,
    kSinF32,
    kCosF32,
    kFmaMix,
    kCndmask,
    kCvtF16,
    kMulLo,
    kAdd3,
    kFmacF32,
    kCndmaskS,
    kNumOps
};

const char *const kNames[kNumOps] = {"v_fma_f32",   "v_fma_f64", "v_add_f64",     "v_mad_u64_u32",
                                     "v_lshl_add_u32", "v_alignbit_b32", "v_add_u32", "v_sin_f32",
                                     "v_cos_f32",   "v_fma_mix_f32", "v_cndmask_b32", "v_cvt_f32_f16",
                                     "v_mul_lo_u32", "v_add3_u32", "v_fmac_f32",  "v_cndmask_b32_e64"};

template <int OP>
__device__ __forceinline__ void step32(uint32_t &x, uint32_t y, uint32_t z)
{
    if constexpr (OP == kFmaF32) asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(x) : "v"(y), "v"(z));
    if constexpr (OP == kLshlAdd) asm volatile("v_lshl_add_u32 %0, %0, 3, %1" : "+v"(x) : "v"(y));
    if constexpr (OP == kAlignbit) asm volatile("v_alignbit_b32 %0, %1, %0, 9" : "+v"(x) : "v"(y));
    if constexpr (OP == kAddU32) asm volatile("v_add_u32 %0, %0, %1" : "+v"(x) : "v"(y));
    if constexpr (OP == kSinF32) asm volatile("v_sin_f32 %0, %0" : "+v"(x));
    if constexpr (OP == kCosF32) asm volatile("v_cos_f32 %0, %0" : "+v"(x));
    if constexpr (OP == kFmaMix) asm volatile("v_fma_mix_f32 %0, %1, %2, %0 op_sel_hi:[0,1,0]" : "+v"(x) : "v"(y), "v"(z));
    if constexpr (OP == kCndmask) asm volatile("v_cndmask_b32 %0, %0, %1, vcc" : "+v"(x) : "v"(y));
    if constexpr (OP == kCvtF16) asm volatile("v_cvt_f32_f16 %0, %0" : "+v"(x));
    if constexpr (OP == kMulLo) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x) : "v"(y));
    if constexpr (OP == kAdd3) asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(x) : "v"(y), "v"(z));
    if constexpr (OP == kFmacF32) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(x) : "v"(y), "v"(z));
    // the select mask in an SGPR pair written once, as the scorers' masked walks do
    if constexpr (OP == kCndmaskS) asm volatile("v_cndmask_b32_e64 %0, %0, %1, s[20:21]" : "+v"(x) : "v"(y));
}

template <int OP>
__device__ __forceinline__ void step64(uint64_t &x, uint64_t y, uint32_t z)
{
    if constexpr (OP == kFmaF64) asm volatile("v_fma_f64 %0, %1, %0, %1" : "+v"(x) : "v"(y));
    if constexpr (OP == kAddF64) asm volatile("v_add_f64 %0, %0, %1" : "+v"(x) : "v"(y));
    if constexpr (OP == kMadU64) asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(x) : "v"(z), "v"(z) : "vcc");
}

constexpr bool is64(int op) { return op == kFmaF64 || op == kAddF64 || op == kMadU64; }

// clk[0..1]: cycle and wall counters at the start of the first wave, clk[2..3] at its end.
template <int OP>
__global__ __launch_bounds__(256) void k_probe(int iters, uint32_t *sink, uint64_t *clk)
{
    const bool timer = blockIdx.x == 0 && threadIdx.x == 0;
    if (timer) {
        clk[0] = (uint64_t)clock64();
        clk[1] = (uint64_t)wall_clock64();
    }
    const uint32_t t = threadIdx.x + 1;
    uint32_t acc = 0;
    if constexpr (is64(OP)) {
        uint64_t a[8];
        const uint64_t y = 0x3FF0000000000001ull;  // 1 + 2^-52: values stay finite over the run
#pragma unroll
        for (int c = 0; c < 8; ++c) a[c] = 0x3FF0000000000000ull + t + c;
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int c = 0; c < 8; ++c) step64<OP>(a[c], y, t);
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) acc ^= (uint32_t)a[c] ^ (uint32_t)(a[c] >> 32);
    } else {
        uint32_t a[8];
        const uint32_t y = 0x3F800001u, z = 0x3C000000u;
#pragma unroll
        for (int c = 0; c < 8; ++c) a[c] = 0x3F000000u + t * 8 + c;
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int c = 0; c < 8; ++c) step32<OP>(a[c], y, z);
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) acc ^= a[c];
    }
    if (acc == 0x12345678u) sink[0] = acc;  // keeps the chains live; practically never stored
    if (timer) {
        clk[2] = (uint64_t)clock64();
        clk[3] = (uint64_t)wall_clock64();
    }
}

template <int OP>
hipError_t launch(int grid, int iters, uint32_t *sink, uint64_t *clk, hipStream_t st)
{
    hipLaunchKernelGGL(k_probe<OP>, dim3(grid), dim3(256), 0, st, iters, sink, clk);
    return hipGetLastError();
}

hipError_t launch_op(int op, int grid, int iters, uint32_t *sink, uint64_t *clk, hipStream_t st)
{
    switch (op) {
    case kFmaF32: return launch<kFmaF32>(grid, iters, sink, clk, st);
    case kFmaF64: return launch<kFmaF64>(grid, iters, sink, clk, st);
    case kAddF64: return launch<kAddF64>(grid, iters, sink, clk, st);
    case kMadU64: return launch<kMadU64>(grid, iters, sink, clk, st);
    case kLshlAdd: return launch<kLshlAdd>(grid, iters, sink, clk, st);
    case kAlignbit: return launch<kAlignbit>(grid, iters, sink, clk, st);
    case kAddU32: return launch<kAddU32>(grid, iters, sink, clk, st);
    case kSinF32: return launch<kSinF32>(grid, iters, sink, clk, st);
    case kCosF32: return launch<kCosF32>(grid, iters, sink, clk, st);
    case kFmaMix: return launch<kFmaMix>(grid, iters, sink, clk, st);
    case kCndmask: return launch<kCndmask>(grid, iters, sink, clk, st);
    case kCvtF16: return launch<kCvtF16>(grid, iters, sink, clk, st);
    case kMulLo: return launch<kMulLo>(grid, iters, sink, clk, st);
    case kAdd3: return launch<kAdd3>(grid, iters, sink, clk, st);
    case kFmacF32: return launch<kFmacF32>(grid, iters, sink, clk, st);
    case kCndmaskS: return launch<kCndmaskS>(grid, iters, sink, clk, st);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------- memory-side probes

// Streaming read of n4 16-byte words, `reps` passes, every lane a grid-stride walk; the sum keeps
// the loads live.
__global__ __launch_bounds__(256) void k_stream_read(const float4 *p, int64_t n4, int reps, float *sink)
{
    float acc = 0.0f;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int r = 0; r < reps; ++r)
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) {
            const float4 v = p[i];
            acc += (v.x + v.y) + (v.z + v.w);
        }
    if (acc == 1.2345e-30f) sink[0] = acc;
}

// LDS reads of 8 bytes per lane from a 16 KB table (2048 elements): at rows drawn by a per-lane
// linear congruential sequence (random banks, as the scorers' gathers) or at consecutive rows
// (lane l reads element base + l: conflict-free). Eight independent sequences per lane.
template <bool RANDOM>
__global__ __launch_bounds__(256) void k_lds_read(int iters, float *sink)
{
    __shared__ float2 tab[2048];
    for (int i = threadIdx.x; i < 2048; i += 256) tab[i] = make_float2((float)i, 1.0f);
    __syncthreads();
    uint32_t st[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) st[c] = (blockIdx.x * 256u + threadIdx.x) * 2654435761u + c * 40503u + 1u;
    float acc = 0.0f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            uint32_t e;
            if (RANDOM) {
                st[c] = st[c] * 1664525u + 1013904223u;
                e = st[c] >> 21;  // 11 bits: 0 .. 2047
            } else {
                e = ((uint32_t)(it * 8 + c) * 64u + threadIdx.x) & 2047u;
            }
            const float2 v = tab[e];
            acc += v.x * v.y;
        }
    }
    if (acc == 1.2345e-30f) sink[0] = acc;
}

}  // namespace

extern "C" {

// Bytes per second of a streaming read of `bytes` (a multiple of 16) repeated `reps` times per
// launch, after one untimed launch (which leaves the buffer in the caches it fits). A buffer larger
// than the MALL measures HBM; one between the L2s and the MALL measures the MALL. Returns 0, or a
// negative value on a HIP error or a bad argument.
int stt_probe_stream(int device, int64_t bytes, int reps, double *gbps_out, double *ms_out)
{
    if (bytes < 16 || bytes % 16 || reps < 1 || !gbps_out || !ms_out) return -1;
    if (hipSetDevice(device) != hipSuccess) return -2;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return -2;
    void *buf = nullptr;
    float *sink = nullptr;
    if (hipMalloc(&buf, (size_t)bytes) != hipSuccess) return -3;
    if (hipMalloc(&sink, 64) != hipSuccess) { (void)hipFree(buf); return -3; }
    int rc = 0;
    if (hipMemset(buf, 0, (size_t)bytes) != hipSuccess) rc = -4;
    const int grid = prop.multiProcessorCount * 8;
    const int64_t n4 = bytes / 16;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    if (!rc) {
        hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, nullptr, (const float4 *)buf, n4, reps, sink);
        (void)hipEventRecord(e0, nullptr);
        hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, nullptr, (const float4 *)buf, n4, reps, sink);
        (void)hipEventRecord(e1, nullptr);
        if (hipGetLastError() != hipSuccess) rc = -4;
    }
    float ms = 0.0f;
    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = -5;
    if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = -5;
    if (!rc) {
        *ms_out = ms;
        *gbps_out = (double)bytes * reps / (ms * 1e-3) / 1e9;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    (void)hipFree(buf);
    return rc;
}

// Bytes per second of 8-byte LDS reads, every CU running 8 workgroups of 256 lanes (each with its
// own 16 KB table: 8 waves per SIMD), `iters` x 8 reads per lane: random rows (random = 1) or
// conflict-free rows.
int stt_probe_lds(int device, int random, int iters, double *gbps_out, double *ms_out)
{
    if (iters < 1 || !gbps_out || !ms_out) return -1;
    if (hipSetDevice(device) != hipSuccess) return -2;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return -2;
    float *sink = nullptr;
    if (hipMalloc(&sink, 64) != hipSuccess) return -3;
    const int grid = prop.multiProcessorCount * 8;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    int rc = 0;
    auto go = [&](int it) {
        if (random) hipLaunchKernelGGL(k_lds_read<true>, dim3(grid), dim3(256), 0, nullptr, it, sink);
        else hipLaunchKernelGGL(k_lds_read<false>, dim3(grid), dim3(256), 0, nullptr, it, sink);
    };
    go(iters / 8 + 1);
    (void)hipEventRecord(e0, nullptr);
    go(iters);
    (void)hipEventRecord(e1, nullptr);
    if (hipGetLastError() != hipSuccess) rc = -4;
    float ms = 0.0f;
    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = -5;
    if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = -5;
    if (!rc) {
        *ms_out = ms;
        *gbps_out = (double)grid * 256.0 * iters * 8.0 * 8.0 / (ms * 1e-3) / 1e9;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    return rc;
}

int stt_probe_count(void) { return kNumOps; }

const char *stt_probe_name(int op) { return op >= 0 && op < kNumOps ? kNames[op] : "?"; }

// Issue rate of instruction class `op` on `device`: lane-instructions per shader clock per CU
// (rate_out), the shader clock in MHz measured during the launch (mhz_out) and the kernel time
// in ms (ms_out). Returns 0, or a negative value on a HIP error or a bad argument.
int stt_probe_issue(int device, int op, int iters, double *rate_out, double *mhz_out, double *ms_out)
{
    if (op < 0 || op >= kNumOps || iters < 1 || !rate_out || !mhz_out || !ms_out) return -1;
    if (hipSetDevice(device) != hipSuccess) return -2;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return -2;
    int wall_khz = 0;
    if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || wall_khz <= 0)
        return -2;
    const int n_cu = prop.multiProcessorCount;
    const int grid = n_cu * 8;  // 8 workgroups of 4 waves per CU: 8 waves per SIMD
    uint32_t *sink = nullptr;
    uint64_t *clk = nullptr;
    if (hipMalloc(&sink, 64) != hipSuccess) return -3;
    if (hipMalloc(&clk, 64) != hipSuccess) { (void)hipFree(sink); return -3; }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    int rc = 0;
    // one warm-up launch, then the timed one
    if (launch_op(op, grid, iters / 8 + 1, sink, clk, nullptr) != hipSuccess) rc = -4;
    (void)hipEventRecord(e0, nullptr);
    if (!rc && launch_op(op, grid, iters, sink, clk, nullptr) != hipSuccess) rc = -4;
    (void)hipEventRecord(e1, nullptr);
    uint64_t h[4] = {0, 0, 0, 0};
    float ms = 0.0f;
    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = -5;
    if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = -5;
    if (!rc && hipMemcpy(h, clk, sizeof h, hipMemcpyDeviceToHost) != hipSuccess) rc = -5;
    if (!rc) {
        const double wall_s = (double)(h[3] - h[1]) / ((double)wall_khz * 1e3);
        const double mhz = wall_s > 0 ? (double)(h[2] - h[0]) / wall_s / 1e6 : 0.0;
        const double lane_instr = (double)grid * 256.0 * (double)iters * 32.0;
        *mhz_out = mhz;
        *ms_out = ms;
        *rate_out = lane_instr / ((double)ms * 1e-3 * mhz * 1e6 * (double)n_cu);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    (void)hipFree(clk);
    return rc;
}

}  // extern "C"
