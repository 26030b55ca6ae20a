// Measured peaks of the resources the kernel-matrix build is bound by, so that
// every roofline fraction can be stated against the chip as measured here as
// well as against its published figures:
//   HBM copy          bytes read + written per second by a plain streaming copy
//   MFMA BF16 / FP32  flops per second of independent v_mfma_f32_32x32x16_bf16 /
//                     v_mfma_f32_32x32x2f32 chains (the distance tiles' products)
//   v_exp_f32         exponentials per second (the tuning sums' exp per grid point)
//   VALU FMA          lane operations per second of v_fma_f32 chains (the
//                     direct-difference tiles, the selection epilogue)
// Each kernel keeps enough independent chains per wavefront to cover the
// instruction latency and launches enough wavefronts to fill every CU.
#include <algorithm>
#include <vector>

#include "kvb_ctx.h"
#include "kvb_device.h"

namespace kvb {

typedef __bf16 pbf16x8 __attribute__((ext_vector_type(8)));
typedef float pf32x16 __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256) void k_peak_copy(const float4* __restrict__ in, float4* __restrict__ out,
                                                   int64_t n4)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n4; i += stride) out[i] = in[i];
}

// Four independent accumulators per wavefront; the operands depend on the
// lane so that nothing folds at compile time; the sums are written so that
// nothing is dead.
__global__ __launch_bounds__(256) void k_peak_mfma_bf16(int iters, float* __restrict__ sink)
{
    const int lane = threadIdx.x & 63;
    pbf16x8 a, b;
    for (int e = 0; e < 8; ++e) {
        a[e] = static_cast<__bf16>(1.0f + 0.001f * static_cast<float>(lane + e));
        b[e] = static_cast<__bf16>(0.5f - 0.001f * static_cast<float>(lane - e));
    }
    pf32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
    for (int i = 0; i < iters; ++i) {
        c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c3, 0, 0, 0);
    }
    float s = 0.f;
    for (int r = 0; r < 16; ++r) s += c0[r] + c1[r] + c2[r] + c3[r];
    sink[static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_mfma_f32(int iters, float* __restrict__ sink)
{
    const int lane = threadIdx.x & 63;
    const float a = 1.0f + 0.001f * static_cast<float>(lane), b = 0.5f - 0.001f * static_cast<float>(lane);
    pf32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
    for (int i = 0; i < iters; ++i) {
        c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c3, 0, 0, 0);
    }
    float s = 0.f;
    for (int r = 0; r < 16; ++r) s += c0[r] + c1[r] + c2[r] + c3[r];
    sink[static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

// y <- 2^(-y) stays in [1/2, 1] for y in [0, 1]: one v_exp_f32 (negated
// source) per step, eight independent chains per lane
__global__ __launch_bounds__(256) void k_peak_exp(int iters, float* __restrict__ sink)
{
    float y[8];
    for (int c = 0; c < 8; ++c) y[c] = 0.01f * static_cast<float>((threadIdx.x + c) & 63);
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < 8; ++c) y[c] = __builtin_amdgcn_exp2f(-y[c]);
    float s = 0.f;
    for (int c = 0; c < 8; ++c) s += y[c];
    sink[static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

// y <- y * a + b with |a| < 1: eight independent v_fma_f32 chains per lane
__global__ __launch_bounds__(256) void k_peak_fma(int iters, float a, float* __restrict__ sink)
{
    float y[8];
    for (int c = 0; c < 8; ++c) y[c] = 0.01f * static_cast<float>((threadIdx.x + c) & 63);
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < 8; ++c) y[c] = fmaf(y[c], a, 0.25f);
    float s = 0.f;
    for (int c = 0; c < 8; ++c) s += y[c];
    sink[static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

}  // namespace kvb

using kvbh::fail;

int kvb_peak_probe(kvb_ctx ctx, int32_t kind, double* rate_host, double* ms_host)
{
    if (kvbh::check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, rate_host != nullptr, "rate_host is required");
    KVB_REQUIRE(ctx, kind >= KVB_PEAK_HBM_COPY && kind <= KVB_PEAK_VALU_FMA, "unknown peak kind %d", kind);
    KVB_DEVICE_WORK(ctx);
    hipStream_t st = ctx->stream;
    constexpr int BLOCKS = 256 * 16, THREADS = 256, REPS = 5;
    const size_t sink_bytes = sizeof(float) * BLOCKS * THREADS;
    const int64_t copy_bytes = int64_t(1) << 31;   // 2 GiB read + 2 GiB written per launch
    const size_t need = kind == KVB_PEAK_HBM_COPY ? size_t(2 * copy_bytes) : sink_bytes;
    void* buf = nullptr;
    if (hipMalloc(&buf, need) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, KVB_E_NOMEM, "hipMalloc of %zu probe bytes failed", need);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = KVB_OK;
    double per_launch = 0.0;   // work units per launch
    const int iters = 4096;
    auto launch = [&]() {
        switch (kind) {
        case KVB_PEAK_HBM_COPY: {
            const int64_t n4 = copy_bytes / 16;
            float4* in = static_cast<float4*>(buf);
            hipLaunchKernelGGL(kvb::k_peak_copy, dim3(BLOCKS * 2), dim3(THREADS), 0, st, in, in + n4, n4);
            per_launch = 2.0 * static_cast<double>(copy_bytes);
            break;
        }
        case KVB_PEAK_MFMA_BF16:
            hipLaunchKernelGGL(kvb::k_peak_mfma_bf16, dim3(BLOCKS), dim3(THREADS), 0, st, iters,
                               static_cast<float*>(buf));
            per_launch = double(BLOCKS) * (THREADS / 64) * iters * 4 * (2.0 * 32 * 32 * 16);
            break;
        case KVB_PEAK_MFMA_F32:
            hipLaunchKernelGGL(kvb::k_peak_mfma_f32, dim3(BLOCKS), dim3(THREADS), 0, st, iters / 4,
                               static_cast<float*>(buf));
            per_launch = double(BLOCKS) * (THREADS / 64) * (iters / 4) * 4 * (2.0 * 32 * 32 * 2);
            break;
        case KVB_PEAK_EXP:
            hipLaunchKernelGGL(kvb::k_peak_exp, dim3(BLOCKS), dim3(THREADS), 0, st, iters, static_cast<float*>(buf));
            per_launch = double(BLOCKS) * THREADS * iters * 8;
            break;
        default:
            hipLaunchKernelGGL(kvb::k_peak_fma, dim3(BLOCKS), dim3(THREADS), 0, st, iters, 0.5f,
                               static_cast<float*>(buf));
            per_launch = double(BLOCKS) * THREADS * iters * 8;
            break;
        }
    };
    if (kind == KVB_PEAK_HBM_COPY && hipMemsetAsync(buf, 0, need, st) != hipSuccess) rc = KVB_E_HIP;
    if (rc == KVB_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) rc = KVB_E_HIP;
    std::vector<float> ms(REPS, 0.f);
    if (rc == KVB_OK) {
        launch();   // warm-up
        for (int r = 0; r < REPS && rc == KVB_OK; ++r) {
            if (hipEventRecord(e0, st) != hipSuccess) rc = KVB_E_HIP;
            launch();
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms[r], e0, e1) != hipSuccess)
                rc = KVB_E_HIP;
        }
        if (hipGetLastError() != hipSuccess) rc = KVB_E_HIP;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (rc != KVB_OK) return fail(ctx, rc, "peak probe %d failed", kind);
    std::sort(ms.begin(), ms.end());
    const double best = ms[0];
    *rate_host = per_launch / (best * 1e-3);
    if (ms_host) *ms_host = best;
    return KVB_OK;
}
