// Kernels of the learned partitioner's MLP (gfx950): BF16 MFMA GEMMs with
// fused epilogues, layout helpers, soft-target softmax cross-entropy, Adam,
// top-P routing and a counter-based generator for seeded parameters.
//
// Every GEMM here is C[M, N] = A[M, K] . B[N, K]^T with A and B row-major BF16
// (K contiguous), FP32 accumulation on v_mfma_f32_32x32x16_bf16; one
// wavefront computes one 32 x 32 output tile. M, N are multiples of 32 and K a
// multiple of 16 (the caller pads).
#include "kvb_device.h"
#include "kvb_kernels.h"

namespace kvb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    const uint32_t u = __float_as_uint(f);
    const uint32_t r = ((u >> 16) & 1u) + 0x7FFFu;
    return static_cast<uint16_t>((u + r) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

// Epilogue: v = acc (+ bias[col]); relu: v = max(v, 0); mask: v = 0 where
// mask_ref[row, col] <= 0; then optional float32 and BF16 stores.
__global__ __launch_bounds__(256) void k_gemm_nt(const uint16_t* __restrict__ A, int lda,
                                                 const uint16_t* __restrict__ B, int ldb, int M, int N, int K,
                                                 const float* __restrict__ bias, int relu,
                                                 const float* __restrict__ mask_ref, int ldm,
                                                 float* __restrict__ Cf, int ldcf, uint16_t* __restrict__ Cb,
                                                 int ldcb)
{
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int tiles_n = N / 32;
    const int tile = blockIdx.x * 4 + wave;
    if (tile >= (M / 32) * tiles_n) return;
    const int m0 = (tile / tiles_n) * 32, n0 = (tile % tiles_n) * 32;
    const int half = lane >> 5;
    const uint16_t* ap = A + static_cast<size_t>(m0 + (lane & 31)) * lda + half * 8;
    const uint16_t* bp = B + static_cast<size_t>(n0 + (lane & 31)) * ldb + half * 8;
    f32x16 acc = {};
    for (int k = 0; k < K; k += 16) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(ap + k);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(bp + k);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    const int col = n0 + (lane & 31);
    const float bcol = bias ? bias[col] : 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = m0 + 8 * (r / 4) + 4 * half + (r % 4);
        float v = acc[r] + bcol;
        if (relu) v = fmaxf(v, 0.f);
        if (mask_ref && mask_ref[static_cast<size_t>(row) * ldm + col] <= 0.f) v = 0.f;
        if (Cf) Cf[static_cast<size_t>(row) * ldcf + col] = v;
        if (Cb) Cb[static_cast<size_t>(row) * ldcb + col] = f2bf(v);
    }
}

// dst[c, r] = src[r, c] for a rows x cols BF16 matrix (32 x 32 LDS tiles).
__global__ __launch_bounds__(256) void k_transpose_bf16(const uint16_t* __restrict__ src, int rows, int cols,
                                                        uint16_t* __restrict__ dst)
{
    __shared__ uint16_t t[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int j = ty; j < 32; j += 8) {
        const int r = by + j, c = bx + tx;
        t[j][tx] = (r < rows && c < cols) ? src[static_cast<size_t>(r) * cols + c] : static_cast<uint16_t>(0);
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int c = bx + j, r = by + tx;
        if (c < cols && r < rows) dst[static_cast<size_t>(c) * rows + r] = t[tx][j];
    }
}

// Rows of a float32 matrix [valid, cols] (optionally gathered through idx) to
// BF16 [rows, ldd]; columns cols..ldd-1 and rows valid..rows-1 are zero.
__global__ __launch_bounds__(256) void k_cast_rows_bf16(const float* __restrict__ src, int cols,
                                                        const int32_t* __restrict__ idx, int valid, int rows,
                                                        int ldd, uint16_t* __restrict__ dst)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(rows) * ldd) return;
    const int r = static_cast<int>(t / ldd), c = static_cast<int>(t % ldd);
    if (c >= cols || r >= valid) {
        dst[t] = 0;
        return;
    }
    const int sr = idx ? idx[r] : r;
    dst[t] = f2bf(src[static_cast<size_t>(sr) * cols + c]);
}

__global__ __launch_bounds__(256) void k_cast_bf16(const float* __restrict__ src, int64_t cnt,
                                                   uint16_t* __restrict__ dst)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < cnt) dst[t] = f2bf(src[t]);
}

// out[c] = sum_r src[r, c] in a fixed order (float64 accumulation).
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ src, int rows, int cols,
                                                float* __restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += static_cast<double>(src[static_cast<size_t>(r) * cols + c]);
    out[c] = static_cast<float>(s);
}

// Soft-target cross-entropy, one wavefront per row of logits Z [B, NB]:
// target t_b = (1/ks) #{r : lab[i, r] == b} (a histogram built in LDS);
// loss_i = logsumexp(z) - sum_b t_b z_b; dZ = (softmax(z) - t) / B (float32 and
// BF16 copies); row losses to row_loss. Dynamic LDS: 4 * NB ints.
__global__ __launch_bounds__(256) void k_softmax_xent(const float* __restrict__ Z, int B, int NB,
                                                      const int32_t* __restrict__ lab, int ks,
                                                      float* __restrict__ dZ, uint16_t* __restrict__ dZb,
                                                      double* __restrict__ row_loss)
{
    extern __shared__ int s_hist[];
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int i = blockIdx.x * 4 + wave;
    if (i >= B) return;
    int* hist = s_hist + wave * NB;
    for (int b = lane; b < NB; b += WAVE) hist[b] = 0;
    wave_lds_sync();
    const int32_t* li = lab + static_cast<size_t>(i) * ks;
    for (int r = lane; r < ks; r += WAVE) {
        const int b = li[r];
        if (b >= 0 && b < NB) atomicAdd(&hist[b], 1);
    }
    wave_lds_sync();
    const float* z = Z + static_cast<size_t>(i) * NB;
    float mx = -INFINITY;
    for (int b = lane; b < NB; b += WAVE) mx = fmaxf(mx, z[b]);
    mx = wave_max_f32(mx);
    double se = 0.0, tz = 0.0;
    for (int b = lane; b < NB; b += WAVE) {
        se += exp(static_cast<double>(z[b]) - static_cast<double>(mx));
        tz += static_cast<double>(hist[b]) * static_cast<double>(z[b]);
    }
    se = wave_sum_f64(se);
    tz = wave_sum_f64(tz) / ks;
    const double lse = static_cast<double>(mx) + log(se);
    const double invB = 1.0 / B;
    for (int b = lane; b < NB; b += WAVE) {
        const double p = exp(static_cast<double>(z[b]) - lse);
        const float g = static_cast<float>((p - static_cast<double>(hist[b]) / ks) * invB);
        dZ[static_cast<size_t>(i) * NB + b] = g;
        dZb[static_cast<size_t>(i) * NB + b] = f2bf(g);
    }
    if (lane == 0) row_loss[i] = lse - tz;
}

__global__ void k_sum_f64(const double* __restrict__ v, int cnt, double scale, double* __restrict__ out, int add)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int t = 0; t < cnt; ++t) s += v[t];
    out[0] = (add ? out[0] : 0.0) + s * scale;
}

// Adam on float32 master parameters with a BF16 shadow (bias-corrected moments).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m1, float* __restrict__ m2, int64_t cnt, float lr,
                                              float b1, float b2, float eps, float c1, float c2,
                                              uint16_t* __restrict__ pb)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const float gt = g[t];
    const float a = b1 * m1[t] + (1.f - b1) * gt;
    const float v = b2 * m2[t] + (1.f - b2) * gt * gt;
    m1[t] = a;
    m2[t] = v;
    const float w = p[t] - lr * (a / c1) / (sqrtf(v / c2) + eps);
    p[t] = w;
    if (pb) pb[t] = f2bf(w);
}

// Top-P buckets of each logits row (descending value, ties to the smaller
// bucket id); home = the first. One wavefront per row, P rounds of a
// wavefront arg-max over the row with earlier winners excluded.
template <int PMAX>
__global__ __launch_bounds__(256) void k_route_topp(const float* __restrict__ Z, int rows, int NB, int P,
                                                    int32_t* __restrict__ home, int32_t* __restrict__ probe)
{
    const int lane = lane_id();
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= rows) return;
    const float* z = Z + static_cast<size_t>(i) * NB;
    int chosen[PMAX];
#pragma unroll
    for (int u = 0; u < PMAX; ++u) chosen[u] = -1;
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        if (p < P) {
            float bv = -INFINITY;
            int bi = 0x7fffffff;
            for (int b = lane; b < NB; b += WAVE) {
                bool taken = false;
#pragma unroll
                for (int u = 0; u < PMAX; ++u) taken |= (chosen[u] == b);
                float v = z[b];
                if (v != v) v = -INFINITY;   // a NaN logit ranks last
                if (!taken && (v > bv || (v == bv && b < bi))) {
                    bv = v;
                    bi = b;
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const float ov = __shfl_xor(bv, o, WAVE);
                const int oi = __shfl_xor(bi, o, WAVE);
                if (ov > bv || (ov == bv && oi < bi)) {
                    bv = ov;
                    bi = oi;
                }
            }
            chosen[p] = bi;
            if (lane == 0) probe[static_cast<size_t>(i) * P + p] = bi;
        }
    }
    if (lane == 0 && home) home[i] = chosen[0];
}

// SplitMix64 (Steele, Lea and Flood; Vigna's constants) at counter c from seed,
// and a standard normal from two of its uniforms (Box-Muller).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double sm_normal(uint64_t seed, uint64_t c)
{
    const double u1 = (static_cast<double>(splitmix64(seed, 2 * c) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = static_cast<double>(splitmix64(seed, 2 * c + 1) >> 11) * (1.0 / 9007199254740992.0);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// p[t] = scale * N(0, 1) draw number (offset + t) of the seeded stream.
__global__ __launch_bounds__(256) void k_fill_normal(float* __restrict__ p, int64_t cnt, uint64_t seed,
                                                     uint64_t offset, float scale)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < cnt) p[t] = scale * static_cast<float>(sm_normal(seed, offset + static_cast<uint64_t>(t)));
}

// ------------------------------------------------------------------ launchers
hipError_t launch_gemm_nt(const uint16_t* A, int lda, const uint16_t* B, int ldb, int M, int N, int K,
                          const float* bias, int relu, const float* mask_ref, int ldm, float* Cf, int ldcf,
                          uint16_t* Cb, int ldcb, hipStream_t st)
{
    if (M % 32 || N % 32 || K % 16) return hipErrorInvalidValue;
    const int tiles = (M / 32) * (N / 32);
    hipLaunchKernelGGL(k_gemm_nt, dim3((tiles + 3) / 4), dim3(256), 0, st, A, lda, B, ldb, M, N, K, bias, relu,
                       mask_ref, ldm, Cf, ldcf, Cb, ldcb);
    return hipGetLastError();
}

hipError_t launch_transpose_bf16(const uint16_t* src, int rows, int cols, uint16_t* dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_transpose_bf16, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(256), 0, st, src, rows, cols,
                       dst);
    return hipGetLastError();
}

hipError_t launch_cast_rows_bf16(const float* src, int cols, const int32_t* idx, int valid, int rows, int ldd,
                                 uint16_t* dst, hipStream_t st)
{
    const int64_t tot = static_cast<int64_t>(rows) * ldd;
    hipLaunchKernelGGL(k_cast_rows_bf16, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0, st, src, cols,
                       idx, valid, rows, ldd, dst);
    return hipGetLastError();
}

hipError_t launch_cast_bf16(const float* src, int64_t cnt, uint16_t* dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_cast_bf16, dim3(static_cast<unsigned>((cnt + 255) / 256)), dim3(256), 0, st, src, cnt, dst);
    return hipGetLastError();
}

hipError_t launch_colsum(const float* src, int rows, int cols, float* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_colsum, dim3((cols + 255) / 256), dim3(256), 0, st, src, rows, cols, out);
    return hipGetLastError();
}

hipError_t launch_softmax_xent(const float* Z, int B, int NB, const int32_t* lab, int ks, float* dZ, uint16_t* dZb,
                               double* row_loss, double* loss_out, int add, hipStream_t st)
{
    hipLaunchKernelGGL(k_softmax_xent, dim3((B + 3) / 4), dim3(256), 4 * NB * sizeof(int), st, Z, B, NB, lab, ks, dZ,
                       dZb, row_loss);
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(64), 0, st, row_loss, B, 1.0 / B, loss_out, add);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m1, float* m2, int64_t cnt, float lr, float b1, float b2,
                       float eps, float c1, float c2, uint16_t* pb, hipStream_t st)
{
    hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>((cnt + 255) / 256)), dim3(256), 0, st, p, g, m1, m2, cnt, lr,
                       b1, b2, eps, c1, c2, pb);
    return hipGetLastError();
}

hipError_t launch_route_topp(const float* Z, int rows, int NB, int P, int32_t* home, int32_t* probe, hipStream_t st)
{
    if (P < 1 || P > 32 || P > NB) return hipErrorInvalidValue;
    if (P <= 8)
        hipLaunchKernelGGL(k_route_topp<8>, dim3((rows + 3) / 4), dim3(256), 0, st, Z, rows, NB, P, home, probe);
    else
        hipLaunchKernelGGL(k_route_topp<32>, dim3((rows + 3) / 4), dim3(256), 0, st, Z, rows, NB, P, home, probe);
    return hipGetLastError();
}

hipError_t launch_fill_normal(float* p, int64_t cnt, uint64_t seed, uint64_t offset, float scale, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_normal, dim3(static_cast<unsigned>((cnt + 255) / 256)), dim3(256), 0, st, p, cnt, seed,
                       offset, scale);
    return hipGetLastError();
}

}  // namespace kvb
