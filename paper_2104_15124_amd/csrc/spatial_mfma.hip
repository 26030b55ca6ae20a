// Spatial order and distance bounds for the matrix-core k-NN scan.
//
// Samples of a low intrinsic dimension (the manifold setting of Section 2)
// concentrate near a few principal directions. An orthonormal basis P of the
// top PR principal directions of the centred samples y is found by subspace
// iteration on their covariance; the projections z = P^T y order the samples
// along a Morton curve of their first PCODE coordinates, optionally refined by
// median splits inside groups of 64 tiles (k_kd_local). Query blocks and
// candidate tiles of consecutive curve positions are then compact in z, and
// because an orthonormal projection never lengthens a vector,
//   |y_i - y_j|^2 >= |z_i - z_j|^2 >= (gap between the boxes of their z)^2,
// a candidate tile whose box lies farther from a query block's box than all
// of the block's current thresholds holds no neighbour of any of its queries
// and is skipped (selection kernel, knn_mfma.hip). The bound is made rigorous
// for the rounding of P, of z and of the box gaps by the margins set there.
#include <rocprim/device/device_radix_sort.hpp>

#include "kvb_device.h"
#include "kvb_kernels.h"

namespace kvb {

constexpr int COV_ROWS = 32;      // rows staged per step
constexpr int COV_ENTRIES = 2048; // covariance entries per block (8 per thread)
constexpr int COV_SAMPLE = 32768; // rows sampled for the covariance

__device__ __forceinline__ void tri_index(int e, int m, int& a, int& b)
{
    // e-th entry of the upper triangle (a <= b), row by row
    a = 0;
    int rem = e;
    while (rem >= m - a) {
        rem -= m - a;
        ++a;
    }
    b = a + rem;
}

// Partial sums of y y^T over the sampled rows (every `stride`-th row), y = x - mu,
// for the entries chunk blockIdx.y of the upper triangle.
__global__ __launch_bounds__(256) void k_cov_partial(const float* __restrict__ X, int n, int m,
                                                     const double* __restrict__ mu, int stride, int rows_per_block,
                                                     double* __restrict__ part)
{
    __shared__ float sy[COV_ROWS][256 + 1];
    const int ntri = m * (m + 1) / 2;
    const int e0 = blockIdx.y * COV_ENTRIES;
    int ea[8], eb[8];
    double acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int e = e0 + threadIdx.x + 256 * u;
        acc[u] = 0.0;
        ea[u] = -1;
        eb[u] = 0;
        if (e < ntri) tri_index(e, m, ea[u], eb[u]);
    }
    const int s_begin = blockIdx.x * rows_per_block;
    const int nsample = (n + stride - 1) / stride;
    const int s_end = min(nsample, s_begin + rows_per_block);
    for (int s0 = s_begin; s0 < s_end; s0 += COV_ROWS) {
        __syncthreads();
        for (int t = threadIdx.x; t < COV_ROWS * m; t += 256) {
            const int r = t / m, c = t % m;
            const int srow = s0 + r;
            sy[r][c] = srow < s_end
                           ? static_cast<float>(static_cast<double>(X[static_cast<size_t>(srow) * stride * m + c]) - mu[c])
                           : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (ea[u] < 0) continue;
            double a = 0.0;
            for (int r = 0; r < COV_ROWS; ++r)
                a += static_cast<double>(sy[r][ea[u]]) * static_cast<double>(sy[r][eb[u]]);
            acc[u] += a;
        }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int e = e0 + threadIdx.x + 256 * u;
        if (e < ntri) part[static_cast<size_t>(blockIdx.x) * ntri + e] = acc[u];
    }
}

__global__ __launch_bounds__(256) void k_cov_reduce(const double* __restrict__ part, int nparts, int m,
                                                    double* __restrict__ C)
{
    const int ntri = m * (m + 1) / 2;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= ntri) return;
    double s = 0.0;
    for (int b = 0; b < nparts; ++b) s += part[static_cast<size_t>(b) * ntri + e];
    int a, b;
    tri_index(e, m, a, b);
    C[static_cast<size_t>(a) * m + b] = s;
    C[static_cast<size_t>(b) * m + a] = s;
}

// Subspace iteration for the top PR eigenvectors of the covariance C (one
// block): V <- orthonormalise(C V) from a fixed full-rank starting basis. The
// product uses the whole block; modified Gram-Schmidt runs in the first
// wavefront (float64, wavefront reductions in a fixed order). Columns of
// negligible norm (a covariance of rank below PR) are set to zero, so the
// nonzero columns of P stay orthonormal.
__global__ __launch_bounds__(256) void k_subspace(const double* __restrict__ C, int m, int iters,
                                                  float* __restrict__ P)
{
    __shared__ double V[256 * PR_DIMS];
    __shared__ double W[256 * PR_DIMS];
    for (int t = threadIdx.x; t < m * PR_DIMS; t += 256) {
        const int a = t / PR_DIMS, j = t % PR_DIMS;
        W[t] = (a % PR_DIMS == j ? 1.0 : 0.0) + 1e-3 * static_cast<double>((a * 7 + j * 13) % 17) / 17.0;
    }
    __syncthreads();
    double trace = 0.0;
    for (int a = 0; a < m; ++a) trace += C[static_cast<size_t>(a) * m + a];
    const double tiny = 1e-24 * (trace > 0.0 ? trace * trace : 1.0);
    for (int it = 0; it <= iters; ++it) {
        if (it > 0) {
            for (int t = threadIdx.x; t < m * PR_DIMS; t += 256) {
                const int a = t / PR_DIMS, j = t % PR_DIMS;
                double s = 0.0;
                for (int b = 0; b < m; ++b) s += C[static_cast<size_t>(a) * m + b] * V[b * PR_DIMS + j];
                W[t] = s;
            }
            __syncthreads();
        }
        if (threadIdx.x < WAVE) {
            const int lane = threadIdx.x;
            // Gram-Schmidt twice keeps the columns orthonormal to rounding level
            for (int pass = 0; pass < 2; ++pass)
            for (int j = 0; j < PR_DIMS; ++j) {
                for (int l = 0; l < j; ++l) {
                    double d = 0.0;
                    for (int a = lane; a < m; a += WAVE) d += W[a * PR_DIMS + j] * W[a * PR_DIMS + l];
                    d = wave_sum_f64(d);
                    for (int a = lane; a < m; a += WAVE) W[a * PR_DIMS + j] -= d * W[a * PR_DIMS + l];
                }
                double nn = 0.0;
                for (int a = lane; a < m; a += WAVE) nn += W[a * PR_DIMS + j] * W[a * PR_DIMS + j];
                nn = wave_sum_f64(nn);
                const double inv = (pass == 1 || nn > (it == 0 ? 1e-24 : tiny)) && nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
                for (int a = lane; a < m; a += WAVE) W[a * PR_DIMS + j] *= inv;
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < m * PR_DIMS; t += 256) V[t] = W[t];
        __syncthreads();
    }
    for (int t = threadIdx.x; t < m * PR_DIMS; t += 256) P[t] = static_cast<float>(V[t]);
    __syncthreads();
    // |P^T v|^2 <= lambda_max(P P^T) |v|^2 = lambda_max(P^T P) |v|^2, and the
    // largest eigenvalue of the Gram matrix G = P^T P of the float32 basis is at
    // most its largest absolute row sum: pscale = 1 / sqrt(that), rounded down
    if (threadIdx.x == 0) {
        double rmax = 0.0;
        for (int j = 0; j < PR_DIMS; ++j) {
            double row = 0.0;
            for (int l = 0; l < PR_DIMS; ++l) {
                double g = 0.0;
                for (int a = 0; a < m; ++a)
                    g += static_cast<double>(P[a * PR_DIMS + j]) * static_cast<double>(P[a * PR_DIMS + l]);
                row += fabs(g);
            }
            rmax = fmax(rmax, row);
        }
        P[m * PR_DIMS] = rmax > 0.0 ? static_cast<float>((1.0 - 1e-6) / sqrt(rmax * (1.0 + 1e-9))) : 1.f;
    }
}

// z_i = P^T y_i (float32, y = x - mu as in the operands), one thread per row;
// per-block minima / maxima of the first PCODE coordinates for the code range.
__global__ __launch_bounds__(256) void k_project(const float* __restrict__ X, int n, int m,
                                                 const double* __restrict__ mu, const float* __restrict__ P,
                                                 float* __restrict__ z, float* __restrict__ zpart)
{
    __shared__ float slo[PCODE_DIMS][256], shi[PCODE_DIMS][256];
    const int i = blockIdx.x * 256 + threadIdx.x;
    float zc[PR_DIMS];
#pragma unroll
    for (int c = 0; c < PR_DIMS; ++c) zc[c] = 0.f;
    if (i < n) {
        const float* x = X + static_cast<size_t>(i) * m;
        for (int k = 0; k < m; ++k) {
            const float y = static_cast<float>(static_cast<double>(x[k]) - mu[k]);
#pragma unroll
            for (int c = 0; c < PR_DIMS; ++c) zc[c] = fmaf(y, P[k * PR_DIMS + c], zc[c]);
        }
#pragma unroll
        for (int c = 0; c < PR_DIMS; ++c) z[static_cast<size_t>(i) * PR_DIMS + c] = zc[c];
    }
#pragma unroll
    for (int c = 0; c < PCODE_DIMS; ++c) {
        slo[c][threadIdx.x] = i < n ? zc[c] : __uint_as_float(0x7F800000u);
        shi[c][threadIdx.x] = i < n ? zc[c] : -__uint_as_float(0x7F800000u);
    }
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o)
#pragma unroll
            for (int c = 0; c < PCODE_DIMS; ++c) {
                slo[c][threadIdx.x] = fminf(slo[c][threadIdx.x], slo[c][threadIdx.x + o]);
                shi[c][threadIdx.x] = fmaxf(shi[c][threadIdx.x], shi[c][threadIdx.x + o]);
            }
        __syncthreads();
    }
    if (threadIdx.x < PCODE_DIMS) {
        zpart[static_cast<size_t>(blockIdx.x) * 2 * PCODE_DIMS + threadIdx.x] = slo[threadIdx.x][0];
        zpart[static_cast<size_t>(blockIdx.x) * 2 * PCODE_DIMS + PCODE_DIMS + threadIdx.x] = shi[threadIdx.x][0];
    }
}

// Range of the first PCODE projected coordinates from the block partials (one
// block): zr = [lo, hi] per coordinate.
__global__ __launch_bounds__(256) void k_zrange(const float* __restrict__ zpart, int nparts, float* __restrict__ zr)
{
    __shared__ float slo[PCODE_DIMS][256], shi[PCODE_DIMS][256];
    float lo[PCODE_DIMS], hi[PCODE_DIMS];
#pragma unroll
    for (int c = 0; c < PCODE_DIMS; ++c) {
        lo[c] = __uint_as_float(0x7F800000u);
        hi[c] = -__uint_as_float(0x7F800000u);
    }
    for (int b = threadIdx.x; b < nparts; b += 256)
#pragma unroll
        for (int c = 0; c < PCODE_DIMS; ++c) {
            lo[c] = fminf(lo[c], zpart[static_cast<size_t>(b) * 2 * PCODE_DIMS + c]);
            hi[c] = fmaxf(hi[c], zpart[static_cast<size_t>(b) * 2 * PCODE_DIMS + PCODE_DIMS + c]);
        }
#pragma unroll
    for (int c = 0; c < PCODE_DIMS; ++c) {
        slo[c][threadIdx.x] = lo[c];
        shi[c][threadIdx.x] = hi[c];
    }
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o)
#pragma unroll
            for (int c = 0; c < PCODE_DIMS; ++c) {
                slo[c][threadIdx.x] = fminf(slo[c][threadIdx.x], slo[c][threadIdx.x + o]);
                shi[c][threadIdx.x] = fmaxf(shi[c][threadIdx.x], shi[c][threadIdx.x + o]);
            }
        __syncthreads();
    }
    if (threadIdx.x < PCODE_DIMS) {
        zr[threadIdx.x] = slo[threadIdx.x][0];
        zr[PCODE_DIMS + threadIdx.x] = shi[threadIdx.x][0];
    }
}

// Morton code of the first PCODE projected coordinates, 8 bits each, over
// their range zr; value = sample index (stable sort: ties by index).
__global__ __launch_bounds__(256) void k_zcodes(const float* __restrict__ z, int n, const float* __restrict__ zr,
                                                uint32_t* __restrict__ code, int32_t* __restrict__ vals)
{
    __shared__ float s_lo[PCODE_DIMS], s_scale[PCODE_DIMS];
    if (threadIdx.x < PCODE_DIMS) {
        const int c = threadIdx.x;
        const float lo = zr[c], hi = zr[PCODE_DIMS + c];
        s_lo[c] = lo;
        s_scale[c] = hi > lo ? 256.f / (hi - lo) : 0.f;
    }
    __syncthreads();
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    uint32_t q[PCODE_DIMS];
#pragma unroll
    for (int c = 0; c < PCODE_DIMS; ++c) {
        const float t = (z[static_cast<size_t>(i) * PR_DIMS + c] - s_lo[c]) * s_scale[c];
        q[c] = min(static_cast<uint32_t>(fminf(fmaxf(t, 0.f), 255.f)), 255u);
    }
    uint32_t zc = 0;
    for (int b = 7; b >= 0; --b)
#pragma unroll
        for (int c = 0; c < PCODE_DIMS; ++c) zc = (zc << 1) | ((q[c] >> b) & 1u);
    code[i] = zc;
    vals[i] = i;
}

// pos[perm[p]] = p; cid[p] = perm[p] for p < n, -1 on the padding up to 32 tiles;
// zs[p] = z[perm[p]]. pos and cid may be null (orders that a later call
// replaces need only zs).
__global__ __launch_bounds__(256) void k_curve_maps(const int32_t* __restrict__ perm, int n, int npad,
                                                    const float* __restrict__ z, int32_t* __restrict__ pos,
                                                    int32_t* __restrict__ cid, float* __restrict__ zs)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npad) return;
    if (p < n) {
        const int i = perm[p];
        if (pos) pos[i] = p;
        if (cid) cid[p] = i;
#pragma unroll
        for (int c = 0; c < PR_DIMS; ++c) zs[static_cast<size_t>(p) * PR_DIMS + c] = z[static_cast<size_t>(i) * PR_DIMS + c];
    } else if (cid) {
        cid[p] = -1;
    }
}

// Boxes of groups of `span` consecutive rows (rows beyond `rows` ignored): over
// projected rows (boxes = 0) or over boxes (boxes = 1). Layout [group][2][PR].
__global__ __launch_bounds__(256) void k_zboxes(const float* __restrict__ src, int rows, int span, int groups,
                                                int boxes, float* __restrict__ out)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= groups * PR_DIMS) return;
    const int g = t / PR_DIMS, c = t % PR_DIMS;
    const int r0 = g * span, r1 = min(rows, r0 + span);
    float lo = __uint_as_float(0x7F800000u), hi = -__uint_as_float(0x7F800000u);
    for (int r = r0; r < r1; ++r) {
        if (boxes) {
            lo = fminf(lo, src[static_cast<size_t>(r) * 2 * PR_DIMS + c]);
            hi = fmaxf(hi, src[static_cast<size_t>(r) * 2 * PR_DIMS + PR_DIMS + c]);
        } else {
            const float v = src[static_cast<size_t>(r) * PR_DIMS + c];
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
        }
    }
    out[static_cast<size_t>(g) * 2 * PR_DIMS + c] = lo;
    out[static_cast<size_t>(g) * 2 * PR_DIMS + PR_DIMS + c] = hi;
}

// Median splits inside each group of KD_GROUP consecutive curve positions (256
// tiles): the group is halved at its middle position along the widest side of
// its box in z, each half likewise, down to 32-position tiles. A curve jump
// inside a group then falls between tiles instead of inside one, and every
// tile is the leaf of a balanced split of its group, so the tiles' boxes are
// compact (the first split of a group that straddles two distant regions
// separates them). Positions beyond n (last group) stay at the group's end.
// One workgroup per group; the halving is a bitonic sort in LDS of the keys
// (segment, coordinate on the segment's widest side, local index).
constexpr int KD_LOG = 13;
constexpr int KD_GROUP = 1 << KD_LOG;   // 8192 positions, 256 tiles
constexpr int KD_LEVELS = KD_LOG - 5;   // halvings down to 32
constexpr int KD_THREADS = 1024;
constexpr int KD_PER = KD_GROUP / KD_THREADS;

__global__ __launch_bounds__(KD_THREADS) void k_kd_local(int32_t* __restrict__ perm, const float* __restrict__ zs,
                                                         int n)
{
    __shared__ uint64_t s_key[KD_GROUP];
    __shared__ int32_t s_id[KD_GROUP];
    __shared__ uint32_t s_lo[1 << (KD_LEVELS - 1)][PR_DIMS], s_hi[1 << (KD_LEVELS - 1)][PR_DIMS];
    __shared__ int s_dim[1 << (KD_LEVELS - 1)];
    const int tid = threadIdx.x;
    const int g0 = blockIdx.x * KD_GROUP;
    const int m = min(KD_GROUP, n - g0);
    constexpr uint64_t PAD = ~0ull;
    for (int e = tid; e < KD_GROUP; e += KD_THREADS) {
        s_id[e] = e < m ? perm[g0 + e] : -1;
        s_key[e] = e < m ? static_cast<uint64_t>(e) : PAD;   // current order: local index in the low bits
    }
    __syncthreads();
    for (int l = 0; l < KD_LEVELS; ++l) {
        const int shift = KD_LOG - l;   // position >> shift = segment at this level
        const int nseg = 1 << l;
        for (int e = tid; e < nseg * PR_DIMS; e += KD_THREADS) {
            s_lo[e / PR_DIMS][e % PR_DIMS] = ~0u;
            s_hi[e / PR_DIMS][e % PR_DIMS] = 0u;
        }
        __syncthreads();
        // boxes: each thread owns KD_PER consecutive positions (one segment)
        {
            const int p0 = tid * KD_PER;
            const int seg = p0 >> shift;
            uint32_t lo[PR_DIMS], hi[PR_DIMS];
#pragma unroll
            for (int c = 0; c < PR_DIMS; ++c) {
                lo[c] = ~0u;
                hi[c] = 0u;
            }
            bool any = false;
            for (int j = 0; j < KD_PER; ++j) {
                const uint64_t k = s_key[p0 + j];
                if (k == PAD) continue;
                const int o = static_cast<int>(k & 0xFFFFu);
                any = true;
#pragma unroll
                for (int c = 0; c < PR_DIMS; ++c) {
                    const uint32_t v = float_order_bits(zs[static_cast<size_t>(g0 + o) * PR_DIMS + c]);
                    lo[c] = min(lo[c], v);
                    hi[c] = max(hi[c], v);
                }
            }
            if (any) {
#pragma unroll
                for (int c = 0; c < PR_DIMS; ++c) {
                    atomicMin(&s_lo[seg][c], lo[c]);
                    atomicMax(&s_hi[seg][c], hi[c]);
                }
            }
        }
        __syncthreads();
        if (tid < nseg) {
            int best = 0;
            float wbest = -1.f;
            for (int c = 0; c < PR_DIMS; ++c) {
                const float w = s_hi[tid][c] >= s_lo[tid][c]
                                    ? order_bits_float(s_hi[tid][c]) - order_bits_float(s_lo[tid][c]) : -1.f;
                if (w > wbest) {
                    wbest = w;
                    best = c;
                }
            }
            s_dim[tid] = best;
        }
        __syncthreads();
        // keys: segment (bits 48..), coordinate on its widest side (16..47), local index (0..15)
        for (int p = tid; p < KD_GROUP; p += KD_THREADS) {
            const uint64_t k = s_key[p];
            if (k == PAD) continue;
            const int o = static_cast<int>(k & 0xFFFFu);
            const int seg = p >> shift;
            const uint32_t v = float_order_bits(zs[static_cast<size_t>(g0 + o) * PR_DIMS + s_dim[seg]]);
            s_key[p] = (static_cast<uint64_t>(seg) << 48) | (static_cast<uint64_t>(v) << 16) | static_cast<uint64_t>(o);
        }
        __syncthreads();
        // ascending bitonic sort of each segment's keys (a segment's keys share
        // its high bits, so sorting the segments sorts the group; PAD keys sort
        // last): the networks of size seg_size, the last merge ascending in
        // every segment
        const int seg_size = 1 << shift;
        for (int k = 2; k <= seg_size; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int t = tid; t < KD_GROUP / 2; t += KD_THREADS) {
                    const int i = 2 * t - (t & (j - 1));
                    const int q = i + j;
                    const uint64_t a = s_key[i], b = s_key[q];
                    const bool up = k == seg_size || (i & k) == 0;
                    if ((a > b) == up) {
                        s_key[i] = b;
                        s_key[q] = a;
                    }
                }
                __syncthreads();
            }
        }
    }
    for (int p = tid; p < m; p += KD_THREADS) perm[g0 + p] = s_id[static_cast<int>(s_key[p] & 0xFFFFu)];
}

// The same halving for the levels above: groups of KG_GROUP consecutive curve
// positions (4096 tiles) are halved along the widest side of each segment's
// box down to segments of KD_GROUP positions, which k_kd_local then finishes.
// One workgroup of 16 wavefronts per group; wavefront w owns the positions
// [w KG_WPOS, (w + 1) KG_WPOS) of the group, lane l the ones congruent to l
// mod 64 (loads and stores of consecutive lanes are consecutive), and a
// wavefront's positions lie in one segment at every level. The segments'
// arrangements (local indices into the group's curve order, whose coordinates
// zs never move) live in two global buffers used in turn. A level: the
// segments' boxes (wavefront reductions, then LDS atomics on order bits), a
// histogram of each segment's widest coordinate over KG_BINS bins of its
// extent, the bin holding the segment's middle rank, then every element
// placed in the order (wavefront, position): the elements of the lower bins
// first, then those of the middle bin up to the middle position, the rest of
// that bin after it, the upper bins last; ranks come from ballots, so the
// result does not depend on the timing of the atomics.
constexpr int KG_LOG = 17;
constexpr int KG_GROUP = 1 << KG_LOG;
constexpr int KG_LEVELS = KG_LOG - KD_LOG;
constexpr int KG_THREADS = 1024;
constexpr int KG_WAVES = KG_THREADS / WAVE;
constexpr int KG_WPOS = KG_GROUP / KG_WAVES;    // 8192 positions per wavefront
constexpr int KG_BINS = 1024;
constexpr int KG_SEGS = 1 << (KG_LEVELS - 1);
constexpr int KG_U = 4;                         // positions per lane in flight

__device__ __forceinline__ int kg_bin(float v, float lo, float scale)
{
    const int b = static_cast<int>((v - lo) * scale);
    return b < 0 ? 0 : (b >= KG_BINS ? KG_BINS - 1 : b);
}

__global__ __launch_bounds__(KG_THREADS) void k_kd_group(const int32_t* __restrict__ perm,
                                                         const float* __restrict__ zs, int n,
                                                         int32_t* __restrict__ ord_a, int32_t* __restrict__ ord_b,
                                                         int32_t* __restrict__ perm_out)
{
    __shared__ uint32_t s_lo[KG_SEGS][PR_DIMS], s_hi[KG_SEGS][PR_DIMS];
    __shared__ int s_dim[KG_SEGS];
    __shared__ int s_hist[KG_SEGS][KG_BINS];
    __shared__ int s_bstar[KG_SEGS], s_below[KG_SEGS], s_take[KG_SEGS], s_cmed[KG_SEGS];
    __shared__ int s_wcnt[KG_WAVES][3];
    const int tid = threadIdx.x;
    const int lane = tid % WAVE, w = tid / WAVE;
    const int g0 = blockIdx.x * KG_GROUP;
    const int m = min(KG_GROUP, n - g0);
    const int wb = w * KG_WPOS;   // this wavefront's first position
    const uint64_t below_me = (1ull << lane) - 1ull;
    int32_t* cur = ord_a + g0;
    int32_t* nxt = ord_b + g0;
    for (int p = wb + lane; p < min(wb + KG_WPOS, m); p += WAVE) cur[p] = p;
    __syncthreads();
    for (int l = 0; l < KG_LEVELS; ++l) {
        const int shift = KG_LOG - l;   // position >> shift = segment
        const int S = 1 << shift, H = S >> 1;
        const int nseg = 1 << l;
        const int seg = wb >> shift;
        const int s0 = seg << shift;
        for (int e = tid; e < nseg * PR_DIMS; e += KG_THREADS) {
            s_lo[e / PR_DIMS][e % PR_DIMS] = ~0u;
            s_hi[e / PR_DIMS][e % PR_DIMS] = 0u;
        }
        for (int e = tid; e < nseg * KG_BINS; e += KG_THREADS) s_hist[e / KG_BINS][e % KG_BINS] = 0;
        __syncthreads();
        {
            uint32_t lo[PR_DIMS], hi[PR_DIMS];
#pragma unroll
            for (int c = 0; c < PR_DIMS; ++c) {
                lo[c] = ~0u;
                hi[c] = 0u;
            }
            for (int p = wb + lane; p < min(wb + KG_WPOS, m); p += WAVE) {
                const float4* z = reinterpret_cast<const float4*>(zs + static_cast<size_t>(g0 + cur[p]) * PR_DIMS);
                const float4 za = z[0], zb = z[1];
                const float zv[PR_DIMS] = {za.x, za.y, za.z, za.w, zb.x, zb.y, zb.z, zb.w};
#pragma unroll
                for (int c = 0; c < PR_DIMS; ++c) {
                    const uint32_t v = float_order_bits(zv[c]);
                    lo[c] = min(lo[c], v);
                    hi[c] = max(hi[c], v);
                }
            }
#pragma unroll
            for (int c = 0; c < PR_DIMS; ++c) {
#pragma unroll
                for (int o = 1; o < WAVE; o <<= 1) {
                    lo[c] = min(lo[c], xor_lane(lo[c], o));
                    hi[c] = max(hi[c], xor_lane(hi[c], o));
                }
            }
            if (lane == 0 && wb < m) {
#pragma unroll
                for (int c = 0; c < PR_DIMS; ++c) {
                    atomicMin(&s_lo[seg][c], lo[c]);
                    atomicMax(&s_hi[seg][c], hi[c]);
                }
            }
        }
        __syncthreads();
        if (tid < nseg) {
            int best = 0;
            float wbest = -1.f;
            for (int c = 0; c < PR_DIMS; ++c) {
                const float wd = s_hi[tid][c] >= s_lo[tid][c]
                                     ? order_bits_float(s_hi[tid][c]) - order_bits_float(s_lo[tid][c]) : -1.f;
                if (wd > wbest) {
                    wbest = wd;
                    best = c;
                }
            }
            s_dim[tid] = best;
        }
        __syncthreads();
        const int d = s_dim[seg];
        const float lo = order_bits_float(s_lo[seg][d]), hi = order_bits_float(s_hi[seg][d]);
        const float scale = hi > lo ? static_cast<float>(KG_BINS) / (hi - lo) : 0.f;
        const int pe = min(wb + KG_WPOS, m);
        // the coordinate on side d of the positions p, p + 64, ... (KG_U of them)
        auto side = [&](int p, int (&o)[KG_U], float (&v)[KG_U]) {
#pragma unroll
            for (int u = 0; u < KG_U; ++u) o[u] = p + u * WAVE < pe ? cur[p + u * WAVE] : 0;
#pragma unroll
            for (int u = 0; u < KG_U; ++u)
                v[u] = p + u * WAVE < pe ? zs[static_cast<size_t>(g0 + o[u]) * PR_DIMS + d] : 0.f;
        };
        for (int p = wb + lane; p < pe; p += KG_U * WAVE) {
            int o[KG_U];
            float v[KG_U];
            side(p, o, v);
#pragma unroll
            for (int u = 0; u < KG_U; ++u)
                if (p + u * WAVE < pe) atomicAdd(&s_hist[seg][kg_bin(v[u], lo, scale)], 1);
        }
        __syncthreads();
        if (tid < nseg) {
            // the first L = min(real, H) positions of the segment take the lower side
            const int real = max(0, min(S, m - (tid << shift)));
            const int L = min(real, H);
            int b = KG_BINS, below = real;   // no split: every element stays on the lower side
            if (real > H) {
                int acc = 0;
                for (b = 0; b < KG_BINS - 1; ++b) {
                    const int c = s_hist[tid][b];
                    if (acc + c >= L) break;
                    acc += c;
                }
                below = acc;
            }
            s_bstar[tid] = b;
            s_below[tid] = below;
            s_take[tid] = L - below;
            s_cmed[tid] = b < KG_BINS ? s_hist[tid][b] : 0;
        }
        __syncthreads();
        const int bs = s_bstar[seg];
        // this wavefront's count of each class (wave-uniform)
        int nl = 0, nm = 0, nr = 0;
        for (int p = wb + lane; p - lane < pe; p += KG_U * WAVE) {
            int o[KG_U];
            float v[KG_U];
            side(p, o, v);
#pragma unroll
            for (int u = 0; u < KG_U; ++u) {
                const bool in = p + u * WAVE < pe;
                const int b = kg_bin(v[u], lo, scale);
                nl += __popcll(__ballot(in && b < bs));
                nm += __popcll(__ballot(in && b == bs));
                nr += __popcll(__ballot(in && b > bs));
            }
        }
        if (lane == 0) {
            s_wcnt[w][0] = nl;
            s_wcnt[w][1] = nm;
            s_wcnt[w][2] = nr;
        }
        __syncthreads();
        // ranks: the wavefronts of the segment before this one, then this one's running counts
        int xl = 0, xm = 0, xr = 0;
        for (int q = s0 / KG_WPOS; q < w; ++q) {
            xl += s_wcnt[q][0];
            xm += s_wcnt[q][1];
            xr += s_wcnt[q][2];
        }
        const int below = s_below[seg], take = s_take[seg], cmed = s_cmed[seg];
        for (int p = wb + lane; p - lane < pe; p += KG_U * WAVE) {
            int o[KG_U];
            float v[KG_U];
            side(p, o, v);
#pragma unroll
            for (int u = 0; u < KG_U; ++u) {
                const bool in = p + u * WAVE < pe;
                const int b = kg_bin(v[u], lo, scale);
                const uint64_t ml = __ballot(in && b < bs), mm = __ballot(in && b == bs),
                               mr = __ballot(in && b > bs);
                if (in) {
                    int q;
                    if (b < bs) {
                        q = s0 + xl + __popcll(ml & below_me);
                    } else if (b == bs) {
                        const int r = xm + __popcll(mm & below_me);
                        q = r < take ? s0 + below + r : s0 + H + (r - take);
                    } else {
                        q = s0 + H + (cmed - take) + xr + __popcll(mr & below_me);
                    }
                    nxt[q] = o[u];
                }
                xl += __popcll(ml);
                xm += __popcll(mm);
                xr += __popcll(mr);
            }
        }
        __syncthreads();
        int32_t* t = cur;
        cur = nxt;
        nxt = t;
    }
    for (int p = wb + lane; p < min(wb + KG_WPOS, m); p += WAVE) perm_out[g0 + p] = perm[g0 + cur[p]];
}

// ------------------------------------------------------------------ launchers
int cov_partials() { return 32; }
int cov_chunks(int m) { return (m * (m + 1) / 2 + COV_ENTRIES - 1) / COV_ENTRIES; }
int project_blocks(int n) { return (n + 255) / 256; }

hipError_t launch_principal_basis(const float* X, int n, int m, const double* mu, double* part, double* C, float* P,
                                  hipStream_t st)
{
    if (m < 1 || m > 256) return hipErrorInvalidValue;
    const int stride = n > COV_SAMPLE ? n / COV_SAMPLE : 1;
    const int nsample = (n + stride - 1) / stride;
    const int nb = cov_partials();
    const int rpb = (nsample + nb - 1) / nb;
    hipLaunchKernelGGL(k_cov_partial, dim3(nb, cov_chunks(m)), dim3(256), 0, st, X, n, m, mu, stride, rpb, part);
    const int ntri = m * (m + 1) / 2;
    hipLaunchKernelGGL(k_cov_reduce, dim3((ntri + 255) / 256), dim3(256), 0, st, part, nb, m, C);
    hipLaunchKernelGGL(k_subspace, dim3(1), dim3(256), 0, st, C, m, 20, P);
    return hipGetLastError();
}

hipError_t launch_curve_order(const float* X, int n, int m, const double* mu, const float* P, float* z, float* zpart,
                              uint32_t* code, uint32_t* scode, int32_t* vals, int32_t* perm, void* sort_tmp,
                              size_t sort_bytes, int32_t* pos, int32_t* cid, float* zs, float* tbox, float* sbox,
                              float* tree, bool median_splits, hipStream_t st)
{
    const int nb = project_blocks(n);
    hipLaunchKernelGGL(k_project, dim3(nb), dim3(256), 0, st, X, n, m, mu, P, z, zpart);
    float* zr = zpart + static_cast<size_t>(nb) * 2 * PCODE_DIMS;   // one more partial's room
    hipLaunchKernelGGL(k_zrange, dim3(1), dim3(256), 0, st, zpart, nb, zr);
    hipLaunchKernelGGL(k_zcodes, dim3(nb), dim3(256), 0, st, z, n, zr, code, vals);
    size_t tb = sort_bytes;
    hipError_t e = rocprim::radix_sort_pairs(sort_tmp, tb, code, scode, vals, perm, static_cast<size_t>(n), 0u,
                                             8u * PCODE_DIMS, st);
    if (e != hipSuccess) return e;
    const int ntiles = (n + 31) / 32, npad = ntiles * 32;
    // with median splits the final order's maps are written at the end; the
    // splits read only zs
    hipLaunchKernelGGL(k_curve_maps, dim3((npad + 255) / 256), dim3(256), 0, st, perm, n, npad, z,
                       median_splits ? nullptr : pos, median_splits ? nullptr : cid, zs);
    if (median_splits) {
        // the median splits inside each 4096-tile group of the curve down to
        // 256-tile segments (they read the curve's coordinates; code and scode
        // hold the arrangements, vals the new order), then inside each of those
        // down to single tiles, then the maps of the final order
        int32_t* split_order = vals;
        hipLaunchKernelGGL(k_kd_group, dim3((n + KG_GROUP - 1) / KG_GROUP), dim3(KG_THREADS), 0, st, perm, zs, n,
                           reinterpret_cast<int32_t*>(code), reinterpret_cast<int32_t*>(scode), split_order);
        hipLaunchKernelGGL(k_curve_maps, dim3((npad + 255) / 256), dim3(256), 0, st, split_order, n, npad, z, nullptr,
                           nullptr, zs);
        hipLaunchKernelGGL(k_kd_local, dim3((n + KD_GROUP - 1) / KD_GROUP), dim3(KD_THREADS), 0, st, split_order, zs,
                           n);
        hipLaunchKernelGGL(k_curve_maps, dim3((npad + 255) / 256), dim3(256), 0, st, split_order, n, npad, z, pos, cid,
                           zs);
    }
    hipLaunchKernelGGL(k_zboxes, dim3((ntiles * PR_DIMS + 255) / 256), dim3(256), 0, st, zs, n, 32, ntiles, 0, tbox);
    const int nsb = (ntiles + SB_TILES_MFMA - 1) / SB_TILES_MFMA;
    hipLaunchKernelGGL(k_zboxes, dim3((nsb * PR_DIMS + 255) / 256), dim3(256), 0, st, tbox, ntiles, SB_TILES_MFMA, nsb,
                       1, sbox);
    // the box tree: each level's boxes over groups of 64 boxes of the level below
    const TreeLayout t = tree_layout(ntiles);
    for (int l = 1; l <= t.top; ++l) {
        const float* src = l == 1 ? tbox : tree + static_cast<size_t>(t.off[l - 1]) * 2 * PR_DIMS;
        hipLaunchKernelGGL(k_zboxes, dim3((t.cnt[l] * PR_DIMS + 255) / 256), dim3(256), 0, st, src, t.cnt[l - 1],
                           TREE_FAN, t.cnt[l], 1, tree + static_cast<size_t>(t.off[l]) * 2 * PR_DIMS);
    }
    return hipGetLastError();
}

TreeLayout tree_layout(int ntiles)
{
    TreeLayout t = {};
    t.cnt[0] = ntiles;
    int l = 0, nodes = 0;
    while (t.cnt[l] > TREE_FAN && l + 1 < TREE_LEVELS) {
        ++l;
        t.cnt[l] = (t.cnt[l - 1] + TREE_FAN - 1) / TREE_FAN;
        t.off[l] = nodes;
        nodes += t.cnt[l];
    }
    t.top = l;
    t.nodes = nodes;
    return t;
}

size_t curve_sort_bytes(int n)
{
    size_t b = 0;
    (void)rocprim::radix_sort_pairs(nullptr, b, static_cast<const uint32_t*>(nullptr), static_cast<uint32_t*>(nullptr),
                                    static_cast<const int32_t*>(nullptr), static_cast<int32_t*>(nullptr),
                                    static_cast<size_t>(n), 0u, 8u * PCODE_DIMS, nullptr);
    return b;
}

}  // namespace kvb
