// Matrix-core distance tiles for the k-NN selection (gfx950 MFMA).
//
// For m >= 9 the squared distances are a dense contraction: with samples
// centred on their column mean (y = x - mu), the selection score
//   s_ij = |y_j|^2 - 2 y_i . y_j = |y_i - y_j|^2 - |y_i|^2
// ranks the candidates j of row i exactly like the squared distance. It is one
// GEMM-shaped product of a query operand and a candidate operand, both laid
// out by the prep kernel with the norm folded into the contraction:
//   query     a_i = [-2 t_1(y_i), ..., -2 t_P(y_i), 1, 1, 1, 0...]
//   candidate b_j = [  u_1(y_j), ...,    u_P(y_j), n1, n2, n3, 0...]
// so that a_i . b_j = s_ij up to the rounding of the operands. In BF16 mode the
// coordinates are split into two or three BF16 terms (hi + lo, or
// hi + mid + lo) and the product pairs listed below; the norm is split into
// three BF16 terms. In FP32 mode the operands are y itself.
//
// Tiles are 32 queries x 32 candidates (v_mfma_f32_32x32x16_bf16 or
// v_mfma_f32_32x32x2_f32, FP32 accumulation). A workgroup of four or eight
// wavefronts stages 32 candidates at a time in LDS (two stages; the next tile
// is prefetched into registers while the current one is consumed); every
// wavefront keeps its query fragments in registers and loads a stage's
// candidate fragments in one batch before the MFMA chain. Scores at or below a query's threshold are appended
// to that query's LDS buffer; a buffer that may not absorb another tile is merged into
// the query's sorted list (in global scratch) by the wavefront bitonic merge,
// which lowers the threshold.
//
// Certificate bound. After the scan, every candidate that is not on a row's
// list has a score >= s_last (the list's last score). The epilogue turns
// s_last into a lower bound on the true squared distance of any such
// candidate, from the operand and accumulation error model:
//   |x_i - x_j|^2 >= (sqrt(max(0, s_last + |y_i|^2 - E_i)) - c (|y_i| + R))^2,
//   E_i = g (R + 1.05 |y_i|)^2 + h R^2 + x |y_i| R,
// with R = max_j |y_j|, g the accumulation bound (K + 4) 2^-24, h the norm
// representation bound, x the cross-term bound of the chosen split and c the
// centring rounding bound. The refine step compares it with the largest kept
// exact distance.
#include "knn_mfma_common.h"

namespace kvb {

// ------------------------------------------------------------------ prep
// Column sums (float64) over blocks of rows, then the fixed-order mean. For
// m <= 256 the block's threads form T = 256 / m row lanes of m columns: thread
// (j, c) sums column c over rows r0 + j, r0 + j + T, ... (consecutive threads
// read consecutive columns of a row), and the T partial sums of a column are
// added in the order j = 0, 1, ... . Wider rows: one thread per column.
__global__ __launch_bounds__(256) void k_colsum_partial(const float* __restrict__ X, int n, int m, int rows_per_block,
                                                        double* __restrict__ part)
{
    __shared__ double s_part[256];
    const int r0 = blockIdx.x * rows_per_block;
    const int r1 = min(n, r0 + rows_per_block);
    if (m <= 256) {
        const int T = 256 / m;
        const int j = threadIdx.x / m, c = threadIdx.x % m;
        double s = 0.0;
        if (j < T)
            for (int r = r0 + j; r < r1; r += T) s += static_cast<double>(X[static_cast<size_t>(r) * m + c]);
        s_part[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x < m) {
            double t = 0.0;
            for (int q = 0; q < T; ++q) t += s_part[q * m + threadIdx.x];
            part[static_cast<size_t>(blockIdx.x) * m + threadIdx.x] = t;
        }
        return;
    }
    for (int c = threadIdx.x; c < m; c += blockDim.x) {
        double s = 0.0;
        for (int r = r0; r < r1; ++r) s += static_cast<double>(X[static_cast<size_t>(r) * m + c]);
        part[static_cast<size_t>(blockIdx.x) * m + c] = s;
    }
}

// The block partials of each column added in a fixed order: for m <= 256,
// thread (j, c) sums the partials j, j + T, ... of column c, and the T sums
// are added in the order j = 0, 1, ... .
__global__ __launch_bounds__(256) void k_colsum_finish(const double* __restrict__ part, int nb, int m, int n,
                                                       double* __restrict__ mu)
{
    __shared__ double s_part[256];
    if (m <= 256) {
        const int T = 256 / m;
        const int j = threadIdx.x / m, c = threadIdx.x % m;
        double s = 0.0;
        if (j < T)
            for (int b = j; b < nb; b += T) s += part[static_cast<size_t>(b) * m + c];
        s_part[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x < m) {
            double t = 0.0;
            for (int q = 0; q < T; ++q) t += s_part[q * m + threadIdx.x];
            mu[threadIdx.x] = t / static_cast<double>(n);
        }
        return;
    }
    for (int c = threadIdx.x; c < m; c += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[static_cast<size_t>(b) * m + c];
        mu[c] = s / static_cast<double>(n);
    }
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    const uint32_t u = __float_as_uint(f);
    const uint32_t r = ((u >> 16) & 1u) + 0x7FFFu;
    return static_cast<uint16_t>((u + r) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

// Position of candidate-operand element (row i, column c) in the tile-major
// fragment order used by the selection kernel: 32-row tiles, each laid out as
// [k-step][lane half][row][fragment element], i.e. exactly the LDS image that
// the MFMA B-operand reads, so a tile streams in with contiguous copies.
__device__ __forceinline__ size_t bpos(int i, int c, int kpad, int kstep, int vec)
{
    const int s = c / kstep, w = c % kstep, h = w / vec, v = w % vec;
    return static_cast<size_t>(i / 32) * 32 * kpad + ((s * 2 + h) * 32 + (i % 32)) * vec + v;
}

// One wavefront per row: y = x - mu (float32), the operand terms, |y|^2
// (float64, kept as float32 for the certificate) and the running max |y|.
// split: 0 = float32 operands, 1 = one BF16 term, 3 = hi/lo pairs, 6 = hi/mid/lo pairs.
// Rows n..npad-1 pad the last 32-row tile with zeros. With brow non-null the
// candidate operand row of sample i is written at row brow[i] instead of i
// (the bucket order of the learned partitioner; npad == n).
// sum over aligned groups of lpr lanes (16, 32 or 64), every lane of a group
// receiving it; the xor stages below lpr are those of wave_sum_f64, so where
// the lanes of a group beyond the row hold 0 the row's sum is the same
__device__ __forceinline__ double group_sum_f64(double v, int lpr)
{
    if (lpr > 32) v += shfl_xor_f64(v, 32);
    if (lpr > 16) v += shfl_xor_f64(v, 16);
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) v += shfl_xor_f64(v, o);
    return v;
}

static int prep_blocks(int npad) { return std::max(1, std::min(4096, (npad + 3) / 4)); }

__global__ __launch_bounds__(256) void k_prep_rows(const float* __restrict__ X, int n, int npad, int m,
                                                   const double* __restrict__ mu, int split, int kpad,
                                                   void* __restrict__ Aq, void* __restrict__ Bc,
                                                   float* __restrict__ ynorm2, unsigned* __restrict__ rmax_bits,
                                                   const int* __restrict__ brow, const int* __restrict__ arow)
{
    // rows are taken in a grid-stride loop, 64 / lpr rows per wavefront (lpr
    // lanes per row, the power of two >= m from 16 on); the largest norm is
    // folded per block and published with one atomic (an atomic per row
    // serialises millions of updates of one address)
    const int lane = lane_id();
    const int lpr = m <= 16 ? 16 : m <= 32 ? 32 : WAVE;
    const int rpw = WAVE / lpr, gl = lane % lpr;
    float wmax = 0.f;
    for (int i0 = (blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * rpw; i0 < npad;
         i0 += gridDim.x * 4 * rpw) {
        const int i = i0 + lane / lpr;
        const bool live = i < npad;   // rows past npad (last wavefront): nothing written
        const bool real = i < n;
        const int ib = (brow && real) ? brow[i] : i;   // candidate operand row
        const int ia = (arow && real) ? arow[i] : i;   // query operand row
        const float* x = X + static_cast<size_t>(real ? i : 0) * m;
        double nrm = 0.0;
        if (split == 0) {
            constexpr int KS = 2, VE = 1;
            float* A = static_cast<float*>(Aq) + static_cast<size_t>(ia) * kpad;
            float* B = static_cast<float*>(Bc);
            for (int c = gl; c < m; c += lpr) {
                const float y = real ? static_cast<float>(static_cast<double>(x[c]) - mu[c]) : 0.0f;
                nrm += static_cast<double>(y) * static_cast<double>(y);
                if (real) A[c] = -2.0f * y;
                if (live) B[bpos(ib, c, kpad, KS, VE)] = y;
            }
            nrm = group_sum_f64(nrm, lpr);
            for (int c = m + gl; c < kpad; c += lpr) {
                if (real) A[c] = (c == m) ? 1.0f : 0.0f;
                if (live) B[bpos(ib, c, kpad, KS, VE)] = (c == m) ? static_cast<float>(nrm) : 0.0f;
            }
        } else {
            constexpr int KS = 16, VE = 8;
            uint16_t* A = static_cast<uint16_t*>(Aq) + static_cast<size_t>(ia) * kpad;
            uint16_t* B = static_cast<uint16_t*>(Bc);
            for (int c = gl; c < m; c += lpr) {
                const float y = real ? static_cast<float>(static_cast<double>(x[c]) - mu[c]) : 0.0f;
                nrm += static_cast<double>(y) * static_cast<double>(y);
                const uint16_t hi = f32_to_bf16_rne(y);
                const float r1 = y - bf16_to_f32(hi);
                const uint16_t mid = f32_to_bf16_rne(r1);
                const float r2 = r1 - bf16_to_f32(mid);
                const uint16_t lo = f32_to_bf16_rne(r2);
                // -2 t is exact in BF16 (a power-of-two scaling)
                const uint16_t hi2 = f32_to_bf16_rne(-2.0f * bf16_to_f32(hi));
                const uint16_t mid2 = f32_to_bf16_rne(-2.0f * bf16_to_f32(mid));
                const uint16_t lo2 = f32_to_bf16_rne(-2.0f * bf16_to_f32(lo));
                uint16_t a[6], b[6];
                int P = 1;
                if (split == 1) {
                    a[0] = hi2; b[0] = hi;
                } else if (split == 3) {                     // (hi,hi) (hi,lo) (lo,hi), the second term as lo
                    a[0] = hi2; b[0] = hi;
                    a[1] = hi2; b[1] = mid;
                    a[2] = mid2; b[2] = hi;
                    P = 3;
                } else {                                     // (hi,hi) (hi,mid) (mid,hi) (hi,lo) (lo,hi) (mid,mid)
                    a[0] = hi2; b[0] = hi;
                    a[1] = hi2; b[1] = mid;
                    a[2] = mid2; b[2] = hi;
                    a[3] = hi2; b[3] = lo;
                    a[4] = lo2; b[4] = hi;
                    a[5] = mid2; b[5] = mid;
                    P = 6;
                }
                for (int t = 0; t < P; ++t) {
                    if (real) A[t * m + c] = a[t];
                    if (live) B[bpos(ib, t * m + c, kpad, KS, VE)] = b[t];
                }
            }
            nrm = group_sum_f64(nrm, lpr);
            const int P = split;
            const uint16_t n1 = f32_to_bf16_rne(static_cast<float>(nrm));
            const double r1 = nrm - static_cast<double>(bf16_to_f32(n1));
            const uint16_t n2 = f32_to_bf16_rne(static_cast<float>(r1));
            const double r2 = r1 - static_cast<double>(bf16_to_f32(n2));
            const uint16_t n3 = f32_to_bf16_rne(static_cast<float>(r2));
            const uint16_t one = f32_to_bf16_rne(1.0f);
            for (int c = P * m + gl; c < kpad; c += lpr) {
                const int t = c - P * m;
                if (real) A[c] = t < 3 ? one : static_cast<uint16_t>(0);
                if (live)
                    B[bpos(ib, c, kpad, KS, VE)] = t == 0   ? n1
                                                   : t == 1 ? n2
                                                   : t == 2 ? n3
                                                            : static_cast<uint16_t>(0);
            }
        }
        if (real && gl == 0) {
            ynorm2[ia] = static_cast<float>(nrm);   // by query operand row
            wmax = fmaxf(wmax, static_cast<float>(sqrt(nrm) * (1.0 + 1e-6)));
        }
    }
    __shared__ float s_wmax[4];
    wmax = wave_max_f32(wmax);
    if (lane == 0) s_wmax[threadIdx.x >> 6] = wmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float bm = fmaxf(fmaxf(s_wmax[0], s_wmax[1]), fmaxf(s_wmax[2], s_wmax[3]));
        if (bm > 0.f) atomicMax(rmax_bits, __float_as_uint(bm));
    }
}

// k_prep_rows for FP32 operands of rows of at most PREP_THREAD_M coordinates,
// by operand row (the BF16 split terms stay with the wavefront per row, whose
// 2-byte query operand writes coalesce):
// thread r prepares operand row r from input row r (r >= n: a padding row of
// zeros), with the same values as
// k_prep_rows (|y|^2 summed over the row in column order). Consecutive
// threads then write consecutive query operand rows and, in the candidate
// operand, whose k-step blocks hold 32 consecutive rows, consecutive
// addresses.
constexpr int PREP_THREAD_M = 64;

__global__ __launch_bounds__(256) void k_prep_rows_thread(const float* __restrict__ X, int n, int npad, int m,
                                                          const double* __restrict__ mu, int split, int kpad,
                                                          void* __restrict__ Aq, void* __restrict__ Bc,
                                                          float* __restrict__ ynorm2, unsigned* __restrict__ rmax_bits)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    float wmax = 0.f;
    if (r < npad) {
        const int i = r < n ? r : -1;
        const bool real = i >= 0;
        const int ib = r, ia = r;
        const float* x = X + static_cast<size_t>(real ? i : 0) * m;
        double nrm = 0.0;
        {
            constexpr int KS = 2, VE = 1;
            float* A = static_cast<float*>(Aq) + static_cast<size_t>(ia) * kpad;
            float* B = static_cast<float*>(Bc);
            const bool vec = (m % 4 == 0) && (kpad % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0) &&
                             ((reinterpret_cast<uintptr_t>(Aq) & 15) == 0);
            if (vec) {
                for (int c = 0; c < m; c += 4) {
                    const float4 xv = real ? *reinterpret_cast<const float4*>(x + c) : make_float4(0.f, 0.f, 0.f, 0.f);
                    const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
                    float ys[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        ys[u] = real ? static_cast<float>(static_cast<double>(xs[u]) - mu[c + u]) : 0.0f;
                        nrm += static_cast<double>(ys[u]) * static_cast<double>(ys[u]);
                        B[bpos(ib, c + u, kpad, KS, VE)] = ys[u];
                    }
                    if (real)
                        *reinterpret_cast<float4*>(A + c) = make_float4(-2.0f * ys[0], -2.0f * ys[1], -2.0f * ys[2],
                                                                        -2.0f * ys[3]);
                }
                for (int c = m; c < kpad; c += 4) {
                    float av[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        av[u] = (c + u == m) ? 1.0f : 0.0f;
                        B[bpos(ib, c + u, kpad, KS, VE)] = (c + u == m) ? static_cast<float>(nrm) : 0.0f;
                    }
                    if (real) *reinterpret_cast<float4*>(A + c) = make_float4(av[0], av[1], av[2], av[3]);
                }
            } else {
                for (int c = 0; c < m; ++c) {
                    const float y = real ? static_cast<float>(static_cast<double>(x[c]) - mu[c]) : 0.0f;
                    nrm += static_cast<double>(y) * static_cast<double>(y);
                    if (real) A[c] = -2.0f * y;
                    B[bpos(ib, c, kpad, KS, VE)] = y;
                }
                for (int c = m; c < kpad; ++c) {
                    if (real) A[c] = (c == m) ? 1.0f : 0.0f;
                    B[bpos(ib, c, kpad, KS, VE)] = (c == m) ? static_cast<float>(nrm) : 0.0f;
                }
            }
        }
        if (real) {
            ynorm2[ia] = static_cast<float>(nrm);
            wmax = static_cast<float>(sqrt(nrm) * (1.0 + 1e-6));
        }
    }
    // the block's largest norm published with one atomic (one per wavefront
    // made 125k updates of one address at n = 8M)
    __shared__ float s_wmax[4];
    wmax = wave_max_f32(wmax);
    if (lane_id() == 0) s_wmax[threadIdx.x >> 6] = wmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float bm = fmaxf(fmaxf(s_wmax[0], s_wmax[1]), fmaxf(s_wmax[2], s_wmax[3]));
        if (bm > 0.f) atomicMax(rmax_bits, __float_as_uint(bm));
    }
}

// ------------------------------------------------------------------ select
// Curve-order scan: the own tile, then alternately outward to the right and
// to the left, skipping what lies beyond the workgroup's current threshold.
// Picking the next tile is a ballot over a window of 64 tiles whose bounds to
// the workgroup's box (bw) and to this wavefront's box (ww) one load gave
// every lane. Before a new tile window is loaded, a window of 64 superblock
// bounds (SB_TILES_MFMA tiles each, also one load) moves the scan past the
// superblocks beyond reach, so sparse scans do not load tile windows of
// tiles that are all far away. The scan state is the same in every wavefront
// of the workgroup.
struct CurveScan {
    int cur_r, cur_l;     // next candidate tile on each side
    int rt0, lt0;         // tile windows: lane l is tile rt0 + l / lt0 - l
    int rsb0, lsb0;       // superblock windows: lane l is superblock rsb0 + l / lsb0 - l
    bool go_right;
    float rbw, rww, lbw, lww;   // tile bounds
    float rsbw, lsbw;           // superblock bounds (workgroup box)

    __device__ __forceinline__ void init(int own_t)
    {
        cur_r = own_t;
        cur_l = own_t - 1;
        rt0 = lt0 = rsb0 = lsb0 = -4 * WAVE;
        go_right = true;
        rbw = rww = lbw = lww = rsbw = lsbw = 0.f;
    }

    __device__ __forceinline__ static void load_box(const float* __restrict__ src_f, float (&b)[2 * PR_DIMS])
    {
        const float4* src = reinterpret_cast<const float4*>(src_f);
#pragma unroll
        for (int v = 0; v < PR_DIMS / 2; ++v) {
            const float4 q = src[v];
            b[4 * v] = q.x;
            b[4 * v + 1] = q.y;
            b[4 * v + 2] = q.z;
            b[4 * v + 3] = q.w;
        }
    }

    // bounds of tile t (NaN: no such tile, never within reach; -inf: own tile)
    __device__ __forceinline__ static void tile_window(int t, int own_t, int tend, const CurveArgs& crv,
                                                       const float* qlo, const float* qhi, const float* wlo,
                                                       const float* whi, const BoxBound& bb, float& bw, float& ww)
    {
        bw = __uint_as_float(0x7FC00000u);
        ww = bw;
        if (t < 0 || t >= tend) return;
        if (t == own_t) {
            bw = -__uint_as_float(0x7F800000u);
            ww = bw;
            return;
        }
        float b[2 * PR_DIMS];
        load_box(crv.tbox + static_cast<size_t>(t) * 2 * PR_DIMS, b);
        bw = box_bound(b, qlo, qhi, bb);
        ww = box_bound(b, wlo, whi, bb);
    }

    // bound of superblock sb (NaN: none; -inf: the own tile's)
    __device__ __forceinline__ static float sb_window(int sb, int own_sb, int nsb, const CurveArgs& crv,
                                                      const float* qlo, const float* qhi, const BoxBound& bb)
    {
        if (sb < 0 || sb >= nsb) return __uint_as_float(0x7FC00000u);
        if (sb == own_sb) return -__uint_as_float(0x7F800000u);
        float b[2 * PR_DIMS];
        load_box(crv.sbox + static_cast<size_t>(sb) * 2 * PR_DIMS, b);
        return box_bound(b, qlo, qhi, bb);
    }

    // next tile whose workgroup bound is <= thr, or -1; wb: its wavefront bound
    __device__ __forceinline__ int next(float thr, int own_t, int tend, const CurveArgs& crv, const float* qlo,
                                        const float* qhi, const float* wlo, const float* whi, const BoxBound& bb,
                                        float& wb)
    {
        constexpr int ST = SB_TILES_MFMA;
        const int own_sb = own_t / ST, nsb = (tend + ST - 1) / ST;
        const int lane = lane_id();
        while (cur_r < tend || cur_l >= 0) {
            if ((go_right && cur_r < tend) || cur_l < 0) {
                go_right = false;
                while (cur_r < tend) {
                    if (cur_r >= rt0 + WAVE) {
                        // first superblock within reach at or after cur_r's
                        const int sb = cur_r / ST;
                        if (sb >= rsb0 + WAVE || sb < rsb0) {
                            rsb0 = sb;
                            rsbw = sb_window(rsb0 + lane, own_sb, nsb, crv, qlo, qhi, bb);
                        }
                        const uint64_t ms = __ballot(rsbw <= thr) & (~0ull << (sb - rsb0));
                        if (!ms) {
                            cur_r = (rsb0 + WAVE) * ST;
                            continue;
                        }
                        const int nsbr = rsb0 + __builtin_ctzll(ms);
                        if (nsbr != sb) cur_r = nsbr * ST;
                        if (cur_r >= tend) break;
                        rt0 = cur_r;
                        tile_window(rt0 + lane, own_t, tend, crv, qlo, qhi, wlo, whi, bb, rbw, rww);
                    }
                    const uint64_t m = __ballot(rbw <= thr) & (~0ull << (cur_r - rt0));
                    if (m) {
                        const int l = __builtin_ctzll(m);
                        wb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rww), l));
                        cur_r = rt0 + l + 1;
                        return rt0 + l;
                    }
                    cur_r = rt0 + WAVE;
                }
            } else {
                go_right = true;
                while (cur_l >= 0) {
                    if (cur_l <= lt0 - WAVE || cur_l > lt0) {
                        // first superblock within reach at or before cur_l's
                        const int sb = cur_l / ST;
                        if (sb > lsb0 || sb <= lsb0 - WAVE) {
                            lsb0 = sb;
                            lsbw = sb_window(lsb0 - lane, own_sb, nsb, crv, qlo, qhi, bb);
                        }
                        const uint64_t ms = __ballot(lsbw <= thr) & (~0ull << (lsb0 - sb));
                        if (!ms) {
                            cur_l = (lsb0 - WAVE + 1) * ST - 1;
                            continue;
                        }
                        const int nsbl = lsb0 - __builtin_ctzll(ms);
                        if (nsbl != sb) cur_l = nsbl * ST + ST - 1;
                        lt0 = cur_l;
                        tile_window(lt0 - lane, own_t, tend, crv, qlo, qhi, wlo, whi, bb, lbw, lww);
                    }
                    const uint64_t m = __ballot(lbw <= thr) & (~0ull << (lt0 - cur_l));
                    if (m) {
                        const int l = __builtin_ctzll(m);
                        wb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lww), l));
                        cur_l = lt0 - l - 1;
                        return lt0 - l;
                    }
                    cur_l = lt0 - WAVE;
                }
            }
        }
        return -1;
    }
};

// WV wavefronts per workgroup share every candidate stage; each wavefront owns
// 32 queries. The first CAP / 32 tiles of a scan that starts from empty
// lists are written into the lists directly and sorted once; afterwards keys
// at or below a query's threshold collect in its LDS buffer of BUF keys, which
// is merged into the list whenever the next tile's keys would not fit.
//
// MODE 0: queries and candidates in sample order, every tile scanned.
//
// MODE 1 (learned): bucketed search of the learned partitioner. Workgroup w
// takes work item (bucket b, first query entry t0): its queries are entries
// t0 .. min(t0 + 32 WV, qptr[b + 1]) - 1 of qids, its candidates the tiles
// tptr[b] .. tptr[b + 1] - 1 of the bucket-ordered candidate operand, whose
// rows map to sample ids through cid (-1 for padding). Lists of queries are
// created on the first probe pass and merged into on later ones (the list's
// kp-th score is the starting threshold); no certificate is computed.
//
// MODE 2 (curve order): operands are laid out in the Morton order of the
// samples' principal projections (spatial_mfma.hip); curve position p holds
// sample crv.perm[p]. Queries, candidate keys, lists and bounds all refer to
// curve positions (the refine step maps them to sample ids while it reads the
// candidates from a curve-ordered copy of the samples). A workgroup's queries
// are consecutive positions; it scans
// tiles outward from its own along the curve and skips every tile (or, where
// the scan enters one, every superblock of SB_TILES_MFMA tiles) whose
// projected box is farther from the workgroup's query box than the largest
// distance threshold of its queries (the bound and its rounding margins are
// derived with the pruning test below). The thresholds are exchanged between
// the wavefronts through a double-buffered LDS array at each stage barrier, so
// all wavefronts take the same skipping decisions. The certificate epilogue
// is that of MODE 0: a skipped candidate lies beyond the threshold at the
// time of the skip, hence beyond every later one.
// Curve scans run as two 4-wavefront workgroups per CU where both fit in LDS
// (two candidate stages and 40-entry query buffers each): a wavefront's list
// merge then holds up three others at the tile barrier instead of seven, and
// the other workgroup keeps the CU busy meanwhile.
constexpr int CURVE_PAIR_BUF = 40;
template <class Tr, int KS>
constexpr bool curve_pair()
{
    return 2 * (2 * KS * 64 * static_cast<int>(sizeof(typename Tr::frag)) + 4 * 32 * CURVE_PAIR_BUF * 8 + 2048) <=
           160 * 1024;
}

template <class Tr, int KS, int WV, int E, int MODE>
__global__ __launch_bounds__(64 * WV, (MODE == 2 && WV == 4 && curve_pair<Tr, KS>()) ? 2 : 1) void k_select_mfma(
    const typename Tr::elem* __restrict__ Aq,
                                                          const typename Tr::elem* __restrict__ Bc, int n, int kp,
                                                          const float* __restrict__ ynorm2,
                                                          const unsigned* __restrict__ rmax_bits, ErrModel em,
                                                          uint64_t* __restrict__ lists, float* __restrict__ lb_out,
                                                          BucketArgs ba, CurveArgs crv,
                                                          unsigned long long* __restrict__ pair_count)
{
    constexpr bool LEARNED = MODE == 1;
    constexpr bool CURVE = MODE == 2;
    using elem = typename Tr::elem;
    using frag = typename Tr::frag;
    constexpr int CAP = WAVE * E;
    constexpr int kpad = KS * Tr::KSTEP;        // padded contraction length
    constexpr int NQ = 32;                      // queries per wavefront
    // per-query LDS buffer entries (curve scans in pairs of 4-wavefront workgroups: 40)
    constexpr int BUF = (MODE == 2 && WV == 4 && curve_pair<Tr, KS>()) ? CURVE_PAIR_BUF : WV == 8 ? 48 : 64;
    // two candidate stages, fragment-major: [stage][k-step][half][row] so that
    // lane l reads consecutive fragments (no bank conflicts). The next tile is
    // prefetched into registers while the current one is consumed.
    constexpr int STAGE_BYTES = KS * 64 * static_cast<int>(sizeof(frag));
    constexpr int CHUNKS = STAGE_BYTES / 16;                 // 16-byte pieces per tile
    constexpr int PF = (CHUNKS + 64 * WV - 1) / (64 * WV);  // pieces per thread
    __shared__ __attribute__((aligned(16))) frag s_tile[2][KS][2][32];
    __shared__ uint64_t s_buf[WV][NQ][BUF];

    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int half = lane >> 5;
    __shared__ int s_qid[WV][NQ];

    // query ids of this wavefront (-1: none) and the candidate tile range
    int q0 = 0, tbeg = 0, tend = 0;
    if constexpr (LEARNED) {
        const int w = blockIdx.x;
        if (w >= *ba.n_work) return;   // whole workgroup
        const int2 wk = ba.work[w];
        const int qend = ba.qptr[wk.x + 1];
        q0 = wk.y + wave * NQ;
        tbeg = ba.tptr[wk.x];
        tend = ba.tptr[wk.x + 1];
        if (lane < NQ) s_qid[wave][lane] = q0 + lane < qend ? ba.qids[q0 + lane] : -1;
    } else if constexpr (CURVE) {
        q0 = (xcd_block() * WV + wave) * NQ;
        tend = (n + 31) / 32;
        if (lane < NQ) s_qid[wave][lane] = q0 + lane < n ? q0 + lane : -1;   // curve positions
    } else {
        q0 = (blockIdx.x * WV + wave) * NQ;
        tend = (n + 31) / 32;
        if (lane < NQ) s_qid[wave][lane] = q0 + lane < n ? q0 + lane : -1;
    }
    wave_lds_sync();

    frag qa[KS];
    {
        // query operand row: curve position (MODE 2) or sample id
        int row = CURVE ? min(q0 + (lane & 31), n - 1) : s_qid[wave][lane & 31];
        if (row < 0) row = max(s_qid[wave][0], 0);
        const elem* src = Aq + static_cast<size_t>(row) * kpad + half * Tr::VEC;
#pragma unroll
        for (int s = 0; s < KS; ++s) qa[s] = Tr::load(src + s * Tr::KSTEP);
    }
    float tauv[16];
    if (LEARNED && !ba.first) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int qid = s_qid[wave][acc_row(r, half)];
            tauv[r] = qid >= 0 ? key_dist(lists[static_cast<size_t>(qid) * CAP + (kp - 1)]) : -__uint_as_float(0x7F800000u);
        }
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r)
            tauv[r] = (!LEARNED || s_qid[wave][acc_row(r, half)] >= 0) ? __uint_as_float(0x7F800000u)
                                                                      : -__uint_as_float(0x7F800000u);
        for (int q = 0; q < NQ; ++q) {
            const int qg = s_qid[wave][q];
            if (qg >= 0)
                for (int t = lane; t < CAP; t += WAVE) lists[static_cast<size_t>(qg) * CAP + t] = KEY_INF;
        }
    }
    wave_lds_sync();
    const int nq_valid = __popcll(__ballot(lane < NQ && s_qid[wave][lane] >= 0));
    unsigned long long pairs = 0;

    // a tile of the tile-major candidate operand is one contiguous block, laid
    // out exactly like an LDS stage: it moves as 16-byte pieces
    // the query fragments have landed before the loop, so the only vector
    // loads in flight inside it are the next tile's prefetch
    int qrow[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) qrow[r] = s_qid[wave][acc_row(r, half)];

    // MODE 2: the query boxes in projected space (s_qbox[w]: wavefront w's,
    // s_qbox[WV]: the workgroup's), the squared norms of the queries
    // (thresholds are kept as scores s = |y_j|^2 - 2 y_i.y_j, the distance
    // threshold is s + |y_i|^2) and the scan cursor
    __shared__ float s_qbox[WV + 1][2][PR_DIMS];
    __shared__ float s_thr[2][WV];
    const float* qlo = &s_qbox[WV][0][0];
    const float* qhi = &s_qbox[WV][1][0];
    const float* wlo = &s_qbox[wave][0][0];
    const float* whi = &s_qbox[wave][1][0];
    // |y_i|^2 of the queries for the distance thresholds: in registers, or in
    // LDS for short contractions (measured faster there; the long ones are
    // short of LDS instead)
    constexpr bool YQ_LDS = KS <= 8;
    __shared__ float s_yq[WV][NQ];
    float yq[YQ_LDS ? 1 : 16];
    CurveScan scan;
    scan.init(0);
    int own_t = 0;
    BoxBound bb = {0.f, 1.f, 0.f};
    if constexpr (CURVE) {
        if constexpr (YQ_LDS) {
            if (lane < NQ) s_yq[wave][lane] = s_qid[wave][lane] >= 0 ? ynorm2[s_qid[wave][lane]] : 0.f;
        } else {
#pragma unroll
            for (int r = 0; r < 16; ++r) yq[r] = qrow[r] >= 0 ? ynorm2[qrow[r]] : 0.f;
        }
#pragma unroll
        for (int c = 0; c < PR_DIMS; ++c) {
            const bool ok = lane < NQ && q0 + lane < n;
            const float v = ok ? crv.zs[static_cast<size_t>(q0 + lane) * PR_DIMS + c] : 0.f;
            float lo = ok ? v : __uint_as_float(0x7F800000u), hi = ok ? v : -__uint_as_float(0x7F800000u);
#pragma unroll
            for (int o = WAVE / 2; o > 0; o >>= 1) {
                lo = fminf(lo, shfl_xor_f32(lo, o));
                hi = fmaxf(hi, shfl_xor_f32(hi, o));
            }
            if (lane == 0) {
                s_qbox[wave][0][c] = lo;
                s_qbox[wave][1][c] = hi;
            }
        }
        __syncthreads();
        if (threadIdx.x < PR_DIMS) {
            const int c = threadIdx.x;
            float lo = s_qbox[0][0][c], hi = s_qbox[0][1][c];
            for (int w = 1; w < WV; ++w) {
                lo = fminf(lo, s_qbox[w][0][c]);
                hi = fmaxf(hi, s_qbox[w][1][c]);
            }
            s_qbox[WV][0][c] = lo;
            s_qbox[WV][1][c] = hi;
        }
        __syncthreads();
        own_t = min(tend - 1, (xcd_block() * WV * NQ + WV * NQ / 2) / 32);
        const float R = __uint_as_float(*rmax_bits);
        bb.zerr = crv.zcoef * R;
        bb.pscale = *crv.pscale;
        bb.yerr = crv.ycoef * R;
        scan.init(own_t);
    }
    __builtin_amdgcn_s_waitcnt(0);
    u32x4 pf[PF];
    int cid_pf = -1;
    int tile = -1;
    float wb_pf = 0.f;   // MODE 2: bound of the prefetched tile to this wavefront's box
    if (tbeg < tend)
        tile = CURVE ? scan.next(__uint_as_float(0x7F800000u), own_t, tend, crv, qlo, qhi, wlo, whi, bb, wb_pf)
                     : tbeg;
    if (tile >= 0) {
        const u32x4* g = reinterpret_cast<const u32x4*>(Bc + static_cast<size_t>(tile) * 32 * kpad);
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int ch = threadIdx.x + u * 64 * WV;
            if (ch < CHUNKS) pf[u] = g[ch];
        }
        if constexpr (LEARNED) cid_pf = ba.cid[static_cast<size_t>(tile) * 32 + (lane & 31)];
        if constexpr (CURVE) cid_pf = tile * 32 + (lane & 31) < n ? tile * 32 + (lane & 31) : -1;
    }
    // the buffers' fill, wave-uniform: query q's count in byte q % 4 of
    // cntw[q / 4] (every index below is a compile-time constant, so they stay
    // in scalar registers; BUF <= 64 fits a byte)
    static_assert(BUF <= 255, "a buffer count must fit a byte");
    uint32_t cntw[NQ / 4];
#pragma unroll
    for (int i = 0; i < NQ / 4; ++i) cntw[i] = 0u;
    auto cnt_of = [&](int q) { return static_cast<int>((cntw[q >> 2] >> (8 * (q & 3))) & 0xFFu); };
    // lists that start empty are filled by the first tiles without merging
    bool filling = !LEARNED || ba.first;
    const int fill_tiles = CAP / 32;   // the whole list capacity: a tighter first threshold
    // MODE 2: this wavefront's largest distance threshold, an upper bound of
    // s + |y_i|^2 over its queries; recomputed only after thresholds change
    float wthr = __uint_as_float(0x7F800000u);
    bool thr_dirty = true;
    for (int it = 0; tile >= 0; ++it) {
        const int stage = it & 1;
        if constexpr (CURVE) {
            if (thr_dirty) {
                float t = -__uint_as_float(0x7F800000u);
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    if (qrow[r] >= 0) {
                        const float y2 = YQ_LDS ? s_yq[wave][acc_row(r, half)] : yq[YQ_LDS ? 0 : r];
                        t = fmaxf(t, fmaxf(tauv[r] + y2, 0.f) * (1.f + 4.8e-7f));
                    }
                // read from one lane: the compiler then sees a wave-uniform
                // value and keeps the branches on it (and the counts) scalar
                wthr = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wave_max_f32(t))));
                thr_dirty = false;
            }
            if (lane == 0) s_thr[stage][wave] = wthr;
        }
        {
            u32x4* d = reinterpret_cast<u32x4*>(&s_tile[stage][0][0][0]);
#pragma unroll
            for (int u = 0; u < PF; ++u) {
                const int ch = threadIdx.x + u * 64 * WV;
                if (ch < CHUNKS) d[ch] = pf[u];
            }
        }
        const int cid_cur = cid_pf;
        const float wb_cur = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wb_pf)));
        __syncthreads();                 // stage visible; the other stage's readers finished a tile ago
        float thr = __uint_as_float(0x7F800000u);
        if constexpr (CURVE) {
            thr = s_thr[stage][0];
#pragma unroll
            for (int w = 1; w < WV; ++w) thr = fmaxf(thr, s_thr[stage][w]);
        }
        int next;
        if constexpr (CURVE)
            next = scan.next(thr, own_t, tend, crv, qlo, qhi, wlo, whi, bb, wb_pf);
        else
            next = tile + 1 < tend ? tile + 1 : -1;
        if (next >= 0) {
            const u32x4* g = reinterpret_cast<const u32x4*>(Bc + static_cast<size_t>(next) * 32 * kpad);
#pragma unroll
            for (int u = 0; u < PF; ++u) {
                const int ch = threadIdx.x + u * 64 * WV;
                if (ch < CHUNKS) pf[u] = g[ch];
            }
            if constexpr (LEARNED) cid_pf = ba.cid[static_cast<size_t>(next) * 32 + (lane & 31)];
            if constexpr (CURVE) cid_pf = next * 32 + (lane & 31) < n ? next * 32 + (lane & 31) : -1;
        }
        // MODE 2, after the fill: a tile the workgroup scans may still lie
        // beyond this wavefront's own box and thresholds
        if constexpr (CURVE) {
            if (!filling && wb_cur > wthr) {
                tile = next;
                continue;
            }
        }
        // all fragment reads are issued before the products (up to 16 at a
        // time), and even / odd K-steps go to two accumulators, so the chain of
        // dependent MFMAs is half as long and does not wait on each LDS read
        f32x16 acc;
        {
            constexpr int BATCH = KS <= 16 ? KS : 4;
            const f32x16 zero = {};
            f32x16 acc0 = zero, acc1 = zero;
#pragma unroll
            for (int s0 = 0; s0 < KS; s0 += BATCH) {
                frag bfr[BATCH];
#pragma unroll
                for (int u = 0; u < BATCH; ++u)
                    if (s0 + u < KS) bfr[u] = s_tile[stage][s0 + u][half][lane & 31];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < BATCH; ++u) {
                    const int s = s0 + u;
                    if (s < KS) {
                        if (s % 2 == 0)
                            acc0 = Tr::mma(qa[s], bfr[u], acc0);
                        else
                            acc1 = Tr::mma(qa[s], bfr[u], acc1);
                    }
                }
            }
            acc = KS > 1 ? acc0 + acc1 : acc0;
        }

        const int cand = MODE != 0 ? cid_cur : tile * 32 + (lane & 31);
        const bool valid = MODE != 0 ? cand >= 0 : cand < n;
        pairs += static_cast<unsigned long long>(nq_valid) *
                 static_cast<unsigned long long>(__popcll(__ballot(valid) & 0xFFFFFFFFull));
        if (filling) {
            // the first CAP / 32 tiles go straight into the (empty) lists
            const int slot = it * 32 + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (qrow[r] >= 0)
                    lists[static_cast<size_t>(qrow[r]) * CAP + slot] =
                        valid ? make_key(acc[r], static_cast<uint32_t>(cand)) : KEY_INF;
            if (it + 1 == fill_tiles || next < 0) {
                filling = false;
                // the lists' stores complete before other lanes read them
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                for (int q = 0; q < NQ; ++q) {
                    const int qg = s_qid[wave][q];
                    if (qg < 0) continue;
                    const float nt = sort_query_list<E>(lists + static_cast<size_t>(qg) * CAP, kp);
                    const int rr = 4 * (q / 8) + (q % 4), hh = (q / 4) & 1;
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        if (r == rr && half == hh) tauv[r] = nt;
                    thr_dirty = true;
                }
            }
            tile = next;
            continue;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float sc = acc[r];
            uint64_t mask = __ballot(valid && sc <= tauv[r]);
            if (mask) {
                const int qa_ = acc_row(r, 0), qb_ = acc_row(r, 1);
                uint32_t ma = static_cast<uint32_t>(mask), mb = static_cast<uint32_t>(mask >> 32);
                int ca = cnt_of(qa_), cb = cnt_of(qb_);
                const bool fa = ca + __popc(ma) > BUF, fb = cb + __popc(mb) > BUF;
                if (fa || fb) {
                    // a full buffer is merged before this tile's keys are added,
                    // so every merge takes nearly BUF keys
                    wave_lds_sync();
                    if (fa) {
                        const int qg = s_qid[wave][qa_];
                        float nt = -__uint_as_float(0x7F800000u);
                        if (qg >= 0)
                            nt = merge_query_list<E>(lists + static_cast<size_t>(qg) * CAP, &s_buf[wave][qa_][0], ca,
                                                     kp);
                        if (half == 0) tauv[r] = nt;
                        thr_dirty = true;
                        ca = 0;
                        cntw[qa_ >> 2] &= ~(0xFFu << (8 * (qa_ & 3)));
                    }
                    if (fb) {
                        const int qg = s_qid[wave][qb_];
                        float nt = -__uint_as_float(0x7F800000u);
                        if (qg >= 0)
                            nt = merge_query_list<E>(lists + static_cast<size_t>(qg) * CAP, &s_buf[wave][qb_][0], cb,
                                                     kp);
                        if (half == 1) tauv[r] = nt;
                        thr_dirty = true;
                        cb = 0;
                        cntw[qb_ >> 2] &= ~(0xFFu << (8 * (qb_ & 3)));
                    }
                    wave_lds_sync();
                    mask = __ballot(valid && sc <= tauv[r]);
                    ma = static_cast<uint32_t>(mask);
                    mb = static_cast<uint32_t>(mask >> 32);
                }
                // slot: the half's count plus the rank among the half's
                // passing lanes (mbcnt64 counts the lower half's lanes too in
                // the upper half)
                const int pa = __popc(ma), pb = __popc(mb);
                const int slot0 = half ? qb_ * BUF + cb - pa : qa_ * BUF + ca;
                if (valid && sc <= tauv[r])
                    (&s_buf[wave][0][0])[slot0 + mbcnt64(mask)] = make_key(sc, static_cast<uint32_t>(cand));
                cntw[qa_ >> 2] += static_cast<uint32_t>(pa) << (8 * (qa_ & 3));
                cntw[qb_ >> 2] += static_cast<uint32_t>(pb) << (8 * (qb_ & 3));
            }
        }
        tile = next;
    }
    wave_lds_sync();
    {
        // the last merges in a loop that is not unrolled: query q's count
        // moved to lane q
        int cnt_lane = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (lane == q) cnt_lane = cnt_of(q);
        uint64_t nonempty = __ballot(cnt_lane > 0);
        while (nonempty) {
            const int q = __builtin_ctzll(nonempty);
            nonempty &= nonempty - 1;
            const int qg = s_qid[wave][q];
            if (qg >= 0)
                merge_query_list<E>(lists + static_cast<size_t>(qg) * CAP, &s_buf[wave][q][0],
                                    __builtin_amdgcn_readlane(cnt_lane, q), kp);
            wave_lds_sync();
        }
    }
    if (pair_count && lane == 0) atomicAdd(pair_count, pairs);

    if constexpr (LEARNED) return;
    // certificate lower bound for the candidates left out of each list
    const double R = static_cast<double>(__uint_as_float(*rmax_bits));
    if (lane < NQ) {
        const int qg = s_qid[wave][lane];
        if (qg >= 0) {
            const float sl = key_dist(lists[static_cast<size_t>(qg) * CAP + (kp - 1)]);
            const double yi2 = static_cast<double>(ynorm2[qg]);
            const double yi = sqrt(yi2);
            const double Ei =
                em.gamma * (R + 1.05 * yi) * (R + 1.05 * yi) + em.norm * R * R + em.cross * yi * R + 1e-30;
            const double t = static_cast<double>(sl) + yi2 - Ei;
            double D = t > 0.0 ? sqrt(t) : 0.0;
            D -= em.center * (yi + R);
            D = D > 0.0 ? D : 0.0;
            lb_out[qg] = static_cast<float>(D * D * (1.0 - 1.0 / 1048576.0));
        }
    }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_colmean(const float* X, int n, int m, double* colpart, int colblocks, double* mu, hipStream_t st)
{
    const int rpb = (n + colblocks - 1) / colblocks;
    hipLaunchKernelGGL(k_colsum_partial, dim3(colblocks), dim3(256), 0, st, X, n, m, rpb, colpart);
    hipLaunchKernelGGL(k_colsum_finish, dim3(1), dim3(256), 0, st, colpart, colblocks, m, n, mu);
    return hipGetLastError();
}

// sample-order operand rows (no row maps): one thread per row for short rows
static void launch_rows(const float* X, int n, int npad, int m, const double* mu, int split, int kpad, void* Aq,
                        void* Bc, float* ynorm2, unsigned* rmax_bits, const int* brow, const int* arow, hipStream_t st)
{
    if (m <= PREP_THREAD_M && split == 0 && !brow && !arow)
        hipLaunchKernelGGL(k_prep_rows_thread, dim3((npad + 255) / 256), dim3(256), 0, st, X, n, npad, m, mu, split,
                           kpad, Aq, Bc, ynorm2, rmax_bits);
    else
        hipLaunchKernelGGL(k_prep_rows, dim3(prep_blocks(npad)), dim3(256), 0, st, X, n, npad, m, mu, split, kpad, Aq,
                           Bc, ynorm2, rmax_bits, brow, arow);
}

hipError_t launch_prep_rows(const float* X, int n, int m, const double* mu, int split, int kpad, void* Aq, void* Bc,
                            float* ynorm2, unsigned* rmax_bits, const int* brow, const int* arow, hipStream_t st)
{
    const int npad = brow ? n : (n + 31) / 32 * 32;
    launch_rows(X, n, npad, m, mu, split, kpad, Aq, Bc, ynorm2, rmax_bits, brow, arow, st);
    return hipGetLastError();
}

// Xs holds the samples in curve order, so operand row p is input row p: the
// sample-order kernels without row maps, reading and writing rows in order
hipError_t launch_prep_rows_curve(const float* Xs, int n, int m, const double* mu, int split, int kpad, void* Aq,
                                  void* Bc, float* ynorm2, unsigned* rmax_bits, hipStream_t st)
{
    const int npad = (n + 31) / 32 * 32;
    launch_rows(Xs, n, npad, m, mu, split, kpad, Aq, Bc, ynorm2, rmax_bits, nullptr, nullptr, st);
    return hipGetLastError();
}

hipError_t launch_prep(const float* X, int n, int m, int split, int kpad, double* colpart, int colblocks,
                       double* mu, void* Aq, void* Bc, float* ynorm2, unsigned* rmax_bits, const int* brow,
                       const int* arow, hipStream_t st)
{
    const int rpb = (n + colblocks - 1) / colblocks;
    // with a row map the padding rows of the last tile are filled separately
    const int npad = brow ? n : (n + 31) / 32 * 32;
    hipLaunchKernelGGL(k_colsum_partial, dim3(colblocks), dim3(256), 0, st, X, n, m, rpb, colpart);
    hipLaunchKernelGGL(k_colsum_finish, dim3(1), dim3(256), 0, st, colpart, colblocks, m, n, mu);
    launch_rows(X, n, npad, m, mu, split, kpad, Aq, Bc, ynorm2, rmax_bits, brow, arow, st);
    return hipGetLastError();
}

template <class Tr, int KS, int WV>
static hipError_t launch_sel(const void* Aq, const void* Bc, int n, int kp, const float* ynorm2, const unsigned* rmax,
                             ErrModel em, uint64_t* lists, int cap, float* lb, const BucketArgs* ba, int max_work,
                             const CurveArgs* crv, unsigned long long* pairs, hipStream_t st)
{
    using elem = typename Tr::elem;
    const int rows_per_block = WV * 32;
    const dim3 block(64 * WV);
    const elem* A = static_cast<const elem*>(Aq);
    const elem* B = static_cast<const elem*>(Bc);
    // the lists buffer holds n * cap keys; only capacities 128 and 256 exist
    if (kp > cap) return hipErrorInvalidValue;
    if (cap != 128 && cap != 256) return hipErrorInvalidValue;
    const BucketArgs nb = {};
    const CurveArgs nc = {};
    if (ba) {
        if (max_work <= 0) return hipSuccess;
        const dim3 grid(max_work);
        if (cap == 128)
            hipLaunchKernelGGL((k_select_mfma<Tr, KS, WV, 2, 1>), grid, block, 0, st, A, B, n, kp, ynorm2, rmax, em,
                               lists, lb, *ba, nc, pairs);
        else
            hipLaunchKernelGGL((k_select_mfma<Tr, KS, WV, 4, 1>), grid, block, 0, st, A, B, n, kp, ynorm2, rmax, em,
                               lists, lb, *ba, nc, pairs);
        return hipGetLastError();
    }
    const dim3 grid((n + rows_per_block - 1) / rows_per_block);
    if (crv) {
        // curve-ordered workgroup scan (long contractions; the short ones walk
        // the box tree in knn_tree.hip)
        constexpr int WC = curve_pair<Tr, KS>() ? 4 : WV;
        const dim3 gridc((n + WC * 32 - 1) / (WC * 32)), blockc(64 * WC);
        if (cap == 128)
            hipLaunchKernelGGL((k_select_mfma<Tr, KS, WC, 2, 2>), gridc, blockc, 0, st, A, B, n, kp, ynorm2, rmax, em,
                               lists, lb, nb, *crv, pairs);
        else
            hipLaunchKernelGGL((k_select_mfma<Tr, KS, WC, 4, 2>), gridc, blockc, 0, st, A, B, n, kp, ynorm2, rmax, em,
                               lists, lb, nb, *crv, pairs);
        return hipGetLastError();
    }
    if (cap == 128)
        hipLaunchKernelGGL((k_select_mfma<Tr, KS, WV, 2, 0>), grid, block, 0, st, A, B, n, kp, ynorm2, rmax, em, lists,
                           lb, nb, nc, pairs);
    else
        hipLaunchKernelGGL((k_select_mfma<Tr, KS, WV, 4, 0>), grid, block, 0, st, A, B, n, kp, ynorm2, rmax, em, lists,
                           lb, nb, nc, pairs);
    return hipGetLastError();
}

// Instantiated contraction lengths (in MFMA K-steps); the operand K is padded
// with zeros up to the next one. WV (wavefronts per workgroup) is 8 where the
// two LDS stages and the query buffers fit in LDS, else 4.
static const int kBf16Steps[] = {2, 3, 4, 5, 6, 7, 8, 10, 13, 16, 20, 25, 32};
static const int kF32Steps[] = {2, 4, 6, 8, 10, 12, 16, 24, 32, 48, 64, 96, 128};

int mfma_kstep(int split) { return split == 0 ? TraitsF32::KSTEP : TraitsBF16::KSTEP; }

int mfma_pick_ksteps(int split, int needed)
{
    const int* lst = split == 0 ? kF32Steps : kBf16Steps;
    const int cnt = split == 0 ? static_cast<int>(sizeof(kF32Steps) / sizeof(int))
                               : static_cast<int>(sizeof(kBf16Steps) / sizeof(int));
    for (int t = 0; t < cnt; ++t)
        if (lst[t] >= needed) return lst[t];
    return -1;
}

#define KVB_SEL_CASE(TR, K, WV) \
    case K: return launch_sel<TR, K, WV>(Aq, Bc, n, kp, ynorm2, rmax, em, lists, cap, lb, ba, max_work, crv, pairs, st);

int select_mfma_queries_per_block(int split, int kpad)
{
    const int ks = kpad / mfma_kstep(split);
    const bool four = split == 0 ? ks >= 64 : ks >= 32;
    return (four ? 4 : 8) * 32;
}

hipError_t launch_select_mfma(int split, const void* Aq, const void* Bc, int n, int kpad, int kp, const float* ynorm2,
                              const unsigned* rmax, ErrModel em, uint64_t* lists, int cap, float* lb,
                              const BucketArgs* ba, int max_work, const CurveArgs* crv, unsigned long long* pairs,
                              hipStream_t st)
{
    const int ks = kpad / mfma_kstep(split);
    if (split == 0) {
        switch (ks) {
            KVB_SEL_CASE(TraitsF32, 2, 8)
            KVB_SEL_CASE(TraitsF32, 4, 8)
            KVB_SEL_CASE(TraitsF32, 6, 8)
            KVB_SEL_CASE(TraitsF32, 8, 8)
            KVB_SEL_CASE(TraitsF32, 10, 8)
            KVB_SEL_CASE(TraitsF32, 12, 8)
            KVB_SEL_CASE(TraitsF32, 16, 8)
            KVB_SEL_CASE(TraitsF32, 24, 8)
            KVB_SEL_CASE(TraitsF32, 32, 8)
            KVB_SEL_CASE(TraitsF32, 48, 8)
            KVB_SEL_CASE(TraitsF32, 64, 4)
            KVB_SEL_CASE(TraitsF32, 96, 4)
            KVB_SEL_CASE(TraitsF32, 128, 4)
        default: return hipErrorInvalidValue;
        }
    }
    switch (ks) {
        KVB_SEL_CASE(TraitsBF16, 2, 8)
        KVB_SEL_CASE(TraitsBF16, 3, 8)
        KVB_SEL_CASE(TraitsBF16, 4, 8)
        KVB_SEL_CASE(TraitsBF16, 5, 8)
        KVB_SEL_CASE(TraitsBF16, 6, 8)
        KVB_SEL_CASE(TraitsBF16, 7, 8)
        KVB_SEL_CASE(TraitsBF16, 8, 8)
        KVB_SEL_CASE(TraitsBF16, 10, 8)
        KVB_SEL_CASE(TraitsBF16, 13, 8)
        KVB_SEL_CASE(TraitsBF16, 16, 8)
        KVB_SEL_CASE(TraitsBF16, 20, 8)
        KVB_SEL_CASE(TraitsBF16, 25, 8)
        KVB_SEL_CASE(TraitsBF16, 32, 4)
    default: return hipErrorInvalidValue;
    }
}
#undef KVB_SEL_CASE

}  // namespace kvb
