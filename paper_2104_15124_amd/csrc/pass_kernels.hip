// O(nk) passes over the k-NN pattern (gfx950): bandwidths, the epsilon
// tuning sums, the density estimate and the alpha/Markov normalisation.
// These kernels stream idx/d2 (8 bytes per stored entry) and gather per-sample
// vectors of neighbours; they are bound by HBM bandwidth except the tuning
// pass, which evaluates one exponential per grid point and entry.
//
// One wavefront owns one row for the row-wise passes (k <= 256 entries, lanes
// strided over them), so row sums reduce inside the wavefront in a fixed
// butterfly order and no atomics are needed. The same passes also run over a
// general CSR pattern (rows of any length, given by rowptr), such as the union
// pattern E u E^T.
#include "kvb_device.h"
#include "kvb_kernels.h"

namespace kvb {

// b_i = sqrt(sum_{r=1..k0} d2[i, r])  (Section 2.1, bandwidth eq.; r = 0 is i itself)
__global__ __launch_bounds__(256) void k_adhoc_bandwidth(const float* __restrict__ d2, int n, int k, int k0,
                                                         float* __restrict__ b)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* row = d2 + static_cast<size_t>(i) * k;
    double s = 0.0;
    for (int r = 1; r <= k0; ++r) s += static_cast<double>(row[r]);
    b[i] = static_cast<float>(sqrt(s));
}

// The k-NN rows in the order of the curve the matrix-core k-NN scanned (row p
// = sample cid[p]), their neighbours as curve positions (pos of the sample
// id), and the bandwidth of each (as k_adhoc_bandwidth). The passes that
// follow then gather the per-sample vectors of a row's neighbours from curve
// positions near the row's own: neighbouring rows share cache lines.
// One wavefront per row.
__global__ __launch_bounds__(256) void k_curve_rows(const int32_t* __restrict__ idx, const float* __restrict__ d2,
                                                    int n, int k, int k0, const int32_t* __restrict__ cid,
                                                    const int32_t* __restrict__ pos, int32_t* __restrict__ idx_c,
                                                    float* __restrict__ d2_c, float* __restrict__ b_c)
{
    const int lane = lane_id();
    const int p = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (p >= n) return;
    const int i = cid[p];
    const int32_t* irow = idx + static_cast<size_t>(i) * k;
    const float* drow = d2 + static_cast<size_t>(i) * k;
    for (int r = lane; r < k; r += WAVE) {
        idx_c[static_cast<size_t>(p) * k + r] = pos[irow[r]];
        d2_c[static_cast<size_t>(p) * k + r] = drow[r];
    }
    if (lane == 0) {
        double s = 0.0;
        for (int r = 1; r <= k0; ++r) s += static_cast<double>(drow[r]);
        b_c[p] = static_cast<float>(sqrt(s));
    }
}

// out[i] = in[pos[i]] for up to three per-sample vectors (null: skipped): the
// curve-ordered vectors back in sample order, written in order (the gathers
// read 4-byte values from arrays small enough to stay in the caches, where
// the scatter out[cid[p]] = in[p] wrote 4-byte values to random places)
__global__ __launch_bounds__(256) void k_gather_samples(const int32_t* __restrict__ pos, int n,
                                                        const float* __restrict__ a_c, float* __restrict__ a,
                                                        const float* __restrict__ b_c, float* __restrict__ b,
                                                        const float* __restrict__ c_c, float* __restrict__ c)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int p = pos[i];
    if (a) a[i] = a_c[p];
    if (b) b[i] = b_c[p];
    if (c) c[i] = c_c[p];
}

// Row sums of exp(-d2/(e rho_i rho_j)): the argument in float64, the kernel
// value in float32 (its relative error, about x 2^-24 at argument x, stays far
// inside the 1e-5 entry tolerance where the terms matter), the sum in float64;
// four rows per wavefront, 16 lanes per row (entries strided by 16), the
// group's partial sums reduced in a fixed butterfly order. Every lane of the
// group returns the row's sum.
constexpr int RL = 16;   // lanes per row in the row-sum passes

__device__ __forceinline__ double row_kernel_sum16(const int32_t* __restrict__ irow, const float* __restrict__ drow,
                                                   int k, const float* __restrict__ rho, double inv_e_rhoi, int gl)
{
    // four entries per lane at a time: their loads and gathers are in flight
    // together; the sum still runs entry by entry
    constexpr int B = 4;
    double s = 0.0;
    for (int r0 = gl; r0 < k; r0 += B * RL) {
        float dv[B];
        int jv[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int r = r0 + u * RL;
            dv[u] = r < k ? drow[r] : 0.f;
            jv[u] = r < k ? irow[r] : 0;
        }
        float rj[B];
#pragma unroll
        for (int u = 0; u < B; ++u) rj[u] = rho[jv[u]];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            if (r0 + u * RL < k) {
                const double x = static_cast<double>(dv[u]) * inv_e_rhoi / static_cast<double>(rj[u]);
                s += static_cast<double>(expf(-static_cast<float>(x)));
            }
        }
    }
#pragma unroll
    for (int o = 1; o < RL; o <<= 1) s += shfl_xor_f64(s, o);
    return s;
}

// Row i spans entries [rowptr_i, rowptr_{i+1}), or [i k, (i + 1) k) when rowptr is null.
__device__ __forceinline__ int64_t row_begin(const int64_t* __restrict__ rowptr, int i, int k)
{
    return rowptr ? rowptr[i] : static_cast<int64_t>(i) * k;
}
__device__ __forceinline__ int row_length(const int64_t* __restrict__ rowptr, int i, int k)
{
    return rowptr ? static_cast<int>(rowptr[i + 1] - rowptr[i]) : k;
}

// Row sums of the 4 its rows [base, base + 4 its) of a wavefront (its <= 16):
// four rows at a time, RL lanes per row, each sum formed exactly as
// row_kernel_sum16 forms it; the sum of row base + t is handed to lane t, so
// that the per-row epilogue (float64 powers) runs once per 4 its rows with that
// many lanes busy rather than once per four rows. Rows of a fixed k <= 64
// entries issue the next four rows' loads before the current four are summed.
// w is the width gathered by column (b or rho); rows at or past n sum to 0.
constexpr int ROWSUM_WAVES = 8192;   // fewest wavefronts a launch is given (8 per SIMD)

__host__ __device__ constexpr int rowsum_its(int n)
{
    return n >= 16 * 4 * ROWSUM_WAVES ? 16 : (n / (4 * ROWSUM_WAVES) > 1 ? n / (4 * ROWSUM_WAVES) : 1);
}

// blocks of four wavefronts, 16 rowsum_its(n) rows each
static int rowsum_blocks(int n) { return (n + 16 * rowsum_its(n) - 1) / (16 * rowsum_its(n)); }

__device__ __forceinline__ double wave_row_sums(const int32_t* __restrict__ idx, const float* __restrict__ d2,
                                                const int64_t* __restrict__ rowptr, int n, int k,
                                                const float* __restrict__ w, double e, int base, int its)
{
    constexpr int GROUPS = WAVE / RL;   // rows summed at a time
    const int lane = lane_id();
    const int g = lane / RL, gl = lane % RL;
    double mine = 0.0;
    if (rowptr == nullptr && k <= 4 * RL) {
        int jv[4];
        float dv[4];
        auto load = [&](int it, int (&jo)[4], float (&dout)[4]) {
            const int i = base + GROUPS * it + g;
            const size_t rb = static_cast<size_t>(i < n ? i : 0) * k;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int r = gl + u * RL;
                const bool ok = i < n && r < k;
                dout[u] = ok ? d2[rb + r] : 0.f;
                jo[u] = ok ? idx[rb + r] : 0;
            }
        };
        load(0, jv, dv);
#pragma unroll 1
        for (int it = 0; it < its; ++it) {
            const int i = base + GROUPS * it + g;
            float rj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) rj[u] = w[jv[u]];
            const double wi = static_cast<double>(w[i < n ? i : n - 1]);
            int jn[4];
            float dn[4];
            if (it + 1 < its) load(it + 1, jn, dn);
            const double inv = 1.0 / (e * wi);
            double s = 0.0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (i < n && gl + u * RL < k) {
                    const double x = static_cast<double>(dv[u]) * inv / static_cast<double>(rj[u]);
                    s += static_cast<double>(expf(-static_cast<float>(x)));
                }
            }
#pragma unroll
            for (int o = 1; o < RL; o <<= 1) s += shfl_xor_f64(s, o);
            const double t = __longlong_as_double(
                static_cast<long long>(shfl_u64(static_cast<uint64_t>(__double_as_longlong(s)), RL * (lane % GROUPS))));
            if (lane / GROUPS == it) mine = t;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                jv[u] = jn[u];
                dv[u] = dn[u];
            }
        }
        return mine;
    }
#pragma unroll 1
    for (int it = 0; it < its; ++it) {
        const int i = base + GROUPS * it + g;
        const int ic = i < n ? i : n - 1;
        const int64_t rb = row_begin(rowptr, ic, k);
        const double wi = static_cast<double>(w[ic]);
        const double s = row_kernel_sum16(idx + rb, d2 + rb, i < n ? row_length(rowptr, ic, k) : 0, w,
                                          1.0 / (e * wi), gl);
        const double t = __longlong_as_double(
            static_cast<long long>(shfl_u64(static_cast<uint64_t>(__double_as_longlong(s)), RL * (lane % GROUPS))));
        if (lane / GROUPS == it) mine = t;
    }
    return mine;
}

// psi_i = sum_r K_ir / (n (pi e b_i^2)^{d/2}), rho_i = 2 psi_i^beta
// (Section 2.1 density eqs.; Algorithm 1 caption). 4 rowsum_its(n) rows per
// wavefront (64 from n = 2^19 on).
__global__ __launch_bounds__(256) void k_density(const int32_t* __restrict__ idx, const float* __restrict__ d2,
                                                 const int64_t* __restrict__ rowptr, int n, int k,
                                                 const float* __restrict__ b, double e,
                                                 const double* __restrict__ e_dev, double d, double beta,
                                                 float* __restrict__ rho, float* __restrict__ psi)
{
    if (e_dev) e = *e_dev;
    const int its = rowsum_its(n);
    const int base = (blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * 4 * its;
    if (base >= n) return;
    const double s = wave_row_sums(idx, d2, rowptr, n, k, b, e, base, its);
    const int i = base + lane_id();
    if (lane_id() < 4 * its && i < n) {
        const double bi = static_cast<double>(b[i]);
        const double pi = 3.14159265358979323846;
        const double w = static_cast<double>(n) * pow(pi * e * bi * bi, 0.5 * d);
        const double p = s / w;
        rho[i] = static_cast<float>(2.0 * pow(p, beta));
        if (psi) psi[i] = static_cast<float>(p);
    }
}

// ------------------------------------------------------------------ tuning sums
// Block partials of chi[g] = sum over entries of exp(-x / e_g), x = d2/(rho_i rho_j).
// Each thread forms x for its entries and accumulates exp2(x c_g) for a group
// of 64 grid points in registers (c_g = -log2(e)/e_g, float32 per thread over
// its few entries; hardware exp2, whose flush of results below 2^-126 is far
// below the sum's rounding since every row contributes exp(0) = 1); the
// per-thread sums are then reduced in float64 in a fixed order.
constexpr int CHI_BLOCK = 256;
constexpr int CHI_GROUP = 64;   // grid points per register group

// ln e_g = ln e_min + g (ln e_max - ln e_min) / (G - 1)
__device__ __forceinline__ double grid_log(double lo, double hi, int G, int g)
{
    return lo + (static_cast<double>(g) * (hi - lo)) / static_cast<double>(G - 1);
}
constexpr int CHI_MIN_ENTRIES_PER_BLOCK = 4096;
constexpr int CHI_BATCH = 4;
constexpr int CHI_MAX_BLOCKS = 1024;

// CSR: rows given by rowptr [n + 1] (k unused) and, when rowid is not null,
// the row of every entry; otherwise k entries per row.
template <bool CSR>
__global__ __launch_bounds__(CHI_BLOCK) void k_chi_partial(const int32_t* __restrict__ idx,
                                                           const float* __restrict__ d2,
                                                           const int64_t* __restrict__ rowptr,
                                                           const int32_t* __restrict__ rowid, int n,
                                                           const float* __restrict__ rho, int64_t nnz, int k,
                                                           int G, double e_min, double e_max,
                                                           const double* __restrict__ scale_dev, int64_t per_block,
                                                           double* __restrict__ partial)
{
    const double sc = scale_dev ? *scale_dev : 1.0;
    const double log_emin = log(e_min * sc), log_emax = log(e_max * sc);
    __shared__ float s_c[256 + CHI_GROUP];
    __shared__ double sred[CHI_BLOCK / WAVE][CHI_GROUP];
    __shared__ float s_tr[WAVE][CHI_GROUP + 1];   // one wavefront's partials, transposed
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    if (CSR) nnz = rowptr[n];   // the launch is sized for an upper bound
    const int64_t base = static_cast<int64_t>(blockIdx.x) * per_block;
    const int64_t end = min(base + per_block, nnz);
    for (int g = threadIdx.x; g < 256 + CHI_GROUP; g += CHI_BLOCK)
        s_c[g] = g < G ? static_cast<float>(-1.4426950408889634 / exp(grid_log(log_emin, log_emax, G, g))) : 0.f;
    __syncthreads();
    for (int g0 = 0; g0 < G; g0 += CHI_GROUP) {
        // the group's coefficients are wave-uniform: held in scalar registers
        float cg[CHI_GROUP];
#pragma unroll
        for (int t = 0; t < CHI_GROUP; ++t)
            cg[t] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s_c[g0 + t])));
        float acc[CHI_GROUP];
#pragma unroll
        for (int t = 0; t < CHI_GROUP; ++t) acc[t] = 0.f;
        // CHI_BATCH entries per thread at a time (their loads and gathers in
        // flight together); the accumulation order stays entry by entry
        // the row of entry p = i k + r is tracked incrementally (no division
        // per entry): consecutive entries of a thread are CHI_BLOCK apart
        const int di = CSR ? 0 : CHI_BLOCK / k, dr = CSR ? 0 : CHI_BLOCK % k;
        int64_t irow, rend = 0;
        int rcol = 0;
        if (CSR && rowid) {
            irow = 0;
        } else if (CSR) {
            // the row holding the thread's first entry: last i with rowptr_i <= p
            const int64_t p = min(base + threadIdx.x, nnz - 1);
            int lo = 0, hi = n;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (rowptr[mid] <= p)
                    lo = mid;
                else
                    hi = mid;
            }
            irow = lo;
            rend = rowptr[lo + 1];
        } else {
            irow = (base + threadIdx.x) / k;
            rcol = static_cast<int>((base + threadIdx.x) - irow * k);
        }
        for (int64_t p0 = base + threadIdx.x; p0 < end; p0 += CHI_BATCH * CHI_BLOCK) {
            float dv[CHI_BATCH];
            int jv[CHI_BATCH];
            int64_t iv[CHI_BATCH];
#pragma unroll
            for (int u = 0; u < CHI_BATCH; ++u) {
                const int64_t p = p0 + u * CHI_BLOCK;
                const bool ok = p < end;
                dv[u] = ok ? d2[p] : 0.f;
                jv[u] = ok ? idx[p] : 0;
                if (CSR && rowid) {
                    iv[u] = ok ? rowid[p] : 0;
                } else if (CSR) {
                    // p < nnz = rowptr_n, so the walk stops at a row below n
                    if (ok) {
                        while (p >= rend) {
                            ++irow;
                            rend = rowptr[irow + 1];
                        }
                    }
                    iv[u] = ok ? irow : 0;
                } else {
                    iv[u] = ok ? irow : 0;
                    irow += di;
                    rcol += dr;
                    if (rcol >= k) {
                        rcol -= k;
                        ++irow;
                    }
                }
            }
            float x[CHI_BATCH];
#pragma unroll
            for (int u = 0; u < CHI_BATCH; ++u)
                x[u] = static_cast<float>(static_cast<double>(dv[u]) /
                                          (static_cast<double>(rho[iv[u]]) * static_cast<double>(rho[jv[u]])));
#pragma unroll
            for (int u = 0; u < CHI_BATCH; ++u) {
                if (p0 + u * CHI_BLOCK < end) {
#pragma unroll
                    for (int t = 0; t < CHI_GROUP; ++t) acc[t] += __builtin_amdgcn_exp2f(x[u] * cg[t]);
                }
            }
        }
        // fixed-order reduction: the wavefronts in turn store their partials
        // transposed, lane t sums grid point t over the 64 lanes in float64;
        // then the wavefronts in order
#pragma unroll 1
        for (int w = 0; w < CHI_BLOCK / WAVE; ++w) {
            if (wave == w) {
#pragma unroll
                for (int t = 0; t < CHI_GROUP; ++t) s_tr[lane][t] = acc[t];
                wave_lds_sync();
                double v = 0.0;
                for (int l = 0; l < WAVE; ++l) v += static_cast<double>(s_tr[l][lane]);
                sred[w][lane] = v;
            }
            __syncthreads();
        }
        if (threadIdx.x < CHI_GROUP && g0 + threadIdx.x < G) {
            double s = 0.0;
            for (int w = 0; w < CHI_BLOCK / WAVE; ++w) s += sred[w][threadIdx.x];
            partial[static_cast<size_t>(blockIdx.x) * G + g0 + threadIdx.x] = s;
        }
        __syncthreads();
    }
}

// Fixed-order reduction of the block partials, then slopes and the optimum
// (Section 2.3): slope_g = (ln chi_{g+1} - ln chi_g) / (ln e_{g+1} - ln e_g),
// g* = first argmax, e* = e_{g*}, dimension estimate 2 slope_{g*}.
// chi[g] = the sum of the block partials of grid point g: one workgroup per
// grid point, thread t summing blocks t, t + 256, ... in order, then a fixed
// tree over the threads. nnz_dev (or null): the pattern's entry count on the
// device; blocks past it hold zero partials and are skipped (adding zeros
// would change nothing).
__global__ __launch_bounds__(256) void k_chi_reduce(const double* __restrict__ partial, int nblocks, int G,
                                                    const int64_t* __restrict__ nnz_dev, int64_t per_block,
                                                    TuneResult* __restrict__ out)
{
    if (nnz_dev) nblocks = static_cast<int>(min(static_cast<int64_t>(nblocks), (*nnz_dev + per_block - 1) / per_block));
    __shared__ double red[256];
    const int g = blockIdx.x;
    double a = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) a += partial[static_cast<size_t>(b) * G + g];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out->chi[g] = red[0];
}

// Slopes and the optimum (Section 2.3): slope_g = (ln chi_{g+1} - ln chi_g) /
// (ln e_{g+1} - ln e_g), g* = first argmax, e* = e_{g*}, dimension estimate
// 2 slope_{g*}.
__global__ __launch_bounds__(256) void k_chi_finish(int G, double e_min, double e_max,
                                                    const double* __restrict__ scale_dev,
                                                    TuneResult* __restrict__ out)
{
    const double sc = scale_dev ? *scale_dev : 1.0;
    const double log_emin = log(e_min * sc), log_emax = log(e_max * sc);
    __shared__ double slope[256];
    if (threadIdx.x + 1 < G) {
        const int t = threadIdx.x;
        const double el = exp(grid_log(log_emin, log_emax, G, t));
        const double er = exp(grid_log(log_emin, log_emax, G, t + 1));
        slope[t] = (log(out->chi[t + 1]) - log(out->chi[t])) / (log(er) - log(el));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int best = 0;
        double best_s = -1.0 / 0.0;
        for (int t = 0; t + 1 < G; ++t) {
            if (slope[t] > best_s) {
                best_s = slope[t];
                best = t;
            }
        }
        out->g_star = best;
        out->e_star = exp(grid_log(log_emin, log_emax, G, best));
        out->dim = 2.0 * best_s;
    }
}

// ------------------------------------------------------------------ grid scale
// Block partial sums of ln(ref_i) and ln(rho_i) in float64.
__global__ __launch_bounds__(256) void k_logsum_partial(const float* __restrict__ ref, const float* __restrict__ rho,
                                                        int n, double* __restrict__ partial)
{
    __shared__ double sa[4], sb[4];
    double a = 0.0, c = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        a += log(static_cast<double>(ref[i]));
        c += log(static_cast<double>(rho[i]));
    }
    a = wave_sum_f64(a);
    c = wave_sum_f64(c);
    if ((threadIdx.x & 63) == 0) {
        sa[threadIdx.x >> 6] = a;
        sb[threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = sa[0] + sa[1] + sa[2] + sa[3];
        partial[2 * blockIdx.x + 1] = sb[0] + sb[1] + sb[2] + sb[3];
    }
}

__global__ __launch_bounds__(256) void k_logsum_finish(const double* __restrict__ partial, int nblocks, int n,
                                                      double* __restrict__ out)
{
    __shared__ double sa[256], sc[256];
    double a = 0.0, c = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) {
        a += partial[2 * b];
        c += partial[2 * b + 1];
    }
    sa[threadIdx.x] = a;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sa[threadIdx.x] += sa[threadIdx.x + o];
            sc[threadIdx.x] += sc[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double l2 = 2.0 * (sa[0] - sc[0]) / static_cast<double>(n) / log(2.0);
        out[0] = ldexp(1.0, static_cast<int>(round(l2)));
    }
}

// ------------------------------------------------------------------ normalisation
// q_i = P_i^{-d} sum_r K_ir, P_i = rho_i/2; stores qa_i = q_i^{-alpha} (Section 2.2)
__global__ __launch_bounds__(256) void k_qpass(const int32_t* __restrict__ idx, const float* __restrict__ d2,
                                               const int64_t* __restrict__ rowptr, int n, int k,
                                               const float* __restrict__ rho, double e,
                                               const double* __restrict__ e_dev, double alpha, double d,
                                               double* __restrict__ qa)
{
    if (e_dev) e = *e_dev;
    const int its = rowsum_its(n);
    const int base = (blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * 4 * its;
    if (base >= n) return;
    const double s = wave_row_sums(idx, d2, rowptr, n, k, rho, e, base, its);
    const int i = base + lane_id();
    if (lane_id() < 4 * its && i < n) {
        const double P = 0.5 * static_cast<double>(rho[i]);
        const double q = pow(P, -d) * s;
        qa[i] = pow(q, -alpha);
    }
}

// Ascending sort of one 32-bit key per lane across the wavefront: the bitonic
// network of bitonic_sort with one key per lane, each exchange a compare, a
// constant lane mask and a select.
__device__ __forceinline__ uint32_t wave_sort_u32(uint32_t v)
{
#pragma unroll
    for (int kb = 2; kb <= WAVE; kb <<= 1) {
#pragma unroll
        for (int j = kb >> 1; j > 0; j >>= 1) {
            const uint32_t o = xor_lane(v, j);
            const uint64_t up = kb < WAVE ? lanes_bit_clear(kb) : ~0ull;
            const uint64_t keep_min = ~(up ^ lanes_bit_clear(j));
            const uint64_t take = __ballot(o < v) ^ ~keep_min;
            v = __builtin_amdgcn_inverse_ballot_w64(take) ? o : v;
        }
    }
    return v;
}

// Kt_ir = K_ir qa_i qa_j (K_ir in float32 as in the row sums), D_i = sum_r Kt_ir
// (float64: each lane's terms compensated, the lanes added in a fixed xor
// butterfly), then the requested
// output kind, the row sorted by column. For KVB_OUT_SYMMETRIC this pass
// stores Kt and the finishing pass divides by S_i S_j.
template <int E>
__global__ __launch_bounds__(256) void k_assemble(const int32_t* __restrict__ idx, const float* __restrict__ d2,
                                                  int n, int k, const float* __restrict__ rho, double e,
                                                  const double* __restrict__ e_dev, const double* __restrict__ qa,
                                                  int out_kind,
                                                  int64_t* __restrict__ rowptr, int32_t* __restrict__ col,
                                                  float* __restrict__ val, double* __restrict__ Pout,
                                                  double* __restrict__ Dout, const int32_t* __restrict__ rowmap,
                                                  const int32_t* __restrict__ sid)
{
    if (e_dev) e = *e_dev;
    const int lane = lane_id();
    const int p = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (p >= n) return;
    // stored row p is output row i; with a row map (curve-ordered rows, see
    // k_curve_rows) idx holds curve positions for the gathers and sid the
    // sample ids of output row i, which are the columns
    const int i = rowmap ? rowmap[p] : p;
    const int32_t* irow = idx + static_cast<size_t>(p) * k;
    const int32_t* srow = rowmap ? sid + static_cast<size_t>(i) * k : irow;
    const float* drow = d2 + static_cast<size_t>(p) * k;
    const double ri = static_cast<double>(rho[p]);
    const double inv = 1.0 / (e * ri);
    const double qai = qa[p];
    double kt[E];
    int cj[E];
    Comp64 acc;
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int r = s * WAVE + lane;
        kt[s] = 0.0;
        cj[s] = -1;
        if (r < k) {
            const int j = irow[r];
            const double x = static_cast<double>(drow[r]) * inv / static_cast<double>(rho[j]);
            kt[s] = static_cast<double>(expf(-static_cast<float>(x))) * qai * qa[j];
            cj[s] = srow[r];
            acc.add(kt[s]);
        }
    }
    // the lanes' compensated sums of at most E terms, added in a fixed xor
    // butterfly (every lane ends with the same D_i; at most 64 E positive
    // float64 terms)
    double Di = acc.value();
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) Di += shfl_xor_f64(Di, o);
    const double Pi = 0.5 * ri;
    if (E == 1 && n < (1 << 26)) {
        // one entry per lane (k <= 64) and columns below 2^26: 32-bit keys
        // column << 6 | lane, sorted across the wavefront; each value is then
        // read from the lane its key names
        float v = 0.f;
        if (cj[0] >= 0) {
            double w;
            if (out_kind == KVB_OUT_MARKOV)
                w = kt[0] / Di;
            else if (out_kind == KVB_OUT_GENERATOR)
                w = (kt[0] / Di - (cj[0] == i ? 1.0 : 0.0)) / (e * Pi * Pi);
            else
                w = kt[0];
            v = static_cast<float>(w);
        }
        uint32_t key = cj[0] >= 0 ? ((static_cast<uint32_t>(cj[0]) << 6) | static_cast<uint32_t>(lane)) : ~0u;
        key = wave_sort_u32(key);
        const float vs = __uint_as_float(static_cast<uint32_t>(
            __shfl(static_cast<int>(__float_as_uint(v)), static_cast<int>(key & 63u), WAVE)));
        if (lane < k) {
            col[static_cast<size_t>(i) * k + lane] = static_cast<int32_t>(key >> 6);
            val[static_cast<size_t>(i) * k + lane] = vs;
        }
        if (lane == 0) {
            rowptr[i] = static_cast<int64_t>(i) * k;
            if (i == n - 1) rowptr[n] = static_cast<int64_t>(n) * k;
            if (Pout) Pout[i] = Pi;
            Dout[i] = Di;
        }
        return;
    }
    uint64_t key[E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
        float v = 0.f;
        if (cj[s] >= 0) {
            double w;
            if (out_kind == KVB_OUT_MARKOV)
                w = kt[s] / Di;
            else if (out_kind == KVB_OUT_GENERATOR)
                w = (kt[s] / Di - (cj[s] == i ? 1.0 : 0.0)) / (e * Pi * Pi);
            else
                w = kt[s];
            v = static_cast<float>(w);
        }
        // sort key: column in the high word, value bits ride along
        key[s] = cj[s] >= 0 ? ((static_cast<uint64_t>(static_cast<uint32_t>(cj[s])) << 32) | __float_as_uint(v))
                            : ~0ull;
    }
    bitonic_sort<E>(key);
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int r = s * WAVE + lane;
        if (r < k) {
            col[static_cast<size_t>(i) * k + r] = static_cast<int32_t>(key[s] >> 32);
            val[static_cast<size_t>(i) * k + r] = __uint_as_float(static_cast<uint32_t>(key[s]));
        }
    }
    if (lane == 0) {
        rowptr[i] = static_cast<int64_t>(i) * k;
        if (i == n - 1) rowptr[n] = static_cast<int64_t>(n) * k;
        if (Pout) Pout[i] = Pi;
        Dout[i] = Di;
    }
}

// Lhat_ir = (Kt_ir / (S_i S_j) - [j == i] / P_i^2) / e, S = P sqrt(D)
__global__ __launch_bounds__(256) void k_symmetric_finish(int64_t nnz, int k, const int32_t* __restrict__ col,
                                                          const float* __restrict__ rho, const double* __restrict__ D,
                                                          double e, const double* __restrict__ e_dev,
                                                          float* __restrict__ val)
{
    if (e_dev) e = *e_dev;
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const int64_t i = p / k;
    const int j = col[p];
    const double Pi = 0.5 * static_cast<double>(rho[i]), Pj = 0.5 * static_cast<double>(rho[j]);
    const double Si = Pi * sqrt(D[i]), Sj = Pj * sqrt(D[j]);
    const double w = (static_cast<double>(val[p]) / (Si * Sj) - (j == i ? 1.0 / (Pi * Pi) : 0.0)) / e;
    val[p] = static_cast<float>(w);
}

// The normalisation over a CSR pattern whose rows are already ordered by
// column: one wavefront per row of any length. Kt_ir is formed as in
// k_assemble (lanes strided over the row); D_i is a compensated float64 sum,
// the lanes' (sum, compensation) pairs combined in a fixed butterfly, since a
// row here may hold thousands of entries; the output value, written in place, takes Kt_ir from registers
// for a row's first 128 entries and forms it again, identically, beyond. For KVB_OUT_SYMMETRIC the value is Kt and
// k_symmetric_rows finishes it.
__global__ __launch_bounds__(256) void k_assemble_rows(const int64_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ col, const float* __restrict__ d2,
                                                       int n, const float* __restrict__ rho, double e,
                                                       const double* __restrict__ e_dev,
                                                       const double* __restrict__ qa, int out_kind,
                                                       float* __restrict__ val, double* __restrict__ Pout,
                                                       double* __restrict__ Dout)
{
    if (e_dev) e = *e_dev;
    const int lane = lane_id();
    const int i = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (i >= n) return;
    const int64_t rb = rowptr[i], re = rowptr[i + 1];
    const double ri = static_cast<double>(rho[i]);
    const double inv = 1.0 / (e * ri);
    const double qai = qa[i];
    // the row's first KEEP * 64 values stay in registers for the second sweep
    constexpr int KEEP = 2;
    double kv[KEEP];
    Comp64 acc;
    int s = 0;
    for (int64_t p = rb + lane; p < re; p += WAVE, ++s) {
        const int j = col[p];
        const double x = static_cast<double>(d2[p]) * inv / static_cast<double>(rho[j]);
        const double kt = static_cast<double>(expf(-static_cast<float>(x))) * qai * qa[j];
#pragma unroll
        for (int u = 0; u < KEEP; ++u)
            if (s == u) kv[u] = kt;
        acc.add(kt);
    }
    double Ds = acc.s, Dc = acc.c;
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        const double os = shfl_xor_f64(Ds, o), oc = shfl_xor_f64(Dc, o);
        const double t = Ds + os;
        Dc += oc + ((fabs(Ds) >= fabs(os)) ? ((Ds - t) + os) : ((os - t) + Ds));
        Ds = t;
    }
    const double Di = Ds + Dc;
    const double Pi = 0.5 * ri;
    s = 0;
    for (int64_t p = rb + lane; p < re; p += WAVE, ++s) {
        const int j = col[p];
        double kt = 0.0;
#pragma unroll
        for (int u = 0; u < KEEP; ++u)
            if (s == u) kt = kv[u];
        if (s >= KEEP) {
            const double x = static_cast<double>(d2[p]) * inv / static_cast<double>(rho[j]);
            kt = static_cast<double>(expf(-static_cast<float>(x))) * qai * qa[j];
        }
        double w;
        if (out_kind == KVB_OUT_MARKOV)
            w = kt / Di;
        else if (out_kind == KVB_OUT_GENERATOR)
            w = (kt / Di - (j == i ? 1.0 : 0.0)) / (e * Pi * Pi);
        else
            w = kt;
        val[p] = static_cast<float>(w);
    }
    if (lane == 0) {
        if (Pout) Pout[i] = Pi;
        Dout[i] = Di;
    }
}

// Lhat_ir = (Kt_ir / (S_i S_j) - [j == i] / P_i^2) / e over a CSR pattern
__global__ __launch_bounds__(256) void k_symmetric_rows(const int64_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col, int n,
                                                        const float* __restrict__ rho, const double* __restrict__ D,
                                                        double e, const double* __restrict__ e_dev,
                                                        float* __restrict__ val)
{
    if (e_dev) e = *e_dev;
    const int lane = lane_id();
    const int i = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (i >= n) return;
    const double Pi = 0.5 * static_cast<double>(rho[i]);
    const double Si = Pi * sqrt(D[i]);
    for (int64_t p = rowptr[i] + lane; p < rowptr[i + 1]; p += WAVE) {
        const int j = col[p];
        const double Pj = 0.5 * static_cast<double>(rho[j]);
        const double Sj = Pj * sqrt(D[j]);
        val[p] = static_cast<float>((static_cast<double>(val[p]) / (Si * Sj) - (j == i ? 1.0 / (Pi * Pi) : 0.0)) / e);
    }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_adhoc_bandwidth(const float* d2, int n, int k, int k0, float* b, hipStream_t st)
{
    hipLaunchKernelGGL(k_adhoc_bandwidth, dim3((n + 255) / 256), dim3(256), 0, st, d2, n, k, k0, b);
    return hipGetLastError();
}

hipError_t launch_density(const int32_t* idx, const float* d2, int n, int k, const float* b, double e,
                          const double* e_dev, double d, double beta, float* rho, float* psi, hipStream_t st)
{
    hipLaunchKernelGGL(k_density, dim3(rowsum_blocks(n)), dim3(256), 0, st, idx, d2, nullptr, n, k, b,
                       e, e_dev, d, beta, rho, psi);
    return hipGetLastError();
}

static int64_t chi_per_block(int64_t nnz)
{
    int64_t per = (nnz + CHI_MAX_BLOCKS - 1) / CHI_MAX_BLOCKS;
    per = (per + CHI_BLOCK - 1) / CHI_BLOCK * CHI_BLOCK;
    return per < CHI_MIN_ENTRIES_PER_BLOCK ? CHI_MIN_ENTRIES_PER_BLOCK : per;
}

int chi_num_blocks(int64_t nnz)
{
    const int64_t per = chi_per_block(nnz);
    return static_cast<int>((nnz + per - 1) / per);
}

hipError_t launch_chi(const int32_t* idx, const float* d2, const float* rho, int64_t nnz, int k, int G, double e_min,
                      double e_max, const double* scale_dev, double* partial, TuneResult* out, hipStream_t st)
{
    const int nb = chi_num_blocks(nnz);
    hipLaunchKernelGGL(k_chi_partial<false>, dim3(nb), dim3(CHI_BLOCK), 0, st, idx, d2, nullptr, nullptr, 0, rho, nnz,
                       k, G, e_min, e_max, scale_dev, chi_per_block(nnz), partial);
    hipLaunchKernelGGL(k_chi_reduce, dim3(G), dim3(256), 0, st, partial, nb, G, nullptr, 0, out);
    hipLaunchKernelGGL(k_chi_finish, dim3(1), dim3(256), 0, st, G, e_min, e_max, scale_dev, out);
    return hipGetLastError();
}

int logsum_num_blocks(int n) { return min(1024, (n + 255) / 256); }

hipError_t launch_grid_scale(const float* ref, const float* rho, int n, double* partial, double* out,
                             hipStream_t st)
{
    const int nb = logsum_num_blocks(n);
    hipLaunchKernelGGL(k_logsum_partial, dim3(nb), dim3(256), 0, st, ref, rho, n, partial);
    hipLaunchKernelGGL(k_logsum_finish, dim3(1), dim3(256), 0, st, partial, nb, n, out);
    return hipGetLastError();
}

hipError_t launch_qpass(const int32_t* idx, const float* d2, int n, int k, const float* rho, double e,
                        const double* e_dev, double alpha, double d, double* qa, hipStream_t st)
{
    hipLaunchKernelGGL(k_qpass, dim3(rowsum_blocks(n)), dim3(256), 0, st, idx, d2, nullptr, n, k, rho,
                       e, e_dev, alpha, d, qa);
    return hipGetLastError();
}

hipError_t launch_assemble(const int32_t* idx, const float* d2, int n, int k, const float* rho, double e,
                           const double* e_dev, const double* qa, int out_kind, int64_t* rowptr, int32_t* col, float* val,
                           double* P, double* D, hipStream_t st, const int32_t* rowmap, const int32_t* sid,
                           const float* rho_out)
{
    const dim3 grid((n + 3) / 4), block(256);
    if (k <= 64)
        hipLaunchKernelGGL((k_assemble<1>), grid, block, 0, st, idx, d2, n, k, rho, e, e_dev, qa, out_kind, rowptr, col,
                           val, P, D, rowmap, sid);
    else if (k <= 128)
        hipLaunchKernelGGL((k_assemble<2>), grid, block, 0, st, idx, d2, n, k, rho, e, e_dev, qa, out_kind, rowptr, col,
                           val, P, D, rowmap, sid);
    else
        hipLaunchKernelGGL((k_assemble<4>), grid, block, 0, st, idx, d2, n, k, rho, e, e_dev, qa, out_kind, rowptr, col,
                           val, P, D, rowmap, sid);
    if (out_kind == KVB_OUT_SYMMETRIC) {
        const int64_t nnz = static_cast<int64_t>(n) * k;
        hipLaunchKernelGGL(k_symmetric_finish, dim3(static_cast<unsigned>((nnz + 255) / 256)), dim3(256), 0, st,
                           nnz, k, col, rowmap ? rho_out : rho, D, e, e_dev, val);
    }
    return hipGetLastError();
}

hipError_t launch_curve_rows(const int32_t* idx, const float* d2, int n, int k, int k0, const int32_t* cid,
                             const int32_t* pos, int32_t* idx_c, float* d2_c, float* b_c, hipStream_t st)
{
    hipLaunchKernelGGL(k_curve_rows, dim3((n + 3) / 4), dim3(256), 0, st, idx, d2, n, k, k0, cid, pos, idx_c, d2_c,
                       b_c);
    return hipGetLastError();
}

hipError_t launch_gather_samples(const int32_t* pos, int n, const float* a_c, float* a, const float* b_c, float* b,
                                 const float* c_c, float* c, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_samples, dim3((n + 255) / 256), dim3(256), 0, st, pos, n, a_c, a, b_c, b, c_c, c);
    return hipGetLastError();
}

// ---- the same passes over a CSR pattern
hipError_t launch_density_csr(const int64_t* rowptr, const int32_t* col, const float* d2, int n, const float* b,
                              double e, const double* e_dev, double d, double beta, float* rho, float* psi,
                              hipStream_t st)
{
    hipLaunchKernelGGL(k_density, dim3(rowsum_blocks(n)), dim3(256), 0, st, col, d2, rowptr, n, 0, b,
                       e, e_dev, d, beta, rho, psi);
    return hipGetLastError();
}

int chi_csr_blocks(int64_t nnz_hint, int64_t nnz_cap)
{
    const int64_t per = chi_per_block(nnz_hint);
    return static_cast<int>((nnz_cap + per - 1) / per);
}

// rowid [nnz_cap] int32: each entry's row, filled by k_row_ids (every row's
// entries in [rowptr_i, rowptr_{i+1}))
__global__ __launch_bounds__(256) void k_row_ids(const int64_t* __restrict__ rowptr, int n, int32_t* __restrict__ rowid)
{
    const int lane = lane_id();
    const int i = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (i >= n) return;
    for (int64_t p = rowptr[i] + lane; p < rowptr[i + 1]; p += WAVE) rowid[p] = i;
}

hipError_t launch_row_ids(const int64_t* rowptr, int n, int32_t* rowid, hipStream_t st)
{
    hipLaunchKernelGGL(k_row_ids, dim3((n + 3) / 4), dim3(256), 0, st, rowptr, n, rowid);
    return hipGetLastError();
}

hipError_t launch_chi_csr(const int64_t* rowptr, const int32_t* rowid, const int32_t* col, const float* d2, int n,
                          int64_t nnz_hint, int64_t nnz_cap, const float* rho, int G, double e_min, double e_max,
                          const double* scale_dev, double* partial, TuneResult* out, hipStream_t st)
{
    // blocks sized for the expected count; enough of them for the largest
    const int nb = chi_csr_blocks(nnz_hint, nnz_cap);
    hipLaunchKernelGGL(k_chi_partial<true>, dim3(nb), dim3(CHI_BLOCK), 0, st, col, d2, rowptr, rowid, n, rho, nnz_cap,
                       0, G, e_min, e_max, scale_dev, chi_per_block(nnz_hint), partial);
    hipLaunchKernelGGL(k_chi_reduce, dim3(G), dim3(256), 0, st, partial, nb, G, rowptr + n, chi_per_block(nnz_hint),
                       out);
    hipLaunchKernelGGL(k_chi_finish, dim3(1), dim3(256), 0, st, G, e_min, e_max, scale_dev, out);
    return hipGetLastError();
}

hipError_t launch_qpass_csr(const int64_t* rowptr, const int32_t* col, const float* d2, int n, const float* rho,
                            double e, const double* e_dev, double alpha, double d, double* qa, hipStream_t st)
{
    hipLaunchKernelGGL(k_qpass, dim3(rowsum_blocks(n)), dim3(256), 0, st, col, d2, rowptr, n, 0, rho,
                       e, e_dev, alpha, d, qa);
    return hipGetLastError();
}

hipError_t launch_assemble_rows(const int64_t* rowptr, const int32_t* col, const float* d2, int n, const float* rho,
                                double e, const double* e_dev, const double* qa, int out_kind, float* val, double* P,
                                double* D, hipStream_t st)
{
    const dim3 grid((n + 3) / 4), block(256);
    hipLaunchKernelGGL(k_assemble_rows, grid, block, 0, st, rowptr, col, d2, n, rho, e, e_dev, qa, out_kind, val, P,
                       D);
    if (out_kind == KVB_OUT_SYMMETRIC)
        hipLaunchKernelGGL(k_symmetric_rows, grid, block, 0, st, rowptr, col, n, rho, D, e, e_dev, val);
    return hipGetLastError();
}

}  // namespace kvb
