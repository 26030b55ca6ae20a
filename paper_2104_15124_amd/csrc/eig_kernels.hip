// Leading eigenpairs of a symmetric CSR matrix (gfx950): Lanczos with full
// reorthogonalisation.
//
// The paper's use of the kernel matrix is spectral: the eigenpairs of the
// symmetric conjugate Lhat = e^{-1}(S^{-1} Kt S^{-1} - P^{-2}) (Section 2.2)
// approximate those of the Kolmogorov operator (Sections 2.2 and 5), and a
// sparse eigensolver is the most expensive step after the matrix itself
// (Section 4). Lhat is negative semi-definite; the wanted eigenvalues are the
// ones nearest zero, the top of its spectrum.
//
// Lanczos (Lanczos 1950; Golub and Van Loan, Section 10.1) builds an
// orthonormal basis v_0..v_{m-1} of the Krylov space of a seeded start vector
// with A v_j = beta_{j-1} v_{j-1} + alpha_j v_j + beta_j v_{j+1}. Rounding
// destroys the orthogonality as Ritz values converge, so every new vector is
// orthogonalised against all previous ones, twice (classical Gram-Schmidt
// repeated). The eigenpairs of the m x m tridiagonal T = tridiag(beta, alpha,
// beta) are the Ritz pairs; a Ritz vector is V s, its residual norm
// |beta_{m-1} s_{m-1}|. The small eigenproblem is solved on the host for the
// wanted pairs only: eigenvalues by bisection on the Sturm count, eigenvectors
// by inverse iteration (Golub and Van Loan, Sections 8.4 and 8.2).
//
// On the device: the matrix-vector product (one wavefront per row, FP64
// accumulation of float32 entries), the projections V^T w (one workgroup per
// basis vector and row chunk, then a fixed-order sum over the chunks), w -= V h (one thread per row), norms and Ritz vectors. Every reduction has a fixed order, so results are reproducible.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "kvb_ctx.h"
#include "kvb_device.h"

namespace kvb {

// y = A x, one wavefront per row, lanes strided over the row, butterfly sum
__global__ __launch_bounds__(256) void k_spmv(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                              const float* __restrict__ val, const double* __restrict__ x, int n,
                                              double* __restrict__ y)
{
    const int lane = lane_id();
    const int i = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (i >= n) return;
    double s = 0.0;
    for (int64_t p = rowptr[i] + lane; p < rowptr[i + 1]; p += WAVE)
        s += static_cast<double>(val[p]) * x[col[p]];
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) s += shfl_xor_f64(s, o);
    if (lane == 0) y[i] = s;
}

// h[c] = V[c] . w, one workgroup per column: the threads stride over the
// rows, then a fixed-order reduction (wavefront butterflies, then the four
// wavefronts in order)
__global__ __launch_bounds__(256) void k_project(const double* __restrict__ V, int64_t ldv,
                                                 const double* __restrict__ w, int n, double* __restrict__ h)
{
    __shared__ double red[4];
    const double* vc = V + static_cast<size_t>(blockIdx.x) * ldv;
    double s = 0.0;
    for (int r = threadIdx.x; r < n; r += 256) s += vc[r] * w[r];
    s = wave_sum_f64(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) h[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// part[s * ldp + c] = V[c][rows of chunk s] . w[same rows]: grid (ncol, chunks),
// so that a few columns still spread over the whole chip; the same fixed-order
// reduction within each workgroup as k_project
__global__ __launch_bounds__(256) void k_project_part(const double* __restrict__ V, int64_t ldv,
                                                      const double* __restrict__ w, int n, int chunk, int ldp,
                                                      double* __restrict__ part)
{
    __shared__ double red[4];
    const double* vc = V + static_cast<size_t>(blockIdx.x) * ldv;
    const int64_t r0 = static_cast<int64_t>(blockIdx.y) * chunk;
    const int64_t r1 = r0 + chunk < n ? r0 + chunk : n;
    double s = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) s += vc[r] * w[r];
    s = wave_sum_f64(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[static_cast<size_t>(blockIdx.y) * ldp + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// h[c] = sum over chunks s, in order, of part[s * ldp + c]
__global__ __launch_bounds__(256) void k_project_sum(const double* __restrict__ part, int ncol, int nchunk,
                                                     int ldp, double* __restrict__ h)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    double s = 0.0;
    for (int q = 0; q < nchunk; ++q) s += part[static_cast<size_t>(q) * ldp + c];
    h[c] = s;
}

// w[r] -= sum_c V[c][r] h[c]
__global__ __launch_bounds__(256) void k_subtract_span(const double* __restrict__ V, int64_t ldv, int ncol,
                                                       const double* __restrict__ h, int n, double* __restrict__ w)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double s = 0.0;
#pragma unroll 8
    for (int c = 0; c < ncol; ++c) s += V[static_cast<size_t>(c) * ldv + r] * h[c];
    w[r] -= s;
}

// out[r] = x[r] * scale
__global__ __launch_bounds__(256) void k_scale(const double* __restrict__ x, double scale, int n,
                                               double* __restrict__ out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) out[r] = x[r] * scale;
}

// ab[0] = h[0] on the first Gram-Schmidt pass, ab[0] += h[0] on the second
__global__ void k_alpha_add(const double* __restrict__ h, int first, double* __restrict__ ab)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) ab[0] = first ? h[0] : ab[0] + h[0];
}

// b = sqrt(nrm2[0]); out[r] = x[r] * (1 / b); the first thread stores b
__global__ __launch_bounds__(256) void k_scale_by_norm(const double* __restrict__ x, const double* __restrict__ nrm2,
                                                       int n, double* __restrict__ out, double* __restrict__ b)
{
    const double bj = sqrt(nrm2[0]);
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) b[0] = bj;
    if (r < n) out[r] = x[r] * (1.0 / bj);
}

// the seeded start vector: SplitMix64 (Steele, Lea and Flood 2014) of
// seed + r mapped to [-1, 1)
__global__ __launch_bounds__(256) void k_start_vector(uint64_t seed, int n, double* __restrict__ v)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (static_cast<uint64_t>(r) + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    v[r] = static_cast<double>(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Y[i][r] = sum_c V[c][r] S[c][i] (Ritz vectors), S column-major [m][nev] as S[c * nev + i]
__global__ __launch_bounds__(256) void k_ritz(const double* __restrict__ V, int64_t ldv, int m,
                                              const double* __restrict__ S, int nev, int n, double* __restrict__ Y)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    for (int i = 0; i < nev; ++i) {
        double s = 0.0;
        for (int c = 0; c < m; ++c) s += V[static_cast<size_t>(c) * ldv + r] * S[static_cast<size_t>(c) * nev + i];
        Y[static_cast<size_t>(i) * n + r] = s;
    }
}

// Spectral solution of the Kolmogorov problem (Section 3.1): with unit
// eigenvectors y_j of Lhat and S = P D^{1/2},
//   t = S g;  c_j = y_j . t;  f = S^{-1} sum_j y_j c_j / lambda_j;  g_l = S^{-1} sum_j y_j c_j.
__global__ __launch_bounds__(256) void k_weight(const double* __restrict__ P, const double* __restrict__ D,
                                                const double* __restrict__ g, int n, double* __restrict__ t)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) t[r] = P[r] * sqrt(D[r]) * g[r];
}

__global__ __launch_bounds__(256) void k_expand(const double* __restrict__ Y, int nvec, const double* __restrict__ cf,
                                                const double* __restrict__ cg, const double* __restrict__ P,
                                                const double* __restrict__ D, int n, double* __restrict__ f,
                                                double* __restrict__ gl)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double sf = 0.0, sg = 0.0;
    for (int j = 0; j < nvec; ++j) {
        const double y = Y[static_cast<size_t>(j) * n + r];
        sf += y * cf[j];
        sg += y * cg[j];
    }
    const double is = 1.0 / (P[r] * sqrt(D[r]));
    f[r] = sf * is;
    if (gl) gl[r] = sg * is;
}

// Carre du champ (Section 3.2): with p_j = y_j . S u and q_j = y_j . S v,
//   U = S^{-1} sum_j p_j y_j,  LU = S^{-1} sum_j lambda_j p_j y_j  (and V, LV from q),
//   t1 = S U V,  t2 = S (LU V + U LV).
__global__ __launch_bounds__(256) void k_cdc_products(const double* __restrict__ Y, int nvec,
                                                      const double* __restrict__ coef, const double* __restrict__ P,
                                                      const double* __restrict__ D, int n, double* __restrict__ t1,
                                                      double* __restrict__ t2)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    // coef: p, lambda p, q, lambda q (nvec each)
    double U = 0.0, LU = 0.0, V = 0.0, LV = 0.0;
    for (int j = 0; j < nvec; ++j) {
        const double y = Y[static_cast<size_t>(j) * n + r];
        U += coef[j] * y;
        LU += coef[nvec + j] * y;
        V += coef[2 * nvec + j] * y;
        LV += coef[3 * nvec + j] * y;
    }
    const double S = P[r] * sqrt(D[r]), is = 1.0 / S;
    U *= is;
    LU *= is;
    V *= is;
    LV *= is;
    t1[r] = S * U * V;
    t2[r] = S * (LU * V + U * LV);
}

// C[l][j][k] = <phi_l, phi_j phi_k>_S = sqrt(n) sum_r y_l y_j y_k / S_r for j <= k
// (one workgroup per pair (j, k), all l at once; the tensor is symmetric)
constexpr int CDC_MAX = 64;
__global__ __launch_bounds__(256) void k_cdc_tensor(const double* __restrict__ Y, int nvec,
                                                    const double* __restrict__ P, const double* __restrict__ D, int n,
                                                    const int* __restrict__ pair_j, const int* __restrict__ pair_k,
                                                    double* __restrict__ C)
{
    __shared__ double red[4][CDC_MAX];
    const int j = pair_j[blockIdx.x], k = pair_k[blockIdx.x];
    double acc[CDC_MAX];
#pragma unroll
    for (int l = 0; l < CDC_MAX; ++l) acc[l] = 0.0;
    for (int r = threadIdx.x; r < n; r += 256) {
        const double w = Y[static_cast<size_t>(j) * n + r] * Y[static_cast<size_t>(k) * n + r] / (P[r] * sqrt(D[r]));
#pragma unroll
        for (int l = 0; l < CDC_MAX; ++l)
            if (l < nvec) acc[l] += Y[static_cast<size_t>(l) * n + r] * w;
    }
    const double rn = sqrt(static_cast<double>(n));
#pragma unroll
    for (int l = 0; l < CDC_MAX; ++l) {
        const double s = wave_sum_f64(acc[l]);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][l] = s;
    }
    __syncthreads();
    // each sorted triple l <= j <= k is written, with its permutations, by the
    // one workgroup of the pair (j, k), so every entry has a single writer
    for (int l = threadIdx.x; l <= j; l += 256) {
        const double v = ((red[0][l] + red[1][l]) + (red[2][l] + red[3][l])) * rn;
        const size_t nv = static_cast<size_t>(nvec);
        C[(l * nv + j) * nv + k] = v;
        C[(l * nv + k) * nv + j] = v;
        C[(j * nv + l) * nv + k] = v;
        C[(j * nv + k) * nv + l] = v;
        C[(k * nv + l) * nv + j] = v;
        C[(k * nv + j) * nv + l] = v;
    }
}

// Particle update of the density-evolution example (Section 5.3, explicit
// step of the sample SDE): x' = x + dt (u - grad f) + sqrt(dt) sigma w, with
// x, x' [n, m] float32 row-major, u and w [n, m] float64 row-major (or null:
// zero), grad [m, n] float64 (one gradient component per row).
__global__ __launch_bounds__(256) void k_advect(const float* __restrict__ X, int n, int m,
                                                const double* __restrict__ u, const double* __restrict__ grad,
                                                const double* __restrict__ w, double dt, double sdt,
                                                float* __restrict__ Xo)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(n) * m) return;
    const int r = static_cast<int>(t / m), s = static_cast<int>(t - static_cast<int64_t>(r) * m);
    double v = -grad[static_cast<size_t>(s) * n + r];
    if (u) v += u[t];
    double x = static_cast<double>(X[t]) + dt * v;
    if (w) x += sdt * w[t];
    Xo[t] = static_cast<float>(x);
}

}  // namespace kvb

namespace {

// split of the Lanczos projections over rows: chunks of at least 8192 rows,
// at most 64 chunks
constexpr int PROJ_MIN_CHUNK = 8192;
constexpr int PROJ_MAX_CHUNKS = 64;

using namespace kvbh;

// Number of eigenvalues of the symmetric tridiagonal T = tridiag(b, a, b)
// below x: the negative pivots of the LDL^T factorisation of T - x I
// (Sylvester's law of inertia; the Sturm sequence count).
int count_below(const std::vector<double>& a, const std::vector<double>& b, int m, double x, double tiny)
{
    int c = 0;
    double q = a[0] - x;
    if (q == 0.0) q = -tiny;
    c += q < 0.0;
    for (int i = 1; i < m; ++i) {
        q = a[i] - x - b[i - 1] * b[i - 1] / q;
        if (q == 0.0) q = -tiny;
        c += q < 0.0;
    }
    return c;
}

// Solve (T - theta I) y = rhs in place: Gaussian elimination with partial
// pivoting on the tridiagonal band (row swaps fill one extra superdiagonal).
void shifted_solve(const std::vector<double>& a, const std::vector<double>& b, int m, double theta, double tiny,
                   std::vector<double>& y)
{
    std::vector<double> lo(m, 0.0), d(m), up(m, 0.0), up2(m, 0.0);
    std::vector<char> swapped(m, 0);
    for (int i = 0; i < m; ++i) d[i] = a[i] - theta;
    for (int i = 0; i + 1 < m; ++i) {
        lo[i] = b[i];
        up[i] = b[i];
    }
    for (int i = 0; i + 1 < m; ++i) {
        if (std::fabs(d[i]) >= std::fabs(lo[i])) {
            if (d[i] == 0.0) d[i] = tiny;
            const double f = lo[i] / d[i];
            lo[i] = f;
            d[i + 1] -= f * up[i];
        } else {
            // rows i and i + 1 trade places; row i + 1's entries move up
            const double f = d[i] / lo[i];
            d[i] = lo[i];
            lo[i] = f;
            const double u = up[i];
            up[i] = d[i + 1];
            d[i + 1] = u - f * d[i + 1];
            if (i + 2 < m) {
                up2[i] = up[i + 1];
                up[i + 1] = -f * up[i + 1];
            }
            swapped[i] = 1;
        }
    }
    if (d[m - 1] == 0.0) d[m - 1] = tiny;
    for (int i = 0; i + 1 < m; ++i) {
        if (swapped[i]) {
            const double t = y[i];
            y[i] = y[i + 1];
            y[i + 1] = t - lo[i] * y[i + 1];
        } else {
            y[i + 1] -= lo[i] * y[i];
        }
    }
    y[m - 1] /= d[m - 1];
    if (m > 1) y[m - 2] = (y[m - 2] - up[m - 2] * y[m - 1]) / d[m - 2];
    for (int i = m - 3; i >= 0; --i) y[i] = (y[i] - up[i] * y[i + 1] - up2[i] * y[i + 2]) / d[i];
}

// The nev largest eigenpairs of T (descending): each eigenvalue by bisection
// on the Sturm count to the resolution of double precision, its eigenvector
// by inverse iteration (three solves with T - theta I), orthogonalised against
// the vectors of nearby eigenvalues already found.
void top_eigenpairs(const std::vector<double>& a, const std::vector<double>& b, int m, int nev,
                    std::vector<double>& theta, std::vector<double>& Y)
{
    double lo = a[0], hi = a[0], norm = 0.0;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
        norm = std::max(norm, std::fabs(a[i]) + r);
    }
    const double tiny = 1e-300 + 2.2e-16 * norm;
    theta.assign(nev, 0.0);
    Y.assign(size_t(nev) * m, 0.0);
    for (int q = 0; q < nev; ++q) {
        const int idx = m - 1 - q;   // ascending rank of the wanted eigenvalue
        double l = lo, h = hi;
        for (int it = 0; it < 2000 && h - l > 4.4e-16 * std::max(std::fabs(l), std::fabs(h)) + 1e-300; ++it) {
            const double mid = 0.5 * (l + h);
            if (mid <= l || mid >= h) break;
            if (count_below(a, b, m, mid, tiny) > idx)
                h = mid;
            else
                l = mid;
        }
        theta[q] = 0.5 * (l + h);
        std::vector<double> y(m);
        double y0 = 0.0;
        for (int i = 0; i < m; ++i) {
            y[i] = 1.0 + 0.01 * std::sin(1.0 + 7.0 * i + 3.0 * q);
            y0 += y[i] * y[i];
        }
        y0 = std::sqrt(y0);
        for (int i = 0; i < m; ++i) y[i] /= y0;
        for (int it = 0; it < 3; ++it) {
            const std::vector<double> prev = y;
            shifted_solve(a, b, m, theta[q], tiny, y);
            for (int p = 0; p < q; ++p) {
                if (std::fabs(theta[p] - theta[q]) > 1e-3 * norm) continue;
                double dot = 0.0;
                for (int i = 0; i < m; ++i) dot += Y[size_t(p) * m + i] * y[i];
                for (int i = 0; i < m; ++i) y[i] -= dot * Y[size_t(p) * m + i];
            }
            // normalise after scaling by the largest entry: a pivot at the
            // floor (T - theta I exactly singular, as for T = 0) makes the
            // entries as large as 1/tiny, whose squares would overflow
            double amax = 0.0;
            for (int i = 0; i < m; ++i) amax = std::max(amax, std::fabs(y[i]));
            if (!(amax > 0.0) || !std::isfinite(amax)) {
                y = prev;   // keep the last unit iterate
                break;
            }
            double nrm = 0.0;
            for (int i = 0; i < m; ++i) {
                y[i] /= amax;
                nrm += y[i] * y[i];
            }
            nrm = std::sqrt(nrm);
            for (int i = 0; i < m; ++i) y[i] /= nrm;
        }
        for (int i = 0; i < m; ++i) Y[size_t(q) * m + i] = y[i];
    }
}

}  // namespace

extern "C" {

int kvb_lanczos_prefix(const double* alpha_host, const double* beta_host, int32_t ncv, int32_t* m_host)
{
    if (!alpha_host || !beta_host || !m_host || ncv < 1) return KVB_E_INVALID;
    // the steps up to the first breakdown (beta_j = 0 up to underflow: an
    // invariant subspace) or all ncv of them; every coefficient used must be
    // finite, and a NaN beta is not a breakdown
    int32_t m = 0;
    for (int32_t j = 0; j < ncv; ++j) {
        const double a = alpha_host[j], b = beta_host[j];
        *m_host = m;
        if (!std::isfinite(a) || !std::isfinite(b) || b < 0.0) return KVB_E_INVALID;
        m = j + 1;
        if (b <= 1e-300) break;
    }
    *m_host = m;
    return KVB_OK;
}

int kvb_eigsh(kvb_ctx ctx, const int64_t* rowptr, const int32_t* col, const float* val, int64_t n, int64_t nnz,
              int32_t nev, int32_t ncv, double tol, uint64_t seed, double* evals_host, double* resid_host,
              double* evecs)
{
    if (!ctx) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31)");
    KVB_REQUIRE(ctx, nev >= 1 && ncv >= nev && ncv <= 4096 && ncv <= n, "need 1 <= nev <= ncv <= min(4096, n)");
    KVB_REQUIRE(ctx, tol > 0 && std::isfinite(tol), "tol must be finite and > 0");
    KVB_REQUIRE(ctx, aligned(val), "val must be a non-null float32 device pointer");
    KVB_REQUIRE(ctx, evals_host != nullptr, "evals_host must be non-null");
    KVB_REQUIRE(ctx, evecs == nullptr || aligned(evecs), "evecs must be aligned");
    KVB_TRY(check_pattern(ctx, rowptr, col, n, nnz));
    const int nn = static_cast<int>(n);
    const int64_t ldv = (n + 63) / 64 * 64;
    const size_t need = round256(size_t(ncv + 1) * ldv * sizeof(double)) + round256(size_t(ldv) * sizeof(double)) +
                        2 * round256(size_t(ncv + 1) * sizeof(double)) +
                        round256(size_t(ncv) * nev * sizeof(double)) +
                        round256(size_t(PROJ_MAX_CHUNKS) * (ncv + 1) * sizeof(double)) +
                        round256(2 * size_t(ncv) * sizeof(double)) + 2048;
    int rc = ensure_scratch(ctx, need);
    if (rc) return rc;
    Carve cv(ctx->scratch);
    double* V = cv.take<double>(size_t(ncv + 1) * ldv);
    double* w = cv.take<double>(ldv);
    double* h = cv.take<double>(ncv + 1);
    double* hsum = cv.take<double>(ncv + 1);
    double* S = cv.take<double>(size_t(ncv) * nev);
    const int ldp = ncv + 1;
    double* part = cv.take<double>(size_t(PROJ_MAX_CHUNKS) * ldp);
    hipStream_t st = ctx->stream;
    const dim3 blk(256), rows_grid((nn + 255) / 256), spmv_grid((nn + 3) / 4);
    double* ab = cv.take<double>(2 * size_t(ncv));   // alpha_0..alpha_{ncv-1}, then beta_0..beta_{ncv-1}
    // row chunks of the projections: at least PROJ_MIN_CHUNK rows, a multiple
    // of 256, at most PROJ_MAX_CHUNKS of them
    int chunk = std::max(PROJ_MIN_CHUNK, (nn + PROJ_MAX_CHUNKS - 1) / PROJ_MAX_CHUNKS);
    chunk = (chunk + 255) / 256 * 256;
    const int nchunk = (nn + chunk - 1) / chunk;

    // hd[0..ncol) = B[:, :ncol]^T x on the device, B's columns ldv apart
    auto project_cols = [&](const double* B, const double* x, int ncol, double* hd) -> hipError_t {
        hipLaunchKernelGGL(kvb::k_project_part, dim3(ncol, nchunk), blk, 0, st, B, ldv, x, nn, chunk, ldp, part);
        hipLaunchKernelGGL(kvb::k_project_sum, dim3((ncol + 255) / 256), blk, 0, st, part, ncol, nchunk, ldp, hd);
        return hipGetLastError();
    };
    auto project = [&](const double* x, int ncol, double* hd) -> hipError_t {
        return project_cols(V, x, ncol, hd);
    };
    // ||x||
    auto norm = [&](double* x, double* out) -> int {
        KVB_HIP(ctx, project_cols(x, x, 1, h));
        KVB_HIP(ctx, hipMemcpyAsync(out, h, sizeof(double), hipMemcpyDeviceToHost, st));
        KVB_HIP(ctx, hipStreamSynchronize(st));
        *out = std::sqrt(*out);
        return KVB_OK;
    };

    hipLaunchKernelGGL(kvb::k_start_vector, rows_grid, blk, 0, st, seed, nn, w);
    double b0 = 0.0;
    KVB_TRY(norm(w, &b0));
    KVB_REQUIRE(ctx, b0 > 0, "start vector vanished");
    hipLaunchKernelGGL(kvb::k_scale, rows_grid, blk, 0, st, w, 1.0 / b0, nn, V);
    // The steps run without a host round trip: alpha_j and beta_j stay on the
    // device until the end. A breakdown (beta_j = 0, an invariant subspace)
    // is found afterwards; the steps after it hold non-finite values that no
    // Ritz vector uses.
    double* alpha_d = ab;
    double* beta_d = ab + ncv;
    for (int j = 0; j < ncv; ++j) {
        double* vj = V + size_t(j) * ldv;
        hipLaunchKernelGGL(kvb::k_spmv, spmv_grid, blk, 0, st, rowptr, col, val, vj, nn, w);
        // two passes of classical Gram-Schmidt against v_0..v_j; alpha_j is
        // the first pass's coefficient on v_j plus the second's correction
        for (int pass = 0; pass < 2; ++pass) {
            KVB_HIP(ctx, project(w, j + 1, hsum));
            hipLaunchKernelGGL(kvb::k_subtract_span, rows_grid, blk, 0, st, V, ldv, j + 1, hsum, nn, w);
            hipLaunchKernelGGL(kvb::k_alpha_add, dim3(1), dim3(64), 0, st, hsum + j, pass == 0 ? 1 : 0,
                               alpha_d + j);
        }
        // beta_j = ||w||, v_{j+1} = w / beta_j (V has room for v_ncv)
        KVB_HIP(ctx, project_cols(w, w, 1, h));
        hipLaunchKernelGGL(kvb::k_scale_by_norm, rows_grid, blk, 0, st, w, h, nn, V + size_t(j + 1) * ldv,
                           beta_d + j);
        KVB_HIP(ctx, hipGetLastError());
    }
    std::vector<double> abh(2 * size_t(ncv));
    KVB_HIP(ctx, hipMemcpyAsync(abh.data(), ab, sizeof(double) * abh.size(), hipMemcpyDeviceToHost, st));
    KVB_HIP(ctx, hipStreamSynchronize(st));
    int m = 0;
    if (kvb_lanczos_prefix(abh.data(), abh.data() + ncv, ncv, &m) != KVB_OK)
        return fail(ctx, KVB_E_INVALID, "non-finite Lanczos coefficient after %d steps: the matrix or the "
                    "start vector holds non-finite values", m);
    std::vector<double> alpha(abh.begin(), abh.begin() + m);
    std::vector<double> beta(abh.begin() + ncv, abh.begin() + ncv + m);
    if (m < ncv) beta[size_t(m) - 1] = 0.0;   // invariant subspace found: the Ritz pairs are exact
    KVB_REQUIRE(ctx, nev <= m, "the Krylov space closed after %d steps, below nev = %d", m, nev);
    // Ritz pairs of T
    std::vector<double> theta, Yt;
    top_eigenpairs(alpha, beta, m, nev, theta, Yt);
    double scale = 0.0;
    for (int i = 0; i < m; ++i)
        scale = std::max(scale, std::fabs(alpha[i]) + (i > 0 ? std::fabs(beta[i - 1]) : 0.0) +
                                    (i + 1 < m ? std::fabs(beta[i]) : 0.0));
    bool converged = true;
    std::vector<double> Ssel(size_t(m) * nev);
    for (int q = 0; q < nev; ++q) {
        evals_host[q] = theta[q];
        const double res = std::fabs(beta[m - 1] * Yt[size_t(q) * m + m - 1]);
        if (resid_host) resid_host[q] = res;
        if (res > tol * scale) converged = false;
        for (int c = 0; c < m; ++c) Ssel[size_t(c) * nev + q] = Yt[size_t(q) * m + c];
    }
    if (evecs) {
        KVB_HIP(ctx, hipMemcpyAsync(S, Ssel.data(), sizeof(double) * Ssel.size(), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(kvb::k_ritz, rows_grid, blk, 0, st, V, ldv, m, S, nev, nn, evecs);
        KVB_HIP(ctx, hipGetLastError());
        KVB_HIP(ctx, hipStreamSynchronize(st));
    }
    return converged ? KVB_OK : KVB_W_NOT_CONVERGED;
}

int kvb_kolmogorov_solve(kvb_ctx ctx, const double* evecs, const double* evals_host, int32_t nvec, int32_t skip,
                         const double* P, const double* D, const double* g, int64_t n, double* f, double* g_proj,
                         double* coef_host)
{
    if (!ctx) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31)");
    KVB_REQUIRE(ctx, nvec >= 1 && skip >= 0 && skip < nvec && nvec <= 1024, "need 0 <= skip < nvec <= 1024");
    KVB_REQUIRE(ctx, evals_host != nullptr, "evals_host must be non-null");
    KVB_REQUIRE(ctx, aligned(evecs) && aligned(P) && aligned(D) && aligned(g) && aligned(f),
                "evecs, P, D, g, f must be non-null float64 device pointers");
    KVB_REQUIRE(ctx, g_proj == nullptr || aligned(g_proj), "g_proj must be aligned");
    const int l = nvec - skip;
    for (int j = skip; j < nvec; ++j)
        KVB_REQUIRE(ctx, evals_host[j] != 0.0 && std::isfinite(evals_host[j]),
                    "eigenvalue %d is zero or not finite: skip the null pairs", j);
    const int nn = static_cast<int>(n);
    int rc = ensure_scratch(ctx, round256(size_t(nn) * sizeof(double)) + 3 * round256(size_t(l) * sizeof(double)) + 1024);
    if (rc) return rc;
    Carve cv(ctx->scratch);
    double* t = cv.take<double>(nn);
    double* c = cv.take<double>(l);
    double* cf = cv.take<double>(l);
    double* cg = cv.take<double>(l);
    hipStream_t st = ctx->stream;
    const double* Y = evecs + size_t(skip) * nn;
    const dim3 blk(256), rows_grid((nn + 255) / 256);
    hipLaunchKernelGGL(kvb::k_weight, rows_grid, blk, 0, st, P, D, g, nn, t);
    hipLaunchKernelGGL(kvb::k_project, dim3(l), blk, 0, st, Y, static_cast<int64_t>(nn), t, nn, c);
    KVB_HIP(ctx, hipGetLastError());
    std::vector<double> ch(l), fh(l);
    KVB_HIP(ctx, hipMemcpyAsync(ch.data(), c, sizeof(double) * l, hipMemcpyDeviceToHost, st));
    KVB_HIP(ctx, hipStreamSynchronize(st));
    for (int j = 0; j < l; ++j) fh[j] = ch[j] / evals_host[skip + j];
    KVB_HIP(ctx, hipMemcpyAsync(cf, fh.data(), sizeof(double) * l, hipMemcpyHostToDevice, st));
    KVB_HIP(ctx, hipMemcpyAsync(cg, ch.data(), sizeof(double) * l, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(kvb::k_expand, rows_grid, blk, 0, st, Y, l, cf, cg, P, D, nn, f, g_proj);
    KVB_HIP(ctx, hipGetLastError());
    KVB_HIP(ctx, hipStreamSynchronize(st));
    if (coef_host) {
        // the paper's coefficients g~_j = <phi_j, g>_S with <phi_i, phi_j>_S = delta_ij, phi_j = sqrt(n) S^{-1} y_j
        const double rn = 1.0 / std::sqrt(static_cast<double>(n));
        for (int j = 0; j < l; ++j) coef_host[j] = ch[j] * rn;
    }
    return KVB_OK;
}

int kvb_carre_du_champ(kvb_ctx ctx, const double* evecs, const double* evals_host, int32_t nvec, const double* P,
                       const double* D, const double* u, const double* v, int64_t n, double* grad, double* C)
{
    if (!ctx) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31)");
    KVB_REQUIRE(ctx, nvec >= 1 && nvec <= 1024, "need 1 <= nvec <= 1024");
    KVB_REQUIRE(ctx, C == nullptr || nvec <= kvb::CDC_MAX, "the coefficient tensor needs nvec <= %d", kvb::CDC_MAX);
    KVB_REQUIRE(ctx, evals_host != nullptr, "evals_host must be non-null");
    KVB_REQUIRE(ctx, aligned(evecs) && aligned(P) && aligned(D) && aligned(u) && aligned(v) && aligned(grad),
                "evecs, P, D, u, v, grad must be non-null float64 device pointers");
    KVB_REQUIRE(ctx, C == nullptr || aligned(C), "C must be aligned");
    const int nn = static_cast<int>(n);
    const int npairs = nvec * (nvec + 1) / 2;
    int rc = ensure_scratch(ctx, 4 * round256(size_t(nn) * sizeof(double)) + 6 * round256(size_t(nvec) * sizeof(double)) +
                                     2 * round256(size_t(npairs) * sizeof(int)) + 2048);
    if (rc) return rc;
    Carve cv(ctx->scratch);
    double* su = cv.take<double>(nn);
    double* sv = cv.take<double>(nn);
    double* t1 = cv.take<double>(nn);
    double* t2 = cv.take<double>(nn);
    double* pq = cv.take<double>(2 * size_t(nvec));
    double* coef = cv.take<double>(4 * size_t(nvec));
    double* ab = cv.take<double>(2 * size_t(nvec));
    int* pj = cv.take<int>(npairs);
    int* pk = cv.take<int>(npairs);
    hipStream_t st = ctx->stream;
    const dim3 blk(256), rows_grid((nn + 255) / 256);
    hipLaunchKernelGGL(kvb::k_weight, rows_grid, blk, 0, st, P, D, u, nn, su);
    hipLaunchKernelGGL(kvb::k_weight, rows_grid, blk, 0, st, P, D, v, nn, sv);
    hipLaunchKernelGGL(kvb::k_project, dim3(nvec), blk, 0, st, evecs, static_cast<int64_t>(nn), su, nn, pq);
    hipLaunchKernelGGL(kvb::k_project, dim3(nvec), blk, 0, st, evecs, static_cast<int64_t>(nn), sv, nn, pq + nvec);
    KVB_HIP(ctx, hipGetLastError());
    std::vector<double> h(2 * size_t(nvec)), c4(4 * size_t(nvec));
    KVB_HIP(ctx, hipMemcpyAsync(h.data(), pq, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
    KVB_HIP(ctx, hipStreamSynchronize(st));
    for (int j = 0; j < nvec; ++j) {
        c4[j] = h[j];
        c4[nvec + j] = evals_host[j] * h[j];
        c4[2 * nvec + j] = h[nvec + j];
        c4[3 * nvec + j] = evals_host[j] * h[nvec + j];
    }
    KVB_HIP(ctx, hipMemcpyAsync(coef, c4.data(), sizeof(double) * c4.size(), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(kvb::k_cdc_products, rows_grid, blk, 0, st, evecs, nvec, coef, P, D, nn, t1, t2);
    hipLaunchKernelGGL(kvb::k_project, dim3(nvec), blk, 0, st, evecs, static_cast<int64_t>(nn), t1, nn, ab);
    hipLaunchKernelGGL(kvb::k_project, dim3(nvec), blk, 0, st, evecs, static_cast<int64_t>(nn), t2, nn, ab + nvec);
    KVB_HIP(ctx, hipGetLastError());
    KVB_HIP(ctx, hipMemcpyAsync(h.data(), ab, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
    KVB_HIP(ctx, hipStreamSynchronize(st));
    // expansion coefficient of phi_l in grad u . grad v, in the y basis: (lambda_l a_l - b_l) / 2
    for (int l = 0; l < nvec; ++l) c4[l] = 0.5 * (evals_host[l] * h[l] - h[nvec + l]);
    KVB_HIP(ctx, hipMemcpyAsync(coef, c4.data(), sizeof(double) * nvec, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(kvb::k_expand, rows_grid, blk, 0, st, evecs, nvec, coef, coef, P, D, nn, grad,
                       static_cast<double*>(nullptr));
    KVB_HIP(ctx, hipGetLastError());
    if (C) {
        std::vector<int> hj(npairs), hk(npairs);
        int q = 0;
        for (int j = 0; j < nvec; ++j)
            for (int k = j; k < nvec; ++k) {
                hj[q] = j;
                hk[q] = k;
                ++q;
            }
        KVB_HIP(ctx, hipMemcpyAsync(pj, hj.data(), sizeof(int) * npairs, hipMemcpyHostToDevice, st));
        KVB_HIP(ctx, hipMemcpyAsync(pk, hk.data(), sizeof(int) * npairs, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(kvb::k_cdc_tensor, dim3(npairs), blk, 0, st, evecs, nvec, P, D, nn, pj, pk, C);
        KVB_HIP(ctx, hipGetLastError());
    }
    KVB_HIP(ctx, hipStreamSynchronize(st));
    return KVB_OK;
}

int kvb_advect(kvb_ctx ctx, const float* X, int64_t n, int32_t m, const double* velocity, const double* grad,
               const double* noise, double dt, double sigma, float* X_out)
{
    if (!ctx) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, n >= 1 && n < (int64_t(1) << 31) && m >= 1 && n * m < (int64_t(1) << 40), "bad n or m");
    KVB_REQUIRE(ctx, std::isfinite(dt) && dt >= 0 && std::isfinite(sigma), "dt must be finite and >= 0, sigma finite");
    KVB_REQUIRE(ctx, aligned(X) && aligned(grad) && aligned(X_out), "X, grad, X_out must be non-null device pointers");
    KVB_REQUIRE(ctx, (velocity == nullptr || aligned(velocity)) && (noise == nullptr || aligned(noise)),
                "velocity and noise must be aligned");
    const int64_t total = n * m;
    hipLaunchKernelGGL(kvb::k_advect, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, ctx->stream, X,
                       static_cast<int>(n), m, velocity, grad, noise, dt, std::sqrt(dt) * sigma, X_out);
    KVB_HIP(ctx, hipGetLastError());
    return KVB_OK;
}

}  // extern "C"
