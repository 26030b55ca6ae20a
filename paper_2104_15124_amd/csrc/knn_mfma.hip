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
// v_mfma_f32_32x32x2_f32, FP32 accumulation). A workgroup of four wavefronts
// stages 32 or 64 candidates at a time in LDS with asynchronous global->LDS
// loads (double-buffered, so the next stage streams in while the current one
// is consumed); every wavefront keeps its query fragments in registers. Scores at or below a query's threshold are appended
// to that query's 64-entry LDS buffer; a buffer past half full is merged into
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
#include "kvb_device.h"
#include "kvb_kernels.h"

namespace kvb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ------------------------------------------------------------------ prep
// Column sums (float64) over blocks of rows, then the fixed-order mean.
__global__ __launch_bounds__(256) void k_colsum_partial(const float* __restrict__ X, int n, int m, int rows_per_block,
                                                        double* __restrict__ part)
{
    const int r0 = blockIdx.x * rows_per_block;
    const int r1 = min(n, r0 + rows_per_block);
    for (int c = threadIdx.x; c < m; c += blockDim.x) {
        double s = 0.0;
        for (int r = r0; r < r1; ++r) s += static_cast<double>(X[static_cast<size_t>(r) * m + c]);
        part[static_cast<size_t>(blockIdx.x) * m + c] = s;
    }
}

__global__ __launch_bounds__(256) void k_colsum_finish(const double* __restrict__ part, int nb, int m, int n,
                                                       double* __restrict__ mu)
{
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
// Rows n..npad-1 pad the last 32-row tile with zeros.
__global__ __launch_bounds__(256) void k_prep_rows(const float* __restrict__ X, int n, int npad, int m,
                                                   const double* __restrict__ mu, int split, int kpad,
                                                   void* __restrict__ Aq, void* __restrict__ Bc,
                                                   float* __restrict__ ynorm2, unsigned* __restrict__ rmax_bits)
{
    const int lane = lane_id();
    const int i = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (i >= npad) return;
    const bool real = i < n;
    const float* x = X + static_cast<size_t>(real ? i : 0) * m;
    double nrm = 0.0;
    if (split == 0) {
        constexpr int KS = 2, VE = 1;
        float* A = static_cast<float*>(Aq) + static_cast<size_t>(i) * kpad;
        float* B = static_cast<float*>(Bc);
        for (int c = lane; c < m; c += WAVE) {
            const float y = real ? static_cast<float>(static_cast<double>(x[c]) - mu[c]) : 0.0f;
            nrm += static_cast<double>(y) * static_cast<double>(y);
            if (real) A[c] = -2.0f * y;
            B[bpos(i, c, kpad, KS, VE)] = y;
        }
        nrm = wave_sum_f64(nrm);
        for (int c = m + lane; c < kpad; c += WAVE) {
            if (real) A[c] = (c == m) ? 1.0f : 0.0f;
            B[bpos(i, c, kpad, KS, VE)] = (c == m) ? static_cast<float>(nrm) : 0.0f;
        }
    } else {
        constexpr int KS = 16, VE = 8;
        uint16_t* A = static_cast<uint16_t*>(Aq) + static_cast<size_t>(i) * kpad;
        uint16_t* B = static_cast<uint16_t*>(Bc);
        for (int c = lane; c < m; c += WAVE) {
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
                B[bpos(i, t * m + c, kpad, KS, VE)] = b[t];
            }
        }
        nrm = wave_sum_f64(nrm);
        const int P = split;
        const uint16_t n1 = f32_to_bf16_rne(static_cast<float>(nrm));
        const double r1 = nrm - static_cast<double>(bf16_to_f32(n1));
        const uint16_t n2 = f32_to_bf16_rne(static_cast<float>(r1));
        const double r2 = r1 - static_cast<double>(bf16_to_f32(n2));
        const uint16_t n3 = f32_to_bf16_rne(static_cast<float>(r2));
        const uint16_t one = f32_to_bf16_rne(1.0f);
        for (int c = P * m + lane; c < kpad; c += WAVE) {
            const int t = c - P * m;
            if (real) A[c] = t < 3 ? one : static_cast<uint16_t>(0);
            B[bpos(i, c, kpad, KS, VE)] = t == 0 ? n1 : t == 1 ? n2 : t == 2 ? n3 : static_cast<uint16_t>(0);
        }
    }
    if (real && lane == 0) {
        ynorm2[i] = static_cast<float>(nrm);
        atomicMax(rmax_bits, __float_as_uint(static_cast<float>(sqrt(nrm) * (1.0 + 1e-6))));
    }
}

// ------------------------------------------------------------------ select
struct TraitsBF16 {
    using elem = uint16_t;
    using frag = bf16x8;
    static constexpr int KSTEP = 16;   // K per MFMA
    static constexpr int VEC = 8;      // K elements per lane per MFMA
    __device__ static __forceinline__ f32x16 mma(frag a, frag b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ frag load(const elem* p) { return *reinterpret_cast<const frag*>(p); }
    // each lane copies one 16-byte fragment; LDS destination = base + lane * 16
    __device__ static __forceinline__ void async_copy(const elem* g, frag* lds_base)
    {
        __builtin_amdgcn_global_load_lds((const void*)g, (__attribute__((address_space(3))) void*)lds_base, 16, 0, 0);
    }
};

struct TraitsF32 {
    using elem = float;
    using frag = float;
    static constexpr int KSTEP = 2;
    static constexpr int VEC = 1;
    __device__ static __forceinline__ f32x16 mma(frag a, frag b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ frag load(const elem* p) { return *p; }
    // each lane copies one 4-byte fragment; LDS destination = base + lane * 4
    __device__ static __forceinline__ void async_copy(const elem* g, frag* lds_base)
    {
        __builtin_amdgcn_global_load_lds((const void*)g, (__attribute__((address_space(3))) void*)lds_base, 4, 0, 0);
    }
};

constexpr int SEL_WAVES = 4;
constexpr int SEL_BUF = 64;   // per-query LDS buffer entries

// Output row (query) of accumulator register r in lane half h of a 32x32 tile.
__host__ __device__ constexpr int acc_row(int r, int h) { return 8 * (r / 4) + 4 * h + (r % 4); }

template <class Tr, int KS, int QT, int TW, int E>
__global__ __launch_bounds__(256) void k_select_mfma(const typename Tr::elem* __restrict__ Aq,
                                                     const typename Tr::elem* __restrict__ Bc, int n, int kp,
                                                     const float* __restrict__ ynorm2,
                                                     const unsigned* __restrict__ rmax_bits, ErrModel em,
                                                     uint64_t* __restrict__ lists, float* __restrict__ lb_out)
{
    using elem = typename Tr::elem;
    using frag = typename Tr::frag;
    constexpr int CAP = WAVE * E;
    constexpr int KSMAX = KS;
    constexpr int kpad = KS * Tr::KSTEP;        // padded contraction length
    constexpr int ks = KS;
    constexpr int NQ = 32 * QT;                 // queries per wavefront
    constexpr int NSUB = TW / 32;               // 32-candidate sub-tiles per stage
    // candidate tiles, fragment-major: [stage][sub][k-step][half][row] so that
    // lane l reads consecutive fragments (no bank conflicts); two stages
    // alternate between async global->LDS loads and MFMA consumption
    __shared__ frag s_tile[2][NSUB][KSMAX][2][32];
    __shared__ uint64_t s_buf[SEL_WAVES][NQ][SEL_BUF];
    __shared__ int s_cnt[SEL_WAVES][NQ];

    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int half = lane >> 5;
    const int q0 = (blockIdx.x * SEL_WAVES + wave) * NQ;

    frag qa[QT][KSMAX];
#pragma unroll
    for (int qt = 0; qt < QT; ++qt) {
        const int row = min(q0 + qt * 32 + (lane & 31), n - 1);
        const elem* src = Aq + static_cast<size_t>(row) * kpad + half * Tr::VEC;
#pragma unroll
        for (int s = 0; s < KS; ++s) qa[qt][s] = Tr::load(src + s * Tr::KSTEP);
    }
    float tauv[QT][16];
#pragma unroll
    for (int qt = 0; qt < QT; ++qt)
#pragma unroll
        for (int r = 0; r < 16; ++r) tauv[qt][r] = __uint_as_float(0x7F800000u);
    for (int q = lane; q < NQ; q += WAVE) s_cnt[wave][q] = 0;
    for (int q = 0; q < NQ; ++q) {
        const int qg = q0 + q;
        if (qg < n)
            for (int t = lane; t < CAP; t += WAVE) lists[static_cast<size_t>(qg) * CAP + t] = KEY_INF;
    }
    wave_lds_sync();

    // one async load instruction moves the 64 fragments (2 halves x 32 rows)
    // of one k-step of one sub-tile: a contiguous block of the tile-major
    // candidate operand; the four wavefronts share the work. Tiles past the
    // padded end are skipped (their candidates are masked out).
    const int ntiles = (n + 31) / 32;
    auto issue = [&](int stage, int c0) {
        for (int j = wave; j < NSUB * ks; j += SEL_WAVES) {
            const int sub = j / ks, s = j % ks;
            const int tile = c0 / 32 + sub;
            if (tile >= ntiles) continue;
            const elem* g = Bc + static_cast<size_t>(tile) * 32 * kpad + (s * 64 + lane) * Tr::VEC;
            Tr::async_copy(g, &s_tile[stage][sub][s][0][0]);
        }
    };

    uint64_t nonempty = 0;   // queries with buffered entries (wave-uniform)
    auto merge_query = [&](int q) {
        const int qg = q0 + q;
        const int c = s_cnt[wave][q];
        uint64_t b = lane < c ? s_buf[wave][q][lane] : KEY_INF;
        float nt = __uint_as_float(0x7F800000u);
        if (qg < n) {
            uint64_t L[E];
            uint64_t* dst = lists + static_cast<size_t>(qg) * CAP;
#pragma unroll
            for (int s = 0; s < E; ++s) L[s] = dst[s * WAVE + lane];
            merge_into_list<E>(L, b);
#pragma unroll
            for (int s = 0; s < E; ++s) dst[s * WAVE + lane] = L[s];
            nt = key_dist(list_at<E>(L, kp - 1));
        }
        if (lane == 0) s_cnt[wave][q] = 0;
        // the query's threshold sits in one accumulator slot of one lane half
        const int qt = q / 32, mrow = q % 32;
        const int rr = 4 * (mrow / 8) + (mrow % 4), hh = (mrow / 4) & 1;
#pragma unroll
        for (int t = 0; t < QT; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (t == qt && r == rr && half == hh) tauv[t][r] = nt;
    };

    issue(0, 0);
    int stage = 0;
    for (int c0 = 0; c0 < n; c0 += TW, stage ^= 1) {
        __builtin_amdgcn_s_waitcnt(0);   // this wavefront's loads of the current stage have landed
        __syncthreads();                 // ... and every other wavefront's; the other stage is free
        if (c0 + TW < n) issue(stage ^ 1, c0 + TW);
        f32x16 acc[NSUB][QT];
        const f32x16 zero = {};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
#pragma unroll
            for (int sub = 0; sub < NSUB; ++sub) {
                const frag b = s_tile[stage][sub][s][half][lane & 31];
#pragma unroll
                for (int qt = 0; qt < QT; ++qt) acc[sub][qt] = Tr::mma(qa[qt][s], b, s == 0 ? zero : acc[sub][qt]);
            }
        }
#pragma unroll
        for (int sub = 0; sub < NSUB; ++sub) {
            const int cand = c0 + sub * 32 + (lane & 31);
            const bool valid = cand < n;
            uint64_t flush = 0;
#pragma unroll
            for (int qt = 0; qt < QT; ++qt) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float sc = acc[sub][qt][r];
                    const uint64_t mask = __ballot(valid && sc <= tauv[qt][r]);
                    if (mask) {
                        const int qa_ = qt * 32 + acc_row(r, 0), qb_ = qt * 32 + acc_row(r, 1);
                        const uint32_t ma = static_cast<uint32_t>(mask), mb = static_cast<uint32_t>(mask >> 32);
                        const int ca = ma ? s_cnt[wave][qa_] : 0;
                        const int cb = mb ? s_cnt[wave][qb_] : 0;
                        const uint32_t hm = half ? mb : ma;
                        const int l31 = lane & 31;
                        if ((hm >> l31) & 1u) {
                            const int pos = (half ? cb : ca) + __popc(hm & ((1u << l31) - 1u));
                            s_buf[wave][half ? qb_ : qa_][pos] = make_key(sc, static_cast<uint32_t>(cand));
                        }
                        const int na = ca + __popc(ma), nb = cb + __popc(mb);
                        if (lane == 0 && ma) s_cnt[wave][qa_] = na;
                        if (lane == 32 && mb) s_cnt[wave][qb_] = nb;
                        if (ma) nonempty |= 1ull << qa_;
                        if (mb) nonempty |= 1ull << qb_;
                        if (na > SEL_BUF / 2) flush |= 1ull << qa_;
                        if (nb > SEL_BUF / 2) flush |= 1ull << qb_;
                    }
                }
            }
            if (flush) {
                wave_lds_sync();
                while (flush) {
                    const int q = __builtin_ctzll(flush);
                    flush &= flush - 1;
                    merge_query(q);
                    nonempty &= ~(1ull << q);
                    wave_lds_sync();
                }
            }
        }
    }
    wave_lds_sync();
    while (nonempty) {
        const int q = __builtin_ctzll(nonempty);
        nonempty &= nonempty - 1;
        merge_query(q);
        wave_lds_sync();
    }
    // certificate lower bound for the candidates left out of each list
    const double R = static_cast<double>(__uint_as_float(*rmax_bits));
    for (int q = lane; q < NQ; q += WAVE) {
        const int qg = q0 + q;
        if (qg >= n) continue;
        const float sl = key_dist(lists[static_cast<size_t>(qg) * CAP + (kp - 1)]);
        const double yi2 = static_cast<double>(ynorm2[qg]);
        const double yi = sqrt(yi2);
        const double Ei = em.gamma * (R + 1.05 * yi) * (R + 1.05 * yi) + em.norm * R * R + em.cross * yi * R + 1e-30;
        const double t = static_cast<double>(sl) + yi2 - Ei;
        double D = t > 0.0 ? sqrt(t) : 0.0;
        D -= em.center * (yi + R);
        D = D > 0.0 ? D : 0.0;
        lb_out[qg] = static_cast<float>(D * D * (1.0 - 1.0 / 1048576.0));
    }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_prep(const float* X, int n, int m, int split, int kpad, double* colpart, int colblocks,
                       double* mu, void* Aq, void* Bc, float* ynorm2, unsigned* rmax_bits, hipStream_t st)
{
    const int rpb = (n + colblocks - 1) / colblocks;
    const int npad = (n + 31) / 32 * 32;
    hipLaunchKernelGGL(k_colsum_partial, dim3(colblocks), dim3(256), 0, st, X, n, m, rpb, colpart);
    hipLaunchKernelGGL(k_colsum_finish, dim3(1), dim3(256), 0, st, colpart, colblocks, m, n, mu);
    hipLaunchKernelGGL(k_prep_rows, dim3((npad + 3) / 4), dim3(256), 0, st, X, n, npad, m, mu, split, kpad, Aq, Bc,
                       ynorm2, rmax_bits);
    return hipGetLastError();
}

template <class Tr, int KS, int QT, int TW>
static hipError_t launch_sel(const void* Aq, const void* Bc, int n, int kp, const float* ynorm2, const unsigned* rmax,
                             ErrModel em, uint64_t* lists, int cap, float* lb, hipStream_t st)
{
    using elem = typename Tr::elem;
    const int rows_per_block = SEL_WAVES * 32 * QT;
    const dim3 grid((n + rows_per_block - 1) / rows_per_block), block(256);
    const elem* A = static_cast<const elem*>(Aq);
    const elem* B = static_cast<const elem*>(Bc);
    // the lists buffer holds n * cap keys; only capacities 128 and 256 exist
    if (kp > cap) return hipErrorInvalidValue;
    if (cap == 128)
        hipLaunchKernelGGL((k_select_mfma<Tr, KS, QT, TW, 2>), grid, block, 0, st, A, B, n, kp, ynorm2, rmax, em, lists,
                           lb);
    else if (cap == 256)
        hipLaunchKernelGGL((k_select_mfma<Tr, KS, QT, TW, 4>), grid, block, 0, st, A, B, n, kp, ynorm2, rmax, em, lists,
                           lb);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Instantiated contraction lengths (in MFMA K-steps); the operand K is padded
// with zeros up to the next one. QT (query tiles per wavefront) and TW
// (candidates per LDS stage) are chosen so that registers and LDS fit.
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

#define KVB_SEL_CASE(TR, K, QT, TW) \
    case K: return launch_sel<TR, K, QT, TW>(Aq, Bc, n, kp, ynorm2, rmax, em, lists, cap, lb, st);

hipError_t launch_select_mfma(int split, const void* Aq, const void* Bc, int n, int kpad, int kp, const float* ynorm2,
                              const unsigned* rmax, ErrModel em, uint64_t* lists, int cap, float* lb, hipStream_t st)
{
    const int ks = kpad / mfma_kstep(split);
    if (split == 0) {
        switch (ks) {
            KVB_SEL_CASE(TraitsF32, 2, 2, 64)
            KVB_SEL_CASE(TraitsF32, 4, 2, 64)
            KVB_SEL_CASE(TraitsF32, 6, 2, 64)
            KVB_SEL_CASE(TraitsF32, 8, 2, 32)
            KVB_SEL_CASE(TraitsF32, 10, 2, 32)
            KVB_SEL_CASE(TraitsF32, 12, 2, 32)
            KVB_SEL_CASE(TraitsF32, 16, 2, 32)
            KVB_SEL_CASE(TraitsF32, 24, 2, 32)
            KVB_SEL_CASE(TraitsF32, 32, 2, 32)
            KVB_SEL_CASE(TraitsF32, 48, 1, 64)
            KVB_SEL_CASE(TraitsF32, 64, 1, 64)
            KVB_SEL_CASE(TraitsF32, 96, 1, 32)
            KVB_SEL_CASE(TraitsF32, 128, 1, 32)
        default: return hipErrorInvalidValue;
        }
    }
    switch (ks) {
        KVB_SEL_CASE(TraitsBF16, 2, 2, 32)
        KVB_SEL_CASE(TraitsBF16, 3, 2, 32)
        KVB_SEL_CASE(TraitsBF16, 4, 2, 32)
        KVB_SEL_CASE(TraitsBF16, 5, 2, 32)
        KVB_SEL_CASE(TraitsBF16, 6, 2, 32)
        KVB_SEL_CASE(TraitsBF16, 7, 2, 32)
        KVB_SEL_CASE(TraitsBF16, 8, 2, 32)
        KVB_SEL_CASE(TraitsBF16, 10, 1, 64)
        KVB_SEL_CASE(TraitsBF16, 13, 1, 64)
        KVB_SEL_CASE(TraitsBF16, 16, 1, 64)
        KVB_SEL_CASE(TraitsBF16, 20, 1, 32)
        KVB_SEL_CASE(TraitsBF16, 25, 1, 32)
        KVB_SEL_CASE(TraitsBF16, 32, 1, 32)
    default: return hipErrorInvalidValue;
    }
}
#undef KVB_SEL_CASE

}  // namespace kvb
