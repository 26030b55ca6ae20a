// Exact k-nearest-neighbour kernels (gfx950).
//
// The method needs, for every sample, its k-1 nearest other samples in the
// order I(x, k) of Section 2.1 (ties to the smaller index); this fixes the
// sparsity pattern of every kernel matrix in Sections 2.1-2.2. The paper's
// brute-force construction (Section 4, Algorithm 1) evaluates all n^2 pairs;
// its rows are independent, which is the parallelism used here.
//
// Pipeline of kvb_knn for one row i:
//   select   stream all n candidates through a distance test and keep the
//            k' = k + margin smallest (distance, index) keys in a register
//            list (one wavefront owns R rows; lanes hold candidates);
//   refine   recompute the k' candidates' squared distances in float64
//            (rounded to float32), drop i itself, sort, decide membership at the
//            k-th neighbour in float64, and check a certificate that no
//            dropped candidate can be nearer than the k-th kept one;
//   fallback rows without a certificate are recomputed by an exact float64
//            radix selection over all n samples.
#include <algorithm>

#include "kvb_device.h"
#include "kvb_kernels.h"

namespace kvb {

// -------------------------------------------------------------------- select
// Direct-difference distance tiles for small m (VALU: m subtractions and m
// multiply-adds per pair; the query coordinates are wave-uniform).
//
// The samples are visited in a spatial order: sorted along a Morton (Z-order)
// curve of their coordinates, cut into tiles of 64 consecutive samples (one
// candidate per lane) and superblocks of 16 tiles, each with its axis-aligned
// bounding box. A wavefront owns R consecutive sorted rows. It first scores
// its own tile and the nearest tiles along the curve, which sets tight
// thresholds, then tests every superblock box (64 per instruction, one per
// lane) and, inside the superblocks within reach, every tile box (16 lanes),
// and scores only the tiles whose box lies within some row's current
// threshold of that row's point. A candidate skipped for a row is therefore at
// least as far as that row's threshold, which only decreases afterwards; this
// keeps the certificate of
// the refine step valid: the box bound is computed in float32 with at most
// (m + 2) roundings, inside the relative margin the refine step allows for
// the selection scores.
//
// Candidates passing the current threshold of a row are appended to a
// 64-entry LDS buffer; a full buffer is merged into the row's register list by
// a bitonic network, which also tightens the threshold. Keys carry curve
// positions; the re-rank maps them to original indices and breaks ties on
// those, so ties order as in I(x, k).
struct SpatialView {
    const float* Xs;      // [n, m] coordinates in curve order
    const float* tbox;    // [tiles, 2, m]: lower corner, then upper corner
    const float* sbox;    // [superblocks, 2, m]
};

constexpr int TILE = 64;
constexpr int SB_TILES = 16;

// Whether a box may hold a candidate for any of the wavefront's rows: the
// squared gap from row r's point to the box against row r's own threshold.
// (Testing the rows' common bounding box instead lets a wavefront whose rows
// straddle a jump of the curve scan far too many tiles.)
template <int M, int R>
__device__ __forceinline__ bool box_near_rows(const float* __restrict__ b, const float (&q)[R][M],
                                              const float (&tau)[R])
{
    float lo[M], hi[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        lo[c] = b[c];
        hi[c] = b[M + c];
    }
    bool near = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const float g = fmaxf(fmaxf(lo[c] - q[r][c], q[r][c] - hi[c]), 0.f);
            s = fmaf(g, g, s);
        }
        near = near || s <= tau[r];
    }
    return near;
}

constexpr int SEED_TILES = 3;   // curve neighbours on each side scored before any box test
constexpr int TILE_BATCH = 2;   // tiles of a superblock whose loads are in flight together

// Upper bound on the kp-th smallest of the wavefront's NS x 64 non-negative
// values (+inf marks none): bisection on the float bit pattern down to bit
// 18 (a relative resolution of 2^-5), by ballot counts; +inf when fewer
// than kp values are finite.
template <int NS>
__device__ __forceinline__ float seed_threshold(const float (&d)[NS], int kp)
{
    int total = 0;
#pragma unroll
    for (int u = 0; u < NS; ++u) total += __popcll(__ballot(d[u] < __uint_as_float(0x7F800000u)));
    if (total < kp) return __uint_as_float(0x7F800000u);
    uint32_t P = 0;
    for (int b = 30; b >= 18; --b) {
        const uint32_t cand = P | (1u << b);
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < NS; ++u) cnt += __popcll(__ballot(__float_as_uint(d[u]) < cand));
        if (cnt < kp) P = cand;
    }
    return __uint_as_float(P | ((1u << 18) - 1u));
}

template <int M>
__device__ __forceinline__ void load_tile(const SpatialView& sv, int n, int t, int lane, float (&x)[M], uint32_t& jo)
{
    const int jp = min(t * TILE + lane, n - 1);
#pragma unroll
    for (int c = 0; c < M; ++c) x[c] = sv.Xs[static_cast<size_t>(jp) * M + c];
    jo = static_cast<uint32_t>(jp);   // curve position; the refine step maps it to the sample id
}

// Score one tile of 64 candidates against the wavefront's R rows and append
// the keys that pass each row's threshold (see k_select_direct).
template <int M, int R, int E>
__device__ __forceinline__ void score_tile(const float (&q)[R][M], const float (&x)[M], uint32_t jo, bool valid, int n,
                                           int t, int kp, int rows_here, int lane, uint64_t* buf, uint64_t (&L)[R][E],
                                           float (&tau)[R], int (&bc)[R], unsigned long long& pairs)
{
    pairs += static_cast<unsigned long long>(min(TILE, n - t * TILE)) * rows_here;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float tt = q[r][0] - x[0];
        float d = tt * tt;
#pragma unroll
        for (int c = 1; c < M; ++c) {
            tt = q[r][c] - x[c];
            d = fmaf(tt, tt, d);
        }
        uint64_t mask = __ballot(valid && d <= tau[r]);
        if (mask) {
            int cnt = __popcll(mask);
            if (bc[r] + cnt > WAVE) {
                wave_lds_sync();
                uint64_t b = lane < bc[r] ? buf[r * WAVE + lane] : KEY_INF;
                merge_into_list<E>(L[r], b);
                bc[r] = 0;
                tau[r] = key_dist(list_at<E>(L[r], kp - 1));
                mask = __ballot(valid && d <= tau[r]);
                cnt = __popcll(mask);
                wave_lds_sync();
            }
            if ((mask >> lane) & 1ull) buf[r * WAVE + bc[r] + mbcnt64(mask)] = make_key(d, jo);
            bc[r] += cnt;
        }
    }
}

template <int M, int R, int E>
__global__ __launch_bounds__(256) void k_select_direct(SpatialView sv, int n, int kp,
                                                       uint64_t* __restrict__ keys_out,
                                                       float* __restrict__ slast_out,
                                                       unsigned long long* __restrict__ pair_count)
{
    __shared__ uint64_t sbuf[4][R][WAVE];
    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int row0 = (blockIdx.x * 4 + wave) * R;   // curve position of the first row
    if (row0 >= n) return;

    float q[R][M];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int p = min(row0 + r, n - 1);
#pragma unroll
        for (int c = 0; c < M; ++c) q[r][c] = sv.Xs[static_cast<size_t>(p) * M + c];
    }
    uint64_t L[R][E];
    float tau[R];
    int bc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int s = 0; s < E; ++s) L[r][s] = KEY_INF;
        tau[r] = __uint_as_float(0x7F800000u);
        bc[r] = 0;
    }
    uint64_t* buf = &sbuf[wave][0][0];
    const int rows_here = min(R, n - row0);
    unsigned long long pairs = 0;

    const int ntiles = (n + TILE - 1) / TILE;
    const int nsb = (ntiles + SB_TILES - 1) / SB_TILES;
    const int own_t = row0 / TILE;
    // seed: the own tile and its curve neighbours, unconditionally. Each row's
    // first threshold is a coarse upper bound of the kp-th smallest seed
    // distance (valid for the whole scan: the kp-th smallest of a subset is at
    // least the kp-th smallest overall), so the seeds append little more than kp.
    constexpr int NS = 2 * SEED_TILES + 1;
    const int a0 = max(0, own_t - SEED_TILES), a1 = min(ntiles - 1, own_t + SEED_TILES);
    float xs[NS][M];
    uint32_t js[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) load_tile<M>(sv, n, min(a0 + u, a1), lane, xs[u], js[u]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float ds[NS];
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            float tt = q[r][0] - xs[u][0];
            float d = tt * tt;
#pragma unroll
            for (int c = 1; c < M; ++c) {
                tt = q[r][c] - xs[u][c];
                d = fmaf(tt, tt, d);
            }
            const bool ok = (a0 + u <= a1) && ((a0 + u) * TILE + lane < n);
            ds[u] = ok ? d : __uint_as_float(0x7F800000u);
        }
        tau[r] = seed_threshold<NS>(ds, kp);
    }
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const int t = a0 + u;
        if (t <= a1)
            score_tile<M, R, E>(q, xs[u], js[u], t * TILE + lane < n, n, t, kp, rows_here, lane, buf, L, tau, bc,
                                pairs);
    }
    // then every superblock within reach of some row (boxes tested 64 at a
    // time, one per lane), inside it every tile within reach (16 lanes), the
    // tiles' loads issued TILE_BATCH at a time
    for (int sb0 = 0; sb0 < nsb; sb0 += WAVE) {
        const int sbl = sb0 + lane;
        bool near = false;
        if (sbl < nsb) near = box_near_rows<M, R>(sv.sbox + static_cast<size_t>(sbl) * 2 * M, q, tau);
        uint64_t sbm = __ballot(near);
        while (sbm) {
            const int sb = sb0 + __builtin_ctzll(sbm);
            sbm &= sbm - 1;
            const int tl = sb * SB_TILES + lane;
            bool tnear = false;
            if (lane < SB_TILES && tl < ntiles && (tl < a0 || tl > a1))
                tnear = box_near_rows<M, R>(sv.tbox + static_cast<size_t>(tl) * 2 * M, q, tau);
            uint64_t tm = __ballot(tnear);
            while (tm) {
                int tb[TILE_BATCH];
                float xb[TILE_BATCH][M];
                uint32_t jb[TILE_BATCH];
#pragma unroll
                for (int u = 0; u < TILE_BATCH; ++u) {
                    tb[u] = -1;
                    jb[u] = 0;
                    if (tm) {
                        tb[u] = sb * SB_TILES + __builtin_ctzll(tm);
                        tm &= tm - 1;
                        load_tile<M>(sv, n, tb[u], lane, xb[u], jb[u]);
                    }
                }
#pragma unroll
                for (int u = 0; u < TILE_BATCH; ++u)
                    if (tb[u] >= 0)
                        score_tile<M, R, E>(q, xb[u], jb[u], tb[u] * TILE + lane < n, n, tb[u], kp, rows_here, lane,
                                            buf, L, tau, bc, pairs);
            }
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (bc[r] > 0) {
            uint64_t b = lane < bc[r] ? buf[r * WAVE + lane] : KEY_INF;
            merge_into_list<E>(L[r], b);
        }
        if (row0 + r < n) {
            const int i = row0 + r;   // lists are stored by curve position
            uint64_t* dst = keys_out + static_cast<size_t>(i) * kp;
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const int t = s * WAVE + lane;
                if (t < kp) dst[t] = L[r][s];
            }
            const float sl = key_dist(list_at<E>(L[r], kp - 1));
            if (lane == 0) slast_out[i] = sl;
        }
    }
    if (pair_count && lane == 0) atomicAdd(pair_count, pairs);
}

// ---- spatial order of the direct path
// Bounding box of the samples: per-block partial minima / maxima, then one block.
__global__ __launch_bounds__(256) void k_bbox_partial(const float* __restrict__ X, int n, int m, int rows_per_block,
                                                      float* __restrict__ part)
{
    __shared__ float sl[256], sh[256];
    const int r0 = blockIdx.x * rows_per_block, r1 = min(n, r0 + rows_per_block);
    for (int c = 0; c < m; ++c) {
        float lo = __uint_as_float(0x7F800000u), hi = -__uint_as_float(0x7F800000u);
        for (int r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
            const float v = X[static_cast<size_t>(r) * m + c];
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
        }
        sl[threadIdx.x] = lo;
        sh[threadIdx.x] = hi;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (threadIdx.x < o) {
                sl[threadIdx.x] = fminf(sl[threadIdx.x], sl[threadIdx.x + o]);
                sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + o]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            part[static_cast<size_t>(blockIdx.x) * 2 * m + c] = sl[0];
            part[static_cast<size_t>(blockIdx.x) * 2 * m + m + c] = sh[0];
        }
        __syncthreads();
    }
}

// Morton code of every sample: each coordinate quantised to b = min(31, 32 / m) bits
// over the bounding box (the box partials are reduced here, redundantly per
// thread: at most 1024 partials of 2m values), bits interleaved from the most
// significant. value = sample index, so a stable sort breaks ties by index.
__global__ __launch_bounds__(256) void k_morton(const float* __restrict__ X, int n, int m, int bits,
                                                const float* __restrict__ part, int nparts,
                                                uint32_t* __restrict__ code, int32_t* __restrict__ vals)
{
    __shared__ float s_lo[8], s_scale[8];
    if (threadIdx.x < m) {
        const int c = threadIdx.x;
        float lo = __uint_as_float(0x7F800000u), hi = -__uint_as_float(0x7F800000u);
        for (int b = 0; b < nparts; ++b) {
            lo = fminf(lo, part[static_cast<size_t>(b) * 2 * m + c]);
            hi = fmaxf(hi, part[static_cast<size_t>(b) * 2 * m + m + c]);
        }
        const float ext = hi - lo;
        s_lo[c] = lo;
        s_scale[c] = ext > 0.f ? static_cast<float>(1ull << bits) / ext : 0.f;
    }
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t qc[8];
    const uint32_t qmax = static_cast<uint32_t>((1ull << bits) - 1);
    for (int c = 0; c < m; ++c) {
        const float t = (X[static_cast<size_t>(i) * m + c] - s_lo[c]) * s_scale[c];
        const float tc = fminf(fmaxf(t, 0.f), static_cast<float>(qmax));
        qc[c] = min(static_cast<uint32_t>(tc), qmax);
    }
    uint32_t z = 0;
    for (int b = bits - 1; b >= 0; --b)
        for (int c = 0; c < m; ++c) z = (z << 1) | ((qc[c] >> b) & 1u);
    code[i] = z;
    vals[i] = i;
}

__global__ __launch_bounds__(256) void k_gather_rows(const float* __restrict__ X, int n, int m,
                                                     const int32_t* __restrict__ perm, float* __restrict__ Xs)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(n) * m) return;
    const int p = static_cast<int>(t / m), c = static_cast<int>(t % m);
    Xs[t] = X[static_cast<size_t>(perm[p]) * m + c];
}

// the same with four coordinates per thread (m a multiple of 4, rows 16-byte aligned)
__global__ __launch_bounds__(256) void k_gather_rows4(const float4* __restrict__ X, int n, int m4,
                                                      const int32_t* __restrict__ perm, float4* __restrict__ Xs)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(n) * m4) return;
    const int p = static_cast<int>(t / m4), c = static_cast<int>(t % m4);
    Xs[t] = X[static_cast<size_t>(perm[p]) * m4 + c];
}

// Xs[p] = X[perm[p]], float4 pieces where the rows allow
static void gather_rows(const float* X, int n, int m, const int32_t* perm, float* Xs, hipStream_t st)
{
    const bool v4 =
        m % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0 && (reinterpret_cast<uintptr_t>(Xs) & 15) == 0;
    const int64_t tot = static_cast<int64_t>(n) * (v4 ? m / 4 : m);
    const dim3 grid(static_cast<unsigned>((tot + 255) / 256));
    if (v4)
        hipLaunchKernelGGL(k_gather_rows4, grid, dim3(256), 0, st, reinterpret_cast<const float4*>(X), n, m / 4, perm,
                           reinterpret_cast<float4*>(Xs));
    else
        hipLaunchKernelGGL(k_gather_rows, grid, dim3(256), 0, st, X, n, m, perm, Xs);
}

// Box of `span` consecutive rows starting at row `first` of each group g
// (rows beyond n are ignored); used for tiles over Xs and for superblocks over
// tile boxes (span 16, rows = boxes, with `boxes` set).
__global__ __launch_bounds__(256) void k_group_boxes(const float* __restrict__ src, int rows, int m, int span,
                                                     int groups, int boxes, float* __restrict__ out)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(groups) * m) return;
    const int g = static_cast<int>(t / m), c = static_cast<int>(t % m);
    const int r0 = g * span, r1 = min(rows, r0 + span);
    float lo = __uint_as_float(0x7F800000u), hi = -__uint_as_float(0x7F800000u);
    for (int r = r0; r < r1; ++r) {
        if (boxes) {
            lo = fminf(lo, src[static_cast<size_t>(r) * 2 * m + c]);
            hi = fmaxf(hi, src[static_cast<size_t>(r) * 2 * m + m + c]);
        } else {
            const float v = src[static_cast<size_t>(r) * m + c];
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
        }
    }
    out[static_cast<size_t>(g) * 2 * m + c] = lo;
    out[static_cast<size_t>(g) * 2 * m + m + c] = hi;
}

// -------------------------------------------------------------------- refine
// Squared distances of row a to the rows b_s = B + j_s m (where act_s), each
// accumulated in float64 over the columns in order (the difference of two
// float32 values is exact in float64) and rounded once to float32: the same
// operations as dist2_f64, so these agree bit for bit with the exact path's
// distances. On gfx950 an unpacked float64 FMA issues at the float32 rate,
// so this costs about three instructions per coordinate. The coordinates are
// read CH at a time (float4 pieces when vec4), so that a chunk's loads are in
// flight together.
template <int E, int CH>
__device__ __forceinline__ void dist2_rows_ch(const float* __restrict__ a, const float* __restrict__ B, int m,
                                              const int (&j)[E], const bool (&act)[E], bool vec4, float (&out)[E])
{
    double acc[E];
#pragma unroll
    for (int s = 0; s < E; ++s) acc[s] = 0.0;
    for (int c0 = 0; c0 < m; c0 += CH) {
        float av[CH], bv[E][CH];
        if (vec4) {
#pragma unroll
            for (int u = 0; u < CH / 4; ++u) {
                if (c0 + 4 * u < m) {
                    const float4 q = *reinterpret_cast<const float4*>(a + c0 + 4 * u);
                    av[4 * u] = q.x;
                    av[4 * u + 1] = q.y;
                    av[4 * u + 2] = q.z;
                    av[4 * u + 3] = q.w;
                }
            }
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const float* b = B + static_cast<size_t>(j[s]) * m;
#pragma unroll
                for (int u = 0; u < CH / 4; ++u) {
                    if (act[s] && c0 + 4 * u < m) {
                        const float4 q = *reinterpret_cast<const float4*>(b + c0 + 4 * u);
                        bv[s][4 * u] = q.x;
                        bv[s][4 * u + 1] = q.y;
                        bv[s][4 * u + 2] = q.z;
                        bv[s][4 * u + 3] = q.w;
                    }
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < CH; ++t)
                if (c0 + t < m) av[t] = a[c0 + t];
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const float* b = B + static_cast<size_t>(j[s]) * m;
#pragma unroll
                for (int t = 0; t < CH; ++t)
                    if (act[s] && c0 + t < m) bv[s][t] = b[c0 + t];
            }
        }
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            if (c0 + t < m) {
#pragma unroll
                for (int s = 0; s < E; ++s)
                    if (act[s]) {
                        const double d = static_cast<double>(av[t]) - static_cast<double>(bv[s][t]);
                        acc[s] = fma(d, d, acc[s]);
                    }
            }
        }
    }
#pragma unroll
    for (int s = 0; s < E; ++s) out[s] = static_cast<float>(acc[s]);
}

// the chunk fitted to m (8 coordinates at most for four key slots)
template <int E>
__device__ __forceinline__ void dist2_rows(const float* __restrict__ a, const float* __restrict__ B, int m,
                                           const int (&j)[E], const bool (&act)[E], bool vec4, float (&out)[E])
{
    if (m <= 4)
        dist2_rows_ch<E, 4>(a, B, m, j, act, vec4, out);
    else if (m <= 8 || E >= 4)
        dist2_rows_ch<E, 8>(a, B, m, j, act, vec4, out);
    else
        dist2_rows_ch<E, 16>(a, B, m, j, act, vec4, out);
}

__device__ __forceinline__ double dist2_f64(const float* __restrict__ a, const float* __restrict__ b, int m)
{
    double s = 0.0;
    for (int c = 0; c < m; ++c) {
        const double t = static_cast<double>(a[c]) - static_cast<double>(b[c]);
        s = fma(t, t, s);
    }
    return s;
}

// Squared distances of a row's candidates computed cooperatively: groups of
// LPC lanes share one candidate (coalesced reads of its row, float4 where the
// rows are 16-byte aligned), accumulate in float64 (differences of float32
// values and their squares are exact or nearly so in float64) and reduce
// inside the group; the result reaches the lane that owns the candidate's key.
// d[s] receives the distance of key slot s of this lane (unchanged where the
// key is KEY_INF or the row itself).
template <int E, int LPC>
__device__ __forceinline__ void group_distances(const float* __restrict__ X, int m, int i, int kp, bool vec4,
                                                const uint64_t (&v)[E], double (&d)[E])
{
    constexpr int CPW = WAVE / LPC;   // candidates per pass
    // pieces of the row per lane: float4 pieces (m <= 16 LPC) or floats (m <= 16 LPC)
    constexpr int QMAX = 16;
    const int lane = lane_id();
    const int g = lane / LPC, gl = lane % LPC;
    const float* xi = X + static_cast<size_t>(i) * m;
    float4 q4[4];
    float q1[QMAX];
    const int nit = vec4 ? (m + 4 * LPC - 1) / (4 * LPC) : (m + LPC - 1) / LPC;
#pragma unroll
    for (int it = 0; it < QMAX; ++it) {
        q1[it] = 0.f;
        if (!vec4 && it < nit) {
            const int c = gl + LPC * it;
            if (c < m) q1[it] = xi[c];
        }
    }
#pragma unroll
    for (int it = 0; it < 4; ++it) {
        q4[it] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (vec4 && it < nit) {
            const int c = 4 * (gl + LPC * it);
            if (c < m) q4[it] = *reinterpret_cast<const float4*>(xi + c);
        }
    }
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int cj = (v[s] != KEY_INF) ? static_cast<int>(key_idx(v[s])) : -1;
        const int tend = min(kp, (s + 1) * WAVE);
        int t0 = s * WAVE;
        if (vec4) {
            // two passes at a time: both candidates' pieces are loaded before
            // either is summed (an invalid slot reads row i and is zeroed)
            for (; t0 < tend; t0 += 2 * CPW) {
                const int t1 = t0 + CPW;
                const int ja = __shfl(cj, (t0 % WAVE) + g, WAVE);
                const int jb = __shfl(cj, (t1 % WAVE) + g, WAVE);
                const bool oka = ja >= 0 && ja != i && t0 + g < tend;
                const bool okb = t1 < tend && jb >= 0 && jb != i && t1 + g < tend;
                const float* xa = X + static_cast<size_t>(oka ? ja : i) * m;
                const float* xb = X + static_cast<size_t>(okb ? jb : i) * m;
                float4 pa[4], pb[4];
#pragma unroll
                for (int it = 0; it < 4; ++it) {
                    const int c = 4 * (gl + LPC * it);
                    const bool in = it < nit && c < m;
                    pa[it] = in ? *reinterpret_cast<const float4*>(xa + c) : make_float4(0.f, 0.f, 0.f, 0.f);
                    pb[it] = in ? *reinterpret_cast<const float4*>(xb + c) : make_float4(0.f, 0.f, 0.f, 0.f);
                }
                double acca = 0.0, accb = 0.0;
#pragma unroll
                for (int it = 0; it < 4; ++it) {
                    const int c = 4 * (gl + LPC * it);
                    if (it < nit && c < m) {
                        const double a0 = static_cast<double>(q4[it].x) - pa[it].x;
                        const double a1 = static_cast<double>(q4[it].y) - pa[it].y;
                        const double a2 = static_cast<double>(q4[it].z) - pa[it].z;
                        const double a3 = static_cast<double>(q4[it].w) - pa[it].w;
                        acca = fma(a0, a0, acca);
                        acca = fma(a1, a1, acca);
                        acca = fma(a2, a2, acca);
                        acca = fma(a3, a3, acca);
                        const double b0 = static_cast<double>(q4[it].x) - pb[it].x;
                        const double b1 = static_cast<double>(q4[it].y) - pb[it].y;
                        const double b2 = static_cast<double>(q4[it].z) - pb[it].z;
                        const double b3 = static_cast<double>(q4[it].w) - pb[it].w;
                        accb = fma(b0, b0, accb);
                        accb = fma(b1, b1, accb);
                        accb = fma(b2, b2, accb);
                        accb = fma(b3, b3, accb);
                    }
                }
                if (!oka) acca = 0.0;
                if (!okb) accb = 0.0;
#pragma unroll
                for (int o = 1; o < LPC; o <<= 1) {
                    acca += shfl_xor_f64(acca, o);
                    accb += shfl_xor_f64(accb, o);
                }
                // the group leaders' sums go to the owner lanes
                const int sa = (lane - (t0 % WAVE)) * LPC;
                const double gota = __shfl(acca, sa >= 0 && sa < WAVE ? sa : 0, WAVE);
                if (lane >= t0 % WAVE && lane < t0 % WAVE + CPW) d[s] = gota;
                const int sb = (lane - (t1 % WAVE)) * LPC;
                const double gotb = __shfl(accb, sb >= 0 && sb < WAVE ? sb : 0, WAVE);
                if (t1 < tend && lane >= t1 % WAVE && lane < t1 % WAVE + CPW) d[s] = gotb;
            }
            continue;
        }
        for (; t0 < tend; t0 += CPW) {
            const int owner = (t0 % WAVE) + g;                 // lane holding this group's candidate
            const int j = __shfl(cj, owner, WAVE);
            double acc = 0.0;
            if (j >= 0 && j != i && t0 + g < kp) {
                const float* xj = X + static_cast<size_t>(j) * m;
#pragma unroll
                for (int it = 0; it < QMAX; ++it) {
                    const int c = gl + LPC * it;
                    if (it < nit && c < m) {
                        const double e0 = static_cast<double>(q1[it]) - xj[c];
                        acc = fma(e0, e0, acc);
                    }
                }
            }
#pragma unroll
            for (int o = 1; o < LPC; o <<= 1) acc += shfl_xor_f64(acc, o);
            // the group leader's sum goes to the owner lane
            const int src = (lane - (t0 % WAVE)) * LPC;
            const double got = __shfl(acc, src >= 0 && src < WAVE ? src : 0, WAVE);
            if (lane >= t0 % WAVE && lane < t0 % WAVE + CPW) d[s] = got;
        }
    }
}

// One wavefront per row. keys: [n, kstride] candidate keys from a select
// kernel (the first kp of each row are used), slast: per row, a bound on the
// candidates the select step dropped, turned into a lower bound on their true
// squared distance by lb_scale (direct tiles: the kp-th score times
// 1/(1 + select error); matrix-core tiles: the bound itself, lb_scale = 1).
// slast == nullptr: no bound (learned routing). LPC == 0: each lane computes
// its own candidates' distances (float64 sums rounded to float32, short rows);
// LPC > 0: groups of LPC lanes per candidate (group_distances, long rows).
// Lists whose recomputed keys are still in ascending order once row i is taken
// out (the common case after the direct tiles, whose float32 scores differ
// from the recomputed distances only in the last bits) skip the sorting
// network.
//
// CV (curve-ordered scans): lists and bounds are stored by curve position r, their
// keys hold curve positions; the candidates are read from the curve-ordered
// copy Xs (neighbouring rows read neighbouring samples) and the keys are
// turned into (distance, sample id) through perm before any ordering.
template <int E, int LPC, bool CV>
__global__ __launch_bounds__(256) void k_refine(const float* __restrict__ X, int n, int m, int k, int kp,
                                                int kstride, const uint64_t* __restrict__ keys,
                                                const float* __restrict__ slast, float lb_scale,
                                                int32_t* __restrict__ idx_out, float* __restrict__ d2_out,
                                                int32_t* __restrict__ flags_out,
                                                int* __restrict__ fb_count, int* __restrict__ fb_list,
                                                float* __restrict__ fb_bound, int force_period,
                                                const float* __restrict__ Xs, const int32_t* __restrict__ perm)
{
    const int lane = lane_id();
    const int r = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // stored row
    if (r >= n) return;
    const int i = CV ? perm[r] : r;   // sample id
    const float* xi = CV ? Xs + static_cast<size_t>(r) * m : X + static_cast<size_t>(i) * m;
    // candidate distances, self removed
    uint64_t v[E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int t = s * WAVE + lane;
        v[s] = t < kp ? keys[static_cast<size_t>(r) * kstride + t] : KEY_INF;
    }
    // list position of row i, if present
    int ps = -1;
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const uint64_t mm = __ballot(v[s] != KEY_INF && static_cast<int>(key_idx(v[s])) == r);
        if (ps < 0 && mm) ps = s * WAVE + __builtin_ctzll(mm);
    }
    if constexpr (LPC == 0) {
        int jr[E];
        bool act[E];
#pragma unroll
        for (int s = 0; s < E; ++s) {
            act[s] = v[s] != KEY_INF && static_cast<int>(key_idx(v[s])) != r;
            jr[s] = act[s] ? static_cast<int>(key_idx(v[s])) : 0;
        }
        const float* Br = CV ? Xs : X;   // the rows the keys refer to
        const bool vec4 = (m % 4 == 0) && ((reinterpret_cast<uintptr_t>(Br) & 15) == 0);
        float dd[E];
        dist2_rows<E>(xi, Br, m, jr, act, vec4, dd);
#pragma unroll
        for (int s = 0; s < E; ++s) {
            if (v[s] == KEY_INF) continue;
            if (!act[s])
                v[s] = KEY_INF;
            else if constexpr (CV)
                v[s] = make_key(dd[s], static_cast<uint32_t>(perm[jr[s]]));
            else
                v[s] = make_key(dd[s], static_cast<uint32_t>(jr[s]));
        }
    } else {
        double dd[E];
#pragma unroll
        for (int s = 0; s < E; ++s) dd[s] = 0.0;
        const float* Xr = CV ? Xs : X;   // the rows the keys refer to
        const bool vec4 = (m % 4 == 0) && ((reinterpret_cast<uintptr_t>(Xr) & 15) == 0);
        group_distances<E, LPC>(Xr, m, r, kp, vec4, v, dd);
#pragma unroll
        for (int s = 0; s < E; ++s) {
            uint64_t key = v[s];
            if (key != KEY_INF) {
                const uint32_t j = key_idx(key);
                key = static_cast<int>(j) == r
                          ? KEY_INF
                          : make_key(static_cast<float>(dd[s]), CV ? static_cast<uint32_t>(perm[j]) : j);
            }
            v[s] = key;
        }
    }
    {
        // the keys one position on, with row i (now KEY_INF) moved past the end
        uint64_t nv[E];
        bool sorted = true;
#pragma unroll
        for (int s = 0; s < E; ++s) {
            uint64_t nx = shfl_u64(v[s], (lane + 1) & (WAVE - 1));
            if (lane == WAVE - 1) nx = (s + 1 < E) ? readlane_u64(v[s + 1 < E ? s + 1 : s], 0) : KEY_INF;
            nv[s] = (ps >= 0 && s * WAVE + lane >= ps) ? nx : v[s];
        }
#pragma unroll
        for (int s = 0; s < E; ++s) {
            uint64_t nx = shfl_u64(nv[s], (lane + 1) & (WAVE - 1));
            if (lane == WAVE - 1) nx = (s + 1 < E) ? readlane_u64(nv[s + 1 < E ? s + 1 : s], 0) : KEY_INF;
            sorted = sorted && !__ballot(nv[s] > nx);
        }
        if (sorted) {
#pragma unroll
            for (int s = 0; s < E; ++s) v[s] = nv[s];
        } else {
            bitonic_sort<E>(v);
        }
    }

    const int kk = k - 1;  // neighbours other than i
    int32_t* orow = idx_out + static_cast<size_t>(i) * k;
    float* drow = d2_out + static_cast<size_t>(i) * k;
    if (lane == 0) {
        orow[0] = i;
        drow[0] = 0.f;
    }
    int flags = 0;
    bool certified = true;
    float bound = __uint_as_float(0x7F800000u);   // upper bound on the true (k-1)-th distance
    if (kk > 0) {
        // relative error bound of the recomputed distances (a few units in
        // the last place), doubled for the band test
        const float dl = 4.8e-7f;
        const float a = key_dist(list_at<E>(v, kk - 1));
        const float lo_edge = a * (1.f - dl) / (1.f + dl);
        const float hi_edge = a * (1.f + dl) / (1.f - dl);
        // positions: sure-in (below lo_edge), band, sure-out (above hi_edge)
        uint64_t band_m[E];
        int c_lo = 0, nband = 0, band_beyond = 0, nvalid = 0;
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int t = s * WAVE + lane;
            const float dv = key_dist(v[s]);
            const bool valid = v[s] != KEY_INF;
            nvalid += __popcll(__ballot(valid));
            const bool in_lo = valid && dv < lo_edge;
            const bool in_band = valid && !in_lo && dv <= hi_edge;
            c_lo += __popcll(__ballot(in_lo));
            band_m[s] = __ballot(in_band);
            nband += __popcll(band_m[s]);
            band_beyond += __popcll(__ballot(in_band && t >= kk));
        }
        // FP64 recheck only when the band straddles the k-th position
        double d64[E];
        int rank[E];
#pragma unroll
        for (int s = 0; s < E; ++s) {
            d64[s] = 0.0;
            rank[s] = 0;
        }
        const bool recheck = band_beyond > 0;
        if (recheck) {
            flags |= KVB_ROW_RECHECK;
#pragma unroll
            for (int s = 0; s < E; ++s)
                if ((band_m[s] >> lane) & 1ull)
                    d64[s] = dist2_f64(xi, X + static_cast<size_t>(key_idx(v[s])) * m, m);
            // rank of every band member among band members by (d64, j)
#pragma unroll
            for (int so = 0; so < E; ++so) {
                uint64_t bm = band_m[so];
                while (bm) {
                    const int src = __builtin_ctzll(bm);
                    bm &= bm - 1;
                    const double od = __shfl(d64[so], src, WAVE);
                    const uint32_t oj = __builtin_amdgcn_readlane(static_cast<int>(key_idx(v[so])), src);
#pragma unroll
                    for (int s = 0; s < E; ++s) {
                        const uint32_t mj = key_idx(v[s]);
                        if ((od < d64[s]) || (od == d64[s] && oj < mj)) rank[s]++;
                    }
                }
            }
        }
        // write the k-1 neighbours and find the largest kept distance
        float kept_max = 0.f;
        int nkept = 0;
        const int need = kk - c_lo;
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int t = s * WAVE + lane;
            const bool valid = v[s] != KEY_INF;
            const float dv = key_dist(v[s]);
            const bool in_lo = valid && dv < lo_edge;
            const bool in_band = (band_m[s] >> lane) & 1ull;
            int pos = -1;
            float outd = dv;
            if (in_lo) {
                pos = t;
            } else if (in_band) {
                if (recheck) {
                    if (rank[s] < need) {
                        pos = c_lo + rank[s];
                        outd = static_cast<float>(d64[s]);
                    }
                } else if (t < kk) {
                    pos = t;
                }
            }
            if (pos >= 0) {
                orow[1 + pos] = static_cast<int32_t>(key_idx(v[s]));
                drow[1 + pos] = outd;
                kept_max = fmaxf(kept_max, dv);
            }
            nkept += __popcll(__ballot(pos >= 0));
        }
        kept_max = wave_max_f32(kept_max);
        // the kept candidates are k-1 samples within this distance of row i
        if (nkept == kk) bound = kept_max * (1.f + dl) * (1.f + 1e-6f);
        if (slast) {
            // certificate: every candidate the select step dropped has a true
            // squared distance >= slast * lb_scale; it must exceed the largest kept
            const float lb = slast[r] * lb_scale;
            const float ub = kept_max * (1.f + dl) * (1.f + 1e-6f);
            certified = lb > ub;
        } else {
            // no bound on the dropped candidates (learned routing): the row is
            // only completed by the exact scan when too few candidates were found
            certified = nvalid >= kk;
        }
    }
    if (!slast) flags |= KVB_ROW_UNCERTIFIED;
    if (force_period > 0 && (i % force_period) == 0) certified = false;
    if (!certified) {
        flags |= KVB_ROW_FALLBACK;
        if (lane == 0) {
            const int slot = atomicAdd(fb_count, 1);
            fb_list[slot] = i;
            fb_bound[slot] = bound;
        }
    }
    if (flags_out && lane == 0) flags_out[i] = flags;
}

// -------------------------------------------------------------------- fallback
// Exact float64 selection for the listed rows, ranked by (d, j).
//
// Bounded pass (rows with a finite bound B >= their true (k-1)-th distance,
// the first FB_MAX_ROWS listed): every block takes chunks of FB_CHUNK samples
// and, row after row (the chunk stays in cache), appends the samples j != i
// with d(i, j) <= B to the row's buffer of FB_CAP entries. All of the row's
// k-1 nearest are among them, so when the buffer holds between k-1 and FB_CAP
// entries the row is finished by ranking the buffer.
//
// Full scan (every other row): an 8-pass radix select on the bits of the
// float64 squared distance (non-negative doubles order like their bit
// patterns) finds the (k-1)-th smallest value V; the neighbours are all j with
// d < V plus the smallest-index j with d == V.
//
// Both compute d in the order of dist2_f64, so they agree on every value and tie.
constexpr int FB_THREADS = 256;
constexpr int FB_CHUNK = 1024;

// m <= FB_LDS_M: blocks stage FB_STAGE consecutive samples in LDS (coalesced,
// row stride m + 1 against bank conflicts), and the listed rows' coordinates,
// bounds and ids once per chunk of up to FB_ROW_FLOATS / m rows; every
// wavefront takes listed rows in turn, one staged sample per lane. A float32
// distance screens each pair first: it errs from the exact one by at most
// (m + 3) 2^-24 relative, so a pair whose float32 distance exceeds the bound by
// (m + 10) 2^-24 cannot be within it; the others are decided in float64 in the
// summation order of dist2_f64.
constexpr int FB_STAGE = 64;
constexpr int FB_LDS_M = 192;
constexpr int FB_LDS_BYTES = 60 * 1024;   // LDS per block: the sample stage, then row chunks
constexpr int FB_ROW_FLOATS = 8192;       // at most this many row coordinates per chunk

// listed rows per LDS chunk: their coordinates (m floats), bound and id each
__host__ __device__ inline int fb_rows_per_chunk(int m)
{
    const int stage = FB_STAGE * (m + 1) * 4;
    int r = (FB_LDS_BYTES - stage) / (4 * m + 12);
    r = r < FB_ROW_FLOATS / m ? r : FB_ROW_FLOATS / m;
    return r < FB_MAX_ROWS ? (r > 1 ? r : 1) : FB_MAX_ROWS;
}
size_t fb_collect_lds_bytes(int m)
{
    const int rch = fb_rows_per_chunk(m);
    return sizeof(float) * (static_cast<size_t>(FB_STAGE) * (m + 1) + static_cast<size_t>(rch) * m) +
           (sizeof(double) + sizeof(int)) * static_cast<size_t>(rch);
}

__global__ __launch_bounds__(FB_THREADS) void k_fb_collect_lds(const float* __restrict__ X, int n, int m,
                                                               const int* __restrict__ fb_count,
                                                               const int* __restrict__ fb_list,
                                                               const float* __restrict__ fb_bound, int rows_cap,
                                                               int* __restrict__ cnt, double* __restrict__ bd,
                                                               int* __restrict__ bj)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char fb_smem[];
    const int total = min(*fb_count, rows_cap);
    if (total == 0) return;
    const int rch = fb_rows_per_chunk(m);
    const int ld = m + 1;
    double* rb = reinterpret_cast<double*>(fb_smem);                  // [rch] screened bounds
    float* xc = reinterpret_cast<float*>(rb + rch);                    // [FB_STAGE][m + 1] samples
    float* xr = xc + FB_STAGE * ld;                                    // [rch][m] listed rows
    int* ri = reinterpret_cast<int*>(xr + static_cast<size_t>(rch) * m);   // [rch] their ids
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
    const double slack = 1.0 + (m + 10) * 0x1p-24;
    for (int r0 = 0; r0 < total; r0 += rch) {
        const int nr = min(rch, total - r0);
        __syncthreads();
        for (int t = threadIdx.x; t < nr; t += FB_THREADS) {
            const float B = fb_bound[r0 + t];
            ri[t] = fb_list[r0 + t];
            rb[t] = B < __uint_as_float(0x7F800000u) ? static_cast<double>(B) : -1.0;   // -1: no bound
        }
        for (int e = threadIdx.x; e < nr * m; e += FB_THREADS) {
            const int t = e / m, c = e - t * m;
            xr[e] = X[static_cast<size_t>(fb_list[r0 + t]) * m + c];
        }
        for (int c0 = blockIdx.x * FB_STAGE; c0 < n; c0 += gridDim.x * FB_STAGE) {
            __syncthreads();
            for (int e = threadIdx.x; e < FB_STAGE * m; e += FB_THREADS) {
                const int r = e / m, c = e - r * m;
                xc[r * ld + c] = c0 + r < n ? X[static_cast<size_t>(c0) * m + e] : 0.f;
            }
            __syncthreads();
            const int j = c0 + lane;
            const float* xj = xc + lane * ld;
            for (int t = wave; t < nr; t += FB_THREADS / WAVE) {
                const double B = rb[t];
                if (B < 0.0) continue;
                const int i = ri[t];
                if (j >= n || j == i) continue;
                const float* xi = xr + t * m;
                float d32 = 0.f;
                for (int c = 0; c < m; ++c) {
                    const float u = xi[c] - xj[c];
                    d32 = fmaf(u, u, d32);
                }
                if (d32 < __uint_as_float(0x7F800000u) && static_cast<double>(d32) > B * slack) continue;
                double d = 0.0;
                for (int c = 0; c < m; ++c) {
                    const double u = static_cast<double>(xi[c]) - static_cast<double>(xj[c]);
                    d = fma(u, u, d);
                }
                if (d <= B) {
                    const int slot = atomicAdd(&cnt[r0 + t], 1);
                    if (slot < FB_CAP) {
                        bd[static_cast<size_t>(r0 + t) * FB_CAP + slot] = d;
                        bj[static_cast<size_t>(r0 + t) * FB_CAP + slot] = j;
                    }
                }
            }
        }
    }
}

// m <= 16: every wavefront takes its own chunks of 64 samples, one per lane,
// with the sample's coordinates in registers (read straight from X: a chunk is
// 64 m consecutive floats), and the listed rows' coordinates, padded to 16,
// as four broadcast float4 reads from LDS; the padding adds exact zeros to
// both sums. Screen and decision as in k_fb_collect_lds.
constexpr int FB_REG_M = 16;
constexpr int FB_REG_ROWS = 768;   // listed rows per LDS chunk (76 bytes each: 57 KB)

size_t fb_collect_reg_bytes() { return static_cast<size_t>(FB_REG_ROWS) * (FB_REG_M * sizeof(float) + sizeof(double) + sizeof(int)); }

__global__ __launch_bounds__(FB_THREADS) void k_fb_collect_reg(const float* __restrict__ X, int n, int m,
                                                               const int* __restrict__ fb_count,
                                                               const int* __restrict__ fb_list,
                                                               const float* __restrict__ fb_bound, int rows_cap,
                                                               int* __restrict__ cnt, double* __restrict__ bd,
                                                               int* __restrict__ bj)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char fb_smem[];
    const int total = min(*fb_count, rows_cap);
    if (total == 0) return;
    float4* xr = reinterpret_cast<float4*>(fb_smem);                                 // [FB_REG_ROWS][4]
    double* rb = reinterpret_cast<double*>(fb_smem + FB_REG_ROWS * FB_REG_M * 4);    // [FB_REG_ROWS]
    int* ri = reinterpret_cast<int*>(rb + FB_REG_ROWS);                              // [FB_REG_ROWS]
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
    const double slack = 1.0 + (m + 10) * 0x1p-24;
    for (int r0 = 0; r0 < total; r0 += FB_REG_ROWS) {
        const int nr = min(FB_REG_ROWS, total - r0);
        __syncthreads();
        for (int t = threadIdx.x; t < nr; t += FB_THREADS) {
            const float B = fb_bound[r0 + t];
            ri[t] = fb_list[r0 + t];
            rb[t] = B < __uint_as_float(0x7F800000u) ? static_cast<double>(B) : -1.0;   // -1: no bound
        }
        float* xrf = reinterpret_cast<float*>(xr);
        for (int e = threadIdx.x; e < nr * FB_REG_M; e += FB_THREADS) {
            const int t = e / FB_REG_M, c = e - t * FB_REG_M;
            xrf[e] = c < m ? X[static_cast<size_t>(fb_list[r0 + t]) * m + c] : 0.f;
        }
        __syncthreads();
        for (int c0 = (blockIdx.x * (FB_THREADS / WAVE) + wave) * WAVE; c0 < n;
             c0 += gridDim.x * FB_THREADS) {
            const int j = c0 + lane;
            float xj[FB_REG_M];
#pragma unroll
            for (int c = 0; c < FB_REG_M; ++c) xj[c] = (j < n && c < m) ? X[static_cast<size_t>(j) * m + c] : 0.f;
            for (int t = 0; t < nr; ++t) {
                const double B = rb[t];
                if (B < 0.0) continue;
                float xi[FB_REG_M];
#pragma unroll
                for (int q = 0; q < FB_REG_M / 4; ++q) {
                    const float4 v = xr[t * (FB_REG_M / 4) + q];
                    xi[4 * q] = v.x;
                    xi[4 * q + 1] = v.y;
                    xi[4 * q + 2] = v.z;
                    xi[4 * q + 3] = v.w;
                }
                float d32 = 0.f;
#pragma unroll
                for (int c = 0; c < FB_REG_M; ++c) {
                    const float u = xi[c] - xj[c];
                    d32 = fmaf(u, u, d32);
                }
                const bool near = !(d32 < __uint_as_float(0x7F800000u)) || static_cast<double>(d32) <= B * slack;
                if (near && j < n && j != ri[t]) {
                    double d = 0.0;
#pragma unroll
                    for (int c = 0; c < FB_REG_M; ++c) {
                        const double u = static_cast<double>(xi[c]) - static_cast<double>(xj[c]);
                        d = fma(u, u, d);
                    }
                    if (d <= B) {
                        const int slot = atomicAdd(&cnt[r0 + t], 1);
                        if (slot < FB_CAP) {
                            bd[static_cast<size_t>(r0 + t) * FB_CAP + slot] = d;
                            bj[static_cast<size_t>(r0 + t) * FB_CAP + slot] = j;
                        }
                    }
                }
            }
        }
    }
}

__global__ __launch_bounds__(FB_THREADS) void k_fb_collect(const float* __restrict__ X, int n, int m,
                                                           const int* __restrict__ fb_count,
                                                           const int* __restrict__ fb_list,
                                                           const float* __restrict__ fb_bound, int rows_cap,
                                                           int* __restrict__ cnt, double* __restrict__ bd,
                                                           int* __restrict__ bj)
{
    __shared__ float xs[1024];
    const int total = min(*fb_count, rows_cap);
    for (int c0 = blockIdx.x * FB_CHUNK; c0 < n && total > 0; c0 += gridDim.x * FB_CHUNK) {
        for (int t = 0; t < total; ++t) {
            const float B = fb_bound[t];
            if (!(B < __uint_as_float(0x7F800000u))) continue;
            const int i = fb_list[t];
            __syncthreads();
            for (int c = threadIdx.x; c < m; c += FB_THREADS) xs[c] = X[static_cast<size_t>(i) * m + c];
            __syncthreads();
            const double Bd = static_cast<double>(B);
#pragma unroll
            for (int u = 0; u < FB_CHUNK / FB_THREADS; ++u) {
                const int j = c0 + u * FB_THREADS + threadIdx.x;
                if (j < n && j != i) {
                    const double d = dist2_f64(xs, X + static_cast<size_t>(j) * m, m);
                    if (d <= Bd) {
                        const int slot = atomicAdd(&cnt[t], 1);
                        if (slot < FB_CAP) {
                            bd[static_cast<size_t>(t) * FB_CAP + slot] = d;
                            bj[static_cast<size_t>(t) * FB_CAP + slot] = j;
                        }
                    }
                }
            }
        }
    }
}

// The row count is *fb_count, or `count` when fb_count is null. Results go to
// row i of idx_out / d2_out, or with `compact` to row t (the list position);
// in compact mode a listed id outside [0, n) yields a row of -1 / NaN.
__global__ __launch_bounds__(FB_THREADS) void k_fallback(const float* __restrict__ X, int n, int m, int k,
                                                         const int* __restrict__ fb_count, int count,
                                                         const int* __restrict__ fb_list, int compact,
                                                         int rows_cap, const int* __restrict__ cnt,
                                                         const double* __restrict__ bd, const int* __restrict__ bj,
                                                         int32_t* __restrict__ idx_out,
                                                         float* __restrict__ d2_out)
{
    __shared__ double s_bd[FB_CAP];
    __shared__ int s_bj[FB_CAP];
    __shared__ unsigned int hist[256];
    __shared__ unsigned long long s_prefix;
    __shared__ int s_remaining;
    __shared__ double cd[256];
    __shared__ int cj[256];
    __shared__ int s_cnt_lt, s_cnt_eq;
    __shared__ int wsum_lt[FB_THREADS / WAVE], wsum_eq[FB_THREADS / WAVE];
    const int tid = threadIdx.x;
    const int total = fb_count ? *fb_count : count;
    const int kk = k - 1;
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int i = fb_list[t];
        const size_t orow = compact ? static_cast<size_t>(t) : static_cast<size_t>(i);
        if (i < 0 || i >= n) {
            if (compact)
                for (int r = tid; r < k; r += FB_THREADS) {
                    idx_out[orow * k + r] = -1;
                    d2_out[orow * k + r] = __uint_as_float(0x7FC00000u);
                }
            continue;
        }
        const float* xi = X + static_cast<size_t>(i) * m;
        if (kk == 0) {
            if (tid == 0) {
                idx_out[orow * k] = i;
                d2_out[orow * k] = 0.f;
            }
            continue;
        }
        const int c = (cnt && t < rows_cap) ? cnt[t] : -1;
        if (c >= kk && c <= FB_CAP) {
            // bounded pass: rank the buffer by (d, j)
            for (int e = tid; e < c; e += FB_THREADS) {
                s_bd[e] = bd[static_cast<size_t>(t) * FB_CAP + e];
                s_bj[e] = bj[static_cast<size_t>(t) * FB_CAP + e];
            }
            __syncthreads();
            for (int e = tid; e < c; e += FB_THREADS) {
                const double d = s_bd[e];
                const int j = s_bj[e];
                int rank = 0;
                for (int u = 0; u < c; ++u) rank += (s_bd[u] < d) || (s_bd[u] == d && s_bj[u] < j);
                if (rank < kk) {
                    idx_out[orow * k + 1 + rank] = j;
                    d2_out[orow * k + 1 + rank] = static_cast<float>(d);
                }
            }
            if (tid == 0) {
                idx_out[orow * k] = i;
                d2_out[orow * k] = 0.f;
            }
            __syncthreads();
            continue;
        }
        if (tid == 0) {
            s_prefix = 0ull;
            s_remaining = kk;
        }
        __syncthreads();
        for (int shift = 56; shift >= 0; shift -= 8) {
            hist[tid] = 0u;
            __syncthreads();
            const unsigned long long pfx = s_prefix;
            const unsigned long long pmask = (shift == 56) ? 0ull : (~0ull << (shift + 8));
            for (int j = tid; j < n; j += FB_THREADS) {
                if (j == i) continue;
                const double d = dist2_f64(xi, X + static_cast<size_t>(j) * m, m);
                const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(d));
                if ((u & pmask) == pfx) atomicAdd(&hist[(u >> shift) & 255ull], 1u);
            }
            __syncthreads();
            if (tid == 0) {
                int rem = s_remaining;
                int b = 0;
                for (; b < 256; ++b) {
                    if (static_cast<int>(hist[b]) >= rem) break;
                    rem -= static_cast<int>(hist[b]);
                }
                s_prefix = pfx | (static_cast<unsigned long long>(b) << shift);
                s_remaining = rem;
            }
            __syncthreads();
        }
        const double V = __longlong_as_double(static_cast<long long>(s_prefix));
        const int need_eq = s_remaining;      // how many d == V entries to take
        const int n_lt = kk - need_eq;        // entries with d < V
        if (tid == 0) {
            s_cnt_lt = 0;
            s_cnt_eq = 0;
        }
        __syncthreads();
        // ordered compaction in index order
        for (int j0 = 0; j0 < n; j0 += FB_THREADS) {
            const int j = j0 + tid;
            double d = 0.0;
            bool lt = false, eq = false;
            if (j < n && j != i) {
                d = dist2_f64(xi, X + static_cast<size_t>(j) * m, m);
                lt = d < V;
                eq = d == V;
            }
            const uint64_t bl = __ballot(lt), be = __ballot(eq);
            const int w = tid / WAVE;
            if ((tid & (WAVE - 1)) == 0) {
                wsum_lt[w] = __popcll(bl);
                wsum_eq[w] = __popcll(be);
            }
            __syncthreads();
            int off_lt = s_cnt_lt, off_eq = s_cnt_eq;
            for (int u = 0; u < w; ++u) {
                off_lt += wsum_lt[u];
                off_eq += wsum_eq[u];
            }
            if (lt) {
                const int p = off_lt + mbcnt64(bl);
                cd[p] = d;
                cj[p] = j;
            }
            if (eq) {
                const int p = off_eq + mbcnt64(be);
                if (p < need_eq) {
                    cd[n_lt + p] = d;
                    cj[n_lt + p] = j;
                }
            }
            __syncthreads();
            if (tid == 0) {
                int a = 0, b = 0;
                for (int u = 0; u < FB_THREADS / WAVE; ++u) {
                    a += wsum_lt[u];
                    b += wsum_eq[u];
                }
                s_cnt_lt += a;
                s_cnt_eq += b;
            }
            __syncthreads();
        }
        // rank by (d, j) and write
        if (tid < kk) {
            const double d = cd[tid];
            const int j = cj[tid];
            int rank = 0;
            for (int u = 0; u < kk; ++u) rank += (cd[u] < d) || (cd[u] == d && cj[u] < j);
            idx_out[orow * k + 1 + rank] = j;
            d2_out[orow * k + 1 + rank] = static_cast<float>(d);
        }
        if (tid == 0) {
            idx_out[orow * k] = i;
            d2_out[orow * k] = 0.f;
        }
        __syncthreads();
    }
}

// -------------------------------------------------------------------- launchers
int spatial_bbox_blocks(int n) { return std::max(1, std::min(1024, (n + 4095) / 4096)); }
int spatial_tiles(int n) { return (n + TILE - 1) / TILE; }
int spatial_superblocks(int n) { return (spatial_tiles(n) + SB_TILES - 1) / SB_TILES; }

// Bits per coordinate of the Morton code: enough cells for a few samples each
// (the tiles stay compact; finer codes only lengthen the sort), at most 32 in all.
int spatial_code_bits(int n, int m)
{
    int lg = 0;
    while ((1ll << lg) < static_cast<long long>(n)) ++lg;
    const int want = std::max(8, (lg + m - 1) / m + 2);
    return std::min(std::min(31, 32 / m), want);
}

hipError_t launch_spatial_codes(const float* X, int n, int m, float* bbox_part, uint32_t* code, int32_t* vals,
                                hipStream_t st)
{
    if (m < 1 || m > 8) return hipErrorInvalidValue;
    const int bits = spatial_code_bits(n, m);
    const int nb = spatial_bbox_blocks(n);
    const int rpb = (n + nb - 1) / nb;
    hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(256), 0, st, X, n, m, rpb, bbox_part);
    hipLaunchKernelGGL(k_morton, dim3((n + 255) / 256), dim3(256), 0, st, X, n, m, bits, bbox_part, nb, code, vals);
    return hipGetLastError();
}

hipError_t launch_spatial_layout(const float* X, int n, int m, const int32_t* perm, float* Xs, float* tbox,
                                 float* sbox, hipStream_t st)
{
    gather_rows(X, n, m, perm, Xs, st);
    const int nt = spatial_tiles(n), ns = spatial_superblocks(n);
    hipLaunchKernelGGL(k_group_boxes, dim3((nt * m + 255) / 256), dim3(256), 0, st, Xs, n, m, TILE, nt, 0, tbox);
    hipLaunchKernelGGL(k_group_boxes, dim3((ns * m + 255) / 256), dim3(256), 0, st, tbox, nt, m, SB_TILES, ns, 1,
                       sbox);
    return hipGetLastError();
}

template <int M, int R>
static hipError_t launch_select_m(const SpatialView& sv, int n, int kp, uint64_t* keys, float* slast,
                                  unsigned long long* pairs, hipStream_t st)
{
    const int rows_per_block = 4 * R;
    const dim3 grid((n + rows_per_block - 1) / rows_per_block), block(256);
    if (kp <= 64)
        hipLaunchKernelGGL((k_select_direct<M, R, 1>), grid, block, 0, st, sv, n, kp, keys, slast, pairs);
    else if (kp <= 128)
        hipLaunchKernelGGL((k_select_direct<M, R, 2>), grid, block, 0, st, sv, n, kp, keys, slast, pairs);
    else
        hipLaunchKernelGGL((k_select_direct<M, R, 4>), grid, block, 0, st, sv, n, kp, keys, slast, pairs);
    return hipGetLastError();
}

hipError_t launch_select_direct(const float* Xs, const float* tbox, const float* sbox, int n, int m, int kp,
                                uint64_t* keys, float* slast, unsigned long long* pairs, hipStream_t st)
{
    const SpatialView sv = {Xs, tbox, sbox};
    // five rows per wavefront up to m = 4: each tile's loads and box tests
    // serve more rows than at four, while the rows' union of near tiles stays
    // small (torus, n = 100k: 438 us at 4 rows, 357 at 5, 365 at 6, 379 at 7);
    // four beyond, where a fifth row's coordinates and list would spill
    switch (m) {
    case 1: return launch_select_m<1, 5>(sv, n, kp, keys, slast, pairs, st);
    case 2: return launch_select_m<2, 5>(sv, n, kp, keys, slast, pairs, st);
    case 3: return launch_select_m<3, 5>(sv, n, kp, keys, slast, pairs, st);
    case 4: return launch_select_m<4, 5>(sv, n, kp, keys, slast, pairs, st);
    case 5: return launch_select_m<5, 4>(sv, n, kp, keys, slast, pairs, st);
    case 6: return launch_select_m<6, 4>(sv, n, kp, keys, slast, pairs, st);
    case 7: return launch_select_m<7, 4>(sv, n, kp, keys, slast, pairs, st);
    case 8: return launch_select_m<8, 4>(sv, n, kp, keys, slast, pairs, st);
    default: return hipErrorInvalidValue;
    }
}

template <int LPC, bool CV>
static void launch_refine_l(const float* X, int n, int m, int k, int kp, int kstride, const uint64_t* keys,
                            const float* slast, float lb_scale, int32_t* idx, float* d2, int32_t* flags, int* fb_count,
                            int* fb_list, float* fb_bound, int force_period, const float* Xs, const int32_t* perm,
                            hipStream_t st)
{
    const dim3 grid((n + 3) / 4), block(256);
    if (kp <= 64)
        hipLaunchKernelGGL((k_refine<1, LPC, CV>), grid, block, 0, st, X, n, m, k, kp, kstride, keys, slast, lb_scale,
                           idx, d2, flags, fb_count, fb_list, fb_bound, force_period, Xs, perm);
    else if (kp <= 128)
        hipLaunchKernelGGL((k_refine<2, LPC, CV>), grid, block, 0, st, X, n, m, k, kp, kstride, keys, slast, lb_scale,
                           idx, d2, flags, fb_count, fb_list, fb_bound, force_period, Xs, perm);
    else
        hipLaunchKernelGGL((k_refine<4, LPC, CV>), grid, block, 0, st, X, n, m, k, kp, kstride, keys, slast, lb_scale,
                           idx, d2, flags, fb_count, fb_list, fb_bound, force_period, Xs, perm);
}

hipError_t launch_refine(const float* X, int n, int m, int k, int kp, int kstride, const uint64_t* keys,
                         const float* slast, float lb_scale, int32_t* idx, float* d2, int32_t* flags,
                         int* fb_count, int* fb_list, float* fb_bound, int force_period, const float* Xs,
                         const int32_t* perm, hipStream_t st)
{
    // rows of up to 24 floats stay with one lane per candidate; longer rows are
    // read by groups of lanes, each lane covering up to 4 float4 pieces (the
    // fewest lanes per candidate: more candidates per pass, fewer passes and
    // shorter group reductions)
#define KVB_REFINE(LPC)                                                                                              \
    do {                                                                                                              \
        if (perm)                                                                                                     \
            launch_refine_l<LPC, true>(X, n, m, k, kp, kstride, keys, slast, lb_scale, idx, d2, flags, fb_count,     \
                                       fb_list, fb_bound, force_period, Xs, perm, st);                                \
        else                                                                                                          \
            launch_refine_l<LPC, false>(X, n, m, k, kp, kstride, keys, slast, lb_scale, idx, d2, flags, fb_count,    \
                                        fb_list, fb_bound, force_period, nullptr, nullptr, st);                       \
    } while (0)
    if (m <= 24)
        KVB_REFINE(0);
    else if (m <= 64)
        KVB_REFINE(4);
    else if (m <= 128)
        KVB_REFINE(8);
    else if (m <= 256)
        KVB_REFINE(16);
    else if (m <= 1024)
        KVB_REFINE(64);
    else
        return hipErrorInvalidValue;
#undef KVB_REFINE
    return hipGetLastError();
}

hipError_t launch_gather_rows(const float* X, int n, int m, const int32_t* perm, float* Xs, hipStream_t st)
{
    gather_rows(X, n, m, perm, Xs, st);
    return hipGetLastError();
}

int fallback_rows_cap(int n) { return n < FB_MAX_ROWS ? n : FB_MAX_ROWS; }

hipError_t launch_fallback(const float* X, int n, int m, int k, const int* fb_count, const int* fb_list,
                           const FallbackWork& fw, int32_t* idx, float* d2, hipStream_t st)
{
    if (m > 1024) return hipErrorInvalidValue;
    const int cap = fallback_rows_cap(n);
    hipError_t e = hipMemsetAsync(fw.cnt, 0, static_cast<size_t>(cap) * sizeof(int), st);
    if (e != hipSuccess) return e;
    if (m <= FB_REG_M) {
        const int waves = (n + WAVE - 1) / WAVE, blocks = (waves + FB_THREADS / WAVE - 1) / (FB_THREADS / WAVE);
        hipLaunchKernelGGL(k_fb_collect_reg, dim3(blocks < 2048 ? blocks : 2048), dim3(FB_THREADS),
                           fb_collect_reg_bytes(), st, X, n, m, fb_count, fb_list, fw.bound, cap, fw.cnt, fw.bd,
                           fw.bj);
    } else if (m <= FB_LDS_M) {
        const int stages = (n + FB_STAGE - 1) / FB_STAGE;
        hipLaunchKernelGGL(k_fb_collect_lds, dim3(stages < 2048 ? stages : 2048), dim3(FB_THREADS),
                           fb_collect_lds_bytes(m), st, X, n, m, fb_count, fb_list, fw.bound, cap, fw.cnt, fw.bd,
                           fw.bj);
    } else {
        const int chunks = (n + FB_CHUNK - 1) / FB_CHUNK;
        hipLaunchKernelGGL(k_fb_collect, dim3(chunks < 2048 ? chunks : 2048), dim3(FB_THREADS), 0, st, X, n, m,
                           fb_count, fb_list, fw.bound, cap, fw.cnt, fw.bd, fw.bj);
    }
    hipLaunchKernelGGL(k_fallback, dim3(512), dim3(FB_THREADS), 0, st, X, n, m, k, fb_count, 0, fb_list, 0, cap,
                       fw.cnt, fw.bd, fw.bj, idx, d2);
    return hipGetLastError();
}

hipError_t launch_exact_rows(const float* X, int n, int m, int k, const int* rows, int nrows, int32_t* idx, float* d2,
                             hipStream_t st)
{
    if (nrows <= 0) return hipSuccess;
    const int grid = nrows < 1024 ? nrows : 1024;
    hipLaunchKernelGGL(k_fallback, dim3(grid), dim3(FB_THREADS), 0, st, X, n, m, k, nullptr, nrows, rows, 1, 0,
                       nullptr, nullptr, nullptr, idx, d2);
    return hipGetLastError();
}

}  // namespace kvb
