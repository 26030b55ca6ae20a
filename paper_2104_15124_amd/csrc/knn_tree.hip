// Exact k-NN selection over curve-ordered matrix-core tiles, pruned by a tree
// of projected boxes (gfx950).
//
// The samples are laid out in the Morton order of their principal projections,
// refined by median splits inside groups of 4096 tiles (spatial_mfma.hip), so
// 32 consecutive positions form a compact tile and 64 consecutive tiles (or
// tree nodes) form a compact node of the level above. One wavefront owns one
// tile of 32 queries and works alone: no workgroup barrier, no shared
// candidate stage. Its scan has two phases.
//
// Fill. The CAP / 32 tiles around its own tile (CAP = the list capacity) are
// scored and written into the query lists in global scratch, which are then
// sorted once; each query's threshold is its list's kp-th score.
//
// Tree walk. From the top level down: a node's (up to 64) children are
// bounded at once, one per lane, against the wavefront's own query box (the
// box of its tile), and a ballot against the wavefront's largest distance
// threshold keeps those within reach. Among a node's pending children the one
// with the smallest bound is taken first (so the thresholds fall early), and
// every child is re-tested against the current threshold when taken, so the
// walk tightens as the lists improve. Every tile
// reached is one 32 x 32 matrix-core product of the query fragments
// (registers) and the candidate fragments (read from the tile-major operand;
// the reads of the next two tiles are issued before the current tile's
// products). A
// score at or below its query's threshold is
// appended to the query's LDS buffer, which is merged into the list when it
// may not absorb another tile (the same merge as the workgroup scans); a
// tile with no such score costs one compare per pair. The climb to the next
// group of tiles is rare and is a call of its own.
//
// A tile is skipped only when the bound of its box to the query box exceeds
// the wavefront's largest threshold at that time, which bounds every one of
// its queries' final thresholds; the certificate epilogue of the workgroup
// scans (knn_mfma.hip) therefore holds unchanged: every candidate missing from
// a list has a score at or above the list's last.
#include "knn_mfma_common.h"

namespace kvb {

namespace {

constexpr int TW = 4;        // wavefronts per workgroup (independent)
constexpr int TBUF = 32;     // per-query LDS buffer entries
// one tile adds up to 32 keys to a query's buffer right after its merge
static_assert(TBUF >= 32, "a query's buffer must absorb a whole tile");
constexpr int TNQ = 32;      // queries per wavefront

// one wavefront's LDS state
struct TreeLds {
    uint64_t buf[TNQ][TBUF];            // per-query buffers of appended keys
    float tau[TNQ];                     // score thresholds (the lists' kp-th scores; -inf: no query)
    float yq[TNQ];                      // |y_q|^2
    float thr[TNQ];                     // distance thresholds (score + |y_q|^2, rounded up)
    float box[2 * PR_DIMS];             // the query tile's box
    float bnd[TREE_LEVELS - 1][WAVE];   // walk: bounds of the pending children of level l >= 1 in row l - 1
    uint64_t mask[TREE_LEVELS];         //       pending children
    int base[TREE_LEVELS];              //       first child
    int lvl;                            //       level of the current pending list
};

// the same, through a pointer in the LDS address space (ds_* instructions in
// the functions that receive a wavefront's state by pointer)
typedef __attribute__((address_space(3))) TreeLds TreeLdsL;

// the tree's shape, shared by the workgroup
struct TreeShape {
    int top;
    int cnt[TREE_LEVELS];
    int off[TREE_LEVELS];
};

// The lane of `m` holding the smallest bound (bounds are >= 0, so their bits
// order like unsigned integers; the low 6 bits carry the lane, which breaks
// ties towards the lower lane and costs a relative 2^-17 of resolution).
__device__ __forceinline__ int nearest_lane(uint64_t m, float bound)
{
    const int lane = lane_id();
    uint32_t key = ((m >> lane) & 1ull) ? ((__float_as_uint(bound) & ~63u) | static_cast<uint32_t>(lane)) : ~0u;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) key = min(key, xor_lane(key, o));
    return static_cast<int>(__builtin_amdgcn_readfirstlane(key) & 63u);
}

__device__ __forceinline__ const float* node_box(const float* tbox, const float* tree, const TreeShape* sh, int level,
                                                 int v)
{
    return level == 0 ? tbox + static_cast<size_t>(v) * 2 * PR_DIMS
                      : tree + (static_cast<size_t>(sh->off[level]) + v) * 2 * PR_DIMS;
}

// A group of up to 64 tiles (level 0), one per lane: first tile, pending
// tiles and each lane's tile bound. base < 0: the walk is over.
struct TileGroup {
    uint64_t mask;
    int base;
    float bnd;
};

// Bounds of the children first .. first + 63 of level `level` to the query box
// (the tiles of the fill range [f0, f0 + nfill) are left out).
__device__ __forceinline__ float child_bound(const float* tbox, const float* tree, const TreeShape* sh, int level,
                                            int first, const float* qbox, BoxBound bb, int f0, int nfill, bool& take)
{
    const int lane = lane_id();
    const int v = first + lane;
    take = lane < min(TREE_FAN, sh->cnt[level] - first);
    if (level == 0) take = take && (v < f0 || v >= f0 + nfill);
    return take ? box_bound(node_box(tbox, tree, sh, level, v), qbox, qbox + PR_DIMS, bb) : __builtin_nanf("");
}

// The next group of tiles within reach of thr, after the current one is
// exhausted: up the levels until a pending child within reach, the nearest
// one taken, then down to its tiles. Whole wavefront.
__device__ __forceinline__ TileGroup climb(TreeLds* Wg, const TreeShape* sh, const float* tbox, const float* tree,
                                        BoxBound bb, float thr, int f0, int nfill)
{
    TreeLdsL* W = (TreeLdsL*)Wg;
    const int lane = lane_id();
    int lvl = W->lvl;
    if (lvl == 0) {
        if (sh->top == 0) return {0ull, -1, 0.f};
        lvl = 1;
    }
    while (true) {
        const float bl = W->bnd[lvl - 1][lane];
        const uint64_t m = W->mask[lvl] & __ballot(bl <= thr);
        if (!m) {
            if (lvl == sh->top) {
                W->lvl = lvl;
                return {0ull, -1, 0.f};
            }
            ++lvl;
            continue;
        }
        const int c = nearest_lane(m, bl);
        const int first = (W->base[lvl] + c) * TREE_FAN;
        wave_lds_sync();
        if (lane == 0) W->mask[lvl] = m & ~(1ull << c);
        bool take;
        float qb[2 * PR_DIMS];
#pragma unroll
        for (int c2 = 0; c2 < 2 * PR_DIMS; ++c2) qb[c2] = W->box[c2];
        const float b = child_bound(tbox, tree, sh, lvl - 1, first, qb, bb, f0, nfill, take);
        const uint64_t mt = __ballot(take);
        --lvl;
        if (lvl == 0) {
            wave_lds_sync();
            if (lane == 0) W->lvl = 0;
            wave_lds_sync();
            return {mt, first, b};
        }
        W->bnd[lvl - 1][lane] = b;
        if (lane == 0) {
            W->mask[lvl] = mt;
            W->base[lvl] = first;
        }
        wave_lds_sync();
    }
}

}  // namespace

// Waves per SIMD the register file allows: the query fragments and the two
// candidate tile buffers (3 KS fragments) dominate the kernel's registers.
// Tiles in flight: three. The third one's fragments (KS x fragment
// registers) can cost a wavefront per SIMD, and that still pays: on the 8M
// mixture the BF16 select at three tiles and three wavefronts per SIMD
// measured 126 ms against 131 ms at two tiles and four; a fourth tile
// measured no faster than three.
template <class Tr, int KS>
constexpr int tree_depth()
{
    return 3;
}

template <class Tr, int KS>
constexpr int tree_waves()
{
    constexpr int fr = 3 * KS * static_cast<int>(sizeof(typename Tr::frag) / 4);
    return fr <= 32 ? 4 : fr <= 64 ? 3 : 2;
}

template <class Tr, int KS, int E>
__global__ __launch_bounds__(64 * TW, (tree_waves<Tr, KS>())) void k_select_tree(
    const typename Tr::elem* __restrict__ Aq, const typename Tr::elem* __restrict__ Bc, int n, int kp,
    const float* __restrict__ ynorm2, const unsigned* __restrict__ rmax_bits, ErrModel em,
    uint64_t* __restrict__ lists, float* __restrict__ lb_out, CurveArgs crv,
    unsigned long long* __restrict__ pair_count)
{
    using elem = typename Tr::elem;
    using frag = typename Tr::frag;
    constexpr int CAP = WAVE * E;
    constexpr int kpad = KS * Tr::KSTEP;
    constexpr int FILL = CAP / 32;
    constexpr float INF = __builtin_inff();
    __shared__ TreeLds s_w[TW];
    __shared__ TreeShape s_shape;

    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int half = lane >> 5, l31 = lane & 31;
    if (threadIdx.x == 0) {
        s_shape.top = crv.layout.top;
        for (int l = 0; l < TREE_LEVELS; ++l) {
            s_shape.cnt[l] = crv.layout.cnt[l];
            s_shape.off[l] = crv.layout.off[l];
        }
    }
    __syncthreads();   // the only workgroup barrier: before any wavefront may leave
    const int ntiles = crv.layout.cnt[0];
    const int t0 = xcd_block() * TW + wave;     // this wavefront's query tile
    if (t0 >= ntiles) return;
    TreeLds& W = s_w[wave];
    const int q0 = t0 * TNQ;
    const int nq_valid = min(TNQ, n - q0);
    uint64_t* lists_q0 = lists + static_cast<size_t>(q0) * CAP;

    // query fragments: curve position q0 + l31 (the last tile's padding rows
    // repeat a real row; their results are never stored)
    frag qa[KS];
    {
        const elem* src = Aq + static_cast<size_t>(min(q0 + l31, n - 1)) * kpad + half * Tr::VEC;
#pragma unroll
        for (int s = 0; s < KS; ++s) qa[s] = Tr::load(src + s * Tr::KSTEP);
    }
    if (lane < 2 * PR_DIMS) W.box[lane] = crv.tbox[static_cast<size_t>(t0) * 2 * PR_DIMS + lane];
    if (lane < TNQ) {
        W.yq[lane] = q0 + lane < n ? ynorm2[q0 + lane] : 0.f;
        W.tau[lane] = -INF;
    }
    wave_lds_sync();
    BoxBound bb;
    {
        const float R = __uint_as_float(*rmax_bits);
        bb.zerr = crv.zcoef * R;
        bb.pscale = *crv.pscale;
        bb.yerr = crv.ycoef * R;
    }

    auto load_tile = [&](int t, frag (&b)[KS]) {
        const elem* src = Bc + static_cast<size_t>(t) * 32 * kpad + (half * 32 + l31) * Tr::VEC;
#pragma unroll
        for (int s = 0; s < KS; ++s) b[s] = Tr::load(src + s * 64 * Tr::VEC);
    };
    // one accumulator chain (the wavefronts sharing a SIMD cover its latency)
    auto product = [&](const frag (&b)[KS]) {
        f32x16 a = {};
#pragma unroll
        for (int s = 0; s < KS; ++s) a = Tr::mma(qa[s], b[s], a);
        return a;
    };

    unsigned long long pairs = 0;

    // ---- fill: the FILL tiles around the own tile, written straight into the lists
    const int nfill = min(FILL, ntiles);
    const int f0 = max(0, min(t0 - (FILL / 2 - 1), ntiles - nfill));
    for (int i = 0; i < FILL; ++i) {
        const bool real = i < nfill;
        f32x16 acc = {};
        if (real) {
            frag b[KS];
            load_tile(f0 + i, b);
            acc = product(b);
        }
        const int cand = (f0 + i) * 32 + l31;
        const bool valid = real && cand < n;
        if (real) pairs += static_cast<unsigned long long>(nq_valid) * __popcll(__ballot(valid) & 0xFFFFFFFFull);
        const int slot = i * 32 + l31;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int q = acc_row(r, half);
            if (q < nq_valid)
                lists_q0[static_cast<size_t>(q) * CAP + slot] =
                    valid ? make_key(acc[r], static_cast<uint32_t>(cand)) : KEY_INF;
        }
    }
    // the lists' stores complete before other lanes read them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // each list sorted in place, the next one's loads in flight meanwhile
    // (the 256-key lists keep the plain loop: their inline sort would spill)
    if constexpr (E > 2) {
        for (int q = 0; q < nq_valid; ++q) {
            const float nt = sort_query_list<E>(lists_q0 + static_cast<size_t>(q) * CAP, kp);
            if (lane == 0) W.tau[q] = nt;
        }
    } else {
        uint64_t Ln[E];
#pragma unroll
        for (int s = 0; s < E; ++s) Ln[s] = lists_q0[s * WAVE + lane];
        for (int q = 0; q < nq_valid; ++q) {
            uint64_t L[E];
#pragma unroll
            for (int s = 0; s < E; ++s) L[s] = Ln[s];
            if (q + 1 < nq_valid) {
#pragma unroll
                for (int s = 0; s < E; ++s) Ln[s] = lists_q0[static_cast<size_t>(q + 1) * CAP + s * WAVE + lane];
            }
            bitonic_sort<E>(L);
#pragma unroll
            for (int s = 0; s < E; ++s) lists_q0[static_cast<size_t>(q) * CAP + s * WAVE + lane] = L[s];
            const float nt = key_dist(list_at<E>(L, kp - 1));
            if (lane == 0) W.tau[q] = nt;
        }
    }
    wave_lds_sync();

    // each query's distance threshold (score + |y_q|^2, rounded up) and the
    // wavefront's largest
    auto dist_threshold = [](float score, float yq) { return fmaxf(score + yq, 0.f) * (1.f + 4.8e-7f); };
    if (lane < TNQ) W.thr[lane] = lane < nq_valid ? dist_threshold(W.tau[lane], W.yq[lane]) : -INF;
    wave_lds_sync();
    // (read from one lane, so that the compiler sees a wave-uniform value and
    // keeps the branches on it, and the state they update, scalar)
    auto wave_threshold = [&]() {
        const float t = wave_max_f32(lane < TNQ ? W.thr[lane] : -INF);
        return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(t)));
    };
    float wthr = wave_threshold();

    // ---- tree walk: the current group of tiles in registers, the levels above in LDS
    TileGroup g = {0ull, 0, __builtin_nanf("")};
    if (s_shape.top == 0) {
        bool take;
        g.bnd = child_bound(crv.tbox, crv.tree, &s_shape, 0, 0, W.box, bb, f0, nfill, take);
        g.mask = __ballot(take);
        if (lane == 0) W.lvl = 0;
    } else {
        bool take;
        const int top = s_shape.top;
        W.bnd[top - 1][lane] = child_bound(crv.tbox, crv.tree, &s_shape, top, 0, W.box, bb, f0, nfill, take);
        const uint64_t mt = __ballot(take);
        if (lane == 0) {
            W.mask[top] = mt;
            W.base[top] = 0;
            W.lvl = top;
        }
    }
    wave_lds_sync();
    // next tile within reach of thr (and its bound), or -1
    auto next_tile = [&](float thr, float& tb) -> int {
        while (true) {
            const uint64_t m = g.mask & __ballot(g.bnd <= thr);
            if (m) {
                const int c = nearest_lane(m, g.bnd);
                g.mask = m & ~(1ull << c);
                tb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g.bnd), c));
                return g.base + c;
            }
            g = climb(&W, &s_shape, crv.tbox, crv.tree, bb, thr, f0, nfill);
            if (g.base < 0) return -1;
        }
    };

    // the thresholds in registers: this lane's accumulator register r holds row acc_row(r, half)
    float tauv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) tauv[r] = W.tau[acc_row(r, half)];
    // the buffers' fill, wave-uniform: query q's count in byte q % 4 of cntw[q / 4]
    // (every index below is a compile-time constant, so they stay in scalar registers)
    uint32_t cntw[TNQ / 4];
#pragma unroll
    for (int i = 0; i < TNQ / 4; ++i) cntw[i] = 0u;
    auto cnt_of = [&](int q) { return static_cast<int>((cntw[q >> 2] >> (8 * (q & 3))) & 0xFFu); };
    bool thr_dirty = false;
    // the tiles' fragments stream into registers DEPTH - 1 tiles ahead of
    // the products (a tile with no hits is too short to cover the latency
    // of the next one's loads)
    constexpr int DEPTH = tree_depth<Tr, KS>();
    int tq[DEPTH];        // the tiles in flight, the current one first (-1: none)
    float tbq[DEPTH];     // their bounds when taken
    frag bq[DEPTH][KS];   // their fragments
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) {
        tq[d] = -1;
        tbq[d] = 0.f;
#pragma unroll
        for (int s = 0; s < KS; ++s) bq[d][s] = {};
    }
    tq[0] = next_tile(wthr, tbq[0]);
    if (tq[0] >= 0) load_tile(tq[0], bq[0]);
#pragma unroll
    for (int d = 1; d + 1 < DEPTH; ++d) {
        if (tq[d - 1] >= 0) tq[d] = next_tile(wthr, tbq[d]);
        if (tq[d] >= 0) load_tile(tq[d], bq[d]);
    }
    while (tq[0] >= 0) {
        if (thr_dirty) {
            wthr = wave_threshold();
            thr_dirty = false;
        }
        tq[DEPTH - 1] = tq[DEPTH - 2] >= 0 ? next_tile(wthr, tbq[DEPTH - 1]) : -1;
        if (tq[DEPTH - 1] >= 0) load_tile(tq[DEPTH - 1], bq[DEPTH - 1]);
        const int cur = tq[0];
        const float tb_cur = tbq[0];
        // the current tile may have fallen out of reach since it was taken
        if (tb_cur <= wthr) {
            f32x16 acc = product(bq[0]);
            const int cand = cur * 32 + l31;
            const bool valid = cand < n;
            pairs += static_cast<unsigned long long>(nq_valid) * __popcll(__ballot(valid) & 0xFFFFFFFFull);
            bool hit = false;
#pragma unroll
            for (int r = 0; r < 16; ++r) hit |= acc[r] <= tauv[r];
            if (__ballot(valid && hit)) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float sc = acc[r];
                    uint64_t mask = __ballot(valid && sc <= tauv[r]);
                    if (!mask) continue;
                    const int qa_ = acc_row(r, 0), qb_ = acc_row(r, 1);
                    int ca = cnt_of(qa_), cb = cnt_of(qb_);
                    const bool fa = ca + __popc(static_cast<uint32_t>(mask)) > TBUF;
                    const bool fb = cb + __popc(static_cast<uint32_t>(mask >> 32)) > TBUF;
                    if (fa || fb) {
                        // a full buffer is merged before this tile's keys are added
                        wave_lds_sync();
                        if (fa) {
                            const float nt = merge_query_list32<E>(lists_q0 + static_cast<size_t>(qa_) * CAP,
                                                                 &W.buf[qa_][0], ca, kp);
                            if (half == 0) tauv[r] = nt;
                            if (lane == 0) W.thr[qa_] = dist_threshold(nt, W.yq[qa_]);
                            ca = 0;
                            cntw[qa_ >> 2] &= ~(0xFFu << (8 * (qa_ & 3)));
                        }
                        if (fb) {
                            const float nt = merge_query_list32<E>(lists_q0 + static_cast<size_t>(qb_) * CAP,
                                                                 &W.buf[qb_][0], cb, kp);
                            if (half == 1) tauv[r] = nt;
                            if (lane == 0) W.thr[qb_] = dist_threshold(nt, W.yq[qb_]);
                            cb = 0;
                            cntw[qb_ >> 2] &= ~(0xFFu << (8 * (qb_ & 3)));
                        }
                        thr_dirty = true;
                        wave_lds_sync();
                        mask = __ballot(valid && sc <= tauv[r]);
                    }
                    const int pa = __popc(static_cast<uint32_t>(mask)), pb = __popc(static_cast<uint32_t>(mask >> 32));
                    // slot: the half's count plus the rank among the half's passing lanes
                    // (mbcnt64 counts the lower half's lanes too in the upper half)
                    const int slot0 = half ? qb_ * TBUF + cb - pa : qa_ * TBUF + ca;
                    if (valid && sc <= tauv[r]) (&W.buf[0][0])[slot0 + mbcnt64(mask)] = make_key(sc, static_cast<uint32_t>(cand));
                    cntw[qa_ >> 2] += static_cast<uint32_t>(pa) << (8 * (qa_ & 3));
                    cntw[qb_ >> 2] += static_cast<uint32_t>(pb) << (8 * (qb_ & 3));
                }
            }
        }
#pragma unroll
        for (int d = 0; d + 1 < DEPTH; ++d) {
            tq[d] = tq[d + 1];
            tbq[d] = tbq[d + 1];
#pragma unroll
            for (int s = 0; s < KS; ++s) bq[d][s] = bq[d + 1][s];
        }
    }

    wave_lds_sync();
    if constexpr (E > 2) {
#pragma unroll
        for (int q = 0; q < TNQ; ++q) {
            const int c = cnt_of(q);
            if (c > 0) {
                merge_query_list32<E>(lists_q0 + static_cast<size_t>(q) * CAP, &W.buf[q][0], c, kp);
                wave_lds_sync();
            }
        }
    } else {
        // the last merges, the next list's loads in flight meanwhile (query
        // q's buffer count moved to lane q, so that the loop need not be unrolled)
        int cnt_lane = 0;
#pragma unroll
        for (int q = 0; q < TNQ; ++q)
            if (lane == q) cnt_lane = cnt_of(q);
        uint64_t Ln[E];
#pragma unroll
        for (int s = 0; s < E; ++s) Ln[s] = lists_q0[s * WAVE + lane];
        for (int q = 0; q < nq_valid; ++q) {
            const int c = __builtin_amdgcn_readlane(cnt_lane, q);
            uint64_t L[E];
#pragma unroll
            for (int s = 0; s < E; ++s) L[s] = Ln[s];
            if (q + 1 < nq_valid) {
#pragma unroll
                for (int s = 0; s < E; ++s) Ln[s] = lists_q0[static_cast<size_t>(q + 1) * CAP + s * WAVE + lane];
            }
            if (c > 0) {
                uint64_t B[1] = {lane >= 32 && lane - 32 < c ? W.buf[q][lane - 32] : KEY_INF};
#pragma unroll
                for (int kb = 2; kb <= 32; kb <<= 1) {
#pragma unroll
                    for (int j = kb >> 1; j > 0; j >>= 1) cx_lanes<1>(B, kb, j, lane);
                }
                L[E - 1] = umin64(L[E - 1], B[0]);
                bitonic_merge_asc<E>(L);
#pragma unroll
                for (int s = 0; s < E; ++s) lists_q0[static_cast<size_t>(q) * CAP + s * WAVE + lane] = L[s];
            }
            // the list's kp-th score, for the certificate below
            const float sl = key_dist(list_at<E>(L, kp - 1));
            if (lane == 0) W.tau[q] = sl;
        }
        wave_lds_sync();
    }
    if (pair_count && lane == 0) atomicAdd(pair_count, pairs);

    // certificate lower bound for the candidates left out of each list (the
    // derivation is that of the workgroup scans in knn_mfma.hip)
    const double R = static_cast<double>(__uint_as_float(*rmax_bits));
    if (lane < nq_valid) {
        const int qg = q0 + lane;
        const float sl = E > 2 ? key_dist(lists[static_cast<size_t>(qg) * CAP + (kp - 1)]) : W.tau[lane];
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

// ------------------------------------------------------------------ launcher
template <class Tr, int KS>
static hipError_t launch_tree(const void* Aq, const void* Bc, int n, int kp, const float* ynorm2, const unsigned* rmax,
                              ErrModel em, uint64_t* lists, int cap, float* lb, const CurveArgs& crv,
                              unsigned long long* pairs, hipStream_t st)
{
    using elem = typename Tr::elem;
    if (kp > cap || (cap != 128 && cap != 256)) return hipErrorInvalidValue;
    const int ntiles = (n + 31) / 32;
    if (crv.layout.cnt[0] != ntiles) return hipErrorInvalidValue;
    const dim3 grid((ntiles + TW - 1) / TW), block(64 * TW);
    const elem* A = static_cast<const elem*>(Aq);
    const elem* B = static_cast<const elem*>(Bc);
    if (cap == 128)
        hipLaunchKernelGGL((k_select_tree<Tr, KS, 2>), grid, block, 0, st, A, B, n, kp, ynorm2, rmax, em, lists, lb,
                           crv, pairs);
    else
        hipLaunchKernelGGL((k_select_tree<Tr, KS, 4>), grid, block, 0, st, A, B, n, kp, ynorm2, rmax, em, lists, lb,
                           crv, pairs);
    return hipGetLastError();
}

bool select_tree_fits(int split, int kpad)
{
    // the walk keeps the query fragments and three tile slots in registers;
    // beyond 80 fragment registers it would fall to two wavefronts per SIMD
    // (and spill), where the workgroup scans' LDS-staged tiles do better
    const int ks = kpad / mfma_kstep(split);
    const int fr = split == 0 ? 1 : 4;
    return 4 * ks * fr <= 80;
}

#define KVB_TREE_CASE(TR, K) \
    case K: return launch_tree<TR, K>(Aq, Bc, n, kp, ynorm2, rmax, em, lists, cap, lb, crv, pairs, st);

hipError_t launch_select_tree(int split, const void* Aq, const void* Bc, int n, int kpad, int kp, const float* ynorm2,
                              const unsigned* rmax, ErrModel em, uint64_t* lists, int cap, float* lb,
                              const CurveArgs& crv, unsigned long long* pairs, hipStream_t st)
{
    const int ks = kpad / mfma_kstep(split);
    if (split == 0) {
        switch (ks) {
            KVB_TREE_CASE(TraitsF32, 2)
            KVB_TREE_CASE(TraitsF32, 4)
            KVB_TREE_CASE(TraitsF32, 6)
            KVB_TREE_CASE(TraitsF32, 8)
            KVB_TREE_CASE(TraitsF32, 10)
            KVB_TREE_CASE(TraitsF32, 12)
            KVB_TREE_CASE(TraitsF32, 16)
        default: return hipErrorInvalidValue;
        }
    }
    switch (ks) {
        KVB_TREE_CASE(TraitsBF16, 2)
        KVB_TREE_CASE(TraitsBF16, 3)
        KVB_TREE_CASE(TraitsBF16, 4)
        KVB_TREE_CASE(TraitsBF16, 5)
    default: return hipErrorInvalidValue;
    }
}
#undef KVB_TREE_CASE

}  // namespace kvb
