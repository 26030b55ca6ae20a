// Entry points of the learned partitioner and the routed k-NN search.
//
// The partitioner is an MLP m -> h1 -> h2 -> nb (ReLU) whose argmax over nb
// buckets places each sample in one bucket and whose n_probe largest logits
// choose the buckets a query searches. Training follows the neighbour-
// histogram recipe of Neural LSH (Dong, Indyk, Razenshteyn and Wagner, ICLR
// 2020): a balanced teacher partition of a subsample, and for every training
// sample a soft target equal to the distribution of its exact neighbours over
// the teacher's buckets, fitted by softmax cross-entropy with Adam.
//
// The routed search reuses the matrix-core distance tiles: samples are laid
// out bucket by bucket (each bucket padded to whole 32-row tiles), and for
// each probe slot every bucket's queries scan only that bucket's tiles,
// merging into one running top-(k + margin) list per query. The exact
// re-rank and the float64 boundary decision then run as in the exact modes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "kvb_ctx.h"

using namespace kvbh;

namespace {

constexpr float kAdamB1 = 0.9f, kAdamB2 = 0.999f, kAdamEps = 1e-8f;
constexpr int kRouteChunk = 32768;   // rows per MLP inference chunk

uint64_t host_splitmix(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t gcd_u64(uint64_t a, uint64_t b)
{
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

int ceil_log2(int v)
{
    int b = 0;
    while ((1 << b) < v) ++b;
    return b;
}

int part_alloc(kvb_ctx ctx, int m, int h1, int h2, int nb, int np)
{
    KVB_DEVICE_WORK(ctx);
    part_free(ctx);
    PartState& P = ctx->part;
    P.m = m;
    P.mpad = (m + 31) / 32 * 32;
    P.h1 = h1;
    P.h2 = h2;
    P.nb = nb;
    P.np = np;
    P.off[0] = 0;
    P.off[1] = int64_t(h1) * P.mpad;
    P.off[2] = P.off[1] + h1;
    P.off[3] = P.off[2] + int64_t(h2) * h1;
    P.off[4] = P.off[3] + h2;
    P.off[5] = P.off[4] + int64_t(nb) * h2;
    P.total = (P.off[5] + nb + 63) / 64 * 64;
    const size_t fbytes = round256(size_t(P.total) * sizeof(float));
    const size_t bytes = 4 * fbytes + round256(size_t(P.total) * 2) + round256(size_t(h1) * h2 * 2) +
                         round256(size_t(h2) * nb * 2);
    void* blk = nullptr;
    if (hipMalloc(&blk, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, KVB_E_NOMEM, "hipMalloc of %zu partitioner bytes failed", bytes);
    }
    P.block = blk;
    Carve cv(blk);
    P.p = cv.take<float>(P.total);
    P.m1 = cv.take<float>(P.total);
    P.m2 = cv.take<float>(P.total);
    P.g = cv.take<float>(P.total);
    P.pb = cv.take<uint16_t>(P.total);
    P.w2t = cv.take<uint16_t>(size_t(h1) * h2);
    P.w3t = cv.take<uint16_t>(size_t(h2) * nb);
    KVB_HIP(ctx, hipMemsetAsync(blk, 0, bytes, ctx->stream));
    P.step = 0;
    return KVB_OK;
}

// BF16 copy of the parameters and the transposed weights used by the backward GEMMs.
int refresh_bf16(kvb_ctx ctx)
{
    PartState& P = ctx->part;
    KVB_HIP(ctx, kvb::launch_cast_bf16(P.p, P.total, P.pb, ctx->stream));
    KVB_HIP(ctx, kvb::launch_transpose_bf16(P.pb + P.off[2], P.h2, P.h1, P.w2t, ctx->stream));
    KVB_HIP(ctx, kvb::launch_transpose_bf16(P.pb + P.off[4], P.nb, P.h2, P.w3t, ctx->stream));
    return KVB_OK;
}

// Padded flat layout <-> the exported compact order W1 [h1, m], b1, W2, b2, W3, b3.
int copy_params(kvb_ctx ctx, const float* src, float* dst, bool to_compact)
{
    PartState& P = ctx->part;
    const size_t m = P.m, mp = P.mpad;
    const int64_t rest = P.off[5] + P.nb - P.off[1];
    if (to_compact) {
        KVB_HIP(ctx, hipMemcpy2DAsync(dst, m * 4, src, mp * 4, m * 4, P.h1, hipMemcpyDeviceToDevice, ctx->stream));
        KVB_HIP(ctx, hipMemcpyAsync(dst + int64_t(P.h1) * P.m, src + P.off[1], rest * 4, hipMemcpyDeviceToDevice,
                                    ctx->stream));
    } else {
        KVB_HIP(ctx, hipMemcpy2DAsync(dst, mp * 4, src, m * 4, m * 4, P.h1, hipMemcpyDeviceToDevice, ctx->stream));
        KVB_HIP(ctx, hipMemcpyAsync(dst + P.off[1], src + int64_t(P.h1) * P.m, rest * 4, hipMemcpyDeviceToDevice,
                                    ctx->stream));
    }
    return KVB_OK;
}

// Activations of one batch of B rows (B a multiple of 32), carved from scratch.
struct Acts {
    uint16_t *Xb, *H1b, *H2b;
    float *H1f, *H2f, *Z;
    // backward only
    float *dZ, *dH2f, *dH1f;
    uint16_t *dZb, *dZT, *H2T, *dH2b, *dH2T, *H1T, *dH1b, *dH1T, *XbT;
    double* row_loss;
    int32_t *bidx, *nbrlab;
};

size_t acts_bytes(const PartState& P, int B, int ks, bool train)
{
    size_t s = round256(size_t(B) * P.mpad * 2) + round256(size_t(B) * P.h1 * 2) + round256(size_t(B) * P.h2 * 2) +
               round256(size_t(B) * P.nb * 4);
    if (train) {
        s += round256(size_t(B) * P.h1 * 4) + round256(size_t(B) * P.h2 * 4);
        s += round256(size_t(B) * P.nb * 4) + round256(size_t(B) * P.h2 * 4) + round256(size_t(B) * P.h1 * 4);
        s += 2 * round256(size_t(B) * P.nb * 2) + 3 * round256(size_t(B) * P.h2 * 2) +
             3 * round256(size_t(B) * P.h1 * 2) + round256(size_t(B) * P.mpad * 2);
        s += round256(size_t(B) * 8) + round256(size_t(B) * 4) + round256(size_t(B) * ks * 4);
    }
    return s + 256;
}

Acts carve_acts(Carve& cv, const PartState& P, int B, int ks, bool train)
{
    Acts a = {};
    a.Xb = cv.take<uint16_t>(size_t(B) * P.mpad);
    a.H1b = cv.take<uint16_t>(size_t(B) * P.h1);
    a.H2b = cv.take<uint16_t>(size_t(B) * P.h2);
    a.Z = cv.take<float>(size_t(B) * P.nb);
    if (train) {
        a.H1f = cv.take<float>(size_t(B) * P.h1);
        a.H2f = cv.take<float>(size_t(B) * P.h2);
        a.dZ = cv.take<float>(size_t(B) * P.nb);
        a.dH2f = cv.take<float>(size_t(B) * P.h2);
        a.dH1f = cv.take<float>(size_t(B) * P.h1);
        a.dZb = cv.take<uint16_t>(size_t(B) * P.nb);
        a.dZT = cv.take<uint16_t>(size_t(B) * P.nb);
        a.H2T = cv.take<uint16_t>(size_t(B) * P.h2);
        a.dH2b = cv.take<uint16_t>(size_t(B) * P.h2);
        a.dH2T = cv.take<uint16_t>(size_t(B) * P.h2);
        a.H1T = cv.take<uint16_t>(size_t(B) * P.h1);
        a.dH1b = cv.take<uint16_t>(size_t(B) * P.h1);
        a.dH1T = cv.take<uint16_t>(size_t(B) * P.h1);
        a.XbT = cv.take<uint16_t>(size_t(B) * P.mpad);
        a.row_loss = cv.take<double>(B);
        a.bidx = cv.take<int32_t>(B);
        a.nbrlab = cv.take<int32_t>(size_t(B) * ks);
    }
    return a;
}

// Forward pass over `valid` rows of X (gathered through idx if non-null),
// padded with zero rows to B: logits in a.Z. With train, float32 copies of
// the hidden activations are kept for the ReLU masks of the backward pass.
int mlp_forward(kvb_ctx ctx, const float* X, const int32_t* idx, int valid, int B, Acts& a, bool train)
{
    PartState& P = ctx->part;
    hipStream_t st = ctx->stream;
    KVB_HIP(ctx, kvb::launch_cast_rows_bf16(X, P.m, idx, valid, B, P.mpad, a.Xb, st));
    KVB_HIP(ctx, kvb::launch_gemm_nt(a.Xb, P.mpad, P.pb + P.off[0], P.mpad, B, P.h1, P.mpad, P.p + P.off[1], 1,
                                     nullptr, 0, train ? a.H1f : nullptr, P.h1, a.H1b, P.h1, st));
    KVB_HIP(ctx, kvb::launch_gemm_nt(a.H1b, P.h1, P.pb + P.off[2], P.h1, B, P.h2, P.h1, P.p + P.off[3], 1, nullptr,
                                     0, train ? a.H2f : nullptr, P.h2, a.H2b, P.h2, st));
    KVB_HIP(ctx, kvb::launch_gemm_nt(a.H2b, P.h2, P.pb + P.off[4], P.h2, B, P.nb, P.h2, P.p + P.off[5], 0, nullptr,
                                     0, a.Z, P.nb, nullptr, 0, st));
    return KVB_OK;
}

// Backward pass of the mean soft-target cross-entropy of a batch after
// mlp_forward(train = true): gradients of every parameter into P.g (padded
// layout); the batch's mean loss is added (add = 1) or stored into *loss_dev.
int mlp_backward(kvb_ctx ctx, int B, const int32_t* nbrlab, int ks, Acts& a, double* loss_dev, int add)
{
    PartState& P = ctx->part;
    hipStream_t st = ctx->stream;
    KVB_HIP(ctx, kvb::launch_softmax_xent(a.Z, B, P.nb, nbrlab, ks, a.dZ, a.dZb, a.row_loss, loss_dev, add, st));
    // layer 3: dW3 = dZ^T H2, db3 = colsum dZ, dH2 = (dZ W3) * [H2 > 0]
    KVB_HIP(ctx, kvb::launch_transpose_bf16(a.dZb, B, P.nb, a.dZT, st));
    KVB_HIP(ctx, kvb::launch_transpose_bf16(a.H2b, B, P.h2, a.H2T, st));
    KVB_HIP(ctx, kvb::launch_gemm_nt(a.dZT, B, a.H2T, B, P.nb, P.h2, B, nullptr, 0, nullptr, 0, P.g + P.off[4], P.h2,
                                     nullptr, 0, st));
    KVB_HIP(ctx, kvb::launch_colsum(a.dZ, B, P.nb, P.g + P.off[5], st));
    KVB_HIP(ctx, kvb::launch_gemm_nt(a.dZb, P.nb, P.w3t, P.nb, B, P.h2, P.nb, nullptr, 0, a.H2f, P.h2, a.dH2f, P.h2,
                                     a.dH2b, P.h2, st));
    // layer 2
    KVB_HIP(ctx, kvb::launch_transpose_bf16(a.dH2b, B, P.h2, a.dH2T, st));
    KVB_HIP(ctx, kvb::launch_transpose_bf16(a.H1b, B, P.h1, a.H1T, st));
    KVB_HIP(ctx, kvb::launch_gemm_nt(a.dH2T, B, a.H1T, B, P.h2, P.h1, B, nullptr, 0, nullptr, 0, P.g + P.off[2], P.h1,
                                     nullptr, 0, st));
    KVB_HIP(ctx, kvb::launch_colsum(a.dH2f, B, P.h2, P.g + P.off[3], st));
    KVB_HIP(ctx, kvb::launch_gemm_nt(a.dH2b, P.h2, P.w2t, P.h2, B, P.h1, P.h2, nullptr, 0, a.H1f, P.h1, a.dH1f, P.h1,
                                     a.dH1b, P.h1, st));
    // layer 1
    KVB_HIP(ctx, kvb::launch_transpose_bf16(a.dH1b, B, P.h1, a.dH1T, st));
    KVB_HIP(ctx, kvb::launch_transpose_bf16(a.Xb, B, P.mpad, a.XbT, st));
    KVB_HIP(ctx, kvb::launch_gemm_nt(a.dH1T, B, a.XbT, B, P.h1, P.mpad, B, nullptr, 0, nullptr, 0, P.g + P.off[0],
                                     P.mpad, nullptr, 0, st));
    KVB_HIP(ctx, kvb::launch_colsum(a.dH1f, B, P.h1, P.g + P.off[1], st));
    return KVB_OK;
}

int require_part(kvb_ctx ctx, int m)
{
    if (!ctx->part.ready) return fail(ctx, KVB_E_NOT_TRAINED, "no partitioner: call kvb_part_init or kvb_part_load");
    if (m >= 0 && m != ctx->part.m)
        return fail(ctx, KVB_E_INVALID, "m = %d does not match the partitioner's input dimension %d", m, ctx->part.m);
    return KVB_OK;
}

int ensure_loss(kvb_ctx ctx, int cnt)
{
    if (cnt <= ctx->loss_cap) return KVB_OK;
    KVB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->loss_dev) (void)hipFree(ctx->loss_dev);
    ctx->loss_dev = nullptr;
    ctx->loss_cap = 0;
    if (hipMalloc(reinterpret_cast<void**>(&ctx->loss_dev), size_t(cnt) * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, KVB_E_NOMEM, "hipMalloc of the loss buffer failed");
    }
    ctx->loss_cap = cnt;
    return KVB_OK;
}

struct FileCloser {
    FILE* f;
    ~FileCloser()
    {
        if (f) fclose(f);
    }
};

const char kMagic[8] = {'K', 'V', 'B', 'P', 'A', 'R', 'T', '1'};

}  // namespace

namespace kvbh {

void part_free(kvb_ctx ctx)
{
    PartState& P = ctx->part;
    if (P.block) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(P.block);
    }
    P = PartState();
}

int learned_knn(kvb_ctx ctx, const float* X, int n, int m, int k, int kp, int32_t* idx, float* d2, int32_t* row_flags)
{
    KVB_TRY(require_part(ctx, m));
    const PartState& P = ctx->part;
    KVB_REQUIRE(ctx, int64_t(n) * P.np < (int64_t(1) << 31), "n * n_probe must be below 2^31");
    const int split = ctx->bf16_split;
    const int cap = kp <= 128 ? 128 : 256;
    const int kraw = split * m + 3;
    const int kstep = kvb::mfma_kstep(split);
    const int ks = kvb::mfma_pick_ksteps(split, (kraw + kstep - 1) / kstep);
    if (ks < 0) return fail(ctx, KVB_E_UNSUPPORTED, "m = %d is too large for the BF16 distance tiles", m);
    const int kpad = ks * kstep;
    const size_t esz = sizeof(uint16_t);
    const int NB = P.nb, NP = P.np;
    const int qpb = kvb::select_mfma_queries_per_block(split, kpad);
    const int64_t max_tiles = (int64_t(n) + 31) / 32 + NB;
    const int max_work = (n + qpb - 1) / qpb + NB + 1;
    const int colblocks = std::max(1, std::min(1024, (n + 4095) / 4096));
    const int CH = kRouteChunk;

    // rocPRIM temporary storage for the two sorts
    size_t tmp_m = 0, tmp_q = 0;
    KVB_HIP(ctx, kvb::sort_keys_u64(nullptr, tmp_m, nullptr, nullptr, n, 32 + std::max(1, ceil_log2(NB)), ctx->stream));
    KVB_HIP(ctx, kvb::sort_keys_u64(nullptr, tmp_q, nullptr, nullptr, int64_t(n) * NP, 44 + std::max(1, ceil_log2(NP)),
                                    ctx->stream));
    const size_t tmp_bytes = std::max(tmp_m, tmp_q);

    size_t need = round256(size_t(n) * cap * 8) + round256(size_t(n) * 4) + round256(size_t(n) * kpad * esz) +
                  round256(size_t(max_tiles) * 32 * kpad * esz) + round256(size_t(n) * 4) + round256(size_t(m) * 8) +
                  round256(size_t(colblocks) * m * 8) + 256 + round256(size_t(n) * 4) +
                  round256(size_t(n) * NP * 4) + 2 * round256(size_t(n) * 8) + 2 * round256(size_t(n) * NP * 8) +
                  round256(size_t(NB) * 4) + round256(size_t(NB + 1) * 4) + round256(size_t(max_tiles) * 32 * 4) +
                  round256(size_t(n) * 4) + round256(size_t(NP) * (NB + 1) * 4) +
                  round256(size_t(NP) * max_work * 8) + round256(size_t(NP) * 4) + round256(size_t(n) * NP * 4) +
                  round256(tmp_bytes) + acts_bytes(P, CH, 0, false) + fallback_bytes(n) + 4096;
    KVB_TRY(ensure_scratch(ctx, need));
    Carve cv(ctx->scratch);
    uint64_t* lists = cv.take<uint64_t>(size_t(n) * cap);
    int* fb_list = cv.take<int>(n);
    float* fb_bound = nullptr;
    const kvb::FallbackWork fw = take_fallback(cv, n, &fb_bound);
    void* Aq = cv.take<char>(size_t(n) * kpad * esz);
    void* Bp = cv.take<char>(size_t(max_tiles) * 32 * kpad * esz);
    float* ynorm2 = cv.take<float>(n);
    double* mu = cv.take<double>(m);
    double* colpart = cv.take<double>(size_t(colblocks) * m);
    unsigned* rmax = cv.take<unsigned>(1);
    int32_t* home = cv.take<int32_t>(n);
    int32_t* probe = cv.take<int32_t>(size_t(n) * NP);
    uint64_t* mkeys = cv.take<uint64_t>(n);
    uint64_t* mkeys_s = cv.take<uint64_t>(n);
    uint64_t* qkeys = cv.take<uint64_t>(size_t(n) * NP);
    uint64_t* qkeys_s = cv.take<uint64_t>(size_t(n) * NP);
    int32_t* mstart = cv.take<int32_t>(NB);
    int32_t* tptr = cv.take<int32_t>(NB + 1);
    int32_t* cid = cv.take<int32_t>(size_t(max_tiles) * 32);
    int32_t* brow = cv.take<int32_t>(n);
    int32_t* qptr = cv.take<int32_t>(size_t(NP) * (NB + 1));
    int2* work = cv.take<int2>(size_t(NP) * max_work);
    int32_t* n_work = cv.take<int32_t>(NP);
    int32_t* qids = cv.take<int32_t>(size_t(n) * NP);
    void* tmp = cv.take<char>(tmp_bytes);
    Acts a = carve_acts(cv, P, CH, 0, false);
    hipStream_t st = ctx->stream;

    KVB_HIP(ctx, hipMemsetAsync(ctx->fb_count_dev, 0, sizeof(int), st));
    KVB_HIP(ctx, hipMemsetAsync(ctx->pairs_dev, 0, sizeof(unsigned long long), st));
    {
        Prof pr(ctx, KVB_PROF_ROUTE);
        for (int off = 0; off < n; off += CH) {
            const int valid = std::min(CH, n - off);
            const int B = (valid + 31) / 32 * 32;
            KVB_TRY(mlp_forward(ctx, X + size_t(off) * m, nullptr, valid, B, a, false));
            KVB_HIP(ctx, kvb::launch_route_topp(a.Z, valid, NB, NP, home + off, probe + size_t(off) * NP, st));
        }
    }
    {
        Prof pr(ctx, KVB_PROF_BUCKETS);
        size_t tb = tmp_bytes;
        KVB_HIP(ctx, kvb::launch_member_keys(home, n, mkeys, st));
        KVB_HIP(ctx, kvb::sort_keys_u64(tmp, tb, mkeys, mkeys_s, n, 32 + std::max(1, ceil_log2(NB)), st));
        KVB_HIP(ctx, kvb::launch_bucket_layout(mkeys_s, n, NB, mstart, tptr, cid, max_tiles * 32, brow, st));
        tb = tmp_bytes;
        KVB_HIP(ctx, kvb::launch_query_keys(probe, n, NP, qkeys, st));
        KVB_HIP(ctx, kvb::sort_keys_u64(tmp, tb, qkeys, qkeys_s, int64_t(n) * NP, 44 + std::max(1, ceil_log2(NP)), st));
        KVB_HIP(ctx, kvb::launch_work_layout(qkeys_s, n, NB, NP, qpb, max_work, qptr, work, n_work, qids, st));
    }
    {
        Prof pr(ctx, KVB_PROF_KNN_PREP);
        KVB_HIP(ctx, hipMemsetAsync(rmax, 0, sizeof(unsigned), st));
        KVB_HIP(ctx, kvb::launch_prep(X, n, m, split, kpad, colpart, colblocks, mu, Aq, Bp, ynorm2, rmax, brow, nullptr, st));
    }
    {
        Prof pr(ctx, KVB_PROF_KNN_SELECT);
        const kvb::ErrModel em = {0.0, 0.0, 0.0, 0.0};   // no certificate in this mode
        for (int s = 0; s < NP; ++s) {
            kvb::BucketArgs ba;
            ba.work = work + size_t(s) * max_work;
            ba.n_work = n_work + s;
            ba.qids = qids;
            ba.qptr = qptr + size_t(s) * (NB + 1);
            ba.tptr = tptr;
            ba.cid = cid;
            ba.first = s == 0 ? 1 : 0;
            KVB_HIP(ctx, kvb::launch_select_mfma(split, Aq, Bp, n, kpad, kp, ynorm2, rmax, em, lists, cap, nullptr,
                                                 &ba, max_work, nullptr, ctx->pairs_dev, st));
        }
    }
    {
        Prof pr(ctx, KVB_PROF_KNN_REFINE);
        KVB_HIP(ctx, kvb::launch_refine(X, n, m, k, kp, cap, lists, nullptr, 1.0f, idx, d2, row_flags,
                                        ctx->fb_count_dev, fb_list, fb_bound, static_cast<int>(ctx->force_fallback),
                                        nullptr, nullptr, st));
    }
    {
        Prof pr(ctx, KVB_PROF_KNN_FALLBACK);
        KVB_HIP(ctx, kvb::launch_fallback(X, n, m, k, ctx->fb_count_dev, fb_list, fw, idx, d2, st));
    }
    return KVB_OK;
}

}  // namespace kvbh

extern "C" {

int kvb_part_init(kvb_ctx ctx, int32_t m, int32_t h1, int32_t h2, int32_t n_buckets, int32_t n_probe, uint64_t seed)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, m >= 1 && m <= 1024, "m must be in [1, 1024], got %d", m);
    KVB_REQUIRE(ctx, h1 >= 32 && h1 <= 4096 && h1 % 32 == 0, "h1 must be a multiple of 32 in [32, 4096]");
    KVB_REQUIRE(ctx, h2 >= 32 && h2 <= 4096 && h2 % 32 == 0, "h2 must be a multiple of 32 in [32, 4096]");
    KVB_REQUIRE(ctx, n_buckets >= 32 && n_buckets <= 4096 && n_buckets % 32 == 0,
                "n_buckets must be a multiple of 32 in [32, 4096]");
    KVB_REQUIRE(ctx, n_probe >= 1 && n_probe <= 32 && n_probe <= n_buckets, "n_probe must be in [1, min(32, n_buckets)]");
    KVB_TRY(part_alloc(ctx, m, h1, h2, n_buckets, n_probe));
    PartState& P = ctx->part;
    hipStream_t st = ctx->stream;
    // He initialisation: weights ~ N(0, 2 / fan_in), biases zero
    KVB_HIP(ctx, kvb::launch_fill_normal(P.p + P.off[0], int64_t(h1) * P.mpad, seed, 0, std::sqrt(2.0f / m), st));
    if (P.mpad > m)
        KVB_HIP(ctx, hipMemset2DAsync(P.p + m, size_t(P.mpad) * 4, 0, size_t(P.mpad - m) * 4, h1, st));
    KVB_HIP(ctx, kvb::launch_fill_normal(P.p + P.off[2], int64_t(h2) * h1, seed, uint64_t(1) << 40,
                                         std::sqrt(2.0f / h1), st));
    KVB_HIP(ctx, kvb::launch_fill_normal(P.p + P.off[4], int64_t(n_buckets) * h2, seed, uint64_t(2) << 40,
                                         std::sqrt(2.0f / h2), st));
    KVB_TRY(refresh_bf16(ctx));
    P.ready = true;
    return KVB_OK;
}

int kvb_part_teacher(kvb_ctx ctx, const float* Xs, int64_t ns, int32_t m, int32_t levels, uint64_t seed,
                     int32_t* labels)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, levels >= 1 && levels <= 12, "levels must be in [1, 12], got %d", levels);
    KVB_REQUIRE(ctx, ns >= (int64_t(1) << levels) && ns < (int64_t(1) << 31), "ns must be in [2^levels, 2^31)");
    KVB_REQUIRE(ctx, m >= 1 && m <= 1024, "m must be in [1, 1024]");
    KVB_REQUIRE(ctx, aligned(Xs) && aligned(labels), "Xs and labels must be non-null device pointers");
    const int n = static_cast<int>(ns);
    size_t tmp_bytes = 0;
    KVB_HIP(ctx, kvb::sort_pairs_u64(nullptr, tmp_bytes, nullptr, nullptr, nullptr, nullptr, n, 32 + levels,
                                     ctx->stream));
    const size_t need = 2 * round256(size_t(n) * 8) + 2 * round256(size_t(n) * 4) +
                        round256(size_t((1 << levels) + 1) * 4) + round256(tmp_bytes) + 1024;
    KVB_TRY(ensure_scratch(ctx, need));
    Carve cv(ctx->scratch);
    uint64_t* keys = cv.take<uint64_t>(n);
    uint64_t* skeys = cv.take<uint64_t>(n);
    int32_t* vals = cv.take<int32_t>(n);
    int32_t* svals = cv.take<int32_t>(n);
    int32_t* start = cv.take<int32_t>((1 << levels) + 1);
    void* tmp = cv.take<char>(tmp_bytes);
    for (int l = 0; l < levels; ++l) {
        KVB_HIP(ctx, kvb::launch_teacher_keys(Xs, n, m, l == 0 ? nullptr : labels, l, seed, keys, vals, ctx->stream));
        size_t tb = tmp_bytes;
        KVB_HIP(ctx, kvb::sort_pairs_u64(tmp, tb, keys, skeys, vals, svals, n, 32 + std::max(1, l), ctx->stream));
        KVB_HIP(ctx, kvb::launch_teacher_split(skeys, svals, n, 1 << l, start, labels, ctx->stream));
    }
    return KVB_OK;
}

int kvb_part_train(kvb_ctx ctx, const float* Xs, int64_t ns, int32_t m, const int32_t* labels, const int32_t* idx_s,
                   int32_t ks, int32_t epochs, int32_t batch, float lr, uint64_t seed, float* loss_host)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_TRY(require_part(ctx, m));
    KVB_REQUIRE(ctx, batch >= 32 && batch <= 65536 && batch % 32 == 0, "batch must be a multiple of 32 in [32, 65536]");
    KVB_REQUIRE(ctx, ns >= batch && ns < (int64_t(1) << 31), "ns must be in [batch, 2^31)");
    KVB_REQUIRE(ctx, ks >= 1 && ks <= 4096, "ks must be in [1, 4096]");
    KVB_REQUIRE(ctx, epochs >= 1 && epochs <= 100000, "epochs must be in [1, 100000]");
    KVB_REQUIRE(ctx, lr > 0.f && std::isfinite(lr), "lr must be finite and > 0");
    KVB_REQUIRE(ctx, aligned(Xs) && aligned(labels) && aligned(idx_s),
                "Xs, labels and idx_s must be non-null device pointers");
    PartState& P = ctx->part;
    const int B = batch;
    KVB_TRY(ensure_scratch(ctx, acts_bytes(P, B, ks, true)));
    KVB_TRY(ensure_loss(ctx, epochs));
    Carve cv(ctx->scratch);
    Acts a = carve_acts(cv, P, B, ks, true);
    hipStream_t st = ctx->stream;
    const int64_t nbatch = ns / B;
    for (int e = 0; e < epochs; ++e) {
        // affine permutation t -> (a t + c) mod ns with gcd(a, ns) = 1
        uint64_t pa = host_splitmix(seed, 2 * uint64_t(e)) % uint64_t(ns);
        if (pa == 0) pa = 1;
        while (gcd_u64(pa, uint64_t(ns)) != 1) pa = pa + 1 == uint64_t(ns) ? 1 : pa + 1;
        const uint64_t pc = host_splitmix(seed, 2 * uint64_t(e) + 1) % uint64_t(ns);
        for (int64_t t = 0; t < nbatch; ++t) {
            KVB_HIP(ctx, kvb::launch_batch_gather(ns, pa, pc, t * B, B, idx_s, ks, labels, a.bidx, a.nbrlab, st));
            KVB_TRY(mlp_forward(ctx, Xs, a.bidx, B, B, a, true));
            KVB_TRY(mlp_backward(ctx, B, a.nbrlab, ks, a, ctx->loss_dev + e, t == 0 ? 0 : 1));
            P.step += 1;
            const float c1 = 1.f - std::pow(kAdamB1, float(P.step));
            const float c2 = 1.f - std::pow(kAdamB2, float(P.step));
            KVB_HIP(ctx, kvb::launch_adam(P.p, P.g, P.m1, P.m2, P.total, lr, kAdamB1, kAdamB2, kAdamEps, c1, c2, P.pb,
                                          st));
            KVB_HIP(ctx, kvb::launch_transpose_bf16(P.pb + P.off[2], P.h2, P.h1, P.w2t, st));
            KVB_HIP(ctx, kvb::launch_transpose_bf16(P.pb + P.off[4], P.nb, P.h2, P.w3t, st));
        }
    }
    std::vector<double> lh(epochs);
    KVB_HIP(ctx, hipMemcpyAsync(lh.data(), ctx->loss_dev, sizeof(double) * epochs, hipMemcpyDeviceToHost, st));
    KVB_HIP(ctx, hipStreamSynchronize(st));
    if (loss_host)
        for (int e = 0; e < epochs; ++e) loss_host[e] = static_cast<float>(lh[e] / double(nbatch));
    return KVB_OK;
}

int kvb_part_route(kvb_ctx ctx, const float* X, int64_t n, int32_t* home, int32_t* probe)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_TRY(require_part(ctx, -1));
    KVB_REQUIRE(ctx, n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31)");
    KVB_REQUIRE(ctx, aligned(X) && aligned(probe), "X and probe must be non-null device pointers");
    KVB_REQUIRE(ctx, home == nullptr || aligned(home), "home must be aligned");
    const PartState& P = ctx->part;
    const int CH = kRouteChunk;
    KVB_TRY(ensure_scratch(ctx, acts_bytes(P, CH, 0, false)));
    Carve cv(ctx->scratch);
    Acts a = carve_acts(cv, P, CH, 0, false);
    const int nn = static_cast<int>(n);
    Prof pr(ctx, KVB_PROF_ROUTE);
    for (int off = 0; off < nn; off += CH) {
        const int valid = std::min(CH, nn - off);
        const int B = (valid + 31) / 32 * 32;
        KVB_TRY(mlp_forward(ctx, X + size_t(off) * P.m, nullptr, valid, B, a, false));
        KVB_HIP(ctx, kvb::launch_route_topp(a.Z, valid, P.nb, P.np, home ? home + off : nullptr,
                                            probe + size_t(off) * P.np, ctx->stream));
    }
    return KVB_OK;
}

int kvb_part_save(kvb_ctx ctx, const char* path)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_TRY(require_part(ctx, -1));
    KVB_REQUIRE(ctx, path != nullptr, "path must be non-null");
    const PartState& P = ctx->part;
    std::vector<float> buf(size_t(P.total) * 3);
    KVB_HIP(ctx, hipMemcpyAsync(buf.data(), P.p, size_t(P.total) * 4, hipMemcpyDeviceToHost, ctx->stream));
    KVB_HIP(ctx, hipMemcpyAsync(buf.data() + P.total, P.m1, size_t(P.total) * 4, hipMemcpyDeviceToHost, ctx->stream));
    KVB_HIP(ctx,
            hipMemcpyAsync(buf.data() + 2 * P.total, P.m2, size_t(P.total) * 4, hipMemcpyDeviceToHost, ctx->stream));
    KVB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    FileCloser fc{fopen(path, "wb")};
    if (!fc.f) return fail(ctx, KVB_E_IO, "cannot open %s for writing", path);
    const int64_t hdr[8] = {P.m, P.h1, P.h2, P.nb, P.np, P.step, P.total, 0};
    bool ok = fwrite(kMagic, 1, 8, fc.f) == 8 && fwrite(hdr, sizeof(hdr), 1, fc.f) == 1 &&
              fwrite(buf.data(), sizeof(float), buf.size(), fc.f) == buf.size();
    ok = (fclose(fc.f) == 0) && ok;
    fc.f = nullptr;
    if (!ok) return fail(ctx, KVB_E_IO, "writing %s failed", path);
    return KVB_OK;
}

int kvb_part_load(kvb_ctx ctx, const char* path)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, path != nullptr, "path must be non-null");
    FileCloser fc{fopen(path, "rb")};
    if (!fc.f) return fail(ctx, KVB_E_IO, "cannot open %s", path);
    char magic[8];
    int64_t hdr[8];
    if (fread(magic, 1, 8, fc.f) != 8 || std::memcmp(magic, kMagic, 8) != 0 || fread(hdr, sizeof(hdr), 1, fc.f) != 1)
        return fail(ctx, KVB_E_IO, "%s is not a partitioner file", path);
    const int64_t m = hdr[0], h1 = hdr[1], h2 = hdr[2], nb = hdr[3], np = hdr[4];
    if (m < 1 || m > 1024 || h1 < 32 || h1 > 4096 || h1 % 32 || h2 < 32 || h2 > 4096 || h2 % 32 || nb < 32 ||
        nb > 4096 || nb % 32 || np < 1 || np > 32 || np > nb)
        return fail(ctx, KVB_E_IO, "%s holds invalid partitioner dimensions", path);
    KVB_TRY(part_alloc(ctx, int(m), int(h1), int(h2), int(nb), int(np)));
    PartState& P = ctx->part;
    if (hdr[6] != P.total) {
        part_free(ctx);
        return fail(ctx, KVB_E_IO, "%s has an inconsistent parameter count", path);
    }
    std::vector<float> buf(size_t(P.total) * 3);
    if (fread(buf.data(), sizeof(float), buf.size(), fc.f) != buf.size()) {
        part_free(ctx);
        return fail(ctx, KVB_E_IO, "%s is truncated", path);
    }
    KVB_HIP(ctx, hipMemcpyAsync(P.p, buf.data(), size_t(P.total) * 4, hipMemcpyHostToDevice, ctx->stream));
    KVB_HIP(ctx, hipMemcpyAsync(P.m1, buf.data() + P.total, size_t(P.total) * 4, hipMemcpyHostToDevice, ctx->stream));
    KVB_HIP(ctx,
            hipMemcpyAsync(P.m2, buf.data() + 2 * P.total, size_t(P.total) * 4, hipMemcpyHostToDevice, ctx->stream));
    P.step = hdr[5];
    KVB_TRY(refresh_bf16(ctx));
    KVB_HIP(ctx, hipStreamSynchronize(ctx->stream));   // the host buffer dies here
    P.ready = true;
    return KVB_OK;
}

int kvb_mlp_forward(kvb_ctx ctx, const float* X, int64_t B, float* logits)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_TRY(require_part(ctx, -1));
    KVB_REQUIRE(ctx, B >= 32 && B <= 65536 && B % 32 == 0, "B must be a multiple of 32 in [32, 65536]");
    KVB_REQUIRE(ctx, aligned(X) && aligned(logits), "X and logits must be non-null device pointers");
    const PartState& P = ctx->part;
    const int b = static_cast<int>(B);
    KVB_TRY(ensure_scratch(ctx, acts_bytes(P, b, 0, false)));
    Carve cv(ctx->scratch);
    Acts a = carve_acts(cv, P, b, 0, false);
    KVB_TRY(mlp_forward(ctx, X, nullptr, b, b, a, false));
    KVB_HIP(ctx, hipMemcpyAsync(logits, a.Z, size_t(b) * P.nb * 4, hipMemcpyDeviceToDevice, ctx->stream));
    return KVB_OK;
}

int kvb_mlp_backward(kvb_ctx ctx, const float* X, int64_t B, const int32_t* nbr_labels, int32_t ks, float* loss_host,
                     float* grads)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_TRY(require_part(ctx, -1));
    KVB_REQUIRE(ctx, B >= 32 && B <= 65536 && B % 32 == 0, "B must be a multiple of 32 in [32, 65536]");
    KVB_REQUIRE(ctx, ks >= 1 && ks <= 4096, "ks must be in [1, 4096]");
    KVB_REQUIRE(ctx, aligned(X) && aligned(nbr_labels) && aligned(grads),
                "X, nbr_labels and grads must be non-null device pointers");
    const PartState& P = ctx->part;
    const int b = static_cast<int>(B);
    KVB_TRY(ensure_scratch(ctx, acts_bytes(P, b, ks, true)));
    KVB_TRY(ensure_loss(ctx, 1));
    Carve cv(ctx->scratch);
    Acts a = carve_acts(cv, P, b, ks, true);
    KVB_TRY(mlp_forward(ctx, X, nullptr, b, b, a, true));
    KVB_TRY(mlp_backward(ctx, b, nbr_labels, ks, a, ctx->loss_dev, 0));
    KVB_TRY(copy_params(ctx, P.g, grads, true));
    double loss = 0.0;
    KVB_HIP(ctx, hipMemcpyAsync(&loss, ctx->loss_dev, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    KVB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (loss_host) *loss_host = static_cast<float>(loss);
    return KVB_OK;
}

int64_t kvb_part_num_params(kvb_ctx ctx)
{
    if (!ctx) return KVB_E_INVALID;
    if (!ctx->part.ready) return fail(ctx, KVB_E_NOT_TRAINED, "no partitioner");
    return ctx->part.nparams();
}

int kvb_part_get_params(kvb_ctx ctx, float* params)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_TRY(require_part(ctx, -1));
    KVB_REQUIRE(ctx, aligned(params), "params must be a non-null device pointer");
    return copy_params(ctx, ctx->part.p, params, true);
}

int kvb_part_set_params(kvb_ctx ctx, const float* params)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_TRY(require_part(ctx, -1));
    KVB_REQUIRE(ctx, aligned(params), "params must be a non-null device pointer");
    PartState& P = ctx->part;
    KVB_TRY(copy_params(ctx, params, P.p, false));
    KVB_HIP(ctx, hipMemsetAsync(P.m1, 0, size_t(P.total) * 4, ctx->stream));
    KVB_HIP(ctx, hipMemsetAsync(P.m2, 0, size_t(P.total) * 4, ctx->stream));
    P.step = 0;
    return refresh_bf16(ctx);
}

}  // extern "C"
