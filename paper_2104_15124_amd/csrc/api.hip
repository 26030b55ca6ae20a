// C ABI of libkvb.so: contexts, argument validation, scratch management and
// the launch sequence of each entry point. The numerical work of every entry
// point runs in the kernels of knn_kernels.hip, knn_mfma.hip and
// pass_kernels.hip; the learned partitioner's entry points are in
// learned_api.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kvb_ctx.h"

namespace {
const char* const kProfNames[KVB_PROF_SLOTS] = {
    "knn_select", "knn_refine", "knn_fallback", "adhoc_bandwidth", "chi_tuning", "density",
    "grid_scale", "q_pass", "assemble", "knn_prep",
    "route", "bucket_build", "union_pattern", "truncate", "curve_rows",
};
}  // namespace

using namespace kvbh;

extern "C" {

int kvb_create(kvb_ctx* out, void* hip_stream)
{
    if (!out) return KVB_E_INVALID;
    *out = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return KVB_E_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return KVB_E_HIP;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return KVB_E_UNSUPPORTED;
    kvb_ctx ctx = new kvb_ctx_s();
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    ctx->device = dev;
    if (hipMalloc(reinterpret_cast<void**>(&ctx->tune_dev), sizeof(kvb::TuneResult)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&ctx->tune_host), sizeof(kvb::TuneResult), hipHostMallocDefault) !=
            hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&ctx->build_dev), sizeof(BuildDev)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&ctx->build_host), sizeof(BuildDev), hipHostMallocDefault) !=
            hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&ctx->fb_count_dev), sizeof(int)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&ctx->pairs_dev), sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&ctx->pairs_host), sizeof(unsigned long long),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&ctx->fb_count_host), sizeof(int), hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&ctx->union_host), 2 * sizeof(unsigned long long),
                      hipHostMallocDefault) != hipSuccess) {
        kvb_destroy(ctx);
        return KVB_E_NOMEM;
    }
    if (noalloc_scratch_init(dev) != KVB_OK) {
        kvb_destroy(ctx);
        return KVB_E_HIP;
    }
    *out = ctx;
    return KVB_OK;
}

int kvb_create_host(kvb_ctx* out)
{
    if (!out) return KVB_E_INVALID;
    kvb_ctx ctx = new kvb_ctx_s();
    ctx->host_only = true;
    ctx->device = -1;
    *out = ctx;
    return KVB_OK;
}

void kvb_destroy(kvb_ctx ctx)
{
    if (!ctx) return;
    if (ctx->host_only) {
        delete ctx;
        return;
    }
    (void)hipStreamSynchronize(ctx->stream);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (const ProfPair& p : ctx->ev_pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->tune_dev) (void)hipFree(ctx->tune_dev);
    if (ctx->tune_host) (void)hipHostFree(ctx->tune_host);
    if (ctx->fb_count_dev) (void)hipFree(ctx->fb_count_dev);
    if (ctx->fb_count_host) (void)hipHostFree(ctx->fb_count_host);
    if (ctx->build_dev) (void)hipFree(ctx->build_dev);
    if (ctx->build_host) (void)hipHostFree(ctx->build_host);
    if (ctx->loss_dev) (void)hipFree(ctx->loss_dev);
    if (ctx->pairs_dev) (void)hipFree(ctx->pairs_dev);
    if (ctx->pairs_host) (void)hipHostFree(ctx->pairs_host);
    if (ctx->union_host) (void)hipHostFree(ctx->union_host);
    part_free(ctx);
    delete ctx;
}

const char* kvb_last_error(kvb_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int kvb_set_option(kvb_ctx ctx, int32_t key, int64_t value)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    switch (key) {
    case KVB_OPT_FORCE_FALLBACK:
        KVB_REQUIRE(ctx, value >= 0, "KVB_OPT_FORCE_FALLBACK must be >= 0");
        ctx->force_fallback = value;
        return KVB_OK;
    case KVB_OPT_SCRATCH_LIMIT:
        KVB_REQUIRE(ctx, value >= 0, "KVB_OPT_SCRATCH_LIMIT must be >= 0");
        ctx->scratch_limit = static_cast<size_t>(value);
        return KVB_OK;
    case KVB_OPT_N_PROBE:
        if (!ctx->part.ready) return fail(ctx, KVB_E_NOT_TRAINED, "KVB_OPT_N_PROBE needs a partitioner");
        KVB_REQUIRE(ctx, value >= 1 && value <= 32 && value <= ctx->part.nb,
                    "KVB_OPT_N_PROBE must be in [1, min(32, n_buckets)]");
        ctx->part.np = static_cast<int>(value);
        return KVB_OK;
    case KVB_OPT_PATTERN:
        KVB_REQUIRE(ctx, value == KVB_PATTERN_KNN || value == KVB_PATTERN_UNION,
                    "KVB_OPT_PATTERN must be KVB_PATTERN_KNN or KVB_PATTERN_UNION");
        ctx->pattern = static_cast<int>(value);
        return KVB_OK;
    case KVB_OPT_CURVE_ORDER:
        KVB_REQUIRE(ctx, value >= 0 && value <= 2, "KVB_OPT_CURVE_ORDER must be 0, 1 or 2");
        ctx->curve_order = static_cast<int>(value);
        return KVB_OK;
    case KVB_OPT_BF16_SPLIT:
        KVB_REQUIRE(ctx, value == 1 || value == 3 || value == 6, "KVB_OPT_BF16_SPLIT must be 1, 3 or 6");
        ctx->bf16_split = static_cast<int>(value);
        return KVB_OK;
    default:
        return fail(ctx, KVB_E_INVALID, "unknown option key %d", key);
    }
}

// The curve order a matrix-core k-NN scanned, left in the context's scratch
// for the passes of kvb_build: cid[p] = sample at curve position p, pos its
// inverse (null when the k-NN did not run in curve order).
struct CurveRows {
    const int32_t* cid = nullptr;
    const int32_t* pos = nullptr;
};

// kvb_knn on the scratch from byte `base` on (the bytes before it are left to
// the caller), reporting the curve order through cr when it ran in one.
static int knn_run(kvb_ctx ctx, size_t base, const float* X, int64_t n, int32_t m, int32_t k, int32_t mode,
                   int32_t margin, int32_t* idx, float* d2, int32_t* row_flags, CurveRows* cr)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31), got %lld", (long long)n);
    KVB_REQUIRE(ctx, m >= 1, "m must be >= 1, got %d", m);
    KVB_REQUIRE(ctx, k >= 1 && k <= n, "k must be in [1, n], got k=%d n=%lld", k, (long long)n);
    KVB_REQUIRE(ctx, margin >= 0, "margin must be >= 0, got %d", margin);
    KVB_REQUIRE(ctx, aligned(X), "X must be a non-null float32 device pointer");
    KVB_REQUIRE(ctx, aligned(idx), "idx must be a non-null int32 device pointer");
    KVB_REQUIRE(ctx, aligned(d2), "d2 must be a non-null float32 device pointer");
    KVB_REQUIRE(ctx, row_flags == nullptr || aligned(row_flags), "row_flags must be aligned");
    KVB_REQUIRE(ctx, mode == KVB_KNN_F32 || mode == KVB_KNN_BF16 || mode == KVB_KNN_LEARNED,
                "unknown k-NN mode %d", mode);
    if (k + margin > 256) return fail(ctx, KVB_E_UNSUPPORTED, "k + margin = %d exceeds 256", k + margin);
    if (m > 1024) return fail(ctx, KVB_E_UNSUPPORTED, "m = %d exceeds 1024", m);

    const int nn = static_cast<int>(n);
    const int kp = static_cast<int>(std::min<int64_t>(k + margin, n));
    if (mode == KVB_KNN_LEARNED) return learned_knn(ctx, X, nn, m, k, kp, idx, d2, row_flags);
    const bool direct = (mode == KVB_KNN_F32 && m <= 8);
    const int split = mode == KVB_KNN_F32 ? 0 : ctx->bf16_split;
    const int cap = kp <= 128 ? 128 : 256;   // list capacities of the matrix-core select kernels
    int kpad = 0;
    if (!direct) {
        const int kraw = split == 0 ? m + 1 : split * m + 3;
        const int kstep = kvb::mfma_kstep(split);
        const int ks = kvb::mfma_pick_ksteps(split, (kraw + kstep - 1) / kstep);
        if (ks < 0)
            return fail(ctx, KVB_E_UNSUPPORTED, "m = %d is too large for the %s distance tiles", m,
                        split == 0 ? "FP32" : "BF16");
        kpad = ks * kstep;
    }
    const int colblocks = std::max(1, std::min(1024, (nn + 4095) / 4096));
    const size_t esz = split == 0 ? sizeof(float) : sizeof(uint16_t);
    size_t need = round256(size_t(nn) * (direct ? kp : cap) * sizeof(uint64_t)) +
                  round256(size_t(nn) * sizeof(float)) + round256(size_t(nn) * sizeof(int)) + fallback_bytes(nn) +
                  2048;
    size_t sort_bytes = 0;
    const int code_bits = direct ? m * kvb::spatial_code_bits(nn, m) : 32;
    if (direct)
        KVB_HIP(ctx, kvb::sort_pairs_u32(nullptr, sort_bytes, nullptr, nullptr, nullptr, nullptr, nn, code_bits,
                                         ctx->stream));
    const int ntiles = kvb::spatial_tiles(nn), nsb = kvb::spatial_superblocks(nn);
    if (direct)
        need += round256(size_t(nn) * m * sizeof(float)) + 2 * round256(size_t(nn) * sizeof(int32_t)) +
                2 * round256(size_t(nn) * sizeof(uint64_t)) + round256(size_t(ntiles) * 2 * m * sizeof(float)) +
                round256(size_t(nsb) * 2 * m * sizeof(float)) +
                round256(size_t(kvb::spatial_bbox_blocks(nn)) * 2 * m * sizeof(float)) + round256(sort_bytes);
    else
        need += 2 * round256(size_t(nn + 31) / 32 * 32 * kpad * esz) + round256(size_t(nn) * sizeof(float)) +
                round256(size_t(m) * sizeof(double)) + round256(size_t(colblocks) * m * sizeof(double)) + 256;
    // curve order of the principal projections (matrix-core modes)
    const bool curve = !direct && ctx->curve_order && m <= 256;
    const int npad32 = (nn + 31) / 32 * 32, ctiles = npad32 / 32;
    const kvb::TreeLayout tl = kvb::tree_layout(ctiles);
    const int csb = (ctiles + kvb::SB_TILES_MFMA - 1) / kvb::SB_TILES_MFMA;
    const size_t ntri = size_t(m) * (m + 1) / 2;
    size_t csort = 0;
    if (curve) {
        csort = kvb::curve_sort_bytes(nn);
        need += round256(size_t(kvb::cov_partials()) * ntri * sizeof(double)) +
                round256(size_t(m) * m * sizeof(double)) + round256((size_t(m) * kvb::PR_DIMS + 1) * sizeof(float)) +
                round256(size_t(nn) * kvb::PR_DIMS * sizeof(float)) +
                round256(size_t(kvb::project_blocks(nn) + 1) * 2 * kvb::PCODE_DIMS * sizeof(float)) +
                2 * round256(size_t(nn) * sizeof(uint32_t)) + 3 * round256(size_t(nn) * sizeof(int32_t)) +
                round256(size_t(npad32) * sizeof(int32_t)) + round256(size_t(npad32) * kvb::PR_DIMS * sizeof(float)) +
                round256(size_t(ctiles) * 2 * kvb::PR_DIMS * sizeof(float)) +
                round256(size_t(std::max(tl.nodes, 1)) * 2 * kvb::PR_DIMS * sizeof(float)) +
                round256(size_t(csb) * 2 * kvb::PR_DIMS * sizeof(float)) + round256(csort) +
                round256(size_t(nn) * m * sizeof(float)) + 512;
    }
    int rc = ensure_scratch(ctx, base + need);
    if (rc) return rc;
    Carve cv(static_cast<char*>(ctx->scratch) + base);
    uint64_t* keys = cv.take<uint64_t>(size_t(nn) * (direct ? kp : cap));
    float* slast = cv.take<float>(nn);
    int* fb_list = cv.take<int>(nn);
    float* fb_bound = nullptr;
    const kvb::FallbackWork fw = take_fallback(cv, nn, &fb_bound);

    KVB_HIP(ctx, hipMemsetAsync(ctx->fb_count_dev, 0, sizeof(int), ctx->stream));
    KVB_HIP(ctx, hipMemsetAsync(ctx->pairs_dev, 0, sizeof(unsigned long long), ctx->stream));
    float lb_scale = 1.0f;
    int kstride = kp;
    float* Xs = nullptr;        // curve-ordered samples (lists are then stored in that order)
    int32_t* perm = nullptr;
    const int32_t* curve_pos = nullptr;
    if (direct) {
        Xs = cv.take<float>(size_t(nn) * m);
        perm = cv.take<int32_t>(nn);
        int32_t* vals = cv.take<int32_t>(nn);
        uint32_t* code = cv.take<uint32_t>(nn);
        uint32_t* scode = cv.take<uint32_t>(nn);
        float* tbox = cv.take<float>(size_t(ntiles) * 2 * m);
        float* sbox = cv.take<float>(size_t(nsb) * 2 * m);
        float* bbox = cv.take<float>(size_t(kvb::spatial_bbox_blocks(nn)) * 2 * m);
        void* sort_tmp = cv.take<char>(sort_bytes);
        {
            Prof pr(ctx, KVB_PROF_KNN_PREP);
            KVB_HIP(ctx, kvb::launch_spatial_codes(X, nn, m, bbox, code, vals, ctx->stream));
            size_t sb = sort_bytes;
            KVB_HIP(ctx, kvb::sort_pairs_u32(sort_tmp, sb, code, scode, vals, perm, nn, code_bits, ctx->stream));
            KVB_HIP(ctx, kvb::launch_spatial_layout(X, nn, m, perm, Xs, tbox, sbox, ctx->stream));
        }
        Prof pr(ctx, KVB_PROF_KNN_SELECT);
        KVB_HIP(ctx, kvb::launch_select_direct(Xs, tbox, sbox, nn, m, kp, keys, slast, ctx->pairs_dev,
                                               ctx->stream));
        // the direct tiles compute each squared distance with at most (m + 2)
        // float32 roundings; (m + 4) 2^-23 bounds their relative error with a
        // factor-2 margin
        const double sel_err = (m + 4) * std::ldexp(1.0, -23);
        lb_scale = static_cast<float>(1.0 / (1.0 + sel_err));
    } else {
        void* Aq = cv.take<char>(size_t(nn) * kpad * esz);
        void* Bc = cv.take<char>(size_t(nn + 31) / 32 * 32 * kpad * esz);   // tile-major, 32-row padded
        float* ynorm2 = cv.take<float>(nn);
        double* mu = cv.take<double>(m);
        double* colpart = cv.take<double>(size_t(colblocks) * m);
        unsigned* rmax = cv.take<unsigned>(1);
        kvb::CurveArgs crv = {};
        {
            Prof pr(ctx, KVB_PROF_KNN_PREP);
            KVB_HIP(ctx, hipMemsetAsync(rmax, 0, sizeof(unsigned), ctx->stream));
            if (curve) {
                double* covpart = cv.take<double>(size_t(kvb::cov_partials()) * ntri);
                double* C = cv.take<double>(size_t(m) * m);
                float* P = cv.take<float>(size_t(m) * kvb::PR_DIMS + 1);
                float* z = cv.take<float>(size_t(nn) * kvb::PR_DIMS);
                float* zpart = cv.take<float>(size_t(kvb::project_blocks(nn) + 1) * 2 * kvb::PCODE_DIMS);
                uint32_t* code = cv.take<uint32_t>(nn);
                uint32_t* scode = cv.take<uint32_t>(nn);
                int32_t* vals = cv.take<int32_t>(nn);
                int32_t* order = cv.take<int32_t>(nn);
                int32_t* pos = cv.take<int32_t>(nn);
                int32_t* cid = cv.take<int32_t>(npad32);
                curve_pos = pos;
                float* zs = cv.take<float>(size_t(npad32) * kvb::PR_DIMS);
                float* tbox = cv.take<float>(size_t(ctiles) * 2 * kvb::PR_DIMS);
                float* tree = cv.take<float>(size_t(std::max(tl.nodes, 1)) * 2 * kvb::PR_DIMS);
                float* sbox = cv.take<float>(size_t(csb) * 2 * kvb::PR_DIMS);
                void* sort_tmp = cv.take<char>(csort);
                KVB_HIP(ctx, kvb::launch_colmean(X, nn, m, colpart, colblocks, mu, ctx->stream));
                KVB_HIP(ctx, kvb::launch_principal_basis(X, nn, m, mu, covpart, C, P, ctx->stream));
                KVB_HIP(ctx, kvb::launch_curve_order(X, nn, m, mu, P, z, zpart, code, scode, vals, order, sort_tmp,
                                                     csort, pos, cid, zs, tbox, sbox, tree, ctx->curve_order == 2,
                                                     ctx->stream));
                // curve-ordered copy of the samples for the refine step
                Xs = cv.take<float>(size_t(nn) * m);
                KVB_HIP(ctx, kvb::launch_gather_rows(X, nn, m, cid, Xs, ctx->stream));
                perm = cid;
                // the padding rows of the last tile hold zeros (their keys are never taken)
                const size_t tile_bytes = size_t(32) * kpad * esz;
                KVB_HIP(ctx, hipMemsetAsync(static_cast<char*>(Bc) + size_t(ctiles - 1) * tile_bytes, 0, tile_bytes,
                                            ctx->stream));
                KVB_HIP(ctx, kvb::launch_prep_rows_curve(Xs, nn, m, mu, split, kpad, Aq, Bc, ynorm2, rmax,
                                                         ctx->stream));
                const double u = std::ldexp(1.0, -24);
                crv.perm = cid;
                crv.zs = zs;
                crv.tbox = tbox;
                crv.sbox = sbox;
                crv.tree = tree;
                crv.layout = tl;
                crv.pscale = P + size_t(m) * kvb::PR_DIMS;
                // a float32 dot product of m terms errs by at most m u |y| |p| (|p| <= 1 + m u)
                crv.zcoef = static_cast<float>((m + 2) * u * 1.01);
                // |y_i - y_j| - |x_i - x_j| <= u (|x_i - mu| + |x_j - mu|) for y = fl(x - mu)
                crv.ycoef = static_cast<float>(2.1 * u);
            } else {
                KVB_HIP(ctx, kvb::launch_prep(X, nn, m, split, kpad, colpart, colblocks, mu, Aq, Bc, ynorm2, rmax,
                                              nullptr, nullptr, ctx->stream));
            }
        }
        // error model of the selection score (derivation in knn_mfma.hip)
        const double u = std::ldexp(1.0, -24);
        double rep = 0.0, drop = 0.0;
        if (split == 1) rep = std::ldexp(1.01, -8);
        if (split == 3) rep = std::ldexp(1.01, -16), drop = std::ldexp(1.03, -16);
        if (split == 6) rep = std::ldexp(1.01, -24), drop = std::ldexp(1.03, -23);
        kvb::ErrModel em;
        em.gamma = (kpad + 4) * u;
        em.norm = 1.01 * u;
        em.cross = 2.0 * (2.0 * rep * (1.0 + rep) + drop);
        em.center = 1.01 * u;
        {
            Prof pr(ctx, KVB_PROF_KNN_SELECT);
            if (curve && kvb::select_tree_fits(split, kpad))
                KVB_HIP(ctx, kvb::launch_select_tree(split, Aq, Bc, nn, kpad, kp, ynorm2, rmax, em, keys, cap, slast,
                                                     crv, ctx->pairs_dev, ctx->stream));
            else
                KVB_HIP(ctx, kvb::launch_select_mfma(split, Aq, Bc, nn, kpad, kp, ynorm2, rmax, em, keys, cap, slast,
                                                     nullptr, 0, curve ? &crv : nullptr, ctx->pairs_dev, ctx->stream));
        }
        kstride = cap;
    }
    {
        Prof pr(ctx, KVB_PROF_KNN_REFINE);
        KVB_HIP(ctx, kvb::launch_refine(X, nn, m, k, kp, kstride, keys, slast, lb_scale, idx, d2, row_flags,
                                        ctx->fb_count_dev, fb_list, fb_bound, static_cast<int>(ctx->force_fallback),
                                        Xs, perm, ctx->stream));
    }
    {
        Prof pr(ctx, KVB_PROF_KNN_FALLBACK);
        KVB_HIP(ctx, kvb::launch_fallback(X, nn, m, k, ctx->fb_count_dev, fb_list, fw, idx, d2, ctx->stream));
    }
    if (cr && curve_pos) {
        cr->cid = perm;
        cr->pos = curve_pos;
    }
    return KVB_OK;
}

int kvb_knn(kvb_ctx ctx, const float* X, int64_t n, int32_t m, int32_t k, int32_t mode, int32_t margin,
            int32_t* idx, float* d2, int32_t* row_flags)
{
    return knn_run(ctx, 0, X, n, m, k, mode, margin, idx, d2, row_flags, nullptr);
}

int kvb_knn_fallback_rows(kvb_ctx ctx, int64_t* count_host)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, count_host != nullptr, "count_host must be non-null");
    KVB_HIP(ctx, hipMemcpyAsync(ctx->fb_count_host, ctx->fb_count_dev, sizeof(int), hipMemcpyDeviceToHost,
                                ctx->stream));
    KVB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *count_host = *ctx->fb_count_host;
    return *count_host > 0 ? KVB_W_FALLBACK : KVB_OK;
}

int kvb_knn_pairs(kvb_ctx ctx, double* pairs_host)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, pairs_host != nullptr, "pairs_host must be non-null");
    KVB_HIP(ctx, hipMemcpyAsync(ctx->pairs_host, ctx->pairs_dev, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                ctx->stream));
    KVB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *pairs_host = static_cast<double>(*ctx->pairs_host);
    return KVB_OK;
}

int kvb_knn_exact_rows(kvb_ctx ctx, const float* X, int64_t n, int32_t m, int32_t k, const int32_t* rows,
                       int64_t nrows, int32_t* idx, float* d2)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31)");
    KVB_REQUIRE(ctx, m >= 1 && m <= 1024, "m must be in [1, 1024], got %d", m);
    KVB_REQUIRE(ctx, k >= 1 && k <= n && k <= 256, "k must be in [1, min(n, 256)], got %d", k);
    KVB_REQUIRE(ctx, nrows >= 0 && nrows < (int64_t(1) << 31), "nrows must be in [0, 2^31)");
    if (nrows == 0) return KVB_OK;
    KVB_REQUIRE(ctx, aligned(X) && aligned(rows) && aligned(idx) && aligned(d2),
                "X, rows, idx and d2 must be non-null device pointers");
    Prof pr(ctx, KVB_PROF_KNN_FALLBACK);
    KVB_HIP(ctx, kvb::launch_exact_rows(X, static_cast<int>(n), m, k, rows, static_cast<int>(nrows), idx, d2,
                                        ctx->stream));
    return KVB_OK;
}

int kvb_bandwidth(kvb_ctx ctx, const int32_t* idx, const float* d2, int64_t n, int32_t k, int32_t mode, int32_t k0,
                  const float* b, double e, double d, double beta, float* rho, float* psi)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31)");
    KVB_REQUIRE(ctx, k >= 1 && k <= 256, "k must be in [1, 256], got %d", k);
    KVB_REQUIRE(ctx, aligned(d2), "d2 must be a non-null float32 device pointer");
    KVB_REQUIRE(ctx, aligned(rho), "rho must be a non-null float32 device pointer");
    const int nn = static_cast<int>(n);
    if (mode == KVB_BW_ADHOC) {
        KVB_REQUIRE(ctx, k0 >= 1 && k0 < k, "k0 must be in [1, k), got k0=%d k=%d", k0, k);
        Prof pr(ctx, KVB_PROF_ADHOC);
        KVB_HIP(ctx, kvb::launch_adhoc_bandwidth(d2, nn, k, k0, rho, ctx->stream));
        return KVB_OK;
    }
    KVB_REQUIRE(ctx, mode == KVB_BW_DENSITY, "unknown bandwidth mode %d", mode);
    KVB_REQUIRE(ctx, aligned(idx), "idx must be a non-null int32 device pointer");
    KVB_REQUIRE(ctx, aligned(b), "b must be a non-null float32 device pointer");
    KVB_REQUIRE(ctx, psi == nullptr || aligned(psi), "psi must be aligned");
    KVB_REQUIRE(ctx, e > 0 && std::isfinite(e), "e must be finite and > 0");
    KVB_REQUIRE(ctx, d > 0 && std::isfinite(d), "d must be finite and > 0");
    KVB_REQUIRE(ctx, std::isfinite(beta), "beta must be finite");
    Prof pr(ctx, KVB_PROF_DENSITY);
    KVB_HIP(ctx, kvb::launch_density(idx, d2, nn, k, b, e, nullptr, d, beta, rho, psi, ctx->stream));
    return KVB_OK;
}

int kvb_grid_scale(kvb_ctx ctx, const float* ref, const float* rho, int64_t n, double* scale_host)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31)");
    KVB_REQUIRE(ctx, aligned(ref) && aligned(rho), "ref and rho must be non-null float32 device pointers");
    KVB_REQUIRE(ctx, scale_host != nullptr, "scale_host must be non-null");
    const int nn = static_cast<int>(n);
    const int nb = kvb::logsum_num_blocks(nn);
    int rc = ensure_scratch(ctx, round256(2 * nb * sizeof(double)) + 512);
    if (rc) return rc;
    Carve cv(ctx->scratch);
    double* part = cv.take<double>(2 * nb);
    double* out = cv.take<double>(1);
    {
        Prof pr(ctx, KVB_PROF_GRID_SCALE);
        KVB_HIP(ctx, kvb::launch_grid_scale(ref, rho, nn, part, out, ctx->stream));
    }
    KVB_HIP(ctx, hipMemcpyAsync(&ctx->tune_host->e_star, out, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    KVB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *scale_host = ctx->tune_host->e_star;
    if (!(std::isfinite(*scale_host) && *scale_host > 0))
        return fail(ctx, KVB_E_INVALID, "grid scale is not finite: inputs must be positive and finite");
    return KVB_OK;
}

int kvb_tune_eps(kvb_ctx ctx, const int32_t* idx, const float* d2, const float* rho, int64_t n, int32_t k,
                 double e_min, double e_max, int32_t G, double* chi_host, double* e_star_host, double* dim_host)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31)");
    KVB_REQUIRE(ctx, k >= 1 && k <= 256, "k must be in [1, 256], got %d", k);
    KVB_REQUIRE(ctx, G >= 3 && G <= 256, "G must be in [3, 256], got %d", G);
    KVB_REQUIRE(ctx, e_min > 0 && e_max > e_min && std::isfinite(e_max), "need 0 < e_min < e_max < inf");
    KVB_REQUIRE(ctx, aligned(idx) && aligned(d2) && aligned(rho), "idx, d2, rho must be non-null device pointers");
    KVB_REQUIRE(ctx, e_star_host != nullptr, "e_star_host must be non-null");
    const int64_t nnz = n * k;
    const int nb = kvb::chi_num_blocks(nnz);
    int rc = ensure_scratch(ctx, round256(size_t(nb) * G * sizeof(double)) + 256);
    if (rc) return rc;
    Carve cv(ctx->scratch);
    double* part = cv.take<double>(size_t(nb) * G);
    {
        Prof pr(ctx, KVB_PROF_CHI);
        KVB_HIP(ctx, kvb::launch_chi(idx, d2, rho, nnz, k, G, e_min, e_max, nullptr, part,
                                     ctx->tune_dev, ctx->stream));
    }
    KVB_HIP(ctx, hipMemcpyAsync(ctx->tune_host, ctx->tune_dev, sizeof(kvb::TuneResult), hipMemcpyDeviceToHost,
                                ctx->stream));
    KVB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const kvb::TuneResult& t = *ctx->tune_host;
    if (chi_host) std::memcpy(chi_host, t.chi, sizeof(double) * G);
    *e_star_host = t.e_star;
    if (dim_host) *dim_host = t.dim;
    return (t.g_star == 0 || t.g_star == G - 2) ? KVB_W_GRID_EDGE : KVB_OK;
}

int kvb_assemble_csr(kvb_ctx ctx, const int32_t* idx, const float* d2, const float* rho, int64_t n, int32_t k,
                     double e, double alpha, double d, int32_t out_kind, int64_t* rowptr, int32_t* col, float* val,
                     double* P, double* D)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31)");
    KVB_REQUIRE(ctx, k >= 1 && k <= 256, "k must be in [1, 256], got %d", k);
    KVB_REQUIRE(ctx, e > 0 && std::isfinite(e), "e must be finite and > 0");
    KVB_REQUIRE(ctx, std::isfinite(alpha) && std::isfinite(d) && d > 0, "alpha must be finite and d > 0");
    KVB_REQUIRE(ctx, out_kind >= KVB_OUT_MARKOV && out_kind <= KVB_OUT_SYMMETRIC, "unknown out_kind %d", out_kind);
    KVB_REQUIRE(ctx, aligned(idx) && aligned(d2) && aligned(rho), "idx, d2, rho must be non-null device pointers");
    KVB_REQUIRE(ctx, aligned(rowptr) && aligned(col) && aligned(val), "rowptr, col, val must be non-null");
    KVB_REQUIRE(ctx, (P == nullptr || aligned(P)) && (D == nullptr || aligned(D)), "P and D must be aligned");
    const int nn = static_cast<int>(n);
    int rc = ensure_scratch(ctx, 2 * round256(size_t(nn) * sizeof(double)) + 256);
    if (rc) return rc;
    Carve cv(ctx->scratch);
    double* qa = cv.take<double>(nn);
    double* Dtmp = cv.take<double>(nn);
    {
        Prof pr(ctx, KVB_PROF_QPASS);
        KVB_HIP(ctx, kvb::launch_qpass(idx, d2, nn, k, rho, e, nullptr, alpha, d, qa, ctx->stream));
    }
    {
        Prof pr(ctx, KVB_PROF_ASSEMBLE);
        KVB_HIP(ctx, kvb::launch_assemble(idx, d2, nn, k, rho, e, nullptr, qa, out_kind, rowptr, col, val, P,
                                          D ? D : Dtmp, ctx->stream));
    }
    return KVB_OK;
}

// ------------------------------------------------------------------ union pattern and CSR passes
// scratch of the transpose-merge: about 17 bytes per directed entry
static size_t union_work_bytes(int n, int64_t nk)
{
    return 2 * round256(size_t(nk) * 4) + round256(size_t(nk)) + round256(size_t(nk) * 8) +
           round256(size_t(n) * 32 * sizeof(uint16_t)) +
           round256((size_t(n) + 1) * 4) + round256((size_t(n) + 1) * 8) + 3 * round256(16) +
           round256(size_t(n) * 4) + round256(kvb::union_scan_bytes(n)) + 2048;
}

static kvb::UnionWork take_union_work(Carve& cv, int n, int64_t nk)
{
    kvb::UnionWork w;
    w.scol = cv.take<int32_t>(nk);
    w.sd2 = cv.take<float>(nk);
    w.flag = cv.take<uint8_t>(nk);
    w.boff = cv.take<uint16_t>(size_t(n) * 32);
    w.rkey = cv.take<uint64_t>(nk);
    w.cnt = cv.take<int>(size_t(n) + 1);
    w.revptr = cv.take<int64_t>(size_t(n) + 1);
    w.bad = cv.take<unsigned long long>(1);
    w.long_count = cv.take<int>(1);
    w.long_rows = cv.take<int>(n);
    w.scan_bytes = kvb::union_scan_bytes(n);
    w.scan_tmp = cv.take<char>(w.scan_bytes);
    return w;
}

int kvb_set_tolerance(kvb_ctx ctx, double delta)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, delta >= 0.0 && delta < 1.0, "delta must lie in [0, 1)");
    ctx->delta = delta;
    return KVB_OK;
}

int kvb_union_pattern(kvb_ctx ctx, const int32_t* idx, const float* d2, int64_t n, int32_t k, int64_t* rowptr,
                      int32_t* col, float* ud2, int64_t cap, int64_t* nnz_host)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31)");
    KVB_REQUIRE(ctx, k >= 1 && k <= 256 && k <= n, "k must be in [1, min(256, n)], got %d", k);
    KVB_REQUIRE(ctx, aligned(idx) && aligned(d2), "idx and d2 must be non-null device pointers");
    KVB_REQUIRE(ctx, aligned(rowptr) && aligned(col) && aligned(ud2), "rowptr, col, ud2 must be non-null");
    KVB_REQUIRE(ctx, nnz_host != nullptr, "nnz_host must be non-null");
    KVB_REQUIRE(ctx, cap >= 0, "cap must be >= 0");
    const int nn = static_cast<int>(n);
    const int64_t nk = n * k;
    int rc = ensure_scratch(ctx, union_work_bytes(nn, nk));
    if (rc) return rc;
    Carve cv(ctx->scratch);
    const kvb::UnionWork w = take_union_work(cv, nn, nk);
    Prof pr(ctx, KVB_PROF_UNION);
    KVB_HIP(ctx, kvb::launch_union_count(idx, d2, nn, k, w, ctx->stream));
    KVB_HIP(ctx, hipMemcpyAsync(ctx->union_host, w.revptr + nn, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    KVB_HIP(ctx, hipMemcpyAsync(ctx->union_host + 1, w.bad, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                ctx->stream));
    KVB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const int64_t total = static_cast<int64_t>(ctx->union_host[0]);
    if (ctx->union_host[1])
        return fail(ctx, KVB_E_INVALID, "idx: a row holds a column outside [0, n) or the same column twice");
    *nnz_host = nk + total;
    if (cap < nk + total)
        return fail(ctx, KVB_E_INVALID, "cap %lld is below the union's %lld entries", static_cast<long long>(cap),
                    static_cast<long long>(nk + total));
    KVB_HIP(ctx, kvb::launch_union_place(nn, k, w, rowptr, col, ud2, ctx->stream));
    return KVB_OK;
}

}  // extern "C"

// shape check of a caller's CSR pattern (synchronises)
int kvbh::check_pattern(kvb_ctx ctx, const int64_t* rowptr, const int32_t* col, int64_t n, int64_t nnz)
{
    KVB_REQUIRE(ctx, n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31)");
    KVB_REQUIRE(ctx, nnz >= 1, "nnz must be >= 1");
    KVB_REQUIRE(ctx, aligned(rowptr) && aligned(col), "rowptr and col must be non-null device pointers");
    int rc = ensure_scratch(ctx, 512);
    if (rc) return rc;
    Carve cv(ctx->scratch);
    unsigned long long* bad = cv.take<unsigned long long>(1);
    KVB_HIP(ctx, kvb::launch_check_csr(rowptr, col, static_cast<int>(n), nnz, bad, ctx->stream));
    KVB_HIP(ctx, hipMemcpyAsync(ctx->union_host, bad, sizeof(unsigned long long), hipMemcpyDeviceToHost, ctx->stream));
    KVB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->union_host[0] & 1)
        return fail(ctx, KVB_E_INVALID, "rowptr must start at 0, never decrease and end at nnz");
    if (ctx->union_host[0] & 2) return fail(ctx, KVB_E_INVALID, "col: a column lies outside [0, n)");
    return KVB_OK;
}

extern "C" {


int kvb_truncate_csr(kvb_ctx ctx, const int64_t* rowptr, const int32_t* col, const float* d2, const float* rho,
                     int64_t n, int64_t nnz, double e, double delta, int64_t* rowptr_out, int32_t* col_out,
                     float* d2_out, int64_t* nnz_host)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, e > 0 && std::isfinite(e), "e must be finite and > 0");
    KVB_REQUIRE(ctx, delta > 0 && delta < 1, "delta must lie in (0, 1)");
    KVB_REQUIRE(ctx, aligned(d2) && aligned(rho), "d2 and rho must be non-null device pointers");
    KVB_REQUIRE(ctx, aligned(rowptr_out) && aligned(col_out) && aligned(d2_out),
                "rowptr_out, col_out, d2_out must be non-null device pointers");
    KVB_TRY(check_pattern(ctx, rowptr, col, n, nnz));
    const int nn = static_cast<int>(n);
    const size_t scan_bytes = kvb::union_scan_bytes(nn);
    int rc = ensure_scratch(ctx, round256((size_t(nn) + 1) * sizeof(int)) + round256(scan_bytes) + 512);
    if (rc) return rc;
    Carve cv(ctx->scratch);
    int* cnt = cv.take<int>(size_t(nn) + 1);
    void* scan_tmp = cv.take<char>(scan_bytes);
    {
        Prof pr(ctx, KVB_PROF_TRUNCATE);
        KVB_HIP(ctx, kvb::launch_truncate(rowptr, col, d2, rho, nn, e, nullptr, -std::log(delta), cnt, scan_tmp,
                                          scan_bytes, rowptr_out, col_out, d2_out, ctx->stream));
    }
    if (nnz_host) {
        KVB_HIP(ctx, hipMemcpyAsync(ctx->union_host, rowptr_out + nn, sizeof(int64_t), hipMemcpyDeviceToHost,
                                    ctx->stream));
        KVB_HIP(ctx, hipStreamSynchronize(ctx->stream));
        *nnz_host = static_cast<int64_t>(ctx->union_host[0]);
    }
    return KVB_OK;
}

int kvb_density_csr(kvb_ctx ctx, const int64_t* rowptr, const int32_t* col, const float* ud2, int64_t n, int64_t nnz,
                    const float* b, double e, double d, double beta, float* rho, float* psi)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, aligned(ud2) && aligned(b) && aligned(rho), "ud2, b, rho must be non-null device pointers");
    KVB_REQUIRE(ctx, psi == nullptr || aligned(psi), "psi must be aligned");
    KVB_REQUIRE(ctx, e > 0 && std::isfinite(e), "e must be finite and > 0");
    KVB_REQUIRE(ctx, d > 0 && std::isfinite(d), "d must be finite and > 0");
    KVB_REQUIRE(ctx, std::isfinite(beta), "beta must be finite");
    KVB_TRY(check_pattern(ctx, rowptr, col, n, nnz));
    Prof pr(ctx, KVB_PROF_DENSITY);
    KVB_HIP(ctx, kvb::launch_density_csr(rowptr, col, ud2, static_cast<int>(n), b, e, nullptr, d, beta, rho, psi,
                                         ctx->stream));
    return KVB_OK;
}

int kvb_tune_eps_csr(kvb_ctx ctx, const int64_t* rowptr, const int32_t* col, const float* ud2, const float* rho,
                     int64_t n, int64_t nnz, double e_min, double e_max, int32_t G, double* chi_host,
                     double* e_star_host, double* dim_host)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, G >= 3 && G <= 256, "G must be in [3, 256], got %d", G);
    KVB_REQUIRE(ctx, e_min > 0 && e_max > e_min && std::isfinite(e_max), "need 0 < e_min < e_max < inf");
    KVB_REQUIRE(ctx, aligned(ud2) && aligned(rho), "ud2 and rho must be non-null device pointers");
    KVB_REQUIRE(ctx, e_star_host != nullptr, "e_star_host must be non-null");
    KVB_TRY(check_pattern(ctx, rowptr, col, n, nnz));
    const int nb = kvb::chi_num_blocks(nnz);
    int rc = ensure_scratch(ctx, round256(size_t(nb) * G * sizeof(double)) + 256);
    if (rc) return rc;
    Carve cv(ctx->scratch);
    double* part = cv.take<double>(size_t(nb) * G);
    {
        Prof pr(ctx, KVB_PROF_CHI);
        KVB_HIP(ctx, kvb::launch_chi_csr(rowptr, nullptr, col, ud2, static_cast<int>(n), nnz, nnz, rho, G, e_min,
                                         e_max, nullptr, part, ctx->tune_dev, ctx->stream));
    }
    KVB_HIP(ctx, hipMemcpyAsync(ctx->tune_host, ctx->tune_dev, sizeof(kvb::TuneResult), hipMemcpyDeviceToHost,
                                ctx->stream));
    KVB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const kvb::TuneResult& t = *ctx->tune_host;
    if (chi_host) std::memcpy(chi_host, t.chi, sizeof(double) * G);
    *e_star_host = t.e_star;
    if (dim_host) *dim_host = t.dim;
    return (t.g_star == 0 || t.g_star == G - 2) ? KVB_W_GRID_EDGE : KVB_OK;
}

int kvb_normalize_csr(kvb_ctx ctx, const int64_t* rowptr, const int32_t* col, const float* ud2, const float* rho,
                      int64_t n, int64_t nnz, double e, double alpha, double d, int32_t out_kind, float* val,
                      double* P, double* D)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, e > 0 && std::isfinite(e), "e must be finite and > 0");
    KVB_REQUIRE(ctx, std::isfinite(alpha) && std::isfinite(d) && d > 0, "alpha must be finite and d > 0");
    KVB_REQUIRE(ctx, out_kind >= KVB_OUT_MARKOV && out_kind <= KVB_OUT_SYMMETRIC, "unknown out_kind %d", out_kind);
    KVB_REQUIRE(ctx, aligned(ud2) && aligned(rho) && aligned(val), "ud2, rho, val must be non-null device pointers");
    KVB_REQUIRE(ctx, (P == nullptr || aligned(P)) && (D == nullptr || aligned(D)), "P and D must be aligned");
    KVB_TRY(check_pattern(ctx, rowptr, col, n, nnz));
    const int nn = static_cast<int>(n);
    int rc = ensure_scratch(ctx, 2 * round256(size_t(nn) * sizeof(double)) + 256);
    if (rc) return rc;
    Carve cv(ctx->scratch);
    double* qa = cv.take<double>(nn);
    double* Dtmp = cv.take<double>(nn);
    {
        Prof pr(ctx, KVB_PROF_QPASS);
        KVB_HIP(ctx, kvb::launch_qpass_csr(rowptr, col, ud2, nn, rho, e, nullptr, alpha, d, qa, ctx->stream));
    }
    {
        Prof pr(ctx, KVB_PROF_ASSEMBLE);
        KVB_HIP(ctx, kvb::launch_assemble_rows(rowptr, col, ud2, nn, rho, e, nullptr, qa, out_kind, val, P,
                                               D ? D : Dtmp, ctx->stream));
    }
    return KVB_OK;
}

// The passes of kvb_build after the k-NN over a CSR pattern: the union E u E^T
// (KVB_PATTERN_UNION) or the directed rows sorted by column, truncated at the
// context's sparsity tolerance when it is set. Enqueued only: the patterns'
// sizes stay on the device (the tuning sums are partitioned for n k entries
// and launched for the largest possible pattern, reading the true count from
// rowptr[n]).
static int build_csr(kvb_ctx ctx, int64_t n, int32_t k, int32_t k0, double d, double alpha, double beta,
                     double e_min, double e_max, int32_t G, int32_t out_kind, const int32_t* idx, const float* d2,
                     float* b, float* rho, float* psi, int64_t* rowptr, int32_t* col, float* val, double* P, double* D)
{
    const int nn = static_cast<int>(n);
    const int64_t nk = n * k;
    const bool uni = ctx->pattern == KVB_PATTERN_UNION;
    const bool trunc = ctx->delta > 0.0;
    const int64_t cap = uni ? n * (2 * int64_t(k) - 1) : nk;
    const int nb = kvb::chi_csr_blocks(nk, cap);
    const int lb = kvb::logsum_num_blocks(nn);
    const size_t scan_bytes = kvb::union_scan_bytes(nn);
    const size_t pat_bytes = round256((size_t(nn) + 1) * 8) + round256(size_t(cap) * 4) * 2;
    const size_t need = union_work_bytes(nn, nk) + pat_bytes * 3 + round256(size_t(cap) * 4) +
                        round256((size_t(nn) + 1) * 4) +
                        round256(scan_bytes) + round256(size_t(nb) * G * sizeof(double)) +
                        round256(size_t(2 * lb) * sizeof(double)) + 2 * round256(size_t(nn) * sizeof(double)) + 4096;
    int rc = ensure_scratch(ctx, need);
    if (rc) return rc;
    Carve cv(ctx->scratch);
    const kvb::UnionWork uw = take_union_work(cv, nn, nk);
    // base pattern: the caller's rowptr/col when it is also the operator pattern
    int64_t* brow = trunc ? cv.take<int64_t>(size_t(nn) + 1) : rowptr;
    int32_t* bcol = trunc ? cv.take<int32_t>(cap) : col;
    float* bd2 = cv.take<float>(cap);
    int64_t* arow = cv.take<int64_t>(size_t(nn) + 1);   // density pattern (truncated)
    int32_t* acol = cv.take<int32_t>(cap);
    float* ad2 = cv.take<float>(cap);
    float* od2 = cv.take<float>(cap);                    // operator pattern distances (truncated)
    int32_t* brid = cv.take<int32_t>(cap);               // row of every base entry
    int* tcnt = cv.take<int>(size_t(nn) + 1);
    void* tscan = cv.take<char>(scan_bytes);
    double* part = cv.take<double>(size_t(nb) * G);
    double* lpart = cv.take<double>(2 * lb);
    double* qa = cv.take<double>(nn);
    double* Dtmp = cv.take<double>(nn);
    BuildDev* bd = ctx->build_dev;
    hipStream_t st = ctx->stream;
    const double L = trunc ? -std::log(ctx->delta) : 0.0;
    {
        Prof pr(ctx, KVB_PROF_ADHOC);
        KVB_HIP(ctx, kvb::launch_adhoc_bandwidth(d2, nn, k, k0, b, st));
    }
    {
        Prof pr(ctx, KVB_PROF_UNION);
        if (uni) {
            KVB_HIP(ctx, kvb::launch_union_count(idx, d2, nn, k, uw, st));
            KVB_HIP(ctx, kvb::launch_union_place(nn, k, uw, brow, bcol, bd2, st));
        } else {
            KVB_HIP(ctx, kvb::launch_sorted_rows(idx, d2, nn, k, brow, bcol, bd2, st));
        }
        KVB_HIP(ctx, kvb::launch_row_ids(brow, nn, brid, st));   // read by both tuning passes
    }
    {
        Prof pr(ctx, KVB_PROF_CHI);
        KVB_HIP(ctx, kvb::launch_chi_csr(brow, brid, bcol, bd2, nn, nk, cap, b, G, e_min, e_max, nullptr, part, &bd->a,
                                         st));
    }
    const int64_t* drow = brow;
    const int32_t* dcol = bcol;
    const float* dd2 = bd2;
    if (trunc) {
        Prof pr(ctx, KVB_PROF_TRUNCATE);
        KVB_HIP(ctx, kvb::launch_truncate(brow, bcol, bd2, b, nn, 0.0, &bd->a.e_star, L, tcnt, tscan, scan_bytes, arow,
                                          acol, ad2, st));
        drow = arow;
        dcol = acol;
        dd2 = ad2;
    }
    {
        Prof pr(ctx, KVB_PROF_DENSITY);
        KVB_HIP(ctx, kvb::launch_density_csr(drow, dcol, dd2, nn, b, 0.0, &bd->a.e_star, d, beta, rho, psi, st));
    }
    {
        Prof pr(ctx, KVB_PROF_GRID_SCALE);
        KVB_HIP(ctx, kvb::launch_grid_scale(b, rho, nn, lpart, &bd->scale, st));
    }
    {
        Prof pr(ctx, KVB_PROF_CHI);
        KVB_HIP(ctx, kvb::launch_chi_csr(brow, brid, bcol, bd2, nn, nk, cap, rho, G, e_min, e_max, &bd->scale, part,
                                         &bd->b, st));
    }
    const float* od = bd2;
    if (trunc) {
        Prof pr(ctx, KVB_PROF_TRUNCATE);
        KVB_HIP(ctx, kvb::launch_truncate(brow, bcol, bd2, rho, nn, 0.0, &bd->b.e_star, L, tcnt, tscan, scan_bytes,
                                          rowptr, col, od2, st));
        od = od2;
    }
    {
        Prof pr(ctx, KVB_PROF_QPASS);
        KVB_HIP(ctx, kvb::launch_qpass_csr(rowptr, col, od, nn, rho, 0.0, &bd->b.e_star, alpha, d, qa, st));
    }
    {
        Prof pr(ctx, KVB_PROF_ASSEMBLE);
        KVB_HIP(ctx, kvb::launch_assemble_rows(rowptr, col, od, nn, rho, 0.0, &bd->b.e_star, qa, out_kind, val, P,
                                               D ? D : Dtmp, st));
    }
    return KVB_OK;
}

int kvb_build(kvb_ctx ctx, const float* X, int64_t n, int32_t m, int32_t k, int32_t mode, int32_t margin, int32_t k0,
              double d, double alpha, double beta, double e_min, double e_max, int32_t G, int32_t out_kind,
              int32_t* idx, float* d2, int32_t* row_flags, float* b, float* rho, float* psi, int64_t* rowptr,
              int32_t* col, float* val, double* P, double* D, double* chi_a_host, double* chi_b_host,
              double* info_host)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, k0 >= 1 && k0 < k, "k0 must be in [1, k), got k0=%d k=%d", k0, k);
    KVB_REQUIRE(ctx, k <= 256, "k must be <= 256, got %d", k);
    KVB_REQUIRE(ctx, G >= 3 && G <= 256, "G must be in [3, 256], got %d", G);
    KVB_REQUIRE(ctx, e_min > 0 && e_max > e_min && std::isfinite(e_max), "need 0 < e_min < e_max < inf");
    KVB_REQUIRE(ctx, d > 0 && std::isfinite(d) && std::isfinite(alpha) && std::isfinite(beta),
                "d must be finite and > 0, alpha and beta finite");
    KVB_REQUIRE(ctx, out_kind >= KVB_OUT_MARKOV && out_kind <= KVB_OUT_SYMMETRIC, "unknown out_kind %d", out_kind);
    KVB_REQUIRE(ctx, aligned(b) && aligned(rho) && (psi == nullptr || aligned(psi)),
                "b and rho must be non-null float32 device pointers");
    KVB_REQUIRE(ctx, aligned(rowptr) && aligned(col) && aligned(val), "rowptr, col, val must be non-null");
    KVB_REQUIRE(ctx, (P == nullptr || aligned(P)) && (D == nullptr || aligned(D)), "P and D must be aligned");
    const bool fixed_k = !(ctx->pattern == KVB_PATTERN_UNION || ctx->delta > 0.0);
    const int nn = static_cast<int>(n);
    const int64_t nnz = n * k;
    const int nb = kvb::chi_num_blocks(nnz);
    const int lb = kvb::logsum_num_blocks(nn);
    // the passes' own scratch; a matrix-core k-NN in curve order also leaves
    // room for the curve-ordered rows (its own scratch follows)
    const bool curve_possible = fixed_k && mode != KVB_KNN_LEARNED && !(mode == KVB_KNN_F32 && m <= 8) &&
                                ctx->curve_order && m <= 256;
    size_t own = round256(size_t(nb) * G * sizeof(double)) + round256(size_t(2 * lb) * sizeof(double)) +
                 2 * round256(size_t(nn) * sizeof(double)) + 1024;
    if (curve_possible)
        own += round256(size_t(nnz) * sizeof(int32_t)) + round256(size_t(nnz) * sizeof(float)) +
               3 * round256(size_t(nn) * sizeof(float));
    own = round256(own);
    CurveRows cr;
    int rc = knn_run(ctx, fixed_k ? own : 0, X, n, m, k, mode, margin, idx, d2, row_flags,
                     curve_possible ? &cr : nullptr);
    if (rc < 0) return rc;
    if (!fixed_k) {
        rc = build_csr(ctx, n, k, k0, d, alpha, beta, e_min, e_max, G, out_kind, idx, d2, b, rho, psi, rowptr, col,
                       val, P, D);
        if (rc < 0) return rc;
        ctx->build_G = G;
        if (!info_host) return KVB_OK;
        return kvb_build_info(ctx, chi_a_host, chi_b_host, info_host);
    }
    rc = ensure_scratch(ctx, own);
    if (rc) return rc;
    Carve cv(ctx->scratch);
    double* part = cv.take<double>(size_t(nb) * G);
    double* lpart = cv.take<double>(2 * lb);
    double* qa = cv.take<double>(nn);
    double* Dtmp = cv.take<double>(nn);
    BuildDev* bd = ctx->build_dev;
    hipStream_t st = ctx->stream;
    // With the curve order: the rows, bandwidths, densities and q in curve
    // order (neighbours as curve positions), the matrix rows written back by
    // sample id. Otherwise every vector by sample id.
    const bool cv_rows = cr.cid != nullptr;
    const int32_t* pidx = idx;
    const float* pd2 = d2;
    float *pb = b, *prho = rho, *ppsi = psi;
    if (cv_rows) {
        int32_t* idx_c = cv.take<int32_t>(size_t(nnz));
        float* d2_c = cv.take<float>(size_t(nnz));
        pb = cv.take<float>(nn);
        prho = cv.take<float>(nn);
        ppsi = cv.take<float>(nn);
        pidx = idx_c;
        pd2 = d2_c;
        Prof pr(ctx, KVB_PROF_CURVE_ROWS);
        KVB_HIP(ctx, kvb::launch_curve_rows(idx, d2, nn, k, k0, cr.cid, cr.pos, idx_c, d2_c, pb, st));
    } else {
        Prof pr(ctx, KVB_PROF_ADHOC);
        KVB_HIP(ctx, kvb::launch_adhoc_bandwidth(d2, nn, k, k0, b, st));
    }
    {
        Prof pr(ctx, KVB_PROF_CHI);
        KVB_HIP(ctx, kvb::launch_chi(pidx, pd2, pb, nnz, k, G, e_min, e_max, nullptr, part, &bd->a, st));
    }
    {
        Prof pr(ctx, KVB_PROF_DENSITY);
        KVB_HIP(ctx, kvb::launch_density(pidx, pd2, nn, k, pb, 0.0, &bd->a.e_star, d, beta, prho,
                                         cv_rows ? ppsi : psi, st));
    }
    {
        Prof pr(ctx, KVB_PROF_GRID_SCALE);
        KVB_HIP(ctx, kvb::launch_grid_scale(pb, prho, nn, lpart, &bd->scale, st));
    }
    {
        Prof pr(ctx, KVB_PROF_CHI);
        KVB_HIP(ctx, kvb::launch_chi(pidx, pd2, prho, nnz, k, G, e_min, e_max, &bd->scale, part, &bd->b, st));
    }
    {
        Prof pr(ctx, KVB_PROF_QPASS);
        KVB_HIP(ctx, kvb::launch_qpass(pidx, pd2, nn, k, prho, 0.0, &bd->b.e_star, alpha, d, qa, st));
    }
    if (cv_rows)
        KVB_HIP(ctx, kvb::launch_gather_samples(cr.pos, nn, pb, b, prho, rho, ppsi, psi, st));
    {
        Prof pr(ctx, KVB_PROF_ASSEMBLE);
        KVB_HIP(ctx, kvb::launch_assemble(pidx, pd2, nn, k, prho, 0.0, &bd->b.e_star, qa, out_kind, rowptr, col, val,
                                          P, D ? D : Dtmp, st, cv_rows ? cr.cid : nullptr, cv_rows ? idx : nullptr,
                                          rho));
    }
    ctx->build_G = G;
    if (!info_host) return KVB_OK;
    return kvb_build_info(ctx, chi_a_host, chi_b_host, info_host);
}

int kvb_build_info(kvb_ctx ctx, double* chi_a_host, double* chi_b_host, double* info_host)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, info_host != nullptr, "info_host must be non-null");
    const int G = ctx->build_G;
    KVB_REQUIRE(ctx, G > 0, "no build has run on this context");
    hipStream_t st = ctx->stream;
    KVB_HIP(ctx, hipMemcpyAsync(ctx->build_host, ctx->build_dev, sizeof(BuildDev), hipMemcpyDeviceToHost, st));
    KVB_HIP(ctx, hipMemcpyAsync(ctx->fb_count_host, ctx->fb_count_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    KVB_HIP(ctx, hipStreamSynchronize(st));
    const BuildDev& h = *ctx->build_host;
    if (chi_a_host) std::memcpy(chi_a_host, h.a.chi, sizeof(double) * G);
    if (chi_b_host) std::memcpy(chi_b_host, h.b.chi, sizeof(double) * G);
    info_host[0] = h.a.e_star;
    info_host[1] = h.a.dim;
    info_host[2] = h.scale;
    info_host[3] = h.b.e_star;
    info_host[4] = h.b.dim;
    info_host[5] = h.a.g_star;
    info_host[6] = h.b.g_star;
    info_host[7] = *ctx->fb_count_host;
    if (!(std::isfinite(h.scale) && h.scale > 0))
        return fail(ctx, KVB_E_INVALID, "grid scale is not finite: bandwidths must be positive and finite");
    const bool edge = h.a.g_star == 0 || h.a.g_star == G - 2 || h.b.g_star == 0 || h.b.g_star == G - 2;
    if (edge) return KVB_W_GRID_EDGE;
    return *ctx->fb_count_host > 0 ? KVB_W_FALLBACK : KVB_OK;
}

const char* kvb_version(void) { return "kvb 0.1 (gfx950)"; }

int kvb_profile_enable(kvb_ctx ctx, int32_t on)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_DEVICE_WORK(ctx);
    int rc = prof_collect(ctx);
    if (rc) return rc;
    for (int s = 0; s < KVB_PROF_SLOTS; ++s) {
        ctx->prof_ms[s] = 0.0;
        ctx->prof_count[s] = 0;
    }
    ctx->prof_on = on != 0;
    // events are created up front, not while timed work is being enqueued
    while (ctx->prof_on && ctx->ev_pool.size() < 512) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) break;
        ctx->ev_pool.push_back(e);
    }
    return KVB_OK;
}

int kvb_profile_read(kvb_ctx ctx, int32_t slot, double* total_ms_host, int64_t* launches_host)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, slot >= 0 && slot < KVB_PROF_SLOTS, "profile slot %d out of range", slot);
    KVB_REQUIRE(ctx, total_ms_host && launches_host, "outputs must be non-null");
    int rc = prof_collect(ctx);
    if (rc) return rc;
    *total_ms_host = ctx->prof_ms[slot];
    *launches_host = ctx->prof_count[slot];
    return KVB_OK;
}

const char* kvb_profile_name(int32_t slot)
{
    return (slot >= 0 && slot < KVB_PROF_SLOTS) ? kProfNames[slot] : "";
}

}  // extern "C"
