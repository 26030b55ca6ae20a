// Context state of libkvb.so and the host helpers shared by the entry points
// (internal: not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "kvb_kernels.h"

namespace kvbh {

struct ProfPair {
    int slot;
    hipEvent_t a, b;
};

// Parameters and training state of the learned partitioner. The parameters
// live in one flat float32 buffer, W1 [h1, mpad] (columns m..mpad-1 zero), b1,
// W2 [h2, h1], b2, W3 [nb, h2], b3, with Adam moments and gradients of the
// same layout and a BF16 copy used by the matrix-core GEMMs.
struct PartState {
    int m = 0, mpad = 0, h1 = 0, h2 = 0, nb = 0, np = 0;
    int64_t off[6] = {};
    int64_t total = 0;
    float* p = nullptr;
    float* m1 = nullptr;
    float* m2 = nullptr;
    float* g = nullptr;
    uint16_t* pb = nullptr;    // BF16 copy of p
    uint16_t* w2t = nullptr;   // BF16 W2^T [h1, h2]
    uint16_t* w3t = nullptr;   // BF16 W3^T [h2, nb]
    void* block = nullptr;     // the one device allocation holding all of the above
    int64_t step = 0;          // Adam steps taken
    bool ready = false;
    int64_t nparams() const { return int64_t(h1) * m + h1 + int64_t(h2) * h1 + h2 + int64_t(nb) * h2 + nb; }
};

// Tuning results of both stages and the grid scale, kept on the device
// between the steps of kvb_build.
struct BuildDev {
    kvb::TuneResult a, b;
    double scale;
    double pad;
};

}  // namespace kvbh

struct kvb_ctx_s {
    hipStream_t stream = nullptr;
    int device = 0;
    bool host_only = false;   // kvb_create_host: validation only, no device work
    std::string err;
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    size_t scratch_limit = 0;
    int64_t force_fallback = 0;
    int bf16_split = 3;
    int curve_order = 2;
    int pattern = KVB_PATTERN_KNN;   // pattern of kvb_build's matrix
    double delta = 0.0;              // sparsity tolerance of kvb_build (0: keep every entry)
    int build_G = 0;   // grid size of the last kvb_build (0: none yet)
    kvb::TuneResult* tune_dev = nullptr;
    kvb::TuneResult* tune_host = nullptr;   // pinned
    kvbh::BuildDev* build_dev = nullptr;    // device-resident tuning results of kvb_build
    kvbh::BuildDev* build_host = nullptr;   // pinned
    int* fb_count_dev = nullptr;            // fallback rows of the last kvb_knn
    int* fb_count_host = nullptr;           // pinned
    unsigned long long* pairs_dev = nullptr;   // candidate pairs scored by the last kvb_knn
    unsigned long long* pairs_host = nullptr;  // pinned
    unsigned long long* union_host = nullptr;  // pinned [2]: reverse entries / check flags, invalid-input flag
    double* loss_dev = nullptr;             // per-epoch losses of kvb_part_train (device)
    int loss_cap = 0;
    kvbh::PartState part;
    // instrumentation: HIP events around each kernel launch on the context stream
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<kvbh::ProfPair> ev_pending;
    double prof_ms[KVB_PROF_SLOTS] = {};
    int64_t prof_count[KVB_PROF_SLOTS] = {};
};

namespace kvbh {

// shape check of a caller's CSR pattern: rowptr[0] = 0, non-decreasing,
// rowptr[n] = nnz, columns in [0, n) (one synchronisation)
int check_pattern(kvb_ctx ctx, const int64_t* rowptr, const int32_t* col, int64_t n, int64_t nnz);

inline int fail(kvb_ctx ctx, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return code;
}

// A host-only context (kvb_create_host) stops where device work would start,
// after all argument checks: at the first KVB_HIP call of an entry point, or
// at KVB_DEVICE_WORK where an entry point allocates or times on the device
// by other means.
#define KVB_DEVICE_WORK(ctx)                                                                   \
    do {                                                                                       \
        if ((ctx) && (ctx)->host_only)                                                         \
            return ::kvbh::fail((ctx), KVB_E_NO_DEVICE, "host-only context: the arguments are valid; nothing ran"); \
    } while (0)

#define KVB_HIP(ctx, call)                                                                     \
    do {                                                                                       \
        KVB_DEVICE_WORK(ctx);                                                                  \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::kvbh::fail((ctx), KVB_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define KVB_REQUIRE(ctx, cond, ...)                                                            \
    do {                                                                                       \
        if (!(cond)) return ::kvbh::fail((ctx), KVB_E_INVALID, __VA_ARGS__);                   \
    } while (0)

#define KVB_TRY(expr)                                                                          \
    do {                                                                                       \
        int rc_ = (expr);                                                                      \
        if (rc_ < 0) return rc_;                                                               \
    } while (0)

template <typename T>
bool aligned(const T* p)
{
    return p != nullptr && (reinterpret_cast<uintptr_t>(p) % alignof(T)) == 0;
}

// Bump allocator over the context scratch buffer; every region is 256-byte aligned.
struct Carve {
    char* base;
    size_t off = 0;
    explicit Carve(void* b) : base(static_cast<char*>(b)) {}
    template <typename T>
    T* take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base + off);
        off += count * sizeof(T);
        return p;
    }
};

inline size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

// scratch of the exact fallback: per-row bounds and the bounded pass buffers
inline size_t fallback_bytes(int n)
{
    const size_t cap = static_cast<size_t>(kvb::fallback_rows_cap(n));
    return round256(size_t(n) * sizeof(float)) + round256(cap * sizeof(int)) +
           round256(cap * kvb::FB_CAP * sizeof(double)) + round256(cap * kvb::FB_CAP * sizeof(int)) + 1024;
}

inline kvb::FallbackWork take_fallback(Carve& cv, int n, float** bound)
{
    const size_t cap = static_cast<size_t>(kvb::fallback_rows_cap(n));
    kvb::FallbackWork fw;
    *bound = cv.take<float>(n);
    fw.bound = *bound;
    fw.cnt = cv.take<int>(cap);
    fw.bd = cv.take<double>(cap * kvb::FB_CAP);
    fw.bj = cv.take<int>(cap * kvb::FB_CAP);
    return fw;
}

inline int ensure_scratch(kvb_ctx ctx, size_t bytes)
{
    if (bytes <= ctx->scratch_bytes) return KVB_OK;
    if (ctx->scratch_limit && bytes > ctx->scratch_limit)
        return fail(ctx, KVB_E_NOMEM, "scratch of %zu bytes exceeds the limit of %zu bytes", bytes,
                    ctx->scratch_limit);
    KVB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->scratch) {
        KVB_HIP(ctx, hipFree(ctx->scratch));
        ctx->scratch = nullptr;
        ctx->scratch_bytes = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, KVB_E_NOMEM, "hipMalloc of %zu scratch bytes failed", bytes);
    }
    ctx->scratch = p;
    ctx->scratch_bytes = bytes;
    return KVB_OK;
}

inline int check_ctx(kvb_ctx ctx) { return ctx ? KVB_OK : KVB_E_INVALID; }

// Looks up (once per device, with that device current) the device address of
// the static scratch array of the allocation-free entry point (noalloc.hip).
int noalloc_scratch_init(int device);

inline hipEvent_t pool_event(kvb_ctx ctx)
{
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one launch sequence with events when instrumentation is on.
struct Prof {
    kvb_ctx ctx;
    int slot;
    hipEvent_t a = nullptr;
    Prof(kvb_ctx c, int s) : ctx(c), slot(s)
    {
        if (ctx->prof_on && (a = pool_event(ctx)) != nullptr) (void)hipEventRecord(a, ctx->stream);
    }
    ~Prof()
    {
        if (!a) return;
        hipEvent_t b = pool_event(ctx);
        if (!b) {
            ctx->ev_pool.push_back(a);
            return;
        }
        (void)hipEventRecord(b, ctx->stream);
        ctx->ev_pending.push_back({slot, a, b});
    }
};

inline int prof_collect(kvb_ctx ctx)
{
    if (ctx->ev_pending.empty()) return KVB_OK;
    KVB_HIP(ctx, hipEventSynchronize(ctx->ev_pending.back().b));
    for (const ProfPair& p : ctx->ev_pending) {
        float ms = 0.f;
        KVB_HIP(ctx, hipEventElapsedTime(&ms, p.a, p.b));
        ctx->prof_ms[p.slot] += ms;
        ctx->prof_count[p.slot] += 1;
        ctx->ev_pool.push_back(p.a);
        ctx->ev_pool.push_back(p.b);
    }
    ctx->ev_pending.clear();
    return KVB_OK;
}

// k-NN through the learned partitioner (learned_api.hip).
int learned_knn(kvb_ctx ctx, const float* X, int n, int m, int k, int kp, int32_t* idx, float* d2,
                int32_t* row_flags);
void part_free(kvb_ctx ctx);

}  // namespace kvbh
