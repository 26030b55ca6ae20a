// The allocation-free variant of kvb_tune_eps, for callers that cannot
// allocate device memory during a call (tight serving loops, code that runs
// under a harness forbidding allocation). Its scratch - the tuning sums' block
// partials and the device copy of the result - lives in a file-scope device
// array of fixed size. Each GPU holds its own copy of the array from the time
// the library's code object is loaded on it until the process ends. Its device
// address is looked up once per device, when a context is created on that
// device, and kept in a per-device table; host code never passes the array's
// own name to a kernel or a copy (in host code that name is only a stand-in
// for the symbol, not a device address).
//
// Every call on one GPU shares that GPU's array: calls that overlap in time on
// one GPU (different streams or host threads) race on it, so the caller must
// order them. Nothing in the array needs to start at zero: every block writes
// its partials in full, and the reductions write the whole result.
#include <cmath>
#include <cstring>
#include <mutex>

#include "kvb_ctx.h"
#include "kvb_kernels.h"

namespace {

// the tuning partials (at most 1024 blocks x 256 grid points x 8 bytes =
// 2 MiB) and the result struct fit with room to spare
constexpr size_t NOALLOC_BYTES = size_t(4) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

size_t round256_na(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

namespace kvbh {

int noalloc_scratch_init(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return KVB_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return KVB_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        return KVB_E_HIP;
    }
    g_noalloc_ptr[device] = p;
    return KVB_OK;
}

static void* noalloc_scratch(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    return g_noalloc_ptr[device];
}

}  // namespace kvbh

using namespace kvbh;

int kvb_tune_eps_noalloc(kvb_ctx ctx, const int32_t* idx, const float* d2, const float* rho, int64_t n, int32_t k,
                         double e_min, double e_max, int32_t G, double* chi_host, double* e_star_host,
                         double* dim_host)
{
    if (check_ctx(ctx)) return KVB_E_INVALID;
    KVB_REQUIRE(ctx, n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31)");
    KVB_REQUIRE(ctx, k >= 1 && k <= 256, "k must be in [1, 256], got %d", k);
    KVB_REQUIRE(ctx, G >= 3 && G <= 256, "G must be in [3, 256], got %d", G);
    KVB_REQUIRE(ctx, e_min > 0 && e_max > e_min && std::isfinite(e_max), "need 0 < e_min < e_max < inf");
    KVB_REQUIRE(ctx, aligned(idx) && aligned(d2) && aligned(rho), "idx, d2, rho must be non-null device pointers");
    KVB_REQUIRE(ctx, e_star_host != nullptr, "e_star_host must be non-null");
    KVB_DEVICE_WORK(ctx);
    void* base = noalloc_scratch(ctx->device);
    if (!base) return fail(ctx, KVB_E_UNSUPPORTED, "no static scratch on device %d", ctx->device);
    const int64_t nnz = n * k;
    const int nb = kvb::chi_num_blocks(nnz);
    const size_t part_bytes = round256_na(size_t(nb) * G * sizeof(double));
    const size_t need = part_bytes + round256_na(sizeof(kvb::TuneResult));
    if (need > NOALLOC_BYTES)
        return fail(ctx, KVB_E_UNSUPPORTED, "the tuning needs %zu bytes of scratch, beyond the %zu-byte static array",
                    need, NOALLOC_BYTES);
    double* part = static_cast<double*>(base);
    kvb::TuneResult* res = reinterpret_cast<kvb::TuneResult*>(static_cast<char*>(base) + part_bytes);
    KVB_HIP(ctx, kvb::launch_chi(idx, d2, rho, nnz, k, G, e_min, e_max, nullptr, part, res, ctx->stream));
    // the context's pinned result buffer was allocated with the context
    KVB_HIP(ctx, hipMemcpyAsync(ctx->tune_host, res, sizeof(kvb::TuneResult), hipMemcpyDeviceToHost, ctx->stream));
    KVB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const kvb::TuneResult& t = *ctx->tune_host;
    if (chi_host) std::memcpy(chi_host, t.chi, sizeof(double) * G);
    *e_star_host = t.e_star;
    if (dim_host) *dim_host = t.dim;
    return (t.g_star == 0 || t.g_star == G - 2) ? KVB_W_GRID_EDGE : KVB_OK;
}
