// The union pattern E u E^T of a directed k-NN pattern (gfx950).
//
// The paper's kernel matrix is symmetric: its brute-force construction sets
// K_ij and K_ji together (Section 4, Algorithm 1). A k-NN row i stores the k
// nearest samples of i, so (i, j) may be stored while (j, i) is not. The
// union pattern stores, in row i, every j with j in N(i) or i in N(j), each
// once, columns ascending, with the squared distance of the pair.
//
// The transpose-merge runs in five data-parallel steps, none of which depends
// on the order in which atomics land:
//   1. each directed row is sorted by column (one wavefront per row);
//   2. every entry (i, j), j != i, looks i up in the sorted row j by binary
//      search; when it is absent, (j, i) is an entry that only the transpose
//      contributes: row j's count is incremented and the pair is appended to
//      a list (the append order is arbitrary);
//   3. an exclusive scan of the counts gives each row's reverse segment and
//      rowptr_i = i k + (reverse entries of rows before i);
//   4. a radix sort of the appended pairs by (row, column) puts each row's
//      reverse entries in its segment, columns ascending;
//   5. every entry's place in its merged row is its rank in its own sorted
//      list plus the number of entries of the other list with a smaller
//      column (a binary search); the two lists are disjoint, so the places
//      are distinct.
// The HBM traffic is a few passes over the n k entries plus the sort of the
// reverse entries; the binary searches gather from rows that stay in L2.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "kvb_device.h"
#include "kvb_kernels.h"

namespace kvb {

// 1. directed row i sorted by column: key = column << 32 | bits of d2
template <int E>
__global__ __launch_bounds__(256) void k_union_sort_rows(const int32_t* __restrict__ idx,
                                                         const float* __restrict__ d2, int n, int k,
                                                         int32_t* __restrict__ scol, float* __restrict__ sd2)
{
    const int lane = lane_id();
    const int i = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (i >= n) return;
    const size_t base = static_cast<size_t>(i) * k;
    uint64_t key[E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int r = s * WAVE + lane;
        key[s] = r < k ? ((static_cast<uint64_t>(static_cast<uint32_t>(idx[base + r])) << 32) |
                          __float_as_uint(d2[base + r]))
                       : ~0ull;
    }
    bitonic_sort<E>(key);
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int r = s * WAVE + lane;
        if (r < k) {
            scol[base + r] = static_cast<int32_t>(key[s] >> 32);
            sd2[base + r] = __uint_as_float(static_cast<uint32_t>(key[s]));
        }
    }
}

// number of entries of the ascending list a[0..len) smaller than v
__device__ __forceinline__ int64_t count_less(const int32_t* __restrict__ a, int64_t len, int32_t v)
{
    int64_t lo = 0, hi = len;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// 2. entries that only the transpose contributes: (j, i) with j in N(i), i not in N(j).
// stats[0] counts them; stats[1] becomes non-zero if a row holds a column
// outside [0, n) or the same column twice (such entries are skipped, so no
// access leaves the arrays).
__global__ __launch_bounds__(256) void k_union_count(const int32_t* __restrict__ scol, const float* __restrict__ sd2,
                                                     int n, int k, int bits, int* __restrict__ cnt,
                                                     unsigned long long* __restrict__ stats,
                                                     uint64_t* __restrict__ rkey, float* __restrict__ rd2)
{
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= static_cast<int64_t>(n) * k) return;
    const int i = static_cast<int>(p / k);
    const int r = static_cast<int>(p - static_cast<int64_t>(i) * k);
    const int j = scol[p];
    if (j < 0 || j >= n || (r > 0 && scol[p - 1] == j)) {
        atomicOr(stats + 1, 1ull);
        return;
    }
    if (j == i) return;
    const int32_t* rj = scol + static_cast<size_t>(j) * k;
    const int64_t at = count_less(rj, k, i);
    if (at < k && rj[at] == i) return;   // mutual: row j stores (j, i) itself
    atomicAdd(cnt + j, 1);
    const unsigned long long slot = atomicAdd(stats, 1ull);
    rkey[slot] = (static_cast<uint64_t>(j) << bits) | static_cast<uint64_t>(i);
    rd2[slot] = sd2[p];
}

// 3. rowptr_i = i k + revptr_i (revptr: exclusive scan of the counts, n + 1 entries)
__global__ __launch_bounds__(256) void k_union_rowptr(const int64_t* __restrict__ revptr, int n, int k,
                                                      int64_t* __restrict__ rowptr)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) rowptr[i] = static_cast<int64_t>(i) * k + revptr[i];
}

// 5a. a directed entry's place: its rank r in the sorted row plus the reverse
// entries of the row with a smaller column
__global__ __launch_bounds__(256) void k_union_place_direct(const int32_t* __restrict__ scol,
                                                            const float* __restrict__ sd2, int n, int k,
                                                            const int64_t* __restrict__ revptr,
                                                            const int32_t* __restrict__ rcol,
                                                            const int64_t* __restrict__ rowptr,
                                                            int32_t* __restrict__ col, float* __restrict__ ud2)
{
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= static_cast<int64_t>(n) * k) return;
    const int i = static_cast<int>(p / k);
    const int r = static_cast<int>(p - static_cast<int64_t>(i) * k);
    const int32_t c = scol[p];
    const int64_t rb = revptr[i];
    const int64_t at = rowptr[i] + r + count_less(rcol + rb, revptr[i + 1] - rb, c);
    col[at] = c;
    ud2[at] = sd2[p];
}

// 5b. a reverse entry's place: its rank in the row's reverse segment plus the
// directed entries of the row with a smaller column. The sorted keys are
// row << bits | column; rcol receives the columns for 5a.
__global__ __launch_bounds__(256) void k_union_split_keys(const uint64_t* __restrict__ skey, int64_t total, int bits,
                                                          int32_t* __restrict__ rcol)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < total) rcol[t] = static_cast<int32_t>(skey[t] & ((1ull << bits) - 1));
}

__global__ __launch_bounds__(256) void k_union_place_reverse(const uint64_t* __restrict__ skey,
                                                             const float* __restrict__ srd2, int64_t total, int bits,
                                                             const int32_t* __restrict__ scol, int k,
                                                             const int64_t* __restrict__ revptr,
                                                             const int64_t* __restrict__ rowptr,
                                                             int32_t* __restrict__ col, float* __restrict__ ud2)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const uint64_t key = skey[t];
    const int j = static_cast<int>(key >> bits);
    const int32_t c = static_cast<int32_t>(key & ((1ull << bits) - 1));
    const int64_t at = rowptr[j] + (t - revptr[j]) + count_less(scol + static_cast<size_t>(j) * k, k, c);
    col[at] = c;
    ud2[at] = srd2[t];
}

// Shape of a caller's CSR pattern: bad |= 1 unless rowptr_0 = 0, rowptr_n = nnz
// and rowptr is non-decreasing; bad |= 2 if a column lies outside [0, n).
__global__ __launch_bounds__(256) void k_check_csr(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                                   int n, int64_t nnz, unsigned long long* __restrict__ bad)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    unsigned long long f = 0;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < nnz || t <= n; t += stride) {
        if (t <= n) {
            const int64_t v = rowptr[t];
            if ((t == 0 && v != 0) || (t == n && v != nnz) || (t < n && rowptr[t + 1] < v)) f |= 1;
        }
        if (t < nnz) {
            const int32_t c = col[t];
            if (c < 0 || c >= n) f |= 2;
        }
    }
    if (f) atomicOr(bad, f);
}

// ------------------------------------------------------------------ launchers
static unsigned grid_of(int64_t cnt) { return static_cast<unsigned>((cnt + 255) / 256); }

int union_key_bits(int n)
{
    int b = 1;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

hipError_t launch_union_count(const int32_t* idx, const float* d2, int n, int k, int32_t* scol, float* sd2, int* cnt,
                              unsigned long long* stats, uint64_t* rkey, float* rd2, hipStream_t st)
{
    const dim3 rows((n + 3) / 4), block(256);
    if (k <= 64)
        hipLaunchKernelGGL((k_union_sort_rows<1>), rows, block, 0, st, idx, d2, n, k, scol, sd2);
    else if (k <= 128)
        hipLaunchKernelGGL((k_union_sort_rows<2>), rows, block, 0, st, idx, d2, n, k, scol, sd2);
    else
        hipLaunchKernelGGL((k_union_sort_rows<4>), rows, block, 0, st, idx, d2, n, k, scol, sd2);
    // n + 1 counts: the last stays zero, so the scan's last entry is the total
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int) * (static_cast<size_t>(n) + 1), st);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(stats, 0, 2 * sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
    const int64_t nk = static_cast<int64_t>(n) * k;
    hipLaunchKernelGGL(k_union_count, dim3(grid_of(nk)), block, 0, st, scol, sd2, n, k, union_key_bits(n), cnt, stats,
                       rkey, rd2);
    return hipGetLastError();
}

size_t union_scan_bytes(int n)
{
    size_t b = 0;
    (void)rocprim::exclusive_scan(nullptr, b, static_cast<const int*>(nullptr), static_cast<int64_t*>(nullptr),
                                  int64_t(0), static_cast<size_t>(n) + 1, rocprim::plus<int64_t>(), nullptr);
    return b;
}

size_t union_sort_bytes(int64_t cap)
{
    size_t b = 0;
    (void)rocprim::radix_sort_pairs(nullptr, b, static_cast<const uint64_t*>(nullptr), static_cast<uint64_t*>(nullptr),
                                    static_cast<const float*>(nullptr), static_cast<float*>(nullptr),
                                    static_cast<size_t>(cap), 0u, 64u, nullptr);
    return b;
}

// cnt must hold n + 1 entries, the last zero: its scan is the total
hipError_t launch_union_scan(void* tmp, size_t tmp_bytes, const int* cnt, int n, int k, int64_t* revptr,
                             int64_t* rowptr, hipStream_t st)
{
    hipError_t e = rocprim::exclusive_scan(tmp, tmp_bytes, cnt, revptr, int64_t(0), static_cast<size_t>(n) + 1,
                                           rocprim::plus<int64_t>(), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_union_rowptr, dim3(grid_of(int64_t(n) + 1)), dim3(256), 0, st, revptr, n, k, rowptr);
    return hipGetLastError();
}

hipError_t launch_union_place(void* tmp, size_t tmp_bytes, const uint64_t* rkey, uint64_t* skey, const float* rd2,
                              float* srd2, int64_t total, const int32_t* scol, const float* sd2, int n, int k,
                              const int64_t* revptr, const int64_t* rowptr, int32_t* rcol, int32_t* col, float* ud2,
                              hipStream_t st)
{
    const int bits = union_key_bits(n);
    if (total > 0) {
        hipError_t e = rocprim::radix_sort_pairs(tmp, tmp_bytes, rkey, skey, rd2, srd2, static_cast<size_t>(total),
                                                 0u, static_cast<unsigned>(2 * bits), st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_union_split_keys, dim3(grid_of(total)), dim3(256), 0, st, skey, total, bits, rcol);
        hipLaunchKernelGGL(k_union_place_reverse, dim3(grid_of(total)), dim3(256), 0, st, skey, srd2, total, bits,
                           scol, k, revptr, rowptr, col, ud2);
    }
    const int64_t nk = static_cast<int64_t>(n) * k;
    hipLaunchKernelGGL(k_union_place_direct, dim3(grid_of(nk)), dim3(256), 0, st, scol, sd2, n, k, revptr, rcol,
                       rowptr, col, ud2);
    return hipGetLastError();
}

hipError_t launch_check_csr(const int64_t* rowptr, const int32_t* col, int n, int64_t nnz, unsigned long long* bad,
                            hipStream_t st)
{
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
    const int64_t cnt = nnz > int64_t(n) + 1 ? nnz : int64_t(n) + 1;
    const int64_t blocks = (cnt + 255) / 256;
    hipLaunchKernelGGL(k_check_csr, dim3(static_cast<unsigned>(blocks < 4096 ? blocks : 4096)), dim3(256), 0, st, rowptr,
                       col, n, nnz, bad);
    return hipGetLastError();
}

}  // namespace kvb
