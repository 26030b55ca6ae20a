// Pattern transforms (gfx950): the union E u E^T of a directed k-NN pattern,
// the threshold truncation of any CSR pattern, and the shape check of a
// caller's CSR pattern.
//
// The paper's kernel matrix is symmetric: its brute-force construction sets
// K_ij and K_ji together (Section 4, Algorithm 1). A k-NN row i stores the k
// nearest samples of i, so (i, j) may be stored while (j, i) is not. The
// union pattern stores, in row i, every j with j in N(i) or i in N(j), each
// once, columns ascending, with the squared distance of the pair.
//
// The transpose-merge runs in data-parallel steps whose result does not depend
// on the order in which atomics land:
//   1. each directed row is sorted by column (one wavefront per row);
//   2. every entry (i, j), j != i, looks i up in the sorted row j by binary
//      search; when it is absent, (j, i) is an entry that only the transpose
//      contributes ("reverse entry"): the entry is flagged and row j's count
//      incremented;
//   3. an exclusive scan of the counts gives each row's reverse segment and
//      rowptr_i = i k + (reverse entries of rows before i);
//   4. the flagged entries are dropped into their rows' segments (slot order
//      arbitrary) as keys i << 32 | bits of d2;
//   5. each segment is sorted (a wavefront in registers up to 256 entries;
//      longer segments, which only hubs of the k-NN graph have, by a
//      workgroup in global memory), so it no longer depends on the slots;
//   6. every entry's place in its merged row is its rank in its own sorted
//      list plus the number of entries of the other list with a smaller
//      column (a binary search); the two lists are disjoint, so the places
//      are distinct.
// No step needs the number of reverse entries on the host, so the whole
// construction can be enqueued without a round trip.
#include "kvb_device.h"
#include "kvb_kernels.h"

#include <rocprim/device/device_scan.hpp>

namespace kvb {

constexpr int SEG_SHORT = 4 * WAVE;   // reverse segments sorted in registers

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

// the same over keys whose high word is the column
__device__ __forceinline__ int64_t count_less_key(const uint64_t* __restrict__ a, int64_t len, int32_t v)
{
    int64_t lo = 0, hi = len;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (static_cast<int32_t>(a[mid] >> 32) < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// 1b. a bucket index of each sorted row: the column range [0, n) is cut into
// UB equal buckets; boff[j][b] (b = 1..UB-1, slot 0 unused) holds the number
// of row j's columns below bucket b, so a column's candidates in row j lie
// between two neighbouring entries of the index (about k / UB of them)
constexpr int UB = 32;

__device__ __forceinline__ int bucket_of(int v, int n) { return static_cast<int>((static_cast<int64_t>(v) * UB) / n); }

__global__ __launch_bounds__(256) void k_union_buckets(const int32_t* __restrict__ scol, int n, int k,
                                                       uint16_t* __restrict__ boff)
{
    const int lane = lane_id();
    const int j = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (j >= n || lane >= UB) return;
    // columns v with bucket_of(v) < b are those below ceil(b n / UB)
    const int64_t bound = (static_cast<int64_t>(lane) * n + UB - 1) / UB;
    const int32_t* row = scol + static_cast<size_t>(j) * k;
    int lo = 0, hi = k;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (row[mid] < bound)
            lo = mid + 1;
        else
            hi = mid;
    }
    boff[static_cast<size_t>(j) * UB + lane] = static_cast<uint16_t>(lo);
}

// the entries of sorted row j that can equal v: [first, last)
__device__ __forceinline__ void bucket_range(const uint16_t* __restrict__ boff, int j, int k, int n, int v, int& first,
                                             int& last)
{
    const int b = bucket_of(v, n);
    const uint16_t* o = boff + static_cast<size_t>(j) * UB;
    first = b == 0 ? 0 : o[b];
    last = b == UB - 1 ? k : o[b + 1];
}

// 2. flag[p] = 1 for entries (i, j) whose transpose (j, i) row j does not
// store; cnt[j] counts them. bad becomes non-zero if a row holds a column
// outside [0, n) or the same column twice (such entries are skipped, so no
// access leaves the arrays).
__global__ __launch_bounds__(256) void k_union_count(const int32_t* __restrict__ scol,
                                                     const uint16_t* __restrict__ boff, int n, int k,
                                                     int* __restrict__ cnt, uint8_t* __restrict__ flag,
                                                     unsigned long long* __restrict__ bad)
{
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= static_cast<int64_t>(n) * k) return;
    const int i = static_cast<int>(p / k);
    const int r = static_cast<int>(p - static_cast<int64_t>(i) * k);
    const int j = scol[p];
    uint8_t f = 0;
    if (j < 0 || j >= n || (r > 0 && scol[p - 1] == j)) {
        atomicOr(bad, 1ull);
    } else if (j != i) {
        const int32_t* rj = scol + static_cast<size_t>(j) * k;
        int first, last;
        bucket_range(boff, j, k, n, i, first, last);
        bool found = false;
        for (int t = first; t < last; ++t) found |= rj[t] == i;
        if (!found) {   // row j does not store (j, i) itself
            atomicAdd(cnt + j, 1);
            f = 1;
        }
    }
    flag[p] = f;
}

// 3. rowptr_i = i k + revptr_i (revptr: exclusive scan of the counts, n + 1 entries)
__global__ __launch_bounds__(256) void k_union_rowptr(const int64_t* __restrict__ revptr, int n, int k,
                                                      int64_t* __restrict__ rowptr)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) rowptr[i] = static_cast<int64_t>(i) * k + revptr[i];
}

// 4. the flagged entries into their rows' reverse segments (fill: zeroed counts)
__global__ __launch_bounds__(256) void k_union_fill(const int32_t* __restrict__ scol, const float* __restrict__ sd2,
                                                    const uint8_t* __restrict__ flag, int n, int k,
                                                    const int64_t* __restrict__ revptr, int* __restrict__ fill,
                                                    uint64_t* __restrict__ rkey)
{
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= static_cast<int64_t>(n) * k || !flag[p]) return;
    const int i = static_cast<int>(p / k);
    const int j = scol[p];
    const int64_t slot = revptr[j] + atomicAdd(fill + j, 1);
    rkey[slot] = (static_cast<uint64_t>(static_cast<uint32_t>(i)) << 32) | __float_as_uint(sd2[p]);
}

// a reverse entry's place in row j: its rank t in the sorted segment plus the
// directed entries of row j with a smaller column
__device__ __forceinline__ void place_reverse(uint64_t key, int64_t t, int j, int k, const int32_t* __restrict__ scol,
                                             const int64_t* __restrict__ rowptr, int32_t* __restrict__ col,
                                             float* __restrict__ ud2)
{
    const int32_t c = static_cast<int32_t>(key >> 32);
    const int64_t at = rowptr[j] + t + count_less(scol + static_cast<size_t>(j) * k, k, c);
    col[at] = c;
    ud2[at] = __uint_as_float(static_cast<uint32_t>(key));
}

// 5a + 6. segments of up to 256 entries: one wavefront per row sorts the
// segment in registers, writes it back sorted (the directed entries' places
// need it) and places its entries. Longer segments are listed for 5b.
template <int E>
__device__ __forceinline__ void sort_place_segment(uint64_t* __restrict__ seg, int L, int j, int k,
                                                   const int32_t* __restrict__ scol,
                                                   const int64_t* __restrict__ rowptr, int32_t* __restrict__ col,
                                                   float* __restrict__ ud2)
{
    const int lane = lane_id();
    uint64_t key[E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int t = s * WAVE + lane;
        key[s] = t < L ? seg[t] : ~0ull;
    }
    bitonic_sort<E>(key);
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int t = s * WAVE + lane;
        if (t < L) {
            seg[t] = key[s];
            place_reverse(key[s], t, j, k, scol, rowptr, col, ud2);
        }
    }
}

__global__ __launch_bounds__(256) void k_union_segments(uint64_t* __restrict__ rkey, int n, int k,
                                                        const int64_t* __restrict__ revptr,
                                                        const int32_t* __restrict__ scol,
                                                        const int64_t* __restrict__ rowptr, int32_t* __restrict__ col,
                                                        float* __restrict__ ud2, int* __restrict__ long_count,
                                                        int* __restrict__ long_rows)
{
    const int j = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (j >= n) return;
    const int64_t b = revptr[j];
    const int64_t L = revptr[j + 1] - b;
    if (L == 0) return;
    if (L <= WAVE)
        sort_place_segment<1>(rkey + b, static_cast<int>(L), j, k, scol, rowptr, col, ud2);
    else if (L <= SEG_SHORT)
        sort_place_segment<4>(rkey + b, static_cast<int>(L), j, k, scol, rowptr, col, ud2);
    else if (lane_id() == 0)
        long_rows[atomicAdd(long_count, 1)] = j;
}

// 5b + 6. a workgroup per listed row sorts its segment in global memory with
// a bitonic network in which every comparator puts the smaller key first
// (each merge stage starts by comparing mirrored positions), so positions at
// or past L act as +inf and need not exist; then it places the entries.
// The barriers order the workgroup's global accesses (one compute unit).
__global__ __launch_bounds__(256) void k_union_long_segments(uint64_t* __restrict__ rkey,
                                                             const int64_t* __restrict__ revptr, int k,
                                                             const int32_t* __restrict__ scol,
                                                             const int64_t* __restrict__ rowptr,
                                                             int32_t* __restrict__ col, float* __restrict__ ud2,
                                                             const int* __restrict__ long_count,
                                                             const int* __restrict__ long_rows)
{
    const int count = *long_count;
    for (int q = blockIdx.x; q < count; q += gridDim.x) {
        const int j = long_rows[q];
        const int64_t b = revptr[j];
        const int64_t L = revptr[j + 1] - b;
        uint64_t* seg = rkey + b;
        int64_t P = 1;
        while (P < L) P <<= 1;
        for (int64_t kb = 2; kb <= P; kb <<= 1) {
            for (int64_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
                const int64_t h = kb >> 1, blk = t / h, off = t - blk * h;
                const int64_t a = blk * kb + off, c = blk * kb + kb - 1 - off;
                if (c < L) {
                    const uint64_t x = seg[a], y = seg[c];
                    if (x > y) {
                        seg[a] = y;
                        seg[c] = x;
                    }
                }
            }
            __syncthreads();
            for (int64_t jj = kb >> 2; jj > 0; jj >>= 1) {
                for (int64_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
                    const int64_t a = (t / jj) * 2 * jj + (t % jj), c = a + jj;
                    if (c < L) {
                        const uint64_t x = seg[a], y = seg[c];
                        if (x > y) {
                            seg[a] = y;
                            seg[c] = x;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int64_t t = threadIdx.x; t < L; t += blockDim.x) place_reverse(seg[t], t, j, k, scol, rowptr, col, ud2);
        __syncthreads();
    }
}

// 6. a directed entry's place: its rank r in the sorted row plus the reverse
// entries of the row with a smaller column
__global__ __launch_bounds__(256) void k_union_place_direct(const int32_t* __restrict__ scol,
                                                            const float* __restrict__ sd2, int n, int k,
                                                            const int64_t* __restrict__ revptr,
                                                            const uint64_t* __restrict__ rkey,
                                                            const int64_t* __restrict__ rowptr,
                                                            int32_t* __restrict__ col, float* __restrict__ ud2)
{
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= static_cast<int64_t>(n) * k) return;
    const int i = static_cast<int>(p / k);
    const int r = static_cast<int>(p - static_cast<int64_t>(i) * k);
    const int32_t c = scol[p];
    const int64_t rb = revptr[i];
    const int64_t at = rowptr[i] + r + count_less_key(rkey + rb, revptr[i + 1] - rb, c);
    col[at] = c;
    ud2[at] = sd2[p];
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

// ------------------------------------------------------------------ threshold truncation
// Section 4: Algorithm 1 stores an entry only when its kernel value exceeds the
// sparsity tolerance delta. Entry (i, j) is kept when x < L, L = -ln(delta)
// (formed on the host), x = (d2 * (1 / (e rho_i))) / rho_j in float64: the
// exponent form of exp(-x) > delta, free of the rounding of exp. One wavefront
// per row; the fill keeps the row's order (ballot and prefix count).
__device__ __forceinline__ bool trunc_keep(const float* __restrict__ d2, const int32_t* __restrict__ col,
                                           const float* __restrict__ rho, int64_t p, double inv, double L)
{
    const double x = static_cast<double>(d2[p]) * inv / static_cast<double>(rho[col[p]]);
    return x < L;
}

__global__ __launch_bounds__(256) void k_trunc_count(const int64_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ col, const float* __restrict__ d2,
                                                     const float* __restrict__ rho, int n, double e,
                                                     const double* __restrict__ e_dev, double L,
                                                     int* __restrict__ cnt)
{
    if (e_dev) e = *e_dev;
    const int lane = lane_id();
    const int i = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (i >= n) return;
    const double inv = 1.0 / (e * static_cast<double>(rho[i]));
    int c = 0;
    for (int64_t p = rowptr[i] + lane; p < rowptr[i + 1]; p += WAVE) c += trunc_keep(d2, col, rho, p, inv, L);
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (lane == 0) cnt[i] = c;
    if (i == n - 1 && lane == 0) cnt[n] = 0;
}

__global__ __launch_bounds__(256) void k_trunc_fill(const int64_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col, const float* __restrict__ d2,
                                                    const float* __restrict__ rho, int n, double e,
                                                    const double* __restrict__ e_dev, double L,
                                                    const int64_t* __restrict__ rowptr_out,
                                                    int32_t* __restrict__ col_out, float* __restrict__ d2_out)
{
    if (e_dev) e = *e_dev;
    const int lane = lane_id();
    const int i = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (i >= n) return;
    const double inv = 1.0 / (e * static_cast<double>(rho[i]));
    int64_t out = rowptr_out[i];
    const uint64_t below = (1ull << lane) - 1;
    for (int64_t p0 = rowptr[i]; p0 < rowptr[i + 1]; p0 += WAVE) {
        const int64_t p = p0 + lane;
        const bool keep = p < rowptr[i + 1] && trunc_keep(d2, col, rho, p, inv, L);
        const uint64_t m = __ballot(keep);
        if (keep) {
            const int64_t at = out + __popcll(m & below);
            col_out[at] = col[p];
            d2_out[at] = d2[p];
        }
        out += __popcll(m);
    }
}

// ------------------------------------------------------------------ launchers
static unsigned grid_of(int64_t cnt) { return static_cast<unsigned>((cnt + 255) / 256); }

constexpr int LONG_SEGMENT_BLOCKS = 256;

size_t union_scan_bytes(int n)
{
    size_t b = 0;
    (void)rocprim::exclusive_scan(nullptr, b, static_cast<const int*>(nullptr), static_cast<int64_t*>(nullptr),
                                  int64_t(0), static_cast<size_t>(n) + 1, rocprim::plus<int64_t>(), nullptr);
    return b;
}

hipError_t launch_union_count(const int32_t* idx, const float* d2, int n, int k, const UnionWork& w, hipStream_t st)
{
    const dim3 rows((n + 3) / 4), block(256);
    if (k <= 64)
        hipLaunchKernelGGL((k_union_sort_rows<1>), rows, block, 0, st, idx, d2, n, k, w.scol, w.sd2);
    else if (k <= 128)
        hipLaunchKernelGGL((k_union_sort_rows<2>), rows, block, 0, st, idx, d2, n, k, w.scol, w.sd2);
    else
        hipLaunchKernelGGL((k_union_sort_rows<4>), rows, block, 0, st, idx, d2, n, k, w.scol, w.sd2);
    // n + 1 counts: the last stays zero, so the scan's last entry is the total
    hipError_t e = hipMemsetAsync(w.cnt, 0, sizeof(int) * (static_cast<size_t>(n) + 1), st);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(w.bad, 0, sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
    const int64_t nk = static_cast<int64_t>(n) * k;
    hipLaunchKernelGGL(k_union_buckets, rows, block, 0, st, w.scol, n, k, w.boff);
    hipLaunchKernelGGL(k_union_count, dim3(grid_of(nk)), block, 0, st, w.scol, w.boff, n, k, w.cnt, w.flag, w.bad);
    size_t scan_bytes = w.scan_bytes;
    e = rocprim::exclusive_scan(w.scan_tmp, scan_bytes, w.cnt, w.revptr, int64_t(0), static_cast<size_t>(n) + 1,
                                rocprim::plus<int64_t>(), st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_union_place(int n, int k, const UnionWork& w, int64_t* rowptr, int32_t* col, float* ud2,
                              hipStream_t st)
{
    const int64_t nk = static_cast<int64_t>(n) * k;
    hipLaunchKernelGGL(k_union_rowptr, dim3(grid_of(int64_t(n) + 1)), dim3(256), 0, st, w.revptr, n, k, rowptr);
    hipError_t e = hipMemsetAsync(w.cnt, 0, sizeof(int) * (static_cast<size_t>(n) + 1), st);   // fill counts
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(w.long_count, 0, sizeof(int), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_union_fill, dim3(grid_of(nk)), dim3(256), 0, st, w.scol, w.sd2, w.flag, n, k, w.revptr, w.cnt,
                       w.rkey);
    hipLaunchKernelGGL(k_union_segments, dim3((n + 3) / 4), dim3(256), 0, st, w.rkey, n, k, w.revptr, w.scol, rowptr,
                       col, ud2, w.long_count, w.long_rows);
    hipLaunchKernelGGL(k_union_long_segments, dim3(LONG_SEGMENT_BLOCKS), dim3(256), 0, st, w.rkey, w.revptr, k, w.scol,
                       rowptr, col, ud2, w.long_count, w.long_rows);
    hipLaunchKernelGGL(k_union_place_direct, dim3(grid_of(nk)), dim3(256), 0, st, w.scol, w.sd2, n, k, w.revptr,
                       w.rkey, rowptr, col, ud2);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_rows_of_k(int n, int k, int64_t* __restrict__ rowptr)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) rowptr[i] = static_cast<int64_t>(i) * k;
}

hipError_t launch_sorted_rows(const int32_t* idx, const float* d2, int n, int k, int64_t* rowptr, int32_t* col,
                              float* sd2, hipStream_t st)
{
    const dim3 rows((n + 3) / 4), block(256);
    if (k <= 64)
        hipLaunchKernelGGL((k_union_sort_rows<1>), rows, block, 0, st, idx, d2, n, k, col, sd2);
    else if (k <= 128)
        hipLaunchKernelGGL((k_union_sort_rows<2>), rows, block, 0, st, idx, d2, n, k, col, sd2);
    else
        hipLaunchKernelGGL((k_union_sort_rows<4>), rows, block, 0, st, idx, d2, n, k, col, sd2);
    hipLaunchKernelGGL(k_rows_of_k, dim3(grid_of(int64_t(n) + 1)), block, 0, st, n, k, rowptr);
    return hipGetLastError();
}

hipError_t launch_truncate(const int64_t* rowptr, const int32_t* col, const float* d2, const float* rho, int n,
                           double e, const double* e_dev, double L, int* cnt, void* scan_tmp, size_t scan_bytes,
                           int64_t* rowptr_out, int32_t* col_out, float* d2_out, hipStream_t st)
{
    const dim3 rows((n + 3) / 4), block(256);
    hipLaunchKernelGGL(k_trunc_count, rows, block, 0, st, rowptr, col, d2, rho, n, e, e_dev, L, cnt);
    hipError_t err = rocprim::exclusive_scan(scan_tmp, scan_bytes, cnt, rowptr_out, int64_t(0),
                                             static_cast<size_t>(n) + 1, rocprim::plus<int64_t>(), st);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_trunc_fill, rows, block, 0, st, rowptr, col, d2, rho, n, e, e_dev, L, rowptr_out, col_out,
                       d2_out);
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
