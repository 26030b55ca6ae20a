// Device work of the learned partitioner outside the MLP: the teacher
// partition (balanced median splits along seeded random directions), batch
// assembly for training, and the bucket layout of the routed search (member
// order, candidate tile offsets, per-probe query groups and work lists).
// Sorting uses rocPRIM's stable device radix sort.
#include <rocprim/device/device_radix_sort.hpp>

#include "kvb_device.h"
#include "kvb_kernels.h"

namespace kvb {

// Component c of the random direction of tree node `node` at `level`: a
// uniform value in [-1, 1) with 24 random bits, from SplitMix64 (Steele, Lea
// and Flood 2014, with Vigna's published constants) evaluated at the counter
// (level << 40) | (node << 20) | c. Exactly representable in float32.
__device__ __forceinline__ double teacher_dir(uint64_t seed, int level, int node, int c)
{
    const uint64_t ctr = (static_cast<uint64_t>(level) << 40) | (static_cast<uint64_t>(node) << 20) |
                         static_cast<uint64_t>(c);
    uint64_t z = seed + (ctr + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return static_cast<double>(z >> 40) * (1.0 / 8388608.0) - 1.0;
}

// key = node << 32 | order bits of float32(projection), value = sample index.
// The projection is accumulated in float64, in column order, one rounding
// per product and per sum (no fused multiply-add), so it is reproducible
// exactly by any IEEE float64 evaluation of the same sum.
__global__ __launch_bounds__(256) void k_teacher_keys(const float* __restrict__ X, int ns, int m,
                                                      const int32_t* __restrict__ node, int level, uint64_t seed,
                                                      uint64_t* __restrict__ keys, int32_t* __restrict__ vals)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    const int v = node ? node[i] : 0;
    const float* x = X + static_cast<size_t>(i) * m;
    double p = 0.0;
    for (int c = 0; c < m; ++c) {
        const double t = static_cast<double>(x[c]) * teacher_dir(seed, level, v, c);
        p = p + t;
    }
    keys[i] = (static_cast<uint64_t>(v) << 32) | float_order_bits(static_cast<float>(p));
    vals[i] = i;
}

// start[v] = first sorted position of node v (nodes are never empty here:
// every node holds at least floor(ns / 2^level) >= 1 samples), start[nodes] = ns.
__global__ __launch_bounds__(256) void k_node_starts(const uint64_t* __restrict__ skeys, int ns, int nodes,
                                                     int32_t* __restrict__ start)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ns) return;
    const uint32_t v = static_cast<uint32_t>(skeys[p] >> 32);
    if (p == 0 || static_cast<uint32_t>(skeys[p - 1] >> 32) != v) start[v] = p;
    if (p == 0) start[nodes] = ns;
}

// The lower floor(size / 2) of each node (by projection, then index) go to
// child 2v, the rest to child 2v + 1.
__global__ __launch_bounds__(256) void k_teacher_split(const uint64_t* __restrict__ skeys,
                                                       const int32_t* __restrict__ svals, int ns,
                                                       const int32_t* __restrict__ start,
                                                       int32_t* __restrict__ node_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ns) return;
    const int v = static_cast<int>(skeys[p] >> 32);
    const int s0 = start[v], size = start[v + 1] - s0;
    node_out[svals[p]] = 2 * v + ((p - s0) >= size / 2 ? 1 : 0);
}

// Batch t of an epoch: rows perm(t0 + r) = (a (t0 + r) + c) mod ns, r < B, and
// the bucket labels of each row's ks neighbours.
__global__ __launch_bounds__(256) void k_batch_gather(int64_t ns, uint64_t a, uint64_t c, int64_t t0, int B,
                                                      const int32_t* __restrict__ idx_s, int ks,
                                                      const int32_t* __restrict__ labels,
                                                      int32_t* __restrict__ bidx, int32_t* __restrict__ nbrlab)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(B) * ks) return;
    const int r = static_cast<int>(t / ks), j = static_cast<int>(t % ks);
    const uint64_t pos = static_cast<uint64_t>(t0 + r);
    const int64_t row = static_cast<int64_t>((static_cast<unsigned __int128>(a) * pos + c) % static_cast<uint64_t>(ns));
    if (j == 0) bidx[r] = static_cast<int32_t>(row);
    nbrlab[t] = labels[idx_s[row * ks + j]];
}

// keys[i] = home[i] << 32 | i
__global__ __launch_bounds__(256) void k_member_keys(const int32_t* __restrict__ home, int n,
                                                     uint64_t* __restrict__ keys)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) keys[i] = (static_cast<uint64_t>(home[i]) << 32) | static_cast<uint32_t>(i);
}

// keys[s n + i] = s << 44 | probe[i, s] << 32 | i
__global__ __launch_bounds__(256) void k_query_keys(const int32_t* __restrict__ probe, int n, int P,
                                                    uint64_t* __restrict__ keys)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(n) * P) return;
    const int i = static_cast<int>(t / P), s = static_cast<int>(t % P);
    keys[static_cast<int64_t>(s) * n + i] = (static_cast<uint64_t>(s) << 44) |
                                            (static_cast<uint64_t>(probe[t]) << 32) | static_cast<uint32_t>(i);
}

__device__ __forceinline__ int lower_bound_u64(const uint64_t* a, int lo, int hi, uint64_t v)
{
    while (lo < hi) {
        const int mid = lo + (hi - lo) / 2;
        if (a[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Exclusive scan of per-thread totals of a 1024-thread block (Hillis-Steele).
__device__ int block_exclusive_scan(int v, int* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int add = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    const int incl = sh[t];
    __syncthreads();
    return incl - v;
}

// Member layout (one 1024-thread block): mstart[b] = first sorted member of
// bucket b; tptr = exclusive scan of ceil(count / 32) over buckets, tptr[nb] = total.
__global__ __launch_bounds__(1024) void k_bucket_layout(const uint64_t* __restrict__ skeys, int n, int nb,
                                                        int32_t* __restrict__ mstart, int32_t* __restrict__ tptr)
{
    __shared__ int sh[1024];
    const int per = (nb + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    int tiles[4] = {0, 0, 0, 0};   // nb <= 4096
    int tot = 0;
    for (int u = 0; u < per; ++u) {
        const int b = b0 + u;
        if (b < nb) {
            const int lo = lower_bound_u64(skeys, 0, n, static_cast<uint64_t>(b) << 32);
            const int hi = lower_bound_u64(skeys, lo, n, static_cast<uint64_t>(b + 1) << 32);
            mstart[b] = lo;
            tiles[u] = (hi - lo + 31) / 32;
            tot += tiles[u];
        }
    }
    int off = block_exclusive_scan(tot, sh);
    for (int u = 0; u < per; ++u) {
        const int b = b0 + u;
        if (b < nb) {
            tptr[b] = off;
            off += tiles[u];
        }
    }
    if (threadIdx.x == 1023) tptr[nb] = off;
}

// Candidate operand rows: member at sorted position p of bucket b sits at
// row 32 tptr[b] + (p - mstart[b]); cid maps rows back to samples (rows of
// padding keep -1), brow maps samples to rows.
__global__ __launch_bounds__(256) void k_member_rows(const uint64_t* __restrict__ skeys, int n,
                                                     const int32_t* __restrict__ mstart,
                                                     const int32_t* __restrict__ tptr, int32_t* __restrict__ cid,
                                                     int32_t* __restrict__ brow)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int b = static_cast<int>(skeys[p] >> 32);
    const int i = static_cast<int>(static_cast<uint32_t>(skeys[p]));
    const int row = 32 * tptr[b] + (p - mstart[b]);
    cid[row] = i;
    brow[i] = row;
}

// Query groups and work items of probe slot s (one 1024-thread block per
// slot): qptr[s][b] = first entry of bucket b among the slot's sorted query
// keys (absolute entry index), qids = sample ids of all entries, and work
// items (b, t0) for chunks of qpb queries.
__global__ __launch_bounds__(1024) void k_work_layout(const uint64_t* __restrict__ qkeys, int n, int nb, int qpb,
                                                      int max_work, int32_t* __restrict__ qptr,
                                                      int2* __restrict__ work, int32_t* __restrict__ n_work)
{
    __shared__ int sh[1024];
    const int s = blockIdx.x;
    const int lo0 = s * n, hi0 = (s + 1) * n;
    int32_t* qp = qptr + static_cast<size_t>(s) * (nb + 1);
    int2* wk = work + static_cast<size_t>(s) * max_work;
    const int per = (nb + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    int starts[4] = {0, 0, 0, 0}, chunks[4] = {0, 0, 0, 0};
    int tot = 0;
    for (int u = 0; u < per; ++u) {
        const int b = b0 + u;
        if (b < nb) {
            const uint64_t base = static_cast<uint64_t>(s) << 44;
            const int lo = lower_bound_u64(qkeys, lo0, hi0, base | (static_cast<uint64_t>(b) << 32));
            const int hi = lower_bound_u64(qkeys, lo, hi0, base | (static_cast<uint64_t>(b + 1) << 32));
            starts[u] = lo;
            qp[b] = lo;
            chunks[u] = (hi - lo + qpb - 1) / qpb;
            tot += chunks[u];
        }
    }
    int off = block_exclusive_scan(tot, sh);
    for (int u = 0; u < per; ++u) {
        const int b = b0 + u;
        if (b < nb)
            for (int c = 0; c < chunks[u]; ++c) {
                if (off < max_work) wk[off] = make_int2(b, starts[u] + c * qpb);
                ++off;
            }
    }
    if (threadIdx.x == 1023) {
        qp[nb] = hi0;
        n_work[s] = off < max_work ? off : max_work;
    }
}

__global__ __launch_bounds__(256) void k_low_words(const uint64_t* __restrict__ keys, int64_t cnt,
                                                   int32_t* __restrict__ out)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < cnt) out[t] = static_cast<int32_t>(static_cast<uint32_t>(keys[t]));
}

__global__ __launch_bounds__(256) void k_fill_i32(int32_t* __restrict__ p, int64_t cnt, int32_t v)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < cnt) p[t] = v;
}

// ------------------------------------------------------------------ launchers
static unsigned blocks_for(int64_t cnt, int per = 256) { return static_cast<unsigned>((cnt + per - 1) / per); }

hipError_t sort_pairs_u64(void* tmp, size_t& tmp_bytes, const uint64_t* kin, uint64_t* kout, const int32_t* vin,
                          int32_t* vout, int cnt, int end_bit, hipStream_t st)
{
    return rocprim::radix_sort_pairs(tmp, tmp_bytes, kin, kout, vin, vout, static_cast<size_t>(cnt), 0,
                                     static_cast<unsigned>(end_bit), st);
}

hipError_t sort_pairs_u32(void* tmp, size_t& tmp_bytes, const uint32_t* kin, uint32_t* kout, const int32_t* vin,
                          int32_t* vout, int cnt, int end_bit, hipStream_t st)
{
    return rocprim::radix_sort_pairs(tmp, tmp_bytes, kin, kout, vin, vout, static_cast<size_t>(cnt), 0,
                                     static_cast<unsigned>(end_bit), st);
}

hipError_t sort_keys_u64(void* tmp, size_t& tmp_bytes, const uint64_t* kin, uint64_t* kout, int64_t cnt,
                         int end_bit, hipStream_t st)
{
    return rocprim::radix_sort_keys(tmp, tmp_bytes, kin, kout, static_cast<size_t>(cnt), 0,
                                    static_cast<unsigned>(end_bit), st);
}

hipError_t launch_teacher_keys(const float* X, int ns, int m, const int32_t* node, int level, uint64_t seed,
                               uint64_t* keys, int32_t* vals, hipStream_t st)
{
    hipLaunchKernelGGL(k_teacher_keys, dim3(blocks_for(ns)), dim3(256), 0, st, X, ns, m, node, level, seed, keys,
                       vals);
    return hipGetLastError();
}

hipError_t launch_teacher_split(const uint64_t* skeys, const int32_t* svals, int ns, int nodes, int32_t* start,
                                int32_t* node_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_node_starts, dim3(blocks_for(ns)), dim3(256), 0, st, skeys, ns, nodes, start);
    hipLaunchKernelGGL(k_teacher_split, dim3(blocks_for(ns)), dim3(256), 0, st, skeys, svals, ns, start, node_out);
    return hipGetLastError();
}

hipError_t launch_batch_gather(int64_t ns, uint64_t a, uint64_t c, int64_t t0, int B, const int32_t* idx_s, int ks,
                               const int32_t* labels, int32_t* bidx, int32_t* nbrlab, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_gather, dim3(blocks_for(static_cast<int64_t>(B) * ks)), dim3(256), 0, st, ns, a, c,
                       t0, B, idx_s, ks, labels, bidx, nbrlab);
    return hipGetLastError();
}

hipError_t launch_member_keys(const int32_t* home, int n, uint64_t* keys, hipStream_t st)
{
    hipLaunchKernelGGL(k_member_keys, dim3(blocks_for(n)), dim3(256), 0, st, home, n, keys);
    return hipGetLastError();
}

hipError_t launch_query_keys(const int32_t* probe, int n, int P, uint64_t* keys, hipStream_t st)
{
    hipLaunchKernelGGL(k_query_keys, dim3(blocks_for(static_cast<int64_t>(n) * P)), dim3(256), 0, st, probe, n, P,
                       keys);
    return hipGetLastError();
}

hipError_t launch_bucket_layout(const uint64_t* skeys, int n, int nb, int32_t* mstart, int32_t* tptr,
                                int32_t* cid, int64_t cid_rows, int32_t* brow, hipStream_t st)
{
    if (nb < 1 || nb > 4096) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bucket_layout, dim3(1), dim3(1024), 0, st, skeys, n, nb, mstart, tptr);
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(cid_rows)), dim3(256), 0, st, cid, cid_rows, -1);
    hipLaunchKernelGGL(k_member_rows, dim3(blocks_for(n)), dim3(256), 0, st, skeys, n, mstart, tptr, cid, brow);
    return hipGetLastError();
}

hipError_t launch_work_layout(const uint64_t* qkeys, int n, int nb, int P, int qpb, int max_work, int32_t* qptr,
                              int2* work, int32_t* n_work, int32_t* qids, hipStream_t st)
{
    if (nb < 1 || nb > 4096) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_work_layout, dim3(P), dim3(1024), 0, st, qkeys, n, nb, qpb, max_work, qptr, work, n_work);
    hipLaunchKernelGGL(k_low_words, dim3(blocks_for(static_cast<int64_t>(n) * P)), dim3(256), 0, st, qkeys,
                       static_cast<int64_t>(n) * P, qids);
    return hipGetLastError();
}

}  // namespace kvb
