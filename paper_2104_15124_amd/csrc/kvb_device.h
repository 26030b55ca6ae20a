// Device-side building blocks shared by the kvb kernels (gfx950, wave64).
//
// Neighbour candidates travel as 64-bit keys: an order-preserving encoding of
// a float32 score in the high word (sign bit flipped for non-negative values,
// all bits flipped for negative ones, so unsigned order equals float order)
// and the column index in the low word. Unsigned key order is therefore the
// (score, index) order of the paper's neighbour ranking I(x, k) (Section 2.1):
// ties between equal scores go to the smaller index. Scores are squared
// distances, or squared distances shifted by a per-row constant.
//
// Per-row candidate lists live in registers, spread over the 64 lanes of a
// wavefront: element t of a list of capacity 64*E sits in slot t / 64 of
// lane t % 64. Sorting and merging use bitonic networks; exchanges between
// lanes go through cross-lane shuffles, exchanges between slots stay in the
// lane.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kvb {

constexpr uint64_t KEY_INF = 0xFF800000FFFFFFFFull;  // score +inf, index 0xffffffff
constexpr int WAVE = 64;

__device__ __forceinline__ uint32_t float_order_bits(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float order_bits_float(uint32_t u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}
__device__ __forceinline__ uint64_t make_key(float d, uint32_t j)
{
    return (static_cast<uint64_t>(float_order_bits(d)) << 32) | j;
}
__device__ __forceinline__ float key_dist(uint64_t k) { return order_bits_float(static_cast<uint32_t>(k >> 32)); }
__device__ __forceinline__ uint32_t key_idx(uint64_t k) { return static_cast<uint32_t>(k); }

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Value of lane (lane ^ j) for j in {1, 2, 4, 8, 16, 32}, without the LDS
// crossbar: DPP quad permutations (j = 1, 2), row shifts (j = 4), a row
// rotation (j = 8), and the gfx950 row-swap permutes (j = 16, 32). Any other
// j falls back to ds_bpermute. Calls with a constant j fold to one path.
__device__ __forceinline__ uint32_t xor_lane(uint32_t v, int j)
{
    const int lane = __lane_id();
    switch (j) {
    case 1: return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);    // quad_perm [1,0,3,2]
    case 2: return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);    // quad_perm [2,3,0,1]
    case 4: {
        const uint32_t up = __builtin_amdgcn_mov_dpp(v, 0x104, 0xF, 0xF, true);   // row_shl:4, lane + 4
        const uint32_t dn = __builtin_amdgcn_mov_dpp(v, 0x114, 0xF, 0xF, true);   // row_shr:4, lane - 4
        return (lane & 4) ? dn : up;
    }
    case 8: return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true);   // row_ror:8
    case 16: {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16) ? r[0] : r[1];
    }
    case 32: {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane & 32) ? r[0] : r[1];
    }
    default: return static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), j, WAVE));
    }
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask)
{
    const uint32_t lo = xor_lane(static_cast<uint32_t>(v), mask);
    const uint32_t hi = xor_lane(static_cast<uint32_t>(v >> 32), mask);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ float shfl_xor_f32(float v, int mask)
{
    return __uint_as_float(xor_lane(__float_as_uint(v), mask));
}

__device__ __forceinline__ double shfl_xor_f64(double v, int mask)
{
    return __longlong_as_double(static_cast<long long>(shfl_xor_u64(static_cast<uint64_t>(__double_as_longlong(v)), mask)));
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src)
{
    int lo = static_cast<int>(static_cast<uint32_t>(v));
    int hi = static_cast<int>(static_cast<uint32_t>(v >> 32));
    lo = __shfl(lo, src, WAVE);
    hi = __shfl(hi, src, WAVE);
    return (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int src)
{
    uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v)), src);
    uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v >> 32)), src);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a < b ? b : a; }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ int mbcnt64(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0));
}

// Order LDS traffic of one wavefront: stores issued before are visible to
// loads of any lane of the same wavefront issued after.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- bitonic networks
// Compare-exchange with partner distance j < 64 (partner in another lane) in a
// bitonic stage of block size kb (ascending where element index & kb == 0).
// The lanes l of a wavefront with bit j of l clear (j a power of two below
// 64), as a lane mask.
__host__ __device__ constexpr uint64_t lanes_bit_clear(int j)
{
    return j == 1    ? 0x5555555555555555ull
           : j == 2  ? 0x3333333333333333ull
           : j == 4  ? 0x0F0F0F0F0F0F0F0Full
           : j == 8  ? 0x00FF00FF00FF00FFull
           : j == 16 ? 0x0000FFFF0000FFFFull
                     : 0x00000000FFFFFFFFull;
}

// The lanes that keep the smaller key of their pair are a constant lane mask
// for each stage and slot (kb, j and s are compile-time constants once the
// networks are unrolled), so each exchange is one 64-bit compare, a scalar
// xor with that mask and two selects.
template <int E, bool DESC = false>
__device__ __forceinline__ void cx_lanes(uint64_t (&v)[E], int kb, int j, int lane)
{
    (void)lane;
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const uint64_t o = shfl_xor_u64(v[s], j);
        // element index i = s * 64 + lane sorts ascending in its block where (i & kb) == 0
        uint64_t up = kb < WAVE ? lanes_bit_clear(kb) : (((s * WAVE) & kb) == 0 ? ~0ull : 0ull);
        if (DESC) up = ~up;
        // in an ascending block the lower lane of a pair keeps the smaller key
        const uint64_t keep_min = ~(up ^ lanes_bit_clear(j));
        // the partner's key is taken where it is the one to keep
        const uint64_t take = __ballot(o < v[s]) ^ ~keep_min;
        v[s] = __builtin_amdgcn_inverse_ballot_w64(take) ? o : v[s];
    }
}

// Compare-exchange with partner distance js*64 (partner in another slot, same lane).
template <int E, bool DESC = false>
__device__ __forceinline__ void cx_slots(uint64_t (&v)[E], int kb, int js, int lane)
{
#pragma unroll
    for (int s = 0; s < E; ++s) {
        int p = s ^ js;
        if (p > s) {
            int i = s * WAVE + lane;
            bool up = ((i & kb) == 0) != DESC;
            uint64_t a = v[s], b = v[p];
            bool sw = up ? (a > b) : (a < b);
            v[s] = sw ? b : a;
            v[p] = sw ? a : b;
        }
    }
}

// Full sort of the 64*E keys held by the wavefront (ascending, or descending
// with DESC).
template <int E, bool DESC = false>
__device__ __forceinline__ void bitonic_sort(uint64_t (&v)[E])
{
    const int lane = lane_id();
#pragma unroll
    for (int kb = 2; kb <= WAVE * E; kb <<= 1) {
#pragma unroll
        for (int j = kb >> 1; j > 0; j >>= 1) {
            // the last stage's direction flag (i & 2N) is 0 for every i, so
            // DESC reverses the whole order
            if (j >= WAVE)
                cx_slots<E, DESC>(v, kb, j / WAVE, lane);
            else
                cx_lanes<E, DESC>(v, kb, j, lane);
        }
    }
}

// Ascending sort of a bitonic sequence of 64*E keys.
template <int E>
__device__ __forceinline__ void bitonic_merge_asc(uint64_t (&v)[E])
{
    const int lane = lane_id();
    constexpr int N = WAVE * E;
#pragma unroll
    for (int j = N >> 1; j > 0; j >>= 1) {
        if (j >= WAVE)
            cx_slots<E>(v, 2 * N, j / WAVE, lane);
        else
            cx_lanes<E>(v, 2 * N, j, lane);
    }
}

// Keep the 64*E smallest of (sorted list L) u (64 unsorted keys b, one per
// lane), sorted ascending in L. The half-cleaner min(L[t], rev(B)[t]) of a
// sorted and a reverse-sorted sequence holds the smallest half as a bitonic
// sequence; only the last slot of L meets real keys of B.
template <int E>
__device__ __forceinline__ void merge_into_list(uint64_t (&L)[E], uint64_t b)
{
    uint64_t B[1] = {b};
    bitonic_sort<1, true>(B);            // descending: B[lane] is the reversed ascending order
    L[E - 1] = umin64(L[E - 1], B[0]);
    bitonic_merge_asc<E>(L);
}

// Key at list position t (wave-uniform t), broadcast to the wavefront.
template <int E>
__device__ __forceinline__ uint64_t list_at(const uint64_t (&L)[E], int t)
{
    const int slot = t / WAVE, src = t % WAVE;
    uint64_t v = L[0];
#pragma unroll
    for (int s = 1; s < E; ++s)
        if (s == slot) v = L[s];
    return readlane_u64(v, src);
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += shfl_xor_f64(v, o);
    return v;
}

__device__ __forceinline__ float wave_max_f32(float v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v = fmaxf(v, shfl_xor_f32(v, o));
    return v;
}

// Neumaier-compensated accumulation (sum, compensation).
struct Comp64 {
    double s = 0.0, c = 0.0;
    __device__ __forceinline__ void add(double x)
    {
        double t = s + x;
        c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
    }
    __device__ __forceinline__ double value() const { return s + c; }
};

}  // namespace kvb
