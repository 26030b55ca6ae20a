// Pieces shared by the matrix-core selection kernels (knn_mfma.hip: the
// all-tiles and learned-bucket scans; knn_tree.hip: the curve-ordered scan
// over the tile-box tree): MFMA operand traits, the accumulator layout, the
// per-query list merge and sort in global scratch, the projected-box distance
// bound and the XCD-aware workgroup order.
#pragma once

#include "kvb_device.h"
#include "kvb_kernels.h"

namespace kvb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct TraitsBF16 {
    using elem = uint16_t;
    using frag = bf16x8;
    static constexpr int KSTEP = 16;   // K per MFMA
    static constexpr int VEC = 8;      // K elements per lane per MFMA
    __device__ static __forceinline__ f32x16 mma(frag a, frag b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ frag load(const elem* p) { return *reinterpret_cast<const frag*>(p); }
};

struct TraitsF32 {
    using elem = float;
    using frag = float;
    static constexpr int KSTEP = 2;
    static constexpr int VEC = 1;
    __device__ static __forceinline__ f32x16 mma(frag a, frag b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ frag load(const elem* p) { return *p; }
};

// Output row (query) of accumulator register r in lane half h of a 32x32 tile.
__host__ __device__ constexpr int acc_row(int r, int h) { return 8 * (r / 4) + 4 * h + (r % 4); }

// Merge query q's LDS buffer into its sorted list in global scratch and return
// the list's kp-th score (the query's new threshold). Whole wavefront.
template <int E>
__device__ __noinline__ float merge_query_list(uint64_t* __restrict__ dst, const uint64_t* buf, int cnt, int kp)
{
    const int lane = lane_id();
    const uint64_t b = lane < cnt ? buf[lane] : KEY_INF;
    uint64_t L[E];
#pragma unroll
    for (int s = 0; s < E; ++s) L[s] = dst[s * WAVE + lane];
    merge_into_list<E>(L, b);
#pragma unroll
    for (int s = 0; s < E; ++s) dst[s * WAVE + lane] = L[s];
    return key_dist(list_at<E>(L, kp - 1));
}

// The same for a buffer of at most 32 keys: they are placed in the upper half
// of the wavefront and sorted there in descending order by the first five
// passes of the bitonic network (15 stages instead of 21), which is already
// the reversed ascending order of the 64-key buffer padded with KEY_INF.
template <int E>
__device__ __noinline__ float merge_query_list32(uint64_t* __restrict__ dst, const uint64_t* buf, int cnt, int kp)
{
    const int lane = lane_id();
    uint64_t B[1] = {lane >= 32 && lane - 32 < cnt ? buf[lane - 32] : KEY_INF};
    uint64_t L[E];
#pragma unroll
    for (int s = 0; s < E; ++s) L[s] = dst[s * WAVE + lane];
#pragma unroll
    for (int kb = 2; kb <= 32; kb <<= 1) {
#pragma unroll
        for (int j = kb >> 1; j > 0; j >>= 1) cx_lanes<1>(B, kb, j, lane);
    }
    L[E - 1] = umin64(L[E - 1], B[0]);
    bitonic_merge_asc<E>(L);
#pragma unroll
    for (int s = 0; s < E; ++s) dst[s * WAVE + lane] = L[s];
    return key_dist(list_at<E>(L, kp - 1));
}

// Lower bound on the squared distance between any query of a workgroup (box
// qlo..qhi of its projected coordinates) and any sample in the projected box
// b ([lower corner, upper corner]), from the box gaps g_c. The computed
// projections differ from the exact P^T y by at most zerr per coordinate,
// |v| >= pscale |P^T v| for every v (the float32 basis is orthonormal only up
// to rounding; pscale is computed from its Gram matrix), and |y_i - y_j|
// exceeds |x_i - x_j| by at most yerr; every float32 step below is taken
// towards a smaller bound.
struct BoxBound {
    float zerr, pscale, yerr;
};

__device__ __forceinline__ float box_bound(const float* __restrict__ b, const float* __restrict__ qlo,
                                           const float* __restrict__ qhi, const BoxBound& bb)
{
    float g2 = 0.f;
#pragma unroll
    for (int c = 0; c < PR_DIMS; ++c) {
        const float g = fmaxf(fmaxf(b[c] - qhi[c], qlo[c] - b[PR_DIMS + c]), 0.f);
        const float gg = fmaxf(g * (1.f - 2.4e-7f) - 2.f * bb.zerr, 0.f);
        g2 = fmaf(gg, gg, g2);
    }
    const float d = sqrtf(g2 * (1.f - 2e-6f)) * bb.pscale - bb.yerr;
    return d > 0.f ? d * d * (1.f - 2e-6f) : 0.f;
}

// Workgroups are dispatched to the 8 XCDs round robin (workgroup b to XCD
// b mod 8). Renumbering them so that each XCD receives one contiguous range of
// curve positions makes the workgroups resident on an XCD at one time
// neighbours along the curve, whose scans read the same candidate tiles
// through that XCD's L2.
__device__ __forceinline__ int xcd_block()
{
    constexpr int XCDS = 8;
    const int b = blockIdx.x, g = gridDim.x;
    const int x = b % XCDS, per = g / XCDS, rem = g % XCDS;
    return x * per + min(x, rem) + b / XCDS;
}

// Sort query q's list in place (whole wavefront) and return its kp-th score.
template <int E>
__device__ __noinline__ float sort_query_list(uint64_t* __restrict__ dst, int kp)
{
    const int lane = lane_id();
    uint64_t L[E];
#pragma unroll
    for (int s = 0; s < E; ++s) L[s] = dst[s * WAVE + lane];
    bitonic_sort<E>(L);
#pragma unroll
    for (int s = 0; s < E; ++s) dst[s * WAVE + lane] = L[s];
    return key_dist(list_at<E>(L, kp - 1));
}

}  // namespace kvb
