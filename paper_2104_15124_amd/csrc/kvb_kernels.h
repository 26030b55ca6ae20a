// Host-side launchers of the kvb kernels (internal to libkvb.so).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kvb.h"

namespace kvb {

// Error model of the MFMA selection scores (see knn_mfma.hip).
struct ErrModel {
    double gamma;   // accumulation bound (K + 4) 2^-24
    double norm;    // relative error of the folded |y_j|^2
    double cross;   // relative bound of the cross term |2 y_i.y_j - computed|
    double center;  // relative rounding of the centred coordinates
};

// Work description of the bucketed (learned-partitioner) selection; see
// k_select_mfma in knn_mfma.hip.
struct BucketArgs {
    const int2* work;    // (bucket, first query entry) per workgroup
    const int* n_work;   // number of valid work items
    const int* qids;     // query sample ids grouped by bucket
    const int* qptr;     // [nb + 1] query entry offsets per bucket
    const int* tptr;     // [nb + 1] candidate tile offsets per bucket
    const int* cid;      // [32 * tiles] sample id of each candidate operand row, -1 for padding
    int first;           // 1: create the query lists, 0: merge into them
};

// Projected dimensions of the curve order (MODE 2 of the matrix-core select):
// boxes use PR_DIMS principal coordinates, the Morton code the first
// PCODE_DIMS of them; superblocks group SB_TILES_MFMA tiles of 32 samples.
constexpr int PR_DIMS = 8;
constexpr int PCODE_DIMS = 4;
constexpr int SB_TILES_MFMA = 16;

// Box tree over the curve-ordered tiles: level 0 holds the tiles' boxes,
// node v of level l >= 1 the box of nodes 64 v .. 64 v + 63 of level l - 1;
// the top level has at most 64 nodes.
constexpr int TREE_FAN = 64;
constexpr int TREE_LEVELS = 6;   // 64^5 tiles of 32 cover every n < 2^31
struct TreeLayout {
    int top;                     // top level (0: the tiles themselves)
    int cnt[TREE_LEVELS];        // nodes per level
    int off[TREE_LEVELS];        // level l >= 1 starts at node off[l] of the node array
    int nodes;                   // nodes of levels >= 1
};
TreeLayout tree_layout(int ntiles);

struct CurveArgs {
    const int* perm;    // [tiles * 32] sample id at each curve position, -1 for padding
    const float* zs;    // [n, PR_DIMS] projected coordinates in curve order
    const float* tbox;  // [tiles, 2, PR_DIMS] boxes of 32-sample tiles
    const float* sbox;  // [superblocks, 2, PR_DIMS] (workgroup scans of knn_mfma.hip)
    const float* tree;  // [layout.nodes, 2, PR_DIMS] boxes of the tree levels >= 1
    TreeLayout layout;
    const float* pscale;// |v| >= *pscale |P^T v| for every v (set with the basis)
    float zcoef;        // computed projected coordinates are within zcoef R of P^T y (R = max |y|)
    float ycoef;        // |y_i - y_j| exceeds |x_i - x_j| by at most ycoef R
};

struct TuneResult {
    double chi[256];
    double e_star;
    double dim;
    int g_star;
    int pad;
};

// k-NN
// direct path (m <= 8): spatial order (Morton codes -> sort -> rows, tile and superblock boxes), then the scan
int spatial_bbox_blocks(int n);
int spatial_tiles(int n);
int spatial_superblocks(int n);
int spatial_code_bits(int n, int m);   // the code has m * spatial_code_bits(n, m) bits
hipError_t launch_spatial_codes(const float* X, int n, int m, float* bbox_part, uint32_t* code, int32_t* vals,
                                hipStream_t st);
hipError_t launch_spatial_layout(const float* X, int n, int m, const int32_t* perm, float* Xs, float* tbox,
                                 float* sbox, hipStream_t st);
// lists [n, kp] and bounds [n] stored by curve position; keys hold curve positions
hipError_t launch_select_direct(const float* Xs, const float* tbox, const float* sbox, int n, int m, int kp,
                                uint64_t* keys, float* slast, unsigned long long* pairs, hipStream_t st);
hipError_t launch_refine(const float* X, int n, int m, int k, int kp, int kstride, const uint64_t* keys,
                         const float* slast, float lb_scale, int32_t* idx, float* d2, int32_t* flags,
                         int* fb_count, int* fb_list, float* fb_bound, int force_period, const float* Xs,
                         const int32_t* perm, hipStream_t st);

// Buffers of the exact fallback's bounded pass (k_fb_collect): rows_cap =
// fallback_rows_cap(n) listed rows with FB_CAP entries each.
constexpr int FB_CAP = 1024;
constexpr int FB_MAX_ROWS = 2048;
struct FallbackWork {
    const float* bound;  // [n] per listed row: bound on its true (k-1)-th distance (+inf: none)
    int* cnt;            // [rows_cap]
    double* bd;          // [rows_cap * FB_CAP] distances
    int* bj;             // [rows_cap * FB_CAP] sample ids
};
int fallback_rows_cap(int n);
// Xs[p] = X[perm[p]] (rows of m floats, p < n)
hipError_t launch_gather_rows(const float* X, int n, int m, const int32_t* perm, float* Xs, hipStream_t st);
hipError_t launch_fallback(const float* X, int n, int m, int k, const int* fb_count, const int* fb_list,
                           const FallbackWork& fw, int32_t* idx, float* d2, hipStream_t st);
hipError_t launch_exact_rows(const float* X, int n, int m, int k, const int* rows, int nrows, int32_t* idx, float* d2,
                             hipStream_t st);

hipError_t launch_prep(const float* X, int n, int m, int split, int kpad, double* colpart, int colblocks,
                       double* mu, void* Aq, void* Bc, float* ynorm2, unsigned* rmax_bits, const int* brow,
                       const int* arow, hipStream_t st);
hipError_t launch_colmean(const float* X, int n, int m, double* colpart, int colblocks, double* mu, hipStream_t st);
hipError_t launch_prep_rows(const float* X, int n, int m, const double* mu, int split, int kpad, void* Aq, void* Bc,
                            float* ynorm2, unsigned* rmax_bits, const int* brow, const int* arow, hipStream_t st);
// the operands in curve order: operand row p from Xs[p], the curve-ordered copy
// of the samples (Xs[p] = X[cid[p]], written by launch_gather_rows), read in order
hipError_t launch_prep_rows_curve(const float* Xs, int n, int m, const double* mu, int split, int kpad, void* Aq,
                                  void* Bc, float* ynorm2, unsigned* rmax_bits, hipStream_t st);
int mfma_kstep(int split);
int mfma_pick_ksteps(int split, int needed);
// ba == nullptr: exact all-pairs selection over n rows; otherwise the bucketed
// selection with max_work workgroups (the kernel skips those beyond *ba->n_work).
hipError_t launch_select_mfma(int split, const void* Aq, const void* Bc, int n, int kpad, int kp, const float* ynorm2,
                              const unsigned* rmax, ErrModel em, uint64_t* lists, int cap, float* lb,
                              const BucketArgs* ba, int max_work, const CurveArgs* crv, unsigned long long* pairs,
                              hipStream_t st);
// curve order of the samples for MODE 2 (spatial_mfma.hip)
int cov_partials();
int cov_chunks(int m);
int project_blocks(int n);
size_t curve_sort_bytes(int n);
// P [m * PR_DIMS + 1]: the basis, then the scale factor of CurveArgs::pscale
hipError_t launch_principal_basis(const float* X, int n, int m, const double* mu, double* part, double* C, float* P,
                                  hipStream_t st);
// zpart [(project_blocks(n) + 1) * 2 * PCODE_DIMS]: block partials, then the reduced range
// tbox [tiles, 2, PR_DIMS]; sbox [superblocks, 2, PR_DIMS]; tree [tree_layout(tiles).nodes, 2, PR_DIMS]
// (the box tree's levels >= 1). median_splits: each group of 4096 consecutive tiles of the curve is then
// halved at its median along the widest side of its box, recursively down to single tiles.
hipError_t launch_curve_order(const float* X, int n, int m, const double* mu, const float* P, float* z, float* zpart,
                              uint32_t* code, uint32_t* scode, int32_t* vals, int32_t* perm, void* sort_tmp,
                              size_t sort_bytes, int32_t* pos, int32_t* cid, float* zs, float* tbox, float* sbox,
                              float* tree, bool median_splits, hipStream_t st);
// curve-ordered exact selection over the box tree (knn_tree.hip); lists [n, cap], lb [n] by curve position.
// select_tree_fits: whether the tree walk suits the contraction length (else the
// workgroup scan of launch_select_mfma with crv runs)
bool select_tree_fits(int split, int kpad);
hipError_t launch_select_tree(int split, const void* Aq, const void* Bc, int n, int kpad, int kp, const float* ynorm2,
                              const unsigned* rmax, ErrModel em, uint64_t* lists, int cap, float* lb,
                              const CurveArgs& crv, unsigned long long* pairs, hipStream_t st);
int select_mfma_queries_per_block(int split, int kpad);

// passes
hipError_t launch_adhoc_bandwidth(const float* d2, int n, int k, int k0, float* b, hipStream_t st);
hipError_t launch_density(const int32_t* idx, const float* d2, int n, int k, const float* b, double e,
                          const double* e_dev, double d, double beta, float* rho, float* psi, hipStream_t st);
int chi_num_blocks(int64_t nnz);
// grid e_g = exp(ln(e_min s) + g (ln(e_max s) - ln(e_min s)) / (G - 1)), s = *scale_dev or 1
hipError_t launch_chi(const int32_t* idx, const float* d2, const float* rho, int64_t nnz, int k, int G, double e_min,
                      double e_max, const double* scale_dev, double* partial, TuneResult* out, hipStream_t st);
int logsum_num_blocks(int n);
hipError_t launch_grid_scale(const float* ref, const float* rho, int n, double* partial, double* out,
                             hipStream_t st);
// e_dev non-null: e is read from device memory (e.g. a TuneResult's e_star)
hipError_t launch_qpass(const int32_t* idx, const float* d2, int n, int k, const float* rho, double e,
                        const double* e_dev, double alpha, double d, double* qa, hipStream_t st);
// rowmap non-null: stored row p (curve order, idx as curve positions, rho and qa by position) is output row
// rowmap[p], whose columns are sid[rowmap[p] * k + r]; rho_out: rho by sample id (the symmetric finish)
hipError_t launch_assemble(const int32_t* idx, const float* d2, int n, int k, const float* rho, double e,
                           const double* e_dev, const double* qa, int out_kind, int64_t* rowptr, int32_t* col,
                           float* val, double* P, double* D, hipStream_t st, const int32_t* rowmap = nullptr,
                           const int32_t* sid = nullptr, const float* rho_out = nullptr);
// the k-NN rows in curve order (row p = sample cid[p]), neighbours as curve positions, and their bandwidths
hipError_t launch_curve_rows(const int32_t* idx, const float* d2, int n, int k, int k0, const int32_t* cid,
                             const int32_t* pos, int32_t* idx_c, float* d2_c, float* b_c, hipStream_t st);
// out[i] = in[pos[i]] for up to three vectors (null pointers skipped)
hipError_t launch_gather_samples(const int32_t* pos, int n, const float* a_c, float* a, const float* b_c, float* b,
                                 const float* c_c, float* c, hipStream_t st);

// learned partitioner: MLP (mlp_kernels.hip)
hipError_t launch_gemm_nt(const uint16_t* A, int lda, const uint16_t* B, int ldb, int M, int N, int K,
                          const float* bias, int relu, const float* mask_ref, int ldm, float* Cf, int ldcf,
                          uint16_t* Cb, int ldcb, hipStream_t st);
hipError_t launch_transpose_bf16(const uint16_t* src, int rows, int cols, uint16_t* dst, hipStream_t st);
hipError_t launch_cast_rows_bf16(const float* src, int cols, const int32_t* idx, int valid, int rows, int ldd,
                                 uint16_t* dst, hipStream_t st);
hipError_t launch_cast_bf16(const float* src, int64_t cnt, uint16_t* dst, hipStream_t st);
hipError_t launch_colsum(const float* src, int rows, int cols, float* out, hipStream_t st);
hipError_t launch_softmax_xent(const float* Z, int B, int NB, const int32_t* lab, int ks, float* dZ, uint16_t* dZb,
                               double* row_loss, double* loss_out, int add, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m1, float* m2, int64_t cnt, float lr, float b1, float b2,
                       float eps, float c1, float c2, uint16_t* pb, hipStream_t st);
hipError_t launch_route_topp(const float* Z, int rows, int NB, int P, int32_t* home, int32_t* probe, hipStream_t st);
hipError_t launch_fill_normal(float* p, int64_t cnt, uint64_t seed, uint64_t offset, float scale, hipStream_t st);

// learned partitioner: teacher, batches, bucket layout (learned_kernels.hip)
hipError_t sort_pairs_u64(void* tmp, size_t& tmp_bytes, const uint64_t* kin, uint64_t* kout, const int32_t* vin,
                          int32_t* vout, int cnt, int end_bit, hipStream_t st);
hipError_t sort_pairs_u32(void* tmp, size_t& tmp_bytes, const uint32_t* kin, uint32_t* kout, const int32_t* vin,
                          int32_t* vout, int cnt, int end_bit, hipStream_t st);
hipError_t sort_keys_u64(void* tmp, size_t& tmp_bytes, const uint64_t* kin, uint64_t* kout, int64_t cnt,
                         int end_bit, hipStream_t st);
hipError_t launch_teacher_keys(const float* X, int ns, int m, const int32_t* node, int level, uint64_t seed,
                               uint64_t* keys, int32_t* vals, hipStream_t st);
hipError_t launch_teacher_split(const uint64_t* skeys, const int32_t* svals, int ns, int nodes, int32_t* start,
                                int32_t* node_out, hipStream_t st);
hipError_t launch_batch_gather(int64_t ns, uint64_t a, uint64_t c, int64_t t0, int B, const int32_t* idx_s, int ks,
                               const int32_t* labels, int32_t* bidx, int32_t* nbrlab, hipStream_t st);
hipError_t launch_member_keys(const int32_t* home, int n, uint64_t* keys, hipStream_t st);
hipError_t launch_query_keys(const int32_t* probe, int n, int P, uint64_t* keys, hipStream_t st);
hipError_t launch_bucket_layout(const uint64_t* skeys, int n, int nb, int32_t* mstart, int32_t* tptr,
                                int32_t* cid, int64_t cid_rows, int32_t* brow, hipStream_t st);
hipError_t launch_work_layout(const uint64_t* qkeys, int n, int nb, int P, int qpb, int max_work, int32_t* qptr,
                              int2* work, int32_t* n_work, int32_t* qids, hipStream_t st);

// ---- union pattern E u E^T and the passes over a CSR pattern
// scratch of the transpose-merge (arrays of n k entries unless noted)
struct UnionWork {
    int32_t* scol;              // directed rows sorted by column
    float* sd2;
    uint8_t* flag;              // entry contributes a reverse entry
    uint16_t* boff;             // [n, 32] bucket index of the sorted rows
    uint64_t* rkey;             // reverse entries (at most n k), by row segment
    int* cnt;                   // [n + 1]
    int64_t* revptr;            // [n + 1]
    unsigned long long* bad;    // [1] invalid-input flag
    int* long_count;            // [1]
    int* long_rows;             // [n]
    void* scan_tmp;
    size_t scan_bytes;
};
size_t union_scan_bytes(int n);
// steps 1-3: sorted rows, flags, counts, revptr (revptr[n] = reverse entries)
hipError_t launch_union_count(const int32_t* idx, const float* d2, int n, int k, const UnionWork& w, hipStream_t st);
// steps 4-6 into rowptr [n + 1], col and ud2 [n k + revptr[n]]
hipError_t launch_union_place(int n, int k, const UnionWork& w, int64_t* rowptr, int32_t* col, float* ud2,
                              hipStream_t st);
// the directed k-NN rows sorted by column as CSR (rowptr_i = i k)
hipError_t launch_sorted_rows(const int32_t* idx, const float* d2, int n, int k, int64_t* rowptr, int32_t* col,
                              float* sd2, hipStream_t st);
// threshold truncation: keep x = d2 / (e rho_i rho_j) < L (L = -ln delta); cnt [n + 1]
// and scan_tmp (union_scan_bytes(n)) are scratch; col_out, d2_out need rowptr[n] entries
hipError_t launch_truncate(const int64_t* rowptr, const int32_t* col, const float* d2, const float* rho, int n,
                           double e, const double* e_dev, double L, int* cnt, void* scan_tmp, size_t scan_bytes,
                           int64_t* rowptr_out, int32_t* col_out, float* d2_out, hipStream_t st);
hipError_t launch_check_csr(const int64_t* rowptr, const int32_t* col, int n, int64_t nnz, unsigned long long* bad,
                            hipStream_t st);
hipError_t launch_density_csr(const int64_t* rowptr, const int32_t* col, const float* d2, int n, const float* b,
                              double e, const double* e_dev, double d, double beta, float* rho, float* psi,
                              hipStream_t st);
// nnz_cap: an upper bound of rowptr[n] (the kernel reads the count from
// rowptr[n]); nnz_hint: the expected count, which sets the block partition
int chi_csr_blocks(int64_t nnz_hint, int64_t nnz_cap);
// rowid [nnz] (or null: the kernel walks rowptr): each entry's row, from launch_row_ids
hipError_t launch_row_ids(const int64_t* rowptr, int n, int32_t* rowid, hipStream_t st);
hipError_t launch_chi_csr(const int64_t* rowptr, const int32_t* rowid, const int32_t* col, const float* d2, int n,
                          int64_t nnz_hint, int64_t nnz_cap, const float* rho, int G, double e_min, double e_max,
                          const double* scale_dev, double* partial, TuneResult* out, hipStream_t st);
hipError_t launch_qpass_csr(const int64_t* rowptr, const int32_t* col, const float* d2, int n, const float* rho,
                            double e, const double* e_dev, double alpha, double d, double* qa, hipStream_t st);
hipError_t launch_assemble_rows(const int64_t* rowptr, const int32_t* col, const float* d2, int n, const float* rho,
                                double e, const double* e_dev, const double* qa, int out_kind, float* val, double* P,
                                double* D, hipStream_t st);

}  // namespace kvb
