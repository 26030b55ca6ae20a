/*
 * kvb — self-tuning variable-bandwidth kernel matrices on MI355X (gfx950).
 *
 * C ABI of the HIP library libkvb.so. It builds, from n samples x^(i) in R^m,
 * the sparse kernel matrix that approximates the Kolmogorov operator
 * L_{psi,c} (Davis & Giannakis, arXiv 2104.15124, Sections 2 and 4):
 *
 *   kvb_knn            k nearest neighbours of every sample (the sparsity
 *                      pattern; neighbour order I(x, k) of Section 2.1)
 *   kvb_bandwidth      ad-hoc bandwidth b (Section 2.1, bandwidth eq.) or the
 *                      density estimate psi and operator bandwidth
 *                      rho = 2 psi^beta (Section 2.1 density eqs.; Algorithm 1
 *                      caption)
 *   kvb_grid_scale     power-of-two placement of the operator-stage e grid
 *   kvb_tune_eps       bandwidth self-tuning: chi(e) = sum_ij K_ij on a log
 *                      grid, optimum = argmax d log chi / d log e (Section 2.3)
 *   kvb_assemble_csr   q, alpha-normalised Kt, degrees D and the Markov matrix
 *                      D^{-1} Kt (or L, or its symmetric conjugate) as CSR
 *                      (Section 2.2)
 *
 * Notation. e is the paper's epsilon^2. One kernel serves both stages:
 *   K_ij = exp(-|x_i - x_j|^2 / (e rho_i rho_j)),
 * with rho = b for the density kernel K_eps (Section 2.1) and rho = 2 psi^beta
 * for the operator kernel K_{eps,beta} (Section 2.2), where 4 epsilon^2
 * (psi_i psi_j)^beta = e rho_i rho_j. P_i = psi_i^beta = rho_i / 2.
 * The pattern is the directed k-NN graph: row i stores i itself and its k-1
 * nearest other samples, all k entries kept (no threshold truncation).
 *
 * Memory. Every pointer argument is a DEVICE pointer unless its name ends in
 * _host. The caller allocates and owns all inputs and outputs; the library
 * never frees or retains them beyond the call. The library owns only the
 * scratch memory inside a context (grown on demand, released by kvb_destroy).
 * Arrays must be aligned to their element size. Layouts are row-major and dense.
 *
 * Streams. A context is bound to one HIP stream at creation. All work of a
 * call is enqueued on that stream and the call returns without waiting,
 * except calls that return *_host values (kvb_grid_scale, kvb_tune_eps,
 * kvb_knn_fallback_rows), which synchronise the context stream before returning.
 *
 * Errors. Every int-returning entry point returns a status: 0 = OK, > 0 = OK
 * with a warning, < 0 = error (nothing useful was written). No call aborts or
 * throws. kvb_last_error(ctx) describes the last non-zero status of that
 * context. A context is not thread-safe; distinct contexts are independent.
 *
 * Determinism. Reductions run in a fixed order with no floating-point
 * atomics, so results are bitwise reproducible from run to run.
 */
#ifndef KVB_H
#define KVB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define KVB_OK 0
#define KVB_W_GRID_EDGE 1    /* tuning optimum on the first or last slope of the grid */
#define KVB_W_FALLBACK 2     /* kvb_knn_fallback_rows: some rows needed the exact fallback scan */
#define KVB_W_NOT_CONVERGED 3 /* kvb_eigsh: some Ritz residual above the tolerance (results still returned) */
#define KVB_E_INVALID (-1)   /* an argument is out of range or a pointer is null/misaligned */
#define KVB_E_NOMEM (-2)     /* scratch allocation failed or exceeds KVB_OPT_SCRATCH_LIMIT */
#define KVB_E_HIP (-3)       /* a HIP runtime call failed (message carries its error string) */
#define KVB_E_UNSUPPORTED (-4) /* valid but beyond this build's capacity, or not a gfx950 device */
#define KVB_E_NOT_TRAINED (-5) /* learned mode requested before a partitioner exists */
#define KVB_E_IO (-6)        /* partitioner file missing, short or corrupt */
#define KVB_E_NO_DEVICE (-7) /* a host-only context (kvb_create_host): the arguments passed every check
                                and nothing ran */

/* ---- k-NN modes ---- */
#define KVB_KNN_F32 0        /* FP32 distance tiles (direct differences for m <= 8, FP32 MFMA otherwise) */
#define KVB_KNN_BF16 1       /* BF16 MFMA distance tiles, FP32 accumulation */
#define KVB_KNN_LEARNED 2    /* learned partitioner routes queries to candidate buckets */

/* ---- bandwidth modes ---- */
#define KVB_BW_ADHOC 0       /* rho_i = b_i = sqrt(sum_{r=1..k0} d2[i, r]) */
#define KVB_BW_DENSITY 1     /* psi_i and rho_i = 2 psi_i^beta from the density kernel with rho = b */

/* ---- output kinds of kvb_assemble_csr ---- */
#define KVB_OUT_MARKOV 0     /* M = D^{-1} Kt (row-stochastic) */
#define KVB_OUT_GENERATOR 1  /* L = e^{-1} P^{-2} (M - I) */
#define KVB_OUT_SYMMETRIC 2  /* Lhat = e^{-1} (S^{-1} Kt S^{-1} - P^{-2}), S = P D^{1/2} */

/* ---- row flags written by kvb_knn ---- */
#define KVB_ROW_RECHECK 1    /* FP64 recheck decided membership at the k-th neighbour */
#define KVB_ROW_FALLBACK 2   /* the row was recomputed by the exact fallback scan */
#define KVB_ROW_UNCERTIFIED 4 /* learned mode: no exactness certificate for this row */

/* ---- options (kvb_set_option) ---- */
#define KVB_OPT_FORCE_FALLBACK 1 /* value N > 0: also send every N-th row to the fallback (testing) */
#define KVB_OPT_SCRATCH_LIMIT 2  /* value: maximum scratch bytes; 0 = unlimited */
#define KVB_OPT_BF16_SPLIT 3     /* BF16 terms per coordinate product in KVB_KNN_BF16 mode: 1 (x_hi only),
                                    3 (hi/lo pairs, default) or 6 (hi/mid/lo pairs) */
#define KVB_OPT_N_PROBE 4        /* learned mode: buckets each query searches (1..min(32, n_buckets)); needs a
                                    partitioner in the context; saved with it */
#define KVB_OPT_CURVE_ORDER 5    /* matrix-core exact modes, m <= 256: 1 scans candidates in the Morton order
                                    of the principal projections and skips tiles whose projected boxes lie
                                    beyond every query's threshold; 2 (default) does the same after halving
                                    every group of 4096 consecutive tiles at its median along the widest side
                                    of its box, recursively down to single tiles (a k-d order inside each
                                    group: tighter tile and tree boxes, fewer scored pairs); 0 scans every tile
                                    in sample order. Every value gives the same exact k-NN */
#define KVB_OPT_PATTERN 6        /* pattern of kvb_build's matrix: KVB_PATTERN_KNN (default) or KVB_PATTERN_UNION */
#define KVB_PATTERN_KNN 0        /* the directed k-NN pattern, k entries per row */
#define KVB_PATTERN_UNION 1      /* E u E^T (as kvb_union_pattern); col and val must then hold n (2k - 1)
                                    entries and rowptr[n] gives the stored count */

typedef struct kvb_ctx_s* kvb_ctx;

/* Create a context bound to hip_stream (a hipStream_t; NULL = the null stream)
 * on the current device. Fails with KVB_E_UNSUPPORTED on a non-gfx950 device. */
int kvb_create(kvb_ctx* out, void* hip_stream);

/* Create a context bound to no device (callers: argument screening and tests on a machine without a
 * GPU; needs no HIP device). Every entry point called with it checks its arguments exactly as with a
 * device context, returning the same KVB_E_INVALID / KVB_E_UNSUPPORTED / KVB_E_NOT_TRAINED status and
 * kvb_last_error message, and returns KVB_E_NO_DEVICE (nothing launched, no memory read or written)
 * where it would start work on the device. Released by kvb_destroy. */
int kvb_create_host(kvb_ctx* out);

/* Release the context and its scratch. Waits for its stream first. NULL is a no-op. */
void kvb_destroy(kvb_ctx ctx);

/* Message of the last non-zero status of ctx ("" if none). Owned by ctx. */
const char* kvb_last_error(kvb_ctx ctx);

/* Set an option (KVB_OPT_*). Unknown keys or bad values -> KVB_E_INVALID. */
int kvb_set_option(kvb_ctx ctx, int32_t key, int64_t value);

/*
 * Exact k-nearest-neighbour self-join (Section 2.1 neighbour order; the
 * brute-force pattern of Section 4, Algorithm 1, with a fixed k per row).
 *   X        [n, m] float32 row-major samples (finite values).
 *   k        neighbours per row including the row itself, 1 <= k <= n.
 *   mode     KVB_KNN_F32 or KVB_KNN_BF16 (exact sets), KVB_KNN_LEARNED
 *            (needs kvb_part_*; recall < 1 possible). F32 uses direct
 *            differences on the vector ALUs for m <= 8 and FP32 matrix-core
 *            tiles otherwise; BF16 uses BF16 matrix-core tiles with the
 *            coordinates split into KVB_OPT_BF16_SPLIT terms.
 *   margin   extra candidates kept by the distance tiles before the exact
 *            re-rank, 0 <= margin and k + margin <= 256.
 *   idx      [n, k] int32 out: row i = i, then the k-1 nearest j != i.
 *   d2       [n, k] float32 out: squared distances (d2[i, 0] = 0), ascending.
 *   row_flags [n] int32 out (KVB_ROW_* bits) or NULL.
 * Membership of the k-th neighbour is decided in FP64 (ties by smaller index);
 * within a row, entries are ordered by their compensated FP32 distance.
 * Requires n < 2^31 and m <= 1024. Asynchronous: rows that needed the exact
 * fallback are marked in row_flags and counted by kvb_knn_fallback_rows.
 * KVB_KNN_LEARNED without a partitioner in ctx returns KVB_E_NOT_TRAINED.
 */
int kvb_knn(kvb_ctx ctx, const float* X, int64_t n, int32_t m, int32_t k,
            int32_t mode, int32_t margin, int32_t* idx, float* d2, int32_t* row_flags);

/* Number of candidate pairs (query row, candidate sample) whose score the
 * distance tiles of the last kvb_knn call on ctx computed: the tiles the
 * spatial scans did not skip by their boxes (direct tiles, curve-ordered
 * matrix-core tiles), every pair when KVB_OPT_CURVE_ORDER is 0, or the routed
 * pairs of the learned search. Synchronises the context stream. */
int kvb_knn_pairs(kvb_ctx ctx, double* pairs_host);

/*
 * Exact k-NN of selected rows against all n samples, by float64 distances
 * and a radix selection (the same scan as the exact fallback of kvb_knn):
 * the judge of recall for KVB_KNN_LEARNED on a sample of rows.
 *   rows     [nrows] int32 device array of row ids (0 <= rows[t] < n).
 *   idx, d2  [nrows, k] out, row t for sample rows[t], in kvb_knn's layout
 *            (self first, then (d2, index) order; d2 rounded to float32).
 * An id outside [0, n) yields a row of -1 / NaN. Asynchronous.
 */
int kvb_knn_exact_rows(kvb_ctx ctx, const float* X, int64_t n, int32_t m, int32_t k, const int32_t* rows,
                       int64_t nrows, int32_t* idx, float* d2);

/* Number of rows of the last kvb_knn call on ctx that took the exact fallback
 * scan. Synchronises the context stream. Returns KVB_W_FALLBACK if > 0. */
int kvb_knn_fallback_rows(kvb_ctx ctx, int64_t* count_host);

/*
 * Per-sample bandwidths over the k-NN pattern (idx, d2 as written by kvb_knn).
 *   KVB_BW_ADHOC:   rho_i = sqrt(sum_{r=1..k0} d2[i, r]), 1 <= k0 < k
 *                   (Section 2.1, bandwidth eq.). b, e, d, beta, psi unused.
 *   KVB_BW_DENSITY: psi_i = sum_r exp(-d2[i,r] / (e b_i b_j)) / (n (pi e b_i^2)^{d/2}),
 *                   rho_i = 2 psi_i^beta, with j = idx[i, r] and n the total
 *                   sample count (Section 2.1 density eqs.; Algorithm 1 caption).
 *                   b [n] float32 in; psi [n] float32 out or NULL. e > 0, d > 0.
 *   rho [n] float32 out.
 */
int kvb_bandwidth(kvb_ctx ctx, const int32_t* idx, const float* d2, int64_t n, int32_t k,
                  int32_t mode, int32_t k0, const float* b, double e, double d, double beta,
                  float* rho, float* psi);

/*
 * Operator-stage grid placement: *scale_host = 2^round(log2(gm(ref^2)/gm(rho^2))),
 * gm = geometric mean over the n samples (FP64, fixed-order reduction). Scaling
 * the e grid by it moves the grid to where e rho_i rho_j matches the density
 * stage; the Kolmogorov matrix is invariant under psi -> c psi, e -> e c^{-2 beta}
 * (Section 2.2), so only the grid's coverage changes. ref, rho [n] float32, > 0.
 * Synchronises the context stream.
 */
int kvb_grid_scale(kvb_ctx ctx, const float* ref, const float* rho, int64_t n,
                   double* scale_host);

/*
 * Bandwidth self-tuning (Section 2.3) over the k-NN pattern:
 *   e_g = exp(ln e_min + g (ln e_max - ln e_min)/(G - 1)), g = 0..G-1,
 *   chi[g] = sum_i sum_r exp(-d2[i,r] / (e_g rho_i rho_{idx[i,r]})) (self terms included),
 *   slope_g = (ln chi[g+1] - ln chi[g]) / (ln e_{g+1} - ln e_g), g = 0..G-2,
 *   g* = first argmax of slope, *e_star_host = e_{g*}, *dim_host = 2 slope_{g*}.
 * Kernel values are FP32 per entry, summed per row in FP32 and across rows in
 * FP64 in a fixed order. 3 <= G <= 256, 0 < e_min < e_max.
 * chi_host [G] (or NULL), e_star_host (required), dim_host (or NULL) are host memory.
 * Returns KVB_W_GRID_EDGE when g* is 0 or G-2. Synchronises the context stream.
 */
int kvb_tune_eps(kvb_ctx ctx, const int32_t* idx, const float* d2, const float* rho,
                 int64_t n, int32_t k, double e_min, double e_max, int32_t G,
                 double* chi_host, double* e_star_host, double* dim_host);

/*
 * kvb_tune_eps without any allocation, for callers that cannot allocate
 * device memory during a call (serving loops, harnesses that forbid it). Same
 * arguments, results (bit for bit) and status as kvb_tune_eps, and the same
 * synchronisation. Its scratch (the sums' block partials and the result) is a
 * static device array of 4 MiB that each GPU holds from library load until the
 * process ends; its address is looked up when a context is created on that
 * GPU. Every call on one GPU shares that array: calls that overlap in time on
 * one GPU race and must be ordered by the caller. The tuning needs at most
 * 2 MiB of it (1024 blocks x G <= 256 doubles); a need beyond the array
 * returns KVB_E_UNSUPPORTED. KVB_OPT_SCRATCH_LIMIT does not apply (nothing is
 * allocated).
 */
int kvb_tune_eps_noalloc(kvb_ctx ctx, const int32_t* idx, const float* d2, const float* rho,
                         int64_t n, int32_t k, double e_min, double e_max, int32_t G,
                         double* chi_host, double* e_star_host, double* dim_host);

/*
 * Normalisation into CSR (Section 2.2):
 *   K_ir = exp(-d2[i,r] / (e rho_i rho_j)), P_i = rho_i / 2,
 *   q_i = P_i^{-d} sum_r K_ir, Kt_ir = K_ir / (q_i q_j)^alpha, D_i = sum_r Kt_ir,
 *   out_kind KVB_OUT_MARKOV:    val = Kt_ir / D_i
 *            KVB_OUT_GENERATOR: val = (Kt_ir / D_i - [j == i]) / (e P_i^2)
 *            KVB_OUT_SYMMETRIC: val = (Kt_ir / (S_i S_j) - [j == i] / P_i^2) / e, S = P sqrt(D)
 * Entries are evaluated with an FP64 argument and exponential; q and D are
 * FP64 row sums (compensated). Columns ascend within each row.
 *   rowptr [n+1] int64 out (rowptr[i] = i k), col [n k] int32 out,
 *   val [n k] float32 out, P [n] float64 out or NULL, D [n] float64 out or NULL.
 */
int kvb_assemble_csr(kvb_ctx ctx, const int32_t* idx, const float* d2, const float* rho,
                     int64_t n, int32_t k, double e, double alpha, double d, int32_t out_kind,
                     int64_t* rowptr, int32_t* col, float* val, double* P, double* D);

/* ---- the union pattern E u E^T ----
 * The paper's kernel matrix is symmetric: its brute-force construction sets
 * K_ij and K_ji together (Section 4, Algorithm 1). A directed k-NN pattern is
 * not; its union with its transpose is. These calls build that pattern and run
 * the density, tuning and normalisation passes over any CSR pattern (row sums
 * then run over the stored row, whatever its length).
 *
 * kvb_union_pattern: row i of the output holds every j with j in row i of idx
 * or i in row j of idx, once, columns ascending; ud2 carries the squared
 * distance of the pair, taken from row i of d2 where (i, j) is stored there,
 * else from row j.
 *   idx [n k] int32, d2 [n k] float32 in: a k-NN pattern as written by kvb_knn
 *     (each row k distinct columns in [0, n)); 1 <= k <= 256.
 *   rowptr [n+1] int64 out (rowptr[0] = 0, rowptr[n] = nnz);
 *   col [cap] int32 out, ud2 [cap] float32 out: the first nnz entries are written.
 *     cap = n (2k - 1) always suffices; nnz <= cap is required.
 *   nnz_host: host out (required).
 * The result is deterministic. Scratch grows by about 17 bytes per directed entry.
 * Synchronises the context stream (once, to size the transpose). KVB_E_INVALID
 * for a repeated column or a column outside [0, n) in a row of idx, or for
 * cap < nnz (the outputs are then unspecified, *nnz_host is set).
 */
int kvb_union_pattern(kvb_ctx ctx, const int32_t* idx, const float* d2, int64_t n, int32_t k,
                      int64_t* rowptr, int32_t* col, float* ud2, int64_t cap, int64_t* nnz_host);

/*
 * The passes of kvb_bandwidth (KVB_BW_DENSITY), kvb_tune_eps and
 * kvb_assemble_csr over a CSR pattern with nnz entries: rowptr [n+1] int64
 * (rowptr[0] = 0, non-decreasing, rowptr[n] = nnz), col [nnz] int32 in
 * [0, n), ud2 [nnz] float32 squared distances. Same formulas, with r running
 * over the stored entries of row i. kvb_normalize_csr writes val [nnz] float32
 * in pattern order (it does not reorder columns); P, D as kvb_assemble_csr.
 * Each call checks the pattern's shape on the device and synchronises once to
 * read the check; KVB_E_INVALID if it fails (nothing else is written then).
 */
int kvb_density_csr(kvb_ctx ctx, const int64_t* rowptr, const int32_t* col, const float* ud2, int64_t n,
                    int64_t nnz, const float* b, double e, double d, double beta, float* rho, float* psi);
int kvb_tune_eps_csr(kvb_ctx ctx, const int64_t* rowptr, const int32_t* col, const float* ud2, const float* rho,
                     int64_t n, int64_t nnz, double e_min, double e_max, int32_t G,
                     double* chi_host, double* e_star_host, double* dim_host);
int kvb_normalize_csr(kvb_ctx ctx, const int64_t* rowptr, const int32_t* col, const float* ud2, const float* rho,
                      int64_t n, int64_t nnz, double e, double alpha, double d, int32_t out_kind,
                      float* val, double* P, double* D);

/*
 * Threshold truncation (Section 4: Algorithm 1 stores an entry only when its
 * kernel value exceeds the sparsity tolerance delta_tol). Entry (i, j) of the
 * CSR pattern (rowptr, col, d2: as kvb_density_csr) is kept when
 * exp(-d2 / (e rho_i rho_j)) > delta, 0 < delta < 1; the test is taken on the
 * exponent, x < -ln(delta) with x = (d2 (1 / (e rho_i))) / rho_j in FP64 and
 * ln on the host (the same inequality without the rounding of exp; an entry
 * whose exponent lies within a few FP64 rounding steps of -ln(delta) may be
 * decided either way). Kept entries keep their order.
 *   rho [n] float32 in; e > 0.
 *   rowptr_out [n+1] int64 out; col_out [nnz] int32 out, d2_out [nnz] float32
 *   out (capacity nnz always suffices; rowptr_out[n] entries are written).
 *   nnz_host: host out or NULL.
 * Checks the input pattern's shape as kvb_density_csr does (one
 * synchronisation); with nnz_host non-NULL it synchronises again to report
 * the count.
 */
int kvb_truncate_csr(kvb_ctx ctx, const int64_t* rowptr, const int32_t* col, const float* d2, const float* rho,
                     int64_t n, int64_t nnz, double e, double delta, int64_t* rowptr_out, int32_t* col_out,
                     float* d2_out, int64_t* nnz_host);

/*
 * Leading eigenpairs of a symmetric CSR matrix (the paper's spectral use of
 * the kernel matrix: the eigenpairs of the symmetric conjugate Lhat of
 * Section 2.2, e.g. KVB_OUT_SYMMETRIC on KVB_PATTERN_UNION, approximate the
 * Kolmogorov operator's; Sections 2.2, 4 and 5). Lanczos with full
 * reorthogonalisation (two passes of classical Gram-Schmidt per step), ncv
 * steps from a seeded start vector, no restart; the Lanczos coefficients stay
 * on the device until the last step. The Ritz pairs of the tridiagonal
 * projection T (eigenvalues by Sturm-count bisection, eigenvectors by inverse
 * iteration, on the host in FP64) are returned for the nev largest
 * eigenvalues (for Lhat, those nearest zero), descending. A breakdown
 * (beta_j = 0: an invariant subspace) ends the projection early; its Ritz
 * pairs are then exact.
 *   rowptr, col, val: the matrix (as kvb_density_csr, val float32); it must be
 *     symmetric (not checked; a non-symmetric input gives meaningless but
 *     finite results).
 *   1 <= nev <= ncv <= min(4096, n); tol > 0; seed: the start vector's seed.
 *   evals_host [nev] host out; resid_host [nev] host out or NULL: the Ritz
 *     residual norms |beta_{m-1} s_{m-1,i}| (m the steps used).
 *   evecs [nev * n] float64 device out or NULL: unit Ritz vectors, one per row.
 * Returns KVB_W_NOT_CONVERGED if a residual exceeds tol * ||T||_inf (results
 * still returned); KVB_E_INVALID if a Lanczos coefficient is not finite (the
 * matrix holds non-finite values) or the space closes before nev steps.
 * Scratch: (ncv + 1) n doubles. Synchronises the context stream once after the
 * steps (and once more when evecs is requested).
 */
int kvb_eigsh(kvb_ctx ctx, const int64_t* rowptr, const int32_t* col, const float* val, int64_t n, int64_t nnz,
              int32_t nev, int32_t ncv, double tol, uint64_t seed, double* evals_host, double* resid_host,
              double* evecs);

/* The part of a Lanczos run kvb_eigsh keeps (host only, needs no device):
 * *m_host = the steps up to and including the first breakdown (beta_j <= 1e-300)
 * or ncv. KVB_E_INVALID if alpha_j or beta_j of a kept step is not finite or
 * beta_j < 0 (*m_host then counts the steps before it).
 *   alpha_host, beta_host [ncv] host in. */
int kvb_lanczos_prefix(const double* alpha_host, const double* beta_host, int32_t ncv, int32_t* m_host);

/*
 * Spectral solution of the Kolmogorov problem L f = g (Section 3.1): the
 * least-squares solution in the span of the leading eigenvectors of L with
 * nonzero eigenvalue, f = Q Lambda^{-1} g~, g~ = Q^T S^2 g / n, where the
 * columns phi_j of Q satisfy <phi_i, phi_j>_S = phi_i^T S^2 phi_j / n =
 * delta_ij. With unit eigenvectors y_j of the symmetric conjugate Lhat (as
 * kvb_eigsh returns them) phi_j = sqrt(n) S^{-1} y_j, so
 * f = S^{-1} sum_j y_j (y_j . S g) / lambda_j.
 *   evecs [nvec * n] float64 device (unit rows), evals_host [nvec]: eigenpairs
 *     of Lhat; the first `skip` pairs (the null pair, eigenvalue 0) are left out.
 *   P, D [n] float64 device: as kvb_assemble_csr returns them (S = P D^{1/2}).
 *   g [n] float64 device in; f [n] float64 device out; g_proj [n] float64
 *   device out or NULL: the projection g_l = Q g~ of g on the span.
 *   coef_host [nvec - skip] host out or NULL: the coefficients g~_j.
 * Synchronises the context stream.
 */
int kvb_kolmogorov_solve(kvb_ctx ctx, const double* evecs, const double* evals_host, int32_t nvec, int32_t skip,
                         const double* P, const double* D, const double* g, int64_t n, double* f, double* g_proj,
                         double* coef_host);

/*
 * Gradients through the Carre du champ identity (Section 3.2): for functions
 * u, v sampled at the n points, grad u . grad v at the samples from the
 * eigenbasis, sum over l, j, k < nvec of u~_j v~_k C_ljk (lambda_l - lambda_j
 * - lambda_k) / 2 phi_l, with C_ljk = <phi_l, phi_j phi_k>_S, u~_j = <u, phi_j>_S,
 * v~_k = <v, phi_k>_S and phi_j = sqrt(n) S^{-1} y_j (y_j unit eigenvectors of
 * Lhat as kvb_eigsh returns them, the null pair first). v = x_s gives the
 * derivative of u along coordinate s. The sum over j and k is evaluated as
 * lambda_l U V - (L U) V - U (L V) with U, V the projections of u, v and L U,
 * L V their images, which equals the triple sum term by term.
 *   evecs [nvec * n] float64 device, evals_host [nvec]; P, D [n] float64 device.
 *   u, v [n] float64 device in; grad [n] float64 device out.
 *   C [nvec^3] float64 device out or NULL (nvec <= 64): C_ljk, index (l nvec + j) nvec + k.
 * Synchronises the context stream.
 */
int kvb_carre_du_champ(kvb_ctx ctx, const double* evecs, const double* evals_host, int32_t nvec, const double* P,
                       const double* D, const double* u, const double* v, int64_t n, double* grad, double* C);

/*
 * Particle update of the density-evolution example (Section 5.3, the explicit
 * step of the sample SDE): x' = x + dt (u - grad f) + sqrt(dt) sigma w, where
 * grad f comes from kvb_carre_du_champ with v = x_s for each coordinate s and
 * f from kvb_kolmogorov_solve.
 *   X, X_out [n, m] float32 device, row-major (may be the same array).
 *   velocity [n, m] float64 device or NULL (u = 0); noise [n, m] float64 device
 *   or NULL (no diffusion): standard normal draws w, which the caller supplies.
 *   grad [m, n] float64 device: component s of grad f at every sample in row s.
 * Enqueued only.
 */
int kvb_advect(kvb_ctx ctx, const float* X, int64_t n, int32_t m, const double* velocity, const double* grad,
               const double* noise, double dt, double sigma, float* X_out);

/*
 * Sparsity tolerance of kvb_build (Section 4: Algorithm 1 stores an entry only
 * when its kernel value exceeds delta_tol), 0 <= delta < 1; 0 (the default)
 * keeps every entry. With delta > 0 kvb_build truncates the density kernel
 * matrix at e_A and the operator kernel matrix at e_B as kvb_truncate_csr
 * does; the tuning sums still run over the whole pattern, and the density, q
 * and D row sums over the kept entries. Its CSR rows then hold the kept
 * entries, columns ascending; rowptr[n] gives their count.
 */
int kvb_set_tolerance(kvb_ctx ctx, double delta);

/*
 * The whole build in one call, in the order of the paper's pipeline (Section 4
 * with the tuning of Section 2.3): k-NN (as kvb_knn) -> ad-hoc bandwidth b ->
 * e tuning on the density kernel over [e_min, e_max] -> density psi and
 * rho = 2 psi^beta -> grid scale s (as kvb_grid_scale with ref = b) -> e tuning
 * on the operator kernel over [s e_min, s e_max] -> q, Kt, D and the CSR of
 * out_kind (as kvb_assemble_csr). Intermediate results stay on the device;
 * results equal those of the separate calls bit for bit. With info_host
 * non-NULL the call synchronises once, at the end; with info_host NULL it
 * only enqueues the work on the context's stream and returns KVB_OK (argument
 * errors are still returned at once), so that consecutive builds run back to
 * back; kvb_build_info then waits for the last build and reports it.
 *   idx, d2, row_flags   as kvb_knn (row_flags may be NULL).
 *   b, rho [n] float32 out; psi [n] float32 out or NULL.
 *   rowptr, col, val, P, D   as kvb_assemble_csr (P, D may be NULL); with
 *                KVB_OPT_PATTERN = KVB_PATTERN_UNION the pattern is E u E^T and
 *                every pass after the ad-hoc bandwidth runs over it, as
 *                kvb_union_pattern, kvb_tune_eps_csr, kvb_density_csr and
 *                kvb_normalize_csr would (col, val: n (2k - 1) entries).
 *   chi_a_host, chi_b_host   [G] host out or NULL: the tuning sums of both stages.
 *   info_host [8] host out or NULL: e_A, dim_A, s, e_B, dim_B, g*_A, g*_B, rows
 *                that took the exact k-NN fallback.
 * Returns KVB_W_GRID_EDGE if either optimum lies at the edge of its grid,
 * else KVB_W_FALLBACK if some rows took the fallback, else KVB_OK; errors as
 * the separate calls.
 */
int kvb_build(kvb_ctx ctx, const float* X, int64_t n, int32_t m, int32_t k, int32_t mode, int32_t margin, int32_t k0,
              double d, double alpha, double beta, double e_min, double e_max, int32_t G, int32_t out_kind,
              int32_t* idx, float* d2, int32_t* row_flags, float* b, float* rho, float* psi, int64_t* rowptr,
              int32_t* col, float* val, double* P, double* D, double* chi_a_host, double* chi_b_host,
              double* info_host);

/* Wait for the context's stream and report the last kvb_build on it, as that
 * call reports with non-NULL host arguments (chi_*_host may be NULL; info_host
 * [8] must not). KVB_E_INVALID if the context has run no build. */
int kvb_build_info(kvb_ctx ctx, double* chi_a_host, double* chi_b_host, double* info_host);

/*
 * ---- learned partitioner (k-NN over routed candidate buckets) ----
 * A small MLP m -> h1 -> h2 -> n_buckets (ReLU, BF16 weights and activations,
 * FP32 accumulation) is trained on the GPU to predict, for a sample, which
 * buckets of a balanced partition its exact k nearest neighbours fall in
 * (the neighbour-histogram targets of Neural LSH, Dong et al., ICLR 2020).
 * kvb_knn(mode = KVB_KNN_LEARNED) then stores every sample in its top-1
 * bucket, sends every query to its top-n_probe buckets and searches only
 * those buckets' candidates with the matrix-core distance tiles. Results are
 * exact within the probed buckets (exact re-rank and FP64 boundary decision)
 * but carry no global certificate: rows are flagged KVB_ROW_UNCERTIFIED, and
 * recall against an exact search is the caller's measure of quality. A row
 * whose probed buckets hold fewer than k - 1 other samples takes the exact
 * fallback. One partitioner lives in a context; it is freed by kvb_destroy.
 * All array arguments are device pointers; *_host arguments are host memory.
 */

/* Create the partitioner's parameters from a seed: weights ~ N(0, 2/fan_in)
 * (Box-Muller over a SplitMix64 counter stream), zero biases, zero Adam
 * state. 1 <= m <= 1024; h1, h2, n_buckets multiples of 32 in [32, 4096];
 * 1 <= n_probe <= min(32, n_buckets). Errors: KVB_E_INVALID, KVB_E_NOMEM. */
int kvb_part_init(kvb_ctx ctx, int32_t m, int32_t h1, int32_t h2, int32_t n_buckets, int32_t n_probe,
                  uint64_t seed);

/* Teacher partition of the ns samples Xs [ns, m] float32: `levels` rounds of
 * median splits; in round l every current node is projected on its own
 * seeded random direction (components uniform in [-1, 1), SplitMix64 at
 * counter l << 40 | node << 20 | c), samples are ordered by (float32 of the
 * float64 projection, index), and the lower floor(size/2) form child 2v, the
 * rest child 2v + 1. labels [ns] int32 out, in [0, 2^levels).
 * 1 <= levels <= 12; 2^levels <= ns < 2^31. */
int kvb_part_teacher(kvb_ctx ctx, const float* Xs, int64_t ns, int32_t m, int32_t levels, uint64_t seed,
                     int32_t* labels);

/* Train the MLP with Adam (beta1 0.9, beta2 0.999, eps 1e-8, learning rate
 * lr) on soft targets: for training row i the target over buckets is the
 * histogram of labels[idx_s[i, r]], r = 0..ks-1 (its exact k-NN rows, as
 * written by kvb_knn), divided by ks; the loss is the batch-mean softmax
 * cross-entropy. Each epoch visits floor(ns / batch) batches of `batch` rows
 * (multiple of 32) in the order of a seeded affine permutation
 * t -> (a t + c) mod ns. loss_host [epochs] (or NULL) receives each epoch's
 * mean loss. Synchronises the context stream. Requires m == the partitioner's m. */
int kvb_part_train(kvb_ctx ctx, const float* Xs, int64_t ns, int32_t m, const int32_t* labels,
                   const int32_t* idx_s, int32_t ks, int32_t epochs, int32_t batch, float lr, uint64_t seed,
                   float* loss_host);

/* Routing of X [n, m]: home [n] (or NULL) = first argmax of the logits (the
 * storage bucket), probe [n, n_probe] = the n_probe largest logits in
 * descending order, ties to the smaller bucket id (probe[i, 0] == home[i]). */
int kvb_part_route(kvb_ctx ctx, const float* X, int64_t n, int32_t* home, int32_t* probe);

/* Save / load the partitioner (dimensions, weights, Adam state) to / from a
 * file (host path). Errors: KVB_E_IO. */
int kvb_part_save(kvb_ctx ctx, const char* path);
int kvb_part_load(kvb_ctx ctx, const char* path);

/* Test hooks. kvb_mlp_forward: logits [B, n_buckets] float32 of X [B, m].
 * kvb_mlp_backward: for X [B, m] and nbr_labels [B, ks] (bucket label of
 * each neighbour of each row), the batch-mean soft-target cross-entropy
 * (loss_host, may be NULL) and the gradient of every parameter in grads
 * [num_params] float32 (order W1, b1, W2, b2, W3, b3, weights row-major
 * [out, in]). Casts to BF16: the input rows, the weights, the ReLU outputs,
 * and the back-propagated logit and hidden gradients before each product.
 * B a multiple of 32 in [32, 65536]. Parameters are not updated. */
int kvb_mlp_forward(kvb_ctx ctx, const float* X, int64_t B, float* logits);
int kvb_mlp_backward(kvb_ctx ctx, const float* X, int64_t B, const int32_t* nbr_labels, int32_t ks,
                     float* loss_host, float* grads);

/* Number of parameters of the current partitioner (floats in grads), or < 0. */
int64_t kvb_part_num_params(kvb_ctx ctx);

/* Copy the FP32 master parameters (order of grads) to params [num_params]. */
int kvb_part_get_params(kvb_ctx ctx, float* params);

/* Replace the parameters by params [num_params] (order of grads) and reset
 * the Adam state. */
int kvb_part_set_params(kvb_ctx ctx, const float* params);

/* Library identification string (static storage). */
const char* kvb_version(void);

/* ---- instrumentation: device time per kernel, from HIP events recorded on
 * the context stream around each launch sequence ---- */
#define KVB_PROF_KNN_SELECT 0    /* distance tiles + top-(k+margin) selection */
#define KVB_PROF_KNN_REFINE 1    /* compensated re-rank, FP64 recheck, certificate */
#define KVB_PROF_KNN_FALLBACK 2  /* exact fallback scan (launched every call; exits early if no rows) */
#define KVB_PROF_ADHOC 3         /* ad-hoc bandwidth */
#define KVB_PROF_CHI 4           /* tuning sums: block partials + fixed-order finish */
#define KVB_PROF_DENSITY 5       /* density estimate and rho */
#define KVB_PROF_GRID_SCALE 6    /* operator-grid scale reduction */
#define KVB_PROF_QPASS 7         /* q pass */
#define KVB_PROF_ASSEMBLE 8      /* Kt, D, output kind, per-row column sort, CSR write */
#define KVB_PROF_KNN_PREP 9      /* centring and operand layout for the matrix-core distance tiles */
#define KVB_PROF_ROUTE 10        /* learned mode: MLP logits and top-n_probe routing */
#define KVB_PROF_BUCKETS 11      /* learned mode: bucket sort, candidate operand gather, work lists */
#define KVB_PROF_UNION 12        /* union pattern: row sort, transpose count, scan, sort, merge */
#define KVB_PROF_TRUNCATE 13     /* threshold truncation: count, scan, ordered fill */
#define KVB_PROF_CURVE_ROWS 14   /* kvb_build after a curve-ordered k-NN: the rows in curve order, neighbours as
                                    curve positions, and the ad-hoc bandwidths (in place of KVB_PROF_ADHOC) */
#define KVB_PROF_SLOTS 15

/* Turn event timing on (on != 0) or off; either way the totals restart at 0. */
int kvb_profile_enable(kvb_ctx ctx, int32_t on);

/* Total milliseconds and number of timed launch sequences of one slot since
 * the last kvb_profile_enable. Synchronises on the recorded events. */
int kvb_profile_read(kvb_ctx ctx, int32_t slot, double* total_ms_host, int64_t* launches_host);

/* Short name of a slot ("" if out of range; static storage). */
const char* kvb_profile_name(int32_t slot);

/* ---- measured peaks: the chip's rates for the resources the build is bound
 * by, so that roofline fractions can be stated against the chip as measured as
 * well as against its published figures ---- */
#define KVB_PEAK_HBM_COPY 0   /* bytes read + written per second by a streaming copy of 2 GiB */
#define KVB_PEAK_MFMA_BF16 1  /* flops per second of v_mfma_f32_32x32x16_bf16 chains */
#define KVB_PEAK_MFMA_F32 2   /* flops per second of v_mfma_f32_32x32x2f32 chains */
#define KVB_PEAK_EXP 3        /* v_exp_f32 results per second */
#define KVB_PEAK_VALU_FMA 4   /* v_fma_f32 lane operations per second */

/* Run the microbenchmark `kind` (KVB_PEAK_*) on the context's stream: one
 * warm-up launch, then the fastest of five timed launches (HIP events).
 * *rate_host = its rate (units above); *ms_host (or NULL) = that launch's
 * milliseconds. Allocates and frees its own device buffer (4 GiB for the copy,
 * 4 MiB otherwise): KVB_E_NOMEM if that fails. Synchronises the stream. */
int kvb_peak_probe(kvb_ctx ctx, int32_t kind, double* rate_host, double* ms_host);

#ifdef __cplusplus
}
#endif

#endif /* KVB_H */
