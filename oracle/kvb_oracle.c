/*
 * Plain FP64 CPU oracle for the sparse self-tuning variable-bandwidth kernel
 * matrix of Davis & Giannakis (arXiv 2104.15124).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously correct reference
 * that the HIP library is checked against. Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it. It shares no
 * code, header, table or helper with the HIP library.
 *
 * Every step follows the paper's definitions in their stated order, in double
 * precision, with inputs upcast from float32:
 *   knn          exact nearest neighbours (the "brute force" algorithm of
 *                Section 4, Algorithm 1; the neighbour ordering I(x, k) of
 *                Section 2.1 with the convention I(x^(i), 0) = i)
 *   adhoc_bw     b_i^2 = sum_{r=1..k0} |x_i - x_{I(x_i, r)}|^2   (Section 2.1, bandwidth eq.)
 *   chi          chi(e) = sum_ij K_ij, slope = d log chi / d log e,
 *                optimum = argmax slope, dimension = 2 max slope  (Section 2.3)
 *   density      psi_i = sum_j K_ij / (n (pi e b_i^2)^{d/2}),
 *                P_i = psi_i^beta, rho_i = 2 P_i      (Section 2.1 density eqs.; Algorithm 1 caption)
 *   normalize    K_ij = exp(-D2/(e rho_i rho_j)), q_i = P_i^{-d} sum_j K_ij,
 *                Kt_ij = K_ij/(q_i q_j)^alpha, D_i = sum_j Kt_ij,
 *                M = D^{-1} Kt, L = e^{-1} P^{-2} (M - I),
 *                Lhat = e^{-1} (S^{-1} Kt S^{-1} - P^{-2}), S = P D^{1/2}
 *                (Section 2.2, kernel, normaliser, Kolmogorov-matrix and
 *                symmetric-conjugate equations)
 *
 * Notation: e stands for the paper's epsilon^2 (it parameterises epsilon^2 =
 * 2^xi in Section 2.3); the density kernel uses rho = b and the operator kernel
 * uses rho = 2 psi^beta, which turns 4 epsilon^2 (psi_i psi_j)^beta into
 * e rho_i rho_j.
 *
 *   truncate     keep K_ij > delta_tol only (Section 4, Algorithm 1)
 *
 * The passes after the neighbour search take a general CSR pattern
 * (rowptr, col, dist2) so that the same code serves the directed k-NN
 * pattern, the symmetrised union pattern used by the spectral checks and
 * their threshold-truncated forms.
 *
 * Summations run in a fixed sequential order so results are reproducible.
 * OpenMP parallelises only over independent rows.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Squared Euclidean distance in double precision from float32 coordinates. */
static double dist2_f64(const float* a, const float* b, int32_t m)
{
    double s = 0.0;
    for (int32_t c = 0; c < m; ++c) {
        double t = (double)a[c] - (double)b[c];
        s += t * t;
    }
    return s;
}

/* (d, j) lexicographic order: distance first, index breaks ties. */
static int key_less(double da, int64_t ja, double db, int64_t jb)
{
    return da < db || (da == db && ja < jb);
}

/*
 * Exact k-NN of one row i against all n samples, on the calling thread: i
 * itself (distance 0), then the k-1 samples j != i first in (D2_ij, j) order,
 * kept in a bounded insertion list.
 */
static int oracle_knn_rows_serial(const float* X, int64_t n, int32_t m, int32_t k, int64_t i, int32_t* idx,
                                  double* d2)
{
    int32_t kk = k - 1;
    double* bd = (double*)malloc(sizeof(double) * (size_t)(kk > 0 ? kk : 1));
    int64_t* bj = (int64_t*)malloc(sizeof(int64_t) * (size_t)(kk > 0 ? kk : 1));
    if (!bd || !bj) {
        free(bd);
        free(bj);
        return ORC_ENOMEM;
    }
    const float* xi = X + (size_t)i * (size_t)m;
    int32_t cnt = 0;
    for (int64_t j = 0; j < n && kk > 0; ++j) {
        if (j == i) continue;
        double s = dist2_f64(xi, X + (size_t)j * (size_t)m, m);
        if (cnt < kk || key_less(s, j, bd[cnt - 1], bj[cnt - 1])) {
            int32_t p = (cnt < kk) ? cnt++ : cnt - 1;
            while (p > 0 && key_less(s, j, bd[p - 1], bj[p - 1])) {
                bd[p] = bd[p - 1];
                bj[p] = bj[p - 1];
                --p;
            }
            bd[p] = s;
            bj[p] = j;
        }
    }
    idx[0] = (int32_t)i;
    d2[0] = 0.0;
    for (int32_t r = 0; r < kk; ++r) {
        idx[1 + r] = (int32_t)bj[r];
        d2[1 + r] = bd[r];
    }
    free(bd);
    free(bj);
    return ORC_OK;
}

/*
 * Exact k-NN self-join over rows [row_begin, row_end) against all n samples.
 * Row i of the output holds i itself (distance 0) and then the k-1 samples
 * j != i that come first in the (D2_ij, j) order. A bounded insertion list
 * keeps the k-1 best seen so far; it is the first k-1 entries of the fully
 * sorted candidate list. Output rows are indexed from row_begin.
 */
int oracle_knn_rows(const float* X, int64_t n, int32_t m, int32_t k,
                    int64_t row_begin, int64_t row_end,
                    int32_t* idx, double* d2)
{
    if (!X || !idx || !d2 || n < 1 || m < 1 || k < 1 || k > n ||
        row_begin < 0 || row_end > n || row_begin > row_end)
        return ORC_EINVAL;
    int err = ORC_OK;
#pragma omp parallel
    {
        int32_t kk = k - 1;
        double* bd = (double*)malloc(sizeof(double) * (size_t)(kk > 0 ? kk : 1));
        int64_t* bj = (int64_t*)malloc(sizeof(int64_t) * (size_t)(kk > 0 ? kk : 1));
        if (!bd || !bj) {
#pragma omp atomic write
            err = ORC_ENOMEM;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = row_begin; i < row_end; ++i) {
            if (!bd || !bj) continue;
            const float* xi = X + (size_t)i * (size_t)m;
            int32_t cnt = 0;
            for (int64_t j = 0; j < n && kk > 0; ++j) {
                if (j == i) continue;
                double s = dist2_f64(xi, X + (size_t)j * (size_t)m, m);
                if (cnt < kk || key_less(s, j, bd[cnt - 1], bj[cnt - 1])) {
                    int32_t p = (cnt < kk) ? cnt++ : cnt - 1;
                    while (p > 0 && key_less(s, j, bd[p - 1], bj[p - 1])) {
                        bd[p] = bd[p - 1];
                        bj[p] = bj[p - 1];
                        --p;
                    }
                    bd[p] = s;
                    bj[p] = j;
                }
            }
            int64_t o = (i - row_begin) * (int64_t)k;
            idx[o] = (int32_t)i;
            d2[o] = 0.0;
            for (int32_t r = 0; r < kk; ++r) {
                idx[o + 1 + r] = (int32_t)bj[r];
                d2[o + 1 + r] = bd[r];
            }
        }
        free(bd);
        free(bj);
    }
    return err;
}

int oracle_knn(const float* X, int64_t n, int32_t m, int32_t k, int32_t* idx, double* d2)
{
    return oracle_knn_rows(X, n, m, k, 0, n, idx, d2);
}

/* Exact k-NN of the listed rows (any order, each in [0, n)) against all n
 * samples; output row t belongs to sample rows[t]. The same search as
 * oracle_knn_rows, one list row per thread. */
int oracle_knn_list(const float* X, int64_t n, int32_t m, int32_t k, const int64_t* rows, int64_t nrows,
                    int32_t* idx, double* d2)
{
    if (!X || !rows || !idx || !d2 || n < 1 || m < 1 || k < 1 || k > n || nrows < 0) return ORC_EINVAL;
    for (int64_t t = 0; t < nrows; ++t)
        if (rows[t] < 0 || rows[t] >= n) return ORC_EINVAL;
    int err = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nrows; ++t) {
        int rc = oracle_knn_rows_serial(X, n, m, k, rows[t], idx + t * (int64_t)k, d2 + t * (int64_t)k);
        if (rc != ORC_OK) {
#pragma omp atomic write
            err = rc;
        }
    }
    return err;
}

/* b_i = sqrt(sum_{r=1..k0} d2[i, r]) over the k-NN rows (self at r = 0 is skipped). */
int oracle_adhoc_bandwidth(const double* d2, int64_t n, int32_t k, int32_t k0, double* b)
{
    if (!d2 || !b || n < 1 || k0 < 1 || k0 >= k) return ORC_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t r = 1; r <= k0; ++r) s += d2[i * (int64_t)k + r];
        b[i] = sqrt(s);
    }
    return ORC_OK;
}

/* Logarithmic grid e_g = exp(ln e_min + g (ln e_max - ln e_min)/(G-1)). */
static double grid_value(double e_min, double e_max, int32_t G, int32_t g)
{
    double lo = log(e_min), hi = log(e_max);
    return exp(lo + (double)g * (hi - lo) / (double)(G - 1));
}

/*
 * Bandwidth self-tuning (Section 2.3). chi[g] = sum over stored (i, j) of
 * exp(-D2_ij / (e_g rho_i rho_j)); slope[g] = (ln chi[g+1] - ln chi[g]) /
 * (ln e_{g+1} - ln e_g) for g = 0..G-2; the optimum is the first g that
 * maximises slope; the intrinsic-dimension estimate is 2 slope[g*].
 * Returns 1 when the optimum sits on the grid edge (g* = 0 or G-2), else 0.
 */
int oracle_chi(const int64_t* rowptr, const int32_t* col, const double* dist2,
               const double* rho, int64_t n, double e_min, double e_max, int32_t G,
               double* chi, double* e_grid, double* slope,
               int32_t* g_star, double* e_star, double* dim)
{
    if (!rowptr || !col || !dist2 || !rho || !chi || n < 1 || G < 3 ||
        !(e_min > 0.0) || !(e_max > e_min))
        return ORC_EINVAL;
    double* rowpart = (double*)malloc(sizeof(double) * (size_t)n);
    if (!rowpart) return ORC_ENOMEM;
    for (int32_t g = 0; g < G; ++g) {
        double e = grid_value(e_min, e_max, G, g);
        if (e_grid) e_grid[g] = e;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
                s += exp(-dist2[p] / (e * rho[i] * rho[col[p]]));
            rowpart[i] = s;
        }
        double tot = 0.0;
        for (int64_t i = 0; i < n; ++i) tot += rowpart[i];
        chi[g] = tot;
    }
    free(rowpart);
    int32_t best = 0;
    double best_s = -INFINITY;
    for (int32_t g = 0; g + 1 < G; ++g) {
        double el = grid_value(e_min, e_max, G, g), er = grid_value(e_min, e_max, G, g + 1);
        double s = (log(chi[g + 1]) - log(chi[g])) / (log(er) - log(el));
        if (slope) slope[g] = s;
        if (s > best_s) {
            best_s = s;
            best = g;
        }
    }
    if (g_star) *g_star = best;
    if (e_star) *e_star = grid_value(e_min, e_max, G, best);
    if (dim) *dim = 2.0 * best_s;
    return (best == 0 || best == G - 2) ? 1 : 0;
}

/*
 * Density estimate (Section 2.1) and operator bandwidth (Algorithm 1 caption):
 * psi_i = sum_j exp(-D2_ij/(e b_i b_j)) / (n (pi e b_i^2)^{d/2}),
 * P_i = psi_i^beta, rho_i = 2 P_i. n is the total number of samples.
 */
int oracle_density(const int64_t* rowptr, const int32_t* col, const double* dist2,
                   const double* b, int64_t n, double e, double d, double beta,
                   double* psi, double* rho)
{
    if (!rowptr || !col || !dist2 || !b || !psi || !rho || n < 1 || !(e > 0.0) || !(d > 0.0))
        return ORC_EINVAL;
    const double pi = 3.14159265358979323846;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            s += exp(-dist2[p] / (e * b[i] * b[col[p]]));
        double w = (double)n * pow(pi * e * b[i] * b[i], 0.5 * d);
        psi[i] = s / w;
        rho[i] = 2.0 * pow(psi[i], beta);
    }
    return ORC_OK;
}

/*
 * Power-of-two rescaling of the operator-stage epsilon grid:
 * s = 2^round(log2(gm(ref^2) / gm(rho^2))), gm = geometric mean over i.
 * The Kolmogorov matrix is invariant under psi -> c psi with e -> e c^{-2 beta},
 * so the scale only moves the grid to where the operator kernel lives.
 */
double oracle_grid_scale(const double* ref, const double* rho, int64_t n)
{
    double a = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        a += log(ref[i]);
        c += log(rho[i]);
    }
    double l2 = 2.0 * (a - c) / (double)n / log(2.0);
    return ldexp(1.0, (int)round(l2));
}

/*
 * Operator normalisation (Section 2.2) over a CSR pattern whose distances are
 * dist2. Outputs, per stored entry p of row i with column j:
 *   out_kind 0: M_ij   = Kt_ij / D_i                       (Markov matrix D^{-1} Kt)
 *   out_kind 1: L_ij   = (M_ij - [i == j]) / (e P_i^2)      (discrete Kolmogorov matrix)
 *   out_kind 2: Lhat_ij = (Kt_ij/(S_i S_j) - [i == j]/P_i^2)/e  (symmetric conjugate)
 * with K_ij = exp(-D2_ij/(e rho_i rho_j)), P_i = rho_i/2, q_i = P_i^{-d} sum_j K_ij,
 * Kt_ij = K_ij/(q_i q_j)^alpha, D_i = sum_j Kt_ij, S_i = P_i sqrt(D_i).
 * q, P, D (length n) are returned when non-null.
 */
int oracle_normalize(const int64_t* rowptr, const int32_t* col, const double* dist2,
                     const double* rho, int64_t n, double e, double alpha, double d,
                     int32_t out_kind, double* val, double* q_out, double* P_out,
                     double* D_out)
{
    if (!rowptr || !col || !dist2 || !rho || !val || n < 1 || !(e > 0.0) ||
        out_kind < 0 || out_kind > 2)
        return ORC_EINVAL;
    double* q = (double*)malloc(sizeof(double) * (size_t)n);
    double* P = (double*)malloc(sizeof(double) * (size_t)n);
    double* D = (double*)malloc(sizeof(double) * (size_t)n);
    if (!q || !P || !D) {
        free(q); free(P); free(D);
        return ORC_ENOMEM;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        P[i] = 0.5 * rho[i];
        double s = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            s += exp(-dist2[p] / (e * rho[i] * rho[col[p]]));
        q[i] = pow(P[i], -d) * s;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int32_t j = col[p];
            double K = exp(-dist2[p] / (e * rho[i] * rho[j]));
            double Kt = K / pow(q[i] * q[j], alpha);
            val[p] = Kt;
            s += Kt;
        }
        D[i] = s;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int32_t j = col[p];
            double Kt = val[p];
            double v;
            if (out_kind == 0) {
                v = Kt / D[i];
            } else if (out_kind == 1) {
                v = (Kt / D[i] - (j == i ? 1.0 : 0.0)) / (e * P[i] * P[i]);
            } else {
                double Si = P[i] * sqrt(D[i]), Sj = P[j] * sqrt(D[j]);
                v = (Kt / (Si * Sj) - (j == i ? 1.0 / (P[i] * P[i]) : 0.0)) / e;
            }
            val[p] = v;
        }
    }
    if (q_out) memcpy(q_out, q, sizeof(double) * (size_t)n);
    if (P_out) memcpy(P_out, P, sizeof(double) * (size_t)n);
    if (D_out) memcpy(D_out, D, sizeof(double) * (size_t)n);
    free(q); free(P); free(D);
    return ORC_OK;
}

/*
 * Threshold truncation (Section 4: Algorithm 1 and the k-d tree algorithm
 * store an entry only when its kernel value exceeds the sparsity tolerance
 * delta_tol). Entry (i, j) of the pattern is kept when
 * K_ij = exp(-D2_ij / (e rho_i rho_j)) > delta, 0 < delta < 1, evaluated as
 * written, in double precision. Kept entries keep their order; rowptr_out
 * (length n + 1) and the kept columns and distances are written. *nnz_out
 * receives rowptr_out[n].
 */
int oracle_truncate(const int64_t* rowptr, const int32_t* col, const double* dist2, const double* rho, int64_t n,
                    double e, double delta, int64_t* rowptr_out, int32_t* col_out, double* dist2_out,
                    int64_t* nnz_out)
{
    if (!rowptr || !col || !dist2 || !rho || !rowptr_out || !col_out || !dist2_out || n < 1 || !(e > 0.0) ||
        !(delta > 0.0 && delta < 1.0))
        return ORC_EINVAL;
    int64_t out = 0;
    for (int64_t i = 0; i < n; ++i) {
        rowptr_out[i] = out;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            const double K = exp(-dist2[p] / (e * rho[i] * rho[col[p]]));
            if (K > delta) {
                col_out[out] = col[p];
                dist2_out[out] = dist2[p];
                ++out;
            }
        }
    }
    rowptr_out[n] = out;
    if (nnz_out) *nnz_out = out;
    return ORC_OK;
}

/*
 * Reorder every row of a fixed-width pattern (k entries per row) so that
 * columns ascend; values move with their columns. Used to lay the k-NN
 * pattern out as CSR.
 */
int oracle_sort_rows_by_col(int64_t n, int32_t k, int32_t* col, double* val)
{
    if (!col || !val || n < 0 || k < 1) return ORC_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int32_t* c = col + i * (int64_t)k;
        double* v = val + i * (int64_t)k;
        for (int32_t a = 1; a < k; ++a) {
            int32_t cc = c[a];
            double vv = v[a];
            int32_t b = a;
            while (b > 0 && c[b - 1] > cc) {
                c[b] = c[b - 1];
                v[b] = v[b - 1];
                --b;
            }
            c[b] = cc;
            v[b] = vv;
        }
    }
    return ORC_OK;
}
