/*
 * Runs every entry of the FP64 oracle (oracle/kvb_oracle.c) on small inputs
 * with known answers, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py compiles and runs
 * it on the CPU). Each check restates a closed form of the method:
 *   chain x_i = (i, 0, 0): row i = i, i-1, i+1, i-2, ... (ties by index);
 *   b_i^2 = 2 (1 + 4 + 9 + 16) = 60 for interior rows (Section 2.1, bandwidth eq.);
 *   Markov rows sum to 1 and L 1 = 0 (Section 2.2);
 *   truncation keeps the entries above delta, the diagonal always (Section 4);
 *   the grid scale of b = [1, 4], rho = [1, 1] is 4.
 * Exit status 0 when every check holds; the sanitizers abort on any fault.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_knn_rows(const float*, int64_t, int32_t, int32_t, int64_t, int64_t, int32_t*, double*);
int oracle_knn(const float*, int64_t, int32_t, int32_t, int32_t*, double*);
int oracle_knn_list(const float*, int64_t, int32_t, int32_t, const int64_t*, int64_t, int32_t*, double*);
int oracle_adhoc_bandwidth(const double*, int64_t, int32_t, int32_t, double*);
int oracle_chi(const int64_t*, const int32_t*, const double*, const double*, int64_t, double, double, int32_t,
               double*, double*, double*, int32_t*, double*, double*);
int oracle_density(const int64_t*, const int32_t*, const double*, const double*, int64_t, double, double, double,
                   double*, double*);
double oracle_grid_scale(const double*, const double*, int64_t);
int oracle_normalize(const int64_t*, const int32_t*, const double*, const double*, int64_t, double, double, double,
                     int32_t, double*, double*, double*, double*);
int oracle_truncate(const int64_t*, const int32_t*, const double*, const double*, int64_t, double, double, int64_t*,
                    int32_t*, double*, int64_t*);
int oracle_sort_rows_by_col(int64_t, int32_t, int32_t*, double*);

static int failures = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++failures;                                            \
        }                                                          \
    } while (0)

int main(void)
{
    enum { N = 40, M = 3, K = 9, K0 = 8, G = 16 };
    float* X = calloc((size_t)N * M, sizeof(float));
    int32_t* idx = malloc(sizeof(int32_t) * N * K);
    double* d2 = malloc(sizeof(double) * N * K);
    for (int i = 0; i < N; ++i) X[i * M] = (float)i;
    CHECK(oracle_knn(X, N, M, K, idx, d2) == 0);
    const int i = 20;
    const int want[K] = {20, 19, 21, 18, 22, 17, 23, 16, 24};
    for (int r = 0; r < K; ++r) CHECK(idx[i * K + r] == want[r]);
    CHECK(idx[0] == 0 && idx[1] == 1 && idx[K - 1] == 8);
    /* the same rows through the row-range and row-list forms */
    int32_t idx2[2 * K];
    double d22[2 * K];
    int64_t rows[2] = {i, 0};
    CHECK(oracle_knn_list(X, N, M, K, rows, 2, idx2, d22) == 0);
    for (int r = 0; r < K; ++r) CHECK(idx2[r] == idx[i * K + r] && idx2[K + r] == idx[r]);
    CHECK(oracle_knn_rows(X, N, M, K, i, i + 1, idx2, d22) == 0 && idx2[2] == 21);
    int64_t bad_rows[1] = {N};
    CHECK(oracle_knn_list(X, N, M, K, bad_rows, 1, idx2, d22) < 0);
    CHECK(oracle_knn(X, N, M, N + 1, idx, d2) < 0);

    double* b = malloc(sizeof(double) * N);
    CHECK(oracle_adhoc_bandwidth(d2, N, K, K0, b) == 0);
    CHECK(fabs(b[i] * b[i] - 60.0) < 1e-12);
    CHECK(fabs(b[0] * b[0] - 204.0) < 1e-12);
    CHECK(oracle_adhoc_bandwidth(d2, N, K, K, b) < 0);

    int64_t* rowptr = malloc(sizeof(int64_t) * (N + 1));
    for (int r = 0; r <= N; ++r) rowptr[r] = (int64_t)r * K;
    double chi[G], eg[G], slope[G];
    int32_t gs = -1;
    double es = 0.0, dim = 0.0;
    CHECK(oracle_chi(rowptr, idx, d2, b, N, 1e-3, 1e1, G, chi, eg, slope, &gs, &es, &dim) >= 0);
    CHECK(gs >= 0 && gs <= G - 2 && es == eg[gs] && dim == 2.0 * slope[gs]);
    for (int g = 1; g < G; ++g) CHECK(chi[g] >= chi[g - 1]);
    CHECK(chi[0] >= N && chi[G - 1] <= (double)N * K);
    CHECK(oracle_chi(rowptr, idx, d2, b, N, 1.0, 0.5, G, chi, eg, slope, &gs, &es, &dim) < 0);

    double* psi = malloc(sizeof(double) * N);
    double* rho = malloc(sizeof(double) * N);
    CHECK(oracle_density(rowptr, idx, d2, b, N, es, 1.0, -0.5, psi, rho) == 0);
    for (int r = 0; r < N; ++r) CHECK(psi[r] > 0.0 && fabs(rho[r] - 2.0 / sqrt(psi[r])) < 1e-12 * rho[r]);

    double one4[2] = {1.0, 4.0}, ones[2] = {1.0, 1.0};
    CHECK(oracle_grid_scale(one4, ones, 2) == 4.0);

    double* val = malloc(sizeof(double) * N * K);
    double *q = malloc(sizeof(double) * N), *P = malloc(sizeof(double) * N), *D = malloc(sizeof(double) * N);
    for (int kind = 0; kind < 3; ++kind) {
        CHECK(oracle_normalize(rowptr, idx, d2, rho, N, 0.5, -0.25, 1.0, kind, val, q, P, D) == 0);
        for (int r = 0; r < N; ++r) {
            double s = 0.0;
            for (int p = r * K; p < (r + 1) * K; ++p) s += val[p];
            if (kind == 0) CHECK(fabs(s - 1.0) < 1e-13);
            if (kind == 1) CHECK(fabs(s) < 1e-9 * (1.0 + fabs(val[r * K])));
        }
    }
    CHECK(oracle_normalize(rowptr, idx, d2, rho, N, 0.5, -0.25, 1.0, 3, val, q, P, D) < 0);

    int64_t* rp2 = malloc(sizeof(int64_t) * (N + 1));
    int32_t* c2 = malloc(sizeof(int32_t) * N * K);
    double* dd2 = malloc(sizeof(double) * N * K);
    int64_t nnz = -1;
    CHECK(oracle_truncate(rowptr, idx, d2, rho, N, 0.5, 1e-2, rp2, c2, dd2, &nnz) == 0);
    CHECK(nnz == rp2[N] && nnz >= N && nnz <= (int64_t)N * K);
    for (int r = 0; r < N; ++r) CHECK(rp2[r + 1] > rp2[r] && c2[rp2[r]] == r);
    CHECK(oracle_truncate(rowptr, idx, d2, rho, N, 0.5, 1.0, rp2, c2, dd2, &nnz) < 0);

    CHECK(oracle_sort_rows_by_col(N, K, idx, val) == 0);
    for (int r = 0; r < N; ++r)
        for (int p = r * K + 1; p < (r + 1) * K; ++p) CHECK(idx[p] > idx[p - 1]);

    free(X); free(idx); free(d2); free(b); free(rowptr); free(psi); free(rho); free(val); free(q); free(P);
    free(D); free(rp2); free(c2); free(dd2);
    if (failures) fprintf(stderr, "%d checks failed\n", failures);
    else printf("oracle sanitized run: all checks passed\n");
    return failures ? 1 : 0;
}
