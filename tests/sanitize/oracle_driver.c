/* Host driver of the FP64 oracle (oracle/oracle.c), built with the address
 * and undefined-behaviour sanitizers by tests/test_sanitizers.py.  Runs every
 * oracle function on random small CSR panels (ragged P, empty rows, empty
 * blocks) and checks the results against dense products and set scans done
 * here, so that out-of-bounds accesses and undefined behaviour in any of them
 * are reported.  Exit status 0 = every check passed. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_threads(void);
void oracle_partition(int64_t, int64_t, int32_t, int32_t, int64_t*, int64_t*, int64_t*);
void oracle_block_nnz(const int64_t*, const int32_t*, int64_t, int64_t, int64_t, int32_t, int64_t*);
int64_t oracle_select(const int64_t*, const int32_t*, int64_t, int64_t, int64_t, int32_t, int32_t*, int64_t*, int32_t*);
void oracle_pack(const void*, int64_t, int64_t, int64_t, const int32_t*, int64_t, void*, int64_t);
void oracle_spmm(const int64_t*, const int32_t*, const float*, int64_t, int64_t, const int32_t*, const float*,
                 int64_t, int64_t, double*, int64_t, int);
void oracle_spmm_rows(const int64_t*, const int32_t*, const float*, int64_t, const int64_t*, int64_t,
                      const int32_t*, const float*, int64_t, int64_t, double*, int64_t, int);
void oracle_spmm_t(const int64_t*, const int32_t*, const float*, int64_t, int64_t, const int32_t*, const float*,
                   int64_t, int64_t, double*, int64_t, int);
void oracle_spmm_t_sampled(const int64_t*, const float*, int64_t, int64_t, const int32_t*, const int64_t*,
                           const float*, int64_t, int64_t, double*, int64_t, int);
void oracle_sddmm(const int64_t*, const int32_t*, int64_t, int64_t, const int32_t*, const float*, int64_t,
                  const float*, int64_t, int64_t, double*, int);
int64_t oracle_select_c_rows(const int64_t*, const int32_t*, int64_t, int64_t, int64_t, int32_t, int32_t*, int64_t*);
void oracle_partial_c(const int64_t*, const int32_t*, const float*, int64_t, int64_t, int32_t,
                      const int32_t*, const int64_t*, const float*, int64_t, int64_t, double*, int64_t, int);
void oracle_aggregate_c(int64_t, int32_t, const int32_t*, const int64_t*, const double*, const float*,
                        int64_t, int64_t, double*, int64_t);

static int fails = 0;
#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);      \
      ++fails;                                                            \
    }                                                                     \
  } while (0)

static uint64_t st = 88172645463325252ull;
static uint64_t rnd(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return st; }
static int close_to(double a, double b) { return fabs(a - b) <= 1e-9 * (1.0 + fabs(b)); }

int main(void) {
  for (int trial = 0; trial < 60; ++trial) {
    const int64_t n_rows = 1 + (int64_t)(rnd() % 40), n_cols = 1 + (int64_t)(rnd() % 40);
    const int32_t P = 1 + (int32_t)(rnd() % 6), p = (int32_t)(rnd() % P);
    const int64_t N = 1 + (int64_t)(rnd() % 5);
    /* dense pattern with empty rows and an empty column range */
    double* A = calloc((size_t)(n_rows * n_cols), sizeof(double));
    const int64_t hole = (int64_t)(rnd() % n_cols);
    for (int64_t i = 0; i < n_rows; ++i)
      for (int64_t j = 0; j < n_cols; ++j)
        if (i % 5 != 3 && j != hole && rnd() % 4 == 0) A[i * n_cols + j] = (double)(int)(rnd() % 7) - 3.0 + 0.5;
    int64_t* rp = malloc((size_t)(n_rows + 1) * sizeof(int64_t));
    int64_t nnz = 0;
    rp[0] = 0;
    for (int64_t i = 0; i < n_rows; ++i) {
      for (int64_t j = 0; j < n_cols; ++j) nnz += A[i * n_cols + j] != 0.0;
      rp[i + 1] = nnz;
    }
    int32_t* col = malloc((size_t)(nnz ? nnz : 1) * sizeof(int32_t));
    float* vals = malloc((size_t)(nnz ? nnz : 1) * sizeof(float));
    int64_t k = 0;
    for (int64_t i = 0; i < n_rows; ++i)
      for (int64_t j = 0; j < n_cols; ++j)
        if (A[i * n_cols + j] != 0.0) { col[k] = (int32_t)j; vals[k] = (float)A[i * n_cols + j]; ++k; }
    float* B = malloc((size_t)(n_cols * N) * sizeof(float));
    float* G = malloc((size_t)(n_rows * N) * sizeof(float));
    for (int64_t i = 0; i < n_cols * N; ++i) B[i] = (float)((int)(rnd() % 9) - 4) * 0.25f;
    for (int64_t i = 0; i < n_rows * N; ++i) G[i] = (float)((int)(rnd() % 9) - 4) * 0.25f;

    int64_t rb, re, K;
    oracle_partition(n_rows, n_cols, P, p, &rb, &re, &K);
    const int64_t M = re - rb, nz0 = rp[rb], pn = rp[re] - nz0;
    int64_t* bn = calloc((size_t)P, sizeof(int64_t));
    oracle_block_nnz(rp, col, rb, re, K, P, bn);
    int64_t sum = 0;
    for (int32_t q = 0; q < P; ++q) sum += bn[q];
    CHECK(sum == pn);
    int32_t* uc = malloc((size_t)(pn ? pn : 1) * sizeof(int32_t));
    int64_t* off = malloc((size_t)(P + 1) * sizeof(int64_t));
    int32_t* cm = malloc((size_t)(pn ? pn : 1) * sizeof(int32_t));
    const int64_t U = oracle_select(rp, col, rb, re, K, P, uc, off, cm);
    CHECK(off[P] == U);
    for (int64_t t = 0; t < pn; ++t) CHECK(uc[cm[t]] == col[nz0 + t]);
    for (int64_t u = 1; u < U; ++u) CHECK(uc[u] > uc[u - 1]);
    /* pack, then every product against the dense definition */
    float* Bp = malloc((size_t)((U ? U : 1) * N) * sizeof(float));
    oracle_pack(B, N, N, 4, uc, U, Bp, N);
    for (int64_t u = 0; u < U; ++u) CHECK(memcmp(Bp + u * N, B + (int64_t)uc[u] * N, (size_t)N * 4) == 0);
    double* Y = malloc((size_t)((M ? M : 1) * N) * sizeof(double));
    double* Y2 = malloc((size_t)((M ? M : 1) * N) * sizeof(double));
    oracle_spmm(rp, col, vals, rb, re, cm, Bp, N, N, Y, N, 0);
    oracle_spmm(rp, col, vals, rb, re, NULL, B, N, N, Y2, N, 0);
    for (int64_t i = 0; i < M; ++i)
      for (int64_t j = 0; j < N; ++j) {
        double d = 0;
        for (int64_t c = 0; c < n_cols; ++c) d += A[(rb + i) * n_cols + c] * B[c * N + j];
        CHECK(close_to(Y[i * N + j], d));
        CHECK(Y2[i * N + j] == Y[i * N + j]);
      }
    int64_t* rows = malloc((size_t)(M ? M : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < M; ++i) rows[i] = M - 1 - i;
    oracle_spmm_rows(rp, col, vals, rb, rows, M, cm, Bp, N, N, Y2, N, 0);
    for (int64_t i = 0; i < M; ++i)
      for (int64_t j = 0; j < N; ++j) CHECK(Y2[i * N + j] == Y[(M - 1 - i) * N + j]);
    double* dBp = calloc((size_t)((U ? U : 1) * N), sizeof(double));
    oracle_spmm_t(rp, col, vals, rb, re, cm, G + 0, N, N, dBp, N, 0);
    for (int64_t u = 0; u < U; ++u)
      for (int64_t j = 0; j < N; ++j) {
        double d = 0;
        for (int64_t i = 0; i < M; ++i) d += A[(rb + i) * n_cols + uc[u]] * G[i * N + j];
        CHECK(close_to(dBp[u * N + j], d));
      }
    int64_t* slot = malloc((size_t)(U ? U : 1) * sizeof(int64_t));
    for (int64_t u = 0; u < U; ++u) slot[u] = (u % 2 == 0) ? u / 2 : -1;
    double* samp = calloc((size_t)(((U + 1) / 2 + 1) * N), sizeof(double));
    oracle_spmm_t_sampled(rp, vals, rb, re, cm, slot, G, N, N, samp, N, 0);
    for (int64_t u = 0; u < U; u += 2)
      for (int64_t j = 0; j < N; ++j) CHECK(close_to(samp[(u / 2) * N + j], dBp[u * N + j]));
    double* dv = malloc((size_t)(pn ? pn : 1) * sizeof(double));
    oracle_sddmm(rp, col, rb, re, cm, G, N, Bp, N, N, dv, 0);
    for (int64_t i = 0; i < M; ++i)
      for (int64_t t = rp[rb + i]; t < rp[rb + i + 1]; ++t) {
        double d = 0;
        for (int64_t j = 0; j < N; ++j) d += (double)G[i * N + j] * B[(int64_t)col[t] * N + j];
        CHECK(close_to(dv[t - nz0], d));
      }
    /* row-based scheme: partial rows summed back give Y */
    int32_t* rs = malloc((size_t)(pn ? pn : 1) * sizeof(int32_t));
    int64_t* roff = malloc((size_t)(P + 1) * sizeof(int64_t));
    const int64_t R = oracle_select_c_rows(rp, col, rb, re, K, P, rs, roff);
    CHECK(roff[P] == R);
    double* Cp = malloc((size_t)((R ? R : 1) * N) * sizeof(double));
    oracle_partial_c(rp, col, vals, rb, K, P, rs, roff, B, N, N, Cp, N, 0);
    oracle_aggregate_c(M, P, rs, roff, Cp, NULL, N, N, Y2, N);
    for (int64_t i = 0; i < M * N; ++i) CHECK(close_to(Y2[i], Y[i]));
    free(A); free(rp); free(col); free(vals); free(B); free(G); free(bn); free(uc); free(off); free(cm);
    free(Bp); free(Y); free(Y2); free(rows); free(dBp); free(slot); free(samp); free(dv); free(rs); free(roff);
    free(Cp);
  }
  printf("oracle driver (%d threads): %d failed checks\n", oracle_threads(), fails);
  return fails ? 1 : 0;
}
