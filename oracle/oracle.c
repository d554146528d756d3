/*
 * FP64 CPU oracle for the per-rank, column-based (sparsity-aware) SpMM path
 * of SHIRO (distributed SpMM with a 1D row partition).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header
 * or constant with the GPU library and is never on the product path.
 *
 * Every routine is the plain definition of what the method computes, written
 * as simple loops, in double precision:
 *   - the 1D row partition and column blocks       (Sec. 2.2; Table 1: M, K)
 *   - Cols(A^(p,q)) as a sorted set                 (Table 1; Sec. 3.1, column-based scheme)
 *   - the packed rows of B for those columns        (Sec. 3.1 Eq. V_col; Sec. 5.1 stage 3)
 *   - the local product C = A B over packed rows,
 *     summed over all blocks of the panel           (Sec. 2.1; Sec. 2.2 stages 3-4; Sec. 5.1 stage 5)
 *   - the gradients of L = <G, A B>: A^T G and the
 *     sampled products G_i . b_j at the nonzeros    (not in the paper; needed by GNN
 *                                                    training, Sec. 7.6)
 *   - the row-based scheme: Rows(A^(p,q)) as sorted
 *     sets, the owner's partial C rows over them,
 *     and their sum into the panel's rows           (Table 1; Sec. 3.1 row-based scheme,
 *                                                    Eq. V_row; Sec. 5.1 stages 3 and 5)
 * No blocking, fusion or reordering beyond the definitions.  OpenMP splits
 * independent output rows (or independent output columns for the scatter)
 * across threads; the sum for every output element is taken in ascending
 * nonzero order, so the result does not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

int oracle_threads(void) { return omp_get_max_threads(); }

/* ---- 1D row partition (Sec. 2.2; Table 1) -------------------------------
 * Panel p of P holds rows [p*M, min(n_rows, (p+1)*M)) with M = ceil(n_rows/P).
 * Column block q holds columns [q*K, min(n_cols, (q+1)*K)), K = ceil(n_cols/P).
 */
void oracle_partition(int64_t n_rows, int64_t n_cols, int32_t P, int32_t p,
                      int64_t* row_begin, int64_t* row_end, int64_t* K_out) {
  int64_t M = (n_rows + P - 1) / P;
  int64_t K = (n_cols + P - 1) / P;
  int64_t b = (int64_t)p * M;
  int64_t e = b + M;
  if (b > n_rows) b = n_rows;
  if (e > n_rows) e = n_rows;
  *row_begin = b;
  *row_end = e;
  *K_out = K;
}

/* Nonzeros of the panel in each column block: block of column c is c / K. */
void oracle_block_nnz(const int64_t* row_ptr, const int32_t* col, int64_t row_begin,
                      int64_t row_end, int64_t K, int32_t P, int64_t* block_nnz) {
  for (int32_t q = 0; q < P; ++q) block_nnz[q] = 0;
  for (int64_t k = row_ptr[row_begin]; k < row_ptr[row_end]; ++k) block_nnz[col[k] / K] += 1;
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* ---- Cols(A^(p,q)) for every block q (Table 1; Sec. 3.1) ----------------
 * Cols_q is the set of column ids with at least one nonzero in block q,
 * listed in ascending order (a set has no order; ascending is the reading
 * taken).  unique_cols holds Cols_0, Cols_1, ... back to back; block_off is
 * the exclusive sum of |Cols_q| (P+1 entries).  colmap[k] is the position of
 * col[k] in that concatenation (panel nonzero k, counted from the panel's
 * first nonzero).  Returns U = sum_q |Cols_q|.
 */
int64_t oracle_select(const int64_t* row_ptr, const int32_t* col, int64_t row_begin,
                      int64_t row_end, int64_t K, int32_t P, int32_t* unique_cols,
                      int64_t* block_off, int32_t* colmap) {
  int64_t nz0 = row_ptr[row_begin], nz1 = row_ptr[row_end];
  int64_t nnz = nz1 - nz0;
  int64_t* cnt = (int64_t*)calloc((size_t)P + 1, sizeof(int64_t));
  for (int64_t k = nz0; k < nz1; ++k) cnt[col[k] / K + 1] += 1;
  for (int32_t q = 0; q < P; ++q) cnt[q + 1] += cnt[q];
  /* bucket the column ids of each block, then sort and drop repeats */
  int32_t* bucket = (int32_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
  int64_t* fill = (int64_t*)malloc((size_t)P * sizeof(int64_t));
  for (int32_t q = 0; q < P; ++q) fill[q] = cnt[q];
  for (int64_t k = nz0; k < nz1; ++k) bucket[fill[col[k] / K]++] = col[k];
  int64_t* usize = (int64_t*)calloc((size_t)P, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t q = 0; q < P; ++q) {
    int32_t* s = bucket + cnt[q];
    int64_t m = cnt[q + 1] - cnt[q];
    qsort(s, (size_t)m, sizeof(int32_t), cmp_i32);
    int64_t u = 0;
    for (int64_t i = 0; i < m; ++i)
      if (u == 0 || s[i] != s[u - 1]) s[u++] = s[i];
    usize[q] = u;
  }
  block_off[0] = 0;
  for (int32_t q = 0; q < P; ++q) block_off[q + 1] = block_off[q] + usize[q];
  for (int32_t q = 0; q < P; ++q)
    memcpy(unique_cols + block_off[q], bucket + cnt[q], (size_t)usize[q] * sizeof(int32_t));
  /* colmap by binary search of col[k] inside Cols_q */
#pragma omp parallel for schedule(static)
  for (int64_t k = nz0; k < nz1; ++k) {
    int64_t q = col[k] / K;
    int64_t lo = block_off[q], hi = block_off[q + 1];
    while (lo < hi) {
      int64_t mid = lo + (hi - lo) / 2;
      if (unique_cols[mid] < col[k]) lo = mid + 1; else hi = mid;
    }
    colmap[k - nz0] = (int32_t)lo;
  }
  int64_t U = block_off[P];
  free(cnt); free(bucket); free(fill); free(usize);
  return U;
}

/* ---- Pack (Sec. 3.1 column-based scheme; Sec. 5.1 stage 3) --------------
 * Bpacked[u, :] = B[unique_cols[u], :], an exact copy of elem_bytes-wide
 * elements (4 for float32, 2 for bfloat16).
 */
void oracle_pack(const void* B, int64_t ldb, int64_t N, int64_t elem_bytes,
                 const int32_t* unique_cols, int64_t U, void* Bpacked, int64_t ldp) {
#pragma omp parallel for schedule(static)
  for (int64_t u = 0; u < U; ++u)
    memcpy((char*)Bpacked + (size_t)(u * ldp * elem_bytes),
           (const char*)B + (size_t)((int64_t)unique_cols[u] * ldb * elem_bytes),
           (size_t)(N * elem_bytes));
}

/* ---- Local SpMM with aggregation (Sec. 2.1; Sec. 2.2 stages 3-4) --------
 * Y[i, j] = sum_k vals[k] * Bp[colmap[k], j] over the nonzeros k of panel row
 * i (all column blocks, ascending k), in double.  Y is (row_end-row_begin)xN.
 * With colmap = NULL the product is taken against the unpacked B rows:
 * Y[i, j] = sum_k vals[k] * B[col[k], j] (the definition C = A B itself).
 * abs_mode != 0 computes |A| |B| instead (the error-metric denominator).
 */
void oracle_spmm(const int64_t* row_ptr, const int32_t* col, const float* vals,
                 int64_t row_begin, int64_t row_end, const int32_t* colmap,
                 const float* Bsrc, int64_t ldb, int64_t N, double* Y, int64_t ldy,
                 int abs_mode) {
  int64_t nz0 = row_ptr[row_begin];
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = row_begin; i < row_end; ++i) {
    double* y = Y + (i - row_begin) * ldy;
    for (int64_t j = 0; j < N; ++j) y[j] = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      int64_t r = colmap ? (int64_t)colmap[k - nz0] : (int64_t)col[k];
      double a = (double)vals[k];
      const float* b = Bsrc + r * ldb;
      if (abs_mode) {
        a = fabs(a);
        for (int64_t j = 0; j < N; ++j) y[j] += a * fabs((double)b[j]);
      } else {
        for (int64_t j = 0; j < N; ++j) y[j] += a * b[j];
      }
    }
  }
}

/* The same definition for a list of panel rows (sampled checks at full size).
 * rows[s] is a panel-local row index; Y is nrows x N. */
void oracle_spmm_rows(const int64_t* row_ptr, const int32_t* col, const float* vals,
                      int64_t row_begin, const int64_t* rows, int64_t nrows,
                      const int32_t* colmap, const float* Bsrc, int64_t ldb, int64_t N,
                      double* Y, int64_t ldy, int abs_mode) {
  int64_t nz0 = row_ptr[row_begin];
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t s = 0; s < nrows; ++s) {
    int64_t i = row_begin + rows[s];
    double* y = Y + s * ldy;
    for (int64_t j = 0; j < N; ++j) y[j] = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      int64_t r = colmap ? (int64_t)colmap[k - nz0] : (int64_t)col[k];
      double a = abs_mode ? fabs((double)vals[k]) : (double)vals[k];
      const float* b = Bsrc + r * ldb;
      for (int64_t j = 0; j < N; ++j) y[j] += a * (abs_mode ? fabs((double)b[j]) : b[j]);
    }
  }
}

/* ---- Gradient of L = <G, A B> with respect to B -------------------------
 * dX[target(k), :] += vals[k] * G[i(k), :] for every panel nonzero k, i.e.
 * dX = A^T G, by scattering each nonzero (COO order).  target(k) is colmap[k]
 * (packed rows, dX is U x N) or col[k] when colmap is NULL (dX is n_cols x
 * N).  dX must be zeroed by the caller.  Threads own disjoint column slices
 * of dX, so each element sums in ascending k.  abs_mode: |A|^T |G|.
 */
void oracle_spmm_t(const int64_t* row_ptr, const int32_t* col, const float* vals,
                   int64_t row_begin, int64_t row_end, const int32_t* colmap,
                   const float* G, int64_t ldg, int64_t N, double* dX, int64_t ldx,
                   int abs_mode) {
  int64_t nz0 = row_ptr[row_begin];
#pragma omp parallel
  {
    int nt = omp_get_num_threads(), t = omp_get_thread_num();
    int64_t j0 = N * t / nt, j1 = N * (t + 1) / nt;
    for (int64_t i = row_begin; i < row_end; ++i) {
      const float* g = G + (i - row_begin) * ldg;
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        int64_t r = colmap ? (int64_t)colmap[k - nz0] : (int64_t)col[k];
        double a = abs_mode ? fabs((double)vals[k]) : (double)vals[k];
        double* x = dX + r * ldx;
        for (int64_t j = j0; j < j1; ++j) x[j] += a * (abs_mode ? fabs((double)g[j]) : g[j]);
      }
    }
  }
}

/* A^T G restricted to the packed rows listed in targets[0..nt) (sampled
 * checks at full size): out[s, :] = sum over k with colmap[k] == targets[s]
 * of vals[k] * G[i(k), :], ascending k.  slot[u] must be -1 or the index s
 * of u in targets (length U, prepared by the caller). */
void oracle_spmm_t_sampled(const int64_t* row_ptr, const float* vals, int64_t row_begin,
                           int64_t row_end, const int32_t* colmap, const int64_t* slot,
                           const float* G, int64_t ldg, int64_t N, double* out, int64_t ldo,
                           int abs_mode) {
  int64_t nz0 = row_ptr[row_begin];
#pragma omp parallel
  {
    int nt = omp_get_num_threads(), t = omp_get_thread_num();
    int64_t j0 = N * t / nt, j1 = N * (t + 1) / nt;
    for (int64_t i = row_begin; i < row_end; ++i) {
      const float* g = G + (i - row_begin) * ldg;
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        int64_t s = slot[colmap[k - nz0]];
        if (s < 0) continue;
        double a = abs_mode ? fabs((double)vals[k]) : (double)vals[k];
        double* x = out + s * ldo;
        for (int64_t j = j0; j < j1; ++j) x[j] += a * (abs_mode ? fabs((double)g[j]) : g[j]);
      }
    }
  }
}

/* ---- Gradient of L = <G, A B> with respect to the values ----------------
 * dvals[k] = sum_j G[i(k), j] * Bsrc[r(k), j]: the dense-dense product
 * G B^T sampled at the nonzeros of A.  r(k) = colmap[k] or col[k].
 * abs_mode: sum_j |G| |B| (the denominator of the error metric).
 */
void oracle_sddmm(const int64_t* row_ptr, const int32_t* col, int64_t row_begin,
                  int64_t row_end, const int32_t* colmap, const float* G, int64_t ldg,
                  const float* Bsrc, int64_t ldb, int64_t N, double* dvals, int abs_mode) {
  int64_t nz0 = row_ptr[row_begin];
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = row_begin; i < row_end; ++i) {
    const float* g = G + (i - row_begin) * ldg;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      int64_t r = colmap ? (int64_t)colmap[k - nz0] : (int64_t)col[k];
      const float* b = Bsrc + r * ldb;
      double s = 0.0;
      for (int64_t j = 0; j < N; ++j) s += abs_mode ? fabs((double)g[j]) * fabs((double)b[j]) : (double)g[j] * (double)b[j];
      dvals[k - nz0] = s;
    }
  }
}

/* ---- Rows(A^(p,q)) for every block q (Table 1; Sec. 3.1 row-based scheme) -
 * Rows_q is the set of panel rows (panel-local index i = global row -
 * row_begin) holding at least one nonzero in block q, listed ascending.
 * row_sel holds Rows_0, Rows_1, ... back to back; rblock_off is the
 * exclusive sum of |Rows_q| (P+1 entries).  Returns R = sum_q |Rows_q|.
 * last[q] remembers the last row added to Rows_q, so a row enters each set
 * once whatever the order of its nonzeros.
 */
int64_t oracle_select_c_rows(const int64_t* row_ptr, const int32_t* col, int64_t row_begin,
                             int64_t row_end, int64_t K, int32_t P, int32_t* row_sel,
                             int64_t* rblock_off) {
  int64_t* cnt = (int64_t*)calloc((size_t)P, sizeof(int64_t));
  int64_t* last = (int64_t*)malloc((size_t)P * sizeof(int64_t));
  for (int32_t q = 0; q < P; ++q) last[q] = -1;
  for (int64_t g = row_begin; g < row_end; ++g)
    for (int64_t k = row_ptr[g]; k < row_ptr[g + 1]; ++k) {
      int64_t q = col[k] / K;
      if (last[q] != g) {
        last[q] = g;
        cnt[q] += 1;
      }
    }
  rblock_off[0] = 0;
  for (int32_t q = 0; q < P; ++q) rblock_off[q + 1] = rblock_off[q] + cnt[q];
  for (int32_t q = 0; q < P; ++q) {
    last[q] = -1;
    cnt[q] = rblock_off[q];
  }
  for (int64_t g = row_begin; g < row_end; ++g)
    for (int64_t k = row_ptr[g]; k < row_ptr[g + 1]; ++k) {
      int64_t q = col[k] / K;
      if (last[q] != g) {
        last[q] = g;
        row_sel[cnt[q]++] = (int32_t)(g - row_begin);
      }
    }
  int64_t R = rblock_off[P];
  free(cnt);
  free(last);
  return R;
}

/* ---- Partial C rows computed by the owner (Sec. 3.1 row-based scheme;
 * Sec. 5.1 stage 3: the remote computation) --------------------------------
 * For entry e = rblock_off[q] + t (row i = Rows_q[t]):
 *   Cp[e, j] = sum over nonzeros k of panel row i with col[k] in block q of
 *              vals[k] * B[col[k], j],
 * ascending k, in double.  abs_mode != 0 computes |A| |B| instead.
 */
void oracle_partial_c(const int64_t* row_ptr, const int32_t* col, const float* vals,
                      int64_t row_begin, int64_t K, int32_t P, const int32_t* row_sel,
                      const int64_t* rblock_off, const float* B, int64_t ldb, int64_t N,
                      double* Cp, int64_t ldc, int abs_mode) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t q = 0; q < P; ++q) {
    for (int64_t e = rblock_off[q]; e < rblock_off[q + 1]; ++e) {
      double* c = Cp + e * ldc;
      for (int64_t j = 0; j < N; ++j) c[j] = 0.0;
      int64_t g = row_begin + row_sel[e];
      for (int64_t k = row_ptr[g]; k < row_ptr[g + 1]; ++k) {
        if (col[k] / K != q) continue;
        double a = (double)vals[k];
        const float* b = B + (int64_t)col[k] * ldb;
        if (abs_mode) {
          a = fabs(a);
          for (int64_t j = 0; j < N; ++j) c[j] += a * fabs((double)b[j]);
        } else {
          for (int64_t j = 0; j < N; ++j) c[j] += a * b[j];
        }
      }
    }
  }
}

/* ---- Aggregation on the receiver (Sec. 5.1 stage 5) ----------------------
 * Y[i, :] = sum over blocks q, ascending, of the partial row of i in block q:
 *   Y[Rows_q[t], :] += Cp[rblock_off[q] + t, :].
 * Rows in no Rows_q stay 0.  Y is M x N (panel rows), in double; the partial
 * rows are given in double (Cp) or, if Cp is NULL, in float (Cpf).
 */
void oracle_aggregate_c(int64_t M, int32_t P, const int32_t* row_sel, const int64_t* rblock_off,
                        const double* Cp, const float* Cpf, int64_t ldc, int64_t N, double* Y,
                        int64_t ldy) {
  for (int64_t i = 0; i < M; ++i)
    for (int64_t j = 0; j < N; ++j) Y[i * ldy + j] = 0.0;
  for (int32_t q = 0; q < P; ++q)
    for (int64_t e = rblock_off[q]; e < rblock_off[q + 1]; ++e) {
      double* y = Y + (int64_t)row_sel[e] * ldy;
      if (Cp) {
        for (int64_t j = 0; j < N; ++j) y[j] += Cp[e * ldc + j];
      } else {
        for (int64_t j = 0; j < N; ++j) y[j] += (double)Cpf[e * ldc + j];
      }
    }
}
