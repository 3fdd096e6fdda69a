/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, obviously correct CPU implementation of the exact sparse
 * products over Z/mZ. Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the library never does. It shares no
 * code, header or table with the GPU path.
 *
 * What it computes follows the paper's problem statement:
 *  - residues are represented on [0, m-1] (Section 2.2, "Finite field
 *    representation"); raw input values are mapped there by canon();
 *  - the matrix is given in CSR form, start/colid/data (Section 2.1,
 *    "Sparse Matrix Formats and Multiplication"); duplicate coordinates
 *    simply add, as the loops below visit every stored entry;
 *  - y <- alpha*A*x + beta*y, the apply y <- A*x (alpha=1, beta=0), and the
 *    block form Y <- alpha*A*X + beta*Y (Section 2, opening paragraph);
 *  - the transpose product A^T*x (Section 1 and Section 4);
 *  - the power A^k*V and the projected sequence S_i = U^T A^i V of block
 *    Wiedemann's first step (Section 2.5 "Performance issues", Section 3
 *    step 1, Section 3.1).
 *
 * Every multiply-add is followed by a reduction modulo m, which is the
 * right-hand loop of the paper's Section 2.2 example: no delayed
 * reduction, no blocking, no reordering. Requirements: 2 <= m < 2^31 and
 * every vector entry, alpha and beta already in [0, m-1]; then each
 * intermediate below is < 2^63.
 *
 * Multi-vectors are n x s, row j holding its s residues contiguously with
 * leading dimension ld >= s (the layout Section 2.5 describes as traversing
 * A once with x and y read and written contiguously).
 *
 * Threads: built plainly it runs on one thread; built with -fopenmp (liboracle_omp.so) the
 * rows of a product run on all cores, with identical results.
 *
 * Return value of each entry point: 0 on success, -1 on invalid arguments
 * (modulus out of range, a vector entry not canonical, a column index out
 * of range, a null pointer).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef int64_t i64;
typedef uint64_t u64;

/* the representative of v in [0, m-1] */
static u64 canon(i64 v, u64 m) {
  i64 r = v % (i64)m;
  if (r < 0) r += (i64)m;
  return (u64)r;
}

static int bad_modulus(u64 m) { return m < 2 || m > 2147483647ULL; }

static int check_vec(const i64* v, i64 rows, i64 s, i64 ld, u64 m) {
  for (i64 i = 0; i < rows; ++i)
    for (i64 b = 0; b < s; ++b)
      if (v[i * ld + b] < 0 || (u64)v[i * ld + b] >= m) return -1;
  return 0;
}

static int check_csr(i64 nrows, i64 ncols, const i64* rowptr, const int32_t* col) {
  if (nrows < 0 || ncols < 0 || !rowptr) return -1;
  for (i64 i = 0; i < nrows; ++i) {
    if (rowptr[i + 1] < rowptr[i]) return -1;
    for (i64 k = rowptr[i]; k < rowptr[i + 1]; ++k)
      if (col[k] < 0 || col[k] >= ncols) return -1;
  }
  return 0;
}

/* Y <- alpha*A*X + beta*Y with X: ncols x s (ldx), Y: nrows x s (ldy) */
int oracle_spmm(i64 nrows, i64 ncols, const i64* rowptr, const int32_t* col, const i64* val, u64 m, i64 s,
                u64 alpha, const i64* X, i64 ldx, u64 beta, i64* Y, i64 ldy) {
  if (bad_modulus(m) || alpha >= m || beta >= m || s < 1 || ldx < s || ldy < s) return -1;
  if (check_csr(nrows, ncols, rowptr, col)) return -1;
  if (check_vec(X, ncols, s, ldx, m) || check_vec(Y, nrows, s, ldy, m)) return -1;
  /* rows are independent: the all-cores build (-fopenmp) splits them over threads; the result is the
     same, and the single-thread build ignores the pragma */
#pragma omp parallel for schedule(dynamic, 1024)
  for (i64 i = 0; i < nrows; ++i) {
    for (i64 b = 0; b < s; ++b) {
      u64 acc = 0;
      for (i64 k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        u64 a = canon(val[k], m);
        u64 xv = (u64)X[(i64)col[k] * ldx + b];
        acc = (acc + a * xv) % m;
      }
      u64 yv = (u64)Y[i * ldy + b];
      Y[i * ldy + b] = (i64)((alpha * acc % m + beta * yv % m) % m);
    }
  }
  return 0;
}

/* y <- alpha*A*x + beta*y */
int oracle_spmv(i64 nrows, i64 ncols, const i64* rowptr, const int32_t* col, const i64* val, u64 m,
                u64 alpha, const i64* x, u64 beta, i64* y) {
  return oracle_spmm(nrows, ncols, rowptr, col, val, m, 1, alpha, x, 1, beta, y, 1);
}

/* Y <- alpha*A^T*X + beta*Y with X: nrows x s (ldx), Y: ncols x s (ldy).
 * Entry A[i,j] contributes A[i,j]*X[i] to output row j. */
int oracle_spmm_t(i64 nrows, i64 ncols, const i64* rowptr, const int32_t* col, const i64* val, u64 m, i64 s,
                  u64 alpha, const i64* X, i64 ldx, u64 beta, i64* Y, i64 ldy) {
  if (bad_modulus(m) || alpha >= m || beta >= m || s < 1 || ldx < s || ldy < s) return -1;
  if (check_csr(nrows, ncols, rowptr, col)) return -1;
  if (check_vec(X, nrows, s, ldx, m) || check_vec(Y, ncols, s, ldy, m)) return -1;
  u64* acc = (u64*)calloc((size_t)(ncols > 0 ? ncols : 1) * (size_t)s, sizeof(u64));
  if (!acc) return -1;
  for (i64 i = 0; i < nrows; ++i) {
    for (i64 k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      u64 a = canon(val[k], m);
      i64 j = col[k];
      for (i64 b = 0; b < s; ++b) {
        u64 xv = (u64)X[i * ldx + b];
        acc[j * s + b] = (acc[j * s + b] + a * xv) % m;
      }
    }
  }
  for (i64 j = 0; j < ncols; ++j)
    for (i64 b = 0; b < s; ++b) {
      u64 yv = (u64)Y[j * ldy + b];
      Y[j * ldy + b] = (i64)((alpha * acc[j * s + b] % m + beta * yv % m) % m);
    }
  free(acc);
  return 0;
}

int oracle_spmv_t(i64 nrows, i64 ncols, const i64* rowptr, const int32_t* col, const i64* val, u64 m,
                  u64 alpha, const i64* x, u64 beta, i64* y) {
  return oracle_spmm_t(nrows, ncols, rowptr, col, val, m, 1, alpha, x, 1, beta, y, 1);
}

/* W <- A^k V for square A (n x n), V and W: n x s, ldv/ldw; k >= 0 */
int oracle_power(i64 n, const i64* rowptr, const int32_t* col, const i64* val, u64 m, i64 k, i64 s,
                 const i64* V, i64 ldv, i64* W, i64 ldw) {
  if (bad_modulus(m) || k < 0 || s < 1 || ldv < s || ldw < s) return -1;
  if (check_csr(n, n, rowptr, col) || check_vec(V, n, s, ldv, m)) return -1;
  i64* cur = (i64*)malloc(sizeof(i64) * (size_t)(n > 0 ? n : 1) * (size_t)s);
  i64* nxt = (i64*)malloc(sizeof(i64) * (size_t)(n > 0 ? n : 1) * (size_t)s);
  if (!cur || !nxt) { free(cur); free(nxt); return -1; }
  for (i64 i = 0; i < n; ++i)
    for (i64 b = 0; b < s; ++b) cur[i * s + b] = V[i * ldv + b];
  for (i64 it = 0; it < k; ++it) {
    memset(nxt, 0, sizeof(i64) * (size_t)n * (size_t)s);
    int rc = oracle_spmm(n, n, rowptr, col, val, m, s, 1, cur, s, 0, nxt, s);
    if (rc) { free(cur); free(nxt); return rc; }
    i64* t = cur; cur = nxt; nxt = t;
  }
  for (i64 i = 0; i < n; ++i)
    for (i64 b = 0; b < s; ++b) W[i * ldw + b] = cur[i * s + b];
  free(cur);
  free(nxt);
  return 0;
}

/* S[i][a][b] = sum_k U[k][a] * (A^i V)[k][b] mod m, for i = 0 .. L-1.
 * U and V are n x s (ldu, ldv). S has L*s*s entries. If Wout is not
 * null it receives A^L V (n x s, leading dimension s). */
int oracle_sequence(i64 n, const i64* rowptr, const int32_t* col, const i64* val, u64 m, i64 s,
                    const i64* U, i64 ldu, const i64* V, i64 ldv, i64 L, i64* S, i64* Wout) {
  if (bad_modulus(m) || L < 0 || s < 1 || ldu < s || ldv < s) return -1;
  if (check_csr(n, n, rowptr, col) || check_vec(U, n, s, ldu, m) || check_vec(V, n, s, ldv, m)) return -1;
  i64* W = (i64*)malloc(sizeof(i64) * (size_t)(n > 0 ? n : 1) * (size_t)s);
  i64* Wn = (i64*)malloc(sizeof(i64) * (size_t)(n > 0 ? n : 1) * (size_t)s);
  if (!W || !Wn) { free(W); free(Wn); return -1; }
  for (i64 k = 0; k < n; ++k)
    for (i64 b = 0; b < s; ++b) W[k * s + b] = V[k * ldv + b];
  for (i64 i = 0; i < L; ++i) {
    for (i64 a = 0; a < s; ++a)
      for (i64 b = 0; b < s; ++b) {
        u64 acc = 0;
        for (i64 k = 0; k < n; ++k) acc = (acc + (u64)U[k * ldu + a] * (u64)W[k * s + b]) % m;
        S[(i * s + a) * s + b] = (i64)acc;
      }
    memset(Wn, 0, sizeof(i64) * (size_t)n * (size_t)s);
    int rc = oracle_spmm(n, n, rowptr, col, val, m, s, 1, W, s, 0, Wn, s);
    if (rc) { free(W); free(Wn); return rc; }
    i64* t = W; W = Wn; Wn = t;
  }
  if (Wout)
    for (i64 k = 0; k < n * s; ++k) Wout[k] = W[k];
  free(W);
  free(Wn);
  return 0;
}

/* canonical residues of raw values, for tests that want the reduced matrix */
int oracle_canon(i64 count, const i64* v, u64 m, i64* out) {
  if (bad_modulus(m)) return -1;
  for (i64 k = 0; k < count; ++k) out[k] = (i64)canon(v[k], m);
  return 0;
}
