// FP64 dense linear algebra on the device for the small projected problems (sizes up to a
// few thousand): tiled GEMM, Gauss-Jordan inverse and solve, triangular solves.
// All matrices are column-major with explicit leading dimensions.
#pragma once

#include "common.hpp"

namespace skr {
namespace dense {

// C = alpha * op(A) op(B) + beta * C,  op(X) = X or X^T
void gemm(bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda, const double* B, int ldb,
          double beta, double* C, int ldc, hipStream_t st);
// The same product with the split-K partial products (long reductions with few output
// tiles) in a caller-provided workspace of ws_doubles doubles instead of the device-memory
// cache; gemm_workspace_doubles gives the size it needs (0 when the product is not split).
// Allocates nothing; SKR_EINVAL when the workspace is too small.
void gemm_ws(bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda, const double* B, int ldb,
             double beta, double* C, int ldc, double* ws, size_t ws_doubles, hipStream_t st);
size_t gemm_workspace_doubles(bool ta, bool tb, int m, int n, int k);

// X1 (n x l, row-major, ld ldx) = alpha * sum_j U_j W[j r : (j+1) r, :] + beta * X1, where the
// basis blocks U_j (n x r, row-major) are stored consecutively (block j at U + j n r) and W is
// (nb r) x l column-major with leading dimension ldw.  T is the basis element type.
template <typename T>
void basis_gemm(int n, int r, int nb, int l, double alpha, const T* U, const double* W, int ldw, double beta,
                double* X, int ldx, hipStream_t st);

// Blocked Gauss-Jordan elimination with partial pivoting of the first n columns of the
// n x ncols matrix S (column-major, leading dimension lds), in place and without moving
// rows.  iws holds gj_ints(n) ints (pivot rows, their inverse, flags) and dws gj_doubles(n)
// doubles.  info (device int) is set to 1 + the first column without a nonzero pivot;
// logabsdet (device double, may be null) receives log|det A|.  The results are read with
// gj_inverse (A^{-1}) and gj_solution (A^{-1} B for the columns n .. ncols-1 of S).
void gj_eliminate(int n, int ncols, double* S, int lds, int* iws, double* dws, int* info, double* logabsdet,
                  hipStream_t st);
// Several independent eliminations, each on its own stream (arguments as for gj_eliminate),
// enqueued interleaved launch by launch so that their chains run concurrently.
struct GjJob {
  int n, ncols;
  double* S;
  int lds;
  int* iws;
  double* dws;
  int* info;
  double* logabsdet;
  hipStream_t st;
};
void gj_eliminate_many(const GjJob* jobs, int count);
void gj_inverse(int n, const double* S, int lds, const int* iws, double* X, int ldx, hipStream_t st);
void gj_solution(int n, int nrhs, const double* S, int lds, const int* iws, double* X, int ldx, hipStream_t st);
int gj_ints(int n);
int gj_doubles(int n);
// y = A^{-1} b from the eliminated S of gj_eliminate(n, n, S, ...): y(i) = sum_k S(piv(i), k) b(piv(k)).
// work holds gj_apply_doubles(n) doubles; b and y may not alias.
void gj_apply(int n, const double* S, int lds, const int* iws, const double* b, double* y, double* work,
              hipStream_t st);
int gj_apply_doubles(int n);

// Solve T X = B in place (B <- T^{-1} B), T upper triangular n x n, B n x nrhs.
void trsm_left_upper(int n, int nrhs, const double* T, int ldt, double* B, int ldb, hipStream_t st);
// Solve X T = B in place (B <- B T^{-1}), T upper triangular n x n, B m x n.
void trsm_right_upper(int m, int n, const double* T, int ldt, double* B, int ldb, hipStream_t st);

// Elementwise helpers (column-major m x n views).
void copy(int m, int n, const double* A, int lda, double* B, int ldb, hipStream_t st);
void transpose(int m, int n, const double* A, int lda, double* B, int ldb, hipStream_t st);  // B = A^T
void set_zero(int m, int n, double* A, int lda, hipStream_t st);
// Z = (mu * X + Y / mu) / 2 with mu = *mu_dev; *diff_dev = ||Z - X||_F^2, *norm_dev = ||Z||_F^2,
// *trace_dev = trace(Z) (square only, may be null).  Reductions are deterministic.
void newton_combine(int m, int n, const double* mu_dev, const double* X, int ldx, const double* Y, int ldy, double* Z,
                    int ldz, double* diff_dev, double* norm_dev, double* trace_dev, double* scratch, hipStream_t st);
// *out = ||A||_F^2 (deterministic)
void fro2(int m, int n, const double* A, int lda, double* out, double* scratch, hipStream_t st);

int scratch_doubles();  // size of the `scratch` buffer the reductions need

}  // namespace dense
}  // namespace skr
