// C ABI of the library (declared in skrylov.h): argument checking, error translation,
// the solve entry points, the true-residual evaluation and the adjoint gradients.
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>

#include "dense.hpp"
#include "solver.hpp"

using namespace skr;

skr_op_s* op_create(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind, const double* vals,
                    const double* diag, hipStream_t stream);
void op_set_diag(skr_op_s* op, const double* diag, hipStream_t stream);

namespace {

thread_local std::string g_last_error;

template <class F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return SKR_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return SKR_EINVAL;
  }
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------- wide SpMM, column-major
// Y(:, c) = Op X(:, c) (+ diag o X(:, c)); X, Y column-major n x q with leading dimension n.
__global__ void spmm_wide_kernel(CsrView<double> A, int q, const double* X, double* Y, double* Yneg_target,
                                 int ldy) {
  (void)Yneg_target;
  const int64_t total = (int64_t)A.n * q;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % A.n), c = (int)(e / A.n);
    const double* x = X + (size_t)c * A.n;
    double y = 0.0;
    for (int k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) y += A.val[k] * x[A.colind[k]];
    if (A.diag) y += A.diag[i] * x[i];
    Y[i + (size_t)c * ldy] = y;
  }
}

// column-major n x q block <- alpha * (row-major n x q)
__global__ void rm_to_cm_kernel(int n, int q, const double* src, double alpha, double* dst, int ldd) {
  const int64_t total = (int64_t)n * q;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), c = (int)(e / n);
    dst[i + (size_t)c * ldd] = alpha * src[(size_t)i * q + c];
  }
}

// ---------------------------------------------------------------- Householder TSQR
// R factor of a tall column-major matrix by a tree of Householder QRs of row blocks
// (tall-skinny QR).  Backward stable for any rank, unlike Cholesky-based QR.
constexpr int HQ_T = 1024;
constexpr int HQ_MAXB = 4096;  // rows per block (LDS holds one Householder vector)

// Each workgroup: Householder QR of rows [blk*b, min(n, blk*b+b)) of the q columns of A
// (column-major, leading dimension lda; the block is overwritten), then writes its q x q
// upper-triangular factor (rows beyond the block's row count are zero) to S at rows
// [blk*q, blk*q+q) (column-major, leading dimension lds).
__global__ void __launch_bounds__(HQ_T) house_block_kernel(int n, int q, double* A, int lda, int b, double* S,
                                                            int lds) {
  __shared__ double v[HQ_MAXB];
  __shared__ double sdot[1024];
  __shared__ double red[HQ_T / 64];
  __shared__ double sh_alpha, sh_tau;
  const int blk = blockIdx.x, tid = threadIdx.x;
  const int r0 = blk * b, rows = min(b, n - r0);
  double* Ab = A + r0;
  const int kmax = min(rows, q);
  for (int j = 0; j < kmax; ++j) {
    const int len = rows - j;
    double s2 = 0.0;
    for (int i = tid; i < len; i += HQ_T) {
      const double x = Ab[(j + i) + (size_t)j * lda];
      v[i] = x;
      s2 += x * x;
    }
    s2 = wave_sum(s2);
    if (tid % 64 == 0) red[tid / 64] = s2;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < HQ_T / 64; ++w) t += red[w];
      const double nrm = sqrt(t), x0 = v[0];
      if (nrm == 0.0) {
        sh_alpha = 0.0;
        sh_tau = 0.0;
      } else {
        const double alpha = x0 >= 0.0 ? -nrm : nrm;
        const double v0 = x0 - alpha;
        v[0] = v0;
        sh_alpha = alpha;
        sh_tau = 2.0 / (t - x0 * x0 + v0 * v0);  // 2 / (v^T v)
      }
    }
    __syncthreads();
    const double tau = sh_tau;
    const int ncols = q - j - 1;
    if (tau != 0.0 && ncols > 0) {
      for (int c0 = 0; c0 < ncols; c0 += 1024) {
        const int nc = min(1024, ncols - c0);
        // sdot[c] = v^T A(j:, j+1+c0+c): one wavefront per column, lanes over the rows
        // (coalesced), a fixed-order wavefront sum
        const int lane = tid % 64, wv = tid / 64;
        for (int c = wv; c < nc; c += HQ_T / 64) {
          const double* col = Ab + j + (size_t)(j + 1 + c0 + c) * lda;
          double t = 0.0;
          for (int i = lane; i < len; i += 64) t += v[i] * col[i];
          t = wave_sum(t);
          if (lane == 0) sdot[c] = t;
        }
        __syncthreads();
        for (int64_t e = tid; e < (int64_t)len * nc; e += HQ_T) {
          const int i = (int)(e % len), c = (int)(e / len);
          Ab[(j + i) + (size_t)(j + 1 + c0 + c) * lda] -= tau * sdot[c] * v[i];
        }
        __syncthreads();
      }
    }
    if (tid == 0) Ab[j + (size_t)j * lda] = (tau != 0.0) ? sh_alpha : v[0];
    __syncthreads();
  }
  // write R (upper part of the first min(rows, q) rows) into S
  for (int64_t e = tid; e < (int64_t)q * q; e += HQ_T) {
    const int i = (int)(e % q), c = (int)(e / q);
    double val = 0.0;
    if (i <= c && i < rows) val = Ab[i + (size_t)c * lda];
    S[(size_t)blk * q + i + (size_t)c * lds] = val;
  }
}

// R factor (q x q, column-major) of the column-major n x q matrix L (overwritten).
void tsqr_r(int n, int q, double* L, double* R, hipStream_t st) {
  SKR_REQUIRE(q <= HQ_MAXB / 2, "too many columns for the residual evaluation");
  const int b = std::min(HQ_MAXB, std::max(4 * q, 1024));
  int rows = n, ld = n;
  double* cur = L;
  DBuf<double> bufs[2];
  int which = 0;
  while (true) {
    const int nblk = ceil_div(rows, b);
    DBuf<double>& S = bufs[which];
    S.alloc((size_t)nblk * q * q);
    hipLaunchKernelGGL(house_block_kernel, dim3(nblk), dim3(HQ_T), 0, st, rows, q, cur, ld, b, S.p, nblk * q);
    check_launch("house_block");
    SKR_HIP(hipStreamSynchronize(st));  // the previous level's buffer is released next
    if (nblk == 1) {
      dense::copy(q, q, S.p, nblk * q, R, q, st);
      SKR_HIP(hipStreamSynchronize(st));
      return;
    }
    rows = nblk * q;
    ld = rows;
    cur = S.p;
    which ^= 1;
  }
}

void check_op(const skr_op_s* op) { SKR_REQUIRE(op != nullptr, "null operator"); }

}  // namespace

extern "C" {

int skr_params_default(skr_params* p) {
  if (!p) return SKR_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->k = 2;
  p->maxit = 200;
  p->p = 20;
  p->zeta = 8;
  p->s = 0;
  p->tol = 1e-6;
  p->seed = 0;
  p->precision = SKR_FP64;
  p->sketch = SKR_SKETCH_SPARSE_SIGN;
  p->recover = SKR_RECOVER_STORED;
  p->trunc_tol = 1e-12;
  p->orth = SKR_ORTH_EUCLIDEAN;
  return SKR_OK;
}

int skr_op_create_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind, const double* vals,
                      const double* diag, void* stream, skr_op* out) {
  return guarded([&] {
    SKR_REQUIRE(out, "null output handle");
    *out = op_create(n, nnz, rowptr, colind, vals, diag, as_stream(stream));
    return SKR_OK;
  });
}

int skr_op_set_diag(skr_op op, const double* diag, void* stream) {
  return guarded([&] {
    check_op(op);
    op_set_diag(op, diag, as_stream(stream));
    return SKR_OK;
  });
}

int skr_op_size(skr_op op, int64_t* n, int64_t* nnz) {
  return guarded([&] {
    check_op(op);
    if (n) *n = op->n;
    if (nnz) *nnz = op->nnz;
    return SKR_OK;
  });
}

int skr_op_destroy(skr_op op) {
  delete op;
  return SKR_OK;
}

int skr_solve(skr_op A, skr_op B, const double* C1, const double* C2, int64_t r, const skr_params* params,
              void* stream, skr_result* out) {
  return guarded([&] {
    SKR_REQUIRE(out && params, "null argument");
    check_op(A);
    check_op(B);
    SKR_REQUIRE(r >= 1 && r <= RMAX, "r must be in [1, 16]");
    *out = nullptr;
    skr_result_s* res = run_solve(A, 0, B, 1, C1, C2, (int)r, *params, as_stream(stream));
    *out = res;
    return (int)res->status;
  });
}

int skr_adjoint_solve(skr_op A, skr_op B, const double* G1, const double* G2, int64_t r, const skr_params* params,
                      void* stream, skr_result* out) {
  return guarded([&] {
    SKR_REQUIRE(out && params, "null argument");
    check_op(A);
    check_op(B);
    SKR_REQUIRE(r >= 1 && r <= RMAX, "r must be in [1, 16]");
    *out = nullptr;
    skr_result_s* res = run_solve(A, 1, B, 0, G1, G2, (int)r, *params, as_stream(stream));
    *out = res;
    return (int)res->status;
  });
}

int skr_lyap_solve(skr_op A, const double* C, int64_t r, const skr_params* params, void* stream, skr_result* out) {
  return guarded([&] {
    SKR_REQUIRE(out && params, "null argument");
    check_op(A);
    SKR_REQUIRE(r >= 1 && r <= RMAX, "r must be in [1, 16]");
    *out = nullptr;
    skr_result_s* res = run_solve(A, 0, nullptr, 0, C, C, (int)r, *params, as_stream(stream));
    *out = res;
    return (int)res->status;
  });
}

int skr_result_info(skr_result res, int64_t* ell, int32_t* iters, double* rho_rel, int32_t* status) {
  return guarded([&] {
    SKR_REQUIRE(res, "null result");
    if (ell) *ell = res->ell;
    if (iters) *iters = res->iters;
    if (rho_rel) *rho_rel = res->rho_rel;
    if (status) *status = res->status;
    return SKR_OK;
  });
}

int skr_result_history(skr_result res, int32_t* d, double* rho_rel, int32_t cap, int32_t* len) {
  return guarded([&] {
    SKR_REQUIRE(res, "null result");
    const int32_t nh = (int32_t)res->hist_d.size();
    if (len) *len = nh;
    for (int32_t i = 0; i < std::min(cap, nh); ++i) {
      if (d) d[i] = res->hist_d[i];
      if (rho_rel) rho_rel[i] = res->hist_rho[i];
    }
    return SKR_OK;
  });
}

int skr_result_copy_factors(skr_result res, double* X1, double* X2, void* stream) {
  return guarded([&] {
    SKR_REQUIRE(res, "null result");
    hipStream_t st = as_stream(stream);
    if (X1) SKR_HIP(hipMemcpyAsync(X1, res->X1.p, sizeof(double) * res->n1 * res->ell, hipMemcpyDeviceToDevice, st));
    if (X2) SKR_HIP(hipMemcpyAsync(X2, res->X2.p, sizeof(double) * res->n2 * res->ell, hipMemcpyDeviceToDevice, st));
    return SKR_OK;
  });
}

int skr_result_timing(skr_result res, double* ms_steps, double* ms_proj, double* ms_recover) {
  return guarded([&] {
    SKR_REQUIRE(res, "null result");
    if (ms_steps) *ms_steps = res->ms_steps;
    if (ms_proj) *ms_proj = res->ms_proj;
    if (ms_recover) *ms_recover = res->ms_recover;
    return SKR_OK;
  });
}

int skr_result_kernel_stats(skr_result res, int32_t idx, int32_t* count, const char** name, int64_t* launches,
                            double* ms) {
  return guarded([&] {
    SKR_REQUIRE(res, "null result");
    if (count) *count = KF_COUNT;
    SKR_REQUIRE(idx >= 0 && idx < KF_COUNT, "kernel family index out of range");
    if (name) *name = kernel_family_name(idx);
    if (launches) *launches = res->fam_launches[idx];
    if (ms) *ms = res->fam_ms[idx];
    return SKR_OK;
  });
}

int skr_result_proj_stats(skr_result res, int32_t* newton_iters, int32_t* neg_a, int32_t* neg_b, double* proj_resid) {
  return guarded([&] {
    SKR_REQUIRE(res, "null result");
    if (newton_iters) *newton_iters = res->last_stats.newton_iters;
    if (neg_a) *neg_a = res->last_stats.neg_eigs_a;
    if (neg_b) *neg_b = res->last_stats.neg_eigs_b;
    if (proj_resid) *proj_resid = res->last_stats.proj_resid;
    return SKR_OK;
  });
}

int skr_result_failed_checks(skr_result res, int32_t* failed) {
  return guarded([&] {
    SKR_REQUIRE(res && failed, "null argument");
    *failed = res->failed_checks;
    return SKR_OK;
  });
}

int skr_result_destroy(skr_result res) {
  delete res;
  return SKR_OK;
}

}  // extern "C"

namespace {

// ||opA(A) X + X opB(B)^T... evaluated as ||[A' X1, X1, -C1] [X2, B' X2, C2]^T||_F / ||C1 C2^T||_F
// with A' = A (ta = 0) or A^T (ta = 1) applied to X1 and B' = B^T (tb = 1, the forward
// equation's X B = X1 (B^T X2)^T) or B (tb = 0, the adjoint's L B^T = L1 (B L2)^T).
int true_residual_impl(skr_op A, int ta, skr_op B, int tb, const double* X1, const double* X2, int64_t ell,
                       const double* C1, const double* C2, int64_t r, void* stream, double* rel) {
  return guarded([&] {
    check_op(A);
    check_op(B);
    SKR_REQUIRE(X1 && X2 && C1 && C2 && rel, "null argument");
    SKR_REQUIRE(ell >= 1 && r >= 1, "ell and r must be positive");
    hipStream_t st = as_stream(stream);
    const int n1 = (int)A->n, n2 = (int)B->n, L = (int)ell, R = (int)r;
    const int q = 2 * L + R;
    DBuf<double> Lm((size_t)n1 * q), Rm((size_t)n2 * q), RL((size_t)q * q), RR((size_t)q * q), P((size_t)q * q),
        scratch(dense::scratch_doubles()), out(2);
    auto grid = [](int64_t tot) { return (int)std::min<int64_t>(8192, (tot + 255) / 256); };
    // Lm = [A X1, X1, -C1], Rm = [X2, B^T X2, C2]  (column-major)
    hipLaunchKernelGGL(rm_to_cm_kernel, dim3(grid((int64_t)n1 * L)), dim3(256), 0, st, n1, L, X1, 1.0, Lm.p + (size_t)L * n1, n1);
    hipLaunchKernelGGL(rm_to_cm_kernel, dim3(grid((int64_t)n1 * R)), dim3(256), 0, st, n1, R, C1, -1.0, Lm.p + (size_t)2 * L * n1, n1);
    hipLaunchKernelGGL(rm_to_cm_kernel, dim3(grid((int64_t)n2 * L)), dim3(256), 0, st, n2, L, X2, 1.0, Rm.p, n2);
    hipLaunchKernelGGL(rm_to_cm_kernel, dim3(grid((int64_t)n2 * R)), dim3(256), 0, st, n2, R, C2, 1.0, Rm.p + (size_t)2 * L * n2, n2);
    check_launch("rm_to_cm");
    hipLaunchKernelGGL(spmm_wide_kernel, dim3(grid((int64_t)n1 * L)), dim3(256), 0, st, csr_view<double>(A, ta), L,
                       Lm.p + (size_t)L * n1, Lm.p, nullptr, n1);
    hipLaunchKernelGGL(spmm_wide_kernel, dim3(grid((int64_t)n2 * L)), dim3(256), 0, st, csr_view<double>(B, tb), L,
                       Rm.p, Rm.p + (size_t)L * n2, nullptr, n2);
    check_launch("spmm_wide");
    // ||C1 C2^T||_F via the same route on the r-column factors
    DBuf<double> c1((size_t)n1 * R), c2((size_t)n2 * R), rc1((size_t)R * R), rc2((size_t)R * R), pc((size_t)R * R);
    hipLaunchKernelGGL(rm_to_cm_kernel, dim3(grid((int64_t)n1 * R)), dim3(256), 0, st, n1, R, C1, 1.0, c1.p, n1);
    hipLaunchKernelGGL(rm_to_cm_kernel, dim3(grid((int64_t)n2 * R)), dim3(256), 0, st, n2, R, C2, 1.0, c2.p, n2);
    check_launch("rm_to_cm");
    tsqr_r(n1, q, Lm.p, RL.p, st);
    tsqr_r(n2, q, Rm.p, RR.p, st);
    tsqr_r(n1, R, c1.p, rc1.p, st);
    tsqr_r(n2, R, c2.p, rc2.p, st);
    dense::gemm(false, true, q, q, q, 1.0, RL.p, q, RR.p, q, 0.0, P.p, q, st);
    dense::gemm(false, true, R, R, R, 1.0, rc1.p, R, rc2.p, R, 0.0, pc.p, R, st);
    dense::fro2(q, q, P.p, q, out.p, scratch.p, st);
    dense::fro2(R, R, pc.p, R, out.p + 1, scratch.p, st);
    double h[2];
    SKR_HIP(hipMemcpyAsync(h, out.p, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    SKR_HIP(hipStreamSynchronize(st));
    *rel = std::sqrt(h[0] / h[1]);
    return SKR_OK;
  });
}

}  // namespace

extern "C" {

int skr_true_residual(skr_op A, skr_op B, const double* X1, const double* X2, int64_t ell, const double* C1,
                      const double* C2, int64_t r, void* stream, double* rel) {
  return true_residual_impl(A, 0, B, 1, X1, X2, ell, C1, C2, r, stream, rel);
}

int skr_true_residual_adjoint(skr_op A, skr_op B, const double* L1, const double* L2, int64_t ell, const double* G1,
                              const double* G2, int64_t r, void* stream, double* rel) {
  return true_residual_impl(A, 1, B, 0, L1, L2, ell, G1, G2, r, stream, rel);
}

}  // extern "C"

namespace {

// out_i = -sum_b Z[i][b] X[i][b], Z, X row-major n x l.  Sixteen lanes (one DPP row) per
// matrix row, each striding over the row's columns, so that a row's loads are contiguous;
// the lanes' sums are combined by DPP butterflies.
__global__ void rowdot_kernel(int n, int l, const double* Z, const double* X, double* out) {
  const int lane16 = threadIdx.x % 16;
  const int rows_per_block = blockDim.x / 16;
  for (int i0 = blockIdx.x * rows_per_block; i0 < n; i0 += gridDim.x * rows_per_block) {
    const int i = i0 + threadIdx.x / 16;  // rows beyond n take part in the butterflies only
    double s = 0.0;
    if (i < n)
      for (int b = lane16; b < l; b += 16) s += Z[(size_t)i * l + b] * X[(size_t)i * l + b];
    s += dpp_move<0xB1>(s);   // quad_perm [1,0,3,2]
    s += dpp_move<0x4E>(s);   // quad_perm [2,3,0,1]
    s += dpp_move<0x124>(s);  // row_ror:4
    s += dpp_move<0x128>(s);  // row_ror:8
    if (i < n && lane16 == 0) out[i] = -s;
  }
}

__global__ void dot_kernel(int count, const double* a, const double* b, double* out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int e = threadIdx.x; e < count; e += blockDim.x) s += a[e] * b[e];
  s = wave_sum(s);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)blockDim.x / 64; ++w) t += red[w];
    *out = t;
  }
}

// Row-major M (n x c) viewed as column-major c x n with leading dimension c.
// S = M1^T M2 (c1 x c2, column-major) = reduction over n: gemm(false, true) on the views.
void inner(int n, int c1, int c2, const double* M1, const double* M2, double* S, hipStream_t st) {
  dense::gemm(false, true, c1, c2, n, 1.0, M1, c1, M2, c2, 0.0, S, c1, st);
}
// O (n x c2, row-major) = M (n x c1, row-major) S (c1 x c2, column-major):
// in the column-major views O^T = S^T M^T  -> gemm(true, false).
void outer(int n, int c1, int c2, const double* M, const double* S, double* O, hipStream_t st) {
  dense::gemm(true, false, c2, n, c1, 1.0, S, c1, M, c1, 0.0, O, c2, st);
}

}  // namespace

extern "C" int skr_pairing_grads(int64_t n1, int64_t n2, int64_t r, int64_t q, const double* X1, const double* X2,
                                 int64_t ellx, const double* L1, const double* L2, int64_t elll, const double* C1,
                                 const double* C2, const double* P1, const double* P2, double* loss, double* dC1,
                                 double* dC2, double* dsig, double* dP1, double* dP2, void* stream) {
  return guarded([&] {
    SKR_REQUIRE(n1 > 0 && n2 > 0 && r > 0 && q > 0 && ellx > 0, "sizes must be positive");
    SKR_REQUIRE(X1 && X2 && P1 && P2, "null argument");
    hipStream_t st = as_stream(stream);
    const int N1 = (int)n1, N2 = (int)n2, R = (int)r, Q = (int)q, LX = (int)ellx, LL = (int)elll;
    // loss = <P1^T X1, P2^T X2>.  Temporaries live until the final synchronisation.
    DBuf<double> a((size_t)Q * LX), b((size_t)Q * LX), out(1);
    DBuf<double> sp1((size_t)LX * Q), sp2((size_t)LX * Q);
    DBuf<double> sc1, sc2, ss, Z;
    inner(N1, Q, LX, P1, X1, a.p, st);
    inner(N2, Q, LX, P2, X2, b.p, st);
    hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(256), 0, st, Q * LX, a.p, b.p, out.p);
    check_launch("dot");
    if (dP1) {  // X1 (X2^T P2)
      inner(N2, LX, Q, X2, P2, sp1.p, st);
      outer(N1, LX, Q, X1, sp1.p, dP1, st);
    }
    if (dP2) {  // X2 (X1^T P1)
      inner(N1, LX, Q, X1, P1, sp2.p, st);
      outer(N2, LX, Q, X2, sp2.p, dP2, st);
    }
    if (dC1 || dC2 || dsig) {
      SKR_REQUIRE(L1 && L2 && elll > 0, "adjoint factors required for dC1, dC2, dsig");
      if (dC1) {  // L1 (L2^T C2)
        SKR_REQUIRE(C2, "C2 required for dC1");
        sc1.alloc((size_t)LL * R);
        inner(N2, LL, R, L2, C2, sc1.p, st);
        outer(N1, LL, R, L1, sc1.p, dC1, st);
      }
      if (dC2) {  // L2 (L1^T C1)
        SKR_REQUIRE(C1, "C1 required for dC2");
        sc2.alloc((size_t)LL * R);
        inner(N1, LL, R, L1, C1, sc2.p, st);
        outer(N2, LL, R, L2, sc2.p, dC2, st);
      }
      if (dsig) {  // -rowsum((L1 (L2^T X2)) o X1)
        ss.alloc((size_t)LL * LX);
        Z.alloc((size_t)N1 * LX);
        inner(N2, LL, LX, L2, X2, ss.p, st);
        outer(N1, LL, LX, L1, ss.p, Z.p, st);
        hipLaunchKernelGGL(rowdot_kernel, dim3(std::min(8192, ceil_div(N1, 16))), dim3(256), 0, st, N1, LX, Z.p, X1,
                           dsig);
        check_launch("rowdot");
      }
    }
    double h = 0.0;
    SKR_HIP(hipMemcpyAsync(&h, out.p, sizeof(double), hipMemcpyDeviceToHost, st));
    SKR_HIP(hipStreamSynchronize(st));
    if (loss) *loss = h;
    return SKR_OK;
  });
}

// ------------------------------------------------------------ allocation-free gradients
// skr_pairing_grads_noalloc keeps every temporary in `scratch`, a fixed device array of
// SKR_PAIRING_SCRATCH_BYTES that each device holds from the module load until the process
// ends.  Host code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): the device address comes from hipGetSymbolAddress, taken once
// per device with that device current and kept in g_scratch_dev.
namespace {

constexpr size_t SCRATCH_DOUBLES = SKR_PAIRING_SCRATCH_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[MAX_DEVICES] = {};

double* scratch_on_current_device() {
  int dev = 0;
  SKR_HIP(hipGetDevice(&dev));
  SKR_REQUIRE(dev >= 0 && dev < MAX_DEVICES, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      throw Error(SKR_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_dev[dev];
}

// Offsets of consecutive 256-byte aligned pieces of the scratch array (in doubles).
struct Carver {
  size_t used = 0;
  size_t take(size_t count) {
    const size_t start = (used + 31) / 32 * 32;
    used = start + count;
    return start;
  }
};

}  // namespace

extern "C" int skr_pairing_grads_noalloc(int64_t n1, int64_t n2, int64_t r, int64_t q, const double* X1,
                                         const double* X2, int64_t ellx, const double* L1, const double* L2,
                                         int64_t elll, const double* C1, const double* C2, const double* P1,
                                         const double* P2, double* loss, double* dC1, double* dC2, double* dsig,
                                         double* dP1, double* dP2, void* stream) {
  return guarded([&] {
    SKR_REQUIRE(n1 > 0 && n2 > 0 && r > 0 && q > 0 && ellx > 0, "sizes must be positive");
    SKR_REQUIRE(n1 <= INT_MAX && n2 <= INT_MAX && r <= INT_MAX && q <= INT_MAX && ellx <= INT_MAX && elll <= INT_MAX,
                "sizes must fit in 32 bits");
    SKR_REQUIRE(X1 && X2 && P1 && P2, "null argument");
    const bool adj = dC1 || dC2 || dsig;
    SKR_REQUIRE(!adj || (L1 && L2 && elll > 0), "adjoint factors required for dC1, dC2, dsig");
    SKR_REQUIRE(!dC1 || C2, "C2 required for dC1");
    SKR_REQUIRE(!dC2 || C1, "C1 required for dC2");
    hipStream_t st = as_stream(stream);
    const int N1 = (int)n1, N2 = (int)n2, R = (int)r, Q = (int)q, LX = (int)ellx, LL = (int)elll;
    // Lay out the temporaries as offsets and reject an oversized request before any work
    // is queued.  Z (the rows of L1 (L2^T X2) that the dsig kernel reads) takes what is left,
    // at least one row.
    Carver c;
    const size_t o_a = c.take((size_t)Q * LX), o_b = c.take((size_t)Q * LX), o_out = c.take(1);
    const size_t o_sp1 = dP1 ? c.take((size_t)LX * Q) : 0, o_sp2 = dP2 ? c.take((size_t)LX * Q) : 0;
    const size_t o_sc1 = dC1 ? c.take((size_t)LL * R) : 0, o_sc2 = dC2 ? c.take((size_t)LL * R) : 0;
    const size_t o_ss = dsig ? c.take((size_t)LL * LX) : 0;
    size_t ws_n = 0;  // split-K partials of the longest reduction, reused call after call
    ws_n = std::max(ws_n, dense::gemm_workspace_doubles(false, true, Q, LX, N1));
    ws_n = std::max(ws_n, dense::gemm_workspace_doubles(false, true, Q, LX, N2));
    if (dP1) ws_n = std::max(ws_n, dense::gemm_workspace_doubles(false, true, LX, Q, N2));
    if (dP2) ws_n = std::max(ws_n, dense::gemm_workspace_doubles(false, true, LX, Q, N1));
    if (dC1) ws_n = std::max(ws_n, dense::gemm_workspace_doubles(false, true, LL, R, N2));
    if (dC2) ws_n = std::max(ws_n, dense::gemm_workspace_doubles(false, true, LL, R, N1));
    if (dsig) ws_n = std::max(ws_n, dense::gemm_workspace_doubles(false, true, LL, LX, N2));
    const size_t o_ws = c.take(ws_n);
    int zrows = 0;
    size_t o_z = 0;
    if (dsig) {
      o_z = c.take(0);
      const size_t left = o_z < SCRATCH_DOUBLES ? SCRATCH_DOUBLES - o_z : 0;
      zrows = (int)std::min<size_t>(left / (size_t)LX, (size_t)N1);
      c.used = o_z + (size_t)zrows * LX;
    }
    if (c.used > SCRATCH_DOUBLES || (dsig && zrows < 1))
      throw Error(SKR_EINVAL, "skr_pairing_grads_noalloc: the temporaries of these sizes exceed the " +
                                  std::to_string((long long)SKR_PAIRING_SCRATCH_BYTES) + "-byte device workspace");
    double* base = scratch_on_current_device();
    double *a = base + o_a, *b = base + o_b, *out = base + o_out, *sp1 = base + o_sp1, *sp2 = base + o_sp2;
    double *sc1 = base + o_sc1, *sc2 = base + o_sc2, *ss = base + o_ss, *ws = ws_n ? base + o_ws : nullptr;
    double* Z = base + o_z;
    auto inner_ws = [&](int n, int c1, int c2, const double* M1, const double* M2, double* S) {
      dense::gemm_ws(false, true, c1, c2, n, 1.0, M1, c1, M2, c2, 0.0, S, c1, ws, ws_n, st);
    };
    auto outer_ws = [&](int n, int c1, int c2, const double* M, const double* S, double* O) {
      dense::gemm_ws(true, false, c2, n, c1, 1.0, S, c1, M, c1, 0.0, O, c2, nullptr, 0, st);
    };
    inner_ws(N1, Q, LX, P1, X1, a);
    inner_ws(N2, Q, LX, P2, X2, b);
    hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(256), 0, st, Q * LX, a, b, out);
    check_launch("dot");
    if (dP1) {  // X1 (X2^T P2)
      inner_ws(N2, LX, Q, X2, P2, sp1);
      outer_ws(N1, LX, Q, X1, sp1, dP1);
    }
    if (dP2) {  // X2 (X1^T P1)
      inner_ws(N1, LX, Q, X1, P1, sp2);
      outer_ws(N2, LX, Q, X2, sp2, dP2);
    }
    if (dC1) {  // L1 (L2^T C2)
      inner_ws(N2, LL, R, L2, C2, sc1);
      outer_ws(N1, LL, R, L1, sc1, dC1);
    }
    if (dC2) {  // L2 (L1^T C1)
      inner_ws(N1, LL, R, L1, C1, sc2);
      outer_ws(N2, LL, R, L2, sc2, dC2);
    }
    if (dsig) {  // -rowsum((L1 (L2^T X2)) o X1), zrows rows at a time
      inner_ws(N2, LL, LX, L2, X2, ss);
      for (int i0 = 0; i0 < N1; i0 += zrows) {
        const int rows = std::min(zrows, N1 - i0);
        outer_ws(rows, LL, LX, L1 + (size_t)i0 * LL, ss, Z);
        hipLaunchKernelGGL(rowdot_kernel, dim3(std::min(8192, ceil_div(rows, 16))), dim3(256), 0, st, rows, LX, Z,
                           X1 + (size_t)i0 * LX, dsig + i0);
        check_launch("rowdot");
      }
    }
    double h = 0.0;
    SKR_HIP(hipMemcpyAsync(&h, out, sizeof(double), hipMemcpyDeviceToHost, st));
    SKR_HIP(hipStreamSynchronize(st));
    if (loss) *loss = h;
    return SKR_OK;
  });
}

extern "C" int skr_release_cached_memory(void) {
  return guarded([&] {
    pool_trim();
    return SKR_OK;
  });
}

extern "C" const char* skr_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* skr_version(void) { return "skrylov-gfx950 0.1"; }
