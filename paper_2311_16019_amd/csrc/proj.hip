// Projected Sylvester problem on the device (FP64).
//
// The small equation M_A Y + Y M_B^T = F is solved with the coupled Newton iteration for
// the matrix sign function of Z = [[M_A, F], [0, -M_B^T]]: with A_0 = M_A, B_0 = M_B^T,
// C_0 = F and a scaling mu_k,
//     A_{k+1} = (mu A_k + A_k^{-1}/mu)/2,  B_{k+1} = (mu B_k + B_k^{-1}/mu)/2,
//     C_{k+1} = (mu C_k + A_k^{-1} C_k B_k^{-1}/mu)/2,
// A_k -> sign(M_A), B_k -> sign(M_B^T) and C_k -> 2 Y when both sign limits are the
// identity (all eigenvalues in the open right half plane, the case of the positive real
// operators this solver targets).  Every iteration is two LU-based inversions and two GEMMs,
// which map onto the GPU; the paper solves the same equation with Bartels-Stewart (Sec. 6),
// whose Schur decompositions do not.  When a limit is not the identity the projected
// matrix is indefinite (the paper's Example 4.5 shows this can happen) and the solve
// reports SKR_EPROJ rather than return a wrong Y.
#include <algorithm>
#include <cmath>
#include <vector>

#include "dense.hpp"
#include "proj.hpp"

namespace skr {
namespace {

enum Scal { LDA = 0, LDB, MU, DA, NA, TA, DB, NB_, TB, DC, NC, RHO2, RES2, F2, YN2, SCAL_N };

__global__ void set_scalar_kernel(double* p, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void mu_kernel(double* s, int m, int scale) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    s[MU] = scale ? exp(-(s[LDA] + s[LDB]) / (2.0 * m)) : 1.0;
}

// F: zero except its top-left r x r block = F11 (row-major) ; column-major m x m
__global__ void rhs_kernel(int m, int r, const double* F11, double* F) {
  const size_t total = (size_t)m * m;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    F[e] = (i < r && j < r) ? F11[i * r + j] : 0.0;
  }
}

// rho^2 = ||hh Y[m-r:m, :]||_F^2 + ||Y[:, m-r:m] gh^T||_F^2, hh/gh r x r column-major with ld.
__global__ void rho_kernel(int m, int r, const double* Y, const double* hh, int ldh, const double* gh, int ldg,
                           double* out) {
  __shared__ double red[16];
  double acc = 0.0;
  for (int e = threadIdx.x; e < 2 * m * r; e += blockDim.x) {
    const int which = e / (m * r), rem = e % (m * r);
    const int a = rem % r, j = rem / r;
    double t = 0.0;
    if (which == 0) {  // (hh Y_last)(a, j) = sum_c hh(a,c) Y(m-r+c, j)
      for (int c = 0; c < r; ++c) t += hh[a + (size_t)c * ldh] * Y[(m - r + c) + (size_t)j * m];
    } else {  // (Y_lastcol gh^T)(j, a) = sum_c Y(j, m-r+c) gh(a, c)
      for (int c = 0; c < r; ++c) t += Y[j + (size_t)(m - r + c) * m] * gh[a + (size_t)c * ldg];
    }
    acc += t * t;
  }
  acc = wave_sum(acc);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)blockDim.x / 64; ++w) s += red[w];
    *out = s;
  }
}

// W = M_A Y + Y M_B^T - F has been formed except for "-F"; subtract F's block and reduce.
__global__ void sub_rhs_kernel(int m, int r, const double* F11, double* W) {
  const int e = threadIdx.x;
  if (e < r * r) W[(e / r) + (size_t)(e % r) * m] -= F11[(e / r) * r + e % r];
}

// ---- complete-pivoting low-rank factorisation -------------------------------------
constexpr int ACA_WG = 256, ACA_G = 512;

__global__ void aca_update_kernel(int m, double* R, const double* Y1, const double* Y2, const int* state, double* part,
                                  int* ipart) {
  const int k = state[0], done = state[1];
  if (done) return;
  const double* u = k > 0 ? Y1 + (size_t)(k - 1) * m : nullptr;
  const double* v = k > 0 ? Y2 + (size_t)(k - 1) * m : nullptr;
  double best = -1.0, ss = 0.0;
  long long bidx = -1;
  const size_t total = (size_t)m * m;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    double x = R[e];
    if (u) { x -= u[i] * v[j]; R[e] = x; }
    const double ax = fabs(x);
    ss += x * x;
    if (ax > best) { best = ax; bidx = (long long)e; }
  }
  __shared__ double sb[ACA_WG / 64], sss[ACA_WG / 64];
  __shared__ long long si[ACA_WG / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const long long oi = __shfl_xor(bidx, off, 64);
    if (ob > best || (ob == best && oi >= 0 && (bidx < 0 || oi < bidx))) { best = ob; bidx = oi; }
  }
  ss = wave_sum(ss);
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  if (lane == 0) { sb[wv] = best; si[wv] = bidx; sss[wv] = ss; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = -1.0, s2 = 0.0;
    long long bi = -1;
    for (int w = 0; w < ACA_WG / 64; ++w) {
      s2 += sss[w];
      if (sb[w] > b || (sb[w] == b && si[w] >= 0 && (bi < 0 || si[w] < bi))) { b = sb[w]; bi = si[w]; }
    }
    part[blockIdx.x] = b;
    part[ACA_G + blockIdx.x] = s2;
    reinterpret_cast<long long*>(ipart)[blockIdx.x] = bi;
  }
}

// state: [0] rank so far, [1] done flag; scal: [0] ||Y||_F^2 (set on the first call)
__global__ void aca_select_kernel(int m, int ng, const double* R, double* Y1, double* Y2, int* state,
                                  const double* part, const int* ipart, double* ynorm2, double tol2, int kmax) {
  __shared__ int pi, pj;
  __shared__ double pv;
  __shared__ int stop;
  if (state[1]) return;
  if (threadIdx.x == 0) {
    double b = -1.0, s2 = 0.0;
    long long bi = -1;
    const long long* ip = reinterpret_cast<const long long*>(ipart);
    for (int g = 0; g < ng; ++g) {
      s2 += part[ACA_G + g];
      if (part[g] > b || (part[g] == b && ip[g] >= 0 && (bi < 0 || ip[g] < bi))) { b = part[g]; bi = ip[g]; }
    }
    const int k = state[0];
    if (k == 0) *ynorm2 = s2;
    stop = (k >= kmax) || !(b > 0.0) || bi < 0 || (s2 <= tol2 * *ynorm2);
    if (stop) state[1] = 1;
    pi = (int)(bi % m);
    pj = (int)(bi / m);
    pv = stop ? 1.0 : R[(size_t)pi + (size_t)pj * m];
  }
  __syncthreads();
  if (stop) return;
  const int k = state[0];
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    Y1[(size_t)k * m + i] = R[(size_t)i + (size_t)pj * m];
    Y2[(size_t)k * m + i] = R[(size_t)pi + (size_t)i * m] / pv;
  }
  __syncthreads();
  if (threadIdx.x == 0) state[0] = k + 1;
}

}  // namespace

ProjSolver::ProjSolver(int r, int mmax, hipStream_t st) : r_(r), mmax_(mmax), st_(st) {
  const size_t mm = (size_t)mmax * mmax;
  mbar_u_.alloc((size_t)(mmax + r) * mmax);
  mbar_v_.alloc((size_t)(mmax + r) * mmax);
  a_.alloc(mm); b_.alloc(mm); ai_.alloc(mm); bi_.alloc(mm); c_.alloc(mm); w1_.alloc(mm); w2_.alloc(mm); lu_.alloc(mm);
  ipiv_.alloc(mmax);
  info_.alloc(2);
  scal_.alloc(SCAL_N);
  scratch_.alloc(dense::scratch_doubles());
}

void ProjSolver::form(int d, const ProjSpace& sp, double* Mbar) {
  const int m = d * r_, ld = sp.ld, ldm = m + r_;
  // Mbar = T_{d+1} H_d_bar  ((m + r) x m)
  if (!sp.broken) {
    dense::gemm(false, false, m + r_, m, m + r_, 1.0, sp.T, ld, sp.H, ld, 0.0, Mbar, ldm, st_);
  } else {  // h_{d+1,d} = 0: only T_d H_d, last block row zero
    dense::set_zero(m + r_, m, Mbar, ldm, st_);
    dense::gemm(false, false, m, m, m, 1.0, sp.T, ld, sp.H, ld, 0.0, Mbar, ldm, st_);
  }
  // Mbar <- Mbar T_d^{-1}
  dense::trsm_right_upper(m + r_, m, sp.T, ld, Mbar, ldm, st_);
}

double ProjSolver::solve(int d, const ProjSpace& u, const ProjSpace& v, const double* F11, ProjStats* stats) {
  const int m = d * r_;
  SKR_REQUIRE(m <= mmax_, "projected size exceeds the allocation");
  m_ = m;
  const int ldm = m + r_;
  form(d, u, mbar_u_.p);
  form(d, v, mbar_v_.p);
  dense::copy(m, m, mbar_u_.p, ldm, a_.p, m, st_);
  dense::transpose(m, m, mbar_v_.p, ldm, b_.p, m, st_);
  hipLaunchKernelGGL(rhs_kernel, dim3(std::min(4096, ceil_div((int64_t)m * m, 256))), dim3(256), 0, st_, m, r_, F11,
                     c_.p);
  check_launch("rhs");
  double* s = scal_.p;
  bool scale = true;
  double prev = 1e300;
  int it = 0, extra = -1;
  const int maxit = 100;
  std::vector<double> hs(SCAL_N);
  int hinfo[2];
  for (it = 0; it < maxit; ++it) {
    dense::copy(m, m, a_.p, m, lu_.p, m, st_);
    dense::getrf(m, lu_.p, m, ipiv_.p, info_.p, s + LDA, st_);
    dense::getri(m, lu_.p, m, ipiv_.p, ai_.p, m, st_);
    dense::copy(m, m, b_.p, m, lu_.p, m, st_);
    dense::getrf(m, lu_.p, m, ipiv_.p, info_.p + 1, s + LDB, st_);
    dense::getri(m, lu_.p, m, ipiv_.p, bi_.p, m, st_);
    hipLaunchKernelGGL(mu_kernel, dim3(1), dim3(1), 0, st_, s, m, scale ? 1 : 0);
    check_launch("mu");
    dense::gemm(false, false, m, m, m, 1.0, ai_.p, m, c_.p, m, 0.0, w1_.p, m, st_);
    dense::gemm(false, false, m, m, m, 1.0, w1_.p, m, bi_.p, m, 0.0, w2_.p, m, st_);
    dense::newton_combine(m, m, s + MU, c_.p, m, w2_.p, m, c_.p, m, s + DC, s + NC, nullptr, scratch_.p, st_);
    dense::newton_combine(m, m, s + MU, a_.p, m, ai_.p, m, a_.p, m, s + DA, s + NA, s + TA, scratch_.p, st_);
    dense::newton_combine(m, m, s + MU, b_.p, m, bi_.p, m, b_.p, m, s + DB, s + NB_, s + TB, scratch_.p, st_);
    SKR_HIP(hipMemcpyAsync(hs.data(), s, SCAL_N * sizeof(double), hipMemcpyDeviceToHost, st_));
    SKR_HIP(hipMemcpyAsync(hinfo, info_.p, 2 * sizeof(int), hipMemcpyDeviceToHost, st_));
    SKR_HIP(hipStreamSynchronize(st_));
    if (hinfo[0] || hinfo[1])
      throw Error(SKR_EPROJ, "projected matrix singular during the sign iteration (d = " + std::to_string(d) + ")");
    const double rel = std::sqrt(std::max(hs[DA] / hs[NA], hs[DB] / hs[NB_]));
    if (!std::isfinite(rel))
      throw Error(SKR_EPROJ, "non-finite sign iteration (d = " + std::to_string(d) + ")");
    if (rel < 1e-2) scale = false;
    if (extra >= 0) {
      if (--extra < 0) { ++it; break; }
    } else if (rel < 1e-10 || (rel < 1e-6 && rel > 0.5 * prev)) {
      extra = 1;  // quadratic convergence: one more step reaches rounding level
    }
    prev = rel;
  }
  const int qa = (int)std::lround((m - hs[TA]) / 2.0), qb = (int)std::lround((m - hs[TB]) / 2.0);
  if (stats) {
    stats->newton_iters = it;
    stats->neg_eigs_a = qa;
    stats->neg_eigs_b = qb;
  }
  if (it >= maxit) throw Error(SKR_EPROJ, "sign iteration did not converge (d = " + std::to_string(d) + ")");
  if (qa != 0 || qb != 0)
    throw Error(SKR_EPROJ, "projected matrices have eigenvalues in the left half plane (" + std::to_string(qa) + ", " +
                               std::to_string(qb) + ") at d = " + std::to_string(d) +
                               "; the sign-function solver needs positive real spectra");
  // Y = C / 2:  (mu X + 0 / mu) / 2 with mu = 1
  hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, st_, s + MU, 1.0);
  check_launch("set_scalar");
  dense::copy(m, m, c_.p, m, w1_.p, m, st_);
  dense::set_zero(m, m, w2_.p, m, st_);
  dense::newton_combine(m, m, s + MU, w1_.p, m, w2_.p, m, c_.p, m, s + DC, s + YN2, nullptr, scratch_.p, st_);
  // projected residual ||M_A Y + Y M_B^T - F||_F / ||F||_F (diagnostic)
  dense::gemm(false, false, m, m, m, 1.0, mbar_u_.p, ldm, c_.p, m, 0.0, w1_.p, m, st_);
  dense::gemm(false, true, m, m, m, 1.0, c_.p, m, mbar_v_.p, ldm, 1.0, w1_.p, m, st_);
  hipLaunchKernelGGL(sub_rhs_kernel, dim3(1), dim3(256), 0, st_, m, r_, F11, w1_.p);
  check_launch("sub_rhs");
  dense::fro2(m, m, w1_.p, m, s + RES2, scratch_.p, st_);
  dense::fro2(r_, r_, F11, r_, s + F2, scratch_.p, st_);
  hipLaunchKernelGGL(rho_kernel, dim3(1), dim3(1024), 0, st_, m, r_, c_.p, mbar_u_.p + m + (size_t)(m - r_) * ldm, ldm,
                     mbar_v_.p + m + (size_t)(m - r_) * ldm, ldm, s + RHO2);
  check_launch("rho");
  SKR_HIP(hipMemcpyAsync(hs.data(), s, SCAL_N * sizeof(double), hipMemcpyDeviceToHost, st_));
  SKR_HIP(hipStreamSynchronize(st_));
  if (stats) stats->proj_resid = std::sqrt(hs[RES2] / hs[F2]);
  return std::sqrt(hs[RHO2]);
}

int ProjSolver::factor(double tol) {
  const int m = m_;
  if (!y1_.p) { y1_.alloc((size_t)mmax_ * mmax_); y2_.alloc((size_t)mmax_ * mmax_); }
  if (!acapart_.p) { acapart_.alloc(2 * ACA_G); acaint_.alloc(2 * ACA_G + 4); }
  dense::copy(m, m, c_.p, m, w1_.p, m, st_);
  int* state = acaint_.p + 2 * ACA_G;
  SKR_HIP(hipMemsetAsync(state, 0, 2 * sizeof(int), st_));
  dense::set_zero(m, 1, y1_.p, m, st_);  // a zero Y yields one zero column
  dense::set_zero(m, 1, y2_.p, m, st_);
  const int g = std::max(1, std::min(ACA_G, ceil_div((int64_t)m * m, ACA_WG * 8)));
  const double tol2 = tol > 0 ? tol * tol : 0.0;
  int hstate[2] = {0, 0};
  for (int k = 0; k <= m; ++k) {
    hipLaunchKernelGGL(aca_update_kernel, dim3(g), dim3(ACA_WG), 0, st_, m, w1_.p, y1_.p, y2_.p, state, acapart_.p,
                       acaint_.p);
    check_launch("aca_update");
    hipLaunchKernelGGL(aca_select_kernel, dim3(1), dim3(1024), 0, st_, m, g, w1_.p, y1_.p, y2_.p, state, acapart_.p,
                       acaint_.p, scal_.p + YN2, tol2, m);
    check_launch("aca_select");
    if (k % 16 == 15 || k == m) {
      SKR_HIP(hipMemcpyAsync(hstate, state, 2 * sizeof(int), hipMemcpyDeviceToHost, st_));
      SKR_HIP(hipStreamSynchronize(st_));
      if (hstate[1]) break;
    }
  }
  SKR_HIP(hipMemcpyAsync(hstate, state, 2 * sizeof(int), hipMemcpyDeviceToHost, st_));
  SKR_HIP(hipStreamSynchronize(st_));
  return std::max(1, hstate[0]);
}

}  // namespace skr
