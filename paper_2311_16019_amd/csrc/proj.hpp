// Projected problem of s-PKSM on the device, FP64:
//   M_A = T_{U,d+1} H_d T_{U,d}^{-1} (top dr rows; eqn:Hhat_Ghat), likewise M_B from G, T_V;
//   solve M_A Y + Y M_B^T = E1 beta_1 beta_2^T E1^T (eqn:reduced_sk);
//   rho = sqrt(||hhat E_d^T Y||_F^2 + ||Y E_d ghat^T||_F^2) (eq:resnorm_sk with the whitened
//   subdiagonal blocks hhat = tau_{d+1} h_{d+1,d} tau_d^{-1});
//   low-rank factors Y ~ Y1 Y2^T.
#pragma once

#include <string>

#include <vector>

#include "common.hpp"

namespace skr {

struct ProjSpace {
  const double* H;   // column-major ((maxit+1) r) x (maxit r), leading dimension ld
  const double* T;   // column-major ((maxit+1) r) square, leading dimension ld
  int ld;
  bool broken;       // subdiagonal block of the last column is zero
};

struct ProjStats {
  int newton_iters = 0;
  double proj_resid = 0.0;   // ||M_A Y + Y M_B^T - F||_F / ||F||_F
  int neg_eigs_a = 0, neg_eigs_b = 0;
};

class ProjSolver {
 public:
  ProjSolver(int r, int mmax, hipStream_t st);
  ~ProjSolver();
  ProjSolver(const ProjSolver&) = delete;
  ProjSolver& operator=(const ProjSolver&) = delete;
  // Solve at block step d (m = d r).  F11 is the device r x r block beta_1 beta_2^T
  // (row-major).  Returns rho (absolute).  Throws Error(SKR_EPROJ) when the projected
  // equation cannot be solved by the sign iteration.
  double solve(int d, const ProjSpace& u, const ProjSpace& v, const double* F11, ProjStats* stats);
  // Low-rank factorisation of the last Y by Gaussian elimination with complete pivoting,
  // stopped when ||Y - Y1 Y2^T||_F <= tol ||Y||_F.  Returns ell; Y1, Y2 are m x ell
  // column-major with leading dimension m.
  int factor(double tol);
  // Residual estimate of the truncated Arnoldi method (Algorithm 2):
  // sqrt(d r) (||Y E_d g^T||_F + ||h E_d^T Y||_F) instead of sqrt of the sum of squares.
  void use_truncated_estimate(bool on) { trunc_est_ = on; }
  // Lyapunov equation (M_B = M_A): the sign iterates satisfy B_k = A_k^T, so each step
  // inverts A_k only and transposes.
  void use_lyapunov(bool on) { lyap_ = on; }
  const double* Y1() const { return y1_.p; }
  const double* Y2() const { return y2_.p; }
  int m() const { return m_; }
  const double* Y() const { return c_.p; }
  // Wait for every stream of the solver (after a failed solve, before its buffers are reused).
  void quiesce();

 private:
  void form(int d, const ProjSpace& sp, double* Mbar, hipStream_t st);
  // G = Y P_-(B) for A Y + Y B = F given Al = A (ld lal), B = Mst^T (Mst ld lms), the sign
  // S of B (or of B^T when s_trans) and F from F11 (transposed when f_trans); q = rank P_-.
  void deflate_right(int m, const double* Al, int lal, const double* Mst, int lms, const double* S, int s_trans,
                     const double* F11, int f_trans, int q, double* G);
  int r_, mmax_, m_ = 0;
  bool trunc_est_ = false;
  bool lyap_ = false;
  hipStream_t st_;
  hipStream_t aux_ = nullptr;  // second stream: the two inversions of a Newton step overlap
  hipStream_t cst_ = nullptr;  // third stream: the products for C overlap the next step's eliminations
  hipEvent_t ev_main_ = nullptr, ev_aux_ = nullptr, ev_cin_ = nullptr, ev_c_ = nullptr;
  DBuf<double> lub_;
  DBuf<double> mbar_u_, mbar_v_, a_, b_, ai_, bi_, c_, w1_, w2_, lu_, y1_, y2_;
  DBuf<int> gjw_a_, gjw_b_, info_;
  DBuf<double> gjd_a_, gjd_b_;
  DBuf<double> scal_, scratch_;
  DBuf<double> cscal_, cscratch_;  // mu, change and norm of the C update on its own stream
  DBuf<double> acapart_, dws_, kbuf_;
  // deflated shifted solves: DEFL_NS eliminations at a time, one stream each
  static constexpr int DEFL_NS = 4;
  hipStream_t dst_[DEFL_NS - 2] = {};
  hipEvent_t dev_[DEFL_NS] = {};
  std::vector<DBuf<double>> kbv_;  // one eliminated shifted matrix per distinct shift
  std::vector<DBuf<int>> gjwv_;
  std::vector<DBuf<double>> gjdv_;
  DBuf<double> gapply_;
  DBuf<int> acaint_;
};

}  // namespace skr
