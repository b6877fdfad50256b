// Driver of Algorithm 1 (s-PKSM) on one GPU and the result object.
#pragma once

#include <vector>

#include "op.hpp"
#include "proj.hpp"

namespace skr {
// Kernel families timed with HIP events when params.profile is set.  With the two-pass
// block step "spmm", "dots" and "update" are one kernel each (the CSR block product, the
// window products, the second sweep) and "reduce" the two small reductions of a step.
enum KernelFamily { KF_SPMM = 0, KF_DOTS, KF_REDUCE, KF_UPDATE, KF_SKETCH, KF_WHITEN, KF_COUNT };
inline const char* kernel_family_name(int f) {
  static const char* names[KF_COUNT] = {"spmm", "dots", "reduce", "update", "sketch", "whiten"};
  return (f >= 0 && f < KF_COUNT) ? names[f] : "";
}
}  // namespace skr

struct skr_result_s {
  int64_t fam_launches[skr::KF_COUNT] = {};
  double fam_ms[skr::KF_COUNT] = {};
  int64_t n1 = 0, n2 = 0, ell = 0;
  int32_t iters = 0, status = 0;
  double rho_rel = 0.0;
  std::vector<int32_t> hist_d;
  std::vector<double> hist_rho;
  skr::DBuf<double> X1, X2;  // row-major n x ell
  double ms_steps = 0.0, ms_proj = 0.0, ms_recover = 0.0;
  skr::ProjStats last_stats;
  int32_t failed_checks = 0;  // checks whose projected equation could not be solved (skipped)
};

namespace skr {

// Solve with Krylov spaces K(opU, C1) and K(opV, C2) where opU = A (transposed if tu)
// and opV = B (transposed if tv).  The forward equation uses (A, tu=0) and (B, tv=1).
// B == nullptr (then C2 == C1): the Lyapunov equation opU X + X opU^T = C1 C1^T on the one
// space K(opU, C1) (the V space of B = opU^T, C2 = C1 with S_V = S_U is the same space).
skr_result_s* run_solve(const skr_op_s* A, int tu, const skr_op_s* B, int tv, const double* C1, const double* C2,
                        int r, const skr_params& p, hipStream_t st);

}  // namespace skr
