// Algorithm 1 (s-PKSM) driven from the host, all arithmetic on the device.
//
// Per block step d (both Krylov spaces in every launch):
//   spmm_dot            U~ = Op U_d,  h_{i0,d} = U_{i0}^T U~          (i0 = max(1, d-k+1))
//   axpy_reduce (k x)   U~ -= U_i h_{i,d}; next dot, or the Gram matrix of U~ at i = d
//   gram2 (r > 1)       second Cholesky QR pass; h_{d+1,d} = R
//   normalize           U_{d+1} = U~ R^{-1}
//   sketch              w = S U_{d+1}
//   whiten              Q_{d+1}, T_{d+1} (Prop. 2.1)
// and, when d % p == 0 or d = maxit, the projected solve and the residual estimate
// (one host synchronisation to read rho).  Finally the low-rank factors of Y and the
// recovery X1 = U_d T_U^{-1} Y1, X2 = V_d T_V^{-1} Y2 from the stored basis or by
// regenerating the basis from the stored Hessenberg blocks (two-pass).
//
// With the sketched inner product (params.orth) the step is SpMM, sketch of U~, the
// sketch-space Gram-Schmidt and QR, one update pass over n rows, then the whitening; the
// sketch of U_{d+1} is a by-product of the sketch-space QR.
#include <algorithm>
#include <climits>
#include <cmath>
#include <memory>

#include "blockstep.hpp"
#include "dense.hpp"
#include "solver.hpp"
#include "sorth.hpp"
#include "srht.hpp"
#include "whiten.hpp"

namespace skr {
namespace {

template <typename T>
__global__ void convert_kernel(const double* src, T* dst, size_t count) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x)
    dst[e] = static_cast<T>(src[e]);
}

__global__ void fill_int_kernel(int* p, int v) {
  if (threadIdx.x == 0) *p = v;
}

// beta = T_1 ell for both spaces (T column-major with ld, ell column-major r x r);
// F11 = beta_U beta_V^T (row-major).
// T(i, i) = 1 for i < m (column-major, leading dimension ld); other entries untouched.
__global__ void unit_diag_kernel(int m, double* T, int ld) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) T[i + (size_t)i * ld] = 1.0;
}

__global__ void rhs_block_kernel(int r, const double* TU, int ldu, const double* ellU, const double* TV, int ldv,
                                 const double* ellV, double* F11) {
  __shared__ double bu[RMAX * RMAX], bv[RMAX * RMAX];
  const int e = threadIdx.x;
  if (e < r * r) {
    const int a = e / r, b = e % r;
    double su = 0.0, sv = 0.0;
    for (int c = 0; c < r; ++c) {
      su += TU[a + (size_t)c * ldu] * ellU[c + (size_t)b * r];
      sv += TV[a + (size_t)c * ldv] * ellV[c + (size_t)b * r];
    }
    bu[e] = su;
    bv[e] = sv;
  }
  __syncthreads();
  if (e < r * r) {
    const int a = e / r, b = e % r;
    double t = 0.0;
    for (int c = 0; c < r; ++c) t += bu[a * r + c] * bv[b * r + c];
    F11[e] = t;
  }
}

// COEF <- h_{i,j} block of H (column-major), RFINV <- inverse of h_{j+1,j} (for replay)
__global__ void replay_coef_kernel(int r, const double* Hblk, int ldh, double* small, int want_inv) {
  if (threadIdx.x != 0) return;
  double* coef = small + SmallLayout::COEF;
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < r; ++b) coef[a * r + b] = Hblk[a + (size_t)b * ldh];
  if (want_inv) {
    double* V = small + SmallLayout::RFINV;
    for (int i = 0; i < r * r; ++i) V[i] = 0.0;
    for (int j = 0; j < r; ++j) {
      V[j * r + j] = 1.0 / coef[j * r + j];
      for (int i = j - 1; i >= 0; --i) {
        double s = 0.0;
        for (int k = i + 1; k <= j; ++k) s += coef[i * r + k] * V[k * r + j];
        V[i * r + j] = -s / coef[i * r + i];
      }
    }
  }
}

// COEF <- 0 (so that axpy_reduce with W = Y computes a plain Gram matrix)
__global__ void zero_small_kernel(double* small, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) small[i] = 0.0;
}

// W[(j-1) r : j r, col] <- P_j W[(j-1) r : j r, col] for blocks j = 1 .. d (W column-major,
// leading dimension ldw; P_j row-major r x r at P + j r^2).
// [a | b] -> p for two s x r row-major blocks (both spaces: blockIdx.y)
// the G sketches of a group (s x r row-major each) side by side -> p (s x G r), both spaces
constexpr int GRP_MAX = 16;  // blocks per group at most (r = 1)
struct GroupSrc {
  const double* w[2][GRP_MAX];
  double* p[2];
};
__global__ void pack_group_kernel(int s, int r, int G, GroupSrc src) {
  const int sp = blockIdx.y, L = G * r;
  double* p = src.p[sp];
  const int total = s * L;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int i = e / L, c = e % L, b = c / r;
    const double* w = src.w[sp][0];
#pragma unroll
    for (int t = 1; t < GRP_MAX; ++t)  // constant indices: the array stays in kernel arguments
      if (t == b) w = src.w[sp][t];
    p[e] = w[(size_t)i * r + c % r];
  }
}

__global__ void apply_pending_kernel(int r, int d, int ncol, const double* P, double* W, int ldw) {
  const int total = d * ncol;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int j = 1 + e % d, col = e / d;
    double* w = W + (size_t)(j - 1) * r + (size_t)col * ldw;
    const double* Pj = P + (size_t)j * r * r;
    double x[RMAX];
    for (int c = 0; c < r; ++c) x[c] = w[c];
    for (int a = 0; a < r; ++a) {
      double t = 0.0;
      for (int c = 0; c < r; ++c) t += Pj[a * r + c] * x[c];
      w[a] = t;
    }
  }
}

int step_wgs(int n) {
  int g = ceil_div(n, 4 * WG);
  g = (g + 7) / 8 * 8;
  return std::max(8, std::min(1024, g));
}

// HIP-event timing of kernel families on the solve's stream (params.profile: 1 times every
// family, 2 + f only family f; each timed launch adds two event records to its stream).
class Profiler {
 public:
  Profiler(int mode, hipStream_t st) : on_(mode != 0), only_(mode >= 2 ? mode - 2 : -1), st_(st) {}
  ~Profiler() {
    for (auto& p : pending_) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : pool_) (void)hipEventDestroy(e);
  }
  void begin(int fam, hipStream_t s = nullptr) {
    active_ = on_ && (only_ < 0 || fam == only_);
    if (!active_) return;
    cur_ = {get(), nullptr, fam};
    cur_st_ = s ? s : st_;
    SKR_HIP(hipEventRecord(cur_.a, cur_st_));
  }
  void end() {
    if (!active_) return;
    cur_.b = get();
    SKR_HIP(hipEventRecord(cur_.b, cur_st_));
    pending_.push_back(cur_);
  }
  // call after the stream has been synchronised
  void resolve(skr_result_s* res) {
    for (auto& p : pending_) {
      float ms = 0.f;
      SKR_HIP(hipEventElapsedTime(&ms, p.a, p.b));
      res->fam_launches[p.fam] += 1;
      res->fam_ms[p.fam] += ms;
      pool_.push_back(p.a);
      pool_.push_back(p.b);
    }
    pending_.clear();
  }

 private:
  struct Pair { hipEvent_t a, b; int fam; };
  hipEvent_t get() {
    if (!pool_.empty()) { hipEvent_t e = pool_.back(); pool_.pop_back(); return e; }
    hipEvent_t e;
    SKR_HIP(hipEventCreate(&e));
    return e;
  }
  bool on_, active_ = false;
  int only_;
  hipStream_t st_, cur_st_ = nullptr;
  Pair cur_{};
  std::vector<Pair> pending_;
  std::vector<hipEvent_t> pool_;
};

template <typename T>
struct Space {
  CsrView<T> A;
  int n = 0, nwg = 0, nchunk = 0;
  int nwg2 = 0;  // workgroups of the two-pass sweeps that write partials
  int nslots = 0;
  bool stored = true;
  DBuf<T> basis, work;
  DBuf<double> H, Tm, Q, small, part, skpart, w, w2, c1, c2, wpart, ell;
  DBuf<double> Pall, Gall, Xall, cgs;  // two-pass step: pending factors, Gram blocks, state
  DBuf<int> broken;
  DBuf<uint16_t> tab;
  DBuf<double> skt, sring;  // sketched orthogonalisation: S U~ and the ring of S U_j
  DBuf<double> skpart2, srz2;  // its own sketch workspaces (the sketch of U~ may overlap that of U_j)
  DBuf<double> sopart, sostate;  // partial sums and small state of its sketch-space launches
  int nring = 0;
  SrhtPlan srht;                   // DCT embedding: factorisation and sampled rows
  DBuf<double> srz, srraw;         // its stage-1 workspace and the sketch before the pending factor
  DBuf<int> sroff, srsamp;
  DBuf<double> Z, cz, cstash, zf, fpart, fstate;  // delayed re-orthogonalisation of the sketched QR update
  // sketch of block j: 2G buffers (block index mod 2G, G blocks per whitening group), so
  // that the sketches of the next group can be written while the current one is whitened
  double* wbuf(int j) const { return wq[j % nwq].p; }
  DBuf<double> wq[2 * GRP_MAX];
  int nwq = 4;
  DBuf<double> wgrp;  // whitening in groups: the G sketches side by side (s x G r row-major)
  T* slot(int j) const {  // 1-based basis block j
    const int idx = stored ? (j - 1) : ((j - 1) % nslots);
    return basis.p + (size_t)idx * n * rr;
  }
  int rr = 0;
};

template <typename T>
class Solver {
 public:
  // B == nullptr: the Lyapunov specialisation A X + X A^T = C1 C1^T (one Krylov space; the
  // second space is an empty placeholder that the tandem kernels skip).
  Solver(const skr_op_s* A, int tu, const skr_op_s* B, int tv, int r, const skr_params& p, hipStream_t st)
      : r_(r), p_(p), st_(st), prof_(p.profile, st) {
    lyap_ = (B == nullptr);
    aux_ = stream_acquire();
    aux2_ = stream_acquire();
    for (auto& e : ev_whiten_) SKR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    SKR_HIP(hipEventCreateWithFlags(&ev_block_, hipEventDisableTiming));
    SKR_HIP(hipEventCreateWithFlags(&ev_sketch_, hipEventDisableTiming));
    SKR_HIP(hipEventCreateWithFlags(&ev_aux_done_, hipEventDisableTiming));
    SKR_REQUIRE(r >= 1 && r <= RMAX, "r must be in [1, 16]");
    SKR_REQUIRE(p.k >= 1, "k must be >= 1");
    SKR_REQUIRE(p.maxit >= 1, "maxit must be >= 1");
    SKR_REQUIRE(p.profile >= 0 && p.profile < 2 + KF_COUNT, "profile must be 0, 1 or 2 + a kernel family index");
    SKR_REQUIRE(p.p >= 1, "p must be >= 1");
    SKR_REQUIRE(p.zeta >= 1 && p.zeta <= 64, "zeta must be in [1, 64]");
    SKR_REQUIRE(p.sketch == SKR_SKETCH_SPARSE_SIGN || p.sketch == SKR_SKETCH_SRHT || p.sketch == SKR_SKETCH_NONE,
                "sketch must be SKR_SKETCH_SPARSE_SIGN, SKR_SKETCH_SRHT or SKR_SKETCH_NONE");
    sketched_ = p.sketch != SKR_SKETCH_NONE;
    srht_ = p.sketch == SKR_SKETCH_SRHT;
    SKR_REQUIRE(p.orth == SKR_ORTH_EUCLIDEAN || p.orth == SKR_ORTH_SKETCHED,
                "orth must be SKR_ORTH_EUCLIDEAN or SKR_ORTH_SKETCHED");
    sorth_ = p.orth == SKR_ORTH_SKETCHED;
    resketch_ = sorth_ && sizeof(T) == sizeof(float);
    SKR_REQUIRE(!sorth_ || sketched_, "the sketched inner product needs an embedding");
    SKR_REQUIRE(p.recover == SKR_RECOVER_STORED || p.recover == SKR_RECOVER_TWO_PASS, "invalid recovery mode");
    SKR_REQUIRE(p.tol >= 0.0 && p.trunc_tol >= 0.0, "tolerances must be nonnegative");
    s_ = sketched_ ? p.s : 0;
    if (sketched_) {
      if (s_ == 0) {
        s_ = 2 * (int64_t)p.maxit * r;
        s_ = (s_ + p.zeta - 1) / p.zeta * p.zeta;
      }
      if (!srht_) {
        SKR_REQUIRE(s_ % p.zeta == 0, "s must be a multiple of zeta");
        SKR_REQUIRE(s_ / p.zeta <= 32768, "s / zeta must not exceed 32768");
      }
      SKR_REQUIRE(s_ >= (int64_t)(p.maxit + 1) * r, "s must be at least (maxit+1) r");
      SKR_REQUIRE(s_ < (int64_t(1) << 31), "s too large");
    }
    ld_ = (p.maxit + 1) * r;
    delayed_ = sketched_ && whiten_delayed_supported(r);
    // whitening in groups of G blocks (a G r-wide block per pass): Q is read twice per G
    // blocks.  r = 4: four blocks, 16 columns (the 16-wide kernels need an even s); else pairs
    // when 2r <= 8.  A wider group asks more of the Cholesky QR of the group's remainder: with
    // r = 1 and sixteen blocks per group, a basis that has become numerically dependent (the
    // paper's Ex. 6.1 at nu = 0.001) let a check pass whose estimate no longer matched the true
    // residual, which pairs do not.
    if (delayed_ && !sorth_) {
      if (r == 4 && s_ % 2 == 0) grp_ = 4;
      else if (whiten_delayed_supported(2 * r)) grp_ = 2;
    }
    nwq_ = std::max(4, 2 * grp_);
    fast_ = cgs_supported(r, p.k);
    if (sorth_ && (!fast_ || p.k > 3))
      throw Error(SKR_ENOTSUP, "the sketched-inner-product block step needs r <= 4 and k <= 3");
    if (lyap_ && !fast_) throw Error(SKR_ENOTSUP, "the Lyapunov solve needs the two-pass block step (r <= 4, k <= 10)");
    if (lyap_ && p.recover != SKR_RECOVER_STORED)
      throw Error(SKR_ENOTSUP, "the Lyapunov solve needs stored-basis recovery");
    int dev = 0;
    SKR_HIP(hipGetDevice(&dev));
    int lds = 0;  // one attribute: the whole property structure took about a millisecond per solve
    SKR_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    lds_limit_ = std::max<size_t>(65536, (size_t)lds);
    setup(sp_[0], A, tu);
    setup(sp_[1], lyap_ ? nullptr : B, tv);
    if (srht_) setup_srht();
  }

  ~Solver() {
    if (aux_) (void)hipStreamSynchronize(aux_);
    if (aux2_) (void)hipStreamSynchronize(aux2_);
    (void)hipStreamSynchronize(st_);
    quiet_.enter();  // every buffer below is idle now
    if (ev_block_) (void)hipEventDestroy(ev_block_);
    if (ev_sketch_) (void)hipEventDestroy(ev_sketch_);
    if (ev_aux_done_) (void)hipEventDestroy(ev_aux_done_);
    for (auto e : ev_whiten_)
      if (e) (void)hipEventDestroy(e);
    if (aux_) stream_release(aux_);
    if (aux2_) stream_release(aux2_);
  }
  Solver(const Solver&) = delete;
  Solver& operator=(const Solver&) = delete;

  // The sketch and the sketched QR update of step d run on the auxiliary stream; the
  // solve's stream waits for them before anything reads T, Q or the breakdown flags.
  void join_aux() {  // the whitening stream's last work follows the last sketch
    SKR_HIP(hipEventRecord(ev_aux_done_, aux2_));
    SKR_HIP(hipStreamWaitEvent(st_, ev_aux_done_, 0));
  }

  skr_result_s* run(const double* C1, const double* C2) {
    PoolQuiet quiet;  // entered once all work of this call has completed
    std::unique_ptr<skr_result_s> res(new skr_result_s());
    res->n1 = sp_[0].n;
    res->n2 = lyap_ ? sp_[0].n : sp_[1].n;
    hipEvent_t e0, e1;
    SKR_HIP(hipEventCreate(&e0));
    SKR_HIP(hipEventCreate(&e1));
    struct EvGuard { hipEvent_t a, b; ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } eg{e0, e1};
    SKR_HIP(hipEventRecord(e0, st_));
    init(C1, C2);
    double rhs = 0.0;
    SKR_HIP(hipMemcpyAsync(&rhs_block_host_[0], F11_.p, sizeof(double) * r_ * r_, hipMemcpyDeviceToHost, st_));
    int hb[2];
    SKR_HIP(hipMemcpyAsync(&hb[0], sp_[0].broken.p, sizeof(int), hipMemcpyDeviceToHost, st_));
    SKR_HIP(hipMemcpyAsync(&hb[1], sp_[1].broken.p, sizeof(int), hipMemcpyDeviceToHost, st_));
    SKR_HIP(hipStreamSynchronize(st_));
    if (lyap_) hb[1] = hb[0];
    if (hb[0] != INT_MAX || hb[1] != INT_MAX)
      throw Error(SKR_EINVAL, "right-hand side factor is rank deficient or its sketch is singular");
    for (int i = 0; i < r_ * r_; ++i) rhs += rhs_block_host_[i] * rhs_block_host_[i];
    rhs = std::sqrt(rhs);
    SKR_REQUIRE(rhs > 0.0 && std::isfinite(rhs), "zero or non-finite right-hand side");

    ProjSolver proj(r_, p_.maxit * r_, st_);
    proj.use_truncated_estimate(!sketched_);
    proj.use_lyapunov(lyap_);
    int status = SKR_NOT_CONVERGED, dfinal = 0, dgood = 0;  // dgood: last check whose projected solve succeeded
    double rho_rel = 0.0;
    for (int d = 1; d <= p_.maxit; ++d) {
      block_step(d);
      if (d % p_.p == 0 || d == p_.maxit) {
        if (sketched_) {
          prof_.begin(KF_WHITEN, aux2_);
          flush_whiten(d, aux2_);
          prof_.end();
        }
        join_aux();
        SKR_HIP(hipMemcpyAsync(&hb[0], sp_[0].broken.p, sizeof(int), hipMemcpyDeviceToHost, st_));
        SKR_HIP(hipMemcpyAsync(&hb[1], sp_[1].broken.p, sizeof(int), hipMemcpyDeviceToHost, st_));
        SKR_HIP(hipEventRecord(e1, st_));
        SKR_HIP(hipEventSynchronize(e1));
        if (lyap_) hb[1] = hb[0];
        float ms = 0.f;
        SKR_HIP(hipEventElapsedTime(&ms, e0, e1));
        res->ms_steps += ms;
        prof_.resolve(res.get());
        const int db = std::min(hb[0], hb[1]);
        int dc = std::min(d, db);
        const bool broke = db <= d;
        SKR_REQUIRE(dc >= 1, "breakdown in the first block step");
        SKR_HIP(hipEventRecord(e0, st_));
        auto pspaces = [&](int dd) {
          ProjSpace pu{sp_[0].H.p, sp_[0].Tm.p, ld_, hb[0] == dd};
          ProjSpace pv = lyap_ ? pu : ProjSpace{sp_[1].H.p, sp_[1].Tm.p, ld_, hb[1] == dd};
          return std::make_pair(pu, pv);
        };
        const auto [pu, pv] = pspaces(dc);
        const bool last_check = broke || d == p_.maxit;
        double rho = 0.0;
        bool solved = true;
        try {
          rho = proj.solve(dc, pu, pv, F11_.p, &res->last_stats);
        } catch (const Error& e) {
          // The projected equation could not be solved at this check (its sketched matrices
          // have eigenvalue pairs the sign iteration cannot separate, which happens when the
          // truncated bases are numerically dependent).  Go on to the next check; at the
          // last one, return the factors of the last check that was solved.
          if (e.code != SKR_EPROJ || (last_check && dgood == 0)) throw;
          proj.quiesce();
          solved = false;
          ++res->failed_checks;
        }
        if (!solved && last_check) {
          const auto [gu, gv] = pspaces(dgood);
          rho = proj.solve(dgood, gu, gv, F11_.p, &res->last_stats);
          dc = dgood;
        }
        SKR_HIP(hipEventRecord(e1, st_));
        SKR_HIP(hipEventSynchronize(e1));
        SKR_HIP(hipEventElapsedTime(&ms, e0, e1));
        res->ms_proj += ms;
        SKR_HIP(hipEventRecord(e0, st_));
        if (solved || last_check) {
          rho_rel = rho / rhs;
          if (solved) {
            res->hist_d.push_back(dc);
            res->hist_rho.push_back(rho_rel);
            dgood = dc;
          }
          dfinal = dc;
        }
        if (!solved && last_check) break;  // NOT_CONVERGED with the last solved check
        if (broke) { status = SKR_BREAKDOWN; break; }
        if (solved && rho_rel <= p_.tol) { status = SKR_OK; break; }
      }
    }
    // factors and recovery
    SKR_HIP(hipEventRecord(e0, st_));
    const int m = dfinal * r_;
    int ell = proj.factor(p_.trunc_tol);
    DBuf<double> W1((size_t)m * ell), W2((size_t)m * ell);
    dense::copy(m, ell, proj.Y1(), m, W1.p, m, st_);
    dense::copy(m, ell, proj.Y2(), m, W2.p, m, st_);
    Space<T>& sv = lyap_ ? sp_[0] : sp_[1];  // the second space of the factors
    // the two triangular solves (chains of small launches) concurrently
    SKR_HIP(hipEventRecord(ev_block_, st_));
    SKR_HIP(hipStreamWaitEvent(aux_, ev_block_, 0));
    dense::trsm_left_upper(m, ell, sp_[0].Tm.p, ld_, W1.p, m, st_);
    dense::trsm_left_upper(m, ell, sv.Tm.p, ld_, W2.p, m, aux_);
    SKR_HIP(hipEventRecord(ev_aux_done_, aux_));
    SKR_HIP(hipStreamWaitEvent(st_, ev_aux_done_, 0));
    res->X1.alloc((size_t)sp_[0].n * ell);
    res->X2.alloc((size_t)sv.n * ell);
    if (p_.recover == SKR_RECOVER_STORED) {
      if (fast_ && !sorth_) {  // U_j = U'_j P_j: X = sum_j U'_j (P_j W[j])
        const int g = std::max(1, std::min(4096, ceil_div((int64_t)dfinal * ell, 256)));
        hipLaunchKernelGGL(apply_pending_kernel, dim3(g), dim3(256), 0, st_, r_, dfinal, ell, sp_[0].Pall.p, W1.p, m);
        hipLaunchKernelGGL(apply_pending_kernel, dim3(g), dim3(256), 0, st_, r_, dfinal, ell, sv.Pall.p, W2.p, m);
        check_launch("apply_pending");
      }
      dense::basis_gemm<T>(sp_[0].n, r_, dfinal, ell, 1.0, sp_[0].basis.p, W1.p, m, 0.0, res->X1.p, ell, st_);
      dense::basis_gemm<T>(sv.n, r_, dfinal, ell, 1.0, sv.basis.p, W2.p, m, 0.0, res->X2.p, ell, st_);
    } else {
      replay(C1, C2, dfinal, ell, W1.p, W2.p, res->X1.p, res->X2.p);
    }
    SKR_HIP(hipEventRecord(e1, st_));
    SKR_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    SKR_HIP(hipEventElapsedTime(&ms, e0, e1));
    res->ms_recover = ms;
    res->ell = ell;
    res->iters = dfinal;
    res->status = status;
    res->rho_rel = rho_rel;
    quiet.enter();  // st_ has completed (e1); the projected solver waits for its own streams
    return res.release();
  }

 private:
  void setup(Space<T>& s, const skr_op_s* op, int t) {
    s.A = op ? csr_view<T>(op, t) : CsrView<T>{};  // no operator: an empty space (n = 0)
    s.n = op ? (int)op->n : 0;
    s.rr = r_;
    s.nwg = step_wgs(s.n);
    s.nwg2 = cgs_wgs(s.n);
    s.stored = (p_.recover == SKR_RECOVER_STORED);
    s.nslots = s.stored ? (p_.maxit + 1) : (p_.k + 1);
    s.basis.alloc((size_t)s.nslots * s.n * r_);
    s.work.alloc((size_t)s.n * r_);
    s.H.alloc((size_t)ld_ * p_.maxit * r_);
    s.Tm.alloc((size_t)ld_ * ld_);
    s.Q.alloc((size_t)s_ * ld_);
    s.small.alloc(SmallLayout::SIZE);
    s.part.alloc((size_t)s.nwg * std::max(RMAX * RMAX + 8, (CGS_KMAX + 1) * r_ * r_));
    if (fast_) {
      const size_t rr = (size_t)r_ * r_, nb = (size_t)p_.maxit + 2;
      s.Pall.alloc(nb * rr);
      s.Gall.alloc(nb * rr);
      s.Xall.alloc(nb * CGS_KMAX * rr);
      s.cgs.alloc(cgs_state_doubles());
      s.Pall.zero(st_);
      s.Gall.zero(st_);
      s.Xall.zero(st_);
      s.cgs.zero(st_);
    }
    s.broken.alloc(1);
    s.nchunk = sketch_chunks(s.n, lyap_ ? 1 : 2);
    if (!srht_) s.skpart.alloc((size_t)s.nchunk * s_ * r_);
    s.nwq = nwq_;
    for (int j = 0; j < nwq_; ++j) s.wq[j].alloc((size_t)s_ * r_);
    s.c1.alloc((size_t)ld_ * r_);
    s.c2.alloc((size_t)ld_ * r_);
    const int rw = grp_ * r_;  // width of a whitened block
    s.wpart.alloc(whiten_part_doubles((int)s_, delayed_ ? 2 * rw : rw, p_.maxit * r_));
    if (delayed_ && s.n > 0) {
      s.Z.alloc((size_t)s_ * 2 * rw);
      s.cz.alloc((size_t)ld_ * 2 * rw);
      s.cstash.alloc((size_t)ld_ * rw);
      s.zf.alloc((size_t)s_ * rw);
      if (grp_ > 1) s.wgrp.alloc((size_t)s_ * rw);
      s.fpart.alloc(whiten_fin_doubles());
      s.fstate.alloc(whiten_fin_state_doubles());
    }
    s.ell.alloc((size_t)r_ * r_);
    if (sketched_ && !srht_) s.tab.alloc((size_t)s.n * p_.zeta);
    if (sorth_) {
      if (!srht_) s.skpart2.alloc((size_t)s.nchunk * s_ * r_);
      s.nring = p_.k + 1;
      s.sopart.alloc(sorth_part_doubles());
      s.sostate.alloc(sorth_state_doubles());
      s.skt.alloc((size_t)s_ * r_);
      s.sring.alloc((size_t)s.nring * s_ * r_);
    }
    s.H.zero(st_);
    s.Tm.zero(st_);
    s.small.zero(st_);
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(1), 0, st_, s.broken.p, INT_MAX);
    check_launch("fill_int");
  }

  SpaceStep<T> step_args(Space<T>& s, int d) {
    SpaceStep<T> a{};
    a.A = s.A;
    a.Y = s.work.p;
    a.small = s.small.p;
    a.part = s.part.p;
    a.broken = s.broken.p;
    a.ldh = ld_;
    a.n = s.n;
    a.nwg = s.nwg;
    a.step = d;
    return a;
  }

  double* Hblk(Space<T>& s, int i, int j) {  // 1-based block (i, j)
    return s.H.p + (size_t)(i - 1) * r_ + (size_t)(j - 1) * r_ * ld_;
  }

  // Orthonormalise the start block: U_1 ell = C (Cholesky QR, twice for r > 1).
  void start_block(Space<T>& s, const double* C, SpaceStep<T>& a) {
    const size_t cnt = (size_t)s.n * r_;
    hipLaunchKernelGGL(convert_kernel<T>, dim3(std::min<size_t>(4096, (cnt + 255) / 256)), dim3(256), 0, st_, C,
                       s.work.p, cnt);
    check_launch("convert");
    hipLaunchKernelGGL(zero_small_kernel, dim3(1), dim3(256), 0, st_, s.small.p, (int)SmallLayout::SIZE);
    check_launch("zero_small");
    a.W = s.work.p;
    a.Wn = nullptr;
    a.post = POST_GRAM1;
    a.Hblk = (r_ == 1) ? s.ell.p : nullptr;
    a.ldh = r_;
  }

  CgsPass<T> cgs_args(Space<T>& s, int d, int nw, int i0) {
    CgsPass<T> a{};
    a.A = s.A;
    a.X = d >= 1 ? s.slot(d) : nullptr;
    a.Pd = (d >= 1 && !sorth_) ? s.Pall.p + (size_t)d * r_ * r_ : nullptr;
    a.Y = s.work.p;
    a.Unew = s.slot(d + 1);
    for (int i = 0; i < nw; ++i) a.W[i] = s.slot(i0 + i);
    a.coef = s.cgs.p + cgs_coef_offset();
    a.part = s.part.p;
    a.n = s.n;
    a.nwg = s.nwg2;
    return a;
  }

  CgsSmall cgs_small(Space<T>& s, double* H, int ldh) {
    CgsSmall m{};
    m.part = s.part.p;
    m.nwg = s.nwg2;
    m.Pall = s.Pall.p;
    m.Gall = s.Gall.p;
    m.Xall = s.Xall.p;
    m.state = s.cgs.p;
    m.H = H;
    m.ldh = ldh;
    m.broken = s.broken.p;
    return m;
  }

  // Start block U_1 ell = C with the two-pass kernels (no window): U'_1 = C R1^{-1},
  // ell = R2 R1, P_1 = R2^{-1}.
  void init_two_pass(const double* C1, const double* C2) {
    CgsPass<T> a[2];
    const double* Cs[2] = {C1, C2};
    for (int q = 0; q < 2; ++q) {
      a[q] = cgs_args(sp_[q], 0, 0, 1);
      a[q].src = Cs[q];
    }
    const CgsSmall m0 = cgs_small(sp_[0], sp_[0].ell.p, r_), m1 = cgs_small(sp_[1], sp_[1].ell.p, r_);
    launch_cgs_spmm<T>(r_, a[0], a[1], st_);
    launch_cgs_dots<T>(r_, 0, a[0], a[1], st_);
    launch_cgs_reduce1(r_, 0, 1, 0, m0, m1, st_);
    launch_cgs_pass2<T>(r_, 0, a[0], a[1], st_);
    launch_cgs_reduce2(r_, 0, 1, 0, m0, m1, st_);
  }

  void init(const double* C1, const double* C2) {
    if (sorth_) {
      init_sorth(C1, C2);
      return;
    }
    if (fast_) {
      init_two_pass(C1, C2);
      init_sketch();
      return;
    }
    SpaceStep<T> a0 = step_args(sp_[0], 0), a1 = step_args(sp_[1], 0);
    start_block(sp_[0], C1, a0);
    start_block(sp_[1], C2, a1);
    launch_axpy_reduce<T>(r_, a0, a1, st_);
    if (r_ > 1) {
      a0.post = a1.post = POST_GRAM2;
      a0.Hblk = sp_[0].ell.p;
      a1.Hblk = sp_[1].ell.p;
      launch_gram2<T>(r_, a0, a1, st_);
    }
    a0.Unew = sp_[0].slot(1);
    a1.Unew = sp_[1].slot(1);
    launch_normalize<T>(r_, a0, a1, st_);
    init_sketch();
  }

  // Sketched inner product: U_1 = C ell^{-1} with ell the R factor of S C, so that S U_1
  // has orthonormal columns; S U_1 is taken from the QR of S C.
  void init_sorth(const double* C1, const double* C2) {
    CgsPass<T> a[2];
    const double* Cs[2] = {C1, C2};
    for (int q = 0; q < 2; ++q) {
      a[q] = cgs_args(sp_[q], 0, 0, 1);
      a[q].src = Cs[q];
    }
    launch_cgs_spmm<T>(r_, a[0], a[1], st_);  // U~ = C in the basis precision
    build_tables();
    sketch_work(st_);
    launch_sorth(r_, (int)s_, 0, 1, 0, sorth_args(sp_[0], sp_[0].ell.p, r_, 1),
                 sorth_args(sp_[1], sp_[1].ell.p, r_, 1), lyap_ ? 1 : 2, st_);
    launch_cgs_pass2<T>(r_, 0, a[0], a[1], st_);  // U_1 = U~ ell^{-1}
    if (resketch_) sketch(1, st_);  // the whitening takes S U_1 of the stored (rounded) block
    whiten(0, 0, st_);
    rhs_block();
  }

  // DCT embedding of each space: plan (host, cached), stage-1 workspace, sampled rows
  void setup_srht() {
    const uint64_t seeds[2] = {p_.seed, mix64_host(p_.seed + 1)};
    for (int q = 0; q < 2; ++q) {
      Space<T>& s = sp_[q];
      if (s.n == 0) continue;
      s.srht = srht_plan(s.n, (int)s_, seeds[q]);
      s.srz.alloc(srht_z_doubles(s.n, r_));
      if (sorth_) s.srz2.alloc(srht_z_doubles(s.n, r_));
      s.srraw.alloc((size_t)s_ * r_);
      s.sroff.alloc(s.srht.soff.size());
      s.srsamp.alloc(s.srht.samp.size());
      SKR_HIP(hipMemcpyAsync(s.sroff.p, s.srht.soff.data(), sizeof(int) * s.srht.soff.size(), hipMemcpyHostToDevice,
                             st_));
      SKR_HIP(hipMemcpyAsync(s.srsamp.p, s.srht.samp.data(), sizeof(int) * s.srht.samp.size(),
                             hipMemcpyHostToDevice, st_));
    }
  }

  SrhtSpace<T> srht_args(Space<T>& s, const T* U, double* w, const double* pend, bool second_ws = false) {
    SrhtSpace<T> a{};
    a.U = U;
    a.Z = second_ws ? s.srz2.p : s.srz.p;
    a.soff = s.sroff.p;
    a.samp = s.srsamp.p;
    a.wraw = pend ? s.srraw.p : w;
    a.w = w;
    a.Pend = pend;
    a.n = s.n;
    a.N1 = s.srht.N1;
    a.N2 = s.srht.N2;
    a.P = s.srht.P;
    a.Q = s.srht.Q;
    a.seed = s.srht.seed;
    return a;
  }

  SorthSpace sorth_args(Space<T>& s, double* H, int ldh, int j) {
    return SorthSpace{s.skt.p,  s.sring.p, s.nring,    resketch_ ? nullptr : s.wbuf(j), s.cgs.p + cgs_coef_offset(),
                      H,        ldh,       s.broken.p, s.sopart.p,                      s.sostate.p};
  }

  // w = S U~ for the block in the work buffer (both spaces), in workspaces of its own
  void sketch_work(hipStream_t st) {
    if (srht_) {
      launch_srht<T>(r_, (int)s_, srht_args(sp_[0], sp_[0].work.p, sp_[0].skt.p, nullptr, true),
                     srht_args(sp_[1], sp_[1].work.p, sp_[1].skt.p, nullptr, true), lyap_ ? 1 : 2, lds_limit_, st);
      return;
    }
    SketchSpace<T> k0{sp_[0].work.p, sp_[0].tab.p, sp_[0].skpart2.p, sp_[0].skt.p, sp_[0].n, sp_[0].nchunk, 0};
    SketchSpace<T> k1{sp_[1].work.p, sp_[1].tab.p, sp_[1].skpart2.p, sp_[1].skt.p, sp_[1].n, sp_[1].nchunk, 0};
    launch_sketch_pending<T>(r_, (int)s_, p_.zeta, k0, k1, nullptr, nullptr, lds_limit_, st);
  }

  void build_tables() {
    if (srht_) return;  // the DCT embedding draws its signs on the fly
    const uint64_t seeds[2] = {p_.seed, mix64_host(p_.seed + 1)};
    for (int i = 0; i < 2; ++i)
      if (sp_[i].n > 0)  // the Lyapunov solve's empty placeholder space has no table
        launch_build_sketch_table(sp_[i].tab.p, sp_[i].n, p_.zeta, (int)(s_ / p_.zeta), seeds[i], st_);
  }

  // F11 = (T_U ell_U)(T_V ell_V)^T, the first block of the projected right-hand side
  void rhs_block() {
    F11_.alloc((size_t)r_ * r_);
    hipLaunchKernelGGL(rhs_block_kernel, dim3(1), dim3(256), 0, st_, r_, sp_[0].Tm.p, ld_, sp_[0].ell.p,
                       second().Tm.p, ld_, second().ell.p, F11_.p);
    check_launch("rhs_block");
    rhs_block_host_.assign((size_t)r_ * r_, 0.0);
  }

  // Sketch tables, S U_1, the first whitening step and F11 = beta_1 beta_2^T.
  void init_sketch() {
    if (!sketched_) {  // t-PKSM: T = I, so M = H and beta = ell
      for (int i = 0; i < 2; ++i) {
        hipLaunchKernelGGL(unit_diag_kernel, dim3(ceil_div(ld_, 256)), dim3(256), 0, st_, ld_, sp_[i].Tm.p, ld_);
        check_launch("unit_diag");
      }
      rhs_block();
      return;
    }
    build_tables();
    sketch(1, st_);
    whiten(0, 0, st_);
    rhs_block();
  }

  // The second space of the equation: the V space, or the U space again for Lyapunov.
  const Space<T>& second() const { return lyap_ ? sp_[0] : sp_[1]; }

  static uint64_t mix64_host(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }

  void sketch(int j, hipStream_t s) {
    if (srht_) {
      const size_t off = (size_t)j * r_ * r_;
      const bool pend = fast_ && !sorth_;  // the sketched-inner-product step stores final blocks
      launch_srht<T>(r_, (int)s_, srht_args(sp_[0], sp_[0].slot(j), sp_[0].wbuf(j), pend ? sp_[0].Pall.p + off : nullptr),
                     srht_args(sp_[1], sp_[1].slot(j), sp_[1].wbuf(j), pend ? sp_[1].Pall.p + off : nullptr),
                     lyap_ ? 1 : 2, lds_limit_, s);
      return;
    }
    SketchSpace<T> k0{sp_[0].slot(j), sp_[0].tab.p, sp_[0].skpart.p, sp_[0].wbuf(j), sp_[0].n, sp_[0].nchunk};
    SketchSpace<T> k1{sp_[1].slot(j), sp_[1].tab.p, sp_[1].skpart.p, sp_[1].wbuf(j), sp_[1].n, sp_[1].nchunk};
    const size_t off = (size_t)j * r_ * r_;
    const bool pend = fast_ && !sorth_;  // the sketched-inner-product step stores final blocks
    launch_sketch_pending<T>(r_, (int)s_, p_.zeta, k0, k1, pend ? sp_[0].Pall.p + off : nullptr,
                             pend ? sp_[1].Pall.p + off : nullptr, lds_limit_, s);
  }

  WhitenSpace whiten_space(Space<T>& sp, int d, bool group = false) {
    WhitenSpace w{sp.Q.p, sp.Tm.p, group ? sp.wgrp.p : sp.wbuf(d + 1), sp.c1.p, sp.c2.p, sp.wpart.p, sp.broken.p, ld_};
    w.Z = sp.Z.p;
    w.cz = sp.cz.p;
    w.cstash = sp.cstash.p;
    w.zf = sp.zf.p;
    w.fpart = sp.fpart.p;
    w.fstate = sp.fstate.p;
    return w;
  }

  // Sketched QR update with the sketch of block d + 1 in wbuf(d + 1).  Without delayed
  // re-orthogonalisation (r > 8, or the first block) block d + 1 is appended at once.  With
  // it, the new block is projected once against Q and left pending, and the block pending
  // before is finished and appended in the same two sweeps over Q.  In groups (grp_ > 1),
  // blocks wait until grp_ of them are there, and their sketches go through these steps as
  // one (grp_ r)-wide block.  The host tracks the columns of Q already final (fin_cols_), the
  // width of the pending block (pend_w_) and the blocks waiting (held_);
  // ev_whiten_[j mod nwq_] is recorded after the work that read wbuf(j).
  void whiten(int d, int step, hipStream_t s) {
    const int ns = lyap_ ? 1 : 2;
    if (!delayed_ || d == 0) {
      const WhitenSpace w0 = whiten_space(sp_[0], d), w1 = whiten_space(sp_[1], d);
      launch_whiten(r_, (int)s_, fin_cols_, step, w0, w1, s, ns);
      fin_cols_ += r_;
      SKR_HIP(hipEventRecord(ev_whiten_[(d + 1) % nwq_], s));
      return;
    }
    const bool group = grp_ > 1;
    if (group && ++held_ < grp_) return;  // block d + 1 waits for the rest of its group
    const int w = grp_ * r_;
    if (group) {  // wbuf(d + 2 - grp_) .. wbuf(d + 1) side by side -> wgrp
      GroupSrc src{};
      for (int q = 0; q < 2; ++q) {
        Space<T>& sp = sp_[lyap_ ? 0 : q];
        for (int t = 0; t < GRP_MAX; ++t) src.w[q][t] = sp.wbuf(d + 2 - grp_ + std::min(t, grp_ - 1));
        src.p[q] = sp.wgrp.p;
      }
      const int mv = std::max(1, std::min(2048, ceil_div((int64_t)s_ * w, 256)));
      hipLaunchKernelGGL(pack_group_kernel, dim3(mv, ns), dim3(256), 0, s, (int)s_, r_, grp_, src);
      check_launch("pack_group");
      for (int j = d + 2 - grp_; j <= d + 1; ++j) SKR_HIP(hipEventRecord(ev_whiten_[j % nwq_], s));
      held_ = 0;
    }
    const WhitenSpace w0 = whiten_space(sp_[0], d, group), w1 = whiten_space(sp_[1], d, group);
    const int first_step = d + 1 - grp_;  // the step that produced the new block's first block
    if (pend_w_ == 0) {
      launch_whiten_delayed(w, (int)s_, fin_cols_, first_step, WHITEN_FIRST, w0, w1, s, ns);
    } else {
      launch_whiten_delayed(w, (int)s_, fin_cols_, pend_step_, WHITEN_APPEND, w0, w1, s, ns);
      fin_cols_ += pend_w_;
    }
    pend_w_ = w;
    pend_step_ = first_step;
    if (!group) SKR_HIP(hipEventRecord(ev_whiten_[(d + 1) % nwq_], s));  // the sweeps read wbuf(d + 1)
  }

  // Finish every block up to d + 1 (before a projected solve, which reads all of T): the
  // pending block, then the blocks still waiting for the rest of their group, one by one.
  void flush_whiten(int d, hipStream_t s) {
    if (!delayed_) return;
    const int ns = lyap_ ? 1 : 2;
    if (pend_w_ > 0) {
      const WhitenSpace w0 = whiten_space(sp_[0], d), w1 = whiten_space(sp_[1], d);
      launch_whiten_delayed(pend_w_, (int)s_, fin_cols_, pend_step_, WHITEN_FLUSH, w0, w1, s, ns);
      fin_cols_ += pend_w_;
      pend_w_ = 0;
    }
    for (int j = d + 2 - held_; j <= d + 1; ++j) {  // block j, sketched at step j - 1
      const WhitenSpace w0 = whiten_space(sp_[0], j - 1), w1 = whiten_space(sp_[1], j - 1);
      launch_whiten(r_, (int)s_, fin_cols_, j - 1, w0, w1, s, ns);
      fin_cols_ += r_;
      SKR_HIP(hipEventRecord(ev_whiten_[j % nwq_], s));
    }
    held_ = 0;
    SKR_REQUIRE(fin_cols_ == (d + 1) * r_, "sketched QR update out of step with the block steps");
  }

  // Two-pass block step (r <= 4, k <= 10): pass 1 + reduce 1, pass 2 + reduce 2.
  void block_step_two_pass(int d) {
    const int i0 = std::max(1, d - p_.k + 1), nw = d - i0 + 1;
    CgsPass<T> a[2];
    for (int q = 0; q < 2; ++q) a[q] = cgs_args(sp_[q], d, nw, i0);
    const CgsSmall m0 = cgs_small(sp_[0], sp_[0].H.p, ld_), m1 = cgs_small(sp_[1], sp_[1].H.p, ld_);
    prof_.begin(KF_SPMM);
    launch_cgs_spmm<T>(r_, a[0], a[1], st_);
    prof_.end();
    prof_.begin(KF_DOTS);
    launch_cgs_dots<T>(r_, nw, a[0], a[1], st_);
    prof_.end();
    prof_.begin(KF_REDUCE);
    launch_cgs_reduce1(r_, nw, i0, d, m0, m1, st_);
    prof_.end();
    if (!sp_[0].stored) {
      // ring buffer: slot(d+1) held U_{d+1-nslots}; its sketch (issued earlier on the
      // auxiliary stream) must be complete before the slot is overwritten
      SKR_HIP(hipStreamWaitEvent(st_, ev_sketch_, 0));
    }
    prof_.begin(KF_UPDATE);
    launch_cgs_pass2<T>(r_, nw, a[0], a[1], st_);
    prof_.end();
    prof_.begin(KF_REDUCE);
    launch_cgs_reduce2(r_, nw, i0, d, m0, m1, st_);
    prof_.end();
    after_step(d);
  }

  // Sketched-inner-product block step: U~ = Op U_d and its sketch, the sketch-space
  // Gram-Schmidt and QR (one workgroup per space), then U_{d+1} in one pass over n rows.
  void block_step_sorth(int d) {
    const int i0 = std::max(1, d - p_.k + 1), nw = d - i0 + 1;
    CgsPass<T> a[2];
    for (int q = 0; q < 2; ++q) a[q] = cgs_args(sp_[q], d, nw, i0);
    prof_.begin(KF_SPMM);
    launch_cgs_spmm<T>(r_, a[0], a[1], st_);
    prof_.end();
    prof_.begin(KF_SKETCH);
    sketch_work(st_);
    prof_.end();
    // the sketch-space step writes the whitening input wbuf(d + 1), which the whitening of
    // step d - 4 read
    SKR_HIP(hipStreamWaitEvent(st_, ev_whiten_[(d + 1) % nwq_], 0));
    prof_.begin(KF_REDUCE);
    launch_sorth(r_, (int)s_, nw, i0, d, sorth_args(sp_[0], sp_[0].H.p, ld_, d + 1),
                 sorth_args(sp_[1], sp_[1].H.p, ld_, d + 1), lyap_ ? 1 : 2, st_);
    prof_.end();
    if (resketch_ && !sp_[0].stored) {
      // ring buffer: slot(d+1) held U_{d+1-nslots}, whose sketch runs on the auxiliary stream
      SKR_HIP(hipStreamWaitEvent(st_, ev_sketch_, 0));
    }
    prof_.begin(KF_UPDATE);
    launch_cgs_pass2<T>(r_, nw, a[0], a[1], st_);
    prof_.end();
    after_step(d);
  }

  // U_{d+1} is final: sketch it (stream aux_) and update Q, T (stream aux2_) concurrently
  // with the next block step; the sketch of block d + 2 overlaps this whitening.
  void after_step(int d) {
    if (!sketched_) return;  // t-PKSM: no embedding
    if (sorth_ && !resketch_) {  // S U_{d+1} is already in wbuf(d + 1)
      SKR_HIP(hipEventRecord(ev_block_, st_));
      SKR_HIP(hipStreamWaitEvent(aux2_, ev_block_, 0));
      prof_.begin(KF_WHITEN, aux2_);
      whiten(d, d, aux2_);
      prof_.end();
      return;
    }
    SKR_HIP(hipEventRecord(ev_block_, st_));
    SKR_HIP(hipStreamWaitEvent(aux_, ev_block_, 0));
    // the whitening of block d - 3 read the buffer that the sketch of block d + 1 writes
    SKR_HIP(hipStreamWaitEvent(aux_, ev_whiten_[(d + 1) % nwq_], 0));
    prof_.begin(KF_SKETCH, aux_);
    sketch(d + 1, aux_);
    prof_.end();
    SKR_HIP(hipEventRecord(ev_sketch_, aux_));
    SKR_HIP(hipStreamWaitEvent(aux2_, ev_sketch_, 0));
    prof_.begin(KF_WHITEN, aux2_);
    whiten(d, d, aux2_);
    prof_.end();
  }

  void block_step(int d) {
    if (sorth_) {
      block_step_sorth(d);
      return;
    }
    if (fast_) {
      block_step_two_pass(d);
      return;
    }
    const int i0 = std::max(1, d - p_.k + 1);
    SpaceStep<T> a[2];
    for (int q = 0; q < 2; ++q) {
      Space<T>& s = sp_[q];
      a[q] = step_args(s, d);
      a[q].X = s.slot(d);
      a[q].W = s.slot(i0);
      a[q].post = POST_DOT;
      a[q].Hblk = Hblk(s, i0, d);
    }
    prof_.begin(KF_SPMM);
    launch_spmm_dot<T>(r_, a[0], a[1], st_);
    prof_.end();
    for (int i = i0; i <= d; ++i) {
      for (int q = 0; q < 2; ++q) {
        Space<T>& s = sp_[q];
        a[q].W = s.slot(i);
        if (i < d) {
          a[q].Wn = s.slot(i + 1);
          a[q].post = POST_DOT;
          a[q].Hblk = Hblk(s, i + 1, d);
        } else {
          a[q].Wn = nullptr;
          a[q].post = POST_GRAM1;
          a[q].Hblk = (r_ == 1) ? Hblk(s, d + 1, d) : nullptr;
        }
      }
      prof_.begin(KF_DOTS);
      launch_axpy_reduce<T>(r_, a[0], a[1], st_);
      prof_.end();
    }
    if (r_ > 1) {
      for (int q = 0; q < 2; ++q) {
        a[q].post = POST_GRAM2;
        a[q].Hblk = Hblk(sp_[q], d + 1, d);
      }
      prof_.begin(KF_UPDATE);
      launch_gram2<T>(r_, a[0], a[1], st_);
      prof_.end();
    }
    for (int q = 0; q < 2; ++q) a[q].Unew = sp_[q].slot(d + 1);
    if (!sp_[0].stored) {
      // ring buffer: slot(d+1) held U_{d+1-nslots}; its sketch (issued earlier on the
      // auxiliary stream) must be complete before the slot is overwritten
      SKR_HIP(hipStreamWaitEvent(st_, ev_sketch_, 0));
    }
    prof_.begin(KF_UPDATE);
    launch_normalize<T>(r_, a[0], a[1], st_);
    prof_.end();
    after_step(d);
  }

  // Two-pass recovery: regenerate U_1..U_d from C and the stored H (no inner products) and
  // accumulate X += U_j W[j] in chunks of the ring buffer.
  void replay(const double* C1, const double* C2, int d, int ell, const double* W1, const double* W2, double* X1,
              double* X2) {
    const double* Cs[2] = {C1, C2};
    const double* Ws[2] = {W1, W2};
    double* Xs[2] = {X1, X2};
    // U_1 = C ell^{-1}: reuse the start-block kernels with R taken from ell
    SpaceStep<T> a[2];
    for (int q = 0; q < 2; ++q) {
      Space<T>& s = sp_[q];
      const size_t cnt = (size_t)s.n * r_;
      hipLaunchKernelGGL(convert_kernel<T>, dim3(std::min<size_t>(4096, (cnt + 255) / 256)), dim3(256), 0, st_, Cs[q],
                         s.work.p, cnt);
      check_launch("convert");
      hipLaunchKernelGGL(replay_coef_kernel, dim3(1), dim3(64), 0, st_, r_, s.ell.p, r_, s.small.p, 1);
      check_launch("replay_coef");
      a[q] = step_args(s, 0);
      a[q].Unew = s.slot(1);
    }
    launch_normalize<T>(r_, a[0], a[1], st_);
    // nslots = k + 1 in two-pass mode; accumulate a block into X before its ring slot is
    // overwritten.
    int flushed = 0;  // blocks 1..flushed have been accumulated into X
    bool first = true;
    auto flush = [&](int upto) {
      // accumulate blocks flushed+1 .. upto (contiguous in the ring only when they do not wrap)
      for (int j = flushed + 1; j <= upto; ++j) {
        for (int q = 0; q < 2; ++q) {
          Space<T>& s = sp_[q];
          const int m = d * r_;
          dense::basis_gemm<T>(s.n, r_, 1, ell, 1.0, s.slot(j), Ws[q] + (size_t)(j - 1) * r_, m, first ? 0.0 : 1.0,
                               Xs[q], ell, st_);
        }
        first = false;
      }
      flushed = upto;
    };
    for (int j = 1; j < d; ++j) {
      // before writing slot(j+1) the block j+1-nslots must have been flushed
      const int evict = j + 1 - sp_[0].nslots;
      if (evict >= 1 && flushed < evict) flush(evict);
      for (int q = 0; q < 2; ++q) {
        Space<T>& s = sp_[q];
        a[q] = step_args(s, j);
        a[q].X = s.slot(j);
        a[q].W = s.slot(j);
        a[q].post = POST_DOT;
        a[q].Hblk = nullptr;
      }
      launch_spmm_dot<T>(r_, a[0], a[1], st_);
      const int i0 = std::max(1, j - p_.k + 1);
      for (int i = i0; i <= j; ++i) {
        for (int q = 0; q < 2; ++q) {
          Space<T>& s = sp_[q];
          hipLaunchKernelGGL(replay_coef_kernel, dim3(1), dim3(64), 0, st_, r_, Hblk(s, i, j), ld_, s.small.p, 0);
          check_launch("replay_coef");
          a[q].W = s.slot(i);
          a[q].Wn = s.slot(i);   // the dot result is discarded
          a[q].post = POST_DOT;
          a[q].Hblk = nullptr;
        }
        launch_axpy_reduce<T>(r_, a[0], a[1], st_);
      }
      for (int q = 0; q < 2; ++q) {
        Space<T>& s = sp_[q];
        hipLaunchKernelGGL(replay_coef_kernel, dim3(1), dim3(64), 0, st_, r_, Hblk(s, j + 1, j), ld_, s.small.p, 1);
        check_launch("replay_coef");
        a[q].Unew = s.slot(j + 1);
      }
      launch_normalize<T>(r_, a[0], a[1], st_);
    }
    flush(d);
  }

  PoolQuiet quiet_;  // first member: released last, after every buffer member
  int r_;
  bool fast_ = false;      // two-pass block step (r <= 4, k <= 10)
  bool sketched_ = true;   // s-PKSM; false: t-PKSM (no embedding)
  bool lyap_ = false;      // A X + X A^T = C1 C1^T on one Krylov space
  bool sorth_ = false;     // truncated orthogonalisation in the sketched inner product
  // ... whose whitening takes the sketch of the stored block rather than the sketch-space
  // S U_{d+1}: with an FP32 basis the two differ by the rounding of the stored block, and
  // the sketched QR must describe the basis that the recovery uses
  bool resketch_ = false;
  bool srht_ = false;      // subsampled randomized DCT embedding instead of the sparse sign one
  bool delayed_ = false;   // delayed re-orthogonalisation in the sketched QR update (r <= 8)
  int grp_ = 1;            // ... on groups of grp_ blocks (grp_ r wide)
  int held_ = 0;           // blocks whose sketches wait for the rest of their group
  int nwq_ = 4;            // sketch buffers per space
  int pend_w_ = 0;         // width of the block projected once and not yet appended to Q, T
  int pend_step_ = 0;      // the step that produced its first block
  int fin_cols_ = 0;       // columns of Q and T that are final
  skr_params p_;
  hipStream_t st_;
  int64_t s_ = 0;
  int ld_ = 0;
  size_t lds_limit_ = 65536;
  Space<T> sp_[2];
  Profiler prof_;
  hipStream_t aux_ = nullptr;   // sketches
  hipStream_t aux2_ = nullptr;  // sketched QR updates (whitening)
  hipEvent_t ev_block_ = nullptr, ev_sketch_ = nullptr, ev_aux_done_ = nullptr;
  hipEvent_t ev_whiten_[2 * GRP_MAX] = {};  // last whitening that read wbuf(j), j mod nwq_
  DBuf<double> F11_;
  std::vector<double> rhs_block_host_;
};

}  // namespace

skr_result_s* run_solve(const skr_op_s* A, int tu, const skr_op_s* B, int tv, const double* C1, const double* C2,
                        int r, const skr_params& p, hipStream_t st) {
  SKR_REQUIRE(A, "null operator");
  SKR_REQUIRE(C1 && C2, "null right-hand side factor");
  SKR_REQUIRE(B || C1 == C2, "the Lyapunov solve takes one right-hand side factor");
  if (p.precision == SKR_FP64) {
    Solver<double> s(A, tu, B, tv, r, p, st);
    return s.run(C1, C2);
  }
  SKR_REQUIRE(p.precision == SKR_MIXED, "precision must be SKR_FP64 or SKR_MIXED");
  Solver<float> s(A, tu, B, tv, r, p, st);
  return s.run(C1, C2);
}

}  // namespace skr
