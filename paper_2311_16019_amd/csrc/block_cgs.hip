// Two-pass block step of the truncated block Arnoldi recurrence (the inner loop of
// Algorithm 1), for r <= 4 and k <= 10.
//
// Pass 1 (one sweep):  U~ = Op U_d = (Op U'_d) P_d, stored; the raw products
//     D1raw_i = U'_i^T U~ for the window blocks i = i0 .. d and G0 = U~^T U~.
// Reduce 1 (small FP64 work on one workgroup per space): with the window Gram matrix
// Gw = W^T W of W = [U_i0 .. U_d] (kept from earlier steps, so no pass is spent on it),
//     D1 = W^T U~,  D = D1 - (Gw - I) D1,   G2 = G0 - D1^T D - D^T D1 + D^T Gw D,
// i.e. classical Gram-Schmidt with its reorthogonalisation pass taken on the Gram side, and
// the Gram matrix of U~ - W D without touching the data; R1 = chol(G2).  The blocks D are
// the Hessenberg entries h_{i,d} (Algorithm 1 defines them by modified Gram-Schmidt against
// the same window; in exact arithmetic both give the same blocks).
// Pass 2 (one sweep):  U' = (U~ - W D) R1^{-1}, stored as U'_{d+1}; G' = U'^T U'.
// Reduce 2: R2 = chol(G') (the second Cholesky QR factor from the stored data),
//     h_{d+1,d} = R2 R1,  P_{d+1} = R2^{-1}  (U_{d+1} = U'_{d+1} P_{d+1}, never formed),
// and the cross products U'_i^T U'_{d+1} that later window Gram matrices need, from the
// identities of pass 2 (U'_i^T U' = D1raw_i R1^{-1} - sum_j U'_i^T U'_j C_j).
//
// When G2 has lost most of its digits to cancellation (||U~ - W D|| << ||U~||) the first
// factor is only a scaling and the second Cholesky pass, computed from the data, carries
// the factorisation.  Breakdown is decided after pass 2 on h_{d+1,d} itself, with the
// oracle's thresholds.
#include <climits>

#include "blockstep.hpp"
#include "small_la.hpp"

namespace skr {
namespace {

constexpr int KM = CGS_KMAX;
// Windows of more than CGS_NARROW blocks take the wide kernels (window count at run time).
constexpr int CGS_NARROW = 3;
constexpr int RM = CGS_RMAX;
constexpr int RR_MAX = RM * RM;
constexpr int RED_T = 1024;  // threads of the first reduce kernel
// Threads of the second: it sums 16 values (16 lanes per value), for which 256 suffice.
constexpr int RED2_T = 256;

// Layout of CgsSmall::state (doubles).
struct CgsLayout {
  static constexpr int R1 = 0;                        // r x r
  static constexpr int COEF = R1 + RR_MAX;            // [R1^{-1} | C_0 .. C_{KM-1}]
  static constexpr int D1RAW = COEF + (KM + 1) * RR_MAX;
  static constexpr int XRAW = D1RAW + KM * RR_MAX;    // (KM r)^2, leading dimension KM * RM
  static constexpr int G0TR = XRAW + (KM * RM) * (KM * RM);
  static constexpr int SIZE = G0TR + 8;
};

// Breakdown thresholds (not discussed in the paper; the same values as the FP64 oracle).
constexpr double BREAK_NORM = 1e-12;
constexpr double BREAK_DIAG = 1e-14;
// Below this fraction of ||U~||_F^2, the Gram-side G2 is not trusted for the first factor.
constexpr double G2_TRUST = 1e-8;

struct Rows {
  int space, local, row0, row1;
};

template <typename T>
__device__ inline Rows rows_of(const CgsPass<T>& s0, const CgsPass<T>& s1) {
  const int G = s0.nwg + s1.nwg;
  const int lg = xcd_logical(blockIdx.x, G);
  Rows w;
  w.space = lg < s0.nwg ? 0 : 1;
  w.local = w.space ? lg - s0.nwg : lg;
  const CgsPass<T>& sp = w.space ? s1 : s0;
  const int per = ((sp.n + sp.nwg - 1) / sp.nwg + WG - 1) / WG * WG;
  w.row0 = min(sp.n, w.local * per);
  w.row1 = min(sp.n, w.row0 + per);
  return w;
}

// Workgroup sums of NV per-thread values, written as this workgroup's partials
// part[v * nwg + local] (value-major): wavefront transpose reductions, then the wavefront
// totals added in order.
// Only the first nvalid values are written (a short last group of a wide sweep).
template <int NV>
__device__ inline void write_partials(const double (&acc)[NV], double* part, int nwg, int local, double* scratch,
                                      int nvalid = NV) {
  const int wv = threadIdx.x / 64;
  int idx;
  const double t = wave_transpose_sum<NV>(acc, idx);
  if (idx >= 0) scratch[wv * NV + idx] = t;
  __syncthreads();
  for (int i = threadIdx.x; i < nvalid; i += WG) {
    double u = 0.0;
#pragma unroll
    for (int w = 0; w < WG / 64; ++w) u += scratch[w * NV + i];
    part[(size_t)i * nwg + local] = u;
  }
}

// ------------------------------------------------------------------------- pass 1
// 1a: U~ = (Op U'_d) P_d (or the start block), stored in T.  Few registers, so many
// wavefronts per CU hide the dependent row-pointer -> column -> gather loads.
// Nonzeros of a row whose loads are in flight together: five covers the 2D stencils in one
// batch and keeps the kernel at six wavefronts per SIMD.
constexpr int SPMM_UN = 5;

template <typename T, int R>
__global__ void __launch_bounds__(WG) cgs_spmm_kernel(CgsPass<T> s0, CgsPass<T> s1) {
  constexpr int RR = R * R;
  const Rows wi = rows_of(s0, s1);
  const CgsPass<T>& sp = wi.space ? s1 : s0;
  __shared__ double pd[RR];
  // slice offsets of this workgroup's rows, loaded once instead of per row
  constexpr int MAXSL = 64;
  __shared__ int soff[MAXSL + 1];
  const CsrView<T> A = sp.A;
  const int q0 = wi.row0 / SELL_C;
  const int nsl = (wi.row1 - wi.row0 + SELL_C - 1) / SELL_C;
  const bool pre = A.sell_off && nsl <= MAXSL;
  for (int i = threadIdx.x; i < RR; i += WG) pd[i] = sp.Pd ? sp.Pd[i] : ((i / R == i % R) ? 1.0 : 0.0);
  if (pre)
    for (int i = threadIdx.x; i <= nsl; i += WG) soff[i] = A.sell_off[q0 + i];
  __syncthreads();
  for (int base = wi.row0; base < wi.row1; base += WG) {
    const int row = base + threadIdx.x;
    if (row >= wi.row1) continue;
    double y[R];
    if (sp.src) {
#pragma unroll
      for (int c = 0; c < R; ++c) y[c] = sp.src[(size_t)row * R + c];
    } else {
      double yr[R];
#pragma unroll
      for (int c = 0; c < R; ++c) yr[c] = 0.0;
      if (A.sell_off) {
        // sliced ELL: a wavefront's 64 rows are one slice, so each index load (and each FP32
        // value load) of the wavefront is one contiguous 256-byte access
        const int q = row / SELL_C, l = row % SELL_C;
        const int e0 = pre ? soff[q - q0] : A.sell_off[q];
        const int w = ((pre ? soff[q - q0 + 1] : A.sell_off[q + 1]) - e0) / SELL_C;
        for (int jb = 0; jb < w; jb += SPMM_UN) {
          int cols[SPMM_UN];
          double vv[SPMM_UN];
#pragma unroll
          for (int j = 0; j < SPMM_UN; ++j) {
            const bool ok = jb + j < w;
            cols[j] = ok ? A.sell_col[e0 + (jb + j) * SELL_C + l] : row;
            vv[j] = ok ? static_cast<double>(A.sell_val[e0 + (jb + j) * SELL_C + l]) : 0.0;
          }
#pragma unroll
          for (int j = 0; j < SPMM_UN; ++j) {
            if (jb + j < w) {
              double x[R];
              load_row<T, R>(sp.X, cols[j], x);
#pragma unroll
              for (int c = 0; c < R; ++c) yr[c] += vv[j] * x[c];
            }
          }
        }
      } else {
      const int k0 = A.rowptr[row], k1 = A.rowptr[row + 1];
      // SPMM_UN nonzeros at a time: their indices and values, then their gathers, in flight
      for (int kb = k0; kb < k1; kb += SPMM_UN) {
        int cols[SPMM_UN];
        double vv[SPMM_UN];
#pragma unroll
        for (int j = 0; j < SPMM_UN; ++j) {
          const bool ok = kb + j < k1;
          cols[j] = ok ? A.colind[kb + j] : row;
          vv[j] = ok ? static_cast<double>(A.val[kb + j]) : 0.0;
        }
#pragma unroll
        for (int j = 0; j < SPMM_UN; ++j) {
          if (kb + j < k1) {
            double x[R];
            load_row<T, R>(sp.X, cols[j], x);
#pragma unroll
            for (int c = 0; c < R; ++c) yr[c] += vv[j] * x[c];
          }
        }
      }
      }
      if (A.diag) {
        const double dg = A.diag[row];
        double x[R];
        load_row<T, R>(sp.X, row, x);
#pragma unroll
        for (int c = 0; c < R; ++c) yr[c] += dg * x[c];
      }
#pragma unroll
      for (int b = 0; b < R; ++b) {
        double t = 0.0;
#pragma unroll
        for (int a = 0; a < R; ++a) t += yr[a] * pd[a * R + b];
        y[b] = t;
      }
    }
    store_row<T, R>(sp.Y, row, y);
  }
}

// 1b: the window products U'_i^T U~ and U~^T U~ from the stored (rounded) U~: independent
// streaming loads, two rows per thread in flight.
// Rows are kept in their storage type until used (half the registers in FP32), and only
// the upper triangle of the symmetric U~^T U~ is accumulated; the products are the same
// operations in the same order as for the full matrix, which is mirrored when the partials
// are written.
template <typename T, int R>
__device__ inline void load_raw(const T* __restrict__ p, int row, T (&x)[R]) {
  const T* q = p + (size_t)row * R;
  if constexpr (sizeof(T) == 4 && R == 4) {
    const float4 v = *reinterpret_cast<const float4*>(q);
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
  } else if constexpr (sizeof(T) == 4 && R == 2) {
    const float2 v = *reinterpret_cast<const float2*>(q);
    x[0] = v.x; x[1] = v.y;
  } else if constexpr (sizeof(T) == 8 && R % 2 == 0) {
#pragma unroll
    for (int c = 0; c < R; c += 2) {
      const double2 v = *reinterpret_cast<const double2*>(q + c);
      x[c] = v.x; x[c + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int c = 0; c < R; ++c) x[c] = q[c];
  }
}

template <typename T, int R, int NW>
__global__ void __launch_bounds__(WG) cgs_dots_kernel(CgsPass<T> s0, CgsPass<T> s1) {
  constexpr int RR = R * R, NV = (NW + 1) * RR, NG = R * (R + 1) / 2;
  const Rows wi = rows_of(s0, s1);
  const CgsPass<T>& sp = wi.space ? s1 : s0;
  __shared__ double scratch[(WG / 64) * NV];
  double accw[NW > 0 ? NW * RR : 1], accg[NG];
#pragma unroll
  for (int v = 0; v < (NW > 0 ? NW * RR : 1); ++v) accw[v] = 0.0;
#pragma unroll
  for (int v = 0; v < NG; ++v) accg[v] = 0.0;
  for (int base = wi.row0; base < wi.row1; base += 2 * WG) {
    T y[2][R], w[2][NW > 0 ? NW : 1][R];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int row = base + h * WG + threadIdx.x;
      const bool ok = row < wi.row1;
      const int rr = ok ? row : wi.row0;  // rows past the end read a valid row, weighted 0
      load_raw<T, R>(sp.Y, rr, y[h]);
#pragma unroll
      for (int i = 0; i < NW; ++i) load_raw<T, R>(sp.W[i], rr, w[h][i]);
      if (!ok) {
#pragma unroll
        for (int c = 0; c < R; ++c) y[h][c] = T(0);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      int g = 0;
#pragma unroll
      for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = a; b < R; ++b, ++g) accg[g] += (double)y[h][a] * (double)y[h][b];
#pragma unroll
      for (int i = 0; i < NW; ++i)
#pragma unroll
        for (int a = 0; a < R; ++a)
#pragma unroll
          for (int b = 0; b < R; ++b) accw[i * RR + a * R + b] += (double)w[h][i][a] * (double)y[h][b];
    }
  }
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NW * RR; ++v) acc[v] = accw[v];
  {
    int g = 0;
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int b = a; b < R; ++b, ++g) {
        acc[NW * RR + a * R + b] = accg[g];
        acc[NW * RR + b * R + a] = accg[g];
      }
  }
  write_partials<NV>(acc, sp.part, sp.nwg, wi.local, scratch);
}

// ------------------------------------------------------------------------- pass 2
template <typename T, int R, int NW>
__global__ void __launch_bounds__(WG) cgs_pass2_kernel(CgsPass<T> s0, CgsPass<T> s1) {
  constexpr int RR = R * R;
  const Rows wi = rows_of(s0, s1);
  const CgsPass<T>& sp = wi.space ? s1 : s0;
  __shared__ double cf[(NW + 1) * RR];
  __shared__ double scratch[(WG / 64) * RR];
  for (int i = threadIdx.x; i < (NW + 1) * RR; i += WG) cf[i] = sp.coef[i];
  __syncthreads();
  double acc[RR];
#pragma unroll
  for (int v = 0; v < RR; ++v) acc[v] = 0.0;
  for (int base = wi.row0; base < wi.row1; base += 2 * WG) {  // two rows per thread in flight
    asm volatile("" ::: "memory");  // coefficients re-read from LDS per iteration (registers)
    double y[2][R], w[2][NW > 0 ? NW : 1][R];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int row = base + h * WG + threadIdx.x;
      const bool ok = row < wi.row1;
      const int rr = ok ? row : wi.row0;  // rows past the end read a valid row, weighted 0
      load_row<T, R>(sp.Y, rr, y[h]);
#pragma unroll
      for (int i = 0; i < NW; ++i) load_row<T, R>(sp.W[i], rr, w[h][i]);
      if (!ok) {
#pragma unroll
        for (int c = 0; c < R; ++c) y[h][c] = 0.0;
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int row = base + h * WG + threadIdx.x;
      double u[R];
#pragma unroll
      for (int b = 0; b < R; ++b) {
        double t = 0.0;
#pragma unroll
        for (int a = 0; a <= b; ++a) t += y[h][a] * cf[a * R + b];  // R1^{-1} is upper triangular
        u[b] = t;
      }
#pragma unroll
      for (int i = 0; i < NW; ++i)
#pragma unroll
        for (int b = 0; b < R; ++b) {
          double t = 0.0;
#pragma unroll
          for (int a = 0; a < R; ++a) t += w[h][i][a] * cf[(1 + i) * RR + a * R + b];
          u[b] -= t;
        }
      if (row < wi.row1) {
        store_row<T, R>(sp.Unew, row, u);
#pragma unroll
        for (int a = 0; a < R; ++a)
#pragma unroll
          for (int b = 0; b < R; ++b) acc[a * R + b] += u[a] * u[b];
      }
    }
  }
  write_partials<RR>(acc, sp.part, sp.nwg, wi.local, scratch);
}

// ------------------------------------------------------------------------- long windows
// Window blocks of a wide sweep taken together in one pass over the rows (4 r^2 <= 64
// accumulated products per thread).
constexpr int CGS_GROUP = 4;

// Pass 1b for nw > 3 window blocks: the products U'_i^T U~ in groups of CGS_GROUP blocks,
// one wavefront per group over all of the workgroup's rows (the group wavefronts read the
// same rows of U~ at about the same time, so U~ comes from HBM once: a pass per group over
// the rows re-read it from HBM, 128 MB per step at n = 1e6, r = 4, k = 10), and U~^T U~ in
// the workgroup's last wavefront; each wavefront's totals are its workgroup's partials, in
// the layout of cgs_dots_kernel.
static_assert(CGS_KMAX <= CGS_GROUP * (WG / 64 - 1), "a wavefront per window group and one for U~^T U~");

template <typename T, int R>
__global__ void __launch_bounds__(WG) cgs_dots_wide_kernel(CgsPass<T> s0, CgsPass<T> s1, int nw) {
  constexpr int RR = R * R, NG = R * (R + 1) / 2, GV = CGS_GROUP * RR;
  const Rows wi = rows_of(s0, s1);
  const CgsPass<T>& sp = wi.space ? s1 : s0;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;  // wv is uniform over the wavefront
  const int ngroups = (nw + CGS_GROUP - 1) / CGS_GROUP;
  if (wv < ngroups) {
    const int g0 = wv * CGS_GROUP, ng = min(CGS_GROUP, nw - g0);
    // the group's block pointers, selected with constant indices (a run-time index into the
    // kernel argument would move the argument structure to scratch memory)
    const T* wp[CGS_GROUP];
#pragma unroll
    for (int i = 0; i < CGS_GROUP; ++i) {
      wp[i] = sp.W[0];
#pragma unroll
      for (int t = 0; t < KM; ++t)
        if (t == g0 + i) wp[i] = sp.W[t];
    }
    double accw[GV];
#pragma unroll
    for (int v = 0; v < GV; ++v) accw[v] = 0.0;
    for (int row = wi.row0 + lane; row < wi.row1; row += 64) {
      T y[R], w[CGS_GROUP][R];
      load_raw<T, R>(sp.Y, row, y);
#pragma unroll
      for (int i = 0; i < CGS_GROUP; ++i)
        if (i < ng) load_raw<T, R>(wp[i], row, w[i]);
#pragma unroll
      for (int i = 0; i < CGS_GROUP; ++i)
        if (i < ng)
#pragma unroll
          for (int a = 0; a < R; ++a)
#pragma unroll
            for (int b = 0; b < R; ++b) accw[i * RR + a * R + b] += (double)w[i][a] * (double)y[b];
    }
    // this group's values are window values g0 * RR .. (g0 + ng) * RR (value-major partials)
    int idx;
    const double t = wave_transpose_sum<GV>(accw, idx);
    if (idx >= 0 && idx < ng * RR) sp.part[(size_t)(g0 * RR + idx) * sp.nwg + wi.local] = t;
  } else if (wv == WG / 64 - 1) {
    double accg[NG];
#pragma unroll
    for (int v = 0; v < NG; ++v) accg[v] = 0.0;
    for (int row = wi.row0 + lane; row < wi.row1; row += 64) {
      T y[R];
      load_raw<T, R>(sp.Y, row, y);
      int g = 0;
#pragma unroll
      for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = a; b < R; ++b, ++g) accg[g] += (double)y[a] * (double)y[b];
    }
    double acc[RR];
    int g = 0;
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int b = a; b < R; ++b, ++g) {
        acc[a * R + b] = accg[g];
        acc[b * R + a] = accg[g];
      }
    int idx;
    const double t = wave_transpose_sum<RR>(acc, idx);
    if (idx >= 0) sp.part[(size_t)(nw * RR + idx) * sp.nwg + wi.local] = t;
  }
}

// Pass 2 for nw > 3 window blocks: U' = (U~ - W D) R1^{-1} with all window rows of a row in
// flight together, and the Gram matrix of U'.
template <typename T, int R>
__global__ void __launch_bounds__(WG) cgs_pass2_wide_kernel(CgsPass<T> s0, CgsPass<T> s1, int nw) {
  constexpr int RR = R * R;
  const Rows wi = rows_of(s0, s1);
  const CgsPass<T>& sp = wi.space ? s1 : s0;
  __shared__ double cf[(KM + 1) * RR];
  __shared__ double scratch[(WG / 64) * RR];
  for (int i = threadIdx.x; i < (nw + 1) * RR; i += WG) cf[i] = sp.coef[i];
  __syncthreads();
  double acc[RR];
#pragma unroll
  for (int v = 0; v < RR; ++v) acc[v] = 0.0;
  for (int row = wi.row0 + threadIdx.x; row < wi.row1; row += WG) {
    // the coefficients are read from LDS in every iteration: kept in registers across rows
    // they would take (nw + 1) r^2 of them
    asm volatile("" ::: "memory");
    double y[R], w[KM][R];
    load_row<T, R>(sp.Y, row, y);
#pragma unroll
    for (int i = 0; i < KM; ++i)
      if (i < nw) load_row<T, R>(sp.W[i], row, w[i]);
    double u[R];
#pragma unroll
    for (int b = 0; b < R; ++b) {
      double t = 0.0;
#pragma unroll
      for (int a = 0; a <= b; ++a) t += y[a] * cf[a * R + b];  // R1^{-1} is upper triangular
      u[b] = t;
    }
#pragma unroll
    for (int i = 0; i < KM; ++i)
      if (i < nw)
#pragma unroll
        for (int b = 0; b < R; ++b) {
          double t = 0.0;
#pragma unroll
          for (int a = 0; a < R; ++a) t += w[i][a] * cf[(1 + i) * RR + a * R + b];
          u[b] -= t;
        }
    store_row<T, R>(sp.Unew, row, u);
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int b = 0; b < R; ++b) acc[a * R + b] += u[a] * u[b];
  }
  write_partials<RR>(acc, sp.part, sp.nwg, wi.local, scratch);
}

// ------------------------------------------------------------------------- reductions
// Sum the partials of nv values into out[0..nv): 16 consecutive threads per value (one
// DPP row), each summing a strided subset of the partials; fixed order throughout.
template <int NT>
__device__ inline void sum_partials(const double* part, int nwg, int nv, double* out) {
  const int sub = threadIdx.x % 16;
  const int nround = (nv + NT / 16 - 1) / (NT / 16);  // uniform over the workgroup
  for (int rd = 0; rd < nround; ++rd) {
    const int v = threadIdx.x / 16 + rd * (NT / 16);
    double s = 0.0;
    if (v < nv) {
      const double* p = part + (size_t)v * nwg;
      for (int g0 = 0; g0 < nwg; g0 += 512) {  // 32 independent loads per thread in flight
        double t[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
          const int g = g0 + sub + 16 * u;
          t[u] = (g < nwg) ? p[g] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 32; ++u) s += t[u];
      }
    }
    s += dpp_move<0xB1>(s);
    s += dpp_move<0x4E>(s);
    s += dpp_move<0x124>(s);
    s += dpp_move<0x128>(s);
    if (v < nv && sub == 0) out[v] = s;
  }
}

__global__ void __launch_bounds__(RED_T) cgs_reduce1_kernel(CgsSmall s0, CgsSmall s1, int r, int nw, int i0, int d) {
  const CgsSmall& sm = blockIdx.x ? s1 : s0;
  const int tid = threadIdx.x, RR = r * r, m = nw * r;
  constexpr int LM = KM * RM;  // leading dimension of the (nw r) x (nw r) arrays
  __shared__ double raw[(KM + 1) * RR_MAX];
  __shared__ double P[KM][RR_MAX];
  __shared__ double Xr[LM * LM], T1[LM * LM], Gw[LM * LM];
  __shared__ double D1[LM * RM], D[LM * RM], M1[LM * RM], Z[LM * RM];
  __shared__ double G2[RR_MAX], R1[RR_MAX], R1i[RR_MAX];
  __shared__ double trg0;
  sum_partials<RED_T>(sm.part, sm.nwg, (nw + 1) * RR, raw);
  for (int e = tid; e < nw * RR; e += RED_T) P[e / RR][e % RR] = sm.Pall[(size_t)(i0 + e / RR) * RR + e % RR];
  for (int e = tid; e < m * m; e += RED_T) {
    const int I = e / m, J = e % m, bi = I / r, bj = J / r, a = I % r, b = J % r;
    double v;
    if (bi == bj) v = sm.Gall[(size_t)(i0 + bi) * RR + a * r + b];
    else if (bi < bj) v = sm.Xall[((size_t)(i0 + bj) * KM + (bj - 1 - bi)) * RR + a * r + b];
    else v = sm.Xall[((size_t)(i0 + bi) * KM + (bi - 1 - bj)) * RR + b * r + a];
    Xr[I * LM + J] = v;
  }
  __syncthreads();
  // D1_i = P_i^T D1raw_i (stacked m x r);  T1 = Xr Pbd
  for (int e = tid; e < m * r; e += RED_T) {
    const int I = e / r, b = e % r, i = I / r, a = I % r;
    double t = 0.0;
    for (int c = 0; c < r; ++c) t += P[i][c * r + a] * raw[i * RR + c * r + b];
    D1[I * RM + b] = t;
  }
  for (int e = tid; e < m * m; e += RED_T) {
    const int I = e / m, J = e % m, bj = J / r, b = J % r;
    double t = 0.0;
    for (int c = 0; c < r; ++c) t += Xr[I * LM + bj * r + c] * P[bj][c * r + b];
    T1[I * LM + J] = t;
  }
  __syncthreads();
  // Gw = Pbd^T T1
  for (int e = tid; e < m * m; e += RED_T) {
    const int I = e / m, J = e % m, bi = I / r, a = I % r;
    double t = 0.0;
    for (int c = 0; c < r; ++c) t += P[bi][c * r + a] * T1[(bi * r + c) * LM + J];
    Gw[I * LM + J] = t;
  }
  __syncthreads();
  // D = D1 - (Gw - I) D1
  for (int e = tid; e < m * r; e += RED_T) {
    const int I = e / r, b = e % r;
    double t = 0.0;
    for (int J = 0; J < m; ++J) t += (Gw[I * LM + J] - (I == J ? 1.0 : 0.0)) * D1[J * RM + b];
    D[I * RM + b] = D1[I * RM + b] - t;
  }
  __syncthreads();
  // M1 = Gw D
  for (int e = tid; e < m * r; e += RED_T) {
    const int I = e / r, b = e % r;
    double t = 0.0;
    for (int J = 0; J < m; ++J) t += Gw[I * LM + J] * D[J * RM + b];
    M1[I * RM + b] = t;
  }
  __syncthreads();
  // G2 = G0 - D1^T D - D^T D1 + D^T M1
  const double* G0 = raw + nw * RR;
  for (int e = tid; e < RR; e += RED_T) {
    const int a = e / r, b = e % r;
    double t = 0.0;
    for (int I = 0; I < m; ++I)
      t += D1[I * RM + a] * D[I * RM + b] + D[I * RM + a] * D1[I * RM + b] - D[I * RM + a] * M1[I * RM + b];
    G2[e] = G0[e] - t;
  }
  __syncthreads();
  if (tid == 0) {
    double tr0 = 0.0, tr2 = 0.0;
    for (int a = 0; a < r; ++a) { tr0 += G0[a * r + a]; tr2 += G2[a * r + a]; }
    trg0 = tr0;
    bool ok = (tr2 > G2_TRUST * tr0) && chol_upper(G2, R1, r);
    if (!ok) {  // cancellation: a scaling only; the second factor comes from the data
      const double sc = sqrt(fmax(tr2, 1e-16 * tr0) / r);
      for (int e = 0; e < RR; ++e) R1[e] = (e / r == e % r) ? (sc > 0.0 ? sc : 1.0) : 0.0;
    }
    inv_upper(R1, R1i, r);
  }
  __syncthreads();
  // C_i = P_i D_i R1^{-1}:  Z = D R1^{-1} first
  for (int e = tid; e < m * r; e += RED_T) {
    const int I = e / r, b = e % r;
    double t = 0.0;
    for (int c = 0; c <= b; ++c) t += D[I * RM + c] * R1i[c * r + b];
    Z[I * RM + b] = t;
  }
  __syncthreads();
  double* st = sm.state;
  for (int e = tid; e < nw * RR; e += RED_T) {
    const int i = e / RR, a = (e % RR) / r, b = e % r;
    double t = 0.0;
    for (int c = 0; c < r; ++c) t += P[i][a * r + c] * Z[(i * r + c) * RM + b];
    st[CgsLayout::COEF + (1 + i) * RR + a * r + b] = t;
    st[CgsLayout::D1RAW + i * RR + a * r + b] = raw[i * RR + a * r + b];
    // h_{i0+i, d} = D_i (column-major in H)
    sm.H[((size_t)(i0 + i - 1) * r + a) + ((size_t)(d - 1) * r + b) * sm.ldh] = D[(i * r + a) * RM + b];
  }
  for (int e = tid; e < RR; e += RED_T) {
    st[CgsLayout::R1 + e] = R1[e];
    st[CgsLayout::COEF + e] = R1i[e];
  }
  for (int e = tid; e < m * m; e += RED_T) st[CgsLayout::XRAW + (e / m) * LM + e % m] = Xr[(e / m) * LM + e % m];
  if (tid == 0) st[CgsLayout::G0TR] = trg0;
}

__global__ void __launch_bounds__(RED2_T) cgs_reduce2_kernel(CgsSmall s0, CgsSmall s1, int r, int nw, int i0, int d) {
  const CgsSmall& sm = blockIdx.x ? s1 : s0;
  const int tid = threadIdx.x, RR = r * r;
  constexpr int LM = KM * RM;
  __shared__ double Gp[RR_MAX], R2[RR_MAX], RF[RR_MAX], R2i[RR_MAX];
  __shared__ int ok_sh;
  sum_partials<RED2_T>(sm.part, sm.nwg, RR, Gp);
  __syncthreads();
  const double* st = sm.state;
  if (tid == 0) {
    bool ok = chol_upper(Gp, R2, r);
    if (ok) {
      matmul_small(R2, st + CgsLayout::R1, RF, r);
      double f2 = 0.0, mx = 0.0, mn = 1e308;
      for (int a = 0; a < r; ++a)
        for (int b = a; b < r; ++b) { f2 += RF[a * r + b] * RF[a * r + b]; mx = fmax(mx, fabs(RF[a * r + b])); }
      for (int a = 0; a < r; ++a) mn = fmin(mn, RF[a * r + a]);
      // ||U~ - W D||_F = ||R2 R1||_F against ||Op U_d||_F, and the diagonal of R (the
      // oracle's two breakdown tests)
      ok = (f2 >= BREAK_NORM * BREAK_NORM * st[CgsLayout::G0TR]) && (mn > BREAK_DIAG * mx);
      inv_upper(R2, R2i, r);
    }
    if (!ok) {
      atomicMin(sm.broken, d);
      for (int e = 0; e < RR; ++e) { RF[e] = 0.0; R2i[e] = (e / r == e % r) ? 1.0 : 0.0; Gp[e] = R2i[e]; }
    }
    ok_sh = ok ? 1 : 0;
  }
  __syncthreads();
  const bool ok = ok_sh != 0;
  // h_{d+1,d} = R2 R1 (for the start block: its R factor, ldh = r), P_{d+1}, U'^T U'
  for (int e = tid; e < RR; e += RED2_T) {
    const int a = e / r, b = e % r;
    sm.H[((size_t)d * r + a) + ((size_t)(d > 0 ? d - 1 : 0) * r + b) * sm.ldh] = RF[e];
    sm.Pall[(size_t)(d + 1) * RR + e] = R2i[e];
    sm.Gall[(size_t)(d + 1) * RR + e] = Gp[e];
  }
  // U'_{i0+i}^T U'_{d+1} = D1raw_i R1^{-1} - sum_j U'_{i0+i}^T U'_{i0+j} C_j
  for (int e = tid; e < nw * RR; e += RED2_T) {
    const int i = e / RR, a = (e % RR) / r, b = e % r;
    double t = 0.0;
    if (ok) {
      for (int c = 0; c < r; ++c) t += st[CgsLayout::D1RAW + i * RR + a * r + c] * st[CgsLayout::COEF + c * r + b];
      for (int j = 0; j < nw; ++j)
        for (int c = 0; c < r; ++c)
          t -= st[CgsLayout::XRAW + (i * r + a) * LM + j * r + c] * st[CgsLayout::COEF + (1 + j) * RR + c * r + b];
    }
    sm.Xall[((size_t)(d + 1) * KM + (d - i0 - i)) * RR + a * r + b] = t;
  }
}

// Workgroups of the SpMM sweep: about four rows per thread, so that many wavefronts per CU
// hide the dependent loads (the other sweeps use the fewer workgroups of CgsPass::nwg,
// whose partials the reductions read).
inline int spmm_wgs(int n) {  // two rows per thread: short latency chains, a small tail
  int g = ceil_div(n, 2 * WG);
  g = (g + 7) / 8 * 8;
  return std::max(8, std::min(8192, g));
}

template <typename T, int R, int NW>
void spmm_launch(const CgsPass<T>& a, const CgsPass<T>& b, hipStream_t st) {
  CgsPass<T> a1 = a, b1 = b;
  a1.nwg = spmm_wgs(a.n);
  b1.nwg = spmm_wgs(b.n);
  hipLaunchKernelGGL((cgs_spmm_kernel<T, R>), dim3(a1.nwg + b1.nwg), dim3(WG), 0, st, a1, b1);
}
template <typename T, int R, int NW>
void dots_launch(const CgsPass<T>& a, const CgsPass<T>& b, hipStream_t st) {
  hipLaunchKernelGGL((cgs_dots_kernel<T, R, NW>), dim3(a.nwg + b.nwg), dim3(WG), 0, st, a, b);
}

template <typename T, int R, int NW>
void pass2_launch(const CgsPass<T>& a, const CgsPass<T>& b, hipStream_t st) {
  hipLaunchKernelGGL((cgs_pass2_kernel<T, R, NW>), dim3(a.nwg + b.nwg), dim3(WG), 0, st, a, b);
}

#define SKR_CGS_DISPATCH(FN, r, nw, ...)                                   \
  do {                                                                     \
    SKR_REQUIRE(r >= 1 && r <= RM && nw >= 0 && nw <= CGS_NARROW, "two-pass block step: unsupported r or window"); \
    switch (r * 8 + nw) {                                                  \
      case 8: FN<T, 1, 0>(__VA_ARGS__); break;                             \
      case 9: FN<T, 1, 1>(__VA_ARGS__); break;                             \
      case 10: FN<T, 1, 2>(__VA_ARGS__); break;                            \
      case 11: FN<T, 1, 3>(__VA_ARGS__); break;                            \
      case 16: FN<T, 2, 0>(__VA_ARGS__); break;                            \
      case 17: FN<T, 2, 1>(__VA_ARGS__); break;                            \
      case 18: FN<T, 2, 2>(__VA_ARGS__); break;                            \
      case 19: FN<T, 2, 3>(__VA_ARGS__); break;                            \
      case 24: FN<T, 3, 0>(__VA_ARGS__); break;                            \
      case 25: FN<T, 3, 1>(__VA_ARGS__); break;                            \
      case 26: FN<T, 3, 2>(__VA_ARGS__); break;                            \
      case 27: FN<T, 3, 3>(__VA_ARGS__); break;                            \
      case 32: FN<T, 4, 0>(__VA_ARGS__); break;                            \
      case 33: FN<T, 4, 1>(__VA_ARGS__); break;                            \
      case 34: FN<T, 4, 2>(__VA_ARGS__); break;                            \
      case 35: FN<T, 4, 3>(__VA_ARGS__); break;                            \
    }                                                                      \
  } while (0)

}  // namespace

int cgs_state_doubles() { return CgsLayout::SIZE; }
int cgs_coef_offset() { return CgsLayout::COEF; }

int cgs_wgs(int n) {
  int g = ceil_div(n, 16 * WG);
  g = (g + 7) / 8 * 8;
  return std::max(8, std::min(256, g));
}

template <typename T>
void launch_cgs_spmm(int r, const CgsPass<T>& a, const CgsPass<T>& b, hipStream_t st) {
  SKR_CGS_DISPATCH(spmm_launch, r, 0, a, b, st);
  check_launch("cgs_spmm");
}
template <typename T>
void launch_cgs_dots(int r, int nw, const CgsPass<T>& a, const CgsPass<T>& b, hipStream_t st) {
  if (nw <= CGS_NARROW) {
    SKR_CGS_DISPATCH(dots_launch, r, nw, a, b, st);
  } else {
    SKR_REQUIRE(r >= 1 && r <= RM && nw <= KM, "two-pass block step: unsupported r or window");
    const dim3 g(a.nwg + b.nwg);
    switch (r) {
      case 1: hipLaunchKernelGGL((cgs_dots_wide_kernel<T, 1>), g, dim3(WG), 0, st, a, b, nw); break;
      case 2: hipLaunchKernelGGL((cgs_dots_wide_kernel<T, 2>), g, dim3(WG), 0, st, a, b, nw); break;
      case 3: hipLaunchKernelGGL((cgs_dots_wide_kernel<T, 3>), g, dim3(WG), 0, st, a, b, nw); break;
      default: hipLaunchKernelGGL((cgs_dots_wide_kernel<T, 4>), g, dim3(WG), 0, st, a, b, nw); break;
    }
  }
  check_launch("cgs_dots");
}
template <typename T>
void launch_cgs_pass2(int r, int nw, const CgsPass<T>& a, const CgsPass<T>& b, hipStream_t st) {
  if (nw <= CGS_NARROW) {
    SKR_CGS_DISPATCH(pass2_launch, r, nw, a, b, st);
  } else {
    SKR_REQUIRE(r >= 1 && r <= RM && nw <= KM, "two-pass block step: unsupported r or window");
    const dim3 g(a.nwg + b.nwg);
    switch (r) {
      case 1: hipLaunchKernelGGL((cgs_pass2_wide_kernel<T, 1>), g, dim3(WG), 0, st, a, b, nw); break;
      case 2: hipLaunchKernelGGL((cgs_pass2_wide_kernel<T, 2>), g, dim3(WG), 0, st, a, b, nw); break;
      case 3: hipLaunchKernelGGL((cgs_pass2_wide_kernel<T, 3>), g, dim3(WG), 0, st, a, b, nw); break;
      default: hipLaunchKernelGGL((cgs_pass2_wide_kernel<T, 4>), g, dim3(WG), 0, st, a, b, nw); break;
    }
  }
  check_launch("cgs_pass2");
}

void launch_cgs_reduce1(int r, int nw, int i0, int d, const CgsSmall& a, const CgsSmall& b, hipStream_t st) {
  SKR_REQUIRE(r >= 1 && r <= RM && nw >= 0 && nw <= KM, "two-pass block step: unsupported r or window");
  hipLaunchKernelGGL(cgs_reduce1_kernel, dim3(2), dim3(RED_T), 0, st, a, b, r, nw, i0, d);
  check_launch("cgs_reduce1");
}
void launch_cgs_reduce2(int r, int nw, int i0, int d, const CgsSmall& a, const CgsSmall& b, hipStream_t st) {
  hipLaunchKernelGGL(cgs_reduce2_kernel, dim3(2), dim3(RED2_T), 0, st, a, b, r, nw, i0, d);
  check_launch("cgs_reduce2");
}

template void launch_cgs_spmm<double>(int, const CgsPass<double>&, const CgsPass<double>&, hipStream_t);
template void launch_cgs_spmm<float>(int, const CgsPass<float>&, const CgsPass<float>&, hipStream_t);
template void launch_cgs_dots<double>(int, int, const CgsPass<double>&, const CgsPass<double>&, hipStream_t);
template void launch_cgs_dots<float>(int, int, const CgsPass<float>&, const CgsPass<float>&, hipStream_t);
template void launch_cgs_pass2<double>(int, int, const CgsPass<double>&, const CgsPass<double>&, hipStream_t);
template void launch_cgs_pass2<float>(int, int, const CgsPass<float>&, const CgsPass<float>&, hipStream_t);

}  // namespace skr
