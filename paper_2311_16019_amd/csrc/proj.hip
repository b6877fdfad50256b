// Projected Sylvester problem on the device (FP64).
//
// The small equation M_A Y + Y M_B^T = F is solved with the coupled Newton iteration for
// the matrix sign function of Z = [[M_A, F], [0, -M_B^T]]: with A_0 = M_A, B_0 = M_B^T,
// C_0 = F and a scaling mu_k (Frobenius-norm scaling),
//     A_{k+1} = (mu A_k + A_k^{-1}/mu)/2,  B_{k+1} = (mu B_k + B_k^{-1}/mu)/2,
//     C_{k+1} = (mu C_k + A_k^{-1} C_k B_k^{-1}/mu)/2,
// A_k -> sign(M_A), B_k -> sign(M_B^T) and C_k -> 2 Y when both sign limits are the
// identity (all eigenvalues in the open right half plane, the case of the positive real
// operators this solver targets).  Every iteration is two Gauss-Jordan inversions and the
// products for C (two with q columns while C is kept as L R^T, see solve()), which map onto
// the GPU; the paper solves the same equation with Bartels-Stewart (Sec. 6), whose Schur
// decompositions do not.  Near convergence, up to order NS_MAX_M, the inversions are
// replaced by Newton-Schulz steps (GEMMs only).  When a limit is not the identity the projected matrix
// is indefinite (the paper's Example 4.5 shows this can happen); the traces of the limits
// count the eigenvalues in the left half plane, and the part of Y on them is added by a
// spectral deflation (below).
#include <algorithm>
#include <cmath>
#include <vector>

#include "dense.hpp"
#include "proj.hpp"

namespace skr {
namespace {

// Relative change of the sign iterates below which the inverses are approximated
// (Newton-Schulz); scaling is off by then (it stops below 1e-2).
constexpr double NS_SWITCH = 5e-3;
// Orders up to which Newton-Schulz steps are taken: above it an exact step (two concurrent
// eliminations, with C in factored form) costs less than the eight dense products of a
// Newton-Schulz step (measured on one MI355X: 45 ms against 62 ms at order 6000, about
// equal at 4000).
constexpr int NS_MAX_M = 4096;
// projected residual above which the solution is refined once (iterative refinement)
constexpr double REFINE_AT = 1e-10;

enum Scal { MU = 0, DA, NA, TA, DB, NB_, TB, DC, NC, RHO2, RHO2B, RES2, F2, YN2, AI2, BI2, A2, B2, SCAL_N };

__global__ void set_scalar_kernel(double* p, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void copy_scalar_kernel(const double* src, double* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

// Frobenius-norm scaling of the sign iteration, mu = (||Z^{-1}||_F / ||Z||_F)^(1/2) with the
// diagonal blocks of Z = [[A, C], [0, -B]] standing in for Z (the coupling block C does not
// enter the spectrum); mu = 1 once the iteration is in its quadratic phase.
__global__ void mu_kernel(double* s, int scale) {
  if (threadIdx.x == 0 && blockIdx.x == 0) s[MU] = scale ? pow((s[AI2] + s[BI2]) / (s[A2] + s[B2]), 0.25) : 1.0;
}

// F: zero except its top-left r x r block = F11 (row-major) ; column-major m x m
__global__ void rhs_kernel(int m, int r, const double* F11, double* F) {
  const size_t total = (size_t)m * m;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    F[e] = (i < r && j < r) ? F11[i * r + j] : 0.0;
  }
}

// F = E_r F11 E_r^T in factored form L R^T (m x r each): L = E_r, R = E_r F11^T.
__global__ void frhs_kernel(int m, int r, const double* F11, double* L, double* R) {
  const size_t total = (size_t)m * r;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), t = (int)(e / m);
    L[e] = (i == t) ? 1.0 : 0.0;
    R[e] = (i < r) ? F11[t * r + i] : 0.0;
  }
}

// The right factor of a factored Newton step for C: its first mq entries (the old columns)
// scaled by mu / 2, the next mq (B^{-T} R) by 1 / (2 mu).
__global__ void fscale_kernel(size_t mq, const double* mu_dev, double* R) {
  const double mu = *mu_dev, lo = 0.5 * mu, hi = 0.5 / mu;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < 2 * mq; e += (size_t)gridDim.x * blockDim.x)
    R[e] *= (e < mq) ? lo : hi;
}

// rho^2 = ||hh Y[m-r:m, :]||_F^2 + ||Y[:, m-r:m] gh^T||_F^2, hh/gh r x r column-major with ld.
// out[0] = ||hh Y(m-r:m, :)||_F^2, out[1] = ||Y(:, m-r:m) gh^T||_F^2
__global__ void rho_kernel(int m, int r, const double* Y, const double* hh, int ldh, const double* gh, int ldg,
                           double* out) {
  __shared__ double red[2][16];
  double acc[2] = {0.0, 0.0};
  for (int e = threadIdx.x; e < 2 * m * r; e += blockDim.x) {
    const int which = e / (m * r), rem = e % (m * r);
    const int a = rem % r, j = rem / r;
    double t = 0.0;
    if (which == 0) {  // (hh Y_last)(a, j) = sum_c hh(a,c) Y(m-r+c, j)
      for (int c = 0; c < r; ++c) t += hh[a + (size_t)c * ldh] * Y[(m - r + c) + (size_t)j * m];
    } else {  // (Y_lastcol gh^T)(j, a) = sum_c Y(j, m-r+c) gh(a, c)
      for (int c = 0; c < r; ++c) t += Y[j + (size_t)(m - r + c) * m] * gh[a + (size_t)c * ldg];
    }
    acc[which] += t * t;
  }
  for (int q = 0; q < 2; ++q) {
    const double v = wave_sum(acc[q]);
    if (threadIdx.x % 64 == 0) red[q][threadIdx.x / 64] = v;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double s = 0.0;
    for (int w = 0; w < (int)blockDim.x / 64; ++w) s += red[threadIdx.x][w];
    out[threadIdx.x] = s;
  }
}

__global__ void scale_copy_kernel(size_t count, double alpha, const double* src, double* dst) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x)
    dst[e] = alpha * src[e];
}

// W = M_A Y + Y M_B^T - F has been formed except for "-F"; subtract F's block and reduce.
__global__ void sub_rhs_kernel(int m, int r, const double* F11, double* W) {
  const int e = threadIdx.x;
  if (e < r * r) W[(e / r) + (size_t)(e % r) * m] -= F11[(e / r) * r + e % r];
}

// ---- complete-pivoting low-rank factorisation -------------------------------------
constexpr int ACA_WG = 256, ACA_G = 2048, ACA_UN = 8;

// The residual update R -= u v^T of the previous cross and the partials of the next pivot
// search (largest |R(i, j)|, smallest index on ties) and of ||R||_F^2.  Columns across
// workgroups, rows across threads in batches of ACA_UN with every load issued before the
// batch is used (indices clamped into the column, the extra entries ignored), so that no
// index division is needed and a thread visits its entries in increasing order.
__global__ void __launch_bounds__(ACA_WG) aca_update_kernel(int m, double* R, const double* Y1, const double* Y2,
                                                            const int* state, double* part, int* ipart) {
  const int k = state[0], done = state[1];
  if (done) return;
  const double* u = k > 0 ? Y1 + (size_t)(k - 1) * m : nullptr;
  const double* v = k > 0 ? Y2 + (size_t)(k - 1) * m : nullptr;
  double best = -1.0, ss = 0.0;
  long long bidx = -1;
  for (int j = blockIdx.x; j < m; j += gridDim.x) {
    double* col = R + (size_t)j * m;
    const double vj = u ? v[j] : 0.0;
    for (int i0 = threadIdx.x; i0 < m; i0 += ACA_WG * ACA_UN) {
      double x[ACA_UN], uu[ACA_UN];
#pragma unroll
      for (int t = 0; t < ACA_UN; ++t) {
        const int ic = min(i0 + t * ACA_WG, m - 1);
        x[t] = col[ic];
        uu[t] = u ? u[ic] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < ACA_UN; ++t) {
        const int i = i0 + t * ACA_WG;
        if (i < m) {
          double xv = x[t];
          if (u) {
            xv -= uu[t] * vj;
            col[i] = xv;
          }
          const double ax = fabs(xv);
          ss += xv * xv;
          if (ax > best) { best = ax; bidx = (long long)j * m + i; }
        }
      }
    }
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
  if (threadIdx.x < 64) {  // one wavefront reduces the partials (fixed order)
    const int lane = threadIdx.x;
    double b = -1.0, s2 = 0.0;
    long long bi = -1;
    const long long* ip = reinterpret_cast<const long long*>(ipart);
    for (int g = lane; g < ng; g += 64) {
      s2 += part[ACA_G + g];
      if (part[g] > b || (part[g] == b && ip[g] >= 0 && (bi < 0 || ip[g] < bi))) { b = part[g]; bi = ip[g]; }
    }
    s2 = wave_sum(s2);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(b, off, 64);
      const long long oi = __shfl_xor(bi, off, 64);
      if (ob > b || (ob == b && oi >= 0 && (bi < 0 || oi < bi))) { b = ob; bi = oi; }
    }
    if (lane == 0) {
    const int k = state[0];
    if (k == 0) *ynorm2 = s2;
    stop = (k >= kmax) || !(b > 0.0) || bi < 0 || (s2 <= tol2 * *ynorm2);
    if (stop) state[1] = 1;
    pi = (int)(bi % m);
    pj = (int)(bi / m);
    pv = stop ? 1.0 : R[(size_t)pi + (size_t)pj * m];
    }
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

// ---- spectral deflation of the sign-function solve --------------------------------
// With S_A = sign(A), S_B = sign(B) (the limits of the coupled iteration) its C-limit W
// solves A W + W B = S_A F + F S_B, i.e. W = S_A Y + Y S_B, hence
//     Y = W/2 + P_A Y + Y P_B,   P = (I - S)/2 the spectral projector on the eigenvalues
// in the open left half plane.  Y P_B = Z L^T with P_B = R L^T (R orthonormal, q_B
// columns) and A Z + Z (R^T B R) = F R, a Sylvester equation with a q_B x q_B right
// coefficient solved through its complex Schur form and q_B shifted solves with A.
// P_A Y follows from the transposed equation.

// P = 0.5 (I - S) or 0.5 (I - S^T)
__global__ void half_i_minus_kernel(int m, const double* S, int lds, int trans, double* P) {
  const size_t total = (size_t)m * m;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    const double sv = trans ? S[j + (size_t)i * lds] : S[i + (size_t)j * lds];
    P[e] = 0.5 * ((i == j ? 1.0 : 0.0) - sv);
  }
}

__device__ inline uint64_t hash64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// m x q test matrix with entries uniform in [-1, 1)
__global__ void omega_kernel(int m, int q, uint64_t seed, double* O) {
  const size_t total = (size_t)m * q;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const uint64_t z = hash64(seed + (e + 1) * 0x9E3779B97F4A7C15ull);
    O[e] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

// Orthonormalise the columns of the m x q column-major G in place (classical Gram-Schmidt,
// two passes).  One workgroup.  info = 1 if a column loses more than 1 - 1e-10 of its norm.
__global__ void orth_kernel(int m, int q, double* G, int* info) {
  __shared__ double red[1024 / 64];
  __shared__ double coef[64];
  const int tid = threadIdx.x;
  auto wg_sum = [&](double v) {
    v = wave_sum(v);
    __syncthreads();
    if (tid % 64 == 0) red[tid / 64] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)blockDim.x / 64; ++w) t += red[w];
    return t;
  };
  for (int j = 0; j < q; ++j) {
    double* gj = G + (size_t)j * m;
    const double n0 = sqrt(wg_sum([&] { double a = 0.0; for (int i = tid; i < m; i += blockDim.x) a += gj[i] * gj[i]; return a; }()));
    for (int pass = 0; pass < 2; ++pass) {
      for (int k = 0; k < j; ++k) {
        const double* gk = G + (size_t)k * m;
        double a = 0.0;
        for (int i = tid; i < m; i += blockDim.x) a += gk[i] * gj[i];
        const double c = wg_sum(a);
        if (tid == 0) coef[k] = c;
      }
      __syncthreads();
      for (int i = tid; i < m; i += blockDim.x) {
        double t = gj[i];
        for (int k = 0; k < j; ++k) t -= coef[k] * G[(size_t)k * m + i];
        gj[i] = t;
      }
      __syncthreads();
    }
    const double n1 = sqrt(wg_sum([&] { double a = 0.0; for (int i = tid; i < m; i += blockDim.x) a += gj[i] * gj[i]; return a; }()));
    if (!(n1 > 1e-10 * n0)) {
      if (tid == 0) *info = 1;
      return;
    }
    for (int i = tid; i < m; i += blockDim.x) gj[i] /= n1;
    __syncthreads();
  }
}

// RHS (m x q) = F R with F zero outside its top-left r x r block F(i, a) = F11[i r + a]
// (or F11[a r + i] for the transposed equation).
__global__ void rhs_proj_kernel(int m, int q, int r, const double* F11, int ft, const double* R, double* RHS) {
  const size_t total = (size_t)m * q;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), c = (int)(e / m);
    double t = 0.0;
    if (i < r)
      for (int a = 0; a < r; ++a) t += (ft ? F11[a * r + i] : F11[i * r + a]) * R[a + (size_t)c * m];
    RHS[e] = t;
  }
}

struct cx {
  double re, im;
};
__device__ inline cx cmk(double a, double b) { return {a, b}; }
__device__ inline cx cadd(cx a, cx b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cx csub(cx a, cx b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline cx cmul(cx a, cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cx cconj(cx a) { return {a.re, -a.im}; }
__device__ inline double cabs2(cx a) { return hypot(a.re, a.im); }
__device__ inline cx cscale(cx a, double s) { return {a.re * s, a.im * s}; }
__device__ inline cx csqrt2(cx z) {
  const double r = cabs2(z);
  double a = sqrt(0.5 * (r + z.re)), b = sqrt(0.5 * fmax(r - z.re, 0.0));
  if (z.im < 0) b = -b;
  return {a, b};
}

// Complex Schur form B = Q T Q^H of a small real q x q matrix (column-major), single thread:
// Householder reduction to Hessenberg form, then implicit single-shift QR sweeps with
// Wilkinson shifts and deflation.  T, Q are returned as real/imaginary parts.
__global__ void schur_kernel(int q, const double* B, double* Tre, double* Tim, double* Qre, double* Qim, int* info) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  auto H = [&](int i, int j) -> cx { return cmk(Tre[i + j * q], Tim[i + j * q]); };
  auto setH = [&](int i, int j, cx v) { Tre[i + j * q] = v.re; Tim[i + j * q] = v.im; };
  auto Q = [&](int i, int j) -> cx { return cmk(Qre[i + j * q], Qim[i + j * q]); };
  auto setQ = [&](int i, int j, cx v) { Qre[i + j * q] = v.re; Qim[i + j * q] = v.im; };
  for (int j = 0; j < q; ++j)
    for (int i = 0; i < q; ++i) {
      Tre[i + j * q] = B[i + j * q];
      Tim[i + j * q] = 0.0;
      Qre[i + j * q] = (i == j) ? 1.0 : 0.0;
      Qim[i + j * q] = 0.0;
    }
  // real Householder reduction to upper Hessenberg form
  double v[64];
  for (int k = 0; k + 2 < q; ++k) {
    double nrm2 = 0.0;
    for (int i = k + 1; i < q; ++i) { v[i] = Tre[i + k * q]; nrm2 += v[i] * v[i]; }
    const double nrm = sqrt(nrm2);
    if (nrm == 0.0) continue;
    const double alpha = v[k + 1] >= 0 ? -nrm : nrm;
    v[k + 1] -= alpha;
    double vv = 0.0;
    for (int i = k + 1; i < q; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    for (int j = 0; j < q; ++j) {  // rows k+1.. of H
      double t = 0.0;
      for (int i = k + 1; i < q; ++i) t += v[i] * Tre[i + j * q];
      t *= beta;
      for (int i = k + 1; i < q; ++i) Tre[i + j * q] -= t * v[i];
    }
    for (int i = 0; i < q; ++i) {  // columns k+1.. of H and of Q
      double t = 0.0, u = 0.0;
      for (int j = k + 1; j < q; ++j) { t += Tre[i + j * q] * v[j]; u += Qre[i + j * q] * v[j]; }
      t *= beta;
      u *= beta;
      for (int j = k + 1; j < q; ++j) { Tre[i + j * q] -= t * v[j]; Qre[i + j * q] -= u * v[j]; }
    }
  }
  const double eps = 2.220446049250313e-16;
  int hi = q - 1, its = 0;
  while (hi > 0) {
    int l = 0;
    for (int k = hi; k >= 1; --k) {
      const double sub = cabs2(H(k, k - 1));
      if (sub <= eps * (cabs2(H(k, k)) + cabs2(H(k - 1, k - 1))) || sub == 0.0) {
        setH(k, k - 1, cmk(0, 0));
        l = k;
        break;
      }
    }
    if (l == hi) { --hi; its = 0; continue; }
    if (++its > 100) { *info = 2; return; }
    const cx a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
    const cx half_tr = cscale(cadd(a, d), 0.5), dd = cscale(csub(a, d), 0.5);
    const cx disc = csqrt2(cadd(cmul(dd, dd), cmul(b, c)));
    const cx mu1 = cadd(half_tr, disc), mu2 = csub(half_tr, disc);
    cx mu = cabs2(csub(mu1, d)) < cabs2(csub(mu2, d)) ? mu1 : mu2;
    if (its % 11 == 10) mu = cadd(d, cmk(cabs2(c), 0.0));  // exceptional shift
    cx x = csub(H(l, l), mu), y = H(l + 1, l);
    for (int k = l; k < hi; ++k) {
      const double ax = cabs2(x), ay = cabs2(y), nrm = hypot(ax, ay);
      double cc;
      cx ss;
      if (nrm == 0.0) { cc = 1.0; ss = cmk(0, 0); }
      else if (ax == 0.0) { cc = 0.0; ss = cscale(cconj(y), 1.0 / ay); }
      else { cc = ax / nrm; ss = cscale(cmul(cscale(x, 1.0 / ax), cconj(y)), 1.0 / nrm); }
      for (int j = (k > l ? k - 1 : l); j < q; ++j) {  // rows k, k+1
        const cx h1 = H(k, j), h2 = H(k + 1, j);
        setH(k, j, cadd(cscale(h1, cc), cmul(ss, h2)));
        setH(k + 1, j, csub(cscale(h2, cc), cmul(cconj(ss), h1)));
      }
      const int imax = min(k + 2, hi);
      for (int i = 0; i <= imax; ++i) {  // columns k, k+1
        const cx h1 = H(i, k), h2 = H(i, k + 1);
        setH(i, k, cadd(cscale(h1, cc), cmul(h2, cconj(ss))));
        setH(i, k + 1, csub(cscale(h2, cc), cmul(h1, ss)));
      }
      for (int i = 0; i < q; ++i) {
        const cx q1 = Q(i, k), q2 = Q(i, k + 1);
        setQ(i, k, cadd(cscale(q1, cc), cmul(q2, cconj(ss))));
        setQ(i, k + 1, csub(cscale(q2, cc), cmul(q1, ss)));
      }
      if (k < hi - 1) { x = H(k + 1, k); y = H(k + 2, k); }
    }
  }
  for (int j = 0; j < q; ++j)
    for (int i = j + 1; i < q; ++i) { Tre[i + j * q] = 0.0; Tim[i + j * q] = 0.0; }
}

// rhs2 = [Re; Im] of Rt[:, j] - sum_{i<j} Zt[:, i] T(i, j)
__global__ void cplx_rhs_kernel(int m, int j, int q, const double* Rtre, const double* Rtim, const double* Zre,
                                const double* Zim, const double* Tre, const double* Tim, double* rhs2) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x) {
    double re = Rtre[e + (size_t)j * m], im = Rtim[e + (size_t)j * m];
    for (int i = 0; i < j; ++i) {
      const double zr = Zre[e + (size_t)i * m], zi = Zim[e + (size_t)i * m];
      const double tr = Tre[i + j * q], ti = Tim[i + j * q];
      re -= zr * tr - zi * ti;
      im -= zr * ti + zi * tr;
    }
    rhs2[e] = re;
    rhs2[m + e] = im;
  }
}

// K (2m x 2m) = [[A + a I, -b I], [b I, A + a I]] with a + ib = T(j, j)
__global__ void build_shift_kernel(int m, const double* A, int lda, const double* Tre, const double* Tim, int q, int j,
                                   double* K) {
  const double a = Tre[j + j * q], b = Tim[j + j * q];
  const int n2 = 2 * m;
  const size_t total = (size_t)n2 * n2;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n2), k = (int)(e / n2);
    const int bi = i / m, bk = k / m, ii = i % m, kk = k % m;
    double v;
    if (bi == bk) v = A[ii + (size_t)kk * lda] + (ii == kk ? a : 0.0);
    else v = (ii == kk) ? (bi == 0 ? -b : b) : 0.0;
    K[e] = v;
  }
}

// K (m x m) = A + a I with a = Re T(j, j)
__global__ void build_real_shift_kernel(int m, const double* A, int lda, const double* Tre, int q, int j, double* K) {
  const double a = Tre[j + j * q];
  const size_t total = (size_t)m * m;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), k = (int)(e / m);
    K[e] = A[i + (size_t)k * lda] + (i == k ? a : 0.0);
  }
}

__global__ void negate_kernel(int m, double* x) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x) x[e] = -x[e];
}

__global__ void split_kernel(int m, int j, const double* x, double* Zre, double* Zim) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x) {
    Zre[e + (size_t)j * m] = x[e];
    Zim[e + (size_t)j * m] = x[m + e];
  }
}

// Y += G (or G^T)
__global__ void add_kernel(int m, const double* G, int trans, double* Y) {
  const size_t total = (size_t)m * m;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    Y[e] += trans ? G[j + (size_t)i * m] : G[e];
  }
}

}  // namespace

constexpr int QMAX = 64;  // largest deflated subspace handled

ProjSolver::ProjSolver(int r, int mmax, hipStream_t st) : r_(r), mmax_(mmax), st_(st) {
  const size_t mm = (size_t)mmax * mmax;
  mbar_u_.alloc((size_t)(mmax + r) * mmax);
  mbar_v_.alloc((size_t)(mmax + r) * mmax);
  a_.alloc(mm); b_.alloc(mm); ai_.alloc(mm); bi_.alloc(mm); c_.alloc(mm); w1_.alloc(mm); w2_.alloc(mm); lu_.alloc(mm);
  gjw_a_.alloc(dense::gj_ints(mmax));
  gjw_b_.alloc(dense::gj_ints(mmax));
  gjd_a_.alloc(dense::gj_doubles(mmax));
  gjd_b_.alloc(dense::gj_doubles(mmax));
  lub_.alloc(mm);
  info_.alloc(2 + QMAX);  // [rank loss, Schur, one per shifted solve]
  scal_.alloc(SCAL_N);
  scratch_.alloc(dense::scratch_doubles());
  cscal_.alloc(3);
  cscratch_.alloc(dense::scratch_doubles());
  aux_ = stream_acquire();
  cst_ = stream_acquire();
  SKR_HIP(hipEventCreateWithFlags(&ev_main_, hipEventDisableTiming));
  SKR_HIP(hipEventCreateWithFlags(&ev_aux_, hipEventDisableTiming));
  SKR_HIP(hipEventCreateWithFlags(&ev_cin_, hipEventDisableTiming));
  SKR_HIP(hipEventCreateWithFlags(&ev_c_, hipEventDisableTiming));
  for (auto& d : dst_) d = stream_acquire();
  for (auto& e : dev_) SKR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

ProjSolver::~ProjSolver() {
  for (auto d : dst_)
    if (d) { (void)hipStreamSynchronize(d); stream_release(d); }
  for (auto e : dev_)
    if (e) (void)hipEventDestroy(e);
  if (aux_) (void)hipStreamSynchronize(aux_);
  if (cst_) (void)hipStreamSynchronize(cst_);
  if (ev_main_) (void)hipEventDestroy(ev_main_);
  if (ev_aux_) (void)hipEventDestroy(ev_aux_);
  if (ev_cin_) (void)hipEventDestroy(ev_cin_);
  if (ev_c_) (void)hipEventDestroy(ev_c_);
  if (aux_) stream_release(aux_);
  if (cst_) stream_release(cst_);
}

void ProjSolver::form(int d, const ProjSpace& sp, double* Mbar, hipStream_t st) {
  const int m = d * r_, ld = sp.ld, ldm = m + r_;
  // Mbar = T_{d+1} H_d_bar  ((m + r) x m)
  if (!sp.broken) {
    dense::gemm(false, false, m + r_, m, m + r_, 1.0, sp.T, ld, sp.H, ld, 0.0, Mbar, ldm, st);
  } else {  // h_{d+1,d} = 0: only T_d H_d, last block row zero
    dense::set_zero(m + r_, m, Mbar, ldm, st);
    dense::gemm(false, false, m, m, m, 1.0, sp.T, ld, sp.H, ld, 0.0, Mbar, ldm, st);
  }
  // Mbar <- Mbar T_d^{-1}
  dense::trsm_right_upper(m + r_, m, sp.T, ld, Mbar, ldm, st);
}


void ProjSolver::deflate_right(int m, const double* Al, int lal, const double* Mst, int lms, const double* S,
                               int s_trans, const double* F11, int f_trans, int q, double* G) {
  SKR_REQUIRE(q >= 1 && q <= QMAX, "deflated subspace too large");
  const size_t mq = (size_t)m * q;
  if (!dws_.p || dws_.n < 12 * (size_t)mmax_ * QMAX) dws_.alloc(12 * (size_t)mmax_ * QMAX + 8 * QMAX * QMAX);
  double* P = ai_.p;  // m x m
  double* O = dws_.p;
  double* R = O + mq;
  double* BR = R + mq;
  double* RHS = BR + mq;
  double* Rtre = RHS + mq;
  double* Rtim = Rtre + mq;
  double* Zre = Rtim + mq;
  double* Zim = Zre + mq;
  double* Lt = Zim + mq;       // q x m
  double* Zr = Lt + mq;        // m x q (real Z)
  double* rhs2 = Zr + mq;      // 2m
  double* Bq = rhs2 + 2 * (size_t)m;
  double* Tre = Bq + q * q;
  double* Tim = Tre + q * q;
  double* Qre = Tim + q * q;
  double* Qim = Qre + q * q;
  const int g = std::min(4096, ceil_div((int64_t)m * m, 256));
  hipLaunchKernelGGL(half_i_minus_kernel, dim3(g), dim3(256), 0, st_, m, S, m, s_trans, P);
  check_launch("half_i_minus");
  hipLaunchKernelGGL(omega_kernel, dim3(std::min(1024, ceil_div((int64_t)mq, 256))), dim3(256), 0, st_, m, q,
                     (uint64_t)0x5EED0000ull + (uint64_t)q, O);
  check_launch("omega");
  dense::gemm(false, false, m, q, m, 1.0, P, m, O, m, 0.0, R, m, st_);
  SKR_HIP(hipMemsetAsync(info_.p, 0, 2 * sizeof(int), st_));
  hipLaunchKernelGGL(orth_kernel, dim3(1), dim3(1024), 0, st_, m, q, R, info_.p);
  check_launch("orth");
  dense::gemm(true, false, m, q, m, 1.0, Mst, lms, R, m, 0.0, BR, m, st_);     // B R = Mst^T R
  dense::gemm(true, false, q, q, m, 1.0, R, m, BR, m, 0.0, Bq, q, st_);        // R^T B R
  dense::gemm(true, false, q, m, m, 1.0, R, m, P, m, 0.0, Lt, q, st_);         // L^T = R^T P
  hipLaunchKernelGGL(rhs_proj_kernel, dim3(std::min(1024, ceil_div((int64_t)mq, 256))), dim3(256), 0, st_, m, q, r_,
                     F11, f_trans, R, RHS);
  check_launch("rhs_proj");
  hipLaunchKernelGGL(schur_kernel, dim3(1), dim3(1), 0, st_, q, Bq, Tre, Tim, Qre, Qim, info_.p + 1);
  check_launch("schur");
  int hinfo[2];
  SKR_HIP(hipMemcpyAsync(hinfo, info_.p, 2 * sizeof(int), hipMemcpyDeviceToHost, st_));
  SKR_HIP(hipStreamSynchronize(st_));
  if (hinfo[0]) throw Error(SKR_EPROJ, "rank loss in the deflated spectral subspace");
  if (hinfo[1]) throw Error(SKR_EPROJ, "small Schur decomposition did not converge");
  dense::gemm(false, false, m, q, q, 1.0, RHS, m, Qre, q, 0.0, Rtre, m, st_);
  dense::gemm(false, false, m, q, q, 1.0, RHS, m, Qim, q, 0.0, Rtim, m, st_);
  // Shifted solves (A + lambda_j I) z_j = rhs_j, lambda_j = a_j + i b_j the diagonal of the
  // complex Schur form, in the order of the recurrence.  The matrices do not depend on the
  // recurrence, so they are eliminated first, DEFL_NS at a time on separate streams, and the
  // recurrence then only applies the inverses.  A real matrix's eigenvalues come in
  // conjugate pairs, and K(conj lambda) = P K(lambda) P with P = diag(I, -I) for the real
  // form K(lambda) = [[A + a I, -b I], [b I, A + a I]], so one elimination serves both
  // members of a pair (the second applies it with the imaginary halves negated); a real
  // shift needs only the m x m matrix A + a I, applied to the real and imaginary parts.
  std::vector<double> hT(2 * (size_t)q * q);
  SKR_HIP(hipMemcpyAsync(hT.data(), Tre, sizeof(double) * q * q, hipMemcpyDeviceToHost, st_));
  SKR_HIP(hipMemcpyAsync(hT.data() + (size_t)q * q, Tim, sizeof(double) * q * q, hipMemcpyDeviceToHost, st_));
  SKR_HIP(hipStreamSynchronize(st_));
  const int n2 = 2 * m;
  hipStream_t ss[DEFL_NS] = {st_, aux_, dst_[0], dst_[1]};
  if (!gapply_.p || gapply_.n < dense::gj_apply_doubles(2 * mmax_) + 2 * (size_t)mmax_)
    gapply_.alloc(dense::gj_apply_doubles(2 * mmax_) + 2 * (size_t)mmax_);
  double* sol = gapply_.p + dense::gj_apply_doubles(n2);  // 2m
  struct Rep { int j; bool real; };
  std::vector<Rep> reps;           // eliminations of the current chunk of the recurrence
  std::vector<int> use_rep(q), use_flip(q);
  auto flush = [&](int j0, int j1) {  // eliminate the chunk's matrices, then run j0 .. j1-1
    const int nr = (int)reps.size();
    while ((int)kbv_.size() < nr) {
      kbv_.emplace_back();
      gjwv_.emplace_back();
      gjdv_.emplace_back();
    }
    SKR_HIP(hipEventRecord(ev_main_, st_));
    for (int u = 1; u < std::min(nr, (int)DEFL_NS); ++u) SKR_HIP(hipStreamWaitEvent(ss[u], ev_main_, 0));
    // the shifted matrices, then their eliminations enqueued interleaved over the streams
    std::vector<dense::GjJob> jobs;
    for (int u = 0; u < nr; ++u) {
      const int nn = reps[u].real ? m : n2, j = reps[u].j;
      if (kbv_[u].n < (size_t)4 * mmax_ * mmax_) {
        kbv_[u].alloc((size_t)4 * mmax_ * mmax_);
        gjwv_[u].alloc(dense::gj_ints(2 * mmax_));
        gjdv_[u].alloc(dense::gj_doubles(2 * mmax_));
      }
      hipStream_t su = ss[u % DEFL_NS];
      if (reps[u].real)
        hipLaunchKernelGGL(build_real_shift_kernel, dim3(std::min(8192, ceil_div((int64_t)m * m, 256))), dim3(256), 0,
                           su, m, Al, lal, Tre, q, j, kbv_[u].p);
      else
        hipLaunchKernelGGL(build_shift_kernel, dim3(std::min(8192, ceil_div((int64_t)n2 * n2, 256))), dim3(256), 0,
                           su, m, Al, lal, Tre, Tim, q, j, kbv_[u].p);
      check_launch("build_shift");
      jobs.push_back({nn, nn, kbv_[u].p, nn, gjwv_[u].p, gjdv_[u].p, info_.p + 2 + j, nullptr, su});
    }
    // jobs on the same stream stay in their order: interleave in rounds of DEFL_NS jobs
    for (size_t u0 = 0; u0 < jobs.size(); u0 += DEFL_NS)
      dense::gj_eliminate_many(jobs.data() + u0, (int)std::min<size_t>(DEFL_NS, jobs.size() - u0));
    for (int u = 1; u < std::min(nr, (int)DEFL_NS); ++u) {
      SKR_HIP(hipEventRecord(dev_[u], ss[u]));
      SKR_HIP(hipStreamWaitEvent(st_, dev_[u], 0));
    }
    const int gm = std::min(1024, ceil_div(m, 256));
    for (int j = j0; j < j1; ++j) {
      const int u = use_rep[j];
      hipLaunchKernelGGL(cplx_rhs_kernel, dim3(gm), dim3(256), 0, st_, m, j, q, Rtre, Rtim, Zre, Zim, Tre, Tim, rhs2);
      check_launch("cplx_rhs");
      if (reps[u].real) {
        dense::gj_apply(m, kbv_[u].p, m, gjwv_[u].p, rhs2, sol, gapply_.p, st_);
        dense::gj_apply(m, kbv_[u].p, m, gjwv_[u].p, rhs2 + m, sol + m, gapply_.p, st_);
      } else {
        if (use_flip[j]) hipLaunchKernelGGL(negate_kernel, dim3(gm), dim3(256), 0, st_, m, rhs2 + m);
        dense::gj_apply(n2, kbv_[u].p, n2, gjwv_[u].p, rhs2, sol, gapply_.p, st_);
        if (use_flip[j]) hipLaunchKernelGGL(negate_kernel, dim3(gm), dim3(256), 0, st_, m, sol + m);
      }
      hipLaunchKernelGGL(split_kernel, dim3(gm), dim3(256), 0, st_, m, j, sol, Zre, Zim);
      check_launch("split");
    }
    reps.clear();
  };
  constexpr int REP_CHUNK = 16;  // eliminated matrices held at once
  int j0 = 0;
  for (int j = 0; j < q; ++j) {
    const double a = hT[j + (size_t)j * q], b = hT[(size_t)q * q + j + (size_t)j * q];
    const double sc = std::max({std::fabs(a), std::fabs(b), 1e-300});
    const bool real = std::fabs(b) <= 1e-13 * sc;
    int u = -1, flip = 0;
    for (int v = 0; v < (int)reps.size() && u < 0; ++v) {
      const int i = reps[v].j;
      const double ai = hT[i + (size_t)i * q], bi = hT[(size_t)q * q + i + (size_t)i * q];
      if (reps[v].real != real || std::fabs(a - ai) > 1e-12 * sc) continue;
      if (real || std::fabs(b - bi) <= 1e-12 * sc) u = v;
      else if (std::fabs(b + bi) <= 1e-12 * sc) { u = v; flip = 1; }
    }
    if (u < 0) {
      if ((int)reps.size() == REP_CHUNK) {
        flush(j0, j);
        j0 = j;
      }
      u = (int)reps.size();
      reps.push_back(Rep{j, real});
    }
    use_rep[j] = u;
    use_flip[j] = flip;
  }
  flush(j0, q);
  {
    int hq[QMAX];
    SKR_HIP(hipMemcpyAsync(hq, info_.p + 2, q * sizeof(int), hipMemcpyDeviceToHost, st_));
    SKR_HIP(hipStreamSynchronize(st_));
    for (int j = 0; j < q; ++j)
      if (hq[j]) throw Error(SKR_EPROJ, "singular shifted system in the deflated solve");
  }

  // Z = Re(Zt Q^H) = Zre Qre^T + Zim Qim^T ;  G = Z L^T
  dense::gemm(false, true, m, q, q, 1.0, Zre, m, Qre, q, 0.0, Zr, m, st_);
  dense::gemm(false, true, m, q, q, 1.0, Zim, m, Qim, q, 1.0, Zr, m, st_);
  dense::gemm(false, false, m, m, q, 1.0, Zr, m, Lt, q, 0.0, G, m, st_);
}

void ProjSolver::quiesce() {
  (void)hipStreamSynchronize(st_);
  if (aux_) (void)hipStreamSynchronize(aux_);
  if (cst_) (void)hipStreamSynchronize(cst_);
  for (auto s : dst_)
    if (s) (void)hipStreamSynchronize(s);
}

double ProjSolver::solve(int d, const ProjSpace& u, const ProjSpace& v, const double* F11, ProjStats* stats) {
  const int m = d * r_;
  SKR_REQUIRE(m <= mmax_, "projected size exceeds the allocation");
  m_ = m;
  const int ldm = m + r_;
  // the two spaces' products and triangular solves (chains of small launches) concurrently
  SKR_HIP(hipEventRecord(ev_main_, st_));
  SKR_HIP(hipStreamWaitEvent(aux_, ev_main_, 0));
  form(d, u, mbar_u_.p, st_);
  form(d, v, mbar_v_.p, aux_);
  SKR_HIP(hipEventRecord(ev_aux_, aux_));
  SKR_HIP(hipStreamWaitEvent(st_, ev_aux_, 0));
  double* s = scal_.p;
  std::vector<double> hs(SCAL_N);
  int hinfo[2];
  double pres = 0.0;
  // Pass 0 solves M_A Y + Y M_B^T = F.  When its projected residual misses REFINE_AT and no
  // eigenvalue needed the deflation, pass 1 refines: the same iteration on the residual
  // R = F - (M_A Y + Y M_B^T) gives E with M_A E + E M_B^T = R, and Y <- Y + E (iterative
  // refinement; the sign iteration's error is relative to its right-hand side, so one
  // refinement brings an ill-conditioned projected equation to about the square of it).
  for (int pass = 0; pass < 2; ++pass) {
  dense::copy(m, m, mbar_u_.p, ldm, a_.p, m, st_);
  dense::transpose(m, m, mbar_v_.p, ldm, b_.p, m, st_);
  // While the right-hand side is the rank-r F (pass 0), C is kept in factored form C = L R^T
  // (L in w1_, R in w2_, q columns each): an exact step appends A^{-1} L to L and B^{-T} R to
  // R, two products with q columns instead of two with m.  No truncation: the rank doubles
  // every step, and C is formed once 2q would pass m / 2, before a Newton-Schulz step and
  // after the iteration.
  bool fac = (pass == 0);
  int q = r_;
  auto form_c = [&]() {
    dense::gemm(false, true, m, m, q, 1.0, w1_.p, m, w2_.p, m, 0.0, c_.p, m, st_);
    fac = false;
  };
  if (pass == 0) {
    hipLaunchKernelGGL(frhs_kernel, dim3(std::max(1, std::min(4096, ceil_div((int64_t)m * r_, 256)))), dim3(256), 0,
                       st_, m, r_, F11, w1_.p, w2_.p);
    check_launch("frhs");
  } else {  // Y -> y1_ (free until the factorisation); c = R = -(M_A Y + Y M_B^T - F), left in w1_
    if (!y1_.p) { y1_.alloc((size_t)mmax_ * mmax_); y2_.alloc((size_t)mmax_ * mmax_); }
    dense::copy(m, m, c_.p, m, y1_.p, m, st_);
    hipLaunchKernelGGL(scale_copy_kernel, dim3(std::min(4096, ceil_div((int64_t)m * m, 256))), dim3(256), 0, st_,
                       (size_t)m * m, -1.0, w1_.p, c_.p);
    check_launch("scale_copy");
  }
  bool scale = true;
  double prev = 1e300;
  int it = 0, extra = -1;
  const int maxit = 100;
  // Near convergence the inverses are replaced by the Newton-Schulz approximation
  // X^{-1} ~ X (2I - X^2), which is the Newton step with a first-order inverse: applied to
  // the whole block matrix Z = [[A, C], [0, -B]] it gives A' = A (3I - A^2)/2, the same for B,
  // and C' = (C + 2C - A(AC) + (AC)B - C B^2)/2; it converges quadratically once
  // ||I - Z^2|| < 1 and costs GEMMs only.
  bool schulz = false;
  for (it = 0; it < maxit; ++it) {
    SKR_HIP(hipEventRecord(ev_main_, st_));
    SKR_HIP(hipStreamWaitEvent(aux_, ev_main_, 0));
    if (!schulz) {
      // A_k^{-1} on the solve's stream and B_k^{-1} on the auxiliary stream, concurrently
      // (the two elimination chains enqueued interleaved)
      if (!lyap_) dense::copy(m, m, b_.p, m, lub_.p, m, aux_);
      dense::copy(m, m, a_.p, m, lu_.p, m, st_);
      const dense::GjJob jobs[2] = {{m, m, lu_.p, m, gjw_a_.p, gjd_a_.p, info_.p, nullptr, st_},
                                    {m, m, lub_.p, m, gjw_b_.p, gjd_b_.p, info_.p + 1, nullptr, aux_}};
      dense::gj_eliminate_many(jobs, lyap_ ? 1 : 2);
      // the inverses overwrite what the previous step's product for C still reads
      SKR_HIP(hipStreamWaitEvent(aux_, ev_c_, 0));
      SKR_HIP(hipStreamWaitEvent(st_, ev_c_, 0));
      if (!lyap_) dense::gj_inverse(m, lub_.p, m, gjw_b_.p, bi_.p, m, aux_);
      SKR_HIP(hipEventRecord(ev_aux_, aux_));
      dense::gj_inverse(m, lu_.p, m, gjw_a_.p, ai_.p, m, st_);
      SKR_HIP(hipStreamWaitEvent(st_, ev_aux_, 0));
      if (lyap_) dense::transpose(m, m, ai_.p, m, bi_.p, m, st_);  // B_k = A_k^T
      if (scale) {
        dense::fro2(m, m, ai_.p, m, s + AI2, scratch_.p, st_);
        dense::fro2(m, m, bi_.p, m, s + BI2, scratch_.p, st_);
        dense::fro2(m, m, a_.p, m, s + A2, scratch_.p, st_);
        dense::fro2(m, m, b_.p, m, s + B2, scratch_.p, st_);
      }
      hipLaunchKernelGGL(mu_kernel, dim3(1), dim3(1), 0, st_, s, scale ? 1 : 0);
      check_launch("mu");
      hipLaunchKernelGGL(copy_scalar_kernel, dim3(1), dim3(1), 0, st_, s + MU, cscal_.p);
      check_launch("copy_scalar");
      // A_{k+1} and B_{k+1} first: the host's decision waits for them, and once the products
      // for C below are running they hold every compute unit
      dense::newton_combine(m, m, s + MU, a_.p, m, ai_.p, m, a_.p, m, s + DA, s + NA, s + TA, scratch_.p, st_);
      dense::newton_combine(m, m, s + MU, b_.p, m, bi_.p, m, b_.p, m, s + DB, s + NB_, s + TB, scratch_.p, st_);
      // C_{k+1} = (mu C + mu^{-1} A^{-1} C B^{-1}) / 2
      if (fac && 2 * q > m / 2) form_c();
      if (fac) {
        // L <- [L, A^{-1} L], R <- [mu R, B^{-T} R / mu] / 2
        dense::gemm(false, false, m, q, m, 1.0, ai_.p, m, w1_.p, m, 0.0, w1_.p + (size_t)q * m, m, st_);
        dense::gemm(true, false, m, q, m, 1.0, bi_.p, m, w2_.p, m, 0.0, w2_.p + (size_t)q * m, m, st_);
        hipLaunchKernelGGL(fscale_kernel, dim3(std::max(1, std::min(4096, ceil_div((int64_t)m * q, 128)))), dim3(256), 0,
                           st_, (size_t)m * q, s + MU, w2_.p);
        check_launch("fscale");
        q *= 2;
        SKR_HIP(hipEventRecord(ev_c_, st_));
      } else {
        // on a stream of its own: the host's decision needs only A_{k+1} and B_{k+1}, so the
        // two products for C may overlap the next step's elimination chains (whose inverses
        // wait for them)
        SKR_HIP(hipEventRecord(ev_cin_, st_));
        SKR_HIP(hipStreamWaitEvent(cst_, ev_cin_, 0));
        dense::gemm(false, false, m, m, m, 1.0, ai_.p, m, c_.p, m, 0.0, w1_.p, m, cst_);
        dense::gemm(false, false, m, m, m, 1.0, w1_.p, m, bi_.p, m, 0.0, w2_.p, m, cst_);
        dense::newton_combine(m, m, cscal_.p, c_.p, m, w2_.p, m, c_.p, m, cscal_.p + 1, cscal_.p + 2, nullptr,
                              cscratch_.p, cst_);
        SKR_HIP(hipEventRecord(ev_c_, cst_));
      }
    } else {
      if (fac) form_c();
      // the products below overwrite what the last exact step's product for C still reads
      SKR_HIP(hipStreamWaitEvent(aux_, ev_c_, 0));
      SKR_HIP(hipStreamWaitEvent(st_, ev_c_, 0));
      // B^2 -> lub_, B^{-1} ~ 2B - B B^2 -> bi_ on the auxiliary stream
      if (!lyap_) {
        dense::gemm(false, false, m, m, m, 1.0, b_.p, m, b_.p, m, 0.0, lub_.p, m, aux_);
        dense::copy(m, m, b_.p, m, bi_.p, m, aux_);
        dense::gemm(false, false, m, m, m, -1.0, b_.p, m, lub_.p, m, 2.0, bi_.p, m, aux_);
      }
      SKR_HIP(hipEventRecord(ev_aux_, aux_));
      // A^2 -> lu_, A^{-1} ~ 2A - A A^2 -> ai_
      dense::gemm(false, false, m, m, m, 1.0, a_.p, m, a_.p, m, 0.0, lu_.p, m, st_);
      dense::copy(m, m, a_.p, m, ai_.p, m, st_);
      dense::gemm(false, false, m, m, m, -1.0, a_.p, m, lu_.p, m, 2.0, ai_.p, m, st_);
      if (lyap_) {  // B = A^T: B^2 = (A^2)^T and the approximate inverse transposes too
        dense::transpose(m, m, lu_.p, m, lub_.p, m, st_);
        dense::transpose(m, m, ai_.p, m, bi_.p, m, st_);
      }
      // w2 = 2C + (AC)B - A(AC) - C B^2, the (1,2) block of Z (2I - Z^2)
      dense::gemm(false, false, m, m, m, 1.0, a_.p, m, c_.p, m, 0.0, w1_.p, m, st_);
      dense::copy(m, m, c_.p, m, w2_.p, m, st_);
      dense::gemm(false, false, m, m, m, 1.0, w1_.p, m, b_.p, m, 2.0, w2_.p, m, st_);
      dense::gemm(false, false, m, m, m, -1.0, a_.p, m, w1_.p, m, 1.0, w2_.p, m, st_);
      SKR_HIP(hipStreamWaitEvent(st_, ev_aux_, 0));
      dense::gemm(false, false, m, m, m, -1.0, c_.p, m, lub_.p, m, 1.0, w2_.p, m, st_);
      hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, st_, s + MU, 1.0);
      check_launch("set_scalar");
      dense::newton_combine(m, m, s + MU, c_.p, m, w2_.p, m, c_.p, m, s + DC, s + NC, nullptr, scratch_.p, st_);
      dense::newton_combine(m, m, s + MU, a_.p, m, ai_.p, m, a_.p, m, s + DA, s + NA, s + TA, scratch_.p, st_);
      dense::newton_combine(m, m, s + MU, b_.p, m, bi_.p, m, b_.p, m, s + DB, s + NB_, s + TB, scratch_.p, st_);
    }
    SKR_HIP(hipMemcpyAsync(hs.data(), s, SCAL_N * sizeof(double), hipMemcpyDeviceToHost, st_));
    SKR_HIP(hipMemcpyAsync(hinfo, info_.p, 2 * sizeof(int), hipMemcpyDeviceToHost, st_));
    SKR_HIP(hipStreamSynchronize(st_));
    if (hinfo[0] || (!lyap_ && hinfo[1]))  // the Lyapunov solve does not invert B
      throw Error(SKR_EPROJ, "projected matrix singular during the sign iteration (d = " + std::to_string(d) + ")");
    const double rel = std::sqrt(std::max(hs[DA] / hs[NA], hs[DB] / hs[NB_]));
    if (!std::isfinite(rel))
      throw Error(SKR_EPROJ, "non-finite sign iteration (d = " + std::to_string(d) + ")");
    const bool unscaled = !scale;  // this step used mu = 1
    if (rel < 1e-2) scale = false;
    // Quadratic convergence: the error of the new iterate is about the square of this step's
    // change, so an unscaled step whose change is below 1e-8 after one below 1e-3 (the
    // quadratic phase) leaves it at rounding level; a change below 1e-10 ends the iteration
    // in any case.
    if (rel < 1e-10 || (unscaled && prev < 1e-3 && rel < 1e-8)) { ++it; break; }
    if (schulz) {
      if (rel > 0.25 * prev) schulz = false;  // not contracting quadratically: exact inverses again
    } else if (!scale && rel < NS_SWITCH && m <= NS_MAX_M) {
      schulz = true;
    }
    if (extra >= 0) {
      if (--extra < 0) { ++it; break; }
    } else if (rel < 1e-6 && rel > 0.5 * prev) {
      extra = 1;  // stagnation at rounding level
    }
    prev = rel;
  }
  SKR_HIP(hipStreamWaitEvent(st_, ev_c_, 0));  // C of the last exact step
  if (fac) form_c();
  const int qa = (int)std::lround((m - hs[TA]) / 2.0), qb = (int)std::lround((m - hs[TB]) / 2.0);
  if (stats) {
    if (pass == 0) stats->newton_iters = it;
    stats->neg_eigs_a = qa;
    stats->neg_eigs_b = qb;
  }
  if (it >= maxit) throw Error(SKR_EPROJ, "sign iteration did not converge (d = " + std::to_string(d) + ")");
  if (qa < 0 || qb < 0 || qa > QMAX || qb > QMAX)
    throw Error(SKR_EPROJ, "projected matrices have too many eigenvalues in the left half plane (" +
                               std::to_string(qa) + ", " + std::to_string(qb) + ") at d = " + std::to_string(d));
  // Y = C / 2:  (mu X + 0 / mu) / 2 with mu = 1
  hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, st_, s + MU, 1.0);
  check_launch("set_scalar");
  dense::copy(m, m, c_.p, m, w1_.p, m, st_);
  dense::set_zero(m, m, w2_.p, m, st_);
  dense::newton_combine(m, m, s + MU, w1_.p, m, w2_.p, m, c_.p, m, s + DC, s + YN2, nullptr, scratch_.p, st_);
  if (pass == 1) {  // Y + E
    hipLaunchKernelGGL(add_kernel, dim3(std::min(4096, ceil_div((int64_t)m * m, 256))), dim3(256), 0, st_, m, y1_.p,
                       0, c_.p);
    check_launch("add");
  }
  // eigenvalues in the left half plane: Y = W/2 + P_A Y + Y P_B
  if (qb > 0) {  // Y P_B with A = M_A, B = M_B^T
    deflate_right(m, mbar_u_.p, ldm, mbar_v_.p, ldm, b_.p, 0, F11, 0, qb, bi_.p);
    hipLaunchKernelGGL(add_kernel, dim3(std::min(4096, ceil_div((int64_t)m * m, 256))), dim3(256), 0, st_, m, bi_.p, 0,
                       c_.p);
    check_launch("add");
  }
  if (qa > 0) {  // (P_A Y)^T = Y^T P_{A^T}: transposed equation M_B Y^T + Y^T M_A^T = F^T
    deflate_right(m, mbar_v_.p, ldm, mbar_u_.p, ldm, a_.p, 1, F11, 1, qa, bi_.p);
    hipLaunchKernelGGL(add_kernel, dim3(std::min(4096, ceil_div((int64_t)m * m, 256))), dim3(256), 0, st_, m, bi_.p, 1,
                       c_.p);
    check_launch("add");
  }
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
  pres = std::sqrt(hs[RES2] / hs[F2]);
  if (pass == 1 || pres <= REFINE_AT || qa != 0 || qb != 0) break;
  }
  if (stats) stats->proj_resid = pres;
  if (!(pres <= 1e-6))
    throw Error(SKR_EPROJ, "projected Sylvester residual " + std::to_string(pres) + " at d = " + std::to_string(d));
  if (trunc_est_) return std::sqrt((double)m) * (std::sqrt(hs[RHO2]) + std::sqrt(hs[RHO2B]));
  return std::sqrt(hs[RHO2] + hs[RHO2B]);
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
