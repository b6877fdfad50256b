// Sketch-space part of the sketched-inner-product block step: block Gram-Schmidt of w = S U~
// against the window's sketches, Cholesky QR twice of the remainder, the coefficients of the
// long update U_{d+1} = (U~ - sum_i U_i h_i) R^{-1}, and the breakdown test.  All of it works
// on s-row arrays (s = O(maxit r)), so one workgroup per space suffices.
#include "small_la.hpp"
#include "sorth.hpp"

namespace skr {
namespace {

constexpr int ST = 512;  // threads of the workgroup
constexpr int SKW = 3;   // window blocks
// Breakdown thresholds (not discussed in the paper; the same values as the FP64 oracle):
// the orthogonalised sketch is negligible against S U~, or its R factor is numerically
// singular.
constexpr double BREAK_NORM = 1e-12;
constexpr double BREAK_DIAG = 1e-14;

// out (r x r row-major, LDS) = X^T Y for s x R row-major X, Y.  Thread t owns rows
// t, t + ST, ..; the order of the sums is fixed.
template <int R>
__device__ void wg_cross(const double* X, const double* Y, int s, double* out, double* red) {
  constexpr int RR = R * R;
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  double acc[RR];
#pragma unroll
  for (int p = 0; p < RR; ++p) acc[p] = 0.0;
#pragma unroll 4
  for (int i = tid; i < s; i += ST) {
    double x[R], y[R];
    load_row<double, R>(X, i, x);
    load_row<double, R>(Y, i, y);
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int b = 0; b < R; ++b) acc[a * R + b] += x[a] * y[b];
  }
#pragma unroll
  for (int p = 0; p < RR; ++p) {
    const double v = wave_sum(acc[p]);
    if (lane == 0) red[wv * RR + p] = v;
  }
  __syncthreads();
  if (tid < RR) {
    double t = 0.0;
    for (int q = 0; q < ST / 64; ++q) t += red[q * RR + tid];
    out[tid] = t;
  }
  __syncthreads();
}

// rows of w <- w M for an upper triangular M (row-major)
template <int R>
__device__ void right_upper(double* w, int s, const double* M) {
#pragma unroll 4
  for (int i = threadIdx.x; i < s; i += ST) {
    double x[R], y[R];
    load_row<double, R>(w, i, x);
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k <= c; ++k) t += x[k] * M[k * R + c];
      y[c] = t;
    }
    store_row<double, R>(w, i, y);
  }
}

template <int R>
__global__ void __launch_bounds__(ST) sorth_kernel(SorthSpace a0, SorthSpace a1, int s, int nw, int i0, int d) {
  constexpr int RR = R * R;
  const SorthSpace& a = blockIdx.x ? a1 : a0;
  __shared__ double red[(ST / 64) * RR];
  __shared__ double h[SKW][RR], G[RR], R1[RR], R1i[RR], R2[RR], R2i[RR], RF[RR], RFi[RR];
  __shared__ double nrm0;
  __shared__ int ok_sh;
  const int tid = threadIdx.x;
  double* w = a.w;
  wg_cross<R>(w, w, s, G, red);
  if (tid == 0) {
    double t = 0.0;
    for (int c = 0; c < R; ++c) t += G[c * R + c];
    nrm0 = t;  // ||S U~||_F^2
  }
  // block Gram-Schmidt in the sketched inner product; a thread updates only the rows whose
  // sums it owns, so no barrier is needed between a product and its update
  for (int i = 0; i < nw; ++i) {
    const double* Wi = a.ring + (size_t)((i0 + i) % a.nring) * s * R;
    wg_cross<R>(Wi, w, s, h[i], red);
#pragma unroll 4
    for (int row = tid; row < s; row += ST) {
      double x[R], y[R];
      load_row<double, R>(Wi, row, x);
      load_row<double, R>(w, row, y);
#pragma unroll
      for (int b = 0; b < R; ++b)
#pragma unroll
        for (int c = 0; c < R; ++c) y[b] -= x[c] * h[i][c * R + b];
      store_row<double, R>(w, row, y);
    }
  }
  // Cholesky QR twice of the remainder: w = q R2 R1
  wg_cross<R>(w, w, s, G, red);
  if (tid == 0) {
    double t = 0.0;
    for (int c = 0; c < R; ++c) t += G[c * R + c];
    bool ok = t >= BREAK_NORM * BREAK_NORM * nrm0 && chol_upper(G, R1, R);
    if (ok) inv_upper(R1, R1i, R);
    ok_sh = ok ? 1 : 0;
  }
  __syncthreads();
  bool ok = ok_sh != 0;  // uniform over the workgroup
  if (ok) {
    right_upper<R>(w, s, R1i);
    wg_cross<R>(w, w, s, G, red);
  }
  if (tid == 0) {
    if (ok) ok = chol_upper(G, R2, R);
    if (ok) {
      matmul_small(R2, R1, RF, R);
      inv_upper(R2, R2i, R);
      matmul_small(R1i, R2i, RFi, R);
      double mx = 0.0, mn = 1e308;
      for (int p = 0; p < RR; ++p) mx = fmax(mx, fabs(RF[p]));
      for (int c = 0; c < R; ++c) mn = fmin(mn, RF[c * R + c]);
      ok = mn > BREAK_DIAG * mx;
    }
    if (!ok) {
      atomicMin(a.broken, d);
      for (int p = 0; p < RR; ++p) { RF[p] = 0.0; RFi[p] = 0.0; R2i[p] = 0.0; }
    }
    ok_sh = ok ? 1 : 0;
  }
  __syncthreads();
  ok = ok_sh != 0;
  // S U_{d+1} = w R2^{-1} (zero after a breakdown)
  double* out = a.ring + (size_t)((d + 1) % a.nring) * s * R;
#pragma unroll 4
  for (int i = tid; i < s; i += ST) {
    double x[R], y[R];
    load_row<double, R>(w, i, x);
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k <= c; ++k) t += x[k] * R2i[k * R + c];
      y[c] = ok ? t : 0.0;
    }
    store_row<double, R>(out, i, y);
    store_row<double, R>(a.wout, i, y);
  }
  // coefficients of U_{d+1} = U~ R^{-1} - sum_i U_i (h_i R^{-1}); all zero after a breakdown
  for (int e = tid; e < (nw + 1) * RR; e += ST) {
    const int blk = e / RR, p = e % RR, ra = p / R, cb = p % R;
    double t = 0.0;
    if (blk == 0) {
      t = RFi[p];
    } else {
      for (int c = 0; c < R; ++c) t += h[blk - 1][ra * R + c] * RFi[c * R + cb];
    }
    a.coef[e] = t;
  }
  // h_{i0+i, d} and h_{d+1, d} = R (column-major); for the start block R goes to H itself
  for (int e = tid; e < nw * RR; e += ST) {
    const int i = e / RR, p = e % RR, ra = p / R, cb = p % R;
    a.H[((size_t)(i0 + i - 1) * R + ra) + ((size_t)(d - 1) * R + cb) * a.ldh] = h[i][p];
  }
  for (int p = tid; p < RR; p += ST) {
    const int ra = p / R, cb = p % R;
    a.H[((size_t)d * R + ra) + ((size_t)(d > 0 ? d - 1 : 0) * R + cb) * a.ldh] = RF[p];
  }
}

template <int R>
void launch_r(int s, int nw, int i0, int d, const SorthSpace& a, const SorthSpace& b, int nspaces,
              hipStream_t st) {
  hipLaunchKernelGGL((sorth_kernel<R>), dim3(nspaces), dim3(ST), 0, st, a, b, s, nw, i0, d);
}

}  // namespace

void launch_sorth(int r, int s, int nw, int i0, int d, const SorthSpace& a, const SorthSpace& b, int nspaces,
                  hipStream_t st) {
  SKR_REQUIRE(nw >= 0 && nw <= SKW && (d == 0) == (nw == 0), "sketched orthogonalisation: invalid window");
  SKR_REQUIRE(nw == 0 || (i0 >= 1 && i0 + nw - 1 == d), "sketched orthogonalisation: window must end at d");
  SKR_REQUIRE(a.nring > nw && (nspaces == 1 || b.nring > nw), "sketched orthogonalisation: ring too short");
  SKR_REQUIRE(nspaces == 1 || nspaces == 2, "sketched orthogonalisation: one or two spaces");
  switch (r) {
    case 1: launch_r<1>(s, nw, i0, d, a, b, nspaces, st); break;
    case 2: launch_r<2>(s, nw, i0, d, a, b, nspaces, st); break;
    case 3: launch_r<3>(s, nw, i0, d, a, b, nspaces, st); break;
    case 4: launch_r<4>(s, nw, i0, d, a, b, nspaces, st); break;
    default: throw Error(SKR_ENOTSUP, "sketched orthogonalisation needs r <= 4");
  }
  check_launch("sorth");
}

}  // namespace skr
