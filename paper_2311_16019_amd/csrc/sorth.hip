// Sketch-space part of the sketched-inner-product block step: block Gram-Schmidt of w = S U~
// against the window's sketches, Cholesky QR twice of the remainder, the coefficients of the
// long update U_{d+1} = (U~ - sum_i U_i h_i) R^{-1}, and the breakdown test.  All of it works
// on s-row arrays (s = O(maxit r)), so one workgroup per space suffices.
#include "small_la.hpp"
#include "sorth.hpp"

namespace skr {
namespace {

constexpr int ST = 1024;  // threads of the workgroup
constexpr int SKW = 3;   // window blocks
// Breakdown thresholds (not discussed in the paper; the same values as the FP64 oracle):
// the orthogonalised sketch is negligible against S U~, or its R factor is numerically
// singular.
constexpr double BREAK_NORM = 1e-12;
constexpr double BREAK_DIAG = 1e-14;

// Workgroup sum of per-thread r x r partials into out (LDS); fixed order throughout.
template <int R>
__device__ void wg_reduce(const double (&acc)[R * R], double* out, double* red) {
  constexpr int RR = R * R;
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
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

template <int R>
__device__ inline void cross_add(double (&acc)[R * R], const double (&x)[R], const double (&y)[R]) {
#pragma unroll
  for (int a = 0; a < R; ++a)
#pragma unroll
    for (int b = 0; b < R; ++b) acc[a * R + b] += x[a] * y[b];
}

// y = x M for an upper triangular M (row-major)
template <int R>
__device__ inline void times_upper(const double (&x)[R], const double* M, double (&y)[R]) {
#pragma unroll
  for (int c = 0; c < R; ++c) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k <= c; ++k) t += x[k] * M[k * R + c];
    y[c] = t;
  }
}

// Thread t owns the rows t, t + ST, .. of every s x r array throughout, so an update and
// the products that follow it need no barrier between them.  The passes over the s rows:
//   0       ||w||_F^2 and h_1 = W_1^T w
//   1 .. nw w -= W_i h_i (stored), then h_{i+1} = W_{i+1}^T w, or G = w^T w after the last
//   nw + 1  G' = (w R1^{-1})^T (w R1^{-1})  (Cholesky QR, second pass; nothing stored)
//   nw + 2  S U_{d+1} = w R1^{-1} R2^{-1} into the ring slot and the whitening input
template <int R>
__global__ void __launch_bounds__(ST) sorth_kernel(SorthSpace a0, SorthSpace a1, int s, int nw, int i0, int d) {
  constexpr int RR = R * R;
  const SorthSpace& a = blockIdx.x ? a1 : a0;
  __shared__ double red[(ST / 64) * RR];
  __shared__ double h[SKW][RR], G[RR], N0[RR], R1[RR], R1i[RR], R2[RR], R2i[RR], RF[RR], RFi[RR];
  __shared__ int ok_sh;
  const int tid = threadIdx.x;
  double* w = a.w;
  auto ring = [&](int j) -> double* { return a.ring + (size_t)(j % a.nring) * s * R; };
  {
    double acc[RR], nacc[RR];
#pragma unroll
    for (int p = 0; p < RR; ++p) acc[p] = nacc[p] = 0.0;
    const double* W1 = nw > 0 ? ring(i0) : w;
#pragma unroll 2
    for (int i = tid; i < s; i += ST) {
      double x[R], y[R];
      load_row<double, R>(w, i, y);
      load_row<double, R>(W1, i, x);
      cross_add<R>(acc, x, y);
      cross_add<R>(nacc, y, y);
    }
    wg_reduce<R>(nacc, N0, red);
    wg_reduce<R>(acc, nw > 0 ? h[0] : G, red);
  }
  for (int j = 0; j < nw; ++j) {
    const double* Wj = ring(i0 + j);
    const double* Wn = j + 1 < nw ? ring(i0 + j + 1) : w;
    double acc[RR];
#pragma unroll
    for (int p = 0; p < RR; ++p) acc[p] = 0.0;
#pragma unroll 2
    for (int i = tid; i < s; i += ST) {
      double x[R], y[R], z[R];
      load_row<double, R>(Wj, i, x);
      load_row<double, R>(w, i, y);
#pragma unroll
      for (int b = 0; b < R; ++b)
#pragma unroll
        for (int c = 0; c < R; ++c) y[b] -= x[c] * h[j][c * R + b];
      store_row<double, R>(w, i, y);
      if (j + 1 < nw) {
        load_row<double, R>(Wn, i, z);
      } else {
#pragma unroll
        for (int c = 0; c < R; ++c) z[c] = y[c];
      }
      cross_add<R>(acc, z, y);
    }
    wg_reduce<R>(acc, j + 1 < nw ? h[j + 1] : G, red);
  }
  // Cholesky QR twice of the remainder: w = q R2 R1
  if (tid == 0) {
    double t0 = 0.0, t = 0.0;
    for (int c = 0; c < R; ++c) { t0 += N0[c * R + c]; t += G[c * R + c]; }
    bool ok = t >= BREAK_NORM * BREAK_NORM * t0 && chol_upper(G, R1, R);
    if (ok) inv_upper(R1, R1i, R);
    ok_sh = ok ? 1 : 0;
  }
  __syncthreads();
  bool ok = ok_sh != 0;  // uniform over the workgroup
  if (ok) {
    double acc[RR];
#pragma unroll
    for (int p = 0; p < RR; ++p) acc[p] = 0.0;
#pragma unroll 2
    for (int i = tid; i < s; i += ST) {
      double x[R], y[R];
      load_row<double, R>(w, i, x);
      times_upper<R>(x, R1i, y);
      cross_add<R>(acc, y, y);
    }
    wg_reduce<R>(acc, G, red);
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
      for (int p = 0; p < RR; ++p) { RF[p] = 0.0; RFi[p] = 0.0; }
    }
    ok_sh = ok ? 1 : 0;
  }
  __syncthreads();
  // S U_{d+1} = w R^{-1} (zero after a breakdown)
  double* out = ring(d + 1);
#pragma unroll 2
  for (int i = tid; i < s; i += ST) {
    double x[R], y[R];
    load_row<double, R>(w, i, x);
    times_upper<R>(x, RFi, y);
    store_row<double, R>(out, i, y);
    if (a.wout) store_row<double, R>(a.wout, i, y);
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
