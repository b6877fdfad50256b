// Sketched QR update (Prop. 2.1), FP64.  Q is column-major (s x columns, ld = s) so that
// appending a block writes contiguous memory and the product Q c reads Q with unit stride
// across the threads of a wavefront.
#include <algorithm>

#include "whiten.hpp"

namespace skr {
namespace {

constexpr int WT = 256;      // threads for the streaming whitening kernels
constexpr int FT = 1024;     // threads of the finishing workgroup
constexpr int SPLIT_COLS = 128;

template <int R>
constexpr int jb_of() { return R <= 4 ? 8 : (R <= 8 ? 4 : 2); }

template <int R>
__global__ void __launch_bounds__(WT) qtw_kernel(WhitenSpace a0, WhitenSpace a1, int s, int m, int which) {
  constexpr int JB = jb_of<R>();
  const WhitenSpace& a = blockIdx.y ? a1 : a0;
  const int j0 = blockIdx.x * JB;
  double acc[JB][R];
#pragma unroll
  for (int jb = 0; jb < JB; ++jb)
#pragma unroll
    for (int c = 0; c < R; ++c) acc[jb][c] = 0.0;
  for (int i = threadIdx.x; i < s; i += WT) {
    double wr[R];
#pragma unroll
    for (int c = 0; c < R; ++c) wr[c] = a.w[(size_t)i * R + c];
    double q[JB];
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) q[jb] = (j0 + jb < m) ? a.Q[(size_t)(j0 + jb) * s + i] : 0.0;
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
      for (int c = 0; c < R; ++c) acc[jb][c] += q[jb] * wr[c];
  }
  __shared__ double red[WT / 64][JB * R];
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
#pragma unroll
  for (int jb = 0; jb < JB; ++jb)
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const double v = wave_sum(acc[jb][c]);
      if (lane == 0) red[wv][jb * R + c] = v;
    }
  __syncthreads();
  double* out = which ? a.c2 : a.c1;
  for (int e = threadIdx.x; e < JB * R; e += WT) {
    const int j = j0 + e / R;
    if (j < m) {
      double t = 0.0;
      for (int w = 0; w < WT / 64; ++w) t += red[w][e];
      out[(size_t)j * R + e % R] = t;
    }
  }
}

template <int R>
__global__ void __launch_bounds__(WT) qc_part_kernel(WhitenSpace a0, WhitenSpace a1, int s, int m, int which,
                                                      int cols_per_split) {
  const WhitenSpace& a = blockIdx.z ? a1 : a0;
  const int i = blockIdx.x * WT + threadIdx.x;
  const int j0 = blockIdx.y * cols_per_split, j1 = min(m, j0 + cols_per_split);
  extern __shared__ double cs[];  // the split's rows of c, staged once per workgroup
  const double* c = which ? a.c2 : a.c1;
  for (int e = threadIdx.x; e < (j1 - j0) * R; e += WT) cs[e] = c[(size_t)j0 * R + e];
  __syncthreads();
  if (i >= s) return;
  double acc[R];
#pragma unroll
  for (int cc = 0; cc < R; ++cc) acc[cc] = 0.0;
  int j = j0;
  for (; j + 4 <= j1; j += 4) {
    double q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = a.Q[(size_t)(j + u) * s + i];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int cc = 0; cc < R; ++cc) acc[cc] += q[u] * cs[(j + u - j0) * R + cc];
  }
  for (; j < j1; ++j) {
    const double q = a.Q[(size_t)j * s + i];
#pragma unroll
    for (int cc = 0; cc < R; ++cc) acc[cc] += q * cs[(j - j0) * R + cc];
  }
#pragma unroll
  for (int cc = 0; cc < R; ++cc) a.part[((size_t)blockIdx.y * s + i) * R + cc] = acc[cc];
}

__global__ void wsub_kernel(WhitenSpace a0, WhitenSpace a1, int s, int r, int nsplit) {
  const WhitenSpace& a = blockIdx.y ? a1 : a0;
  const size_t total = (size_t)s * r;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    double t = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) t += a.part[(size_t)sp * total + e];
    a.w[e] -= t;
  }
}

__device__ bool chol_upper_small(const double* G, double* U, int r) {
  for (int i = 0; i < r * r; ++i) U[i] = 0.0;
  for (int j = 0; j < r; ++j) {
    double sd = G[j * r + j];
    for (int k = 0; k < j; ++k) sd -= U[k * r + j] * U[k * r + j];
    if (!(sd > 0.0)) return false;
    const double d = sqrt(sd);
    U[j * r + j] = d;
    for (int i = j + 1; i < r; ++i) {
      double t = G[j * r + i];
      for (int k = 0; k < j; ++k) t -= U[k * r + j] * U[k * r + i];
      U[j * r + i] = t / d;
    }
  }
  return true;
}

__device__ void inv_upper_small(const double* U, double* V, int r) {
  for (int i = 0; i < r * r; ++i) V[i] = 0.0;
  for (int j = 0; j < r; ++j) {
    V[j * r + j] = 1.0 / U[j * r + j];
    for (int i = j - 1; i >= 0; --i) {
      double t = 0.0;
      for (int k = i + 1; k <= j; ++k) t += U[i * r + k] * V[k * r + j];
      V[i * r + j] = -t / U[i * r + i];
    }
  }
}

// Gram matrix of the s x R row-major block w, reduced over the workgroup into G (LDS).
// Small R: every thread accumulates the full R x R outer products of its rows (independent
// loads), then a wavefront + LDS reduction; large R: threads own (a, b) pairs.
template <int R>
__device__ void wg_gram(const double* w, int s, double* G, double* red) {
  constexpr int RR = R * R;
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  if constexpr (R <= 4) {
    double acc[RR];
#pragma unroll
    for (int p = 0; p < RR; ++p) acc[p] = 0.0;
    for (int i = tid; i < s; i += FT) {
      double x[R];
#pragma unroll
      for (int c = 0; c < R; ++c) x[c] = w[(size_t)i * R + c];
#pragma unroll
      for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) acc[a * R + b] += x[a] * x[b];
    }
#pragma unroll
    for (int p = 0; p < RR; ++p) {
      const double v = wave_sum(acc[p]);
      if (lane == 0) red[wv * RR + p] = v;
    }
    __syncthreads();
    if (tid < RR) {
      double t = 0.0;
      for (int q = 0; q < FT / 64; ++q) t += red[q * RR + tid];
      G[tid] = t;
    }
    __syncthreads();
  } else {
    constexpr int PH = FT / RR;
    double acc = 0.0;
    if (tid < PH * RR) {
      const int p = tid % RR, ph = tid / RR, ra = p / R, rb = p % R;
      for (int i = ph; i < s; i += PH) acc += w[(size_t)i * R + ra] * w[(size_t)i * R + rb];
    }
    red[tid] = acc;
    __syncthreads();
    if (tid < RR) {
      double t = 0.0;
      for (int ph = 0; ph < PH; ++ph) t += red[ph * RR + tid];
      G[tid] = t;
    }
    __syncthreads();
  }
}

// One workgroup per space: CholQR2 of the remainder w, then append q to Q and
// [T_H; tau] to T.
template <int R>
__global__ void __launch_bounds__(FT) whiten_finish_kernel(WhitenSpace a0, WhitenSpace a1, int s, int m, int step) {
  const WhitenSpace& a = blockIdx.x ? a1 : a0;
  __shared__ double red[FT];
  __shared__ double G[RMAX * RMAX], R1[RMAX * RMAX], R1i[RMAX * RMAX], R2[RMAX * RMAX], R2i[RMAX * RMAX],
      tau[RMAX * RMAX];
  __shared__ int ok;
  const int tid = threadIdx.x;
  wg_gram<R>(a.w, s, G, red);
  if (tid == 0) {
    ok = chol_upper_small(G, R1, R);
    if (ok) inv_upper_small(R1, R1i, R);
  }
  __syncthreads();
  if (ok) {
    for (int i = tid; i < s; i += FT) {
      double x[R], y[R];
#pragma unroll
      for (int c = 0; c < R; ++c) x[c] = a.w[(size_t)i * R + c];
#pragma unroll
      for (int c = 0; c < R; ++c) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k <= c; ++k) t += x[k] * R1i[k * R + c];
        y[c] = t;
      }
#pragma unroll
      for (int c = 0; c < R; ++c) a.w[(size_t)i * R + c] = y[c];
    }
  }
  __syncthreads();
  if (ok) wg_gram<R>(a.w, s, G, red);
  if (tid == 0) {
    if (ok) ok = chol_upper_small(G, R2, R);
    if (ok) {
      inv_upper_small(R2, R2i, R);
      for (int i = 0; i < R; ++i)
        for (int j = 0; j < R; ++j) {
          double t = 0.0;
          for (int k = 0; k < R; ++k) t += R2[i * R + k] * R1[k * R + j];
          tau[i * R + j] = t;
        }
    } else {
      atomicMin(a.broken, step);
      for (int i = 0; i < R * R; ++i) { tau[i] = (i % (R + 1) == 0) ? 1.0 : 0.0; R2i[i] = 0.0; }
    }
  }
  __syncthreads();
  // q = w R2^{-1} -> Q[:, m : m+R]
  for (int i = tid; i < s; i += FT) {
    double x[R];
#pragma unroll
    for (int c = 0; c < R; ++c) x[c] = a.w[(size_t)i * R + c];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k <= c; ++k) t += x[k] * R2i[k * R + c];
      a.Q[(size_t)(m + c) * s + i] = t;
    }
  }
  // T_H = c1 + c2 above the diagonal block, tau on it
  for (int e = tid; e < m * R; e += FT) {
    const int i = e / R, c = e % R;
    a.T[i + (size_t)(m + c) * a.ldt] = a.c1[e] + a.c2[e];
  }
  if (tid < R * R) {
    const int ra = tid / R, rb = tid % R;
    a.T[(m + ra) + (size_t)(m + rb) * a.ldt] = (ra <= rb) ? tau[ra * R + rb] : 0.0;
  }
}

}  // namespace

int whiten_splits(int m) { return std::max(1, std::min(64, ceil_div(m, SPLIT_COLS))); }
size_t whiten_part_doubles(int s, int r, int maxm) { return (size_t)whiten_splits(maxm) * s * r; }

#define WH_DISPATCH(r, ...)                                                \
  switch (r) {                                                             \
    case 1: { constexpr int RR_ = 1; __VA_ARGS__; } break;                 \
    case 2: { constexpr int RR_ = 2; __VA_ARGS__; } break;                 \
    case 3: { constexpr int RR_ = 3; __VA_ARGS__; } break;                 \
    case 4: { constexpr int RR_ = 4; __VA_ARGS__; } break;                 \
    case 5: { constexpr int RR_ = 5; __VA_ARGS__; } break;                 \
    case 6: { constexpr int RR_ = 6; __VA_ARGS__; } break;                 \
    case 7: { constexpr int RR_ = 7; __VA_ARGS__; } break;                 \
    case 8: { constexpr int RR_ = 8; __VA_ARGS__; } break;                 \
    case 9: { constexpr int RR_ = 9; __VA_ARGS__; } break;                 \
    case 10: { constexpr int RR_ = 10; __VA_ARGS__; } break;               \
    case 11: { constexpr int RR_ = 11; __VA_ARGS__; } break;               \
    case 12: { constexpr int RR_ = 12; __VA_ARGS__; } break;               \
    case 13: { constexpr int RR_ = 13; __VA_ARGS__; } break;               \
    case 14: { constexpr int RR_ = 14; __VA_ARGS__; } break;               \
    case 15: { constexpr int RR_ = 15; __VA_ARGS__; } break;               \
    case 16: { constexpr int RR_ = 16; __VA_ARGS__; } break;               \
    default: throw Error(SKR_ENOTSUP, "block size r must be in [1, 16]");  \
  }

void launch_whiten(int r, int s, int m, int step, const WhitenSpace& a, const WhitenSpace& b, hipStream_t st) {
  if (m > 0) {
    const int nsplit = whiten_splits(m);
    const int cps = ceil_div(m, nsplit);
    for (int pass = 0; pass < 2; ++pass) {
      WH_DISPATCH(r, hipLaunchKernelGGL((qtw_kernel<RR_>), dim3(ceil_div(m, jb_of<RR_>()), 2), dim3(WT), 0, st, a, b, s,
                                        m, pass));
      check_launch("whiten_qtw");
      WH_DISPATCH(r, hipLaunchKernelGGL((qc_part_kernel<RR_>), dim3(ceil_div(s, WT), nsplit, 2), dim3(WT),
                                        sizeof(double) * (size_t)cps * RR_, st, a, b, s, m, pass, cps));
      check_launch("whiten_qc");
      hipLaunchKernelGGL(wsub_kernel, dim3(std::min(1024, ceil_div((int64_t)s * r, 256)), 2), dim3(256), 0, st, a, b,
                         s, r, nsplit);
      check_launch("whiten_sub");
    }
  }
  WH_DISPATCH(r, hipLaunchKernelGGL((whiten_finish_kernel<RR_>), dim3(2), dim3(FT), 0, st, a, b, s, m, step));
  check_launch("whiten_finish");
}

}  // namespace skr
