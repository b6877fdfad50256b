// Sketched QR update (Prop. 2.1), FP64.  Q is column-major (s x columns, ld = s) so that
// appending a block writes contiguous memory and the product Q c reads Q with unit stride
// across the threads of a wavefront.
#include <algorithm>

#include "small_la.hpp"
#include "whiten.hpp"

namespace skr {
namespace {

constexpr int WT = 256;      // threads for the streaming whitening kernels
constexpr int FT = 1024;     // threads of the finishing workgroup

// ---- c = Q^T w, split over row chunks: every wavefront owns 64 / R columns of a tile of
// 4 (64 / R) columns and sums its chunk's rows for all of them; the 64 per-lane values are
// transpose-reduced across the wavefront, and each (chunk, column) partial is written once.
constexpr int QT_ROWS = 1024;  // rows of Q per chunk (fewer partials than 256: 4.9 against 4.2 TB/s)

template <int R>
constexpr int qt_cols() { return 64 / R > 0 ? 64 / R : 1; }

template <int R>
__global__ void __launch_bounds__(WT) qtw_split_kernel(WhitenSpace a0, WhitenSpace a1, int s, int m) {
  constexpr int CW = qt_cols<R>(), NV = CW * R;
  const WhitenSpace& a = blockIdx.z ? a1 : a0;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const int j0 = (blockIdx.x * (WT / 64) + wv) * CW;
  const int r0 = blockIdx.y * QT_ROWS, r1 = min(s, r0 + QT_ROWS);
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  if (j0 < m) {
    for (int i = r0 + lane; i < r1; i += 64) {
      double wr[R];
      load_row<double, R>(a.w, i, wr);
      double q[CW];
#pragma unroll
      for (int jj = 0; jj < CW; ++jj) q[jj] = (j0 + jj < m) ? a.Q[(size_t)(j0 + jj) * s + i] : 0.0;
#pragma unroll
      for (int jj = 0; jj < CW; ++jj)
#pragma unroll
        for (int c = 0; c < R; ++c) acc[jj * R + c] += q[jj] * wr[c];
    }
  }
  int idx;
  const double t = wave_transpose_sum<NV>(acc, idx);
  if (idx >= 0 && j0 + idx / R < m)
    a.part[((size_t)blockIdx.y * m + j0 + idx / R) * R + idx % R] = t;
}

// out = sum over the row chunks of the partials (fixed order)
__global__ void qtw_sum_kernel(WhitenSpace a0, WhitenSpace a1, int m, int r, int nchunk, int which) {
  const WhitenSpace& a = blockIdx.y ? a1 : a0;
  double* out = which ? a.c2 : a.c1;
  const int total = m * r;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    int ch = 0;
    for (; ch + 4 <= nchunk; ch += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) t[u] += a.part[(size_t)(ch + u) * total + e];
    }
    for (; ch < nchunk; ++ch) t[0] += a.part[(size_t)ch * total + e];
    out[e] = (t[0] + t[1]) + (t[2] + t[3]);
  }
}

// ---- w -= Q c in one launch: a workgroup owns 128 rows; its 2 column groups (two
// wavefronts each) take every other column of Q (each load a 1 KiB row segment per group,
// eight columns' loads in flight), and the 2 partial sums are added in order through LDS.
// c is staged through LDS in column chunks.  (32 rows and 8 groups: 4.2 TB/s; this: 4.8.)
constexpr int QC_COLS = 512;
constexpr int QC_ROWS = 128, QC_GROUPS = WT / QC_ROWS, QC_UN = 8;

template <int R>
__global__ void __launch_bounds__(WT) qc_rows_kernel(WhitenSpace a0, WhitenSpace a1, int s, int m, int which) {
  const WhitenSpace& a = blockIdx.y ? a1 : a0;
  const double* c = which ? a.c2 : a.c1;
  __shared__ double cs[QC_COLS * R];
  __shared__ double red[QC_GROUPS][QC_ROWS][R];
  const int lr = threadIdx.x % QC_ROWS, g = threadIdx.x / QC_ROWS;
  const int i = blockIdx.x * QC_ROWS + lr;
  double acc[R];
#pragma unroll
  for (int cc = 0; cc < R; ++cc) acc[cc] = 0.0;
  for (int jc = 0; jc < m; jc += QC_COLS) {
    const int jn = min(QC_COLS, m - jc);
    __syncthreads();
    for (int e = threadIdx.x; e < jn * R; e += WT) cs[e] = c[(size_t)jc * R + e];
    __syncthreads();
    if (i < s) {
      int j = g;
      for (; j + (QC_UN - 1) * QC_GROUPS < jn; j += QC_UN * QC_GROUPS) {
        double q[QC_UN];
#pragma unroll
        for (int u = 0; u < QC_UN; ++u) q[u] = a.Q[(size_t)(jc + j + QC_GROUPS * u) * s + i];
#pragma unroll
        for (int u = 0; u < QC_UN; ++u)
#pragma unroll
          for (int cc = 0; cc < R; ++cc) acc[cc] += q[u] * cs[(j + QC_GROUPS * u) * R + cc];
      }
      for (; j < jn; j += QC_GROUPS) {
        const double q = a.Q[(size_t)(jc + j) * s + i];
#pragma unroll
        for (int cc = 0; cc < R; ++cc) acc[cc] += q * cs[j * R + cc];
      }
    }
  }
#pragma unroll
  for (int cc = 0; cc < R; ++cc) red[g][lr][cc] = acc[cc];
  __syncthreads();
  if (g == 0 && i < s) {
#pragma unroll
    for (int cc = 0; cc < R; ++cc) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < QC_GROUPS; ++q) t += red[q][lr][cc];
      a.w[(size_t)i * R + cc] -= t;
    }
  }
}

// ---- 16-wide sweeps on the matrix cores.  With 16 columns in w (a pair of blocks next to
// the pending pair), the two sweeps are products with an N = 16 operand: Q^T w (m x 16) and
// Q c (s x 16), taken by v_mfma_f64_16x16x4f64 (A(i, k) from lane i + 16 k, B(k, j) from lane
// j + 16 k, D(4 v + g, j) in register v of lane j + 16 g).  They stay bound by the reads of Q;
// the matrix cores replace the 16 multiply-adds per element of Q (and the LDS staging of the
// coefficients and the wavefront transpose reductions) that made the vector kernels latency-
// and occupancy-bound at this width.
typedef double wm_d4 __attribute__((ext_vector_type(4)));
constexpr int QM_UN = 8;  // loads in flight per lane

// c = Q^T w (w with 16 NT columns, row-major) for one chunk of QT_ROWS rows: each wavefront
// owns 16 columns of Q; per pair of MFMA steps lane (i, g) reads rows r + 2 g, r + 2 g + 1 of
// its column (16 bytes) and the same rows of w, one 16-column tile of w per accumulator.
// Partials in the layout of qtw_split_kernel.
template <int NT>
__global__ void __launch_bounds__(WT) qtw_mfma_kernel(WhitenSpace a0, WhitenSpace a1, int s, int m) {
  constexpr int LD = 16 * NT;
  const WhitenSpace& a = blockIdx.z ? a1 : a0;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const int g = lane >> 4, l16 = lane & 15;
  const int j0 = (blockIdx.x * (WT / 64) + wv) * 16;
  if (j0 >= m) return;  // uniform over the wavefront; the kernel has no barrier
  const int r0 = blockIdx.y * QT_ROWS, r1 = min(s, r0 + QT_ROWS);
  const int col = j0 + l16;
  const bool cok = col < m;
  const double* qcol = a.Q + (size_t)(cok ? col : j0) * s;
  wm_d4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = wm_d4{0.0, 0.0, 0.0, 0.0};
  int i = r0;
  // full groups of 8 rows: rows i + 2 g and i + 2 g + 1 for lane group g; s is even, so a
  // 16-byte load at an even row is aligned (Q's columns start at multiples of s doubles)
  for (; i + 8 * QM_UN <= r1; i += 8 * QM_UN) {
    double2 qa[QM_UN];
    double zb0[QM_UN][NT], zb1[QM_UN][NT];
#pragma unroll
    for (int u = 0; u < QM_UN; ++u) {
      const int r = i + 8 * u + 2 * g;
      qa[u] = cok ? *reinterpret_cast<const double2*>(qcol + r) : double2{0.0, 0.0};
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        zb0[u][t] = a.w[(size_t)r * LD + 16 * t + l16];
        zb1[u][t] = a.w[(size_t)(r + 1) * LD + 16 * t + l16];
      }
    }
#pragma unroll
    for (int u = 0; u < QM_UN; ++u)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[u].x, zb0[u][t], acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[u].y, zb1[u][t], acc[t], 0, 0, 0);
      }
  }
  for (; i < r1; i += 4) {  // the rest, 4 rows per step (rows beyond r1 contribute zero)
    const int r = i + g;
    const bool rok = r < r1;
    const double qv = (cok && rok) ? qcol[r] : 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const double zv = rok ? a.w[(size_t)r * LD + 16 * t + l16] : 0.0;
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(qv, zv, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int j = j0 + 4 * v + g;
    if (j < m)
#pragma unroll
      for (int t = 0; t < NT; ++t) a.part[((size_t)blockIdx.y * m + j) * LD + 16 * t + l16] = acc[t][v];
  }
}

// w -= Q c (w and c with 16 NT columns, row-major) for 16 rows per wavefront: lane (i, g)
// reads row i of column j + g of Q and row j + g of c.
template <int NT>
__global__ void __launch_bounds__(WT) qc_mfma_kernel(WhitenSpace a0, WhitenSpace a1, int s, int m, int which) {
  constexpr int LD = 16 * NT;
  const WhitenSpace& a = blockIdx.y ? a1 : a0;
  const double* c = which ? a.c2 : a.c1;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const int g = lane >> 4, l16 = lane & 15;
  const int i0 = (blockIdx.x * (WT / 64) + wv) * 16;
  if (i0 >= s) return;  // uniform over the wavefront; the kernel has no barrier
  const int row = i0 + l16;
  const bool rok = row < s;
  const double* qrow = a.Q + (rok ? row : i0);
  wm_d4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = wm_d4{0.0, 0.0, 0.0, 0.0};
  int j = 0;
  for (; j + 4 * QM_UN <= m; j += 4 * QM_UN) {
    double qa[QM_UN], cb[QM_UN][NT];
#pragma unroll
    for (int u = 0; u < QM_UN; ++u) {
      const int jj = j + 4 * u + g;
      qa[u] = rok ? qrow[(size_t)jj * s] : 0.0;
#pragma unroll
      for (int t = 0; t < NT; ++t) cb[u][t] = c[(size_t)jj * LD + 16 * t + l16];
    }
#pragma unroll
    for (int u = 0; u < QM_UN; ++u)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[u], cb[u][t], acc[t], 0, 0, 0);
  }
  for (; j < m; j += 4) {  // columns beyond m contribute zero
    const int jj = j + g;
    const double qv = (rok && jj < m) ? qrow[(size_t)jj * s] : 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const double cv = (jj < m) ? c[(size_t)jj * LD + 16 * t + l16] : 0.0;
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(qv, cv, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = i0 + 4 * v + g;
    if (r < s)
#pragma unroll
      for (int t = 0; t < NT; ++t) a.w[(size_t)r * LD + 16 * t + l16] -= acc[t][v];
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
__device__ void wg_gram(const double* w, int s, double* G, double* red, int ld = R) {
  constexpr int RR = R * R;
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  if constexpr (R <= 4) {
    double acc[RR];
#pragma unroll
    for (int p = 0; p < RR; ++p) acc[p] = 0.0;
#pragma unroll 4
    for (int i = tid; i < s; i += FT) {  // unrolled: several rows' loads in flight
      double x[R];
#pragma unroll
      for (int c = 0; c < R; ++c) x[c] = w[(size_t)i * ld + c];
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
      for (int i = ph; i < s; i += PH) acc += w[(size_t)i * ld + ra] * w[(size_t)i * ld + rb];
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
#pragma unroll 4
    for (int i = tid; i < s; i += FT) {
      double x[R], y[R];
      load_row<double, R>(a.w, i, x);
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
#pragma unroll 4
  for (int i = tid; i < s; i += FT) {
    double x[R];
    load_row<double, R>(a.w, i, x);
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

// Register-resident finish (R <= 4, s <= FIN_RPT FIN_T): each thread keeps its rows of w in
// registers through both Cholesky QR passes, so w is read once and Q written once.
constexpr int FIN_T = 512, FIN_RPT = 16;

template <int R>
__device__ inline void fin_gram(const double (&x)[FIN_RPT][R], double* G, double* red) {
  constexpr int RR = R * R;
  const int wv = threadIdx.x / 64;
  double acc[RR];
#pragma unroll
  for (int p = 0; p < RR; ++p) acc[p] = 0.0;
#pragma unroll
  for (int q = 0; q < FIN_RPT; ++q)
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int b = 0; b < R; ++b) acc[a * R + b] += x[q][a] * x[q][b];
  int idx;
  const double t = wave_transpose_sum<RR>(acc, idx);
  if (idx >= 0) red[wv * RR + idx] = t;
  __syncthreads();
  if (threadIdx.x < RR) {
    double u = 0.0;
    for (int w = 0; w < FIN_T / 64; ++w) u += red[w * RR + threadIdx.x];
    G[threadIdx.x] = u;
  }
  __syncthreads();
}

template <int R>
__global__ void __launch_bounds__(FIN_T) whiten_finish_reg_kernel(WhitenSpace a0, WhitenSpace a1, int s, int m,
                                                               int step) {
  const WhitenSpace& a = blockIdx.x ? a1 : a0;
  constexpr int RR = R * R;
  __shared__ double red[(FIN_T / 64) * RR];
  __shared__ double G[RR], R1[RR], R1i[RR], R2[RR], R2i[RR], tau[RR];
  __shared__ int ok;
  const int tid = threadIdx.x;
  double x[FIN_RPT][R];
#pragma unroll
  for (int q = 0; q < FIN_RPT; ++q) {
    const int i = tid + q * FIN_T;
    if (i < s) {
      load_row<double, R>(a.w, i, x[q]);
    } else {
#pragma unroll
      for (int c = 0; c < R; ++c) x[q][c] = 0.0;
    }
  }
  fin_gram<R>(x, G, red);
  if (tid == 0) {
    ok = chol_upper_small(G, R1, R);
    if (ok) inv_upper_small(R1, R1i, R);
  }
  __syncthreads();
  if (ok) {
#pragma unroll
    for (int q = 0; q < FIN_RPT; ++q) {
      double y[R];
#pragma unroll
      for (int c = 0; c < R; ++c) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k <= c; ++k) t += x[q][k] * R1i[k * R + c];
        y[c] = t;
      }
#pragma unroll
      for (int c = 0; c < R; ++c) x[q][c] = y[c];
    }
    fin_gram<R>(x, G, red);
  }
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
      for (int i = 0; i < RR; ++i) { tau[i] = (i % (R + 1) == 0) ? 1.0 : 0.0; R2i[i] = 0.0; }
    }
  }
  __syncthreads();
  // q = (w R1^{-1}) R2^{-1} -> Q[:, m : m+R] (zero when the space broke down)
#pragma unroll
  for (int q = 0; q < FIN_RPT; ++q) {
    const int i = tid + q * FIN_T;
    if (i >= s) continue;
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k <= c; ++k) t += x[q][k] * R2i[k * R + c];
      a.Q[(size_t)(m + c) * s + i] = t;
    }
  }
  for (int e = tid; e < m * R; e += FIN_T) {
    const int i = e / R, c = e % R;
    a.T[i + (size_t)(m + c) * a.ldt] = a.c1[e] + a.c2[e];
  }
  if (tid < RR) {
    const int ra = tid / R, rb = tid % R;
    a.T[(m + ra) + (size_t)(m + rb) * a.ldt] = (ra <= rb) ? tau[ra * R + rb] : 0.0;
  }
}

// ---- delayed re-orthogonalisation: small kernels around the 2r-wide sweeps
// mode 0: Z[:, r : 2r] <- w (the new block next to the pending one)
// mode 1: zf <- Z[:, 0 : r] (the pending block, staged contiguously for its last pass)
// mode 2: Z[:, 0 : r] <- w (a first-pass remainder becomes the pending block)
__global__ void dcgs_move_kernel(WhitenSpace a0, WhitenSpace a1, int s, int r, int mode) {
  const WhitenSpace& a = blockIdx.y ? a1 : a0;
  const int total = s * r;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int i = e / r, c = e % r;
    double* z = a.Z + (size_t)i * 2 * r;
    if (mode == 0) z[r + c] = a.w[e];
    else if (mode == 1) a.zf[e] = z[c];
    else z[c] = a.w[e];
  }
}

// Finishing the pending block over many workgroups per space.  Z holds [P'' | w'] (s x 2R,
// row-major): the pending block after both passes against the m columns of Q, and the new
// block after its first pass; cz the products [a | b] of that sweep (m x 2R); cstash the
// pending block's first-pass coefficients (m x R).  Four launches, each a sweep over the
// s rows by FIN_G workgroups; every small factor is computed by each workgroup from the
// previous launch's partial sums, added in workgroup order (the same on every workgroup):
//   1. partials of G1 = P''^T P''
//   2. R1 = chol(G1); P1 = P'' R1^{-1} in place; partials of G2 = P1^T P1
//   3. R2 = chol(G2); q = P1 R2^{-1} -> columns m .. m + R - 1 of Q and Z[:, 0 : R];
//      tau = R2 R1 -> the diagonal block of T; partials of E = q^T w'
//   4. Z[:, 0 : R] <- w' - q E (the next pending block); T(0 : m, m : m + R) = cstash + a,
//      cstash <- [b; E] (its first-pass coefficients against the grown Q)
// A failed Cholesky factorisation marks the space broken at `step` and appends zero columns
// with tau = I (the finish of the non-delayed update does the same).
constexpr int FIN_G = 64;          // workgroups per space (at most)
constexpr int FIN_ROWS_MIN = 512;  // rows per workgroup (at least)
constexpr int FIN_RR = 256;        // R^2 for R <= 16

struct FinRows {
  int g, ng, r0, r1;
};
__device__ inline FinRows fin_rows(int s) {
  FinRows f;
  f.g = blockIdx.x;
  f.ng = gridDim.x;
  const int per = (s + f.ng - 1) / f.ng;
  f.r0 = min(s, f.g * per);
  f.r1 = min(s, f.r0 + per);
  return f;
}
inline int fin_groups(int s) { return std::max(1, std::min(FIN_G, ceil_div(s, FIN_ROWS_MIN))); }

// Sum of the workgroup's per-thread R x R values into part[g * RR + p] (fixed order).
template <int RR>
__device__ inline void fin_write_partials(const double (&acc)[RR], double* part, int g, double* red) {
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
#pragma unroll
  for (int p = 0; p < RR; ++p) {
    const double v = wave_sum(acc[p]);
    if (lane == 0) red[wv * RR + p] = v;
  }
  __syncthreads();
  if (threadIdx.x < RR) {
    double t = 0.0;
    for (int w = 0; w < WT / 64; ++w) t += red[w * RR + threadIdx.x];
    part[(size_t)g * FIN_RR + threadIdx.x] = t;
  }
}

// out[p] = sum over the ng workgroups' partials (fixed order), in LDS
template <int RR>
__device__ inline void fin_sum_partials(const double* part, int ng, double* out) {
  if (threadIdx.x < RR) {
    double t = 0.0;
    for (int g = 0; g < ng; ++g) t += part[(size_t)g * FIN_RR + threadIdx.x];
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

template <int R>
__global__ void __launch_bounds__(WT) fin1_kernel(WhitenSpace a0, WhitenSpace a1, int s) {
  const WhitenSpace& a = blockIdx.y ? a1 : a0;
  constexpr int RR = R * R, L = 2 * R;
  __shared__ double red[(WT / 64) * RR];
  const FinRows f = fin_rows(s);
  double acc[RR];
#pragma unroll
  for (int p = 0; p < RR; ++p) acc[p] = 0.0;
  for (int i = f.r0 + threadIdx.x; i < f.r1; i += WT) {
    const double* z = a.Z + (size_t)i * L;
    double x[R];
#pragma unroll
    for (int c = 0; c < R; ++c) x[c] = z[c];
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
      for (int v = 0; v < R; ++v) acc[u * R + v] += x[u] * x[v];
  }
  fin_write_partials<RR>(acc, a.fpart, f.g, red);
}

template <int R>
__global__ void __launch_bounds__(WT) fin2_kernel(WhitenSpace a0, WhitenSpace a1, int s, int step) {
  const WhitenSpace& a = blockIdx.y ? a1 : a0;
  constexpr int RR = R * R, L = 2 * R;
  __shared__ double red[(WT / 64) * RR];
  __shared__ double G[RR], R1[RR], R1i[RR];
  __shared__ int ok;
  const FinRows f = fin_rows(s);
  fin_sum_partials<RR>(a.fpart, f.ng, G);
  if (threadIdx.x == 0) {
    ok = chol_upper_small(G, R1, R);
    if (ok) inv_upper_small(R1, R1i, R);
    if (f.g == 0) {  // the outcome and R1 for the next launches
      a.fstate[0] = ok ? 1.0 : 0.0;
      for (int p = 0; p < RR; ++p) a.fstate[8 + p] = ok ? R1[p] : 0.0;
      if (!ok) atomicMin(a.broken, step);
    }
  }
  __syncthreads();
  double acc[RR];
#pragma unroll
  for (int p = 0; p < RR; ++p) acc[p] = 0.0;
  if (ok) {
    for (int i = f.r0 + threadIdx.x; i < f.r1; i += WT) {
      double* z = a.Z + (size_t)i * L;
      double y[R];
#pragma unroll
      for (int c = 0; c < R; ++c) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k <= c; ++k) t += z[k] * R1i[k * R + c];
        y[c] = t;
      }
#pragma unroll
      for (int c = 0; c < R; ++c) z[c] = y[c];
#pragma unroll
      for (int u = 0; u < R; ++u)
#pragma unroll
        for (int v = 0; v < R; ++v) acc[u * R + v] += y[u] * y[v];
    }
  }
  fin_write_partials<RR>(acc, a.fpart + (size_t)FIN_G * FIN_RR, f.g, red);
}

template <int R>
__global__ void __launch_bounds__(WT) fin3_kernel(WhitenSpace a0, WhitenSpace a1, int s, int m, int step) {
  const WhitenSpace& a = blockIdx.y ? a1 : a0;
  constexpr int RR = R * R, L = 2 * R;
  __shared__ double red[(WT / 64) * RR];
  __shared__ double G[RR], R2[RR], R2i[RR];
  __shared__ int ok;
  const FinRows f = fin_rows(s);
  fin_sum_partials<RR>(a.fpart + (size_t)FIN_G * FIN_RR, f.ng, G);
  if (threadIdx.x == 0) {
    ok = a.fstate[0] != 0.0;
    if (ok) ok = chol_upper_small(G, R2, R);
    if (ok) inv_upper_small(R2, R2i, R);
    else
      for (int p = 0; p < RR; ++p) R2i[p] = 0.0;
    if (f.g == 0) {
      if (!ok && a.fstate[0] != 0.0) atomicMin(a.broken, step);
      a.fstate[1] = ok ? 1.0 : 0.0;
      for (int u = 0; u < R; ++u)  // tau = R2 R1 on the diagonal block of T (I after a failure)
        for (int v = 0; v < R; ++v) {
          double t = 0.0;
          if (ok)
            for (int k = 0; k < R; ++k) t += R2[u * R + k] * a.fstate[8 + k * R + v];
          else
            t = (u == v) ? 1.0 : 0.0;
          a.T[(m + u) + (size_t)(m + v) * a.ldt] = (u <= v) ? t : 0.0;
        }
    }
  }
  __syncthreads();
  double acc[RR];
#pragma unroll
  for (int p = 0; p < RR; ++p) acc[p] = 0.0;
  for (int i = f.r0 + threadIdx.x; i < f.r1; i += WT) {
    double* z = a.Z + (size_t)i * L;
    double q[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k <= c; ++k) t += z[k] * R2i[k * R + c];
      q[c] = t;
      a.Q[(size_t)(m + c) * s + i] = t;
    }
#pragma unroll
    for (int c = 0; c < R; ++c) z[c] = q[c];
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
      for (int v = 0; v < R; ++v) acc[u * R + v] += q[u] * z[R + v];
  }
  fin_write_partials<RR>(acc, a.fpart + (size_t)2 * FIN_G * FIN_RR, f.g, red);
}

template <int R>
__global__ void __launch_bounds__(WT) fin4_kernel(WhitenSpace a0, WhitenSpace a1, int s, int m) {
  const WhitenSpace& a = blockIdx.y ? a1 : a0;
  constexpr int RR = R * R, L = 2 * R;
  __shared__ double E[RR];
  const FinRows f = fin_rows(s);
  fin_sum_partials<RR>(a.fpart + (size_t)2 * FIN_G * FIN_RR, f.ng, E);
  for (int i = f.r0 + threadIdx.x; i < f.r1; i += WT) {
    double* z = a.Z + (size_t)i * L;
    double v[R];
#pragma unroll
    for (int y = 0; y < R; ++y) {
      double t = z[R + y];
#pragma unroll
      for (int x = 0; x < R; ++x) t -= z[x] * E[x * R + y];
      v[y] = t;
    }
#pragma unroll
    for (int y = 0; y < R; ++y) z[y] = v[y];
  }
  // T column block of the finished block and the pending block's coefficients [b; E],
  // the m R entries split over the workgroups
  const int tot = m * R, per = (tot + f.ng - 1) / f.ng, e0 = f.g * per, e1 = min(tot, e0 + per);
  for (int e = e0 + threadIdx.x; e < e1; e += WT) {
    const int j = e / R, c = e % R;
    const double* czj = a.cz + (size_t)j * L;
    a.T[j + (size_t)(m + c) * a.ldt] = a.cstash[e] + czj[c];
    a.cstash[e] = czj[R + c];
  }
  if (f.g == 0 && threadIdx.x < RR) a.cstash[(size_t)m * R + threadIdx.x] = E[threadIdx.x];
}

// ---- finishing a 16-wide pending block (a group of blocks of 16 columns in all).  The same
// four launches as fin1_kernel .. fin4_kernel; the 16 x 16 products over the rows (the Gram
// matrices and E) are taken on the matrix cores: lane (a, g) of a wavefront supplies element
// (row, a) of the left factor and element (row, b = a) of the right one for rows r + g, and
// the four wavefronts' tiles are added in order through LDS.  The per-row triangular
// products that feed them are formed by each lane for its own element.
constexpr int W16 = 16, L32 = 32, RR16 = 256;

// the workgroup's 16 x 16 tile sums acc (register v of lane a + 16 g holds entry (4 v + g, a))
// into part[g * FIN_RR + p] (p = row * 16 + column), in a fixed order
__device__ inline void fin16_write_tile(const wm_d4& acc, double* part, int g, double* red) {
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64, lg = lane >> 4, l16 = lane & 15;
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wv * RR16 + (4 * v + lg) * W16 + l16] = acc[v];
  __syncthreads();
  if (threadIdx.x < RR16) {
    double t = 0.0;
    for (int w = 0; w < WT / 64; ++w) t += red[w * RR16 + threadIdx.x];
    part[(size_t)g * FIN_RR + threadIdx.x] = t;
  }
}

__global__ void __launch_bounds__(WT) fin1_w16_kernel(WhitenSpace a0, WhitenSpace a1, int s) {
  const WhitenSpace& a = blockIdx.y ? a1 : a0;
  __shared__ double red[(WT / 64) * RR16];
  const FinRows f = fin_rows(s);
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64, lg = lane >> 4, l16 = lane & 15;
  wm_d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int base = f.r0 + 4 * wv; base < f.r1; base += 4 * (WT / 64)) {  // uniform per wavefront
    const int row = base + lg;
    const double x = row < f.r1 ? a.Z[(size_t)row * L32 + l16] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, acc, 0, 0, 0);
  }
  fin16_write_tile(acc, a.fpart, f.g, red);
}

// y(row, a) = sum_{k <= a} z(row, k) Ri(k, a) for the upper triangular Ri (16 x 16, LDS)
__device__ inline double fin16_tri(const double* z, const double* Ri, int a) {
  double t = 0.0;
  for (int k = 0; k <= a; ++k) t += z[k] * Ri[k * W16 + a];
  return t;
}

__global__ void __launch_bounds__(WT) fin2_w16_kernel(WhitenSpace a0, WhitenSpace a1, int s, int step) {
  const WhitenSpace& a = blockIdx.y ? a1 : a0;
  __shared__ double red[(WT / 64) * RR16];
  __shared__ double G[RR16], R1[RR16], R1i[RR16];
  __shared__ int ok;
  const FinRows f = fin_rows(s);
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64, lg = lane >> 4, l16 = lane & 15;
  fin_sum_partials<RR16>(a.fpart, f.ng, G);
  if (threadIdx.x == 0) {
    ok = chol_upper_small(G, R1, W16);
    if (ok) inv_upper_small(R1, R1i, W16);
    if (f.g == 0) {  // the outcome and R1 for the next launches
      a.fstate[0] = ok ? 1.0 : 0.0;
      for (int p = 0; p < RR16; ++p) a.fstate[8 + p] = ok ? R1[p] : 0.0;
      if (!ok) atomicMin(a.broken, step);
    }
  }
  __syncthreads();
  wm_d4 acc = {0.0, 0.0, 0.0, 0.0};
  if (ok) {
    // the Gram matrix of P1 = P'' R1^{-1} from the rows as they are, then P1 written back
    for (int base = f.r0 + 4 * wv; base < f.r1; base += 4 * (WT / 64)) {
      const int row = base + lg;
      const double y = row < f.r1 ? fin16_tri(a.Z + (size_t)row * L32, R1i, l16) : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(y, y, acc, 0, 0, 0);
    }
    __syncthreads();  // every read of this workgroup's rows precedes the writes below
    for (int i = f.r0 + threadIdx.x; i < f.r1; i += WT) {
      double* z = a.Z + (size_t)i * L32;
      double y[W16];
#pragma unroll
      for (int c = 0; c < W16; ++c) y[c] = fin16_tri(z, R1i, c);
#pragma unroll
      for (int c = 0; c < W16; ++c) z[c] = y[c];
    }
  }
  fin16_write_tile(acc, a.fpart + (size_t)FIN_G * FIN_RR, f.g, red);
}

__global__ void __launch_bounds__(WT) fin3_w16_kernel(WhitenSpace a0, WhitenSpace a1, int s, int m, int step) {
  const WhitenSpace& a = blockIdx.y ? a1 : a0;
  __shared__ double red[(WT / 64) * RR16];
  __shared__ double G[RR16], R2[RR16], R2i[RR16];
  __shared__ int ok;
  const FinRows f = fin_rows(s);
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64, lg = lane >> 4, l16 = lane & 15;
  fin_sum_partials<RR16>(a.fpart + (size_t)FIN_G * FIN_RR, f.ng, G);
  if (threadIdx.x == 0) {
    ok = a.fstate[0] != 0.0;
    if (ok) ok = chol_upper_small(G, R2, W16);
    if (ok) inv_upper_small(R2, R2i, W16);
    else
      for (int p = 0; p < RR16; ++p) R2i[p] = 0.0;
    if (f.g == 0) {
      if (!ok && a.fstate[0] != 0.0) atomicMin(a.broken, step);
      a.fstate[1] = ok ? 1.0 : 0.0;
      for (int u = 0; u < W16; ++u)  // tau = R2 R1 on the diagonal block of T (I after a failure)
        for (int v = 0; v < W16; ++v) {
          double t = 0.0;
          if (ok)
            for (int k = 0; k < W16; ++k) t += R2[u * W16 + k] * a.fstate[8 + k * W16 + v];
          else
            t = (u == v) ? 1.0 : 0.0;
          a.T[(m + u) + (size_t)(m + v) * a.ldt] = (u <= v) ? t : 0.0;
        }
    }
  }
  __syncthreads();
  // E = q^T w' with q = P1 R2^{-1} from the rows as they are, then q written to Q and Z
  wm_d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int base = f.r0 + 4 * wv; base < f.r1; base += 4 * (WT / 64)) {
    const int row = base + lg;
    const bool rok = row < f.r1;
    const double* z = a.Z + (size_t)(rok ? row : f.r0) * L32;
    const double q = rok ? fin16_tri(z, R2i, l16) : 0.0;
    const double w = rok ? z[W16 + l16] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(q, w, acc, 0, 0, 0);
  }
  __syncthreads();  // every read of this workgroup's rows precedes the writes below
  for (int i = f.r0 + threadIdx.x; i < f.r1; i += WT) {
    double* z = a.Z + (size_t)i * L32;
    double q[W16];
#pragma unroll
    for (int c = 0; c < W16; ++c) q[c] = fin16_tri(z, R2i, c);
#pragma unroll
    for (int c = 0; c < W16; ++c) {
      a.Q[(size_t)(m + c) * s + i] = q[c];
      z[c] = q[c];
    }
  }
  fin16_write_tile(acc, a.fpart + (size_t)2 * FIN_G * FIN_RR, f.g, red);
}

__global__ void __launch_bounds__(WT) fin4_w16_kernel(WhitenSpace a0, WhitenSpace a1, int s, int m) {
  const WhitenSpace& a = blockIdx.y ? a1 : a0;
  __shared__ double E[RR16];
  const FinRows f = fin_rows(s);
  fin_sum_partials<RR16>(a.fpart + (size_t)2 * FIN_G * FIN_RR, f.ng, E);
  for (int i = f.r0 + threadIdx.x; i < f.r1; i += WT) {
    double* z = a.Z + (size_t)i * L32;
    double q[W16], v[W16];
#pragma unroll
    for (int x = 0; x < W16; ++x) {
      q[x] = z[x];
      v[x] = z[W16 + x];
    }
#pragma unroll 1
    for (int x = 0; x < W16; ++x) {  // v -= q(x) E(x, :), one row of E at a time
      const double qx = q[x];
#pragma unroll
      for (int y = 0; y < W16; ++y) v[y] -= qx * E[x * W16 + y];
    }
#pragma unroll
    for (int y = 0; y < W16; ++y) z[y] = v[y];
  }
  // T column block of the finished block and the pending block's coefficients [b; E],
  // the 16 m entries split over the workgroups
  const int tot = m * W16, per = (tot + f.ng - 1) / f.ng, e0 = f.g * per, e1 = min(tot, e0 + per);
  for (int e = e0 + threadIdx.x; e < e1; e += WT) {
    const int j = e / W16, c = e % W16;
    const double* czj = a.cz + (size_t)j * L32;
    a.T[j + (size_t)(m + c) * a.ldt] = a.cstash[e] + czj[c];
    a.cstash[e] = czj[W16 + c];
  }
  if (f.g == 0 && threadIdx.x < RR16) a.cstash[(size_t)m * W16 + threadIdx.x] = E[threadIdx.x];
}

// T(0 : m, m : m + R) = c1 + c2 (the first- and second-pass coefficients of a flushed block)
__global__ void tcol_kernel(WhitenSpace a0, WhitenSpace a1, int m, int R) {
  const WhitenSpace& a = blockIdx.y ? a1 : a0;
  const int total = m * R;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x)
    a.T[(e / R) + (size_t)(m + e % R) * a.ldt] = a.c1[e] + a.c2[e];
}

}  // namespace

size_t whiten_fin_doubles() { return (size_t)3 * FIN_G * FIN_RR; }
size_t whiten_fin_state_doubles() { return 8 + FIN_RR; }

// partials of Q^T w: one m x r slab per chunk of QT_ROWS rows
size_t whiten_part_doubles(int s, int r, int maxm) { return (size_t)ceil_div(s, QT_ROWS) * maxm * r; }

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

void launch_whiten(int r, int s, int m, int step, const WhitenSpace& a, const WhitenSpace& b, hipStream_t st,
                   int nspaces) {
  const int ns = nspaces == 1 ? 1 : 2;  // grid extent over the spaces: b is skipped when 1
  if (m > 0) {
    const int nchunk = ceil_div(s, QT_ROWS);
    for (int pass = 0; pass < 2; ++pass) {
      WH_DISPATCH(r, {
        const int tile = (WT / 64) * qt_cols<RR_>();
        hipLaunchKernelGGL((qtw_split_kernel<RR_>), dim3(ceil_div(m, tile), nchunk, ns), dim3(WT), 0, st, a, b, s, m);
      });
      check_launch("whiten_qtw");
      hipLaunchKernelGGL(qtw_sum_kernel, dim3(std::min(1024, ceil_div((int64_t)m * r, 256)), ns), dim3(256), 0, st, a,
                         b, m, r, nchunk, pass);
      check_launch("whiten_qtw_sum");
      WH_DISPATCH(r, hipLaunchKernelGGL((qc_rows_kernel<RR_>), dim3(ceil_div(s, QC_ROWS), ns), dim3(WT), 0, st, a, b, s,
                                        m, pass));
      check_launch("whiten_qc");
    }
  }
  if (r <= 4 && s <= FIN_RPT * FIN_T) {
    switch (r) {
      case 1: hipLaunchKernelGGL((whiten_finish_reg_kernel<1>), dim3(ns), dim3(FIN_T), 0, st, a, b, s, m, step); break;
      case 2: hipLaunchKernelGGL((whiten_finish_reg_kernel<2>), dim3(ns), dim3(FIN_T), 0, st, a, b, s, m, step); break;
      case 3: hipLaunchKernelGGL((whiten_finish_reg_kernel<3>), dim3(ns), dim3(FIN_T), 0, st, a, b, s, m, step); break;
      default: hipLaunchKernelGGL((whiten_finish_reg_kernel<4>), dim3(ns), dim3(FIN_T), 0, st, a, b, s, m, step); break;
    }
  } else {
    WH_DISPATCH(r, hipLaunchKernelGGL((whiten_finish_kernel<RR_>), dim3(ns), dim3(FT), 0, st, a, b, s, m, step));
  }
  check_launch("whiten_finish");
}

namespace {

// One sweep pair over the m columns of Q for the R-wide row-major block a.w: the products
// Q^T w summed into c1 (pass 0) or c2 (pass 1), then w -= Q c.
template <int R>
void sweep_pair(int s, int m, int pass, const WhitenSpace& a, const WhitenSpace& b, int ns, hipStream_t st) {
  const int nchunk = ceil_div(s, QT_ROWS);
  // R = 16, 32: the matrix-core sweeps (they read Q in 16-byte pairs of rows: an even s keeps
  // them aligned; 32-wide blocks are only formed for even s); other widths: the vector sweeps
  bool mfma = false;
  if constexpr (R == 16 || R == 32) {
    constexpr int NT = R / 16;
    mfma = s % 2 == 0;
    SKR_REQUIRE(mfma || R == 16, "32-wide sweeps need an even number of sketch rows");
    if (mfma)
      hipLaunchKernelGGL((qtw_mfma_kernel<NT>), dim3(ceil_div(m, (WT / 64) * 16), nchunk, ns), dim3(WT), 0, st, a, b,
                         s, m);
  }
  if constexpr (R <= 16) {
    if (!mfma) {
      const int tile = (WT / 64) * qt_cols<R>();
      hipLaunchKernelGGL((qtw_split_kernel<R>), dim3(ceil_div(m, tile), nchunk, ns), dim3(WT), 0, st, a, b, s, m);
    }
  }
  check_launch("whiten_qtw");
  hipLaunchKernelGGL(qtw_sum_kernel, dim3(std::min(1024, ceil_div((int64_t)m * R, 256)), ns), dim3(256), 0, st, a, b,
                     m, R, nchunk, pass);
  check_launch("whiten_qtw_sum");
  if constexpr (R == 16 || R == 32) {
    if (mfma)
      hipLaunchKernelGGL((qc_mfma_kernel<R / 16>), dim3(ceil_div(s, (WT / 64) * 16), ns), dim3(WT), 0, st, a, b, s, m,
                         pass);
  }
  if constexpr (R <= 16) {
    if (!mfma) hipLaunchKernelGGL((qc_rows_kernel<R>), dim3(ceil_div(s, QC_ROWS), ns), dim3(WT), 0, st, a, b, s, m, pass);
  }
  check_launch("whiten_qc");
}

void finish_block(int r, int s, int m, int step, const WhitenSpace& a, const WhitenSpace& b, int ns, hipStream_t st) {
  if (r <= 4 && s <= FIN_RPT * FIN_T) {
    switch (r) {
      case 1: hipLaunchKernelGGL((whiten_finish_reg_kernel<1>), dim3(ns), dim3(FIN_T), 0, st, a, b, s, m, step); break;
      case 2: hipLaunchKernelGGL((whiten_finish_reg_kernel<2>), dim3(ns), dim3(FIN_T), 0, st, a, b, s, m, step); break;
      case 3: hipLaunchKernelGGL((whiten_finish_reg_kernel<3>), dim3(ns), dim3(FIN_T), 0, st, a, b, s, m, step); break;
      default: hipLaunchKernelGGL((whiten_finish_reg_kernel<4>), dim3(ns), dim3(FIN_T), 0, st, a, b, s, m, step); break;
    }
  } else {
    WH_DISPATCH(r, hipLaunchKernelGGL((whiten_finish_kernel<RR_>), dim3(ns), dim3(FT), 0, st, a, b, s, m, step));
  }
  check_launch("whiten_finish");
}

}  // namespace

void launch_whiten_delayed(int r, int s, int m, int step, int mode, const WhitenSpace& a, const WhitenSpace& b,
                           hipStream_t st, int nspaces) {
  SKR_REQUIRE(whiten_delayed_supported(r) || (r == W16 && s % 2 == 0),
              "delayed re-orthogonalisation needs r <= 8, or 16 with an even s");
  SKR_REQUIRE(m >= 1, "delayed re-orthogonalisation needs a finished first block");
  const int ns = nspaces == 1 ? 1 : 2;
  const int mv = std::max(1, std::min(2048, ceil_div((int64_t)s * r, 256)));
  if (mode == WHITEN_FIRST) {
    // w <- w - Q cstash with cstash = Q^T w, then the remainder becomes the pending block
    WhitenSpace a2 = a, b2 = b;
    a2.c1 = a.cstash;
    b2.c1 = b.cstash;
    WH_DISPATCH(r, sweep_pair<RR_>(s, m, 0, a2, b2, ns, st));
    hipLaunchKernelGGL(dcgs_move_kernel, dim3(mv, ns), dim3(256), 0, st, a, b, s, r, 2);
    check_launch("dcgs_move");
  } else if (mode == WHITEN_APPEND) {
    hipLaunchKernelGGL(dcgs_move_kernel, dim3(mv, ns), dim3(256), 0, st, a, b, s, r, 0);
    check_launch("dcgs_move");
    WhitenSpace a2 = a, b2 = b;  // the 2r-wide sweeps over [pending | new]
    a2.w = a.Z;
    b2.w = b.Z;
    a2.c1 = a.cz;
    b2.c1 = b.cz;
    switch (r) {
      case 1: sweep_pair<2>(s, m, 0, a2, b2, ns, st); break;
      case 2: sweep_pair<4>(s, m, 0, a2, b2, ns, st); break;
      case 3: sweep_pair<6>(s, m, 0, a2, b2, ns, st); break;
      case 4: sweep_pair<8>(s, m, 0, a2, b2, ns, st); break;
      case 5: sweep_pair<10>(s, m, 0, a2, b2, ns, st); break;
      case 6: sweep_pair<12>(s, m, 0, a2, b2, ns, st); break;
      case 7: sweep_pair<14>(s, m, 0, a2, b2, ns, st); break;
      case 8: sweep_pair<16>(s, m, 0, a2, b2, ns, st); break;
      default: sweep_pair<32>(s, m, 0, a2, b2, ns, st); break;
    }
    const dim3 fg(fin_groups(s), ns);
    if (r == W16) {
      hipLaunchKernelGGL(fin1_w16_kernel, fg, dim3(WT), 0, st, a, b, s);
      hipLaunchKernelGGL(fin2_w16_kernel, fg, dim3(WT), 0, st, a, b, s, step);
      hipLaunchKernelGGL(fin3_w16_kernel, fg, dim3(WT), 0, st, a, b, s, m, step);
      hipLaunchKernelGGL(fin4_w16_kernel, fg, dim3(WT), 0, st, a, b, s, m);
    } else {
      WH_DISPATCH(r, {
        hipLaunchKernelGGL((fin1_kernel<RR_>), fg, dim3(WT), 0, st, a, b, s);
        hipLaunchKernelGGL((fin2_kernel<RR_>), fg, dim3(WT), 0, st, a, b, s, step);
        hipLaunchKernelGGL((fin3_kernel<RR_>), fg, dim3(WT), 0, st, a, b, s, m, step);
        hipLaunchKernelGGL((fin4_kernel<RR_>), fg, dim3(WT), 0, st, a, b, s, m);
      });
    }
    check_launch("whiten_finish_delayed");
  } else {
    SKR_REQUIRE(mode == WHITEN_FLUSH, "unknown whitening mode");
    // the pending block, staged contiguously: its second pass, then the usual finish with
    // T = cstash (first pass) + the second pass's coefficients
    hipLaunchKernelGGL(dcgs_move_kernel, dim3(mv, ns), dim3(256), 0, st, a, b, s, r, 1);
    check_launch("dcgs_move");
    WhitenSpace a2 = a, b2 = b;
    a2.w = a.zf;
    b2.w = b.zf;
    a2.c1 = a.cstash;
    b2.c1 = b.cstash;
    a2.c2 = a.cz;
    b2.c2 = b.cz;
    WH_DISPATCH(r, sweep_pair<RR_>(s, m, 1, a2, b2, ns, st));
    if (r == W16) {  // the multi-workgroup finish of a 16-wide block, back in Z[:, 0 : 16]
      hipLaunchKernelGGL(dcgs_move_kernel, dim3(mv, ns), dim3(256), 0, st, a2, b2, s, r, 2);
      const dim3 fg(fin_groups(s), ns);
      hipLaunchKernelGGL(fin1_w16_kernel, fg, dim3(WT), 0, st, a, b, s);
      hipLaunchKernelGGL(fin2_w16_kernel, fg, dim3(WT), 0, st, a, b, s, step);
      hipLaunchKernelGGL(fin3_w16_kernel, fg, dim3(WT), 0, st, a, b, s, m, step);
      hipLaunchKernelGGL(tcol_kernel, dim3(std::max(1, std::min(1024, ceil_div((int64_t)m * r, 256))), ns), dim3(256),
                         0, st, a2, b2, m, r);
      check_launch("whiten_flush_w16");
    } else {
      finish_block(r, s, m, step, a2, b2, ns, st);
    }
  }
}

}  // namespace skr
