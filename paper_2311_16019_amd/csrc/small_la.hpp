// Small dense FP64 helpers shared by the block-step kernels (single-thread r x r
// operations, r <= 16, row-major) and the XCD-aware workgroup numbering.
#pragma once

#include "common.hpp"

namespace skr {

// Logical workgroup id such that each XCD (workgroups are dealt round-robin over the 8
// XCDs by hardware id) owns a contiguous range of logical ids, hence contiguous rows.
__device__ inline int xcd_logical(int g, int G) {
  if (G % 8 != 0) return g;
  return (g % 8) * (G / 8) + g / 8;
}

// ------------------------------------------------------------------ small FP64 helpers
// Upper Cholesky factor of a symmetric r x r matrix G (row-major): U^T U = G.
__device__ inline bool chol_upper(const double* G, double* U, int r) {
  for (int i = 0; i < r * r; ++i) U[i] = 0.0;
  for (int j = 0; j < r; ++j) {
    double s = G[j * r + j];
    for (int k = 0; k < j; ++k) s -= U[k * r + j] * U[k * r + j];
    if (!(s > 0.0)) return false;
    double d = sqrt(s);
    U[j * r + j] = d;
    for (int i = j + 1; i < r; ++i) {
      double t = G[j * r + i];
      for (int k = 0; k < j; ++k) t -= U[k * r + j] * U[k * r + i];
      U[j * r + i] = t / d;
    }
  }
  return true;
}

// Inverse of an upper triangular r x r matrix (row-major).
__device__ inline void inv_upper(const double* U, double* V, int r) {
  for (int i = 0; i < r * r; ++i) V[i] = 0.0;
  for (int j = 0; j < r; ++j) {
    V[j * r + j] = 1.0 / U[j * r + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= j; ++k) s += U[i * r + k] * V[k * r + j];
      V[i * r + j] = -s / U[i * r + i];
    }
  }
}

__device__ inline void matmul_small(const double* A, const double* B, double* C, int r) {
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      double s = 0.0;
      for (int k = 0; k < r; ++k) s += A[i * r + k] * B[k * r + j];
      C[i * r + j] = s;
    }
}

__device__ inline void set_identity(double* A, int r) {
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) A[i * r + j] = (i == j) ? 1.0 : 0.0;
}

constexpr int next_pow2(int v) { return v <= 1 ? 1 : 2 * next_pow2((v + 1) / 2); }

__device__ inline double swap_sum32(double lo, double hi) {  // lanes < 32 keep lo, others hi
  const unsigned long long a = (unsigned long long)__double_as_longlong(lo);
  const unsigned long long b = (unsigned long long)__double_as_longlong(hi);
  const auto l = __builtin_amdgcn_permlane32_swap((unsigned)a, (unsigned)b, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap((unsigned)(a >> 32), (unsigned)(b >> 32), false, false);
  const double x = __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | l[0]));
  const double y = __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | l[1]));
  return x + y;
}
__device__ inline double swap_sum16(double lo, double hi) {  // lanes with bit 4 clear keep lo
  const unsigned long long a = (unsigned long long)__double_as_longlong(lo);
  const unsigned long long b = (unsigned long long)__double_as_longlong(hi);
  const auto l = __builtin_amdgcn_permlane16_swap((unsigned)a, (unsigned)b, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap((unsigned)(a >> 32), (unsigned)(b >> 32), false, false);
  const double x = __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | l[0]));
  const double y = __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | l[1]));
  return x + y;
}
template <int CTRL>
__device__ inline double dpp_keep_sum(double lo, double hi, bool upper) {
  const double send = upper ? lo : hi;
  return (upper ? hi : lo) + dpp_move<CTRL>(send);
}


// Sums over the 64 lanes of a wavefront of NV <= 64 per-lane values at once, by a transpose
// reduction: six exchange stages (lanes paired across 32 and 16 by the gfx950 permlane swaps,
// then mirrored 16-lane rows, mirrored 8-lane halves and quad swaps by DPP), each halving the
// number of values a lane carries; about 2 NV exchanges instead of NV full wavefront sums.
// Returns the total of value idx for the lane that holds it (one lane per value), idx = -1
// for the other lanes.  All 64 lanes must be active.
template <int NV>
__device__ inline double wave_transpose_sum(const double (&acc)[NV], int& idx) {
  constexpr int NP = next_pow2(NV);
  static_assert(NP <= 64, "at most 64 values");
  const int lane = threadIdx.x % 64;
  double v[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) v[i] = (i < NV) ? acc[i] : 0.0;
  if (NP >= 2) {
#pragma unroll
    for (int j = 0; j < NP / 2; ++j) v[j] = swap_sum32(v[j], v[j + NP / 2]);
  } else {
    v[0] = swap_sum32(v[0], v[0]);
  }
  if (NP >= 4) {
#pragma unroll
    for (int j = 0; j < NP / 4; ++j) v[j] = swap_sum16(v[j], v[j + NP / 4]);
  } else {
    v[0] = swap_sum16(v[0], v[0]);
  }
  if (NP >= 8) {
#pragma unroll
    for (int j = 0; j < NP / 8; ++j) v[j] = dpp_keep_sum<0x140>(v[j], v[j + NP / 8], (lane & 8) != 0);
  } else {
    v[0] += dpp_move<0x140>(v[0]);
  }
  if (NP >= 16) {
#pragma unroll
    for (int j = 0; j < NP / 16; ++j) v[j] = dpp_keep_sum<0x141>(v[j], v[j + NP / 16], (lane & 4) != 0);
  } else {
    v[0] += dpp_move<0x141>(v[0]);
  }
  if (NP >= 32) {
#pragma unroll
    for (int j = 0; j < NP / 32; ++j) v[j] = dpp_keep_sum<0x4E>(v[j], v[j + NP / 32], (lane & 2) != 0);
  } else {
    v[0] += dpp_move<0x4E>(v[0]);
  }
  if (NP >= 64) {
    v[0] = dpp_keep_sum<0xB1>(v[0], v[1], (lane & 1) != 0);
  } else {
    v[0] += dpp_move<0xB1>(v[0]);
  }
  constexpr int SH = (NP == 1) ? 6 : (NP == 2) ? 5 : (NP == 4) ? 4 : (NP == 8) ? 3 : (NP == 16) ? 2 : (NP == 32) ? 1 : 0;
  const int i = lane >> SH;
  idx = ((lane & ((1 << SH) - 1)) == 0 && i < NV) ? i : -1;
  return v[0];
}

// Row access of row-major n x R blocks with one vector memory instruction per 16 bytes.
// Every block starts at a multiple of n R sizeof(T) bytes of a hipMalloc allocation, so a
// row of R = 2 or 4 elements is aligned to its vector size.
template <typename T, int R>
__device__ inline void load_row(const T* __restrict__ p, int row, double (&x)[R]) {
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
    for (int c = 0; c < R; ++c) x[c] = static_cast<double>(q[c]);
  }
}

// Stores the row rounded to T; x is replaced by the stored (rounded) values.
template <typename T, int R>
__device__ inline void store_row(T* __restrict__ p, int row, double (&x)[R]) {
  T* q = p + (size_t)row * R;
  if constexpr (sizeof(T) == 4 && R == 4) {
    const float4 v = make_float4((float)x[0], (float)x[1], (float)x[2], (float)x[3]);
    *reinterpret_cast<float4*>(q) = v;
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
  } else if constexpr (sizeof(T) == 4 && R == 2) {
    const float2 v = make_float2((float)x[0], (float)x[1]);
    *reinterpret_cast<float2*>(q) = v;
    x[0] = v.x; x[1] = v.y;
  } else if constexpr (sizeof(T) == 8 && R % 2 == 0) {
#pragma unroll
    for (int c = 0; c < R; c += 2) *reinterpret_cast<double2*>(q + c) = make_double2(x[c], x[c + 1]);
  } else {
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const T t = static_cast<T>(x[c]);
      q[c] = t;
      x[c] = static_cast<double>(t);
    }
  }
}

}  // namespace skr
