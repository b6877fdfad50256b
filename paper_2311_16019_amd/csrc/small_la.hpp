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
