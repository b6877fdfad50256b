// Block-step kernels of the truncated block Arnoldi recurrence (Algorithm 1's inner loop):
// sparse block product, truncated block Gram-Schmidt, Cholesky QR of the new block and
// the sparse sign sketch.  Both Krylov spaces are processed by every launch.
#pragma once

#include "op.hpp"

namespace skr {

// Per-space small state kept on the device (FP64).  Offsets in doubles.
struct SmallLayout {
  static constexpr int COEF = 0;                       // r x r coefficients of the next axpy
  static constexpr int OUT = COEF + RMAX * RMAX;       // reduced output of the last kernel (r*r + 1)
  static constexpr int NRMOP = OUT + RMAX * RMAX + 8;  // ||Op U_d||_F^2
  static constexpr int R1 = NRMOP + 8;                 // first Cholesky factor
  static constexpr int R1INV = R1 + RMAX * RMAX;
  static constexpr int RF = R1INV + RMAX * RMAX;       // final R = R2 R1 (h_{d+1,d})
  static constexpr int RFINV = RF + RMAX * RMAX;
  static constexpr int SIZE = RFINV + RMAX * RMAX;
};

// Post-processing done by the last workgroup of a reduction kernel.
enum PostMode : int {
  POST_DOT = 0,    // h = reduced r x r block: store into H and into COEF
  POST_GRAM1 = 1,  // Cholesky of the Gram matrix of the orthogonalised block
  POST_GRAM2 = 2,  // second Cholesky (CholQR2), final R into H
};

template <typename T>
struct SpaceStep {
  CsrView<T> A;         // operator of this space (spmm only)
  const T* X;           // spmm input block U_d
  T* Y;                 // work block (U tilde), n x r
  const T* W;           // window block U_i (dot partner / axpy source)
  const T* Wn;          // next window block U_{i+1} for the fused dot, or null
  T* Unew;              // destination of the normalised block (normalize only)
  double* small;        // SmallLayout state
  double* part;         // per-workgroup partials
  int* broken;          // first step at which this space broke down (INT_MAX if none)
  double* Hblk;         // destination of h (column-major block in H), or null
  int ldh;
  int n;
  int nwg;              // workgroups of this space
  int step;             // current block step d (1-based) for breakdown bookkeeping
  int post;             // PostMode
};

// Launchers; each processes both spaces in one grid.
template <typename T>
void launch_spmm_dot(int r, const SpaceStep<T>& s0, const SpaceStep<T>& s1, hipStream_t st);
template <typename T>
void launch_axpy_reduce(int r, const SpaceStep<T>& s0, const SpaceStep<T>& s1, hipStream_t st);
template <typename T>
void launch_gram2(int r, const SpaceStep<T>& s0, const SpaceStep<T>& s1, hipStream_t st);
template <typename T>
void launch_normalize(int r, const SpaceStep<T>& s0, const SpaceStep<T>& s1, hipStream_t st);

// Sparse sign embedding table: tab[t*n + j] = bucket | (negative << 15), for t < zeta.
void launch_build_sketch_table(uint16_t* tab, int n, int zeta, int b, uint64_t seed, hipStream_t st);

template <typename T>
struct SketchSpace {
  const T* U;            // n x r block to sketch
  const uint16_t* tab;   // zeta x n table
  double* part;          // [nchunk][s][r] partial sums
  double* w;             // s x r output (row-major), scaled by 1/sqrt(zeta)
  int n, nchunk;
};
template <typename T>
void launch_sketch(int r, int s, int zeta, const SketchSpace<T>& a, const SketchSpace<T>& b,
                   size_t lds_limit, hipStream_t st);

int sketch_chunks(int n);

}  // namespace skr
