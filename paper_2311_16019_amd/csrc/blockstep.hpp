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
  // 1: the block has columns of about unit norm and is accumulated in fixed point
  // (deterministic); 0: unbounded entries (the SpMM output U~), FP64 atomics
  int fixed = 1;
};
template <typename T>
void launch_sketch(int r, int s, int zeta, const SketchSpace<T>& a, const SketchSpace<T>& b,
                   size_t lds_limit, hipStream_t st);

int sketch_chunks(int n, int nspaces);
// Sketch with a pending right factor: w = (S U') P / sqrt(zeta), P (r x r row-major, device)
// or null for the identity.
template <typename T>
void launch_sketch_pending(int r, int s, int zeta, const SketchSpace<T>& a, const SketchSpace<T>& b,
                           const double* Pa, const double* Pb, size_t lds_limit, hipStream_t st);

// ---- Two-pass block step (truncated block classical Gram-Schmidt, reorthogonalised through
// the window Gram matrix, with Cholesky QR twice).  The stored basis block is U'_j with
// U_j = U'_j P_j for a pending r x r factor P_j kept on the device, so that the second
// Cholesky factor never needs a pass of its own.
constexpr int CGS_KMAX = 10;  // window blocks handled by the two-pass step (k <= 10)
constexpr int CGS_RMAX = 4;   // block sizes handled by the two-pass step (r <= 4)

inline bool cgs_supported(int r, int k) { return r <= CGS_RMAX && k <= CGS_KMAX; }

template <typename T>
struct CgsPass {
  CsrView<T> A;               // operator (pass 1)
  const T* X;                 // U'_d, the SpMM input (pass 1)
  const double* src;          // pass 1 reads this n x r FP64 block instead of the SpMM (start block)
  const double* Pd;           // pending factor of X (r x r row-major), null = identity
  T* Y;                       // U~ (pass 1 output, pass 2 input)
  T* Unew;                    // U'_{d+1} (pass 2 output)
  const T* W[CGS_KMAX];       // window blocks U'_{i0} .. U'_d
  const double* coef;         // pass 2: [R1^{-1} | C_0 .. C_{nw-1}], r x r row-major each
  double* part;               // per-workgroup partials, value-major
  int n, nwg;
};

// Per-space small state of the two-pass step (device pointers, FP64, r x r row-major blocks).
struct CgsSmall {
  double* part;               // partials of the pass just run
  int nwg;
  double* Pall;               // P_j at Pall + j r^2 (j = 0 .. maxit + 1)
  double* Gall;               // U'_j^T U'_j at Gall + j r^2
  double* Xall;               // U'_{j-1-t}^T U'_j at Xall + (j KMAX + t) r^2
  double* state;              // CgsLayout
  double* H;                  // Hessenberg matrix (column-major, ldh), or the start block's R
  int ldh;
  int* broken;
};

// Pass 1 is two sweeps: the SpMM (many workgroups) and the window products (CgsPass::nwg
// workgroups, whose partials reduce 1 reads).
template <typename T>
void launch_cgs_spmm(int r, const CgsPass<T>& a, const CgsPass<T>& b, hipStream_t st);
template <typename T>
void launch_cgs_dots(int r, int nw, const CgsPass<T>& a, const CgsPass<T>& b, hipStream_t st);
template <typename T>
void launch_cgs_pass2(int r, int nw, const CgsPass<T>& a, const CgsPass<T>& b, hipStream_t st);
// Small-world work after pass 1 (block step d, window i0 .. d with nw = d - i0 + 1 blocks;
// d = 0, nw = 0 for the start block) and after pass 2.
void launch_cgs_reduce1(int r, int nw, int i0, int d, const CgsSmall& a, const CgsSmall& b, hipStream_t st);
void launch_cgs_reduce2(int r, int nw, int i0, int d, const CgsSmall& a, const CgsSmall& b, hipStream_t st);
int cgs_state_doubles();
int cgs_coef_offset();  // offset of [R1^{-1} | C_0 ..] in CgsSmall::state
int cgs_wgs(int n);     // workgroups per space of the sweeps that write partials

}  // namespace skr
