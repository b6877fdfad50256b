// Sketched QR update of Prop. 2.1 (Algorithm 1's whitening step), FP64 on the device:
// given w = S U_{d+1} (s x r), extend Q_{d} (s x dr, orthonormal columns) and the upper
// triangular T_d (dr x dr) to Q_{d+1}, T_{d+1} by block classical Gram-Schmidt with one
// re-orthogonalisation pass and a Cholesky QR (twice) of the remainder.
#pragma once

#include "common.hpp"

namespace skr {

struct WhitenSpace {
  double* Q;      // column-major s x (maxit+1) r, leading dimension s
  double* T;      // column-major, leading dimension ldt
  double* w;      // s x r row-major: sketch of the new block, overwritten
  double* c1;     // m x r row-major: first-pass coefficients
  double* c2;     // m x r row-major: second-pass coefficients
  double* part;   // partial products of Q^T w, one m x r slab per chunk of rows
  int* broken;    // breakdown marker of this space
  int ldt;
  // Delayed re-orthogonalisation (whiten_delayed_supported): the pending block's remainder
  // and the new block side by side (s x 2r row-major), their products with Q (m x 2r), the
  // pending block's first-pass coefficients (m x r) and an s x r staging block.
  double* Z = nullptr;
  double* cz = nullptr;
  double* cstash = nullptr;
  double* zf = nullptr;
  double* fpart = nullptr;   // workgroup partials of the finishing reductions (whiten_fin_doubles)
  double* fstate = nullptr;  // their outcome: Cholesky success flags (whiten_fin_state_doubles)
};

size_t whiten_fin_doubles();
size_t whiten_fin_state_doubles();

size_t whiten_part_doubles(int s, int r, int maxm);

// Delayed classical Gram-Schmidt with re-orthogonalisation (the DCGS2 scheme of Swirydowicz,
// Langou, Ananthan, Yang and Thomas, Numer. Linear Algebra Appl. 2021, in block form): the
// second pass of block j is taken in the same two sweeps over Q as the first pass of block
// j + 1, so that Q is read twice per block step instead of four times.  Modes:
//   WHITEN_FIRST   no block pending: first pass of the new block (in w) against the m
//                  columns of Q; the remainder becomes the pending block.
//   WHITEN_APPEND  pending block and new block: both against the m columns of Q in 2r-wide
//                  sweeps; the pending block is finished (Cholesky QR twice), appended as
//                  columns m .. m+r-1 of Q and of T; the new block's remainder, projected
//                  off the appended columns too, becomes the pending block.
//   WHITEN_FLUSH   the pending block alone is finished and appended (before a projected
//                  solve, which needs T of every block).
// `step` is the breakdown marker written if the finished block is rank deficient.
enum { WHITEN_FIRST = 0, WHITEN_APPEND = 1, WHITEN_FLUSH = 2 };
inline bool whiten_delayed_supported(int r) { return r <= 8; }
void launch_whiten_delayed(int r, int s, int m, int step, int mode, const WhitenSpace& a, const WhitenSpace& b,
                           hipStream_t st, int nspaces = 2);

// Append the block for step d (m = d r current columns of Q).  `init` = true builds Q_1,
// T_1 from w alone (m = 0).  Processes both spaces in every launch, or only `a` when
// nspaces is 1.
void launch_whiten(int r, int s, int m, int step, const WhitenSpace& a, const WhitenSpace& b, hipStream_t st,
                   int nspaces = 2);

}  // namespace skr
