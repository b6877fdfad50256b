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
};

size_t whiten_part_doubles(int s, int r, int maxm);

// Append the block for step d (m = d r current columns of Q).  `init` = true builds Q_1,
// T_1 from w alone (m = 0).  Processes both spaces in every launch, or only `a` when
// nspaces is 1.
void launch_whiten(int r, int s, int m, int step, const WhitenSpace& a, const WhitenSpace& b, hipStream_t st,
                   int nspaces = 2);

}  // namespace skr
