// Sketched-inner-product orthogonalisation of a new Krylov block (the truncated
// orthogonalisation in the inner product <x, y>_S = (S x)^T (S y), the variant that appendix A
// names as an alternative to the Euclidean one).  The block step becomes
//
//   U~ = Op U_d                                 (SpMM, n rows)
//   w  = S U~                                   (sparse sign sketch, s rows)
//   h_i = (S U_i)^T w,  w <- w - (S U_i) h_i     for the window i = i0 .. d (s rows only)
//   w = q R (Cholesky QR twice),  S U_{d+1} = q  (s rows only)
//   U_{d+1} = (U~ - sum_i U_i h_i) R^{-1}       (one pass over n rows)
//
// so every inner product is taken on s-row sketches and the long vectors are read once per
// pass.  S U_{d+1} is then already known and feeds the sketched QR update of Prop. 2.1 without
// a second sketch.
#pragma once

#include "common.hpp"

namespace skr {

struct SorthSpace {
  double* w;        // s x r row-major: S U~ on entry, overwritten
  double* ring;     // nring slots of s x r: S U_j in slot j % nring
  int nring;
  double* wout;     // s x r: copy of S U_{d+1} for the sketched QR update (which overwrites it),
                    // or null when the update takes a sketch of the stored block instead
  double* coef;     // [R^{-1} | h_{i0} R^{-1} | ..] r x r row-major each, read by the update pass
  double* H;        // column-major, leading dimension ldh; for the start block its R factor
  int ldh;
  int* broken;      // first step at which the space broke down (INT_MAX if none)
  double* part;     // sorth_part_doubles(): per-workgroup partial sums (two sets, alternating)
  double* state;    // sorth_state_doubles(): coefficients and factors passed between launches
};

int sorth_groups(int s);          // workgroups per space of each launch
size_t sorth_part_doubles();
size_t sorth_state_doubles();

// Block step d (d = 0: the start block, nw = 0) on the window i0 .. i0 + nw - 1 (nw <= 3,
// r <= 4): nw + 3 launches, each over both spaces or only `a` when nspaces is 1.
void launch_sorth(int r, int s, int nw, int i0, int d, const SorthSpace& a, const SorthSpace& b, int nspaces,
                  hipStream_t st);

}  // namespace skr
