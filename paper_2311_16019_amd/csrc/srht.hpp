// Subsampled randomized DCT embedding (the trigonometric embedding of Sec. 2.2 that the
// experiments of Sec. 6 use): S x = sqrt(n / s) * DCT2(E x)[rows], with the orthonormal DCT-II,
// a Rademacher diagonal E and s distinct sampled rows.
//
// Random draws (SplitMix64, Steele, Lea and Flood 2014): E_j = -1 when the lowest bit of
// output j + 1 of the generator started at `seed` is set; rows = the s indices i with the
// smallest output i + 1 of the generator started at mix64(seed) (ties by index), ascending.
//
// The DCT of each column is taken through a complex DFT of length n of the reordered
// sequence v = (y_0, y_2, y_4, .., .., y_5, y_3, y_1) (Makhoul 1980):
// DCT2(y)_k ~ Re(exp(-i pi k / (2n)) V_k).  With n = N1 N2 and N1 = P Q the DFT splits as
//   stage 1 (every b < N2):  Z[k1][b] = w_n^{b k1} sum_a v[N2 a + b] w_N1^{a k1}
//            (the length-N1 DFT in LDS as P-point and Q-point passes)
//   stage 2 (sampled k only): V_k = sum_b Z[k mod N1][b] w_N2^{b (k div N1)}
// so only the s sampled outputs of the second stage are formed.
#pragma once

#include <cstdint>
#include <vector>

#include "common.hpp"

namespace skr {

struct SrhtPlan {
  int64_t n = 0;
  int N1 = 0, N2 = 0, P = 0, Q = 0;
  int s = 0;
  uint64_t seed = 0;           // sign seed of this space
  std::vector<int> soff;       // N1 + 1 offsets of the samples grouped by k mod N1
  std::vector<int> samp;       // 2 ints per sample: output row i and frequency k
};

// Factorisation of n and the sampled rows (host; cached by (n, s, seed)).  Throws
// SKR_ENOTSUP when n has no factorisation n = N1 N2, N1 = P Q with P, Q <= 64 and N1, N2 within
// the kernels' shared-memory limits.
SrhtPlan srht_plan(int64_t n, int s, uint64_t seed);

template <typename T>
struct SrhtSpace {
  const T* U;          // n x r row-major block to sketch
  double* Z;           // workspace: r x N1 x N2 complex (interleaved re, im)
  const int* soff;     // device copy of SrhtPlan::soff
  const int* samp;     // device copy of SrhtPlan::samp
  double* wraw;        // s x r: S U before the pending factor
  double* w;           // s x r output
  const double* Pend;  // pending right factor (r x r row-major) or null
  int64_t n;
  int N1, N2, P, Q;
  uint64_t seed;
};

size_t srht_z_doubles(int64_t n, int r);  // size of SrhtSpace::Z
// w = (S U) Pend for one or two spaces (b ignored when nspaces is 1; a space with n = 0 is
// skipped).
template <typename T>
void launch_srht(int r, int s, const SrhtSpace<T>& a, const SrhtSpace<T>& b, int nspaces, size_t lds_limit,
                 hipStream_t st);

}  // namespace skr
