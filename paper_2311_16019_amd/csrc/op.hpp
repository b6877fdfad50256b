// Device-resident sparse operator: CSR of M and of M^T, FP64 and FP32 values.
#pragma once

#include "common.hpp"

struct skr_op_s {
  int64_t n = 0, nnz = 0;
  // index 0: M, index 1: M^T
  skr::DBuf<int32_t> rowptr[2], colind[2];
  skr::DBuf<double> val64[2];
  skr::DBuf<float> val32[2];
  skr::DBuf<double> diag;  // empty when the operator has no diagonal term
  bool has_diag = false;
  // The same matrices sliced into ELL blocks of SELL_C consecutive rows (see sell_build):
  // slice q holds its rows' entries column by column, entry j of row q SELL_C + l at
  // sell_off[q] + j SELL_C + l; rows shorter than the slice's longest row are padded with
  // zero values whose column is the row itself.
  skr::DBuf<int32_t> sell_off[2], sell_col[2];
  skr::DBuf<double> sell_v64[2];
  skr::DBuf<float> sell_v32[2];
};

namespace skr {

// The view the kernels take of one operator orientation.
template <typename T>
struct CsrView {
  int n;
  const int32_t* rowptr;
  const int32_t* colind;
  const T* val;
  const double* diag;  // nullptr when absent
  const int32_t* sell_off;  // sliced-ELL form of the same matrix (nullptr when absent)
  const int32_t* sell_col;
  const T* sell_val;
};

constexpr int SELL_C = 64;  // rows per slice: one wavefront

template <typename T>
CsrView<T> csr_view(const skr_op_s* op, int transpose);

}  // namespace skr
