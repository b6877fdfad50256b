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
};

template <typename T>
CsrView<T> csr_view(const skr_op_s* op, int transpose);

}  // namespace skr
