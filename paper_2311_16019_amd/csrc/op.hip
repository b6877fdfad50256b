// Sparse operator creation: validation and transpose on the host, then upload.
#include <algorithm>
#include <climits>
#include <memory>
#include <vector>

#include "op.hpp"

namespace skr {

template <>
CsrView<double> csr_view<double>(const skr_op_s* op, int t) {
  return {static_cast<int>(op->n), op->rowptr[t].p, op->colind[t].p, op->val64[t].p,
          op->has_diag ? op->diag.p : nullptr, op->sell_off[t].p, op->sell_col[t].p, op->sell_v64[t].p};
}
template <>
CsrView<float> csr_view<float>(const skr_op_s* op, int t) {
  return {static_cast<int>(op->n), op->rowptr[t].p, op->colind[t].p, op->val32[t].p,
          op->has_diag ? op->diag.p : nullptr, op->sell_off[t].p, op->sell_col[t].p, op->sell_v32[t].p};
}

void validate_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind) {
  SKR_REQUIRE(n > 0 && n < (int64_t(1) << 31) - 1, "operator size n must be in [1, 2^31-1)");
  SKR_REQUIRE(nnz >= 0 && nnz < (int64_t(1) << 31), "nnz must fit in int32");
  SKR_REQUIRE(rowptr && (nnz == 0 || colind), "null CSR array");
  SKR_REQUIRE(rowptr[0] == 0 && rowptr[n] == nnz, "rowptr must start at 0 and end at nnz");
  for (int64_t i = 0; i < n; ++i)
    SKR_REQUIRE(rowptr[i + 1] >= rowptr[i], "rowptr must be nondecreasing");
  for (int64_t k = 0; k < nnz; ++k)
    SKR_REQUIRE(colind[k] >= 0 && colind[k] < n, "column index out of range");
}

// Counting-sort transpose of a CSR matrix (column indices of the result come out sorted
// within each row because rows of the input are visited in order).
void transpose_csr(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci, const double* v,
                   std::vector<int32_t>& trp, std::vector<int32_t>& tci, std::vector<double>& tv) {
  trp.assign(n + 1, 0);
  tci.resize(nnz);
  tv.resize(nnz);
  for (int64_t k = 0; k < nnz; ++k) trp[ci[k] + 1]++;
  for (int64_t i = 0; i < n; ++i) trp[i + 1] += trp[i];
  std::vector<int32_t> next(trp.begin(), trp.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      int32_t j = ci[k];
      int32_t pos = next[j]++;
      tci[pos] = static_cast<int32_t>(i);
      tv[pos] = v[k];
    }
}

// Sliced ELL with SELL_C rows per slice: slice q's width is the longest row among rows
// q SELL_C .. q SELL_C + SELL_C - 1; entry j of its row l sits at off[q] + j SELL_C + l.
// Returns false when the padded entry count does not fit in int32.
bool sell_build(int64_t n, const int32_t* rp, const int32_t* ci, const double* v, std::vector<int32_t>& off,
                std::vector<int32_t>& col, std::vector<double>& val) {
  const int64_t ns = (n + SELL_C - 1) / SELL_C;
  off.assign(ns + 1, 0);
  int64_t total = 0;
  for (int64_t q = 0; q < ns; ++q) {
    int32_t w = 0;
    for (int64_t i = q * SELL_C; i < std::min(n, (q + 1) * SELL_C); ++i) w = std::max(w, rp[i + 1] - rp[i]);
    off[q] = static_cast<int32_t>(std::min<int64_t>(total, INT32_MAX));
    total += (int64_t)w * SELL_C;
    if (total >= INT32_MAX) return false;
  }
  off[ns] = static_cast<int32_t>(total);
  col.assign(total, 0);
  val.assign(total, 0.0);
  for (int64_t q = 0; q < ns; ++q) {
    const int32_t w = (off[q + 1] - off[q]) / SELL_C;
    for (int l = 0; l < SELL_C; ++l) {
      const int64_t i = q * SELL_C + l;
      for (int32_t j = 0; j < w; ++j) {
        const int64_t e = off[q] + (int64_t)j * SELL_C + l;
        const int32_t k = (i < n) ? rp[i] + j : 0;
        if (i < n && k < rp[i + 1]) {
          col[e] = ci[k];
          val[e] = v[k];
        } else {
          col[e] = static_cast<int32_t>(i < n ? i : n - 1);  // padding: a valid row, value 0
          val[e] = 0.0;
        }
      }
    }
  }
  return true;
}

}  // namespace skr

using namespace skr;

skr_op_s* op_create(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                    const double* vals, const double* diag, hipStream_t stream) {
  validate_csr(n, nnz, rowptr, colind);
  SKR_REQUIRE(nnz == 0 || vals, "null CSR values");
  std::unique_ptr<skr_op_s> op(new skr_op_s());
  op->n = n;
  op->nnz = nnz;
  std::vector<int32_t> trp, tci;
  std::vector<double> tv;
  transpose_csr(n, nnz, rowptr, colind, vals, trp, tci, tv);
  const int32_t* rps[2] = {rowptr, trp.data()};
  const int32_t* cis[2] = {colind, tci.data()};
  const double* vs[2] = {vals, tv.data()};
  std::vector<float> v32(nnz);
  for (int t = 0; t < 2; ++t) {
    op->rowptr[t].alloc(n + 1);
    op->colind[t].alloc(std::max<int64_t>(nnz, 1));
    op->val64[t].alloc(std::max<int64_t>(nnz, 1));
    op->val32[t].alloc(std::max<int64_t>(nnz, 1));
    SKR_HIP(hipMemcpyAsync(op->rowptr[t].p, rps[t], (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    if (nnz) {
      SKR_HIP(hipMemcpyAsync(op->colind[t].p, cis[t], nnz * sizeof(int32_t), hipMemcpyHostToDevice, stream));
      SKR_HIP(hipMemcpyAsync(op->val64[t].p, vs[t], nnz * sizeof(double), hipMemcpyHostToDevice, stream));
      for (int64_t k = 0; k < nnz; ++k) v32[k] = static_cast<float>(vs[t][k]);
      SKR_HIP(hipMemcpyAsync(op->val32[t].p, v32.data(), nnz * sizeof(float), hipMemcpyHostToDevice, stream));
      // the host staging buffer is reused: wait before overwriting it
      SKR_HIP(hipStreamSynchronize(stream));
    }
  }
  for (int t = 0; t < 2; ++t) {
    std::vector<int32_t> off, col;
    std::vector<double> val;
    if (!sell_build(n, rps[t], cis[t], vs[t], off, col, val)) continue;
    std::vector<float> val32(val.begin(), val.end());
    op->sell_off[t].alloc(off.size());
    op->sell_col[t].alloc(std::max<size_t>(col.size(), 1));
    op->sell_v64[t].alloc(std::max<size_t>(val.size(), 1));
    op->sell_v32[t].alloc(std::max<size_t>(val.size(), 1));
    SKR_HIP(hipMemcpyAsync(op->sell_off[t].p, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    if (!col.empty()) {
      SKR_HIP(hipMemcpyAsync(op->sell_col[t].p, col.data(), col.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
      SKR_HIP(hipMemcpyAsync(op->sell_v64[t].p, val.data(), val.size() * sizeof(double), hipMemcpyHostToDevice, stream));
      SKR_HIP(hipMemcpyAsync(op->sell_v32[t].p, val32.data(), val32.size() * sizeof(float), hipMemcpyHostToDevice,
                             stream));
    }
    SKR_HIP(hipStreamSynchronize(stream));  // host staging vectors go out of scope
  }
  op->diag.alloc(n);
  if (diag) {
    SKR_HIP(hipMemcpyAsync(op->diag.p, diag, n * sizeof(double), hipMemcpyHostToDevice, stream));
    op->has_diag = true;
  }
  SKR_HIP(hipStreamSynchronize(stream));
  return op.release();
}

void op_set_diag(skr_op_s* op, const double* diag, hipStream_t stream) {
  SKR_REQUIRE(op, "null operator");
  if (!diag) {
    op->has_diag = false;
    return;
  }
  SKR_HIP(hipMemcpyAsync(op->diag.p, diag, op->n * sizeof(double), hipMemcpyDeviceToDevice, stream));
  op->has_diag = true;
}
