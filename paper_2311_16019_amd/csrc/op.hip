// Sparse operator creation: validation and transpose on the host, then upload.
#include <algorithm>
#include <memory>

#include "op.hpp"

namespace skr {

template <>
CsrView<double> csr_view<double>(const skr_op_s* op, int t) {
  return {static_cast<int>(op->n), op->rowptr[t].p, op->colind[t].p, op->val64[t].p,
          op->has_diag ? op->diag.p : nullptr};
}
template <>
CsrView<float> csr_view<float>(const skr_op_s* op, int t) {
  return {static_cast<int>(op->n), op->rowptr[t].p, op->colind[t].p, op->val32[t].p,
          op->has_diag ? op->diag.p : nullptr};
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
