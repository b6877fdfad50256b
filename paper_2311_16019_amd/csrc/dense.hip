// FP64 dense kernels for the projected problems: tiled GEMM, triangular solves and
// elementwise helpers (inverses and dense solves are in gauss_jordan.hip).
#include <algorithm>
#include <cmath>
#include <map>

#include <rocblas/rocblas.h>

#include "dense.hpp"

namespace skr {
namespace dense {
namespace {

constexpr int BM = 64, BN = 64, BK = 32, GT = 256;

// Element loaders: op(A)(i, k) and op(B)(k, j).  FAST selects the index that varies
// fastest in memory so that tile loads are coalesced.
struct LoadAN {  // A column-major, not transposed: fast in i
  const double* A; int lda;
  static constexpr bool I_FAST = true;
  __device__ double operator()(int i, int k) const { return A[i + (size_t)k * lda]; }
};
struct LoadAT {  // A^T: fast in k
  const double* A; int lda;
  static constexpr bool I_FAST = false;
  __device__ double operator()(int i, int k) const { return A[k + (size_t)i * lda]; }
};
struct LoadBN {  // B column-major, not transposed: fast in k
  const double* B; int ldb;
  static constexpr bool K_FAST = true;
  __device__ double operator()(int k, int j) const { return B[k + (size_t)j * ldb]; }
};
struct LoadBT {  // B^T: fast in j
  const double* B; int ldb;
  static constexpr bool K_FAST = false;
  __device__ double operator()(int k, int j) const { return B[j + (size_t)k * ldb]; }
};
template <typename T>
struct LoadBasis {  // (i, q) -> U_{q / r}[i][q % r] for consecutive row-major n x r blocks
  const T* U; int n, r;
  static constexpr bool I_FAST = false;
  __device__ double operator()(int i, int q) const {
    const int j = q / r, c = q - j * r;
    return static_cast<double>(U[((size_t)j * n + i) * r + c]);
  }
};
struct StoreCM {  // column-major C; K-slice z writes to C + z * zstride
  double* C; int ldc; double alpha, beta; size_t zstride = 0;
  __device__ void operator()(int i, int j, double v, int z) const {
    double* p = C + (size_t)z * zstride + i + (size_t)j * ldc;
    *p = (beta == 0.0) ? alpha * v : alpha * v + beta * *p;
  }
};
struct StoreRM {  // row-major C (element (i, j) at i*ldc + j)
  double* C; int ldc; double alpha, beta; size_t zstride = 0;
  __device__ void operator()(int i, int j, double v, int z) const {
    double* p = C + (size_t)z * zstride + (size_t)i * ldc + j;
    *p = (beta == 0.0) ? alpha * v : alpha * v + beta * *p;
  }
};

// FP64 GEMM tile on the matrix cores (v_mfma_f64_16x16x4f64; a 16 x 16 x 4 product takes
// A(i, k) from lane i + 16 k, B(k, j) from lane j + 16 k, and leaves D(4 v + g, j) in
// register v of lane j + 16 g).  Workgroup tile BM x BN = 64 x 64 from four wavefronts of
// 32 x 32 (2 x 2 MFMA tiles); K in chunks of BK staged in LDS as [row][k] (k fastest, padded),
// loaded into registers one chunk ahead.  Inside a group of 16 consecutive k, lane group
// g = lane / 16 owns k = 4 g + s at MFMA step s, so each lane reads its four A (and B) values
// of a group as two 16-byte LDS loads.  blockIdx.z selects a K slice of length kchunk.
constexpr int LDK = BK + 2;
constexpr int GPT = BM * BK / GT;  // staged elements of A (and of B) per thread

typedef double gm_d4 __attribute__((ext_vector_type(4)));

template <class LA, class LB, class ST>
__global__ void __launch_bounds__(GT) gemm_kernel(int m, int n, int k, LA la, LB lb, ST st, int kchunk) {
  __shared__ __attribute__((aligned(16))) double As[BM * LDK];
  __shared__ __attribute__((aligned(16))) double Bs[BN * LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int wr = wave >> 1, wc = wave & 1;
  const int i0 = blockIdx.x * BM, j0 = blockIdx.y * BN;
  const int kb = blockIdx.z * kchunk, ke = min(k, kb + kchunk);
  gm_d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = gm_d4{0.0, 0.0, 0.0, 0.0};
  // staging coordinates: element e = tid + GT u of the chunk, coalesced along the fast index
  auto a_coord = [&](int u, int& ii, int& kk) {
    const int e = tid + GT * u;
    if constexpr (LA::I_FAST) { ii = e % BM; kk = e / BM; } else { kk = e % BK; ii = e / BK; }
  };
  auto b_coord = [&](int u, int& jj, int& kk) {
    const int e = tid + GT * u;
    if constexpr (LB::K_FAST) { kk = e % BK; jj = e / BK; } else { jj = e % BN; kk = e / BN; }
  };
  double ra[GPT], rb[GPT];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      int ii, kk, jj, k2;
      a_coord(u, ii, kk);
      ra[u] = (i0 + ii < m && k0 + kk < ke) ? la(i0 + ii, k0 + kk) : 0.0;
      b_coord(u, jj, k2);
      rb[u] = (j0 + jj < n && k0 + k2 < ke) ? lb(k0 + k2, j0 + jj) : 0.0;
    }
  };
  if (kb < ke) fetch(kb);
  for (int k0 = kb; k0 < ke; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      int ii, kk, jj, k2;
      a_coord(u, ii, kk);
      As[ii * LDK + kk] = ra[u];
      b_coord(u, jj, k2);
      Bs[jj * LDK + k2] = rb[u];
    }
    __syncthreads();
    if (k0 + BK < ke) fetch(k0 + BK);
#pragma unroll
    for (int t = 0; t < BK / 16; ++t) {
      double av[2][4], bv[2][4];
#pragma unroll
      for (int r2 = 0; r2 < 2; ++r2) {
        const double* pa = As + (wr * 32 + r2 * 16 + l16) * LDK + 16 * t + 4 * g;
        const double2 a01 = *reinterpret_cast<const double2*>(pa);
        const double2 a23 = *reinterpret_cast<const double2*>(pa + 2);
        av[r2][0] = a01.x; av[r2][1] = a01.y; av[r2][2] = a23.x; av[r2][3] = a23.y;
        const double* pb = Bs + (wc * 32 + r2 * 16 + l16) * LDK + 16 * t + 4 * g;
        const double2 b01 = *reinterpret_cast<const double2*>(pb);
        const double2 b23 = *reinterpret_cast<const double2*>(pb + 2);
        bv[r2][0] = b01.x; bv[r2][1] = b01.y; bv[r2][2] = b23.x; bv[r2][3] = b23.y;
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int r2 = 0; r2 < 2; ++r2)
#pragma unroll
          for (int c2 = 0; c2 < 2; ++c2)
            acc[r2][c2] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[r2][s], bv[c2][s], acc[r2][c2], 0, 0, 0);
    }
  }
#pragma unroll
  for (int r2 = 0; r2 < 2; ++r2)
#pragma unroll
    for (int c2 = 0; c2 < 2; ++c2) {
      const int j = j0 + wc * 32 + c2 * 16 + l16;
      if (j >= n) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wr * 32 + r2 * 16 + 4 * v + g;
        if (i < m) st(i, j, acc[r2][c2][v], blockIdx.z);
      }
    }
}

// C = alpha * sum_z W[z] + beta * C  (column-major m x n, W slices contiguous m x n)
__global__ void splitk_reduce_kernel(int m, int n, int nz, const double* W, double alpha, double beta, double* C,
                                     int ldc) {
  const size_t total = (size_t)m * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    double t = 0.0;
    for (int z = 0; z < nz; ++z) t += W[(size_t)z * total + e];
    const int i = (int)(e % m), j = (int)(e / m);
    double* p = C + i + (size_t)j * ldc;
    *p = (beta == 0.0) ? alpha * t : alpha * t + beta * *p;
  }
}

template <class LA, class LB, class ST>
void run_gemm(int m, int n, int k, LA la, LB lb, ST st, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  dim3 grid(ceil_div(m, BM), ceil_div(n, BN));
  hipLaunchKernelGGL((gemm_kernel<LA, LB, ST>), grid, dim3(GT), 0, s, m, n, k, la, lb, st, std::max(k, 1));
  check_launch("gemm");
}

// Few output tiles and a long reduction: split K over workgroups into partial products
// and sum them in a fixed order (column-major C only).
// Number of K slices and their length for a split-K product, or false when the product
// is not split (many output tiles or a short reduction).
bool splitk_plan(int m, int n, int k, int* nz_out, int* kchunk_out) {
  const int tiles = ceil_div(m, BM) * ceil_div(n, BN);
  if (tiles >= 64 || k < 8192) return false;
  int nz = std::min(512 / tiles + 1, ceil_div(k, 2048));
  nz = std::max(2, std::min(nz, 256));
  const int kchunk = ceil_div(ceil_div(k, nz), BK) * BK;
  *nz_out = ceil_div(k, kchunk);
  *kchunk_out = kchunk;
  return true;
}

// ws: caller-provided room for the nz m x n partial products, or null to take it from the
// device-memory cache.
template <class LA, class LB>
bool run_gemm_splitk(int m, int n, int k, LA la, LB lb, double alpha, double beta, double* C, int ldc, double* ws,
                     hipStream_t s) {
  int nz = 0, kchunk = 0;
  if (!splitk_plan(m, n, k, &nz, &kchunk)) return false;
  DBuf<double> W;
  if (!ws) W.alloc((size_t)nz * m * n);
  double* wp = ws ? ws : W.p;
  StoreCM sw{wp, m, 1.0, 0.0, (size_t)m * n};
  dim3 grid(ceil_div(m, BM), ceil_div(n, BN), nz);
  hipLaunchKernelGGL((gemm_kernel<LA, LB, StoreCM>), grid, dim3(GT), 0, s, m, n, k, la, lb, sw, kchunk);
  check_launch("gemm_splitk");
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3(std::min(2048, ceil_div((int64_t)m * n, 256))), dim3(256), 0, s, m, n,
                     nz, wp, alpha, beta, C, ldc);
  check_launch("splitk_reduce");
  return true;  // W returns to the device-memory cache, which orders its reuse after this work
}

// ----------------------------------------------------------------------- triangular
// Triangular solves by NB x NB diagonal blocks: each diagonal block is inverted once into
// LDS (one thread per column, in registers), then applied as a small dense product;
// the off-diagonal blocks are GEMM updates.
constexpr int NB = 32;

// B[0:nb, :] <- U^{-1} B, U upper triangular (non-unit); one thread per column of B.
__global__ void trsm_lun_diag_kernel(int nb, const double* U, int ldu, double* B, int ldb, int ncols) {
  __shared__ double Us[NB][NB + 1], Ui[NB][NB + 1];
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
    const int i = e % NB, j = e / NB;
    Us[i][j] = (i < nb && j < nb) ? (i <= j ? U[i + (size_t)j * ldu] : 0.0) : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  if (threadIdx.x < NB) {  // column j of U^{-1} (backward substitution on e_j), in registers
    const int j = threadIdx.x;
    double col[NB];
#pragma unroll
    for (int i = NB - 1; i >= 0; --i) {
      double v = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int l = i + 1; l < NB; ++l) v -= Us[i][l] * col[l];
      col[i] = (i <= j) ? v / Us[i][i] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) Ui[i][j] = col[i];
  }
  __syncthreads();
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncols) return;
  double x[NB];
  double* b = B + (size_t)col * ldb;
#pragma unroll
  for (int i = 0; i < NB; ++i) x[i] = (i < nb) ? b[i] : 0.0;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (i < nb) {
      double s = 0.0;
#pragma unroll
      for (int l = i; l < NB; ++l) s += Ui[i][l] * x[l];
      b[i] = s;
    }
  }
}

// B[:, 0:nb] <- B T^{-1}, T upper triangular diagonal block; one thread per row of B.
__global__ void trsm_run_diag_kernel(int nb, const double* T, int ldt, double* B, int ldb, int nrows) {
  __shared__ double Ts[NB][NB + 1], Ti[NB][NB + 1];
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
    const int i = e % NB, j = e / NB;
    Ts[i][j] = (i < nb && j < nb) ? (i <= j ? T[i + (size_t)j * ldt] : 0.0) : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  if (threadIdx.x < NB) {
    const int j = threadIdx.x;
    double col[NB];
#pragma unroll
    for (int i = NB - 1; i >= 0; --i) {
      double v = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int l = i + 1; l < NB; ++l) v -= Ts[i][l] * col[l];
      col[i] = (i <= j) ? v / Ts[i][i] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) Ti[i][j] = col[i];
  }
  __syncthreads();
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nrows) return;
  double x[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) x[c] = (c < nb) ? B[row + (size_t)c * ldb] : 0.0;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c < nb) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l <= c; ++l) s += x[l] * Ti[l][c];
      B[row + (size_t)c * ldb] = s;
    }
  }
}

__global__ void copy_kernel(int m, int n, const double* A, int lda, double* B, int ldb) {
  const size_t total = (size_t)m * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    B[i + (size_t)j * ldb] = A[i + (size_t)j * lda];
  }
}

__global__ void transpose_kernel(int m, int n, const double* A, int lda, double* B, int ldb) {
  __shared__ double tile[32][33];
  const int bi = blockIdx.x * 32, bj = blockIdx.y * 32;
  for (int y = threadIdx.y; y < 32; y += blockDim.y) {
    const int i = bi + threadIdx.x, j = bj + y;
    if (i < m && j < n) tile[y][threadIdx.x] = A[i + (size_t)j * lda];
  }
  __syncthreads();
  for (int y = threadIdx.y; y < 32; y += blockDim.y) {
    const int j = bj + threadIdx.x, i = bi + y;  // B(j, i) = A(i, j)
    if (i < m && j < n) B[j + (size_t)i * ldb] = tile[threadIdx.x][y];
  }
}

__global__ void zero_kernel(int m, int n, double* A, int lda) {
  const size_t total = (size_t)m * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x)
    A[e % m + (e / m) * (size_t)lda] = 0.0;
}

constexpr int RED_WG = 256, RED_MAXG = 1024;

__global__ void combine_kernel(int m, int n, const double* mu_dev, const double* X, int ldx, const double* Y, int ldy,
                               double* Z, int ldz, double* part) {
  const double mu = *mu_dev;
  const size_t total = (size_t)m * n;
  double d2 = 0.0, z2 = 0.0, tr = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    const double x = X[i + (size_t)j * ldx];
    const double z = 0.5 * (mu * x + Y[i + (size_t)j * ldy] / mu);
    Z[i + (size_t)j * ldz] = z;
    d2 += (z - x) * (z - x);
    z2 += z * z;
    if (i == j) tr += z;
  }
  __shared__ double red[3][RED_WG / 64];
  d2 = wave_sum(d2); z2 = wave_sum(z2); tr = wave_sum(tr);
  if (threadIdx.x % 64 == 0) { red[0][threadIdx.x / 64] = d2; red[1][threadIdx.x / 64] = z2; red[2][threadIdx.x / 64] = tr; }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int w = 0; w < RED_WG / 64; ++w) s += red[threadIdx.x][w];
    part[threadIdx.x * RED_MAXG + blockIdx.x] = s;
  }
}

__global__ void fro2_kernel(int m, int n, const double* A, int lda, double* part) {
  const size_t total = (size_t)m * n;
  double s2 = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const double a = A[e % m + (e / m) * (size_t)lda];
    s2 += a * a;
  }
  __shared__ double red[RED_WG / 64];
  s2 = wave_sum(s2);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < RED_WG / 64; ++w) s += red[w];
    part[blockIdx.x] = s;
  }
}

// Sum `ng` partials of each of `nq` quantities in a fixed order (one wavefront per quantity).
__global__ void finalize_kernel(const double* part, int ng, int nq, double* o0, double* o1, double* o2) {
  const int q = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (q >= nq) return;
  double s = 0.0;
  for (int g = lane; g < ng; g += 64) s += part[q * RED_MAXG + g];
  s = wave_sum(s);
  double* o = q == 0 ? o0 : (q == 1 ? o1 : o2);
  if (lane == 0 && o) *o = s;
}

int red_grid(size_t total) { return (int)std::max<size_t>(1, std::min<size_t>(RED_MAXG, (total + RED_WG * 4 - 1) / (RED_WG * 4))); }

}  // namespace

int scratch_doubles() { return 3 * RED_MAXG; }

size_t gemm_workspace_doubles(bool ta, bool tb, int m, int n, int k) {
  int nz = 0, kchunk = 0;
  if (k <= 0 || ta == tb || !splitk_plan(m, n, k, &nz, &kchunk)) return 0;
  return (size_t)nz * m * n;
}

void gemm_ws(bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda, const double* B, int ldb,
             double beta, double* C, int ldc, double* ws, size_t ws_doubles, hipStream_t st) {
  if (gemm_workspace_doubles(ta, tb, m, n, k) > ws_doubles) throw Error(SKR_EINVAL, "gemm workspace too small");
  StoreCM sc{C, ldc, alpha, beta};
  if (k <= 0) {  // C = beta C
    if (beta == 0.0) set_zero(m, n, C, ldc, st);
    else if (beta != 1.0) throw Error(SKR_ENOTSUP, "gemm with k = 0 and beta != 0, 1");
    return;
  }
  if (ta && !tb && run_gemm_splitk(m, n, k, LoadAT{A, lda}, LoadBN{B, ldb}, alpha, beta, C, ldc, ws, st)) return;
  if (!ta && tb && run_gemm_splitk(m, n, k, LoadAN{A, lda}, LoadBT{B, ldb}, alpha, beta, C, ldc, ws, st)) return;
  if (!ta && !tb) run_gemm(m, n, k, LoadAN{A, lda}, LoadBN{B, ldb}, sc, st);
  else if (ta && !tb) run_gemm(m, n, k, LoadAT{A, lda}, LoadBN{B, ldb}, sc, st);
  else if (!ta && tb) run_gemm(m, n, k, LoadAN{A, lda}, LoadBT{B, ldb}, sc, st);
  else run_gemm(m, n, k, LoadAT{A, lda}, LoadBT{B, ldb}, sc, st);
}

// Large plain products (the projected solve's order-m products and the outer-panel updates of
// the two-level Gauss-Jordan elimination) go to rocBLAS's FP64 GEMM, which runs at 64-67
// TFLOP/s for orders 4000-6000 on MI355X against 35-38 for the tile kernel above; with atomics
// disallowed its results do not depend on scheduling.  One handle per thread and device, kept
// for the life of the process (the library is thread-safe per solve, a handle is not).
namespace {
constexpr double LIB_GEMM_MIN_FLOP = 1.0e9;  // 2 m n k
constexpr int LIB_GEMM_MIN_DIM = 256;

rocblas_handle lib_handle() {
  thread_local std::map<int, rocblas_handle> handles;
  int dev = 0;
  SKR_HIP(hipGetDevice(&dev));
  auto it = handles.find(dev);
  if (it != handles.end()) return it->second;
  rocblas_handle h = nullptr;
  if (rocblas_create_handle(&h) != rocblas_status_success) throw Error(SKR_EHIP, "rocblas_create_handle failed");
  if (rocblas_set_atomics_mode(h, rocblas_atomics_not_allowed) != rocblas_status_success ||
      rocblas_set_pointer_mode(h, rocblas_pointer_mode_host) != rocblas_status_success)
    throw Error(SKR_EHIP, "rocblas handle set-up failed");
  handles.emplace(dev, h);
  return h;
}

bool lib_gemm(bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda, const double* B, int ldb,
              double beta, double* C, int ldc, hipStream_t st) {
  if (2.0 * m * n * k < LIB_GEMM_MIN_FLOP || std::min(m, n) < LIB_GEMM_MIN_DIM) return false;
  rocblas_handle h = lib_handle();
  if (rocblas_set_stream(h, st) != rocblas_status_success) throw Error(SKR_EHIP, "rocblas_set_stream failed");
  const rocblas_status rs = rocblas_dgemm(h, ta ? rocblas_operation_transpose : rocblas_operation_none,
                                          tb ? rocblas_operation_transpose : rocblas_operation_none, m, n, k, &alpha,
                                          A, lda, B, ldb, &beta, C, ldc);
  if (rs != rocblas_status_success) throw Error(SKR_EHIP, std::string("rocblas_dgemm failed: ") + rocblas_status_to_string(rs));
  return true;
}
}  // namespace

void gemm(bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda, const double* B, int ldb,
          double beta, double* C, int ldc, hipStream_t st) {
  StoreCM sc{C, ldc, alpha, beta};
  if (k <= 0) {  // C = beta C
    if (beta == 0.0) set_zero(m, n, C, ldc, st);
    else if (beta != 1.0) throw Error(SKR_ENOTSUP, "gemm with k = 0 and beta != 0, 1");
    return;
  }
  if (lib_gemm(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, st)) return;
  if (ta && !tb && run_gemm_splitk(m, n, k, LoadAT{A, lda}, LoadBN{B, ldb}, alpha, beta, C, ldc, nullptr, st)) return;
  if (!ta && tb && run_gemm_splitk(m, n, k, LoadAN{A, lda}, LoadBT{B, ldb}, alpha, beta, C, ldc, nullptr, st)) return;
  if (!ta && !tb) run_gemm(m, n, k, LoadAN{A, lda}, LoadBN{B, ldb}, sc, st);
  else if (ta && !tb) run_gemm(m, n, k, LoadAT{A, lda}, LoadBN{B, ldb}, sc, st);
  else if (!ta && tb) run_gemm(m, n, k, LoadAN{A, lda}, LoadBT{B, ldb}, sc, st);
  else run_gemm(m, n, k, LoadAT{A, lda}, LoadBT{B, ldb}, sc, st);
}

namespace {

// ---------------------------------------------------------------------------------------
// Basis products X = alpha * [U_1 ... U_nb] W + beta * X on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64).  A 16 x 16 x 4 product takes A(i, k) from lane i + 16 k, B(k, j)
// from lane j + 16 k, and leaves D(4 v + g, j) in register v of lane j + 16 g.
//
// The reduction index q = (block, column) is walked in chunks of BG_KC.  Within a group of
// 16 consecutive q, lane group g (= lane / 16) owns q = 4 g + s for the four MFMA steps
// s = 0..3, so that for r a multiple of 4 a lane's four A values are one contiguous row
// segment of one basis block (a single vector load straight from HBM, no LDS).  The W chunk
// (BG_KC x up to 128 columns) is staged in LDS, column by column with q fastest, and each
// lane reads its four B values of a step group as two 16-byte LDS loads.
// Workgroup: 8 waves x 32 rows = 256 rows of X, all (<= 128) columns of one column chunk;
// the basis is read from HBM exactly once per column chunk.
constexpr int BG_T = 512, BG_WAVES = 8, BG_RS = 2, BG_ROWS = BG_WAVES * BG_RS * 16, BG_KC = 32;
constexpr int BG_LDW = BG_KC + 2;  // padded LDS column of the W chunk (doubles)

typedef double bg_d4 __attribute__((ext_vector_type(4)));

template <typename T, bool VEC>
__device__ inline void bg_load_a(const T* U, int n, int r, int K, int i, int q, double a[4]) {
  if (i >= n || q >= K) {
#pragma unroll
    for (int s = 0; s < 4; ++s) a[s] = 0.0;
    return;
  }
  if constexpr (VEC) {  // r % 4 == 0 and q % 4 == 0: four consecutive entries of one row
    const int j = q / r, c = q - j * r;
    const T* p = U + ((size_t)j * n + i) * r + c;
    if constexpr (sizeof(T) == 4) {
      const float4 v = *reinterpret_cast<const float4*>(p);
      a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
    } else {
      const double2 v0 = *reinterpret_cast<const double2*>(p);
      const double2 v1 = *reinterpret_cast<const double2*>(p + 2);
      a[0] = v0.x; a[1] = v0.y; a[2] = v1.x; a[3] = v1.y;
    }
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int qq = q + s;
      const int j = qq / r, c = qq - j * r;
      a[s] = qq < K ? static_cast<double>(U[((size_t)j * n + i) * r + c]) : 0.0;
    }
  }
}

template <typename T, bool VEC, int NCS>
__global__ void __launch_bounds__(BG_T) basis_mfma_kernel(int n, int r, int K, int l, double alpha, const T* U,
                                                          const double* W, int ldw, double beta, double* X, int ldx) {
  __shared__ __attribute__((aligned(16))) double Ws[NCS * 16 * BG_LDW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, jl = lane & 15;
  const int row0 = blockIdx.x * BG_ROWS + wave * (BG_RS * 16);
  const int col0 = blockIdx.y * 128;
  const int ncol = min(NCS * 16, l - col0);
  bg_d4 acc[BG_RS][NCS];
#pragma unroll
  for (int a = 0; a < BG_RS; ++a)
#pragma unroll
    for (int b = 0; b < NCS; ++b) acc[a][b] = bg_d4{0.0, 0.0, 0.0, 0.0};

  // The next chunk's W entries and A values are loaded into registers while the current
  // chunk is multiplied, so neither HBM (A) nor L2 (W) latency stalls the matrix cores.
  constexpr int TG = BG_KC / 16;                           // 16-wide q groups per chunk
  constexpr int WPT = (NCS * 16 * BG_KC + BG_T - 1) / BG_T;  // staged W entries per thread
  double wreg[WPT], anext[TG][BG_RS][4];
  auto fetch = [&](int q0) {
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
      const int e = tid + BG_T * u;
      const int cc = e / BG_KC, kk = e - cc * BG_KC;
      const int q = q0 + kk;
      wreg[u] = (e < NCS * 16 * BG_KC && cc < ncol && q < K) ? W[q + (size_t)(col0 + cc) * ldw] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < TG; ++t)
#pragma unroll
      for (int rs = 0; rs < BG_RS; ++rs)
        bg_load_a<T, VEC>(U, n, r, K, row0 + rs * 16 + jl, q0 + 16 * t + 4 * g, anext[t][rs]);
  };
  fetch(0);
  for (int q0 = 0; q0 < K; q0 += BG_KC) {
    // stage W(q0 : q0 + KC, col0 : col0 + 16 NCS) with q fastest; zeros outside
    __syncthreads();
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
      const int e = tid + BG_T * u;
      if (e < NCS * 16 * BG_KC) Ws[(e / BG_KC) * BG_LDW + e % BG_KC] = wreg[u];
    }
    __syncthreads();
    double a[TG][BG_RS][4];
#pragma unroll
    for (int t = 0; t < TG; ++t)
#pragma unroll
      for (int rs = 0; rs < BG_RS; ++rs)
#pragma unroll
        for (int s = 0; s < 4; ++s) a[t][rs][s] = anext[t][rs][s];
    if (q0 + BG_KC < K) fetch(q0 + BG_KC);
#pragma unroll
    for (int t = 0; t < TG; ++t) {
#pragma unroll
      for (int cs = 0; cs < NCS; ++cs) {
        const double* wp = Ws + (cs * 16 + jl) * BG_LDW + 16 * t + 4 * g;
        const double2 b01 = *reinterpret_cast<const double2*>(wp);
        const double2 b23 = *reinterpret_cast<const double2*>(wp + 2);
        const double b[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int rs = 0; rs < BG_RS; ++rs)
            acc[rs][cs] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t][rs][s], b[s], acc[rs][cs], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int rs = 0; rs < BG_RS; ++rs)
#pragma unroll
    for (int cs = 0; cs < NCS; ++cs) {
      const int c = cs * 16 + jl;
      if (c >= ncol) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = row0 + rs * 16 + 4 * v + g;
        if (i >= n) continue;
        double* p = X + (size_t)i * ldx + col0 + c;
        *p = beta == 0.0 ? alpha * acc[rs][cs][v] : alpha * acc[rs][cs][v] + beta * *p;
      }
    }
}

template <typename T, bool VEC>
void run_basis_mfma(int n, int r, int K, int l, double alpha, const T* U, const double* W, int ldw, double beta,
                    double* X, int ldx, hipStream_t st) {
  const int ncs = ceil_div(std::min(l, 128), 16);
  dim3 grid(ceil_div(n, BG_ROWS), ceil_div(l, 128));
#define SKR_BG(N)                                                                                                   \
  hipLaunchKernelGGL((basis_mfma_kernel<T, VEC, N>), grid, dim3(BG_T), 0, st, n, r, K, l, alpha, U, W, ldw, beta, X, \
                     ldx)
  if (ncs <= 1) SKR_BG(1);
  else if (ncs <= 2) SKR_BG(2);
  else if (ncs <= 4) SKR_BG(4);
  else SKR_BG(8);
#undef SKR_BG
  check_launch("basis_mfma");
}

}  // namespace

template <typename T>
void basis_gemm(int n, int r, int nb, int l, double alpha, const T* U, const double* W, int ldw, double beta,
                double* X, int ldx, hipStream_t st) {
  if (n <= 0 || l <= 0) return;
  const int K = nb * r;
  if (K <= 0) {
    run_gemm(n, l, K, LoadBasis<T>{U, n, r}, LoadBN{W, ldw}, StoreRM{X, ldx, alpha, beta}, st);
    return;
  }
  if (r % 4 == 0) run_basis_mfma<T, true>(n, r, K, l, alpha, U, W, ldw, beta, X, ldx, st);
  else run_basis_mfma<T, false>(n, r, K, l, alpha, U, W, ldw, beta, X, ldx, st);
}
template void basis_gemm<double>(int, int, int, int, double, const double*, const double*, int, double, double*, int,
                                 hipStream_t);
template void basis_gemm<float>(int, int, int, int, double, const float*, const double*, int, double, double*, int,
                                hipStream_t);

void trsm_left_upper(int n, int nrhs, const double* T, int ldt, double* B, int ldb, hipStream_t st) {
  if (n <= 0 || nrhs <= 0) return;
  const int nblk = ceil_div(n, NB);
  for (int bi = nblk - 1; bi >= 0; --bi) {
    const int b0 = bi * NB, nb = std::min(NB, n - b0);
    hipLaunchKernelGGL(trsm_lun_diag_kernel, dim3(ceil_div(nrhs, 256)), dim3(256), 0, st, nb,
                       T + b0 + (size_t)b0 * ldt, ldt, B + b0, ldb, nrhs);
    check_launch("trsm_lun");
    if (b0 > 0)
      gemm(false, false, b0, nrhs, nb, -1.0, T + (size_t)b0 * ldt, ldt, B + b0, ldb, 1.0, B, ldb, st);
  }
}

void trsm_right_upper(int m, int n, const double* T, int ldt, double* B, int ldb, hipStream_t st) {
  if (m <= 0 || n <= 0) return;
  for (int c0 = 0; c0 < n; c0 += NB) {
    const int nb = std::min(NB, n - c0);
    hipLaunchKernelGGL(trsm_run_diag_kernel, dim3(ceil_div(m, 256)), dim3(256), 0, st, nb,
                       T + c0 + (size_t)c0 * ldt, ldt, B + (size_t)c0 * ldb, ldb, m);
    check_launch("trsm_run");
    const int rest = n - c0 - nb;
    if (rest > 0)
      gemm(false, false, m, rest, nb, -1.0, B + (size_t)c0 * ldb, ldb, T + c0 + (size_t)(c0 + nb) * ldt, ldt, 1.0,
           B + (size_t)(c0 + nb) * ldb, ldb, st);
  }
}

void copy(int m, int n, const double* A, int lda, double* B, int ldb, hipStream_t st) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(copy_kernel, dim3(std::min(4096, ceil_div((int64_t)m * n, 256))), dim3(256), 0, st, m, n, A, lda,
                     B, ldb);
  check_launch("copy");
}

void transpose(int m, int n, const double* A, int lda, double* B, int ldb, hipStream_t st) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(transpose_kernel, dim3(ceil_div(m, 32), ceil_div(n, 32)), dim3(32, 8), 0, st, m, n, A, lda, B,
                     ldb);
  check_launch("transpose");
}

void set_zero(int m, int n, double* A, int lda, hipStream_t st) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(zero_kernel, dim3(std::min(4096, ceil_div((int64_t)m * n, 256))), dim3(256), 0, st, m, n, A, lda);
  check_launch("zero");
}

void newton_combine(int m, int n, const double* mu_dev, const double* X, int ldx, const double* Y, int ldy, double* Z,
                    int ldz, double* diff_dev, double* norm_dev, double* trace_dev, double* scratch, hipStream_t st) {
  const int g = red_grid((size_t)m * n);
  hipLaunchKernelGGL(combine_kernel, dim3(g), dim3(RED_WG), 0, st, m, n, mu_dev, X, ldx, Y, ldy, Z, ldz, scratch);
  check_launch("newton_combine");
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(192), 0, st, scratch, g, 3, diff_dev, norm_dev, trace_dev);
  check_launch("finalize");
}

void fro2(int m, int n, const double* A, int lda, double* out, double* scratch, hipStream_t st) {
  const int g = red_grid((size_t)m * n);
  hipLaunchKernelGGL(fro2_kernel, dim3(g), dim3(RED_WG), 0, st, m, n, A, lda, scratch);
  check_launch("fro2");
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(64), 0, st, scratch, g, 1, out, nullptr, nullptr);
  check_launch("finalize");
}

}  // namespace dense
}  // namespace skr
