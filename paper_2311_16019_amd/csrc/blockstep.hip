// Block-step kernels: CSR block product, truncated block MGS, CholQR2, sparse sign sketch.
//
// Layout: every n x r block is row-major (row i holds the r entries of one grid node),
// so a wavefront of 64 consecutive rows reads 64*r contiguous elements.  Reductions over
// rows (the r x r inner products of the Gram-Schmidt step and the Gram matrices of the
// Cholesky QR) are two-stage and deterministic: each workgroup writes one partial, and
// the last workgroup to arrive sums the partials in workgroup order.
#include <climits>

#include "blockstep.hpp"
#include "small_la.hpp"

namespace skr {
namespace {


// Breakdown thresholds (not discussed in the paper; the same values as the FP64 oracle).
constexpr double BREAK_NORM = 1e-12;
constexpr double BREAK_DIAG = 1e-14;

template <typename T>
__device__ void mark_broken(const SpaceStep<T>& sp, double* sm, int r) {
  atomicMin(sp.broken, sp.step);
  set_identity(sm + SmallLayout::R1, r);
  set_identity(sm + SmallLayout::R1INV, r);
  set_identity(sm + SmallLayout::RF, r);
  set_identity(sm + SmallLayout::RFINV, r);
}

template <typename T>
__device__ bool diag_ok(const double* Rm, int r) {
  double mx = 0.0, mn = 1e308;
  for (int i = 0; i < r; ++i)
    for (int j = i; j < r; ++j) mx = fmax(mx, fabs(Rm[i * r + j]));
  for (int i = 0; i < r; ++i) mn = fmin(mn, Rm[i * r + i]);
  return mn > BREAK_DIAG * mx;
}

// Single-thread post-processing of the reduced r x r output.
template <typename T>
__device__ void post_process(const SpaceStep<T>& sp, int r) {
  double* sm = sp.small;
  const double* out = sm + SmallLayout::OUT;
  const int rr = r * r;
  if (sp.post == POST_DOT) {
    for (int i = 0; i < rr; ++i) sm[SmallLayout::COEF + i] = out[i];
    if (sp.Hblk)
      for (int a = 0; a < r; ++a)
        for (int b = 0; b < r; ++b) sp.Hblk[a + (size_t)b * sp.ldh] = out[a * r + b];
    return;
  }
  if (sp.post == POST_GRAM1) {
    double tr = 0.0;
    for (int i = 0; i < r; ++i) tr += out[i * r + i];
    const double nrm_op2 = sm[SmallLayout::NRMOP];
    bool ok = tr >= BREAK_NORM * BREAK_NORM * nrm_op2 && tr > 0.0;
    if (ok) ok = chol_upper(out, sm + SmallLayout::R1, r);
    if (!ok) {
      mark_broken(sp, sm, r);
    } else {
      inv_upper(sm + SmallLayout::R1, sm + SmallLayout::R1INV, r);
      if (r == 1) {  // normalisation is exact: no second pass
        sm[SmallLayout::RF] = sm[SmallLayout::R1];
        sm[SmallLayout::RFINV] = sm[SmallLayout::R1INV];
      }
    }
  } else {  // POST_GRAM2
    if (*sp.broken == sp.step) return;
    double* R2 = sm + SmallLayout::SIZE;  // scratch past the state (LDS in reduce_post_kernel)
    double* R2i = R2 + RMAX * RMAX;
    if (!chol_upper(out, R2, r)) {
      mark_broken(sp, sm, r);
    } else {
      inv_upper(R2, R2i, r);
      matmul_small(R2, sm + SmallLayout::R1, sm + SmallLayout::RF, r);
      matmul_small(sm + SmallLayout::R1INV, R2i, sm + SmallLayout::RFINV, r);
    }
  }
  // h_{d+1,d} = R into H (both after GRAM2, and after GRAM1 when r == 1)
  if (sp.post == POST_GRAM2 || r == 1) {
    if (*sp.broken != sp.step && !diag_ok<T>(sm + SmallLayout::RF, r)) mark_broken(sp, sm, r);
    if (sp.Hblk) {
      const bool br = (*sp.broken == sp.step);
      for (int a = 0; a < r; ++a)
        for (int b = 0; b < r; ++b)
          sp.Hblk[a + (size_t)b * sp.ldh] = br ? 0.0 : sm[SmallLayout::RF + a * r + b];
    }
  }
}

// Workgroup epilogue: write this workgroup's reduced values as its partial, value-major
// (part[i * nwg + local]) so that the reduction reads each value's partials contiguously.
// The partials are summed in a fixed order by reduce_post_kernel, launched next on the
// same stream (the kernel boundary makes them visible; no device-scope fence is needed).
template <typename T>
__device__ inline void write_partial(const SpaceStep<T>& sp, int local, const double* wg_vals, int nvals) {
  for (int i = threadIdx.x; i < nvals; i += blockDim.x) sp.part[(size_t)i * sp.nwg + local] = wg_vals[i];
}

// One workgroup per space: each wavefront sums the partials of some values (lane-strided,
// coalesced, then a fixed shuffle tree), then one thread post-processes.
template <typename T>
__global__ void __launch_bounds__(256) reduce_post_kernel(SpaceStep<T> s0, SpaceStep<T> s1, int r, int nvals) {
  const SpaceStep<T>& sp = blockIdx.x ? s1 : s0;
  double* out = sp.small + SmallLayout::OUT;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  for (int i = wv; i < nvals; i += 4) {
    const double* p = sp.part + (size_t)i * sp.nwg;
    // up to 16 partials per lane (nwg <= 1024): issue all loads, then add in order
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int w = lane + 64 * q;
      v[q] = (w < sp.nwg) ? p[w] : 0.0;
    }
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) s += v[q];
    s = wave_sum(s);
    if (lane == 0) out[i] = s;
  }
  __syncthreads();
  // post-process on an LDS copy of the small state (the single thread's dependent
  // accesses then hit LDS, not global memory), then write it back
  __shared__ double sm[SmallLayout::SIZE + 2 * RMAX * RMAX];
  for (int i = threadIdx.x; i < SmallLayout::SIZE; i += blockDim.x) sm[i] = sp.small[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    if (nvals > r * r) sm[SmallLayout::NRMOP] = sm[SmallLayout::OUT + r * r];
    SpaceStep<T> loc = sp;
    loc.small = sm;
    post_process(loc, r);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < SmallLayout::SIZE; i += blockDim.x) sp.small[i] = sm[i];
}

// Accumulate r x r products  sum_rows P[row][a] * Q[row][b]  of one tile of WG rows.
// Small r: thread-private accumulators; large r: LDS tiles redistributed over (a, b).
template <int R>
struct PairAcc {
  static constexpr bool PRIVATE = (R <= 6);
  static constexpr int NP = PRIVATE ? R * R : 1;
  double a[NP];
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < NP; ++i) a[i] = 0.0;
  }
};

template <int R>
__device__ inline void pair_accumulate(PairAcc<R>& acc, const double (&p)[R], const double (&q)[R],
                                       double* lds_p, double* lds_q) {
  if constexpr (PairAcc<R>::PRIVATE) {
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int b = 0; b < R; ++b) acc.a[a * R + b] += p[a] * q[b];
  } else {
    const int tid = threadIdx.x;
#pragma unroll
    for (int c = 0; c < R; ++c) {
      lds_p[tid * R + c] = p[c];
      lds_q[tid * R + c] = q[c];
    }
    __syncthreads();
    constexpr int RR = R * R;
    constexpr int PH = WG / RR;
    if (tid < PH * RR) {
      const int pr = tid % RR, ph = tid / RR;
      const int a = pr / R, b = pr % R;
      double s = 0.0;
      for (int j = ph; j < WG; j += PH) s += lds_p[j * R + a] * lds_q[j * R + b];
      acc.a[0] += s;
    }
    __syncthreads();
  }
}

// Reduce the pair accumulators (and one extra scalar) over the workgroup into vals[0..R*R].
template <int R>
__device__ inline void pair_reduce(PairAcc<R>& acc, double extra, double* vals, double* scratch) {
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  constexpr int NW = WG / 64;
  constexpr int RR = R * R;
  if constexpr (PairAcc<R>::PRIVATE) {
#pragma unroll
    for (int i = 0; i < RR; ++i) {
      double v = wave_sum(acc.a[i]);
      if (lane == 0) scratch[wv * (RR + 1) + i] = v;
    }
  } else {
    constexpr int PH = WG / RR;
    // thread tid holds pair tid % RR of phase tid / RR; reduce phases through LDS
    scratch[tid] = (tid < PH * RR) ? acc.a[0] : 0.0;
    __syncthreads();
    if (tid < RR) {
      double s = 0.0;
      for (int ph = 0; ph < PH; ++ph) s += scratch[ph * RR + tid];
      vals[tid] = s;
    }
    __syncthreads();
  }
  double ev = wave_sum(extra);
  if constexpr (PairAcc<R>::PRIVATE) {
    if (lane == 0) scratch[wv * (RR + 1) + RR] = ev;
    __syncthreads();
    if (tid <= RR) {
      double s = 0.0;
      for (int w = 0; w < NW; ++w) s += scratch[w * (RR + 1) + tid];
      vals[tid] = s;
    }
  } else {
    if (lane == 0) scratch[WG + wv] = ev;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < NW; ++w) s += scratch[WG + w];
      vals[RR] = s;
    }
  }
  __syncthreads();
}

template <typename T, int R>
__device__ inline void load_block_row(const T* __restrict__ p, int row, double (&x)[R]) {
  load_row<T, R>(p, row, x);
}

template <typename T, int R>
__device__ inline void store_block_row(T* __restrict__ p, int row, const double (&x)[R]) {
#pragma unroll
  for (int c = 0; c < R; ++c) p[(size_t)row * R + c] = static_cast<T>(x[c]);
}

struct WgInfo {
  int space, local, row0, row1;
};

template <typename T>
__device__ inline WgInfo wg_info(const SpaceStep<T>& s0, const SpaceStep<T>& s1) {
  const int G = s0.nwg + s1.nwg;
  const int lg = xcd_logical(blockIdx.x, G);
  WgInfo w;
  w.space = lg < s0.nwg ? 0 : 1;
  w.local = w.space ? lg - s0.nwg : lg;
  const SpaceStep<T>& sp = w.space ? s1 : s0;
  const int per = ((sp.n + sp.nwg - 1) / sp.nwg + WG - 1) / WG * WG;
  w.row0 = min(sp.n, w.local * per);
  w.row1 = min(sp.n, w.row0 + per);
  return w;
}

constexpr int lds_pair_doubles(int R) { return (R <= 6) ? 1 : WG * R; }

// -------------------------------------------------------------------------------------
// Y = Op X (+ diag o X);  dot partials W^T Y and ||Y||_F^2.
template <typename T, int R>
__global__ void __launch_bounds__(WG) spmm_dot_kernel(SpaceStep<T> s0, SpaceStep<T> s1) {
  const WgInfo wi = wg_info(s0, s1);
  const SpaceStep<T>& sp = wi.space ? s1 : s0;
  __shared__ double lds_p[lds_pair_doubles(R)], lds_q[lds_pair_doubles(R)];
  __shared__ double scratch[WG + 16 + (RMAX * RMAX + 1) * (WG / 64)];
  __shared__ double vals[RMAX * RMAX + 8];
  PairAcc<R> acc;
  acc.zero();
  double sq = 0.0;
  const CsrView<T> A = sp.A;
  for (int base = wi.row0; base < wi.row1; base += WG) {
    const int row = base + threadIdx.x;
    double y[R], w[R];
#pragma unroll
    for (int c = 0; c < R; ++c) { y[c] = 0.0; w[c] = 0.0; }
    if (row < wi.row1) {
      const int k0 = A.rowptr[row], k1 = A.rowptr[row + 1];
      for (int k = k0; k < k1; ++k) {
        const int col = A.colind[k];
        const double v = static_cast<double>(A.val[k]);
        double x[R];
        load_block_row<T, R>(sp.X, col, x);
#pragma unroll
        for (int c = 0; c < R; ++c) y[c] += v * x[c];
      }
      if (A.diag) {
        const double dg = A.diag[row];
        double x[R];
        load_block_row<T, R>(sp.X, row, x);
#pragma unroll
        for (int c = 0; c < R; ++c) y[c] += dg * x[c];
      }
      if constexpr (sizeof(T) == 4) {
        // the stored block is FP32: accumulate the products of the rounded values
#pragma unroll
        for (int c = 0; c < R; ++c) y[c] = static_cast<double>(static_cast<float>(y[c]));
      }
      store_block_row<T, R>(sp.Y, row, y);
      load_block_row<T, R>(sp.W, row, w);
#pragma unroll
      for (int c = 0; c < R; ++c) sq += y[c] * y[c];
    }
    pair_accumulate<R>(acc, w, y, lds_p, lds_q);
  }
  pair_reduce<R>(acc, sq, vals, scratch);
  write_partial(sp, wi.local, vals, R * R + 1);
}

// Y -= W * coef;  then partials of Wn^T Y (dot) or Y^T Y (Gram).
template <typename T, int R>
__global__ void __launch_bounds__(WG) axpy_reduce_kernel(SpaceStep<T> s0, SpaceStep<T> s1) {
  const WgInfo wi = wg_info(s0, s1);
  const SpaceStep<T>& sp = wi.space ? s1 : s0;
  __shared__ double lds_p[lds_pair_doubles(R)], lds_q[lds_pair_doubles(R)];
  __shared__ double scratch[WG + 16 + (RMAX * RMAX + 1) * (WG / 64)];
  __shared__ double vals[RMAX * RMAX + 8];
  __shared__ double coef[RMAX * RMAX];
  for (int i = threadIdx.x; i < R * R; i += WG) coef[i] = sp.small[SmallLayout::COEF + i];
  __syncthreads();
  PairAcc<R> acc;
  acc.zero();
  const bool gram = (sp.Wn == nullptr);
  for (int base = wi.row0; base < wi.row1; base += WG) {
    const int row = base + threadIdx.x;
    double y[R], p[R];
#pragma unroll
    for (int c = 0; c < R; ++c) { y[c] = 0.0; p[c] = 0.0; }
    if (row < wi.row1) {
      double w[R];
      load_block_row<T, R>(sp.Y, row, y);
      load_block_row<T, R>(sp.W, row, w);
#pragma unroll
      for (int c = 0; c < R; ++c) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < R; ++a) s += w[a] * coef[a * R + c];
        y[c] -= s;
      }
      if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int c = 0; c < R; ++c) y[c] = static_cast<double>(static_cast<float>(y[c]));
      }
      store_block_row<T, R>(sp.Y, row, y);
      if (gram) {
#pragma unroll
        for (int c = 0; c < R; ++c) p[c] = y[c];
      } else {
        load_block_row<T, R>(sp.Wn, row, p);
      }
    }
    pair_accumulate<R>(acc, p, y, lds_p, lds_q);
  }
  pair_reduce<R>(acc, 0.0, vals, scratch);
  write_partial(sp, wi.local, vals, R * R);
}

// Gram matrix of Y R1^{-1} (second Cholesky QR pass); Y is not modified.
template <typename T, int R>
__global__ void __launch_bounds__(WG) gram2_kernel(SpaceStep<T> s0, SpaceStep<T> s1) {
  const WgInfo wi = wg_info(s0, s1);
  const SpaceStep<T>& sp = wi.space ? s1 : s0;
  __shared__ double lds_p[lds_pair_doubles(R)], lds_q[lds_pair_doubles(R)];
  __shared__ double scratch[WG + 16 + (RMAX * RMAX + 1) * (WG / 64)];
  __shared__ double vals[RMAX * RMAX + 8];
  __shared__ double rinv[RMAX * RMAX];
  for (int i = threadIdx.x; i < R * R; i += WG) rinv[i] = sp.small[SmallLayout::R1INV + i];
  __syncthreads();
  PairAcc<R> acc;
  acc.zero();
  for (int base = wi.row0; base < wi.row1; base += WG) {
    const int row = base + threadIdx.x;
    double z[R];
#pragma unroll
    for (int c = 0; c < R; ++c) z[c] = 0.0;
    if (row < wi.row1) {
      double y[R];
      load_block_row<T, R>(sp.Y, row, y);
#pragma unroll
      for (int c = 0; c < R; ++c) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a <= c; ++a) s += y[a] * rinv[a * R + c];
        z[c] = s;
      }
    }
    pair_accumulate<R>(acc, z, z, lds_p, lds_q);
  }
  pair_reduce<R>(acc, 0.0, vals, scratch);
  write_partial(sp, wi.local, vals, R * R);
}

// Unew = Y R^{-1}.
template <typename T, int R>
__global__ void __launch_bounds__(WG) normalize_kernel(SpaceStep<T> s0, SpaceStep<T> s1) {
  const WgInfo wi = wg_info(s0, s1);
  const SpaceStep<T>& sp = wi.space ? s1 : s0;
  __shared__ double rinv[RMAX * RMAX];
  for (int i = threadIdx.x; i < R * R; i += WG) rinv[i] = sp.small[SmallLayout::RFINV + i];
  __syncthreads();
  for (int base = wi.row0; base < wi.row1; base += WG) {
    const int row = base + threadIdx.x;
    if (row >= wi.row1) continue;
    double y[R], z[R];
    load_block_row<T, R>(sp.Y, row, y);
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a <= c; ++a) s += y[a] * rinv[a * R + c];
      z[c] = s;
    }
    store_block_row<T, R>(sp.Unew, row, z);
  }
}

// ------------------------------------------------------------------ sparse sign sketch
__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void build_table_kernel(uint16_t* tab, int n, int zeta, int b, uint64_t seed) {
  const int64_t total = (int64_t)n * zeta;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / zeta), t = (int)(e % zeta);
    const uint64_t idx = (uint64_t)zeta * (uint64_t)j + (uint64_t)t + 1ull;
    const uint64_t z = mix64(seed + idx * 0x9E3779B97F4A7C15ull);
    const uint32_t bucket = (uint32_t)(((z >> 32) * (uint64_t)b) >> 32);
    tab[(size_t)t * n + j] = (uint16_t)(bucket | ((uint32_t)(z & 1ull) << 15));
  }
}

constexpr int SK_WG = 1024;

// One workgroup per (chunk of rows, copy t): scatter-add signed rows into an LDS copy of
// the t-th band of the sketch (b x rc values, columns [c0, c0+rc)), then write it out.
// The LDS copy is column-major (acc[c * b + bucket]) so that the 64 random buckets of a
// wavefront's atomics spread over all LDS banks rather than over the few banks that one
// column of a row-major copy maps to.
//
// The band is accumulated in 64-bit fixed point (value x 2^SK_FRAC, rounded to the nearest
// integer): integer addition is associative, so the order in which the atomics land does
// not change the result and every run of a solve produces the same sketch bit for bit.
// The sketched blocks have columns of about unit norm (|entries| <= 2 for the stored
// blocks of the two-pass step, whose pending factor is near the identity), so a bucket's
// sum over one chunk of rows stays far below the 2^(63 - SK_FRAC) = 2048 the format holds;
// the rounding is 2^-53 absolute per contribution, below the FP64 rounding of the entries
// of a unit-norm sketch column.
constexpr int SK_FRAC = 52;

template <typename T, int R>
__global__ void __launch_bounds__(SK_WG) sketch_kernel(SketchSpace<T> a0, SketchSpace<T> a1, int s, int zeta,
                                                        int c0, int rc) {
  extern __shared__ unsigned long long acc[];
  constexpr double SCALE = (double)(1ull << SK_FRAC);
  const int b = s / zeta;
  const int G = zeta * (a0.nchunk + a1.nchunk);
  const int lg = xcd_logical(blockIdx.x, G);
  const int sp_id = lg < zeta * a0.nchunk ? 0 : 1;
  const SketchSpace<T>& sp = sp_id ? a1 : a0;
  const int idx = sp_id ? lg - zeta * a0.nchunk : lg;
  const int t = idx % zeta, chunk = idx / zeta;
  for (int i = threadIdx.x; i < b * rc; i += SK_WG) acc[i] = 0ull;
  __syncthreads();
  const int per = (sp.n + sp.nchunk - 1) / sp.nchunk;
  const int r0 = min(sp.n, chunk * per), r1 = min(sp.n, r0 + per);
  const uint16_t* tab = sp.tab + (size_t)t * sp.n;
  for (int row = r0 + threadIdx.x; row < r1; row += SK_WG) {
    const uint32_t e = tab[row];
    const int bucket = (int)(e & 0x7FFFu);
    const double sg = (e & 0x8000u) ? -1.0 : 1.0;
    double x[R];
    load_block_row<T, R>(sp.U, row, x);
    if (sp.fixed) {
#pragma unroll
      for (int c = 0; c < R; ++c)
        if (c >= c0 && c < c0 + rc) {
          const long long q = __double2ll_rn(sg * x[c] * SCALE);  // two's complement: wraps exactly
          atomicAdd(&acc[(c - c0) * b + bucket], (unsigned long long)q);
        }
    } else {
      double* accd = reinterpret_cast<double*>(acc);
#pragma unroll
      for (int c = 0; c < R; ++c)
        if (c >= c0 && c < c0 + rc) atomicAdd(&accd[(c - c0) * b + bucket], sg * x[c]);
    }
  }
  __syncthreads();
  double* out = sp.part + ((size_t)chunk * s + (size_t)t * b) * R;
  const double* accd = reinterpret_cast<const double*>(acc);
  for (int i = threadIdx.x; i < b * rc; i += SK_WG) {
    const int bk = i / rc, c = i % rc;
    out[(size_t)bk * R + c0 + c] =
        sp.fixed ? (double)(long long)acc[c * b + bk] / SCALE : accd[c * b + bk];
  }
}

// w = (sum over chunks of the partial sketches) P / sqrt(zeta), P (r x r row-major) the
// block's pending right factor or null for the identity.  Each thread sums one entry's
// chunks (all loads in flight), then the rows of the workgroup are multiplied by P in LDS.
constexpr int SK_CHMAX = 32;  // sketch_chunks() never exceeds this
template <typename T>
__global__ void __launch_bounds__(256) sketch_reduce_kernel(SketchSpace<T> a0, SketchSpace<T> a1, const double* P0,
                                                            const double* P1, int s, int r, double scale) {
  const SketchSpace<T>& sp = blockIdx.y ? a1 : a0;
  const double* P = blockIdx.y ? P1 : P0;
  __shared__ double sh[256];
  const size_t total = (size_t)s * r;
  const int rows_per = 256 / r, lr = threadIdx.x / r, c = threadIdx.x % r;
  for (int row0 = blockIdx.x * rows_per; row0 < s; row0 += gridDim.x * rows_per) {
    const int row = row0 + lr;
    const bool mine = lr < rows_per && row < s;
    double t = 0.0;
    if (mine) {
      double v[SK_CHMAX];
#pragma unroll
      for (int ch = 0; ch < SK_CHMAX; ++ch) v[ch] = (ch < sp.nchunk) ? sp.part[(size_t)ch * total + (size_t)row * r + c] : 0.0;
#pragma unroll
      for (int ch = 0; ch < SK_CHMAX; ++ch) t += v[ch];
    }
    sh[threadIdx.x] = t;
    __syncthreads();
    if (mine) {
      double o = t;
      if (P) {
        o = 0.0;
        for (int k = 0; k < r; ++k) o += sh[lr * r + k] * P[k * r + c];
      }
      sp.w[(size_t)row * r + c] = o * scale;
    }
    __syncthreads();
  }
}

template <typename T>
int grid_of(const SpaceStep<T>& a, const SpaceStep<T>& b) {
  return a.nwg + b.nwg;
}

}  // namespace

// Row chunks per space: one workgroup per (chunk, copy); a single space (the Lyapunov
// solve) takes twice as many so that the launch still fills the GPU.
int sketch_chunks(int n, int nspaces) {
  return std::max(1, std::min(nspaces == 1 ? 32 : 16, ceil_div(n, 4 * SK_WG)));
}

#define SKR_DISPATCH_R(r, ...)                                             \
  switch (r) {                                                             \
    case 1: { constexpr int RR_ = 1; __VA_ARGS__; } break;                 \
    case 2: { constexpr int RR_ = 2; __VA_ARGS__; } break;                 \
    case 3: { constexpr int RR_ = 3; __VA_ARGS__; } break;                 \
    case 4: { constexpr int RR_ = 4; __VA_ARGS__; } break;                 \
    case 5: { constexpr int RR_ = 5; __VA_ARGS__; } break;                 \
    case 6: { constexpr int RR_ = 6; __VA_ARGS__; } break;                 \
    case 7: { constexpr int RR_ = 7; __VA_ARGS__; } break;                 \
    case 8: { constexpr int RR_ = 8; __VA_ARGS__; } break;                 \
    case 9: { constexpr int RR_ = 9; __VA_ARGS__; } break;                 \
    case 10: { constexpr int RR_ = 10; __VA_ARGS__; } break;               \
    case 11: { constexpr int RR_ = 11; __VA_ARGS__; } break;               \
    case 12: { constexpr int RR_ = 12; __VA_ARGS__; } break;               \
    case 13: { constexpr int RR_ = 13; __VA_ARGS__; } break;               \
    case 14: { constexpr int RR_ = 14; __VA_ARGS__; } break;               \
    case 15: { constexpr int RR_ = 15; __VA_ARGS__; } break;               \
    case 16: { constexpr int RR_ = 16; __VA_ARGS__; } break;               \
    default: throw Error(SKR_ENOTSUP, "block size r must be in [1, 16]");  \
  }

template <typename T>
void launch_reduce_post(int r, int nvals, const SpaceStep<T>& s0, const SpaceStep<T>& s1, hipStream_t st) {
  hipLaunchKernelGGL((reduce_post_kernel<T>), dim3(2), dim3(256), 0, st, s0, s1, r, nvals);
  check_launch("reduce_post");
}

template <typename T>
void launch_spmm_dot(int r, const SpaceStep<T>& s0, const SpaceStep<T>& s1, hipStream_t st) {
  SKR_DISPATCH_R(r, hipLaunchKernelGGL((spmm_dot_kernel<T, RR_>), dim3(grid_of(s0, s1)), dim3(WG), 0, st, s0, s1));
  check_launch("spmm_dot");
  launch_reduce_post(r, r * r + 1, s0, s1, st);
}
template <typename T>
void launch_axpy_reduce(int r, const SpaceStep<T>& s0, const SpaceStep<T>& s1, hipStream_t st) {
  SKR_DISPATCH_R(r, hipLaunchKernelGGL((axpy_reduce_kernel<T, RR_>), dim3(grid_of(s0, s1)), dim3(WG), 0, st, s0, s1));
  check_launch("axpy_reduce");
  launch_reduce_post(r, r * r, s0, s1, st);
}
template <typename T>
void launch_gram2(int r, const SpaceStep<T>& s0, const SpaceStep<T>& s1, hipStream_t st) {
  SKR_DISPATCH_R(r, hipLaunchKernelGGL((gram2_kernel<T, RR_>), dim3(grid_of(s0, s1)), dim3(WG), 0, st, s0, s1));
  check_launch("gram2");
  launch_reduce_post(r, r * r, s0, s1, st);
}
template <typename T>
void launch_normalize(int r, const SpaceStep<T>& s0, const SpaceStep<T>& s1, hipStream_t st) {
  SKR_DISPATCH_R(r, hipLaunchKernelGGL((normalize_kernel<T, RR_>), dim3(grid_of(s0, s1)), dim3(WG), 0, st, s0, s1));
  check_launch("normalize");
}

void launch_build_sketch_table(uint16_t* tab, int n, int zeta, int b, uint64_t seed, hipStream_t st) {
  SKR_REQUIRE(b >= 1 && b <= 32768, "sketch rows per band s/zeta must be in [1, 32768]");
  const int64_t total = (int64_t)n * zeta;
  const int grid = (int)std::min<int64_t>(4096, (total + 255) / 256);
  hipLaunchKernelGGL(build_table_kernel, dim3(grid), dim3(256), 0, st, tab, n, zeta, b, seed);
  check_launch("build_sketch_table");
}

template <typename T>
void launch_sketch_pending(int r, int s, int zeta, const SketchSpace<T>& a, const SketchSpace<T>& b,
                           const double* Pa, const double* Pb, size_t lds_limit, hipStream_t st) {
  const int bands = s / zeta;
  int rc = (int)std::min<size_t>((size_t)r, lds_limit / (sizeof(double) * (size_t)bands));
  SKR_REQUIRE(rc >= 1, "sketch band does not fit in LDS");
  const int grid = zeta * (a.nchunk + b.nchunk);
  for (int c0 = 0; c0 < r; c0 += rc) {
    const int cn = std::min(rc, r - c0);
    const size_t lds = sizeof(double) * (size_t)bands * cn;
    SKR_DISPATCH_R(r, {
      auto kern = sketch_kernel<T, RR_>;
      if (lds > 65536) SKR_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      hipLaunchKernelGGL(kern, dim3(grid), dim3(SK_WG), lds, st, a, b, s, zeta, c0, cn);
    });
    check_launch("sketch");
  }
  SKR_REQUIRE(a.nchunk <= SK_CHMAX && b.nchunk <= SK_CHMAX, "too many sketch chunks");
  hipLaunchKernelGGL(sketch_reduce_kernel<T>, dim3(std::min(1024, ceil_div((int64_t)s * r, 256)), 2), dim3(256), 0, st, a,
                     b, Pa, Pb, s, r, 1.0 / sqrt((double)zeta));
  check_launch("sketch_reduce");
}

template <typename T>
void launch_sketch(int r, int s, int zeta, const SketchSpace<T>& a, const SketchSpace<T>& b, size_t lds_limit,
                   hipStream_t st) {
  launch_sketch_pending<T>(r, s, zeta, a, b, nullptr, nullptr, lds_limit, st);
}

#define SKR_INST(T)                                                                                  \
  template void launch_spmm_dot<T>(int, const SpaceStep<T>&, const SpaceStep<T>&, hipStream_t);     \
  template void launch_axpy_reduce<T>(int, const SpaceStep<T>&, const SpaceStep<T>&, hipStream_t);  \
  template void launch_gram2<T>(int, const SpaceStep<T>&, const SpaceStep<T>&, hipStream_t);        \
  template void launch_normalize<T>(int, const SpaceStep<T>&, const SpaceStep<T>&, hipStream_t);    \
  template void launch_sketch<T>(int, int, int, const SketchSpace<T>&, const SketchSpace<T>&, size_t, hipStream_t); \
  template void launch_sketch_pending<T>(int, int, int, const SketchSpace<T>&, const SketchSpace<T>&, const double*, \
                                         const double*, size_t, hipStream_t);
SKR_INST(double)
SKR_INST(float)

}  // namespace skr
