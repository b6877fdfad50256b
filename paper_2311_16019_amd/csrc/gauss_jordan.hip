// Blocked Gauss-Jordan elimination with partial pivoting (FP64) for the inverses of the
// projected Newton iteration and for small dense solves.
//
// Rows are never interchanged in memory.  The pivot of column k is the row piv[k], chosen
// by largest modulus among the rows not yet used as pivots, and the eliminated column k
// stores column piv[k] of the accumulated elimination matrix E (E A = Pi, Pi(:, k) =
// e_{piv[k]}).  Afterwards A^{-1}(i, j) = S(piv[i], pos[j]) with pos the inverse of piv,
// and for extra columns B of S the solution of A X = B is X(i, c) = S(piv[i], n + c).
//
// Blocking: columns are eliminated in panels of NB.  Panel b's combined transformation E_b
// differs from the identity only in the panel's pivot rows P_b, and the panel's columns
// K_b hold E_b(:, P_b) once the panel is eliminated, so every other column j receives it as
// one rank-NB update
//     S(:, j) <- S(:, j) + S(:, K_b) a - sum_t a_t e_{P_b[t]},   a = S(P_b, j).
// Launch b runs one workgroup that applies E_{b-1} to the columns of panel b and then
// eliminates panel b in registers (one barrier per column), and many workgroups that apply
// E_{b-1} to all remaining columns: n / NB + 1 launches for the whole elimination.  The
// panel workgroup has one wavefront per SIMD up to order 1024 and two above: the
// per-column pivot search and broadcast are latency chains that more wavefronts would only
// time-share, but the panel width is bounded by the rows each thread holds in registers.
#include <climits>
#include <functional>
#include <memory>
#include <vector>
#include <type_traits>
#include <cmath>

#include "dense.hpp"

namespace skr {
namespace dense {
namespace {

constexpr int GJ_CW = 4;          // columns per strip of an update workgroup
constexpr int GJ_MAXUPD = 511;    // update workgroups per launch

struct GjArgs {
  int n, ncols, ld, b, nblk, nupd;
  // column range of this elimination: columns c0 .. c0 + npiv - 1 are eliminated, and the
  // update workgroups touch only columns c0 .. cend - 1 (the whole matrix for a one-level
  // elimination; one outer panel of a two-level elimination)
  int c0, npiv, cend;
  int want_logdet;    // the final launch sums log|pivot| over all n columns
  int wide;           // columns are 16-byte aligned (even ld, aligned S)
  double* S;
  int* piv;
  int* pos;
  int* used;
  int* info;
  double* pivabs;     // |pivot| of every column (summed as logs by the final launch)
  double* logabsdet;  // sum over all panels (may be null)
};

__global__ void gj_init_kernel(int n, int* used, int* info) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) used[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *info = 0;
}

// Pivot search keys.  64-bit: the IEEE bits of |v| (monotone for nonnegative doubles) with
// the low 24 bits replaced by 2^24 - 1 - row, so that the largest key is the largest
// modulus and, among moduli equal to 28 mantissa bits, the smallest row.  32-bit (at most
// 2048 rows): the upper word of |v| with its low 12 bits replaced by 4095 - row, which
// resolves moduli to 8 mantissa bits: the chosen pivot is within a factor 1 - 2^-8 of the
// column's largest eligible modulus, which keeps partial pivoting's growth bound up to that
// factor per column.  Rows that may not pivot get key 0; every eligible row has a nonzero
// key even when its entry is zero (the row code is at least 2048).
__device__ inline uint64_t pivot_key(double av, int row, uint64_t) {
  const uint64_t bits = (uint64_t)__double_as_longlong(av);
  return (bits & ~0xFFFFFFull) | (uint64_t)(0xFFFFFF - row);
}
__device__ inline uint32_t pivot_key(double av, int row, uint32_t) {
  const uint32_t hi = (uint32_t)((uint64_t)__double_as_longlong(av) >> 32);
  return (hi & ~0xFFFu) | (uint32_t)(0xFFF - row);
}
__device__ inline int key_row(uint64_t key) { return 0xFFFFFF - (int)(key & 0xFFFFFFull); }
__device__ inline int key_row(uint32_t key) { return 0xFFF - (int)(key & 0xFFFu); }

template <int CTRL>
__device__ inline uint64_t dpp_key(uint64_t v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
template <int CTRL>
__device__ inline uint32_t dpp_key(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
__device__ inline uint64_t lane_key(uint64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint32_t lane_key(uint32_t v, int lane) { return (uint32_t)__builtin_amdgcn_readlane((int)v, lane); }

// Maximum over the wavefront, returned uniformly: butterflies within each row of 16 lanes
// (DPP quad permutations and row rotations), then the four row maxima via readlane.
template <typename K>
__device__ inline K wave_max_key(K v) {
  K o;
  o = dpp_key<0xB1>(v);   // quad_perm [1,0,3,2]
  v = o > v ? o : v;
  o = dpp_key<0x4E>(v);   // quad_perm [2,3,0,1]
  v = o > v ? o : v;
  o = dpp_key<0x124>(v);  // row_ror:4
  v = o > v ? o : v;
  o = dpp_key<0x128>(v);  // row_ror:8
  v = o > v ? o : v;
  K m = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const K x = lane_key(v, 16 * r);
    m = x > m ? x : m;
  }
  return m;
}

// One row set per thread: row(q) = threadIdx.x + TG q.
template <int RPT, int TG>
__device__ inline int row_of(int q) { return threadIdx.x + TG * q; }

// Whether the panel workgroup stages the previous panel in LDS (at most 128 KiB).
template <int RPT, int NB, int TG>
constexpr bool gj_stage() { return TG * RPT * NB * 8 <= 128 * 1024; }

// Panel workgroup of launch b: apply E_{b-1} to the columns K_b, then eliminate K_b.
// TG threads per workgroup (one or two wavefronts per SIMD); the previous panel's columns
// are staged in LDS when they fit (STAGE), else read from global memory (L2) column by column.
template <int RPT, int NB, int TG>
__device__ __forceinline__ void panel_workgroup(const GjArgs& g, double* sl) {
  __shared__ int pl[NB];
  __shared__ int pivl[NB];
  __shared__ double amat[NB][NB];
  using Key = std::conditional_t<(TG * RPT <= 2048), uint32_t, uint64_t>;
  __shared__ Key ckey[2][(TG / 64)];
  __shared__ double crow[2][(TG / 64)][NB];
  __shared__ double red[(TG / 64)];
  const int tid = threadIdx.x, wv = tid / 64;
  if (g.b == g.nblk) {  // final launch: log|det A| = sum of log|pivot|, in a fixed order
    if (g.logabsdet && g.want_logdet) {
      double l = 0.0;
      for (int k = tid; k < g.n; k += TG) l += (g.pivabs[k] > 0.0) ? log(g.pivabs[k]) : 0.0;
      l = wave_sum(l);
      if (tid % 64 == 0) red[wv] = l;
      __syncthreads();
      if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < (TG / 64); ++w) t += red[w];
        *g.logabsdet = t;
      }
    }
    return;
  }
  const int k0 = g.c0 + g.b * NB, nbc = min(NB, g.c0 + g.npiv - k0);
  constexpr int ROWS = TG * RPT;
  const int kp0 = k0 - NB;
  constexpr bool STAGE = gj_stage<RPT, NB, TG>();
  if (STAGE && g.b > 0) {
    // The previous panel's columns S(:, K_{b-1}) (panel b-1 is always full) are staged in
    // LDS by direct global-to-LDS loads, issued before this panel's own loads so that both
    // sets are in flight together: sl[t * ROWS + row].  One instruction moves 128 rows of a
    // column (16 bytes per lane) when the columns are 16-byte aligned, else 32 rows (4 bytes
    // per lane).  A lane whose pair of rows straddles row n reads the first entry of the
    // next column, which exists (panel b-1 is not the last column), and lands in an unused
    // LDS row.
    const int lane = tid % 64;
    const bool wide = g.wide != 0;
    const int rows_per = wide ? 128 : 32, nch = (g.n + rows_per - 1) / rows_per;
    for (int e = wv; e < NB * nch; e += (TG / 64)) {
      const int t = e / nch, j = e % nch;
      const double* col = g.S + (size_t)(kp0 + t) * g.ld;
      auto* dst = (__attribute__((address_space(3))) void*)(sl + t * ROWS + rows_per * j);
      if (wide) {
        if (rows_per * j + 2 * lane < g.n) __builtin_amdgcn_global_load_lds(col + rows_per * j + 2 * lane, dst, 16, 0, 0);
      } else {
        const char* cb = reinterpret_cast<const char*>(col) + 256 * j + 4 * lane;
        if (256 * j + 4 * lane < 8 * g.n) __builtin_amdgcn_global_load_lds(cb, dst, 4, 0, 0);
      }
    }
  }
  double x[RPT][NB];
  // bit q: row_of(q) may still pivot (a bit mask in one register rather than RPT lane masks)
  using Mask = std::conditional_t<(RPT > 32), uint64_t, uint32_t>;
  Mask elig = 0;
  {
    // Every lane loads (row and column clamped into the panel, the extra values zeroed
    // afterwards), so that all loads are in flight together: conditional loads became
    // branches with a wait for each row's flag before the next row's loads.
    int usedv[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int rc = min(row_of<RPT, TG>(q), g.n - 1);
#pragma unroll
      for (int c = 0; c < NB; ++c) x[q][c] = g.S[rc + (size_t)(k0 + min(c, nbc - 1)) * g.ld];
      usedv[q] = g.used[rc];
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const bool in = row_of<RPT, TG>(q) < g.n;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (!in || c >= nbc) x[q][c] = 0.0;
      if (in && usedv[q] == 0) elig |= Mask(1) << q;
    }
  }
  if (g.b > 0) {  // the previous panel applied to this panel's columns
    if (tid < NB) pl[tid] = g.piv[kp0 + tid];
    __syncthreads();
    // amat(t, :) = S(P_{b-1}[t], K_b): the pivot rows' entries of this panel, taken from the
    // registers of the threads that own those rows
    int tp[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int row = row_of<RPT, TG>(q);
      tp[q] = -1;
      for (int t = 0; t < NB; ++t)
        if (pl[t] == row) tp[q] = t;
      if (tp[q] >= 0)
#pragma unroll
        for (int c = 0; c < NB; ++c) amat[tp[q]][c] = x[q][c];
    }
    __syncthreads();
#pragma unroll 2
    for (int t = 0; t < NB; ++t) {
      double sv[RPT];
      if constexpr (STAGE) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) sv[q] = sl[t * ROWS + row_of<RPT, TG>(q)];
      } else {  // column t of the previous panel, written by the previous launch (in L2)
        const double* col = g.S + (size_t)(kp0 + t) * g.ld;
#pragma unroll
        for (int q = 0; q < RPT; ++q) sv[q] = col[min(row_of<RPT, TG>(q), g.n - 1)];  // rows past n: unused
      }
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const double a = amat[t][c];
#pragma unroll
        for (int q = 0; q < RPT; ++q) x[q][c] += sv[q] * a;
      }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q)
      if (tp[q] >= 0)
#pragma unroll
        for (int c = 0; c < NB; ++c) x[q][c] -= amat[tp[q]][c];
  }
  // Eliminate the panel's columns: per column one pivot search (keys reduced within each
  // wavefront, then over the (TG / 64) candidates published in LDS) and one barrier; the LDS
  // records are double-buffered so the next column's writes cannot race this column's reads.
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c >= nbc) continue;  // uniform; keeps the loop fully unrollable
    const int buf = c & 1;
    Key key = 0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const Key kq = ((elig >> q) & 1) ? pivot_key(fabs(x[q][c]), row_of<RPT, TG>(q), Key{}) : Key{0};
      key = kq > key ? kq : key;
    }
    const Key wkey = wave_max_key(key);  // uniform over the wavefront
    if (wkey != 0) {
      const int wr = key_row(wkey), wq = wr / TG;  // wq uniform: scalar branches below
      if (wr % TG == tid) {
        ckey[buf][wv] = wkey;
#pragma unroll
        for (int q = 0; q < RPT; ++q)
          if (q == wq)
#pragma unroll
            for (int cc = 0; cc < NB; ++cc) crow[buf][wv][cc] = x[q][cc];
      }
    } else if (tid % 64 == 0) {
      ckey[buf][wv] = 0;
    }
    __syncthreads();
    Key gk = 0;
    int gw = 0;
#pragma unroll
    for (int w = 0; w < (TG / 64); ++w) {
      const Key kw = ckey[buf][w];
      if (kw > gk) { gk = kw; gw = w; }
    }
    const int gr = key_row(gk);
    double ps[NB];
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) ps[cc] = crow[buf][gw][cc];
    const double pv = ps[c];
    const bool ok = (pv != 0.0) && (gk != 0);
    const double inv = ok ? 1.0 / pv : 0.0;
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) ps[cc] *= inv;
    // every row takes the elimination update (no divergent branch); the pivot row's owner
    // then overwrites it with the scaled pivot row
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const double f = x[q][c];
#pragma unroll
      for (int cc = 0; cc < NB; ++cc)
        if (cc != c) x[q][cc] -= f * ps[cc];
      x[q][c] = -f * inv;
    }
    if (gr % TG == tid) {
      const int gq = gr / TG;
#pragma unroll
      for (int q = 0; q < RPT; ++q)
        if (q == gq) {
#pragma unroll
          for (int cc = 0; cc < NB; ++cc) x[q][cc] = (cc == c) ? inv : ps[cc];
          elig &= ~(Mask(1) << q);
        }
    }
    if (tid == 0) {
      pivl[c] = gr;
      g.pivabs[k0 + c] = ok ? fabs(pv) : 0.0;
      if (!ok) atomicCAS(g.info, 0, k0 + c + 1);
    }
  }
  // the barrier that publishes pivl comes before the panel's stores, so that it does not
  // wait for their completion
  __syncthreads();
  if (tid < nbc) {
    const int p = pivl[tid];
    g.piv[k0 + tid] = p;
    g.pos[p] = k0 + tid;
    g.used[p] = 1;
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int row = row_of<RPT, TG>(q);
    if (row >= g.n) continue;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nbc) g.S[row + (size_t)(k0 + c) * g.ld] = x[q][c];
  }
}

// Update workgroup of launch b >= 1: apply E_{b-1} to its strips of columns outside
// K_{b-1} and K_b.
template <int RPT, int NB, int TG>
__device__ __forceinline__ void update_workgroup(const GjArgs& g) {
  __shared__ int pl[NB];
  __shared__ double am[NB][GJ_CW];
  const int tid = threadIdx.x;
  const int kp0 = g.c0 + (g.b - 1) * NB, nbp = min(NB, g.c0 + g.npiv - kp0);
  const int kb0 = g.c0 + g.b * NB, kb1 = (g.b < g.nblk) ? min(g.c0 + g.npiv, kb0 + NB) : kb0;
  if (tid < nbp) pl[tid] = g.piv[kp0 + tid];
  __syncthreads();
  double s[RPT][NB];
  int tp[RPT];
  // clamped, unconditional loads (all in flight together), zeroed afterwards
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int rc = min(row_of<RPT, TG>(q), g.n - 1);
#pragma unroll
    for (int t = 0; t < NB; ++t) s[q][t] = g.S[rc + (size_t)(kp0 + min(t, nbp - 1)) * g.ld];
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int row = row_of<RPT, TG>(q);
#pragma unroll
    for (int t = 0; t < NB; ++t)
      if (row >= g.n || t >= nbp) s[q][t] = 0.0;
    tp[q] = -1;
    for (int t = 0; t < nbp; ++t)
      if (pl[t] == row) tp[q] = t;
  }
  auto skip = [&](int j) { return j >= g.cend || (j >= kp0 && j < kp0 + nbp) || (j >= kb0 && j < kb1); };
  const int nstrips = (g.cend - g.c0 + GJ_CW - 1) / GJ_CW;
  for (int strip = blockIdx.x - 1; strip < nstrips; strip += g.nupd) {
    const int j0 = g.c0 + strip * GJ_CW;
    for (int e = tid; e < NB * GJ_CW; e += TG) {
      const int t = e / GJ_CW, jj = e % GJ_CW, j = j0 + jj;
      am[t][jj] = (t < nbp && !skip(j)) ? g.S[pl[t] + (size_t)j * g.ld] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < GJ_CW; ++jj) {
      const int j = j0 + jj;
      if (skip(j)) continue;
      double* col = g.S + (size_t)j * g.ld;
      double acc[RPT], v[RPT];
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        acc[q] = 0.0;
        v[q] = col[min(row_of<RPT, TG>(q), g.n - 1)];  // rows past n are not stored
      }
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        const double a = am[t][jj];
#pragma unroll
        for (int q = 0; q < RPT; ++q) acc[q] += s[q][t] * a;
      }
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int row = row_of<RPT, TG>(q);
        if (row >= g.n) continue;
        double w = v[q] + acc[q];
        if (tp[q] >= 0) w -= am[tp[q]][jj];
        col[row] = w;
      }
    }
    __syncthreads();
  }
}

template <int RPT, int NB, int TG>
__global__ void __launch_bounds__(TG) gj_step_kernel(GjArgs g) {
  extern __shared__ double sl[];  // TG * RPT * NB doubles when staged, panel workgroup only
  if (blockIdx.x == 0) panel_workgroup<RPT, NB, TG>(g, sl);
  else if (g.b > 0) update_workgroup<RPT, NB, TG>(g);
}

__global__ void gj_gather_inverse_kernel(int n, const double* S, int lds, const int* piv, const int* pos, double* X,
                                         int ldx) {
  const size_t total = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    X[i + (size_t)j * ldx] = S[piv[i] + (size_t)pos[j] * lds];
  }
}

__global__ void gj_gather_solution_kernel(int n, int nrhs, const double* S, int lds, const int* piv, double* X,
                                          int ldx) {
  const size_t total = (size_t)n * nrhs;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), c = (int)(e / n);
    X[i + (size_t)c * ldx] = S[piv[i] + (size_t)(n + c) * lds];
  }
}

// t (partial over a chunk of columns) = S(:, k0:k1) b(piv(k0:k1)); rows across threads.
constexpr int GA_KC = 64;
__global__ void gj_apply_part_kernel(int n, const double* S, int lds, const int* piv, const double* b, double* part) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int k0 = blockIdx.y * GA_KC, k1 = min(n, k0 + GA_KC);
  if (r >= n) return;
  double t = 0.0;
#pragma unroll 8
  for (int k = k0; k < k1; ++k) t += S[r + (size_t)k * lds] * b[piv[k]];
  part[(size_t)blockIdx.y * n + r] = t;
}
// y(i) = sum over chunks of t(piv(i))
__global__ void gj_apply_gather_kernel(int n, int nch, const int* piv, const double* part, double* y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int r = piv[i];
  double t = 0.0;
  for (int c = 0; c < nch; ++c) t += part[(size_t)c * n + r];
  y[i] = t;
}

// Outer panel update of a two-level elimination: after the columns K_B = c0 .. c0 + w - 1
// have been eliminated (their columns hold E_B(:, P_B)), every other column j receives
//     S(:, j) <- S(:, j) + S(:, K_B) a_j - sum_t a_j(t) e_{P_B[t]},   a_j = S(P_B, j),
// as one gather of the pivot rows, two GEMMs on the matrix cores and one scatter.
__global__ void gj_gather_rows_kernel(int w, int c0, int ncols, const double* S, int ld, const int* piv, double* A) {
  const size_t total = (size_t)w * ncols;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int t = (int)(e % w), j = (int)(e / w);
    const bool inside = j >= c0 && j < c0 + w;
    A[e] = inside ? 0.0 : S[piv[c0 + t] + (size_t)j * ld];
  }
}

__global__ void gj_scatter_rows_kernel(int w, int c0, int ncols, double* S, int ld, const int* piv, const double* A) {
  const size_t total = (size_t)w * ncols;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int t = (int)(e % w), j = (int)(e / w);
    if (j >= c0 && j < c0 + w) continue;
    S[piv[c0 + t] + (size_t)j * ld] -= A[e];
  }
}

// The launches of one elimination as a list of closures, so that several eliminations on
// different streams can be enqueued interleaved: enqueued one after the other, the first
// chain's dependent launches fill its queue and hold the host until most of them have run,
// which serialises chains meant to run concurrently.
using GjPlan = std::vector<std::function<void()>>;

// One elimination range (all columns for a one-level elimination, one outer panel of a
// two-level one): launches b = 0 .. nblk of gj_step_kernel.
template <int RPT, int NB, int TG>
void plan_gj_range(GjArgs g, hipStream_t st, GjPlan& plan) {
  g.nblk = (g.npiv + NB - 1) / NB;
  g.nupd = std::min(GJ_MAXUPD, (g.cend - g.c0 + GJ_CW - 1) / GJ_CW);
  const int lds_bytes = gj_stage<RPT, NB, TG>() ? TG * RPT * NB * (int)sizeof(double) : 0;
  if (lds_bytes)
    SKR_HIP(hipFuncSetAttribute((const void*)gj_step_kernel<RPT, NB, TG>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                lds_bytes));
  for (int b = 0; b <= g.nblk; ++b) {
    g.b = b;
    const int grid = (b == 0) ? 1 : 1 + g.nupd;
    // only launches with a previous panel stage it; the update workgroups need no LDS
    const int shm = (b > 0 && b < g.nblk) ? lds_bytes : 0;
    plan.emplace_back([g, grid, shm, st]() {
      hipLaunchKernelGGL((gj_step_kernel<RPT, NB, TG>), dim3(grid), dim3(TG), shm, st, g);
      check_launch("gj_step");
    });
  }
}

// Columns per outer panel of the two-level elimination, used from GJ2_MIN_N rows on: the
// one-level panels there are a few columns wide (all n rows of a panel are held in one
// workgroup's registers) and every panel is a rank-NB update of the whole matrix, a pass
// over n x ncols doubles per few columns; the outer panels turn that traffic into GEMMs.
constexpr int GJ2_W = 256, GJ2_MIN_N = 1025;

template <int RPT, int NB, int TG>
void plan_gj(int n, int ncols, double* S, int lds, int* iws, double* dws, int* info, double* logabsdet,
             hipStream_t st, GjPlan& plan, std::vector<std::unique_ptr<DBuf<double>>>& keep) {
  GjArgs g{};
  g.n = n;
  g.ncols = ncols;
  g.ld = lds;
  g.wide = (lds % 2 == 0) && (reinterpret_cast<uintptr_t>(S) % 16 == 0);
  g.S = S;
  g.piv = iws;
  g.pos = iws + n;
  g.used = iws + 2 * (size_t)n;
  g.info = info;
  g.pivabs = dws;
  g.logabsdet = logabsdet;
  plan.emplace_back([n, used = g.used, info, st]() {
    hipLaunchKernelGGL(gj_init_kernel, dim3(std::max(1, std::min(64, ceil_div(n, 256)))), dim3(256), 0, st, n, used,
                       info);
    check_launch("gj_init");
  });
  if (n < GJ2_MIN_N) {
    g.c0 = 0;
    g.npiv = n;
    g.cend = ncols;
    g.want_logdet = 1;
    plan_gj_range<RPT, NB, TG>(g, st, plan);
    return;
  }
  static_assert(GJ2_W % NB == 0, "outer panels hold whole inner panels");
  const int wmax = std::min(GJ2_W, n);
  // pivot rows of the other columns; reused panel after panel
  keep.emplace_back(new DBuf<double>((size_t)wmax * ncols));
  double* A = keep.back()->p;
  const int* piv = g.piv;
  for (int c0 = 0; c0 < n; c0 += GJ2_W) {
    const int w = std::min(GJ2_W, n - c0);
    g.c0 = c0;
    g.npiv = w;
    g.cend = c0 + w;
    g.want_logdet = (c0 + w == n);
    plan_gj_range<RPT, NB, TG>(g, st, plan);
    if (ncols == w) continue;
    plan.emplace_back([=]() {
      const int grid = std::max(1, std::min(4096, ceil_div((int64_t)w * ncols, 256)));
      hipLaunchKernelGGL(gj_gather_rows_kernel, dim3(grid), dim3(256), 0, st, w, c0, ncols, S, lds, piv, A);
      check_launch("gj_gather_rows");
      const double* K = S + (size_t)c0 * lds;
      if (c0 > 0) gemm(false, false, n, c0, w, 1.0, K, lds, A, w, 1.0, S, lds, st);
      if (c0 + w < ncols)
        gemm(false, false, n, ncols - c0 - w, w, 1.0, K, lds, A + (size_t)(c0 + w) * w, w, 1.0,
             S + (size_t)(c0 + w) * lds, lds, st);
      hipLaunchKernelGGL(gj_scatter_rows_kernel, dim3(grid), dim3(256), 0, st, w, c0, ncols, S, lds, piv, A);
      check_launch("gj_scatter_rows");
    });
  }
}

}  // namespace

int gj_ints(int n) { return 3 * n; }
int gj_apply_doubles(int n) { return ceil_div(n, GA_KC) * n; }

void gj_apply(int n, const double* S, int lds, const int* iws, const double* b, double* y, double* work,
              hipStream_t st) {
  const int nch = ceil_div(n, GA_KC);
  hipLaunchKernelGGL(gj_apply_part_kernel, dim3(ceil_div(n, 256), nch), dim3(256), 0, st, n, S, lds, iws, b, work);
  check_launch("gj_apply");
  hipLaunchKernelGGL(gj_apply_gather_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, nch, iws, work, y);
  check_launch("gj_apply_gather");
}
int gj_doubles(int n) { return n + 1; }

namespace {
void plan_elimination(const GjJob& j, GjPlan& plan, std::vector<std::unique_ptr<DBuf<double>>>& keep) {
  const int n = j.n;
  SKR_REQUIRE(n >= 1 && j.ncols >= n && j.lds >= n, "Gauss-Jordan elimination: bad sizes");
  SKR_REQUIRE(n <= 16384, "Gauss-Jordan elimination supports n <= 16384");
  // RPT rows per thread and panel width NB with RPT * NB <= 64 register doubles.  Up to
  // order 1024 one wavefront per SIMD (256 threads); from 1025 to 8192, two (512 threads),
  // which halves the number of panels (one launch each) for the same registers per thread.
#define SKR_GJ_PLAN(RPT, NB, TG) \
  plan_gj<RPT, NB, TG>(n, j.ncols, j.S, j.lds, j.iws, j.dws, j.info, j.logabsdet, j.st, plan, keep)
  if (n <= 256) SKR_GJ_PLAN(1, 32, 256);
  else if (n <= 512) SKR_GJ_PLAN(2, 32, 256);
  else if (n <= 1024) SKR_GJ_PLAN(4, 16, 256);
  else if (n <= 2048) SKR_GJ_PLAN(4, 16, 512);
  else if (n <= 4096) SKR_GJ_PLAN(8, 8, 512);
  else if (n <= 6144) SKR_GJ_PLAN(12, 4, 512);  // no register spills, unlike 16 rows per thread
  else if (n <= 8192) SKR_GJ_PLAN(16, 4, 512);
  else SKR_GJ_PLAN(64, 1, 256);
#undef SKR_GJ_PLAN
}
}  // namespace

void gj_eliminate_many(const GjJob* jobs, int count) {
  std::vector<GjPlan> plans(count);
  std::vector<std::unique_ptr<DBuf<double>>> keep;  // released (cache-ordered) after the enqueue
  size_t len = 0;
  for (int i = 0; i < count; ++i) {
    plan_elimination(jobs[i], plans[i], keep);
    len = std::max(len, plans[i].size());
  }
  for (size_t t = 0; t < len; ++t)
    for (int i = 0; i < count; ++i)
      if (t < plans[i].size()) plans[i][t]();
}

void gj_eliminate(int n, int ncols, double* S, int lds, int* iws, double* dws, int* info, double* logabsdet,
                  hipStream_t st) {
  const GjJob j{n, ncols, S, lds, iws, dws, info, logabsdet, st};
  gj_eliminate_many(&j, 1);
}

void gj_inverse(int n, const double* S, int lds, const int* iws, double* X, int ldx, hipStream_t st) {
  const int grid = std::max(1, std::min(4096, ceil_div((int64_t)n * n, 256)));
  hipLaunchKernelGGL(gj_gather_inverse_kernel, dim3(grid), dim3(256), 0, st, n, S, lds, iws, iws + n, X, ldx);
  check_launch("gj_inverse");
}

void gj_solution(int n, int nrhs, const double* S, int lds, const int* iws, double* X, int ldx, hipStream_t st) {
  const int grid = std::max(1, std::min(4096, ceil_div((int64_t)n * nrhs, 256)));
  hipLaunchKernelGGL(gj_gather_solution_kernel, dim3(grid), dim3(256), 0, st, n, nrhs, S, lds, iws, X, ldx);
  check_launch("gj_solution");
}

}  // namespace dense
}  // namespace skr
