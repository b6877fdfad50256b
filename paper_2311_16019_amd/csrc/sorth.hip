// Sketch-space part of the sketched-inner-product block step: block Gram-Schmidt of w = S U~
// against the window's sketches, Cholesky QR twice of the remainder, the coefficients of the
// long update U_{d+1} = (U~ - sum_i U_i h_i) R^{-1}, and the breakdown test, all on s-row
// arrays (s = O(maxit r)).
#include "small_la.hpp"
#include "sorth.hpp"

namespace skr {
namespace {

constexpr int SKW = 3;   // window blocks
// Breakdown thresholds (not discussed in the paper; the same values as the FP64 oracle):
// the orthogonalised sketch is negligible against S U~, or its R factor is numerically
// singular.
constexpr double BREAK_NORM = 1e-12;
constexpr double BREAK_DIAG = 1e-14;

template <int R>
__device__ inline void cross_add(double (&acc)[R * R], const double (&x)[R], const double (&y)[R]) {
#pragma unroll
  for (int a = 0; a < R; ++a)
#pragma unroll
    for (int b = 0; b < R; ++b) acc[a * R + b] += x[a] * y[b];
}

// y = x M for an upper triangular M (row-major)
template <int R>
__device__ inline void times_upper(const double (&x)[R], const double* M, double (&y)[R]) {
#pragma unroll
  for (int c = 0; c < R; ++c) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k <= c; ++k) t += x[k] * M[k * R + c];
    y[c] = t;
  }
}

// The step as nw + 3 launches of SG workgroups per space, each owning a slice of the s rows;
// every launch first sums the previous launch's per-workgroup partials (fixed order, the same
// in every workgroup) and then makes one pass over its rows:
//   0         partials of ||w||^2 and of W_1^T w (of w^T w when nw = 0)
//   1 .. nw   h_j from the sums; w -= W_j h_j (stored); partials of W_{j+1}^T w, or of w^T w
//   nw + 1    R1 = chol(w^T w) and the breakdown test; partials of (w R1^{-1})^T (w R1^{-1})
//   nw + 2    R2, R = R2 R1; S U_{d+1} = w R^{-1} into the ring slot (and the whitening
//             input); workgroup 0 writes the coefficients, H and the breakdown marker
// This is the block MGS of the single-pass form, with its reductions spread over the chip.
constexpr int SG_T = 256;  // threads of a workgroup
constexpr int SG_MAX = 64; // workgroups per space
constexpr int PREC = RMAX * RMAX + 1;  // one partial record: r x r values and one scalar
// state layout (doubles)
constexpr int ST_H = 0;                        // SKW r x r coefficient blocks
constexpr int ST_N0 = ST_H + SKW * RMAX * RMAX;
constexpr int ST_R1 = ST_N0 + 1;               // r x r
constexpr int ST_R1I = ST_R1 + RMAX * RMAX;    // r x r
constexpr int ST_OK = ST_R1I + RMAX * RMAX;
constexpr int ST_SIZE = ST_OK + 1;

template <int R>
__device__ void sg_sum(const double* part, int G, double* out) {  // out[0 .. RR] (+ scalar)
  constexpr int RR = R * R;
  if ((int)threadIdx.x <= RR) {
    const int v = threadIdx.x;
    double t = 0.0;
    for (int g = 0; g < G; ++g) t += part[(size_t)g * PREC + (v == RR ? RMAX * RMAX : v)];
    out[v] = t;
  }
  __syncthreads();
}

template <int R>
__device__ void sg_write(const double (&acc)[R * R], double scal, double* part, double* red) {
  constexpr int RR = R * R;
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
#pragma unroll
  for (int p = 0; p <= RR; ++p) {
    const double v = wave_sum(p < RR ? acc[p] : scal);
    if (lane == 0) red[wv * (RR + 1) + p] = v;
  }
  __syncthreads();
  if (tid <= RR) {
    double t = 0.0;
    for (int q = 0; q < SG_T / 64; ++q) t += red[q * (RR + 1) + tid];
    part[(size_t)blockIdx.x * PREC + (tid == RR ? RMAX * RMAX : tid)] = t;
  }
}

template <int R>
__global__ void __launch_bounds__(SG_T) sorth_phase_kernel(SorthSpace a0, SorthSpace a1, int s, int nw, int i0,
                                                            int d, int phase, int G) {
  constexpr int RR = R * R;
  const SorthSpace& a = blockIdx.y ? a1 : a0;
  __shared__ double red[(SG_T / 64) * (RR + 1)];
  __shared__ double sum[RR + 1], M[RR], R2[RR], RF[RR], RFi[RR], R1i[RR];
  __shared__ int ok_sh;
  const int tid = threadIdx.x;
  const int rpg = (s + G - 1) / G, r0 = blockIdx.x * rpg, r1 = min(s, r0 + rpg);
  double* w = a.w;
  double* st = a.state;
  const double* prev = a.part + (size_t)((phase + 1) & 1) * SG_MAX * PREC;
  double* cur = a.part + (size_t)(phase & 1) * SG_MAX * PREC;
  auto ring = [&](int j) -> double* { return a.ring + (size_t)(j % a.nring) * s * R; };
  double acc[RR];
#pragma unroll
  for (int p = 0; p < RR; ++p) acc[p] = 0.0;
  double scal = 0.0;
  if (phase == 0) {
    const double* W1 = nw > 0 ? ring(i0) : w;
    for (int i = r0 + tid; i < r1; i += SG_T) {
      double x[R], y[R];
      load_row<double, R>(w, i, y);
      load_row<double, R>(W1, i, x);
      cross_add<R>(acc, x, y);
#pragma unroll
      for (int c = 0; c < R; ++c) scal += y[c] * y[c];
    }
    sg_write<R>(acc, scal, cur, red);
    return;
  }
  sg_sum<R>(prev, G, sum);
  if (phase <= nw) {
    const int j = phase - 1;  // window block W_{j} (0-based) with h_j = sum
    if (blockIdx.x == 0 && tid < RR) st[ST_H + j * RMAX * RMAX + tid] = sum[tid];
    if (blockIdx.x == 0 && tid == 0 && phase == 1) st[ST_N0] = sum[RR];
    const double* Wj = ring(i0 + j);
    const double* Wn = j + 1 < nw ? ring(i0 + j + 1) : w;
    for (int i = r0 + tid; i < r1; i += SG_T) {
      double x[R], y[R], z[R];
      load_row<double, R>(Wj, i, x);
      load_row<double, R>(w, i, y);
#pragma unroll
      for (int b = 0; b < R; ++b)
#pragma unroll
        for (int c = 0; c < R; ++c) y[b] -= x[c] * sum[c * R + b];
      store_row<double, R>(w, i, y);
      if (j + 1 < nw) {
        load_row<double, R>(Wn, i, z);
      } else {
#pragma unroll
        for (int c = 0; c < R; ++c) z[c] = y[c];
      }
      cross_add<R>(acc, z, y);
    }
    sg_write<R>(acc, 0.0, cur, red);
    return;
  }
  if (phase == nw + 1) {  // sum = w^T w of the remainder
    if (tid == 0) {
      const double n0 = nw > 0 ? st[ST_N0] : sum[RR];
      double t = 0.0;
      for (int c = 0; c < R; ++c) t += sum[c * R + c];
      double R1[RR];
      bool ok = t >= BREAK_NORM * BREAK_NORM * n0 && chol_upper(sum, R1, R);
      if (ok) inv_upper(R1, R1i, R);
      else
        for (int p = 0; p < RR; ++p) R1i[p] = 0.0;
      ok_sh = ok ? 1 : 0;
      if (blockIdx.x == 0) {
        for (int p = 0; p < RR; ++p) { st[ST_R1 + p] = ok ? R1[p] : 0.0; st[ST_R1I + p] = R1i[p]; }
        st[ST_OK] = ok ? 1.0 : 0.0;
      }
    }
    __syncthreads();
    if (ok_sh) {
      for (int i = r0 + tid; i < r1; i += SG_T) {
        double x[R], y[R];
        load_row<double, R>(w, i, x);
        times_upper<R>(x, R1i, y);
        cross_add<R>(acc, y, y);
      }
    }
    sg_write<R>(acc, 0.0, cur, red);
    return;
  }
  // phase nw + 2: sum = Gram of w R1^{-1}
  if (tid == 0) {
    bool ok = st[ST_OK] != 0.0 && chol_upper(sum, R2, R);
    if (ok) {
      double R1[RR], R2i[RR], R1iv[RR];
      for (int p = 0; p < RR; ++p) { R1[p] = st[ST_R1 + p]; R1iv[p] = st[ST_R1I + p]; }
      matmul_small(R2, R1, RF, R);
      inv_upper(R2, R2i, R);
      matmul_small(R1iv, R2i, RFi, R);
      double mx = 0.0, mn = 1e308;
      for (int p = 0; p < RR; ++p) mx = fmax(mx, fabs(RF[p]));
      for (int c = 0; c < R; ++c) mn = fmin(mn, RF[c * R + c]);
      ok = mn > BREAK_DIAG * mx;
    }
    if (!ok)
      for (int p = 0; p < RR; ++p) { RF[p] = 0.0; RFi[p] = 0.0; }
    ok_sh = ok ? 1 : 0;
  }
  __syncthreads();
  // S U_{d+1} = w R^{-1} (zero after a breakdown)
  double* out = ring(d + 1);
  for (int i = r0 + tid; i < r1; i += SG_T) {
    double x[R], y[R];
    load_row<double, R>(w, i, x);
    times_upper<R>(x, RFi, y);
    store_row<double, R>(out, i, y);
    if (a.wout) store_row<double, R>(a.wout, i, y);
  }
  if (blockIdx.x != 0) return;
  if (tid == 0 && !ok_sh) atomicMin(a.broken, d);
  // coefficients of U_{d+1} = U~ R^{-1} - sum_i U_i (h_i R^{-1}); all zero after a breakdown
  for (int e = tid; e < (nw + 1) * RR; e += SG_T) {
    const int blk = e / RR, p = e % RR, ra = p / R, cb = p % R;
    double t = 0.0;
    if (blk == 0) {
      t = RFi[p];
    } else {
      for (int c = 0; c < R; ++c) t += st[ST_H + (blk - 1) * RMAX * RMAX + ra * R + c] * RFi[c * R + cb];
    }
    a.coef[e] = t;
  }
  // h_{i0+i, d} and h_{d+1, d} = R (column-major); for the start block R goes to H itself
  for (int e = tid; e < nw * RR; e += SG_T) {
    const int i = e / RR, p = e % RR, ra = p / R, cb = p % R;
    a.H[((size_t)(i0 + i - 1) * R + ra) + ((size_t)(d - 1) * R + cb) * a.ldh] = st[ST_H + i * RMAX * RMAX + p];
  }
  for (int p = tid; p < RR; p += SG_T) {
    const int ra = p / R, cb = p % R;
    a.H[((size_t)d * R + ra) + ((size_t)(d > 0 ? d - 1 : 0) * R + cb) * a.ldh] = RF[p];
  }
}

template <int R>
void launch_r(int s, int nw, int i0, int d, const SorthSpace& a, const SorthSpace& b, int nspaces,
              hipStream_t st) {
  const int G = sorth_groups(s);
  for (int phase = 0; phase <= nw + 2; ++phase)
    hipLaunchKernelGGL((sorth_phase_kernel<R>), dim3(G, nspaces), dim3(SG_T), 0, st, a, b, s, nw, i0, d, phase, G);
}

}  // namespace

int sorth_groups(int s) { return std::max(1, std::min(SG_MAX, (s + 2 * SG_T - 1) / (2 * SG_T))); }
size_t sorth_part_doubles() { return (size_t)2 * SG_MAX * PREC; }
size_t sorth_state_doubles() { return ST_SIZE; }

void launch_sorth(int r, int s, int nw, int i0, int d, const SorthSpace& a, const SorthSpace& b, int nspaces,
                  hipStream_t st) {
  SKR_REQUIRE(nw >= 0 && nw <= SKW && (d == 0) == (nw == 0), "sketched orthogonalisation: invalid window");
  SKR_REQUIRE(nw == 0 || (i0 >= 1 && i0 + nw - 1 == d), "sketched orthogonalisation: window must end at d");
  SKR_REQUIRE(a.nring > nw && (nspaces == 1 || b.nring > nw), "sketched orthogonalisation: ring too short");
  SKR_REQUIRE(nspaces == 1 || nspaces == 2, "sketched orthogonalisation: one or two spaces");
  switch (r) {
    case 1: launch_r<1>(s, nw, i0, d, a, b, nspaces, st); break;
    case 2: launch_r<2>(s, nw, i0, d, a, b, nspaces, st); break;
    case 3: launch_r<3>(s, nw, i0, d, a, b, nspaces, st); break;
    case 4: launch_r<4>(s, nw, i0, d, a, b, nspaces, st); break;
    default: throw Error(SKR_ENOTSUP, "sketched orthogonalisation needs r <= 4");
  }
  check_launch("sorth");
}

}  // namespace skr
