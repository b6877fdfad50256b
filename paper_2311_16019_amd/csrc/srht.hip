// Subsampled randomized DCT embedding on the device: stage 1 (length-N1 DFTs in LDS, one
// workgroup per tile of consecutive b < N2), stage 2 (the sampled outputs, one workgroup per
// residue k1 = k mod N1, one wavefront per sampled frequency),
// and the pending right factor.  Host side: the factorisation n = N1 N2, N1 = P Q and the
// sampled rows, cached per (n, s, seed).
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "small_la.hpp"
#include "srht.hpp"

namespace skr {
namespace {

constexpr int S1T = 512;      // threads of a stage-1 workgroup
constexpr int S2T = 1024;     // threads of a stage-2 workgroup (one wavefront per sample)
constexpr int CC2MAX = 8;     // columns per stage-2 chunk
constexpr int PQMAX = 64;     // largest direct DFT length of stage 1
constexpr int N1MAX = 3072;   // stage-1 sequence length (LDS: tables + one column)
constexpr int N2MAX = 4096;   // stage-2 sequence length (LDS: twiddles + one column)
constexpr uint64_t GOLDEN = 0x9E3779B97F4A7C15ull;
constexpr int LD = 8;         // global loads in flight per thread in the staging loops
constexpr int S1B = 8;        // widest tile of b per stage-1 workgroup
constexpr size_t S1_SHARE = 52 * 1024;  // stage-1 LDS that leaves room for three workgroups per CU
constexpr size_t S2_SHARE = 80 * 1024;  // stage-2 LDS that leaves room for two workgroups per CU
constexpr double SAMPLE_W = 4.0;        // cost of a sampled-stage multiply-add against a stage-1 one

__host__ __device__ inline uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// exp(-2 pi i t / N) into (re, im), 0 <= t < N
__device__ inline void twiddle(int64_t t, int64_t N, double& re, double& im) {
  double sn, cs;
  sincospi(2.0 * (double)t / (double)N, &sn, &cs);
  re = cs;
  im = -sn;
}

// One workgroup per tile of B consecutive b: the B cc sequences of a column chunk are
// transformed together, so that the Z entries of a tile (consecutive b for one k1) are
// written by one workgroup.  Complex arrays in LDS are planar (real and imaginary parts in
// separate arrays) and sequences are laid out with an odd stride, to spread LDS banks.
template <typename T>
__global__ void __launch_bounds__(S1T) srht_stage1_kernel(SrhtSpace<T> a0, SrhtSpace<T> a1, int r, int cc, int B) {
  const SrhtSpace<T>& a = blockIdx.y ? a1 : a0;
  const int N1 = a.N1, N2 = a.N2, P = a.P, Q = a.Q;
  const int L = N1 | 1;                                   // sequence stride in LDS (odd)
  const int b0 = xcd_logical(blockIdx.x, gridDim.x) * B;  // neighbouring tiles share cache lines of U
  if (a.n == 0 || b0 >= N2) return;                       // uniform over the workgroup
  const int nb = min(B, N2 - b0);
  const int tid = threadIdx.x;
  extern __shared__ double sm[];
  double* wN1r = sm;                 // N1 each: w_N1^j
  double* wN1i = wN1r + N1;
  double* wPr = wN1i + N1;           // P each
  double* wPi = wPr + P;
  double* wQr = wPi + P;             // Q each
  double* wQi = wQr + Q;
  double* bPr = wQi + Q;             // B P each: w_n^{b k1a}
  double* bPi = bPr + B * P;
  double* bQr = bPi + B * P;         // B Q each: w_n^{b P k1b}
  double* bQi = bQr + B * Q;
  double* Tr = bQi + B * Q;          // B cc L each
  double* Ti = Tr + B * cc * L;
  double* xs = Ti + B * cc * L;      // B cc L
  const int64_t n = a.n, h = (n + 1) / 2;
  for (int j = tid; j < N1; j += S1T) twiddle(j, N1, wN1r[j], wN1i[j]);
  for (int j = tid; j < P; j += S1T) twiddle(j, P, wPr[j], wPi[j]);
  for (int j = tid; j < Q; j += S1T) twiddle(j, Q, wQr[j], wQi[j]);
  for (int e = tid; e < nb * P; e += S1T) {
    const int bi = e / P, j = e % P;
    twiddle(((int64_t)(b0 + bi) * j) % n, n, bPr[e], bPi[e]);
  }
  for (int e = tid; e < nb * Q; e += S1T) {
    const int bi = e / Q, j = e % Q;
    twiddle(((int64_t)(b0 + bi) * P * j) % n, n, bQr[e], bQi[e]);
  }
  for (int c0 = 0; c0 < r; c0 += cc) {
    const int ncol = min(cc, r - c0);
    const int nseq = nb * ncol;  // sequence q = bi ncol + cl
    __syncthreads();             // tables written, previous chunk consumed
    // v[N2 a + b] with v the even entries of y = E x followed by the odd ones reversed;
    // LD loads per thread are issued before any of them is used
    for (int e0 = 0; e0 < N1 * nseq; e0 += LD * S1T) {
      double val[LD];
      int64_t rows[LD];
#pragma unroll
      for (int u = 0; u < LD; ++u) {
        const int e = e0 + u * S1T + tid;
        const int aa = e / nseq, q = e % nseq, bi = q / ncol, cl = q % ncol;
        const int64_t m = (int64_t)N2 * aa + b0 + bi;
        rows[u] = m < h ? 2 * m : 2 * (n - 1 - m) + 1;
        val[u] = e < N1 * nseq ? static_cast<double>(a.U[rows[u] * r + c0 + cl]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < LD; ++u) {
        const int e = e0 + u * S1T + tid;
        if (e < N1 * nseq) {
          const int aa = e / nseq, q = e % nseq;
          const double sg = (splitmix_mix(a.seed + (uint64_t)(rows[u] + 1) * GOLDEN) & 1ull) ? -1.0 : 1.0;
          xs[q * L + aa] = sg * val[u];
        }
      }
    }
    __syncthreads();
    // P-point DFTs over a1 (a = Q a1 + a2), times w_N1^{a2 k1a}
    for (int e = tid; e < nseq * N1; e += S1T) {
      const int q = e / N1, rem = e % N1, k1a = rem / Q, a2 = rem % Q;
      const double* xc = xs + q * L + a2;
      double re = 0.0, im = 0.0;
      int idx = 0;
#pragma unroll 4
      for (int a1 = 0; a1 < P; ++a1) {
        const double x = xc[Q * a1];
        re += x * wPr[idx];
        im += x * wPi[idx];
        idx += k1a;
        if (idx >= P) idx -= P;
      }
      const int t = a2 * k1a;  // <= (Q - 1)(P - 1) < N1
      const double tr = wN1r[t], ti = wN1i[t];
      Tr[q * L + rem] = re * tr - im * ti;
      Ti[q * L + rem] = re * ti + im * tr;
    }
    __syncthreads();
    // Q-point DFTs over a2: k1 = k1a + P k1b; times w_n^{b k1}
    for (int e = tid; e < nseq * N1; e += S1T) {
      const int q = e / N1, rem = e % N1, k1a = rem / Q, k1b = rem % Q, bi = q / ncol, cl = q % ncol;
      const int base = q * L + k1a * Q;
      double re = 0.0, im = 0.0;
      int idx = 0;
#pragma unroll 4
      for (int a2 = 0; a2 < Q; ++a2) {
        const double xr = Tr[base + a2], xi = Ti[base + a2];
        const double wr = wQr[idx], wi = wQi[idx];
        re += xr * wr - xi * wi;
        im += xr * wi + xi * wr;
        idx += k1b;
        if (idx >= Q) idx -= Q;
      }
      const int k1 = k1a + P * k1b;
      // w_n^{b k1} = w_n^{b k1a} w_n^{b P k1b}
      const double ur = bPr[bi * P + k1a], ui = bPi[bi * P + k1a];
      const double vr = bQr[bi * Q + k1b], vi = bQi[bi * Q + k1b];
      const double tr = ur * vr - ui * vi, ti = ur * vi + ui * vr;
      double* z = a.Z + 2 * (((int64_t)(c0 + cl) * N1 + k1) * N2 + b0 + bi);  // [column][k1][b]
      z[0] = re * tr - im * ti;
      z[1] = re * ti + im * tr;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(S2T) srht_stage2_kernel(SrhtSpace<T> a0, SrhtSpace<T> a1, int r, int s, int cc) {
  const SrhtSpace<T>& a = blockIdx.y ? a1 : a0;
  const int N1 = a.N1, N2 = a.N2;
  const int k1 = blockIdx.x;
  if (a.n == 0 || k1 >= N1) return;
  const int j0 = a.soff[k1], j1 = a.soff[k1 + 1];
  if (j0 == j1) return;  // uniform: no sampled frequency has this residue
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  extern __shared__ double sm[];
  double* Zr = sm;               // cc N2 each
  double* Zi = Zr + cc * N2;
  const double scale = sqrt(2.0 / (double)s);  // sqrt(n / s) times the DCT's sqrt(2 / n)
  for (int c0 = 0; c0 < r; c0 += cc) {
    const int ncol = min(cc, r - c0);
    __syncthreads();
    for (int e0 = 0; e0 < ncol * N2; e0 += LD * S2T) {
      double zr[LD], zi[LD];
#pragma unroll
      for (int u = 0; u < LD; ++u) {
        const int e = e0 + u * S2T + tid;
        const int cl = e / N2, bb = e % N2;
        zr[u] = zi[u] = 0.0;
        if (e < ncol * N2) {
          const double* z = a.Z + 2 * (((int64_t)(c0 + cl) * N1 + k1) * N2 + bb);
          zr[u] = z[0];
          zi[u] = z[1];
        }
      }
#pragma unroll
      for (int u = 0; u < LD; ++u) {
        const int e = e0 + u * S2T + tid;
        if (e < ncol * N2) {
          Zr[e] = zr[u];
          Zi[e] = zi[u];
        }
      }
    }
    __syncthreads();
    // one wavefront per sample: V_k = sum_b Z[k1][b] w_N2^{b k2}, reduced within the wavefront;
    // lane l takes b = l, l + 64, .., its twiddle advanced by the factor w_N2^{64 k2}
    for (int j = j0 + wv; j < j1; j += S2T / 64) {
      const int i = a.samp[2 * j], k = a.samp[2 * j + 1];
      const unsigned k2 = (unsigned)(k / N1);  // < N2 <= 4096, so 64 k2 fits 32 bits
      double acc[2 * CC2MAX];
#pragma unroll
      for (int v = 0; v < 2 * CC2MAX; ++v) acc[v] = 0.0;
      const int t0 = (int)(((unsigned)lane * k2) % (unsigned)N2), ts = (int)((64u * k2) % (unsigned)N2);
      double wr, wi, sr, si;
      twiddle(t0, N2, wr, wi);
      twiddle(ts, N2, sr, si);
      for (int bb = lane; bb < N2; bb += 64) {
#pragma unroll
        for (int cl = 0; cl < CC2MAX; ++cl) {
          if (cl < ncol) {
            const double zr = Zr[cl * N2 + bb], zi = Zi[cl * N2 + bb];
            acc[2 * cl] += zr * wr - zi * wi;
            acc[2 * cl + 1] += zr * wi + zi * wr;
          }
        }
        const double nr = wr * sr - wi * si;
        wi = wr * si + wi * sr;
        wr = nr;
      }
      double sn, cs;  // DCT2_k = Re(exp(-i pi k / (2n)) V_k)
      sincospi((double)k / (2.0 * (double)a.n), &sn, &cs);
      const double ck = (k == 0) ? 0.70710678118654752440 : 1.0;
#pragma unroll
      for (int cl = 0; cl < CC2MAX; ++cl) {
        if (cl < ncol) {  // uniform
          const double vr = wave_sum(acc[2 * cl]), vi = wave_sum(acc[2 * cl + 1]);
          if (lane == 0) a.wraw[(int64_t)i * r + c0 + cl] = scale * ck * (vr * cs + vi * sn);
        }
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) srht_pending_kernel(SrhtSpace<T> a0, SrhtSpace<T> a1, int r, int s) {
  const SrhtSpace<T>& a = blockIdx.y ? a1 : a0;
  if (a.n == 0 || !a.Pend) return;
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < (int64_t)s * r; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / r;
    const int c = (int)(e % r);
    double t = 0.0;
    for (int k = 0; k < r; ++k) t += a.wraw[i * r + k] * a.Pend[k * r + c];
    a.w[e] = t;
  }
}

struct PlanKey {
  int64_t n;
  int s;
  uint64_t seed;
  bool operator<(const PlanKey& o) const { return std::tie(n, s, seed) < std::tie(o.n, o.s, o.seed); }
};

}  // namespace

SrhtPlan srht_plan(int64_t n, int s, uint64_t seed) {
  static std::mutex mu;
  static std::map<PlanKey, SrhtPlan> cache;
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find({n, s, seed});
    if (it != cache.end()) return it->second;
  }
  SKR_REQUIRE(n >= 1 && n < (int64_t(1) << 31), "DCT embedding: n out of range");
  SKR_REQUIRE(s >= 1 && s <= n, "DCT embedding: s must be in [1, n] (distinct sampled rows)");
  SrhtPlan pl;
  pl.n = n;
  pl.s = s;
  pl.seed = seed;
  // n = N1 N2, N1 = P Q: the cheapest split by n (P + Q) + SAMPLE_W s N2 multiply-adds per
  // column (a multiply-add of the sampled stage weighted by its measured relative cost)
  double best = -1.0;
  for (int64_t N1 = 1; N1 <= std::min<int64_t>(n, N1MAX); ++N1) {
    if (n % N1) continue;
    const int64_t N2 = n / N1;
    if (N2 > N2MAX) continue;
    int bp = 0, bq = 0;
    for (int P = 1; P <= PQMAX; ++P)
      if (N1 % P == 0 && N1 / P <= PQMAX && (bp == 0 || P + N1 / P < bp + bq)) {
        bp = P;
        bq = (int)(N1 / P);
      }
    if (bp == 0) continue;
    const double cost = (double)n * (bp + bq) + SAMPLE_W * (double)s * (double)N2;
    if (best < 0.0 || cost < best) {
      best = cost;
      pl.N1 = (int)N1;
      pl.N2 = (int)N2;
      pl.P = bp;
      pl.Q = bq;
    }
  }
  if (best < 0.0)
    throw Error(SKR_ENOTSUP, "DCT embedding: n has no factorisation n = N1 N2 with N1 = P Q, P, Q <= 64, "
                             "N1 <= 3072, N2 <= 4096");
  // the s rows with the smallest generator outputs (ties by index), in ascending order
  const uint64_t sd = splitmix_mix(seed);
  std::vector<uint64_t> key((size_t)n);
  for (int64_t i = 0; i < n; ++i) key[(size_t)i] = splitmix_mix(sd + (uint64_t)(i + 1) * GOLDEN);
  std::vector<int> idx((size_t)n);
  for (int64_t i = 0; i < n; ++i) idx[(size_t)i] = (int)i;
  auto less = [&](int x, int y) { return key[x] < key[y] || (key[x] == key[y] && x < y); };
  if (s < n) std::nth_element(idx.begin(), idx.begin() + s, idx.end(), less);
  idx.resize((size_t)s);
  std::sort(idx.begin(), idx.end());
  // group the samples by residue k mod N1 (stage 2 runs one workgroup per residue)
  pl.soff.assign((size_t)pl.N1 + 1, 0);
  for (int i = 0; i < s; ++i) pl.soff[(size_t)(idx[i] % pl.N1) + 1] += 1;
  for (int q = 0; q < pl.N1; ++q) pl.soff[q + 1] += pl.soff[q];
  std::vector<int> fill(pl.soff.begin(), pl.soff.end() - 1);
  pl.samp.assign((size_t)2 * s, 0);
  for (int i = 0; i < s; ++i) {
    const int q = idx[i] % pl.N1;
    const int j = fill[q]++;
    pl.samp[2 * j] = i;
    pl.samp[2 * j + 1] = idx[i];
  }
  std::lock_guard<std::mutex> g(mu);
  if (cache.size() >= 16) cache.clear();
  cache[{n, s, seed}] = pl;
  return pl;
}

size_t srht_z_doubles(int64_t n, int r) { return (size_t)2 * n * r; }

template <typename T>
void launch_srht(int r, int s, const SrhtSpace<T>& a, const SrhtSpace<T>& b, int nspaces, size_t lds_limit,
                 hipStream_t st) {
  SKR_REQUIRE(nspaces == 1 || nspaces == 2, "DCT embedding: one or two spaces");
  SKR_REQUIRE(r >= 1, "DCT embedding: r >= 1");
  const SrhtSpace<T>* sp[2] = {&a, &b};
  int maxN1 = 1, maxN2 = 1, maxPQ = 1;
  for (int q = 0; q < nspaces; ++q) {
    if (sp[q]->n == 0) continue;
    SKR_REQUIRE((int64_t)sp[q]->N1 * sp[q]->N2 == sp[q]->n && sp[q]->P * sp[q]->Q == sp[q]->N1,
                "DCT embedding: inconsistent plan");
    maxN1 = std::max(maxN1, sp[q]->N1);
    maxN2 = std::max(maxN2, sp[q]->N2);
    maxPQ = std::max(maxPQ, sp[q]->P + sp[q]->Q);
  }
  const size_t budget = std::min<size_t>(lds_limit, 160 * 1024) - 1024;
  // stage 1: tables 2 (N1 + (B + 1)(P + Q)) doubles and 3 B cc L doubles per column chunk
  // (L = N1 | 1); the widest tile of b (up to S1B) and chunk of columns that keep three
  // workgroups on a compute unit, else one of each within the whole budget
  const size_t L1 = (size_t)(maxN1 | 1);
  auto tab1_of = [&](int Bt) { return (size_t)2 * (maxN1 + (size_t)(Bt + 1) * maxPQ) * sizeof(double); };
  auto seq1 = [&](int Bt) { return (size_t)3 * Bt * L1 * sizeof(double); };
  int B1 = S1B;
  size_t budget1 = S1_SHARE;
  while (B1 > 1 && tab1_of(B1) + seq1(B1) > budget1) B1 /= 2;
  if (tab1_of(B1) + seq1(B1) > budget1) budget1 = budget;
  const size_t tab1 = tab1_of(B1);
  SKR_REQUIRE(tab1 + seq1(B1) <= budget, "DCT embedding: N1 too large for LDS");
  const int cc1 = (int)std::min<size_t>(r, (budget1 - tab1) / seq1(B1));
  const size_t lds1 = tab1 + (size_t)cc1 * seq1(B1);
  // stage 2: 2 cc N2 doubles per column chunk, within a share that leaves room for two
  // workgroups on a compute unit (one column at least)
  const size_t col2 = (size_t)2 * maxN2 * sizeof(double);
  SKR_REQUIRE(col2 <= budget, "DCT embedding: N2 too large for LDS");
  const size_t budget2 = std::max(col2, std::min(budget, S2_SHARE));
  const int cc2 = (int)std::min<size_t>(std::min(r, CC2MAX), budget2 / col2);
  const size_t lds2 = (size_t)cc2 * col2;
  SKR_HIP(hipFuncSetAttribute((const void*)srht_stage1_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds1));
  SKR_HIP(hipFuncSetAttribute((const void*)srht_stage2_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds2));
  SrhtSpace<T> a1 = a, b1 = (nspaces == 2) ? b : a;
  if (nspaces == 1) b1.n = 0;
  hipLaunchKernelGGL(srht_stage1_kernel<T>, dim3((maxN2 + B1 - 1) / B1, 2), dim3(S1T), lds1, st, a1, b1, r, cc1, B1);
  check_launch("srht_stage1");
  hipLaunchKernelGGL(srht_stage2_kernel<T>, dim3(maxN1, 2), dim3(S2T), lds2, st, a1, b1, r, s, cc2);
  check_launch("srht_stage2");
  const bool pend = (a1.n > 0 && a1.Pend) || (b1.n > 0 && b1.Pend);
  if (pend) {
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>(1024, ((int64_t)s * r + 255) / 256));
    hipLaunchKernelGGL(srht_pending_kernel<T>, dim3(g, 2), dim3(256), 0, st, a1, b1, r, s);
    check_launch("srht_pending");
  }
}

template void launch_srht<double>(int, int, const SrhtSpace<double>&, const SrhtSpace<double>&, int, size_t,
                                  hipStream_t);
template void launch_srht<float>(int, int, const SrhtSpace<float>&, const SrhtSpace<float>&, int, size_t,
                                 hipStream_t);

}  // namespace skr
