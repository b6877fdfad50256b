// Shared definitions of the gfx950 sketched-and-truncated Krylov library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "skrylov.h"

namespace skr {

constexpr int RMAX = 16;          // largest supported block size r
constexpr int WG = 256;           // threads per workgroup of the streaming kernels

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define SKR_HIP(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::skr::Error(SKR_EHIP, std::string(#call) + " failed: " + hipGetErrorString(e_)); \
  } while (0)

#define SKR_REQUIRE(cond, msg)                                                            \
  do {                                                                                    \
    if (!(cond)) throw ::skr::Error(SKR_EINVAL, msg);                                     \
  } while (0)

inline void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(SKR_EHIP, std::string("launch of ") + what + " failed: " + hipGetErrorString(e));
}

template <typename T>
T* dmalloc(size_t count) {
  if (count == 0) return nullptr;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(SKR_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
  }
  return static_cast<T*>(p);
}

inline void dfree(void* p) {
  if (p) (void)hipFree(p);
}

// RAII device buffer
template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  explicit DBuf(size_t count) : p(dmalloc<T>(count)), n(count) {}
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { dfree(p); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { dfree(p); }
  void alloc(size_t count) { dfree(p); p = dmalloc<T>(count); n = count; }
  void zero(hipStream_t s) { if (p) SKR_HIP(hipMemsetAsync(p, 0, n * sizeof(T), s)); }
};

inline int ceil_div(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

// ---------------------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------------------

// Sum over a workgroup of WG threads; every thread gets the result.  `red` must hold WG/64
// doubles of shared memory.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace skr
