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

// Cached device allocation (see runtime.hip): blocks released with pool_free are kept and
// handed out again; pool_trim returns the cache to the HIP runtime.
void* pool_alloc(size_t bytes);
void pool_free(void* p);
void pool_trim();
void pool_quiet_enter();
void pool_quiet_leave();
// Quiet scope: once enter() is called (after the owner has waited for all device work on
// the buffers it is about to release), releases on this host thread until the scope ends
// need no device synchronisation before their reuse.
struct PoolQuiet {
  bool on = false;
  void enter() {
    if (!on) { pool_quiet_enter(); on = true; }
  }
  ~PoolQuiet() {
    if (on) pool_quiet_leave();
  }
};
// Streams (non-blocking, default priority) kept for reuse across solves.
hipStream_t stream_acquire();
void stream_release(hipStream_t s);

template <typename T>
T* dmalloc(size_t count) {
  return static_cast<T*>(pool_alloc(count * sizeof(T)));
}

inline void dfree(void* p) { pool_free(p); }

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

// Data-parallel-primitive move of a double across lanes (two 32-bit DPP moves).
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ inline double lane_value(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a wavefront (all lanes active); every lane gets the result.
// Butterflies within each row of 16 lanes by DPP quad permutations and row rotations, then
// the four row sums read with readlane and added in a fixed order: deterministic, and no
// LDS traffic.
__device__ inline double wave_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x124>(v);  // row_ror:4
  v += dpp_move<0x128>(v);  // row_ror:8
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

}  // namespace skr
