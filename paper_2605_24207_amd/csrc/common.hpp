// Shared host/device helpers of librelnn (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <utility>

#include "../../include/relnn.h"

namespace relnn {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);

struct Fail {
  relnn_status st;
};

#define RELNN_REQUIRE(cond, code, ...)          \
  do {                                          \
    if (!(cond)) {                              \
      ::relnn::set_error(__VA_ARGS__);          \
      throw ::relnn::Fail{code};                \
    }                                           \
  } while (0)

#define RELNN_HIP(call)                                                           \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ::relnn::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),   \
                         __FILE__, __LINE__);                                     \
      throw ::relnn::Fail{e_ == hipErrorOutOfMemory ? RELNN_E_OOM : RELNN_E_HIP}; \
    }                                                                             \
  } while (0)

#define RELNN_LAUNCHED() RELNN_HIP(hipGetLastError())

// Runs `body` and maps a Fail (or any C++ exception) to a status.
template <class F>
relnn_status guard(F&& body) {
  try {
    body();
    return RELNN_OK;
  } catch (const Fail& f) {
    return f.st;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return RELNN_E_OOM;
  } catch (...) {
    set_error("unexpected C++ exception");
    return RELNN_E_HIP;
  }
}

// Device buffer owned by host code, freed on scope exit.
struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  explicit DevBuf(size_t bytes) { alloc(bytes); }
  void alloc(size_t bytes) {
    release();
    n = bytes;
    if (bytes) RELNN_HIP(hipMalloc(&p, bytes));
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

// Brackets one kernel launch with HIP events on its stream when timing is
// enabled (relnn_timing_enable); a no-op otherwise.
class KTimer {
 public:
  KTimer(const char* name, hipStream_t s);
  ~KTimer();
  KTimer(const KTimer&) = delete;
  KTimer& operator=(const KTimer&) = delete;

 private:
  const char* name_;
  hipStream_t s_;
  void* a_ = nullptr;
  void* b_ = nullptr;
};

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// A wave-uniform span of `bytes` bytes as a raw buffer resource (the gfx9
// resource word 3 for raw 32-bit access): loads through it take the base
// from scalar registers and a 32-bit lane offset, and read 0 past the end.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// Waves of `kernel` (blocks of `threads` threads, no dynamic LDS) that the
// GPU holds at once: its blocks per CU (the occupancy query, which accounts
// for its registers) times the CUs.  Cached per kernel.  The range-split
// kernels launch at most this many waves, so that all of them run in one
// round instead of a full round followed by a partly empty one.
int64_t resident_waves(const void* kernel, int threads);

// min(cap, the waves of kernel held at once), at least 1
template <class KernelT>
int64_t one_round_units(KernelT kernel, int threads, int64_t cap) {
  const int64_t r = resident_waves(reinterpret_cast<const void*>(kernel), threads);
  return std::max<int64_t>(1, std::min<int64_t>(cap, r));
}
inline int64_t round_up(int64_t a, int64_t b) { return cdiv(a, b) * b; }

// ------------------------------------------------------------------ device
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

}  // namespace relnn
