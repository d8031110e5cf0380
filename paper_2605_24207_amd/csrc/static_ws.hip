// relnn_layer_fwd_static: the forward of relnn_layer_fwd for callers that
// cannot allocate device memory (code under graph capture, serving loops,
// harnesses that forbid allocation).  Its workspace is a file-scope device
// array of kScratchBytes per GPU, which each GPU the library runs on holds
// until the process ends.  Host code never uses the array's name as a
// device address: the address of the array on each device is looked up once
// (hipGetSymbolAddress, with that device current) and kept per device.
#include <mutex>

#include "layer_fwd.hpp"

namespace relnn {

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;   // 32 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up on the
// first call per device).
char* scratch_ptr() {
  int dev = 0;
  RELNN_HIP(hipGetDevice(&dev));
  RELNN_REQUIRE(dev >= 0 && dev < kMaxDevices, RELNN_E_UNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    RELNN_REQUIRE(e == hipSuccess && p != nullptr, RELNN_E_HIP, "hipGetSymbolAddress of the scratch array failed: %s",
                  hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  return static_cast<char*>(g_ptr[dev]);
}

}  // namespace

}  // namespace relnn

using namespace relnn;

extern "C" relnn_status relnn_static_scratch_bytes(size_t* bytes) {
  return guard([&] {
    RELNN_REQUIRE(bytes != nullptr, RELNN_E_INVALID, "bytes is NULL");
    *bytes = kScratchBytes;
  });
}

extern "C" relnn_status relnn_layer_fwd_static(const relnn_index* idx, const relnn_layer_desc* L,
                                               const void* const* emb, const void* W, const float* b,
                                               float* out, float* pre, int32_t* argmax, relnn_stream_t stream) {
  return guard([&] {
    RELNN_REQUIRE(L == nullptr || !(L->flags & RELNN_PLAIN), RELNN_E_UNSUPPORTED,
                  "RELNN_PLAIN runs a library GEMM, which may allocate: not available without allocation");
    const size_t need = layer_fwd_ws_bytes(idx, L);
    RELNN_REQUIRE(need <= kScratchBytes, RELNN_E_RANGE,
                  "this layer needs %zu bytes of workspace, the static scratch holds %zu", need, kScratchBytes);
    layer_fwd_run(idx, L, emb, W, b, out, pre, argmax, scratch_ptr(), kScratchBytes, (hipStream_t)stream);
  });
}
