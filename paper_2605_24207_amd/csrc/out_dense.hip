// Dense layout of a layer's (or a union's) output.  The output content of a
// projected union is the set of head keys that occur (Section 2.2), so the
// library writes one row per group, in key order; chained layers and
// serving may prefer rows addressed by the key itself, with a presence byte
// telling the keys that occur from those that do not (their rows are zero).
#include "common.hpp"

using namespace relnn;

namespace {

unsigned grid_n(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 1 << 16)); }

__global__ void k_zero_rows(float* dense, int64_t n, uint8_t* present, int64_t n_out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    dense[i] = 0.0f;
    if (present && i < n_out) present[i] = 0;
  }
}

// dense[keys[g]] = compact[g], present[keys[g]] = 1 (keys distinct)
__global__ void k_scatter_rows(const int32_t* keys, int64_t G, const float* compact, int h, float* dense,
                               uint8_t* present) {
  const int64_t total = G * h;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = i / h;
    const int c = (int)(i - g * h);
    const int64_t row = keys[g];
    dense[row * h + c] = compact[i];
    if (present && c == 0) present[row] = 1;
  }
}

}  // namespace

extern "C" relnn_status relnn_out_dense(const int32_t* keys, int64_t G, const float* compact, int32_t h,
                                        int64_t n_out, float* dense, uint8_t* present, relnn_stream_t stream) {
  return guard([&] {
    RELNN_REQUIRE(G >= 0 && h > 0 && n_out >= 0, RELNN_E_INVALID, "G, h and n_out must be non-negative, h > 0");
    RELNN_REQUIRE(G == 0 || (keys != nullptr && compact != nullptr), RELNN_E_INVALID, "keys and compact are required");
    RELNN_REQUIRE(n_out == 0 || dense != nullptr, RELNN_E_INVALID, "dense is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (G > 0) {                       // ascending keys: the first and the last bound them all
      int32_t ends[2];
      RELNN_HIP(hipMemcpyAsync(&ends[0], keys, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      RELNN_HIP(hipMemcpyAsync(&ends[1], keys + (G - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
      RELNN_HIP(hipStreamSynchronize(s));
      RELNN_REQUIRE(ends[0] >= 0 && (int64_t)ends[1] < n_out && ends[0] <= ends[1], RELNN_E_RANGE,
                    "keys span [%d, %d], outside [0, %lld)", ends[0], ends[1], (long long)n_out);
    }
    if (n_out > 0) {
      const int64_t n = std::max<int64_t>(n_out * h, n_out);
      k_zero_rows<<<grid_n(n), 256, 0, s>>>(dense, n_out * h, present, n_out);
      RELNN_LAUNCHED();
    }
    if (G > 0) {
      k_scatter_rows<<<grid_n(G * h), 256, 0, s>>>(keys, G, compact, h, dense, present);
      RELNN_LAUNCHED();
    }
  });
}
