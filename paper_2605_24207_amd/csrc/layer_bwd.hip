// Backward of one relational layer (placeholder until the kernels land).
#include "layer_fwd.hpp"

namespace relnn {
size_t bwd_workspace(const relnn_index*, const relnn_layer_desc*, const FwdPlan&) { return 256; }
}  // namespace relnn

using namespace relnn;

extern "C" relnn_status relnn_layer_bwd(const relnn_index*, const relnn_layer_desc*, const void* const*,
                                        const void*, const float*, const float*, const int32_t*,
                                        const float*, float* const*, float*, float*, void*, size_t,
                                        relnn_stream_t) {
  return guard([&] { RELNN_REQUIRE(false, RELNN_E_UNSUPPORTED, "backward not built yet"); });
}
