// k-ary projected union (Section 2.2) of k join results with one head, and
// the union rule's transform after it (Section 3.1).
//
// The union's content is the set of head keys of all branches: their group
// keys are radix-sorted together and deduplicated, and every branch group is
// mapped to its union row by binary search.  The forward evaluates each
// branch's join -> transform with the fused layer kernels, aggregating per
// branch group (SUM for SUM and MEAN, MAX for MAX), then adds (or takes the
// maximum of) the branch partials into the union rows branch by branch (a
// branch maps its groups to distinct rows, so no two writes of one pass
// meet, and the fixed branch order keeps results deterministic).  MEAN
// divides the union's sums by the union's member counts: it is applied once
// over the whole multiset, never as a mean of the branches' means.  The
// union rule's transform (v W_post + b_post, then act_post) runs on the
// union rows as one matrix-core product.  MAX also records each column's
// maximiser as a position in the concatenation of the branches' canonical
// tuple orders: the first maximiser in (branch, position) order.
//
// The backward runs the chain rule the other way: through act_post and the
// union rule's transform on the union rows (dW_post = v^T dU and dV = dU
// W_post^T as matrix-core products), then, branch by branch, the union
// row's gradient is routed to the branch's groups (MEAN divided by the
// union's member count, MAX through the recorded maximisers) and the
// branch's own layer backward carries it to its weights and embeddings.
#include <memory>
#include <vector>

#include "gemm.hpp"
#include "index.hpp"
#include "layer_fwd.hpp"
#include "prims.hpp"

struct relnn_union {
  int device = 0;
  int k = 0;
  int64_t G = 0;
  const relnn_index* br[RELNN_MAX_UNION] = {};
  relnn::DevBuf keys;                   // [G] ascending
  relnn::DevBuf cnt;                    // [G] members of each key over all branches
  relnn::DevBuf map[RELNN_MAX_UNION];   // [G_i] union row of each branch group
  int64_t base[RELNN_MAX_UNION] = {};   // first position of branch i in the concatenated tuple order
};

using namespace relnn;

namespace {

unsigned grid_n(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 1 << 16)); }

// map[q] = position of key[q] in the sorted distinct keys uk[0..G)
__global__ void k_map_keys(const int32_t* key, int64_t n, const int32_t* uk, int64_t G, int32_t* map) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = key[q];
    int64_t lo = 0, hi = G;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (uk[mid] < v) lo = mid + 1; else hi = mid;
    }
    map[q] = (int32_t)lo;
  }
}

// cnt[map[q]] += |group q| (map injective within a branch)
__global__ void k_add_counts(const int32_t* offsets, const int32_t* map, int64_t n, int32_t* cnt) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    cnt[map[q]] += offsets[q + 1] - offsets[q];
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill(float* p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// acc[map[q]][c] (+)= part[q][c] (SUM) or max (MAX: a later branch replaces
// only a strictly smaller value, so ties stay with the earlier branch; the
// maximiser arg becomes base + the branch's own, when arg is given).
__global__ void k_merge(const float* part, const int32_t* part_arg, const int32_t* map, int64_t n, int h, int is_max,
                        int32_t base, float* acc, int32_t* arg) {
  const int64_t total = n * h;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = i / h;
    const int c = (int)(i - q * h);
    const int64_t o = (int64_t)map[q] * h + c;
    const float v = part[i];
    if (is_max) {
      if (v > acc[o]) {
        acc[o] = v;
        if (arg) arg[o] = base + part_arg[i];
      }
    } else {
      acc[o] += v;
    }
  }
}

// d[i] = g[i] * act'(v[i]) (ReLU'(0) = 0; v unused for NONE)
__global__ void k_act_grad(const float* g, const float* v, int64_t n, int act, float* d) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = (act == RELNN_ACT_RELU && !(v[i] > 0.0f)) ? 0.0f : g[i];
}

// The gradient reaching branch group q: row map[q] of dV (MEAN: divided by
// the union row's member count); MAX: the branch's own maximiser position
// where the union's maximiser lies in this branch, else -1 (no tuple) and a
// zero gradient (the layer backward takes a group's whole gradient row for
// an atom keyed by the group, which holds only where the group owns every
// column).
__global__ void k_union_route(const float* dV, const int32_t* cnt, const int32_t* map, int64_t n, int h, int mean,
                              const int32_t* arg, int64_t base, int64_t E, float* dout, int32_t* am) {
  const int64_t total = n * h;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = i / h;
    const int c = (int)(i - q * h);
    const int64_t o = (int64_t)map[q] * h + c;
    float v = dV[o];
    if (mean) v = v / (float)cnt[map[q]];
    dout[i] = v;
    if (arg) {
      const int64_t a = (int64_t)arg[o] - base;
      const bool mine = a >= 0 && a < E;
      am[i] = mine ? (int32_t)a : -1;
      if (!mine) dout[i] = 0.0f;
    }
  }
}

// MEAN: acc /= cnt; pre = acc; without a post transform out = act(acc).
__global__ void k_union_finish(float* acc, const int32_t* cnt, int64_t G, int h, int mean, float* pre, float* out,
                               int act) {
  const int64_t total = G * h;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    float v = acc[i];
    if (mean) v = v / (float)cnt[i / h];
    acc[i] = v;
    if (pre) pre[i] = v;
    if (out) out[i] = act == RELNN_ACT_RELU ? fmaxf(v, 0.0f) : v;
  }
}

struct UnionPlan {
  size_t ws_acc = 0, ws_part[RELNN_MAX_UNION] = {}, ws_arg[RELNN_MAX_UNION] = {}, ws_layer = 0, total = 0;
  size_t layer_bytes = 0;
};

relnn_layer_desc branch_desc(const relnn_layer_desc* L, int agg) {
  relnn_layer_desc d = *L;
  d.agg = agg == RELNN_MAX ? RELNN_MAX : RELNN_SUM;   // MEAN: sums per branch, divided once after the union
  d.act_post = RELNN_ACT_NONE;
  d.flags = 0;
  return d;
}

UnionPlan plan_union(const relnn_union* U, const relnn_layer_desc* const* L, int agg) {
  UnionPlan p;
  const int h = L[0]->h;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += round_up(std::max<size_t>(bytes, 1), 256);
    return o;
  };
  p.ws_acc = take((size_t)std::max<int64_t>(U->G, 1) * h * 4);
  for (int i = 0; i < U->k; ++i) {
    p.ws_part[i] = take((size_t)std::max<int64_t>(U->br[i]->G, 1) * h * 4);
    if (agg == RELNN_MAX) p.ws_arg[i] = take((size_t)std::max<int64_t>(U->br[i]->G, 1) * h * 4);
    const relnn_layer_desc d = branch_desc(L[i], agg);
    p.layer_bytes = std::max(p.layer_bytes, layer_fwd_ws_bytes(U->br[i], &d));
  }
  p.ws_layer = take(p.layer_bytes);
  p.total = off;
  return p;
}

void check_union_args(const relnn_union* U, const relnn_layer_desc* const* L, int agg) {
  RELNN_REQUIRE(U != nullptr && L != nullptr, RELNN_E_INVALID, "union or layer descriptors are NULL");
  RELNN_REQUIRE(agg >= RELNN_SUM && agg <= RELNN_MAX, RELNN_E_INVALID, "unknown aggregate");
  for (int i = 0; i < U->k; ++i) {
    RELNN_REQUIRE(L[i] != nullptr, RELNN_E_INVALID, "layer descriptor %d is NULL", i);
    RELNN_REQUIRE(L[i]->h == L[0]->h, RELNN_E_INVALID, "branch %d has width %d, branch 0 %d", i, L[i]->h, L[0]->h);
    RELNN_REQUIRE((L[i]->flags & ~(RELNN_FUSED | RELNN_DW_ACCUM)) == 0, RELNN_E_UNSUPPORTED,
                  "branch %d: layer flags are not used here", i);
  }
}

}  // namespace

extern "C" relnn_status relnn_union_build(const relnn_index* const* branches, int32_t k, relnn_stream_t stream,
                                          relnn_union** out) {
  return guard([&] {
    RELNN_REQUIRE(out != nullptr, RELNN_E_INVALID, "out is NULL");
    *out = nullptr;
    RELNN_REQUIRE(branches != nullptr && k >= 1 && k <= RELNN_MAX_UNION, RELNN_E_INVALID,
                  "k must be 1..%d", RELNN_MAX_UNION);
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<relnn_union> U(new relnn_union());
    RELNN_HIP(hipGetDevice(&U->device));
    U->k = k;
    int64_t n = 0, e = 0;
    for (int i = 0; i < k; ++i) {
      RELNN_REQUIRE(branches[i] != nullptr, RELNN_E_INVALID, "branch %d is NULL", i);
      U->br[i] = branches[i];
      U->base[i] = e;
      n += branches[i]->G;
      e += branches[i]->E;
    }
    RELNN_REQUIRE(n < (int64_t)INT32_MAX, RELNN_E_RANGE, "too many groups");
    RELNN_REQUIRE(e < (int64_t)INT32_MAX, RELNN_E_RANGE, "too many tuples over all branches");
    // all branch keys, sorted and deduplicated
    DevBuf all(std::max<int64_t>(n, 1) * sizeof(int32_t));
    int64_t o = 0;
    for (int i = 0; i < k; ++i) {
      if (branches[i]->G > 0)
        RELNN_HIP(hipMemcpyAsync(all.as<int32_t>() + o, branches[i]->group_keys, branches[i]->G * sizeof(int32_t),
                                 hipMemcpyDeviceToDevice, s));
      o += branches[i]->G;
    }
    DevBuf seg(std::max<int64_t>(n, 1) * sizeof(int32_t)), offs((n + 1) * sizeof(int32_t));
    U->keys.alloc(std::max<int64_t>(n, 1) * sizeof(int32_t));
    if (n > 0) {
      uint32_t kmin, kmax;
      prim::key_range(all.as<int32_t>(), nullptr, n, &kmin, &kmax, s);
      DevBuf kk(n * sizeof(uint32_t)), tk(n * sizeof(uint32_t)), tv(n * sizeof(int32_t));
      prim::make_keys(all.as<int32_t>(), nullptr, n, kmin, kk.as<uint32_t>(), s);
      prim::radix_sort_pairs(kk.as<uint32_t>(), all.as<int32_t>(), tk.as<uint32_t>(), tv.as<int32_t>(), n,
                             std::max(1, prim::bits_for((uint64_t)(kmax - kmin))), s);
      U->G = prim::segments(all.as<int32_t>(), n, seg.as<int32_t>(), offs.as<int32_t>(), U->keys.as<int32_t>(), s);
    }
    U->cnt.alloc(std::max<int64_t>(U->G, 1) * sizeof(int32_t));
    if (U->G > 0) {
      k_fill_i32<<<grid_n(U->G), 256, 0, s>>>(U->cnt.as<int32_t>(), U->G, 0);
      RELNN_LAUNCHED();
    }
    for (int i = 0; i < k; ++i) {
      const int64_t Gi = branches[i]->G;
      U->map[i].alloc(std::max<int64_t>(Gi, 1) * sizeof(int32_t));
      if (Gi == 0) continue;
      k_map_keys<<<grid_n(Gi), 256, 0, s>>>(branches[i]->group_keys, Gi, U->keys.as<int32_t>(), U->G,
                                             U->map[i].as<int32_t>());
      RELNN_LAUNCHED();
      k_add_counts<<<grid_n(Gi), 256, 0, s>>>(branches[i]->offsets, U->map[i].as<int32_t>(), Gi,
                                               U->cnt.as<int32_t>());
      RELNN_LAUNCHED();
    }
    RELNN_HIP(hipStreamSynchronize(s));
    *out = U.release();
  });
}

extern "C" relnn_status relnn_union_query(const relnn_union* U, int64_t* n_groups) {
  return guard([&] {
    RELNN_REQUIRE(U != nullptr && n_groups != nullptr, RELNN_E_INVALID, "NULL argument");
    *n_groups = U->G;
  });
}

extern "C" relnn_status relnn_union_export(const relnn_union* U, int32_t* keys, int32_t* counts,
                                           relnn_stream_t stream) {
  return guard([&] {
    RELNN_REQUIRE(U != nullptr, RELNN_E_INVALID, "union is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (keys && U->G > 0)
      RELNN_HIP(hipMemcpyAsync(keys, U->keys.p, U->G * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (counts && U->G > 0)
      RELNN_HIP(hipMemcpyAsync(counts, U->cnt.p, U->G * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  });
}

extern "C" relnn_status relnn_union_free(relnn_union* U) {
  return guard([&] { delete U; });
}

extern "C" relnn_status relnn_union_workspace_size(const relnn_union* U, const relnn_layer_desc* const* L,
                                                   int32_t agg, size_t* bytes) {
  return guard([&] {
    RELNN_REQUIRE(bytes != nullptr, RELNN_E_INVALID, "bytes is NULL");
    check_union_args(U, L, agg);
    *bytes = plan_union(U, L, agg).total;
  });
}

extern "C" relnn_status relnn_union_fwd(const relnn_union* U, const relnn_layer_desc* const* L, int32_t agg,
                                        int32_t act_post, const void* const* const* emb, const void* const* W,
                                        const float* const* b, const float* W_post, const float* b_post,
                                        int32_t h_out, float* out, float* pre, int32_t* argmax, void* ws,
                                        size_t ws_bytes, relnn_stream_t stream) {
  return guard([&] {
    check_union_args(U, L, agg);
    RELNN_REQUIRE(act_post == RELNN_ACT_NONE || act_post == RELNN_ACT_RELU, RELNN_E_INVALID, "unknown activation");
    RELNN_REQUIRE(emb != nullptr && W != nullptr, RELNN_E_INVALID, "emb and W are required");
    const int h = L[0]->h;
    RELNN_REQUIRE(W_post != nullptr || h_out == h, RELNN_E_INVALID, "without W_post, h_out must equal h");
    RELNN_REQUIRE(W_post == nullptr || (h_out > 0 && h % 4 == 0), RELNN_E_UNSUPPORTED,
                  "the post transform needs h %% 4 == 0");
    RELNN_REQUIRE(out != nullptr || U->G == 0, RELNN_E_INVALID, "out is NULL");
    const UnionPlan P = plan_union(U, L, agg);
    RELNN_REQUIRE(ws != nullptr && ws_bytes >= P.total, RELNN_E_INVALID, "workspace of %zu bytes given, %zu needed",
                  ws_bytes, P.total);
    RELNN_REQUIRE(((uintptr_t)ws & 255) == 0, RELNN_E_INVALID, "workspace must be 256-byte aligned");
    if (U->G == 0) return;
    hipStream_t s = (hipStream_t)stream;
    char* w = static_cast<char*>(ws);
    float* acc = reinterpret_cast<float*>(w + P.ws_acc);
    const bool is_max = agg == RELNN_MAX;
    k_fill<<<grid_n(U->G * h), 256, 0, s>>>(acc, U->G * h, is_max ? -INFINITY : 0.0f);
    RELNN_LAUNCHED();
    int32_t* arg = is_max ? argmax : nullptr;
    if (arg) {
      k_fill_i32<<<grid_n(U->G * h), 256, 0, s>>>(arg, U->G * h, -1);
      RELNN_LAUNCHED();
    }
    for (int i = 0; i < U->k; ++i) {                      // each branch, then its partials in branch order
      const relnn_index* bi = U->br[i];
      if (bi->G == 0) continue;
      const relnn_layer_desc d = branch_desc(L[i], agg);
      float* part = reinterpret_cast<float*>(w + P.ws_part[i]);
      int32_t* part_arg = arg ? reinterpret_cast<int32_t*>(w + P.ws_arg[i]) : nullptr;
      layer_fwd_run(bi, &d, emb[i], W[i], b ? b[i] : nullptr, part, nullptr, part_arg, w + P.ws_layer,
                    P.layer_bytes, s);
      k_merge<<<grid_n(bi->G * h), 256, 0, s>>>(part, part_arg, U->map[i].as<int32_t>(), bi->G, h, is_max ? 1 : 0,
                                                 (int32_t)U->base[i], acc, arg);
      RELNN_LAUNCHED();
    }
    k_union_finish<<<grid_n(U->G * h), 256, 0, s>>>(acc, U->cnt.as<int32_t>(), U->G, h, agg == RELNN_MEAN ? 1 : 0,
                                                      pre, W_post ? nullptr : out, act_post);
    RELNN_LAUNCHED();
    if (W_post) {                                         // the union rule's transform, once per key
      RowsEpi epi;
      epi.bias = b_post;
      epi.act = act_post;
      gemm_rows(false, acc, false, h, U->G, h, W_post, false, false, h_out, h_out, out, h_out, epi, s);
    }
  });
}

namespace {

struct UnionBwdPlan {
  size_t ws_dV = 0, ws_u = 0, ws_dU = 0, ws_tn = 0, ws_dout = 0, ws_am = 0, ws_layer = 0, total = 0;
  size_t layer_bytes = 0;
};

relnn_layer_desc branch_bwd_desc(const relnn_layer_desc* L, int agg) {
  relnn_layer_desc d = *L;
  d.agg = agg == RELNN_MAX ? RELNN_MAX : RELNN_SUM;   // MEAN: the division is in the routed gradient
  d.act_post = RELNN_ACT_NONE;
  d.flags = L->flags & RELNN_DW_ACCUM;
  return d;
}

UnionBwdPlan plan_union_bwd(const relnn_union* U, const relnn_layer_desc* const* L, int agg, int h_out) {
  UnionBwdPlan p;
  const int h = L[0]->h;
  const int64_t G = std::max<int64_t>(U->G, 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += round_up(std::max<size_t>(bytes, 1), 256);
    return o;
  };
  p.ws_dV = take((size_t)G * h * 4);
  p.ws_u = take((size_t)G * h_out * 4);
  p.ws_dU = take((size_t)G * h_out * 4);
  p.ws_tn = take((size_t)gemm_tn_ws_floats(G, h, h_out) * 4);
  int64_t gmax = 1;
  for (int i = 0; i < U->k; ++i) {
    gmax = std::max<int64_t>(gmax, U->br[i]->G);
    const relnn_layer_desc d = branch_bwd_desc(L[i], agg);
    p.layer_bytes = std::max(p.layer_bytes, layer_bwd_ws_bytes(U->br[i], &d));
  }
  p.ws_dout = take((size_t)gmax * h * 4);
  if (agg == RELNN_MAX) p.ws_am = take((size_t)gmax * h * 4);
  p.ws_layer = take(p.layer_bytes);
  p.total = off;
  return p;
}

}  // namespace

extern "C" relnn_status relnn_union_bwd_workspace_size(const relnn_union* U, const relnn_layer_desc* const* L,
                                                       int32_t agg, int32_t h_out, size_t* bytes) {
  return guard([&] {
    RELNN_REQUIRE(bytes != nullptr, RELNN_E_INVALID, "bytes is NULL");
    check_union_args(U, L, agg);
    RELNN_REQUIRE(h_out > 0, RELNN_E_INVALID, "h_out must be positive");
    *bytes = plan_union_bwd(U, L, agg, h_out).total;
  });
}

extern "C" relnn_status relnn_union_bwd(const relnn_union* U, const relnn_layer_desc* const* L, int32_t agg,
                                        int32_t act_post, const void* const* const* emb, const void* const* W,
                                        const float* const* b, const float* W_post, const float* b_post,
                                        int32_t h_out, const float* pre, const int32_t* argmax, const float* dout,
                                        float* const* const* demb, float* const* dW, float* const* db,
                                        float* dW_post, float* db_post, void* ws, size_t ws_bytes,
                                        relnn_stream_t stream) {
  return guard([&] {
    check_union_args(U, L, agg);
    RELNN_REQUIRE(act_post == RELNN_ACT_NONE || act_post == RELNN_ACT_RELU, RELNN_E_INVALID, "unknown activation");
    RELNN_REQUIRE(emb != nullptr && W != nullptr && demb != nullptr && dW != nullptr, RELNN_E_INVALID,
                  "emb, W, demb and dW are required");
    const int h = L[0]->h;
    const bool post = W_post != nullptr;
    RELNN_REQUIRE(post || h_out == h, RELNN_E_INVALID, "without W_post, h_out must equal h");
    RELNN_REQUIRE(!post || dW_post != nullptr, RELNN_E_INVALID, "dW_post is required with W_post");
    RELNN_REQUIRE(!post || (h % 4 == 0 && h_out % 4 == 0 && h <= 1024 && h_out <= 1024), RELNN_E_UNSUPPORTED,
                  "the post transform's backward needs h and h_out multiples of 4, at most 1024");
    const int64_t G = U->G;
    RELNN_REQUIRE(dout != nullptr || G == 0, RELNN_E_INVALID, "dout is NULL");
    RELNN_REQUIRE(pre != nullptr || G == 0 || (!post && act_post == RELNN_ACT_NONE), RELNN_E_INVALID,
                  "pre is required with W_post or act_post");
    RELNN_REQUIRE(agg != RELNN_MAX || argmax != nullptr || G == 0, RELNN_E_INVALID, "argmax is required for MAX");
    const UnionBwdPlan P = plan_union_bwd(U, L, agg, h_out);
    RELNN_REQUIRE(ws != nullptr && ws_bytes >= P.total, RELNN_E_INVALID, "workspace of %zu bytes given, %zu needed",
                  ws_bytes, P.total);
    RELNN_REQUIRE(((uintptr_t)ws & 255) == 0, RELNN_E_INVALID, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char* w = static_cast<char*>(ws);
    float* dV = reinterpret_cast<float*>(w + P.ws_dV);
    if (post && G == 0) {                                 // nothing flows: the post gradients are zero
      k_fill<<<grid_n((int64_t)h * h_out), 256, 0, s>>>(dW_post, (int64_t)h * h_out, 0.0f);
      RELNN_LAUNCHED();
      if (db_post) {
        k_fill<<<1, 256, 0, s>>>(db_post, h_out, 0.0f);
        RELNN_LAUNCHED();
      }
    } else if (post) {
      float* dU = reinterpret_cast<float*>(w + P.ws_dU);
      if (act_post == RELNN_ACT_RELU) {                   // u = v W_post + b_post, as the forward formed it
        float* u = reinterpret_cast<float*>(w + P.ws_u);
        RowsEpi epi;
        epi.bias = b_post;
        gemm_rows(false, pre, false, h, G, h, W_post, false, false, h_out, h_out, u, h_out, epi, s);
        k_act_grad<<<grid_n(G * h_out), 256, 0, s>>>(dout, u, G * h_out, act_post, dU);
      } else {
        k_act_grad<<<grid_n(G * h_out), 256, 0, s>>>(dout, nullptr, G * h_out, RELNN_ACT_NONE, dU);
      }
      RELNN_LAUNCHED();
      TnB tb;
      tb.B = dU;
      tb.ldb = h_out;
      gemm_tn(false, pre, false, h, nullptr, nullptr, tb, G, h, h_out, nullptr, dW_post, db_post, false,
              reinterpret_cast<float*>(w + P.ws_tn), s);
      gemm_rows(false, dU, false, h_out, G, h_out, W_post, false, true, h_out, h, dV, h, RowsEpi{}, s);
    } else if (G > 0) {
      k_act_grad<<<grid_n(G * h), 256, 0, s>>>(dout, pre, G * h, act_post, dV);
      RELNN_LAUNCHED();
    }
    const bool is_max = agg == RELNN_MAX;
    float* dout_i = reinterpret_cast<float*>(w + P.ws_dout);
    int32_t* am_i = is_max ? reinterpret_cast<int32_t*>(w + P.ws_am) : nullptr;
    for (int i = 0; i < U->k; ++i) {                      // each branch's share, then its layer backward
      const relnn_index* bi = U->br[i];
      if (bi->G > 0) {
        k_union_route<<<grid_n(bi->G * h), 256, 0, s>>>(dV, U->cnt.as<int32_t>(), U->map[i].as<int32_t>(), bi->G, h,
                                                         agg == RELNN_MEAN ? 1 : 0, is_max ? argmax : nullptr,
                                                         U->base[i], bi->E, dout_i, am_i);
        RELNN_LAUNCHED();
      }
      const relnn_layer_desc d = branch_bwd_desc(L[i], agg);
      layer_bwd_run(bi, &d, emb[i], W[i], b ? b[i] : nullptr, nullptr, am_i, dout_i, demb[i], dW[i],
                    db ? db[i] : nullptr, w + P.ws_layer, P.layer_bytes, s);
    }
  });
}
