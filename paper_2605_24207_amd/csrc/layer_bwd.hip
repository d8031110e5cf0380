// Backward of one relational layer: the gradient of sum(out * dout) with
// respect to W, b and every atom's embedding rows (Section 2.3: the
// parameters are the per-tuple embeddings and the transform weights).
//
// With y_tau = act_pre(x_tau W + b), pre_g = alpha_{tau in g} y_tau and
// out_g = act_post(pre_g):
//   dA_g      = dout_g * act_post'(pre_g)                       (ReLU'(0) = 0)
//   dY_tau    = dA_g            (SUM)
//             = dA_g / |g|      (MEAN)
//             = dA_g[j] if tau is the argmax of column j, else 0 (MAX)
//   dY_tau   *= act_pre'(x_tau W + b)   (recomputed mask, only if act_pre)
//   dW        = sum_tau x_tau^T dY_tau,   db = sum_tau dY_tau
//   dz_j[r]  += sum_{tau joined to row r of atom j} (dY_tau W^T)[cols of j]
//
// dz_j always goes through the per-row sums of dY (bwd_linear.hip).  dW and
// db go through the per-group sums of x when dY_tau = dA_g (SUM or MEAN with
// an affine transform); otherwise through the per-tuple product
// sum_tau x_tau^T dY_tau (gemm.hip: the joined rows x_tau gathered again,
// never stored, and dY_tau = dA_g(tau) routed by the maximiser bits and the
// act_pre mask as it is staged), with the atoms keyed by the group column of
// a MAX layer taken over the groups instead.
#include "gemm.hpp"
#include "layer_fwd.hpp"

namespace relnn {

namespace {

// MAX routing as bits: bit c % 32 of word c / 32 of tuple t is set where t
// is its group's maximiser in column c (argmax[g][c] == t).  The argmax row
// of a group is read by its consecutive tuples (from L2 after the first),
// and the sums over joined rows then read 4 bytes per 32 columns of a tuple
// instead of its argmax row.
__global__ void k_own_bits(const int32_t* argmax, const int32_t* tuple_group, int64_t E, int h, int nw,
                           const uint32_t* mask, uint32_t* own) {
  const bool vec = (h & 31) == 0 && (((uintptr_t)argmax) & 15) == 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < E * nw;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = i / nw;
    const int w = (int)(i - t * nw);
    const int32_t* am = argmax + (int64_t)tuple_group[t] * h + 32 * w;
    const int32_t tt = (int32_t)t;
    uint32_t bits = 0;
    if (vec) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int4 v = reinterpret_cast<const int4*>(am)[q];
        bits |= (uint32_t)(v.x == tt) << (4 * q) | (uint32_t)(v.y == tt) << (4 * q + 1) |
                (uint32_t)(v.z == tt) << (4 * q + 2) | (uint32_t)(v.w == tt) << (4 * q + 3);
      }
    } else {
      const int nb = min(32, h - 32 * w);
      for (int b = 0; b < nb; ++b) bits |= (uint32_t)(am[b] == tt) << b;
    }
    own[i] = mask ? bits & mask[i] : bits;           // act_pre: also where x W + b > 0
  }
}

// dA[g][n] = dout[g][n] * act_post'(pre[g][n]) (ReLU'(0) = 0), divided by
// the group's tuple count for MEAN: the per-group part of the routing.
__global__ void k_route_prep(const float* dout, const float* pre, const int32_t* offsets, int64_t G, int h, int agg,
                             int act_post, float* dA) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < G * h;
       i += (int64_t)gridDim.x * blockDim.x) {
    float v = dout[i];
    if (act_post == RELNN_ACT_RELU && !(pre[i] > 0.0f)) v = 0.0f;
    if (agg == RELNN_MEAN) {
      const int64_t g = i / h;
      v = v / (float)(offsets[g + 1] - offsets[g]);
    }
    dA[i] = v;
  }
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 1 << 16));
}

struct BwdPlan {
  FwdPlan F;
  int K = 0;
  size_t ws_mask = 0, ws_fwsw = 0, ws_dA = 0, ws_own = 0, ws_part = 0, ws_prod = 0, total = 0;
  int kv = 0;                // per-tuple dW: atoms 0 .. kv-1 (MAX: the others are keyed by the group column)
  bool xs_dw = false;        // dW through the per-group sums (SUM / MEAN, affine)
  LinBwdPlan lin;
};

BwdPlan plan_bwd(const relnn_index* idx, const relnn_layer_desc* L, const FwdPlan& F) {
  BwdPlan p;
  p.F = F;
  p.K = F.K;
  const int64_t E = idx->E;
  if (L->flags & RELNN_TF_PRODUCT) {                     // dA, maximiser bits, the per-atom passes
    size_t off = 0;
    p.ws_dA = off;
    off += round_up(std::max<int64_t>(idx->G, 1) * L->h * 4, 256);
    p.ws_own = off;
    if (L->agg == RELNN_MAX) off += round_up(std::max<int64_t>(E, 1) * cdiv(L->h, 32) * 4, 256);
    p.ws_prod = off;
    off += prod_bwd_ws_bytes(idx, L);
    p.total = off;
    return p;
  }
  p.xs_dw = L->act_pre == RELNN_ACT_NONE && L->agg != RELNN_MAX;
  size_t off = 0;
  p.ws_mask = off;                                       // act_pre: mask bits [E][ceil(h / 32)]
  if (L->act_pre != RELNN_ACT_NONE) off += round_up(std::max<int64_t>(E, 1) * cdiv(L->h, 32) * 4, 256);
  p.ws_fwsw = off;
  if (L->act_pre != RELNN_ACT_NONE)                     // W swizzled for the mask kernel
    off += round_up((int64_t)F.Kp * L->h * (L->dtype == RELNN_BF16 ? 2 : 4), 256);
  p.ws_dA = off;
  off += round_up(std::max<int64_t>(idx->G, 1) * L->h * 4, 256);
  p.ws_own = off;                                        // MAX: ownership bits [E][ceil(h / 32)]
  if (L->agg == RELNN_MAX) off += round_up(std::max<int64_t>(E, 1) * cdiv(L->h, 32) * 4, 256);
  // MAX without act_pre: trailing atoms keyed by the group column leave the
  // per-tuple dW for a product over the groups (their routed gradients add
  // up to dA_g per group)
  p.kv = L->k;
  if (L->agg == RELNN_MAX && L->act_pre == RELNN_ACT_NONE)
    while (p.kv > 1 && idx->atom_gk[p.kv - 1]) --p.kv;
  p.ws_part = off;
  if (!p.xs_dw) {
    int64_t nf = 0;
    for (int j = 0; j < L->k; ++j)
      nf = std::max(nf, j < p.kv ? gemm_tn_ws_floats(E, L->d[j], L->h) : gk_dw_ws_floats(idx->G, L->d[j], L->h));
    off += round_up(nf * 4, 256);
  }
  p.lin = plan_lin_bwd(idx, L, off, p.xs_dw);
  p.total = p.lin.total;
  return p;
}

}  // namespace

size_t bwd_workspace(const relnn_index* idx, const relnn_layer_desc* L, const FwdPlan& P) {
  return plan_bwd(idx, L, P).total;
}

size_t layer_bwd_ws_bytes(const relnn_index* idx, const relnn_layer_desc* L) {
  return plan_bwd(idx, L, checked_plan(idx, L)).total;
}

void layer_bwd_run(const relnn_index* idx, const relnn_layer_desc* L, const void* const* emb, const void* W,
                   const float* b, const float* pre, const int32_t* argmax, const float* dout, float* const* demb,
                   float* dW, float* db, void* ws, size_t ws_bytes, hipStream_t stream) {
  {
    FwdPlan F = checked_plan(idx, L);
    RELNN_REQUIRE(idx->has_bwd, RELNN_E_INVALID, "the index was built without RELNN_IDX_BWD");
    RELNN_REQUIRE(!(L->flags & RELNN_OUT_BF16), RELNN_E_INVALID, "RELNN_OUT_BF16 is a forward-only flag");
    const bool prod = (L->flags & RELNN_TF_PRODUCT) != 0;
    const BwdPlan P = plan_bwd(idx, L, F);
    RELNN_REQUIRE(emb != nullptr && demb != nullptr && (prod || (W != nullptr && dW != nullptr)), RELNN_E_INVALID,
                  "emb, W, dW and demb are required (W and dW not for the product transform)");
    RELNN_REQUIRE(dout != nullptr || idx->G == 0, RELNN_E_INVALID, "dout is NULL");
    RELNN_REQUIRE(L->act_post == RELNN_ACT_NONE || pre != nullptr || idx->G == 0, RELNN_E_INVALID,
                  "pre is required when act_post is not NONE");
    RELNN_REQUIRE(L->agg != RELNN_MAX || argmax != nullptr || idx->G == 0, RELNN_E_INVALID,
                  "argmax is required for MAX");
    for (int j = 0; j < L->k; ++j) {
      RELNN_REQUIRE(emb[j] != nullptr || idx->n_rows[j] == 0, RELNN_E_INVALID, "emb[%d] is NULL", j);
      RELNN_REQUIRE(demb[j] != nullptr || idx->n_rows[j] == 0, RELNN_E_INVALID, "demb[%d] is NULL", j);
      RELNN_REQUIRE(((uintptr_t)emb[j] & 15) == 0, RELNN_E_UNSUPPORTED, "emb[%d] is not 16-byte aligned", j);
      RELNN_REQUIRE(prod || L->d[j] % 16 == 0, RELNN_E_UNSUPPORTED, "backward needs d[%d] %% 16 == 0", j);
    }
    RELNN_REQUIRE(ws != nullptr && ws_bytes >= P.total, RELNN_E_INVALID,
                  "workspace of %zu bytes given, %zu needed", ws_bytes, P.total);
    RELNN_REQUIRE(((uintptr_t)ws & 255) == 0, RELNN_E_INVALID, "workspace must be 256-byte aligned");
    RELNN_REQUIRE(L->h % 4 == 0, RELNN_E_UNSUPPORTED, "backward needs h %% 4 == 0");
    hipStream_t s = (hipStream_t)stream;
    char* w = static_cast<char*>(ws);
    const int h = L->h;
    const int64_t E = idx->E;
    const bool accum = (L->flags & RELNN_DW_ACCUM) != 0;
    if (prod) {                                  // no weights: the embedding gradients only
      if (E == 0) return;
      float* dA = reinterpret_cast<float*>(w + P.ws_dA);
      k_route_prep<<<grid_for(idx->G * h), 256, 0, s>>>(dout, pre, idx->offsets, idx->G, h, L->agg, L->act_post, dA);
      RELNN_LAUNCHED();
      const int nw = (int)cdiv(h, 32);
      uint32_t* own = nullptr;
      if (L->agg == RELNN_MAX) {
        own = reinterpret_cast<uint32_t*>(w + P.ws_own);
        k_own_bits<<<grid_for(E * nw), 256, 0, s>>>(argmax, idx->tuple_group, E, h, nw, nullptr, own);
        RELNN_LAUNCHED();
      }
      prod_bwd(idx, L, emb, dA, own, nw, demb, w + P.ws_prod, s);
      return;
    }
    if (E == 0) {
      if (!accum) {
        k_fill_f32<<<grid_for((int64_t)P.K * h), 256, 0, s>>>(dW, (int64_t)P.K * h, 0.0f);
        RELNN_LAUNCHED();
        if (db) {
          k_fill_f32<<<1, 256, 0, s>>>(db, h, 0.0f);
          RELNN_LAUNCHED();
        }
      }
      return;
    }
    const Atoms at = make_atoms(L, emb, idx);
    float* dA = reinterpret_cast<float*>(w + P.ws_dA);
    k_route_prep<<<grid_for(idx->G * h), 256, 0, s>>>(dout, pre, idx->offsets, idx->G, h, L->agg, L->act_post, dA);
    RELNN_LAUNCHED();
    const int nw = (int)cdiv(h, 32);
    uint32_t* mask = nullptr;
    if (L->act_pre != RELNN_ACT_NONE) {      // recompute act_pre'(x W + b) per tuple, one bit per column
      FwdArgs a{};
      a.at = at;
      a.rows = idx->rows;
      a.E = E;
      a.K = F.K;
      a.Kp = F.Kp;
      a.h = h;
      a.TM = F.TM;
      a.off_x = (int)F.off_x;
      a.off_y = (int)F.off_y;
      a.Wsw = w + P.ws_fwsw;
      a.b = b;
      a.mask = reinterpret_cast<uint32_t*>(w + P.ws_mask);
      swizzle_w(W, L->dtype, F.K, F.Kp, h, w + P.ws_fwsw, s);
      launch_mask(F, a, L->dtype, s);
      mask = a.mask;
    }
    // routing of dY: one bit per tuple and column, set where the tuple is
    // its group's maximiser (MAX) and where x W + b > 0 (act_pre)
    uint32_t* route = mask;
    if (L->agg == RELNN_MAX) {
      route = reinterpret_cast<uint32_t*>(w + P.ws_own);
      k_own_bits<<<grid_for(E * nw), 256, 0, s>>>(argmax, idx->tuple_group, E, h, nw, mask, route);
      RELNN_LAUNCHED();
    }

    // dW and db
    if (P.xs_dw) {
      lin_bwd_dw(idx, L, P.lin, emb, dA, dW, db, accum, w, s);
    } else {
      // per tuple: dW rows of atom j = sum_tau x_j(tau)^T dY_tau, and db =
      // sum_tau dY_tau with the first atom
      TnB B;
      B.B = dA;
      B.ldb = h;
      B.brow = idx->tuple_group;
      B.own = route;
      B.own_w = nw;
      const bool bf16 = L->dtype == RELNN_BF16;
      float* part = reinterpret_cast<float*>(w + P.ws_part);
      for (int j = 0, koff = 0; j < L->k; koff += L->d[j], ++j) {
        KTimer tm("bwd_dw", s);
        if (j < P.kv)
          gemm_tn(bf16, emb[j], bf16, L->d[j], idx->rows + (int64_t)j * E, nullptr, B, E, L->d[j], h, nullptr,
                  dW + (int64_t)koff * h, j == 0 ? db : nullptr, accum, part, s);
        else
          gk_dw(idx, j, emb[j], bf16, L->d[j], h, dA, dW + (int64_t)koff * h, accum, part, s);
      }
    }

    // dz_j for every atom, in body order (through the per-row sums of dY)
    lin_bwd_dx(idx, L, P.lin, W, dA, route, nw, mask != nullptr, demb, w, s);
  }
}

}  // namespace relnn

using namespace relnn;

extern "C" relnn_status relnn_layer_bwd(const relnn_index* idx, const relnn_layer_desc* L,
                                        const void* const* emb, const void* W, const float* b,
                                        const float* pre, const int32_t* argmax, const float* dout,
                                        float* const* demb, float* dW, float* db, void* ws, size_t ws_bytes,
                                        relnn_stream_t stream) {
  return guard([&] {
    layer_bwd_run(idx, L, emb, W, b, pre, argmax, dout, demb, dW, db, ws, ws_bytes, (hipStream_t)stream);
  });
}
