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
// an affine transform); otherwise this file's per-tuple kernel: the joined
// rows x_tau are gathered again, never stored, and a persistent kernel
// accumulates X^T dY over its contiguous run of tiles on the matrix cores
// (FP32 16x16x4), then the per-block partials are summed in block order.
#include "layer_fwd.hpp"

namespace relnn {

namespace {

constexpr int kDwTM = 32;
constexpr int kDwThreads = 512;
constexpr int kDwMaxB = 24;              // 16x16 accumulator blocks per wave

struct Route {
  const float* dA;          // [G][h] dout * act_post'(pre), / |g| for MEAN
  const int32_t* argmax;    // [G][h] (MAX)
  const int32_t* tuple_group;
  const uint8_t* mask;      // [E][h] (act_pre != NONE)
  int h, agg;
};

// dY of tuple e (group g), column n.
__device__ __forceinline__ float route(const Route& R, int64_t e, int64_t g, int n) {
  const int64_t o = g * R.h + n;
  float v = R.dA[o];
  if (R.agg == RELNN_MAX && R.argmax[o] != (int32_t)e) v = 0.0f;
  if (R.mask && !R.mask[e * R.h + n]) v = 0.0f;
  return v;
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

// ---------------------------------------------------------------- dW, db
struct DwArgs {
  Atoms at;
  const int32_t* rows;      // [k*E]
  int64_t E;
  int K, K16;               // K and K rounded up to 16
  int n0, hn;               // output columns [n0, n0 + hn) of this launch
  Route R;
  int64_t ntiles, nunits;
  float* part;              // [nunits][K16][h]
  float* dbpart;            // [nunits][h]
};

template <class T>
__global__ void __launch_bounds__(kDwThreads) k_bwd_dw(DwArgs a) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  constexpr int TM = kDwTM;
  constexpr int EPC = 16 / sizeof(T);
  const int XS = a.K16 + 4;
  const int DS = a.hn + 4;
  float* Xs = reinterpret_cast<float*>(smem);      // [TM][XS] gathered x, FP32
  float* Ds = Xs + TM * XS;                         // [TM][DS] routed dY
  const int h = a.R.h;
  const int lane = __lane_id();
  const int w = threadIdx.x / 64;
  const int nrb = a.K16 / 16, ncb = a.hn / 16;
  const int nblk = nrb * ncb;
  const int64_t bidx = blockIdx.x;
  const int64_t tb = (a.ntiles * bidx) / a.nunits, te = (a.ntiles * (bidx + 1)) / a.nunits;
  f32x4 acc[kDwMaxB];
#pragma unroll
  for (int q = 0; q < kDwMaxB; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  float dbacc = 0.0f;
  const int cpr = a.K16 / EPC;

  for (int64_t t = tb; t < te; ++t) {
    const int64_t e0 = t * TM;
    const int nv = (int)min<int64_t>(TM, a.E - e0);
    for (int i = threadIdx.x; i < TM * cpr; i += blockDim.x) {
      const int r = i / cpr, c = i - (i / cpr) * cpr;
      const int el = c * EPC;
      float vals[EPC];
#pragma unroll
      for (int u = 0; u < EPC; ++u) vals[u] = 0.0f;
      if (r < nv && el < a.K) {
        int j = 0;
#pragma unroll
        for (int q = 1; q < kMaxAtoms; ++q)
          if (q < a.at.k && el >= a.at.koff[q]) j = q;
        const int64_t row = a.at.rows[j][e0 + r];
        const uint4 raw = *reinterpret_cast<const uint4*>(static_cast<const T*>(a.at.emb[j]) + row * a.at.d[j] +
                                                          (el - a.at.koff[j]));
        const T* tv = reinterpret_cast<const T*>(&raw);
#pragma unroll
        for (int u = 0; u < EPC; ++u) vals[u] = (float)tv[u];
      }
#pragma unroll
      for (int u = 0; u < EPC; ++u) Xs[r * XS + el + u] = vals[u];
    }
    for (int i = threadIdx.x; i < TM * a.hn; i += blockDim.x) {
      const int r = i / a.hn, n = i - (i / a.hn) * a.hn;
      float v = 0.0f;
      if (r < nv) {
        const int64_t e = e0 + r;
        v = route(a.R, e, a.R.tuple_group[e], a.n0 + n);
      }
      Ds[r * DS + n] = v;
    }
    __syncthreads();
    // dW[k][n] += sum_e X[e][k] dY[e][n]: A = X^T (lane: X[e = 4ks + l/16][k]),
    // B = dY (lane: dY[4ks + l/16][n]).
#pragma unroll
    for (int ks = 0; ks < TM / 4; ++ks) {
      const int er = ks * 4 + (lane >> 4);
#pragma unroll
      for (int q = 0; q < kDwMaxB; ++q) {
        const int blk = w + 8 * q;
        if (blk < nblk) {
          const int rb = blk / ncb, cb = blk - (blk / ncb) * ncb;
          const float av = Xs[er * XS + rb * 16 + (lane & 15)];
          const float bv = Ds[er * DS + cb * 16 + (lane & 15)];
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[q], 0, 0, 0);
        }
      }
    }
    if (threadIdx.x < a.hn)
      for (int r = 0; r < nv; ++r) dbacc += Ds[r * DS + threadIdx.x];
    __syncthreads();
  }
  // per-block partials
#pragma unroll
  for (int q = 0; q < kDwMaxB; ++q) {
    const int blk = w + 8 * q;
    if (blk < nblk) {
      const int rb = blk / ncb, cb = blk - (blk / ncb) * ncb;
      const int n = a.n0 + cb * 16 + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = rb * 16 + 4 * (lane >> 4) + i;
        a.part[(bidx * a.K16 + k) * h + n] = acc[q][i];
      }
    }
  }
  if (threadIdx.x < a.hn) a.dbpart[bidx * h + a.n0 + threadIdx.x] = dbacc;
}

// dW[k][n] (+)= sum over blocks b of part[b][k][n], in block order, Kahan.
__global__ void k_dw_reduce(const float* part, const float* dbpart, int64_t nunits, int K, int K16, int h,
                            float* dW, float* db, int accumulate) {
  const int64_t total = (int64_t)K * h + (db ? h : 0);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.0f, c = 0.0f;
    if (i < (int64_t)K * h) {
      const int64_t k = i / h, n = i - (i / h) * h;
      for (int64_t b = 0; b < nunits; ++b) {
        const float y = part[(b * K16 + k) * h + n] - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
      }
      dW[i] = accumulate ? dW[i] + s : s;
    } else {
      const int64_t n = i - (int64_t)K * h;
      for (int64_t b = 0; b < nunits; ++b) {
        const float y = dbpart[b * h + n] - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
      }
      db[n] = accumulate ? db[n] + s : s;
    }
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

int num_cus() {
  static int n = 0;
  if (!n) {
    int dev = 0;
    RELNN_HIP(hipGetDevice(&dev));
    RELNN_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
  }
  return n;
}

struct BwdPlan {
  FwdPlan F;
  int K = 0, K16 = 0, hn = 0;
  int64_t dw_tiles = 0, dw_units = 0;
  size_t dw_lds = 0;
  size_t ws_mask = 0, ws_fwsw = 0, ws_part = 0, ws_dbpart = 0, ws_dA = 0, total = 0;
  bool xs_dw = false;        // dW through the per-group sums (SUM / MEAN, affine)
  LinBwdPlan lin;
};

BwdPlan plan_bwd(const relnn_index* idx, const relnn_layer_desc* L, const FwdPlan& F) {
  BwdPlan p;
  p.F = F;
  p.K = F.K;
  p.K16 = (int)round_up(F.K, 16);
  int hn = (kDwMaxB * 8 * 16 * 16 / p.K16) / 16 * 16;
  p.hn = std::max(16, std::min(L->h, hn));
  const int64_t E = idx->E;
  p.xs_dw = L->act_pre == RELNN_ACT_NONE && L->agg != RELNN_MAX;
  p.dw_tiles = cdiv(E, kDwTM);
  p.dw_units = std::max<int64_t>(1, std::min<int64_t>(p.dw_tiles, num_cus()));
  p.dw_lds = (size_t)kDwTM * (p.K16 + 4) * 4 + (size_t)kDwTM * (p.hn + 4) * 4;
  size_t off = 0;
  p.ws_mask = off;
  if (L->act_pre != RELNN_ACT_NONE) off += round_up(std::max<int64_t>(E, 1) * L->h, 256);
  p.ws_fwsw = off;
  off += round_up(F.ws_carry - F.ws_wsw, 256);          // forward W swizzle (mask kernel)
  p.ws_part = off;
  if (!p.xs_dw) {
    off += round_up(p.dw_units * p.K16 * L->h * 4, 256);
    p.ws_dbpart = off;
    off += round_up(p.dw_units * L->h * 4, 256);
  }
  p.ws_dA = off;
  off += round_up(std::max<int64_t>(idx->G, 1) * L->h * 4, 256);
  p.lin = plan_lin_bwd(idx, L, off, p.xs_dw);
  p.total = p.lin.total;
  return p;
}

template <class KernelT>
void allow_lds(KernelT k, size_t bytes) {
  RELNN_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

}  // namespace

size_t bwd_workspace(const relnn_index* idx, const relnn_layer_desc* L, const FwdPlan& P) {
  return plan_bwd(idx, L, P).total;
}

}  // namespace relnn

using namespace relnn;

extern "C" relnn_status relnn_layer_bwd(const relnn_index* idx, const relnn_layer_desc* L,
                                        const void* const* emb, const void* W, const float* b,
                                        const float* pre, const int32_t* argmax, const float* dout,
                                        float* const* demb, float* dW, float* db, void* ws, size_t ws_bytes,
                                        relnn_stream_t stream) {
  return guard([&] {
    FwdPlan F = checked_plan(idx, L);
    RELNN_REQUIRE(idx->has_bwd, RELNN_E_INVALID, "the index was built without RELNN_IDX_BWD");
    RELNN_REQUIRE(!(L->flags & RELNN_OUT_BF16), RELNN_E_INVALID, "RELNN_OUT_BF16 is a forward-only flag");
    const BwdPlan P = plan_bwd(idx, L, F);
    RELNN_REQUIRE(emb != nullptr && W != nullptr && dW != nullptr && demb != nullptr, RELNN_E_INVALID,
                  "emb, W, dW and demb are required");
    RELNN_REQUIRE(dout != nullptr || idx->G == 0, RELNN_E_INVALID, "dout is NULL");
    RELNN_REQUIRE(L->act_post == RELNN_ACT_NONE || pre != nullptr || idx->G == 0, RELNN_E_INVALID,
                  "pre is required when act_post is not NONE");
    RELNN_REQUIRE(L->agg != RELNN_MAX || argmax != nullptr || idx->G == 0, RELNN_E_INVALID,
                  "argmax is required for MAX");
    for (int j = 0; j < L->k; ++j) {
      RELNN_REQUIRE(emb[j] != nullptr || idx->n_rows[j] == 0, RELNN_E_INVALID, "emb[%d] is NULL", j);
      RELNN_REQUIRE(demb[j] != nullptr || idx->n_rows[j] == 0, RELNN_E_INVALID, "demb[%d] is NULL", j);
      RELNN_REQUIRE(((uintptr_t)emb[j] & 15) == 0, RELNN_E_UNSUPPORTED, "emb[%d] is not 16-byte aligned", j);
      RELNN_REQUIRE(L->d[j] % 16 == 0, RELNN_E_UNSUPPORTED, "backward needs d[%d] %% 16 == 0", j);
    }
    RELNN_REQUIRE(ws != nullptr && ws_bytes >= P.total, RELNN_E_INVALID,
                  "workspace of %zu bytes given, %zu needed", ws_bytes, P.total);
    RELNN_REQUIRE(((uintptr_t)ws & 255) == 0, RELNN_E_INVALID, "workspace must be 256-byte aligned");
    RELNN_REQUIRE(P.xs_dw || P.dw_lds <= 160 * 1024, RELNN_E_UNSUPPORTED,
                  "K = %d, h = %d does not fit the backward LDS tiles", P.K, L->h);
    hipStream_t s = (hipStream_t)stream;
    char* w = static_cast<char*>(ws);
    const int h = L->h;
    const int64_t E = idx->E;
    const bool accum = (L->flags & RELNN_DW_ACCUM) != 0;
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
    Route R{dA, argmax, idx->tuple_group, nullptr, h, L->agg};

    if (L->act_pre != RELNN_ACT_NONE) {      // recompute act_pre'(x W + b) per tuple
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
      a.mask = reinterpret_cast<uint8_t*>(w + P.ws_mask);
      swizzle_w(W, L->dtype, F.K, F.Kp, h, w + P.ws_fwsw, s);
      launch_mask(F, a, L->dtype, s);
      R.mask = a.mask;
    }

    // dW and db
    if (P.xs_dw) {
      lin_bwd_dw(idx, L, P.lin, emb, dA, dW, db, accum, w, s);
    } else {
      DwArgs d{};
      d.at = at;
      d.rows = idx->rows;
      d.E = E;
      d.K = P.K;
      d.K16 = P.K16;
      d.R = R;
      d.ntiles = P.dw_tiles;
      d.nunits = P.dw_units;
      d.part = reinterpret_cast<float*>(w + P.ws_part);
      d.dbpart = reinterpret_cast<float*>(w + P.ws_dbpart);
      for (int n0 = 0; n0 < h; n0 += P.hn) {
        d.n0 = n0;
        d.hn = std::min(P.hn, h - n0);
        KTimer tm("bwd_dw", s);
        if (L->dtype == RELNN_BF16) {
          allow_lds(k_bwd_dw<__bf16>, P.dw_lds);
          k_bwd_dw<__bf16><<<(unsigned)P.dw_units, kDwThreads, P.dw_lds, s>>>(d);
        } else {
          allow_lds(k_bwd_dw<float>, P.dw_lds);
          k_bwd_dw<float><<<(unsigned)P.dw_units, kDwThreads, P.dw_lds, s>>>(d);
        }
        RELNN_LAUNCHED();
      }
      k_dw_reduce<<<grid_for((int64_t)P.K * h + h), 256, 0, s>>>(d.part, d.dbpart, P.dw_units, P.K, P.K16, h, dW,
                                                                   db, accum ? 1 : 0);
      RELNN_LAUNCHED();
    }

    // dz_j for every atom, in body order (through the per-row sums of dY)
    lin_bwd_dx(idx, L, P.lin, W, dA, L->agg == RELNN_MAX ? argmax : nullptr, R.mask, demb, w, s);
  });
}
