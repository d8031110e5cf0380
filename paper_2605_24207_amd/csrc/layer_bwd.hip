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
// (FP32 16x16x4, tiles staged transposed and double-buffered in LDS), then
// the per-block partials are summed in block order.
#include "layer_fwd.hpp"

namespace relnn {

namespace {

constexpr int kDwTM = 32;
constexpr int kDwThreads = 512;
constexpr int kDwTS = kDwTM + 4;         // LDS row stride (floats) of the transposed tiles

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

// MAX routing as bits: bit c % 32 of word c / 32 of tuple t is set where t
// is its group's maximiser in column c (argmax[g][c] == t).  The argmax row
// of a group is read by its consecutive tuples (from L2 after the first),
// and the sums over joined rows then read 4 bytes per 32 columns of a tuple
// instead of its argmax row.
__global__ void k_own_bits(const int32_t* argmax, const int32_t* tuple_group, int64_t E, int h, int nw,
                           uint32_t* own) {
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
    own[i] = bits;
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
  int vec4;                 // h % 4 == 0 and dA / argmax 16-byte aligned: routed dY read 4 columns at a time
  int ncb;                  // column blocks per pass: 1, 2, 4 or 8
};

// Tiles are staged transposed in LDS, XT[k][tuple] and DT[n][tuple] (row
// stride kDwTS floats), double-buffered: the global loads of tile t+1 are in
// flight while tile t is multiplied.  MFMA step s (0..7) of a tile pairs
// tuple 8 (l / 16) + s with lane l, so the 8 steps of a lane read 8
// consecutive tuples of one row: two 16-byte LDS reads per operand per tile.
// Wave w owns the 16x16 output blocks w, w + 8, ... (row block blk / ncb,
// column block blk % ncb).
template <class T>
__device__ __forceinline__ float4 dw_load4(const T* p);
template <>
__device__ __forceinline__ float4 dw_load4<float>(const float* p) {
  return *reinterpret_cast<const float4*>(p);
}
template <>
__device__ __forceinline__ float4 dw_load4<__bf16>(const __bf16* p) {
  const uint2 r = *reinterpret_cast<const uint2*>(p);
  return make_float4(__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xffff0000u), __uint_as_float(r.y << 16),
                     __uint_as_float(r.y & 0xffff0000u));
}

// kRoute: 0 = routed dY one column at a time (any h); otherwise four
// columns per load (h % 4 == 0, aligned inputs), bit 0: MAX routing by
// argmax, bit 1: act_pre mask.  Each variant loads only what it uses, so no
// load sits behind a branch.
template <class T, int QB, int kRoute>
__global__ void __launch_bounds__(kDwThreads) k_bwd_dw(DwArgs a) {
  constexpr bool kVec = kRoute != 0, kArg = (kRoute & 1) != 0, kMask = (kRoute & 2) != 0;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  constexpr int TM = kDwTM;
  static_assert(TM == 32 && kDwThreads == 512, "4x4 staging blocks: 8 tuple groups per tile");
  const int K16 = a.K16, hn = a.hn, h = a.R.h;
  const int lane = __lane_id();
  const int w = threadIdx.x / 64;
  const int tid = threadIdx.x;
  const int nrb = K16 / 16, ncb = a.ncb;                   // ncb divides 8
  const int wu = __builtin_amdgcn_readfirstlane(w);
  const int cb = wu % ncb, rb0 = wu / ncb, rstep = 8 / ncb;  // this wave's blocks: (rb0 + rstep q, cb)
  const int bufsz = (K16 + 16 * ncb) * kDwTS;               // floats per buffer
  float* lds = reinterpret_cast<float*>(smem);
  const int64_t bidx = blockIdx.x;
  const int64_t tb = (a.ntiles * bidx) / a.nunits, te = (a.ntiles * (bidx + 1)) / a.nunits;

  // staging work of this thread: X blocks i = tid, tid + 512 (4 tuples x 4
  // columns each; column chunk kc = i % (K16/4), tuple group i / (K16/4)),
  // and the dY block tid < 2 * 16 ncb (column chunk tid % (4 ncb), tuple
  // group tid / (4 ncb))
  const int kcs = K16 / 4, ncs = 4 * ncb;
  const bool dy_on = tid < 8 * ncs;
  const int dnc = tid % ncs, dtg = tid / ncs;
  constexpr int NXB = 2;                                   // X blocks per thread (K16 <= 512)
  float4 xr[NXB][4];
  // Fixed per-thread load plan.  Every load is issued unconditionally from
  // a clamped, valid address and the value is zeroed afterwards where it
  // lies outside the tile or the columns (a load behind a branch makes the
  // compiler wait for it at the join).  Row and group numbers are loaded
  // one tile ahead of the data that they address.
  const char* xsrc[NXB];
  int xstride[NXB];
  const int32_t* xrows[NXB];
  bool xon[NXB];
#pragma unroll
  for (int bi = 0; bi < NXB; ++bi) {
    const int i = tid + bi * kDwThreads;
    const int kc = i % kcs, tg = i / kcs;
    const int el = 4 * kc;
    const int elc = min(el, a.K - 4);
    int j = 0;
#pragma unroll
    for (int q = 1; q < kMaxAtoms; ++q)
      if (q < a.at.k && elc >= a.at.koff[q]) j = q;
    xsrc[bi] = reinterpret_cast<const char*>(static_cast<const T*>(a.at.emb[j]) + (elc - a.at.koff[j]));
    xstride[bi] = a.at.d[j] * (int)sizeof(T);
    xrows[bi] = a.at.rows[j];
    xon[bi] = tg < 8 && el < a.K;
  }
  int32_t rn[NXB][4], gn[4], gn_prev[4];
  auto fetch_idx = [&](int64_t t) {
    const int64_t e0 = t * TM;
    const int nv = (int)min<int64_t>(TM, a.E - e0);
#pragma unroll
    for (int bi = 0; bi < NXB; ++bi) {
      const int tg = min((tid + bi * kDwThreads) / kcs, 7);
#pragma unroll
      for (int r = 0; r < 4; ++r) rn[bi][r] = xrows[bi][e0 + min(4 * tg + r, nv - 1)];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) gn[r] = a.R.tuple_group[e0 + min(4 * min(dtg, 7) + r, nv - 1)];
  };
  auto keep_groups = [&]() {                                // group numbers of the tile just fetched
#pragma unroll
    for (int r = 0; r < 4; ++r) gn_prev[r] = gn[r];
  };
  // data loads of a tile: raw values only; they are selected (tile rows,
  // columns, MAX routing, act_pre mask) when stashed, after the products of
  // the current tile, so that the loads stay in flight meanwhile
  float4 draw[4];
  int4 amraw[4];
  uint32_t mraw[4];
  auto fetch_data = [&](int64_t t) {
    const int64_t e0 = t * TM;
    const int nv = (int)min<int64_t>(TM, a.E - e0);
#pragma unroll
    for (int bi = 0; bi < NXB; ++bi)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        xr[bi][r] = dw_load4<T>(reinterpret_cast<const T*>(xsrc[bi] + (int64_t)rn[bi][r] * xstride[bi]));
    if constexpr (kVec) {
      const int nc = min(4 * dnc, hn - 4);                    // hn is a multiple of 4 here
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t e = e0 + min(4 * dtg + r, nv - 1);
        const int64_t o = (int64_t)gn[r] * h + a.n0 + nc;
        draw[r] = *reinterpret_cast<const float4*>(a.R.dA + o);
        if constexpr (kArg) amraw[r] = *reinterpret_cast<const int4*>(a.R.argmax + o);
        if constexpr (kMask) mraw[r] = *reinterpret_cast<const uint32_t*>(a.R.mask + e * h + a.n0 + nc);
      }
    }
  };
  // registers -> transposed LDS tiles of buffer b (tile t)
  auto stash = [&](int b, int64_t t) {
    const int64_t e0 = t * TM;
    const int nv = (int)min<int64_t>(TM, a.E - e0);
    float* XT = lds + b * bufsz;
    float* DT = XT + K16 * kDwTS;
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int bi = 0; bi < NXB; ++bi) {
      const int i = tid + bi * kDwThreads;
      const int kc = i % kcs, tg = i / kcs;
      if (tg < 8) {
        float4 x[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = xon[bi] && 4 * tg + r < nv ? xr[bi][r] : z4;
        *reinterpret_cast<float4*>(XT + (4 * kc + 0) * kDwTS + 4 * tg) = make_float4(x[0].x, x[1].x, x[2].x, x[3].x);
        *reinterpret_cast<float4*>(XT + (4 * kc + 1) * kDwTS + 4 * tg) = make_float4(x[0].y, x[1].y, x[2].y, x[3].y);
        *reinterpret_cast<float4*>(XT + (4 * kc + 2) * kDwTS + 4 * tg) = make_float4(x[0].z, x[1].z, x[2].z, x[3].z);
        *reinterpret_cast<float4*>(XT + (4 * kc + 3) * kDwTS + 4 * tg) = make_float4(x[0].w, x[1].w, x[2].w, x[3].w);
      }
    }
    if (dy_on) {
      float4 d[4];
      const int n = 4 * dnc;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int tr = 4 * dtg + r;
        if constexpr (kVec) {
          const int32_t ei = (int32_t)(e0 + min(tr, nv - 1));
          // keep bits of the 4 columns (integer arithmetic: no branches)
          uint32_t keep = (tr < nv && n < hn) ? 15u : 0u;
          if constexpr (kArg) {
            const int4 am = amraw[r];
            keep &= (uint32_t)(am.x == ei) | ((uint32_t)(am.y == ei) << 1) | ((uint32_t)(am.z == ei) << 2) |
                    ((uint32_t)(am.w == ei) << 3);
          }
          if constexpr (kMask) {
            const uint32_t m = mraw[r];
            keep &= (uint32_t)((m & 0xffu) != 0) | ((uint32_t)((m & 0xff00u) != 0) << 1) |
                    ((uint32_t)((m & 0xff0000u) != 0) << 2) | ((uint32_t)((m & 0xff000000u) != 0) << 3);
          }
          const float4 v = draw[r];
          d[r] = make_float4((keep & 1u) ? v.x : 0.0f, (keep & 2u) ? v.y : 0.0f, (keep & 4u) ? v.z : 0.0f,
                             (keep & 8u) ? v.w : 0.0f);
        } else {                                              // any h: one column at a time
          float t4[4] = {0.f, 0.f, 0.f, 0.f};
          if (tr < nv)
            for (int u = 0; u < 4; ++u)
              if (n + u < hn) t4[u] = route(a.R, e0 + tr, gn_prev[r], a.n0 + n + u);
          d[r] = make_float4(t4[0], t4[1], t4[2], t4[3]);
        }
      }
      *reinterpret_cast<float4*>(DT + (4 * dnc + 0) * kDwTS + 4 * dtg) = make_float4(d[0].x, d[1].x, d[2].x, d[3].x);
      *reinterpret_cast<float4*>(DT + (4 * dnc + 1) * kDwTS + 4 * dtg) = make_float4(d[0].y, d[1].y, d[2].y, d[3].y);
      *reinterpret_cast<float4*>(DT + (4 * dnc + 2) * kDwTS + 4 * dtg) = make_float4(d[0].z, d[1].z, d[2].z, d[3].z);
      *reinterpret_cast<float4*>(DT + (4 * dnc + 3) * kDwTS + 4 * dtg) = make_float4(d[0].w, d[1].w, d[2].w, d[3].w);
    }
  };

  f32x4 acc[QB];
#pragma unroll
  for (int q = 0; q < QB; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  float4 dbacc = make_float4(0.f, 0.f, 0.f, 0.f);          // dY column sums of this thread's dY block
  const int lq = 8 * (lane >> 4), lm = lane & 15;

  // the prefetches run unconditionally (the last tiles are fetched again,
  // harmlessly): a skipped load on one path makes the compiler wait for
  // every load where the paths meet
  const int64_t tl = te - 1;
  fetch_idx(tb);
  fetch_data(tb);
  keep_groups();
  fetch_idx(min(tb + 1, tl));
  stash(0, tb);
  __syncthreads();
  for (int64_t t = tb; t < te; ++t) {
    const int b = (int)((t - tb) & 1);
    fetch_data(min(t + 1, tl));
    keep_groups();
    fetch_idx(min(t + 2, tl));
    const float* XT = lds + b * bufsz;
    const float* DT = XT + K16 * kDwTS;
#pragma unroll
    for (int grp = 0; grp < 2; ++grp) {
      const int to = lq + 4 * grp;                            // tuples to .. to+3 of this lane
      const f32x4 bb = *reinterpret_cast<const f32x4*>(DT + (16 * cb + lm) * kDwTS + to);
      const float* xa = XT + (16 * rb0 + lm) * kDwTS + to;
      const int astep = 16 * rstep * kDwTS;
      // the operand of block q + 1 is read while block q is multiplied
      // blocks past the last row block multiply a repeated (valid) operand
      // into accumulators that are never written out
      const int qlast = (nrb - 1 - rb0) / rstep;
      f32x4 an = *reinterpret_cast<const f32x4*>(xa);
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        const f32x4 aa = an;
        if (q + 1 < QB) an = *reinterpret_cast<const f32x4*>(xa + min(q + 1, qlast) * astep);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(aa[u], bb[u], acc[q], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (dy_on) {                                              // db: this thread's dY block, tuple order
      const float* d = DT + (4 * dnc) * kDwTS + 4 * dtg;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        dbacc.x += d[0 * kDwTS + r];
        dbacc.y += d[1 * kDwTS + r];
        dbacc.z += d[2 * kDwTS + r];
        dbacc.w += d[3 * kDwTS + r];
      }
    }
    stash(b ^ 1, min(t + 1, tl));
    __syncthreads();
  }
  // per-block partials
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    const int rb = rb0 + rstep * q;
    if (rb < nrb) {
      const int n = cb * 16 + lm;
      if (n < hn) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = rb * 16 + 4 * (lane >> 4) + i;
          a.part[(bidx * K16 + k) * h + a.n0 + n] = acc[q][i];
        }
      }
    }
  }
  // db partial: the 8 tuple groups of each column, in order
  float* dbs = lds;                                           // [8][16 ncb] (the tiles are no longer read)
  if (dy_on) {
    const float v[4] = {dbacc.x, dbacc.y, dbacc.z, dbacc.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) dbs[dtg * ncs * 4 + 4 * dnc + u] = v[u];
  }
  __syncthreads();
  if (tid < hn) {
    float sdb = 0.0f;
    for (int g8 = 0; g8 < 8; ++g8) sdb += dbs[g8 * ncs * 4 + tid];
    a.dbpart[bidx * h + a.n0 + tid] = sdb;
  }
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
  int K = 0, K16 = 0, hn = 0, ncb = 1;
  int64_t dw_tiles = 0, dw_units = 0;
  size_t dw_lds = 0;
  size_t ws_mask = 0, ws_fwsw = 0, ws_part = 0, ws_dbpart = 0, ws_dA = 0, ws_own = 0, total = 0;
  int kv = 0;                // MAX: atoms dW takes per tuple (the others are keyed by the group column)
  size_t ws_gkpart = 0;
  bool xs_dw = false;        // dW through the per-group sums (SUM / MEAN, affine)
  LinBwdPlan lin;
};

BwdPlan plan_bwd(const relnn_index* idx, const relnn_layer_desc* L, const FwdPlan& F) {
  BwdPlan p;
  p.F = F;
  p.K = F.K;
  p.K16 = (int)round_up(F.K, 16);
  // columns per pass: at most 8 column blocks, 16 accumulator blocks
  // per wave, and two buffers of (K16 + columns) transposed rows in LDS
  const int nrb = p.K16 / 16;
  int ncb = 8;    // a power of two (each wave keeps one column block), at most 16 blocks per wave
  while (ncb > 1 && (16 * (ncb / 2) >= L->h || nrb * ncb > 128 ||
                     (size_t)2 * (p.K16 + 16 * ncb) * kDwTS * 4 > 160 * 1024))
    ncb /= 2;
  p.ncb = ncb;
  p.hn = std::min(L->h, 16 * ncb);
  const int64_t E = idx->E;
  p.xs_dw = L->act_pre == RELNN_ACT_NONE && L->agg != RELNN_MAX;
  p.dw_tiles = cdiv(E, kDwTM);
  p.dw_units = std::max<int64_t>(1, std::min<int64_t>(p.dw_tiles, num_cus()));
  p.dw_lds = (size_t)2 * (p.K16 + 16 * p.ncb) * kDwTS * 4;
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
  p.ws_own = off;                                        // MAX: ownership bits [E][ceil(h / 32)]
  if (L->agg == RELNN_MAX) off += round_up(std::max<int64_t>(E, 1) * cdiv(L->h, 32) * 4, 256);
  // MAX without act_pre: trailing atoms keyed by the group column leave the
  // per-tuple dW for a product over the groups (their routed gradients add
  // up to dA_g per group)
  p.kv = L->k;
  if (L->agg == RELNN_MAX && L->act_pre == RELNN_ACT_NONE)
    while (p.kv > 1 && idx->atom_gk[p.kv - 1]) --p.kv;
  p.ws_gkpart = off;
  if (p.kv < L->k) {
    int64_t nf = 0;
    for (int j = p.kv; j < L->k; ++j) nf = std::max(nf, gk_dw_ws_floats(idx->G, L->d[j], L->h));
    off += round_up(nf * 4, 256);
  }
  p.lin = plan_lin_bwd(idx, L, off, p.xs_dw);
  p.total = p.lin.total;
  return p;
}

template <class KernelT>
void allow_lds(KernelT k, size_t bytes);

// accumulator blocks per wave: 8 or 16 (the plan keeps nblk <= 128)
template <class T, int QB, int kRoute>
void launch_dw_q(const DwArgs& d, int64_t units, size_t lds, hipStream_t s) {
  allow_lds(k_bwd_dw<T, QB, kRoute>, lds);
  k_bwd_dw<T, QB, kRoute><<<(unsigned)units, kDwThreads, lds, s>>>(d);
  RELNN_LAUNCHED();
}
template <class T, int QB>
void launch_dw_r(const DwArgs& d, int64_t units, size_t lds, hipStream_t s) {
  const int route = !d.vec4 ? 0 : (d.R.agg == RELNN_MAX ? 1 : 0) | (d.R.mask ? 2 : 0);
  switch (route) {
    case 1: launch_dw_q<T, QB, 1>(d, units, lds, s); break;
    case 2: launch_dw_q<T, QB, 2>(d, units, lds, s); break;
    case 3: launch_dw_q<T, QB, 3>(d, units, lds, s); break;
    default: launch_dw_q<T, QB, 0>(d, units, lds, s); break;
  }
}
template <class T>
void launch_dw(const DwArgs& d, int64_t nblk, int64_t units, size_t lds, hipStream_t s) {
  RELNN_REQUIRE(nblk <= 128, RELNN_E_HIP, "internal: %lld dW blocks", (long long)nblk);
  if (nblk <= 64)
    launch_dw_r<T, 8>(d, units, lds, s);
  else
    launch_dw_r<T, 16>(d, units, lds, s);
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
      d.at.k = P.kv;                          // per tuple: atoms 0 .. kv-1, the leading rows of dW
      int Kv = 0;
      for (int j = 0; j < P.kv; ++j) Kv += L->d[j];
      d.rows = idx->rows;
      d.E = E;
      d.K = Kv;
      d.K16 = (int)round_up(Kv, 16);
      d.R = R;
      d.ntiles = P.dw_tiles;
      d.nunits = P.dw_units;
      d.part = reinterpret_cast<float*>(w + P.ws_part);
      d.dbpart = reinterpret_cast<float*>(w + P.ws_dbpart);
      const int64_t nblk = (d.K16 / 16) * P.ncb;
      d.ncb = P.ncb;
      d.vec4 = h % 4 == 0 && ((uintptr_t)dA & 15) == 0 && ((uintptr_t)argmax & 15) == 0;
      RELNN_REQUIRE(P.K16 <= 512, RELNN_E_UNSUPPORTED, "dense dW: K = %d too wide", P.K);
      for (int n0 = 0; n0 < h; n0 += P.hn) {
        d.n0 = n0;
        d.hn = std::min(P.hn, h - n0);
        KTimer tm("bwd_dw", s);
        if (L->dtype == RELNN_BF16)
          launch_dw<__bf16>(d, nblk, P.dw_units, P.dw_lds, s);
        else
          launch_dw<float>(d, nblk, P.dw_units, P.dw_lds, s);
      }
      k_dw_reduce<<<grid_for((int64_t)Kv * h + h), 256, 0, s>>>(d.part, d.dbpart, P.dw_units, Kv, d.K16, h, dW,
                                                                  db, accum ? 1 : 0);
      RELNN_LAUNCHED();
      for (int j = P.kv, koff = Kv; j < L->k; koff += L->d[j], ++j) {
        KTimer tm("bwd_dw", s);
        gk_dw(idx, j, emb[j], L->dtype == RELNN_BF16, L->d[j], h, dA, dW + (int64_t)koff * h, accum,
              reinterpret_cast<float*>(w + P.ws_gkpart), s);
      }
    }

    // dz_j for every atom, in body order (through the per-row sums of dY)
    uint32_t* own = nullptr;
    const int nw = (int)cdiv(h, 32);
    if (L->agg == RELNN_MAX) {
      own = reinterpret_cast<uint32_t*>(w + P.ws_own);
      k_own_bits<<<grid_for(E * nw), 256, 0, s>>>(argmax, idx->tuple_group, E, h, nw, own);
      RELNN_LAUNCHED();
    }
    lin_bwd_dx(idx, L, P.lin, W, dA, own, nw, R.mask, demb, w, s);
  });
}
