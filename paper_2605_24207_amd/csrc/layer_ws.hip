// Forward layer, weight-stationary persistent kernel (the fast path).
//
// Same arithmetic as the tile kernel of layer_fwd.hip (gather -> Linear on
// the matrix cores -> per-group reduce -> act_post), organised for gfx950:
//
//  * one block per CU, persistent over a contiguous range of TM-tuple tiles;
//  * NCW = h/32 "compute" waves each hold their 32 output columns of W in
//    VGPRs for the whole kernel (loaded once) and run 32x32 MFMAs
//    (f32 32x32x2 or bf16 32x32x16) with the A operand read from LDS;
//  * 4 "gather" waves stream the joined rows of tile t+1 into the other LDS
//    buffer with 16-byte loads while the compute waves work on tile t, and
//    reduce tile t-1 per group from the FP32 result tile in LDS;
//  * a group that spans tiles is accumulated inside the block (Kahan
//    compensated sum, or max with the earliest maximiser), so a block leaves
//    at most two partials: for the groups cut by its range ends.  k_fixup
//    combines those in block order.
// One __syncthreads per tile separates the stages.
#include <type_traits>

#include "layer_fwd.hpp"

namespace relnn {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kGatherWaves = 4;
constexpr int kHMax = 128;

struct WsArgs {
  Atoms at;
  const int32_t* rows;
  int64_t E;
  const int64_t* E_dev;      // if set: E (and the tile count) come from device memory
  int K, h;
  int64_t ntiles, nunits;
  const void* Wsw;
  const float* b;
  int act_pre;
  Seg sg;
  Sink sink;
  float* carry;
  int32_t* carry_arg;
};

template <class T>
struct WsCfg;
template <>
struct WsCfg<float> {
  static constexpr int TM = 32;    // tuples per tile (one 32-row MFMA block)
  static constexpr int KQ = 8;     // k granularity of the A read (float4 per lane group)
  static constexpr int EPC = 4;
  static constexpr int XPAD = 4;
};
template <>
struct WsCfg<__bf16> {
  static constexpr int TM = 32;
  static constexpr int KQ = 16;
  static constexpr int EPC = 8;
  static constexpr int XPAD = 8;
};

__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
  const float y = x - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}

// W in the per-wave fragment order of the kernel below.
// f32: fragment ks of column block cw, lane l holds W[k][32 cw + l % 32]
//      with k = 8 (ks / 4) + 4 (l / 32) + ks % 4.
// bf16: lane l holds W[16 ks + 8 (l / 32) + i][32 cw + l % 32], i = 0..7.
__global__ void k_ws_swizzle_f32(const float* __restrict__ W, int K, int KP, int h, float* __restrict__ out) {
  const int nks = KP / 2;
  const int64_t total = (int64_t)(h / 32) * nks * 64;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int lane = (int)(i & 63);
    const int64_t f = i >> 6;
    const int ks = (int)(f % nks);
    const int cw = (int)(f / nks);
    const int k = 8 * (ks / 4) + 4 * (lane / 32) + ks % 4;
    out[i] = k < K ? W[(int64_t)k * h + cw * 32 + lane % 32] : 0.0f;
  }
}

// f32, 16-column slices: fragment ks of slice cw, lane l holds
// W[16 (ks / 4) + 4 (l / 16) + ks % 4][16 cw + l % 16].
__global__ void k_ws_swizzle_f16c(const float* __restrict__ W, int K, int KP, int h, float* __restrict__ out) {
  const int nks = KP / 4;
  const int64_t total = (int64_t)(h / 16) * nks * 64;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int lane = (int)(i & 63);
    const int64_t f = i >> 6;
    const int ks = (int)(f % nks);
    const int cw = (int)(f / nks);
    const int k = 16 * (ks / 4) + 4 * (lane / 16) + ks % 4;
    out[i] = k < K ? W[(int64_t)k * h + cw * 16 + lane % 16] : 0.0f;
  }
}

__global__ void k_ws_swizzle_bf16(const __bf16* __restrict__ W, int K, int KP, int h, __bf16* __restrict__ out) {
  const int nks = KP / 16;
  const int64_t total = (int64_t)(h / 32) * nks * 64 * 8;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(i & 7);
    const int lane = (int)((i >> 3) & 63);
    const int64_t f = i >> 9;
    const int ks = (int)(f % nks);
    const int cw = (int)(f / nks);
    const int k = 16 * ks + 8 * (lane / 32) + e;
    out[i] = k < K ? W[(int64_t)k * h + cw * 32 + lane % 32] : (__bf16)0.0f;
  }
}

// Per-group reduce of the FP32 result tile Y (rows = tuples of tile t) by
// threads tid = 0..nthr-1 of the block; keeps the block's open group in
// open_* (double-buffered by tile parity) and writes finished groups or the
// partials of groups cut by the block's range ends.
__device__ __forceinline__ void ws_reduce(const WsArgs& a, int64_t t, const float* Y, int YS, int TM, int64_t tb,
                                          int64_t range_lo, int64_t range_hi, float* open_s, float* open_c,
                                          int32_t* open_a, int tid, int nthr) {
  const int h = a.h;
  const int64_t e0 = t * TM;
  const int nv = (int)min<int64_t>(TM, a.E - e0);
  const int64_t s_first = a.sg.seg_of[e0];
  const int64_t s_last = a.sg.seg_of[e0 + nv - 1];
  const int rd = (int)((t - tb) & 1), wr = rd ^ 1;
  const int64_t work = (s_last - s_first + 1) * h;
  const bool maxagg = a.sink.agg == RELNN_MAX;
  for (int64_t p = tid; p < work; p += nthr) {
    const int64_t s = s_first + p / h;
    const int c = (int)(p - (p / h) * h);
    const int64_t g0 = a.sg.offsets[s], g1 = a.sg.offsets[s + 1];
    const int r0 = (int)(max(g0, e0) - e0);
    const int r1 = (int)(min(g1, e0 + nv) - e0);
    float S, Cc = 0.0f;
    int32_t am = -1;
    const float bc = a.b ? a.b[c] : 0.0f;
    if (maxagg) {
      S = act_apply(a.act_pre, Y[r0 * YS + c] + bc);
      am = (int32_t)(e0 + r0);
      for (int r = r0 + 1; r < r1; ++r) {
        const float y = act_apply(a.act_pre, Y[r * YS + c] + bc);
        if (y > S) {
          S = y;
          am = (int32_t)(e0 + r);
        }
      }
    } else {
      S = 0.0f;
      for (int r = r0; r < r1; ++r) S += act_apply(a.act_pre, Y[r * YS + c] + bc);
    }
    if (s == s_first && g0 < e0 && t > tb) {      // continues the block's open group
      if (maxagg) {
        const float ov = open_s[rd * kHMax + c];
        if (!(S > ov)) {
          S = ov;
          am = open_a[rd * kHMax + c];
        }
      } else {
        float os = open_s[rd * kHMax + c], oc = open_c[rd * kHMax + c];
        kahan_add(os, oc, S);
        S = os;
        Cc = oc;
      }
    }
    if (g1 > e0 + nv) {                          // continues past this tile
      if (e0 + nv < range_hi) {
        open_s[wr * kHMax + c] = S;
        open_c[wr * kHMax + c] = Cc;
        open_a[wr * kHMax + c] = am;
      } else {
        const int slot = (g0 < range_lo) ? 0 : 1;
        a.carry[((int64_t)blockIdx.x * 2 + slot) * h + c] = S - Cc;
        if (a.carry_arg) a.carry_arg[((int64_t)blockIdx.x * 2 + slot) * h + c] = am;
      }
    } else if (g0 >= range_lo) {                  // complete inside this block
      sink_write(a.sink, s, c, h, S - Cc, am, (int32_t)(g1 - g0));
    } else {                                      // cut by the range start
      a.carry[((int64_t)blockIdx.x * 2 + 0) * h + c] = S - Cc;
      if (a.carry_arg) a.carry_arg[((int64_t)blockIdx.x * 2 + 0) * h + c] = am;
    }
  }
}

// KS = 1: one compute wave per 32 output columns.  KS = 2: two, each over
// half of K; both add their partial tile into the zeroed LDS result with
// float atomics -- two addends commute exactly, so the sum is deterministic.
template <class T, int KP, int KS>
__global__ void __launch_bounds__((4 * KS + kGatherWaves) * 64) k_fwd_ws(WsArgs a) {
  if (a.E_dev) {
    a.E = *a.E_dev;
    a.ntiles = (a.E + WsCfg<T>::TM - 1) / WsCfg<T>::TM;
    a.sg.n = a.E;
  }
  using C = WsCfg<T>;
  constexpr int TM = C::TM;
  constexpr int XS = KP + C::XPAD;
  constexpr int CPR = KP / C::EPC;                          // 16-byte chunks per row
  constexpr int CH = (TM * CPR + 255) / 256;                // chunks per gather thread
  constexpr bool BF = sizeof(T) == 2;
  constexpr int NKS = (BF ? KP / 16 : KP / 2) / KS;         // MFMA k steps per compute wave
  constexpr int NRB = TM / 32;                              // 32-row blocks per tile
  constexpr int KW = KP / KS;                               // k range of one compute wave

  extern __shared__ __attribute__((aligned(16))) char smem[];
  T* Xb = reinterpret_cast<T*>(smem);                                        // [2][TM][XS]
  float* Yb = reinterpret_cast<float*>(smem + 2 * TM * XS * sizeof(T));      // [2][TM][YS]
  const int h = a.h;
  const int YS = h + 4;
  float* open_s = Yb + 2 * TM * YS;          // [2][kHMax] running sums of the open group
  float* open_c = open_s + 2 * kHMax;        // [2][kHMax] Kahan compensations
  int32_t* open_a = reinterpret_cast<int32_t*>(open_c + 2 * kHMax);   // [2][kHMax] argmax

  const int ncb = h / 32;
  const int ncw = ncb * KS;
  const int wave = threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  const bool compute = wave < ncw;
  const int cb = wave % ncb;                 // column block of a compute wave
  const int kh = wave / ncb;                 // its k range
  const int gt = threadIdx.x - ncw * 64;     // gather thread id (0..255) if !compute

  const int64_t nb = a.nunits;
  const int64_t bidx = blockIdx.x;
  const int64_t tb = (a.ntiles * bidx) / nb;
  const int64_t te = (a.ntiles * (bidx + 1)) / nb;
  const int64_t range_lo = tb * TM;
  const int64_t range_hi = min<int64_t>(te * TM, a.E);

  // ---- compute waves: W fragments to registers, once
  typedef typename std::conditional<BF, bf16x8, float>::type WFrag;
  WFrag w[NKS];
  if (compute) {
    const WFrag* src = reinterpret_cast<const WFrag*>(a.Wsw) + ((int64_t)cb * NKS * KS + kh * NKS) * 64;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) w[ks] = src[ks * 64 + lane];
  }

  // gather: issue the 16-byte loads of tile t (kept in registers) ...
  auto gather_load = [&](int64_t t, uint4 (&v)[CH], int (&dst)[CH]) {
    const int64_t e0 = t * TM;
    const int nv = (int)min<int64_t>(TM, a.E - e0);
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int i = gt + q * 256;
      v[q] = make_uint4(0, 0, 0, 0);
      dst[q] = -1;
      if (i < TM * CPR) {
        const int r = i / CPR;
        const int c = i - r * CPR;
        const int el = c * C::EPC;
        dst[q] = r * XS + el;
        if (r < nv && el < a.K) {
          int j = 0;
#pragma unroll
          for (int u = 1; u < kMaxAtoms; ++u)
            if (u < a.at.k && el >= a.at.koff[u]) j = u;
          const int64_t row = a.at.rows[j][e0 + r];
          v[q] = *reinterpret_cast<const uint4*>(static_cast<const T*>(a.at.emb[j]) + row * a.at.d[j] +
                                                  (el - a.at.koff[j]));
        }
      }
    }
  };
  // Load + store in batches of 4 chunks: few registers, for the variants
  // whose W slice already fills most of the register file.
  auto gather_copy = [&](int64_t t, T* Xd) {
    const int64_t e0 = t * TM;
    const int nv = (int)min<int64_t>(TM, a.E - e0);
    // Opaque copy of the thread id: stops the compiler from hoisting the
    // per-chunk index math of all tiles out of the tile loop (which would
    // pin dozens of registers next to the W slice).
    int g = gt;
    asm volatile("" : "+v"(g));
#pragma unroll
    for (int q0 = 0; q0 < CH; q0 += 4) {
      uint4 v[4];
      int dst[4];
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int i = g + (q0 + qq) * 256;
        v[qq] = make_uint4(0, 0, 0, 0);
        dst[qq] = -1;
        if (q0 + qq < CH && i < TM * CPR) {
          const int r = i / CPR;
          const int c = i - r * CPR;
          const int el = c * C::EPC;
          dst[qq] = r * XS + el;
          if (r < nv && el < a.K) {
            int j = 0;
#pragma unroll
            for (int u = 1; u < kMaxAtoms; ++u)
              if (u < a.at.k && el >= a.at.koff[u]) j = u;
            const int64_t row = a.at.rows[j][e0 + r];
            v[qq] = *reinterpret_cast<const uint4*>(static_cast<const T*>(a.at.emb[j]) + row * a.at.d[j] +
                                                     (el - a.at.koff[j]));
          }
        }
      }
#pragma unroll
      for (int qq = 0; qq < 4; ++qq)
        if (dst[qq] >= 0) *reinterpret_cast<uint4*>(Xd + dst[qq]) = v[qq];
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  // ... and store them into an LDS tile buffer.
  auto gather_store = [&](T* Xd, const uint4 (&v)[CH], const int (&dst)[CH]) {
#pragma unroll
    for (int q = 0; q < CH; ++q)
      if (dst[q] >= 0) *reinterpret_cast<uint4*>(Xd + dst[q]) = v[q];
  };

  auto reduce = [&](int64_t t, const float* Y) {
    ws_reduce(a, t, Y, YS, TM, tb, range_lo, range_hi, open_s, open_c, open_a, gt, 256);
  };

  if (tb >= te) return;
  if (!compute) {
    gather_copy(tb, Xb);
    if constexpr (KS > 1)
      for (int i = gt; i < 2 * TM * YS; i += 256) Yb[i] = 0.0f;
  }
  __syncthreads();
  for (int64_t t = tb; t <= te; ++t) {
    const int buf = (int)((t - tb) & 1);
    T* X = Xb + buf * TM * XS;
    float* Y = Yb + buf * TM * YS;
    if (compute) {
      if (t < te) {
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) {
          f32x16 acc;
#pragma unroll
          for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
          const T* xr = X + (rb * 32 + (lane & 31)) * XS + kh * KW;
          // A operands one step ahead of the MFMAs; the scheduling barrier
          // keeps the compiler from hoisting every LDS read (and its
          // registers) to the top of the unrolled loop.
          if constexpr (BF) {
            bf16x8 cur = *reinterpret_cast<const bf16x8*>(xr + 8 * (lane >> 5));
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks) {
              bf16x8 nxt = cur;
              if (ks + 1 < NKS) nxt = *reinterpret_cast<const bf16x8*>(xr + 16 * (ks + 1) + 8 * (lane >> 5));
              acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cur, w[ks], acc, 0, 0, 0);
              __builtin_amdgcn_sched_barrier(0);
              cur = nxt;
            }
          } else {
            f32x4 cur = *reinterpret_cast<const f32x4*>(xr + 4 * (lane >> 5));
#pragma unroll
            for (int m = 0; m < NKS / 4; ++m) {
              f32x4 nxt = cur;
              if (m + 1 < NKS / 4) nxt = *reinterpret_cast<const f32x4*>(xr + 8 * (m + 1) + 4 * (lane >> 5));
#pragma unroll
              for (int u = 0; u < 4; ++u)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(cur[u], w[4 * m + u], acc, 0, 0, 0);
              __builtin_amdgcn_sched_barrier(0);
              cur = nxt;
            }
          }
          const int col = cb * 32 + (lane & 31);
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int row = rb * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            if constexpr (KS == 1)
              Y[row * YS + col] = acc[v];
            else
              atomicAdd(&Y[row * YS + col], acc[v]);
          }
        }
      }
    } else {
      const bool more = t + 1 < te;
      uint4 v[CH];
      int dst[CH];
      // f32 tiles are MFMA-bound: store the next tile first and keep few
      // registers live; bf16 tiles are load-bound: reduce while loads fly.
      constexpr bool overlap = BF;
      if (more) gather_load(t + 1, v, dst);
      if (more && !overlap) gather_store(Xb + (buf ^ 1) * TM * XS, v, dst);
      if (t > tb) {
        float* Yp = Yb + (buf ^ 1) * TM * YS;
        reduce(t - 1, Yp);
        if constexpr (KS > 1) {        // zero it for the partial sums of tile t + 1
          for (int i = gt; i < TM * YS; i += 256) Yp[i] = 0.0f;
        }
      }
      if constexpr (overlap) {
        if (more) gather_store(Xb + (buf ^ 1) * TM * XS, v, dst);
      }
    }
    __syncthreads();
  }
}


// FP32 variant: every wave gathers, multiplies and reduces.  A wave owns 16
// output columns (its W slice, KP/4 VGPRs, stays in registers) and runs
// f32 16x16x4 MFMAs over the 32 rows of a tile; the 16-byte loads of tile
// t+1 are issued before the MFMA loop of tile t and land in the other LDS
// buffer after it, so HBM latency hides behind matrix work.
// A lane holds A[row = lane % 16][k = lane / 16]; with one float4 LDS read
// per lane group the four k of MFMA step 4m+u map to physical columns
// 16m + 4 (lane / 16) + u.  W is swizzled to match (k_ws_swizzle_f16c).
template <int KP, int NW>
__global__ void __launch_bounds__(NW * 64) k_fwd_f32(WsArgs a) {
  if (a.E_dev) {
    a.E = *a.E_dev;
    a.ntiles = (a.E + 31) / 32;
    a.sg.n = a.E;
  }
  constexpr int TM = 32;
  constexpr int XS = KP + 4;
  constexpr int CPR = KP / 4;
  constexpr int NKS = KP / 4;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  float* Xb = reinterpret_cast<float*>(smem);          // [2][TM][XS]
  float* Yb = Xb + 2 * TM * XS;                        // [2][TM][YS]
  const int h = a.h;
  const int YS = h + 4;
  float* open_s = Yb + 2 * TM * YS;
  float* open_c = open_s + 2 * kHMax;
  int32_t* open_a = reinterpret_cast<int32_t*>(open_c + 2 * kHMax);
  constexpr int nthr = NW * 64;
  constexpr int CH = (TM * CPR + nthr - 1) / nthr;     // 16-byte chunks per thread
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t nb = a.nunits, bidx = blockIdx.x;
  const int64_t tb = (a.ntiles * bidx) / nb, te = (a.ntiles * (bidx + 1)) / nb;
  const int64_t range_lo = tb * TM, range_hi = min<int64_t>(te * TM, a.E);
  if (tb >= te) return;

  float w[NKS];
  {
    const float* src = static_cast<const float*>(a.Wsw) + (int64_t)wave * NKS * 64;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) w[ks] = src[ks * 64 + lane];
  }

  uint4 v[CH];
  auto load = [&](int64_t t) {
    const int64_t e0 = t * TM;
    const int nv = (int)min<int64_t>(TM, a.E - e0);
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int i = threadIdx.x + q * nthr;
      v[q] = make_uint4(0, 0, 0, 0);
      if (i < TM * CPR) {
        const int r = i / CPR, el = (i - (i / CPR) * CPR) * 4;
        if (r < nv && el < a.K) {
          int j = 0;
#pragma unroll
          for (int u = 1; u < kMaxAtoms; ++u)
            if (u < a.at.k && el >= a.at.koff[u]) j = u;
          const int64_t row = a.at.rows[j][e0 + r];
          v[q] = *reinterpret_cast<const uint4*>(static_cast<const float*>(a.at.emb[j]) + row * a.at.d[j] +
                                                  (el - a.at.koff[j]));
        }
      }
    }
  };
  auto store = [&](float* X) {
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int i = threadIdx.x + q * nthr;
      if (i < TM * CPR) {
        const int r = i / CPR, el = (i - (i / CPR) * CPR) * 4;
        *reinterpret_cast<uint4*>(X + r * XS + el) = v[q];
      }
    }
  };

  load(tb);
  store(Xb);
  __syncthreads();
  for (int64_t t = tb; t < te; ++t) {
    const int buf = (int)((t - tb) & 1);
    const float* X = Xb + buf * TM * XS;
    float* Y = Yb + buf * TM * YS;
    const bool more = t + 1 < te;
    if (more) load(t + 1);
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      const float* xr = X + (rb * 16 + (lane & 15)) * XS + 4 * (lane >> 4);
      f32x4 cur = *reinterpret_cast<const f32x4*>(xr);
#pragma unroll
      for (int m = 0; m < NKS / 4; ++m) {
        f32x4 nxt = cur;
        if (m + 1 < NKS / 4) nxt = *reinterpret_cast<const f32x4*>(xr + 16 * (m + 1));
#pragma unroll
        for (int u = 0; u < 4; ++u)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(cur[u], w[4 * m + u], acc, 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        cur = nxt;
      }
      const int col = wave * 16 + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) Y[(rb * 16 + 4 * (lane >> 4) + i) * YS + col] = acc[i];
    }
    if (more) store(Xb + (buf ^ 1) * TM * XS);
    __syncthreads();
    ws_reduce(a, t, Y, YS, TM, tb, range_lo, range_hi, open_s, open_c, open_a, threadIdx.x, nthr);
  }
}

namespace {

template <class KernelT>
void allow_lds(KernelT k, size_t bytes) {
  RELNN_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

size_t f32_lds(int KP, int h) { return 2 * 32 * (KP + 4) * 4 + 2 * 32 * (h + 4) * 4 + 3 * 2 * kHMax * 4; }

template <int KP, int NW>
void run_f32(const WsArgs& a, hipStream_t s) {
  const size_t lds = f32_lds(KP, a.h);
  allow_lds(k_fwd_f32<KP, NW>, lds);
  KTimer tm("fwd_fused", s);
  k_fwd_f32<KP, NW><<<(unsigned)a.nunits, NW * 64, lds, s>>>(a);
  RELNN_LAUNCHED();
}

template <int KP>
void run_f32_h(const WsArgs& a, hipStream_t s) {
  switch (a.h / 16) {
    case 2: run_f32<KP, 2>(a, s); break;
    case 4: run_f32<KP, 4>(a, s); break;
    case 6: run_f32<KP, 6>(a, s); break;
    default: run_f32<KP, 8>(a, s); break;
  }
}

template <class T>
size_t ws_lds(int KP, int h) {
  const size_t TM = WsCfg<T>::TM;
  return 2 * TM * (KP + WsCfg<T>::XPAD) * sizeof(T) + 2 * TM * (h + 4) * 4 + 3 * 2 * kHMax * 4;
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

template <class T, int KP>
void run(const WsArgs& a0, hipStream_t s) {
  WsArgs a = a0;
  const size_t lds = ws_lds<T>(KP, a.h);
  // two compute waves per column block once one wave's W slice passes 96 VGPRs
  constexpr int KS = 1;
  allow_lds(k_fwd_ws<T, KP, KS>, lds);
  const int threads = ((a.h / 32) * KS + kGatherWaves) * 64;
  KTimer tm("fwd_fused", s);
  k_fwd_ws<T, KP, KS><<<(unsigned)a.nunits, threads, lds, s>>>(a);
  RELNN_LAUNCHED();
}

template <class T>
int pick_kp(int K) {
  const int steps[] = {64, 128, 256, 384};
  const int maxk = 384;
  for (int kp : steps)
    if (K <= kp && kp <= maxk) return kp;
  return 0;
}

}  // namespace

WsPlan plan_ws(int dtype, int K, int h, int64_t E) {
  WsPlan p;
  const bool bf = dtype == RELNN_BF16;
  p.KP = bf ? pick_kp<__bf16>(K) : pick_kp<float>(K);
  if (!p.KP || h % (bf ? 32 : 16) != 0 || h > kHMax) {
    p.KP = 0;
    return p;
  }
  p.TM = bf ? WsCfg<__bf16>::TM : WsCfg<float>::TM;
  p.ntiles = cdiv(E, p.TM);
  p.nunits = std::max<int64_t>(1, std::min<int64_t>(p.ntiles, num_cus()));
  p.wsw_bytes = (size_t)p.KP * h * (bf ? 2 : 4);
  p.carry_elems = (size_t)p.nunits * 2 * h;
  return p;
}

void swizzle_ws(const void* W, int dtype, int K, int KP, int h, void* out, hipStream_t s) {
  const int64_t n = (int64_t)KP * h;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 4096));
  if (dtype == RELNN_BF16)
    k_ws_swizzle_bf16<<<g, 256, 0, s>>>(static_cast<const __bf16*>(W), K, KP, h, static_cast<__bf16*>(out));
  else
    k_ws_swizzle_f16c<<<g, 256, 0, s>>>(static_cast<const float*>(W), K, KP, h, static_cast<float*>(out));
  RELNN_LAUNCHED();
}

void launch_ws(const WsPlan& p, int dtype, const FwdArgs& f, const void* Wsw, float* carry, int32_t* carry_arg,
               hipStream_t s) {
  WsArgs a{};
  a.at = f.at;
  a.rows = f.rows;
  a.E = f.E;
  a.E_dev = f.E_dev;
  a.K = f.K;
  a.h = f.h;
  a.ntiles = p.ntiles;
  a.nunits = p.nunits;
  a.Wsw = Wsw;
  a.b = f.b;
  a.act_pre = f.act_pre;
  a.sg = f.sg;
  a.sink = f.sink;
  a.carry = carry;
  a.carry_arg = carry_arg;
  if (dtype == RELNN_BF16) {
    switch (p.KP) {
      case 64: run<__bf16, 64>(a, s); break;
      case 128: run<__bf16, 128>(a, s); break;
      case 256: run<__bf16, 256>(a, s); break;
      default: run<__bf16, 384>(a, s); break;
    }
  } else {
    switch (p.KP) {
      case 64: run_f32_h<64>(a, s); break;
      case 128: run_f32_h<128>(a, s); break;
      case 256: run_f32_h<256>(a, s); break;
      default: run_f32_h<384>(a, s); break;
    }
  }
  launch_fixup(f.sg, p.TM, f.h, p.ntiles, p.nunits, f.sink, carry, carry_arg, s);
}

}  // namespace relnn
