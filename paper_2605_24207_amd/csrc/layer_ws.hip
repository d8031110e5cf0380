// Forward layer, weight-stationary persistent kernels (the fast path).
//
// Same arithmetic as the tile kernel of layer_fwd.hip (gather -> Linear on
// the matrix cores -> per-group reduce -> act_post), organised for gfx950:
//
//  * one block per CU, persistent over a contiguous range of 32-tuple tiles;
//  * the W slice of a wave stays in VGPRs for the whole kernel (loaded once);
//  * the joined rows of tile t+1 are loaded with 16-byte gathers while
//    tile t is on the matrix cores, then land in the other LDS buffer;
//  * the group structure of each tile (runs of equal group, whether the
//    first run started earlier and the last continues) is staged in LDS
//    with the prefetch, so the per-group reduce reads LDS only;
//  * a group that spans tiles is accumulated inside the block (Kahan
//    compensated sum, or max with the earliest maximiser), so a block
//    leaves at most two partials, for the groups cut by its range ends;
//    k_fixup combines those in block order.
// One __syncthreads per tile separates the stages.
//
// FP32 (k_fwd_f32): all waves alike, 16 output columns each, f32 16x16x4.
// BF16 (k_fwd_ws):  h/32 compute waves (32 columns each, bf16 32x32x16)
//                   plus 4 gather waves that load, stage and reduce.
#include "layer_fwd.hpp"

namespace relnn {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kGatherWaves = 4;
constexpr int kHMax = 128;
constexpr int kTM = 32;                  // tuples per tile, both kernels

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

// Group structure of one tile, staged in LDS.
struct TileInfo {
  int32_t nv;                // tuples in the tile
  int32_t nruns;             // runs of equal group
  int32_t prev_same;         // the first run's group started before the tile
  int32_t next_same;         // the last run's group continues after it
  int32_t rstart[kTM + 1];   // first row of each run, rstart[nruns] = nv
  int32_t rgrp[kTM];         // group of each run
};

// Running state of the group left open at the end of the previous tile
// (double-buffered by tile parity), per output column.
struct OpenState {
  float s[2][kHMax];         // sum (or max)
  float c[2][kHMax];         // Kahan compensation
  int32_t arg[2][kHMax];     // argmax (MAX)
  int32_t n[2][kHMax];       // tuples so far
  int32_t cut[2][kHMax];     // the group started before the block's range
  float bias[kHMax];         // b (zero if none), staged once per block
};

// Stages b in LDS so that the reduce issues no global load of its own
// (such a load would wait for every gather load in flight before it).
__device__ __forceinline__ void stage_bias(OpenState* op, const WsArgs& a, int tid, int nthr) {
  for (int c = tid; c < a.h; c += nthr) op->bias[c] = a.b ? a.b[c] : 0.0f;
}

__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
  const float y = x - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}

// Group ids a wave needs to stage one tile: lane r < nv holds the group of
// row r; lane 0 also holds the groups just before and after the tile (-1
// at the ends of the list).
struct SegLoad {
  int32_t g, before, after;
};

__device__ __forceinline__ SegLoad seg_load(const WsArgs& a, int64_t t) {
  const int lane = __lane_id();
  const int64_t e0 = t * kTM;
  const int nv = (int)min<int64_t>(kTM, a.E - e0);
  SegLoad L{-1, -1, -1};
  if (lane < nv) L.g = a.sg.seg_of[e0 + lane];
  if (lane == 0) {
    if (e0 > 0) L.before = a.sg.seg_of[e0 - 1];
    if (e0 + nv < a.E) L.after = a.sg.seg_of[e0 + nv];
  }
  return L;
}

// Whole wave: turns the loaded group ids into runs (ballot of run starts).
__device__ __forceinline__ void seg_stage(TileInfo* ti, const WsArgs& a, int64_t t, const SegLoad& L) {
  const int lane = __lane_id();
  const int nv = (int)min<int64_t>(kTM, a.E - t * kTM);
  const int32_t prev = __shfl_up(L.g, 1, 64);
  const bool start = lane < nv && (lane == 0 || prev != L.g);
  const uint64_t m = __ballot(start);
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int rank = __popcll(m & lt);
  if (start) {
    ti->rstart[rank] = lane;
    ti->rgrp[rank] = L.g;
  }
  const int32_t first = __shfl(L.g, 0, 64);
  const int32_t last = __shfl(L.g, nv - 1, 64);
  if (lane == 0) {
    const int nr = __popcll(m);
    ti->nv = nv;
    ti->nruns = nr;
    ti->rstart[nr] = nv;
    ti->prev_same = L.before >= 0 && L.before == first;
    ti->next_same = L.after >= 0 && L.after == last;
  }
}

// Per-group reduce of the FP32 result tile Y (rows = tuples of tile t),
// threads tid = 0..nthr-1: bias and act_pre per tuple, then SUM / MEAN /
// MAX per run; finished groups are written, the open group is carried to
// the next tile of the block, groups cut by the block's range ends leave a
// partial (slot 0: cut by the range start, slot 1: runs past the end).
template <bool kStoreOnly>
__device__ __forceinline__ void ws_reduce(const WsArgs& a, int64_t t, const float* Y, int YS, const TileInfo* ti,
                                          int64_t tb, int64_t range_hi, OpenState* op, int tid, int nthr) {
  const int h = a.h;
  const int64_t e0 = t * kTM;
  const int nv = ti->nv, nr = ti->nruns;
  const int rd = (int)((t - tb) & 1), wr = rd ^ 1;
  const bool maxagg = a.sink.agg == RELNN_MAX;
  const int64_t bidx = blockIdx.x;
  for (int p = tid; p < nr * h; p += nthr) {
    const int q = p / h;
    const int c = p - q * h;
    const int r0 = ti->rstart[q], r1 = ti->rstart[q + 1];
    const int64_t s = ti->rgrp[q];
    const float bc = op->bias[c];
    float S, Cc = 0.0f;
    int32_t am = -1;
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
    int32_t cnt = r1 - r0;
    bool cut = false;
    if (q == 0 && ti->prev_same) {
      if (t > tb) {                                // the block's open group
        if (maxagg) {
          const float ov = op->s[rd][c];
          if (!(S > ov)) {
            S = ov;
            am = op->arg[rd][c];
          }
        } else {
          float os = op->s[rd][c], oc = op->c[rd][c];
          kahan_add(os, oc, S);
          S = os;
          Cc = oc;
        }
        cnt += op->n[rd][c];
        cut = op->cut[rd][c] != 0;
      } else {
        cut = true;                                // began before the range
      }
    }
    if (q == nr - 1 && ti->next_same) {            // continues past this tile
      if (e0 + nv < range_hi) {
        op->s[wr][c] = S;
        op->c[wr][c] = Cc;
        op->arg[wr][c] = am;
        op->n[wr][c] = cnt;
        op->cut[wr][c] = cut ? 1 : 0;
      } else {
        const int slot = cut ? 0 : 1;
        a.carry[(bidx * 2 + slot) * h + c] = S - Cc;
        if (a.carry_arg) a.carry_arg[(bidx * 2 + slot) * h + c] = am;
      }
    } else if (!cut) {                             // complete inside this block
      sink_write<kStoreOnly>(a.sink, s, c, h, S - Cc, am, cnt);
    } else {                                       // cut by the range start
      a.carry[(bidx * 2 + 0) * h + c] = S - Cc;
      if (a.carry_arg) a.carry_arg[(bidx * 2 + 0) * h + c] = am;
    }
  }
}

// W in the per-wave fragment order of the BF16 kernel: fragment ks of
// column block cw, lane l holds W[16 ks + 8 (l / 32) + i][32 cw + l % 32],
// i = 0..7.
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

// W for the FP32 kernel, 16-column slices: fragment ks of slice cw, lane l
// holds W[16 (ks / 4) + 4 (l / 16) + ks % 4][16 cw + l % 16].
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

// A tile's row-major copy in LDS is moved in 16-byte chunks; chunk i is row
// i / CPR, elements (i % CPR) * EPC onwards.  Loading takes two stages so
// that no data load waits on its own row index: chunk_row reads the joined
// row of the chunk's atom a tile ahead of chunk_fetch, which reads the 16
// bytes.
struct AtomRef {
  const int32_t* rows;
  const void* emb;
  int d, koff;
};

// The atom that owns Concat column el.  Picked with compile-time indices:
// indexing the argument's arrays with a run-time value would move the whole
// argument to scratch memory.
__device__ __forceinline__ AtomRef atom_of(const Atoms& at, int el) {
  AtomRef r{at.rows[0], at.emb[0], at.d[0], 0};
  auto pick = [&](auto U) {
    constexpr int u = decltype(U)::value;
    if (u < at.k && el >= at.koff[u]) r = AtomRef{at.rows[u], at.emb[u], at.d[u], at.koff[u]};
  };
  static_assert(kMaxAtoms == 4, "one pick per atom after the first");
  pick(std::integral_constant<int, 1>{});
  pick(std::integral_constant<int, 2>{});
  pick(std::integral_constant<int, 3>{});
  return r;
}

// Both stages are branch-free: a chunk outside the tile (row >= nv) or in
// the K..KP pad reads a clamped, valid address and is zeroed when stored,
// so every thread issues the same straight run of loads.
template <class T, int CPR>
__device__ __forceinline__ int32_t chunk_row(const WsArgs& a, int64_t e0, int nv, int i) {
  constexpr int EPC = 16 / sizeof(T);
  const int r = min(i / CPR, nv - 1);
  const int el = min((i % CPR) * EPC, a.K - EPC);
  return atom_of(a.at, el).rows[e0 + r];
}

template <class T, int CPR>
__device__ __forceinline__ uint4 chunk_fetch(const WsArgs& a, int i, int32_t row) {
  constexpr int EPC = 16 / sizeof(T);
  const int el = min((i % CPR) * EPC, a.K - EPC);
  const AtomRef A = atom_of(a.at, el);
  return *reinterpret_cast<const uint4*>(static_cast<const T*>(A.emb) + (int64_t)row * A.d + (el - A.koff));
}

// Whether chunk i holds data (else it is stored as zeros).  Applied when
// the chunk is written to LDS, long after its load was issued: a select
// right after the load lets the compiler turn the load into a branch whose
// zero path must wait for every load in flight.
template <class T, int CPR>
__device__ __forceinline__ bool chunk_valid(const WsArgs& a, int nv, int i) {
  constexpr int EPC = 16 / sizeof(T);
  return i / CPR < nv && (i % CPR) * EPC < a.K;
}

// v, or zeros if !keep (masks on values: a conditional over two uint4
// lvalues would select between their addresses and keep v in scratch).
__device__ __forceinline__ uint4 keep_or_zero(bool keep, uint4 v) {
  const uint32_t m = keep ? 0xffffffffu : 0u;
  return make_uint4(v.x & m, v.y & m, v.z & m, v.w & m);
}

// LDS element offset of chunk i (-1 past the tile).
template <class T, int CPR, int XS>
__device__ __forceinline__ int chunk_dst(int i) {
  constexpr int EPC = 16 / sizeof(T);
  if (i >= kTM * CPR) return -1;
  const int r = i / CPR;
  return r * XS + (i - r * CPR) * EPC;
}

// ---------------------------------------------------------------- BF16
template <int KP>
__global__ void __launch_bounds__((4 + kGatherWaves) * 64) k_fwd_ws(WsArgs a) {
  using T = __bf16;
  if (a.E_dev) {                   // run-time size: as many units as tiles, at most the grid
    a.E = *a.E_dev;
    a.ntiles = (a.E + kTM - 1) / kTM;
    a.sg.n = a.E;
    a.nunits = max<int64_t>(1, min<int64_t>(a.nunits, a.ntiles));
    if ((int64_t)blockIdx.x >= a.nunits) return;
  }
  constexpr int TM = kTM;
  constexpr int XS = KP + 8;
  constexpr int CPR = KP / 8;                               // 16-byte chunks per row
  constexpr int CH = (TM * CPR + 255) / 256;                // chunks per gather thread
  constexpr int NKS = KP / 16;                              // MFMA k steps

  extern __shared__ __attribute__((aligned(16))) char smem[];
  T* Xb = reinterpret_cast<T*>(smem);                                        // [2][TM][XS]
  float* Yb = reinterpret_cast<float*>(smem + 2 * TM * XS * sizeof(T));      // [2][TM][YS]
  const int h = a.h;
  const int YS = h + 4;
  OpenState* op = reinterpret_cast<OpenState*>(Yb + 2 * TM * YS);
  TileInfo* tinfo = reinterpret_cast<TileInfo*>(op + 1);                     // [4]

  const int ncw = h / 32;
  const int wave = threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  const bool compute = wave < ncw;
  const int gt = threadIdx.x - ncw * 64;     // gather thread id (0..255) if !compute
  const bool stager = !compute && gt < 64;   // first gather wave stages the group runs

  const int64_t bidx = blockIdx.x;
  const int64_t tb = (a.ntiles * bidx) / a.nunits;
  const int64_t te = (a.ntiles * (bidx + 1)) / a.nunits;
  const int64_t range_hi = min<int64_t>(te * TM, a.E);
  if (tb >= te) return;
  stage_bias(op, a, threadIdx.x, blockDim.x);

  bf16x8 w[NKS];
  if (compute) {
    const bf16x8* src = reinterpret_cast<const bf16x8*>(a.Wsw) + (int64_t)wave * NKS * 64;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) w[ks] = src[ks * 64 + lane];
  }

  // gather waves: row indices two tiles ahead, data one tile ahead
  int32_t ridx[CH];
  auto load_idx = [&](int64_t t) {
    const int64_t e0 = t * TM;
    const int nv = (int)min<int64_t>(TM, a.E - e0);
#pragma unroll
    for (int q = 0; q < CH; ++q) ridx[q] = chunk_row<T, CPR>(a, e0, nv, gt + q * 256);
  };
  if (!compute) {                            // prologue: tile tb, indices of tb + 1
    load_idx(tb);
    uint4 v[CH];
    const int nv = (int)min<int64_t>(TM, a.E - tb * TM);
#pragma unroll
    for (int q = 0; q < CH; ++q) v[q] = chunk_fetch<T, CPR>(a, gt + q * 256, ridx[q]);
    const SegLoad L = stager ? seg_load(a, tb) : SegLoad{-1, -1, -1};
    if (tb + 1 < te) load_idx(tb + 1);
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int dst = chunk_dst<T, CPR, XS>(gt + q * 256);
      if (dst >= 0) *reinterpret_cast<uint4*>(Xb + dst) = keep_or_zero(chunk_valid<T, CPR>(a, nv, gt + q * 256), v[q]);
    }
    if (stager) seg_stage(&tinfo[0], a, tb, L);
  }
  __syncthreads();
  for (int64_t t = tb; t <= te; ++t) {
    const int buf = (int)((t - tb) & 1);
    if (compute) {
      if (t < te) {
        const T* X = Xb + buf * TM * XS;
        float* Y = Yb + buf * TM * YS;
        f32x16 acc;
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
        const T* xr = X + (lane & 31) * XS + 8 * (lane >> 5);
        // A operands one step ahead of the MFMAs; the scheduling barrier
        // keeps the compiler from hoisting every LDS read (and its
        // registers) to the top of the unrolled loop.
        bf16x8 cur = *reinterpret_cast<const bf16x8*>(xr);
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
          bf16x8 nxt = cur;
          if (ks + 1 < NKS) nxt = *reinterpret_cast<const bf16x8*>(xr + 16 * (ks + 1));
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cur, w[ks], acc, 0, 0, 0);
          __builtin_amdgcn_sched_barrier(0);
          cur = nxt;
        }
        const int col = wave * 32 + (lane & 31);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          Y[row * YS + col] = acc[v];
        }
      }
    } else {
      // load-bound: the data of tile t+1 and the indices of t+2 are in
      // flight while t-1 is reduced
      const bool more = t + 1 < te;
      uint4 v[CH];
      SegLoad L{-1, -1, -1};
      const int nv1 = more ? (int)min<int64_t>(TM, a.E - (t + 1) * TM) : 0;
      if (more) {
#pragma unroll
        for (int q = 0; q < CH; ++q) v[q] = chunk_fetch<T, CPR>(a, gt + q * 256, ridx[q]);
        if (stager) L = seg_load(a, t + 1);
      }
      if (t + 2 < te) load_idx(t + 2);
      if (t > tb)
        ws_reduce<true>(a, t - 1, Yb + (buf ^ 1) * TM * YS, YS, &tinfo[(t - 1 - tb) & 3], tb, range_hi, op, gt, 256);
      if (more) {
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          const int dst = chunk_dst<T, CPR, XS>(gt + q * 256);
          if (dst >= 0)
            *reinterpret_cast<uint4*>(Xb + (buf ^ 1) * TM * XS + dst) =
                keep_or_zero(chunk_valid<T, CPR>(a, nv1, gt + q * 256), v[q]);
        }
        if (stager) seg_stage(&tinfo[(t + 1 - tb) & 3], a, t + 1, L);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- FP32
// Every wave gathers, multiplies and reduces.  A wave owns 16 output
// columns (its W slice, KP/4 VGPRs) and runs f32 16x16x4 MFMAs over the 32
// rows of a tile; the loads of tile t+1 are issued before the MFMA loop of
// tile t and land in the other LDS buffer after it.  A lane holds
// A[row = lane % 16][k = lane / 16]; with one float4 LDS read per lane
// group the four k of MFMA step 4m+u map to columns 16m + 4 (lane / 16) + u,
// and W is swizzled to match (k_ws_swizzle_f16c).
template <int KP, int NW>
__global__ void __launch_bounds__(NW * 64) k_fwd_f32(WsArgs a) {
  if (a.E_dev) {                   // run-time size: as many units as tiles, at most the grid
    a.E = *a.E_dev;
    a.ntiles = (a.E + kTM - 1) / kTM;
    a.sg.n = a.E;
    a.nunits = max<int64_t>(1, min<int64_t>(a.nunits, a.ntiles));
    if ((int64_t)blockIdx.x >= a.nunits) return;
  }
  constexpr int TM = kTM;
  constexpr int XS = KP + 4;
  constexpr int CPR = KP / 4;
  constexpr int NKS = KP / 4;
  constexpr int nthr = NW * 64;
  constexpr int CH = (TM * CPR + nthr - 1) / nthr;     // 16-byte chunks per thread
  extern __shared__ __attribute__((aligned(16))) char smem[];
  float* Xb = reinterpret_cast<float*>(smem);          // [2][TM][XS]
  float* Yb = Xb + 2 * TM * XS;                        // [2][TM][YS]
  const int h = a.h;
  const int YS = h + 4;
  OpenState* op = reinterpret_cast<OpenState*>(Yb + 2 * TM * YS);
  TileInfo* tinfo = reinterpret_cast<TileInfo*>(op + 1);   // [4]
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t tb = (a.ntiles * (int64_t)blockIdx.x) / a.nunits;
  const int64_t te = (a.ntiles * ((int64_t)blockIdx.x + 1)) / a.nunits;
  const int64_t range_hi = min<int64_t>(te * TM, a.E);
  if (tb >= te) return;
  stage_bias(op, a, threadIdx.x, blockDim.x);

  float w[NKS];
  {
    const float* src = static_cast<const float*>(a.Wsw) + (int64_t)wave * NKS * 64;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) w[ks] = src[ks * 64 + lane];
  }

  // row indices two tiles ahead, data one tile ahead
  int32_t ridx[CH];
  uint4 v[CH];
  SegLoad L{-1, -1, -1};
  auto load_idx = [&](int64_t t) {
    const int64_t e0 = t * TM;
    const int nv = (int)min<int64_t>(TM, a.E - e0);
#pragma unroll
    for (int q = 0; q < CH; ++q) ridx[q] = chunk_row<float, CPR>(a, e0, nv, threadIdx.x + q * nthr);
  };
  auto load_data = [&](int64_t t) {
#pragma unroll
    for (int q = 0; q < CH; ++q) v[q] = chunk_fetch<float, CPR>(a, threadIdx.x + q * nthr, ridx[q]);
    if (wave == 0) L = seg_load(a, t);
  };
  auto store = [&](float* X, TileInfo* ti, int64_t t) {
    const int nv = (int)min<int64_t>(TM, a.E - t * TM);
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int dst = chunk_dst<float, CPR, XS>(threadIdx.x + q * nthr);
      if (dst >= 0)
        *reinterpret_cast<uint4*>(X + dst) = keep_or_zero(chunk_valid<float, CPR>(a, nv, threadIdx.x + q * nthr), v[q]);
    }
    if (wave == 0) seg_stage(ti, a, t, L);
  };

  load_idx(tb);
  load_data(tb);
  if (tb + 1 < te) load_idx(tb + 1);
  store(Xb, &tinfo[0], tb);
  __syncthreads();
  for (int64_t t = tb; t < te; ++t) {
    const int buf = (int)((t - tb) & 1);
    const float* X = Xb + buf * TM * XS;
    float* Y = Yb + buf * TM * YS;
    const bool more = t + 1 < te;
    if (more) load_data(t + 1);
    if (t + 2 < te) load_idx(t + 2);
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
    if (more) store(Xb + (buf ^ 1) * TM * XS, &tinfo[(t + 1 - tb) & 3], t + 1);
    __syncthreads();
    ws_reduce<true>(a, t, Y, YS, &tinfo[(t - tb) & 3], tb, range_hi, op, threadIdx.x, nthr);
  }
}

// ---------------------------------------------------------------- pushdown
// Transform pushed below the join (affine tau only): with P_j = Z_j W_j
// computed once per row of atom j, the tuple value is sum_j P_j[r_j] + b.
// This kernel sums the P rows of the atoms that vary inside a group (the
// others, and b, are one constant per group added by the sink) into the
// FP32 tile in LDS, then reduces it per group exactly like the fused
// kernels.  Loads of tile t+1 are in flight while tile t is reduced.
struct PushArgs {
  int n;                                  // atoms gathered per tuple
  const float* P[RELNN_MAX_ATOMS];        // [n_rows_j][h]
  const int32_t* rows[RELNN_MAX_ATOMS];   // [E] joined row per tuple
};

template <int NW>
__global__ void __launch_bounds__(NW * 64) k_push(WsArgs a, PushArgs pa) {
  constexpr int TM = kTM;
  constexpr int nthr = NW * 64;
  constexpr int CH = (TM * (kHMax / 4) + nthr - 1) / nthr;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int h = a.h;
  const int YS = h + 4;
  const int C4 = h / 4;
  float* Yb = reinterpret_cast<float*>(smem);            // [2][TM][YS]
  OpenState* op = reinterpret_cast<OpenState*>(Yb + 2 * TM * YS);
  TileInfo* tinfo = reinterpret_cast<TileInfo*>(op + 1);   // [4]
  const int wave = threadIdx.x / 64;
  const int64_t tb = (a.ntiles * (int64_t)blockIdx.x) / a.nunits;
  const int64_t te = (a.ntiles * ((int64_t)blockIdx.x + 1)) / a.nunits;
  const int64_t range_hi = min<int64_t>(te * TM, a.E);
  if (tb >= te) return;
  stage_bias(op, a, threadIdx.x, blockDim.x);

  f32x4 acc[CH];
  SegLoad L{-1, -1, -1};
  auto load = [&](int64_t t) {
    const int64_t e0 = t * TM;
    const int nv = (int)min<int64_t>(TM, a.E - e0);
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int i = threadIdx.x + q * nthr;
      acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
      const int r = i / C4;
      if (i < TM * C4 && r < nv) {
        const int c4 = i - r * C4;
        for (int j = 0; j < pa.n; ++j)
          acc[q] += *reinterpret_cast<const f32x4*>(pa.P[j] + (int64_t)pa.rows[j][e0 + r] * h + 4 * c4);
      }
    }
    if (wave == 0) L = seg_load(a, t);
  };
  auto store = [&](float* Y, TileInfo* ti, int64_t t) {
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int i = threadIdx.x + q * nthr;
      if (i < TM * C4) {
        const int r = i / C4, c4 = i - (i / C4) * C4;
        *reinterpret_cast<f32x4*>(Y + r * YS + 4 * c4) = acc[q];
      }
    }
    if (wave == 0) seg_stage(ti, a, t, L);
  };

  load(tb);
  store(Yb, &tinfo[0], tb);
  __syncthreads();
  for (int64_t t = tb; t < te; ++t) {
    const int buf = (int)((t - tb) & 1);
    const bool more = t + 1 < te;
    if (more) load(t + 1);
    ws_reduce<false>(a, t, Yb + buf * TM * YS, YS, &tinfo[(t - tb) & 3], tb, range_hi, op, threadIdx.x, nthr);
    if (more) store(Yb + (buf ^ 1) * TM * YS, &tinfo[(t + 1 - tb) & 3], t + 1);
    __syncthreads();
  }
}

namespace {

template <class KernelT>
void allow_lds(KernelT k, size_t bytes) {
  RELNN_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

constexpr size_t kStateBytes = sizeof(OpenState) + 4 * sizeof(TileInfo);

size_t f32_lds(int KP, int h) { return 2 * kTM * (KP + 4) * 4 + 2 * kTM * (h + 4) * 4 + kStateBytes; }
size_t bf16_lds(int KP, int h) { return 2 * kTM * (KP + 8) * 2 + 2 * kTM * (h + 4) * 4 + kStateBytes; }

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
  switch (a.h) {
    case 32: run_f32<KP, 2>(a, s); break;
    case 64: run_f32<KP, 4>(a, s); break;
    case 96: run_f32<KP, 6>(a, s); break;
    default: run_f32<KP, 8>(a, s); break;
  }
}

template <int KP>
void run_bf16(const WsArgs& a, hipStream_t s) {
  const size_t lds = bf16_lds(KP, a.h);
  allow_lds(k_fwd_ws<KP>, lds);
  KTimer tm("fwd_fused", s);
  k_fwd_ws<KP><<<(unsigned)a.nunits, (a.h / 32 + kGatherWaves) * 64, lds, s>>>(a);
  RELNN_LAUNCHED();
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

int pick_kp(int K) {
  for (int kp : {64, 128, 256, 384})
    if (K <= kp) return kp;
  return 0;
}

}  // namespace

void launch_push(const FwdArgs& f, int64_t nunits, int n, const float* const* P, const int32_t* const* rows,
                 float* carry, int32_t* carry_arg, hipStream_t s) {
  RELNN_REQUIRE(f.h % 4 == 0 && f.h <= kHMax, RELNN_E_UNSUPPORTED, "pushdown needs h %% 4 == 0 and h <= %d", kHMax);
  WsArgs a{};
  a.at = f.at;
  a.E = f.E;
  a.h = f.h;
  a.ntiles = cdiv(f.E, kTM);
  a.nunits = std::max<int64_t>(1, std::min<int64_t>(a.ntiles, nunits));
  a.b = nullptr;                      // the bias is part of the group constant
  a.act_pre = RELNN_ACT_NONE;
  a.sg = f.sg;
  a.sink = f.sink;
  a.carry = carry;
  a.carry_arg = carry_arg;
  PushArgs pa{};
  pa.n = n;
  for (int j = 0; j < n; ++j) {
    pa.P[j] = P[j];
    pa.rows[j] = rows[j];
  }
  const size_t lds = 2 * kTM * (f.h + 4) * 4 + kStateBytes;
  allow_lds(k_push<4>, lds);
  {
    KTimer tm("fwd_push", s);
    k_push<4><<<(unsigned)a.nunits, 256, lds, s>>>(a, pa);
    RELNN_LAUNCHED();
  }
  launch_fixup(f.sg, kTM, f.h, a.ntiles, a.nunits, f.sink, carry, carry_arg, s);
}

int64_t push_units(int64_t E) { return std::max<int64_t>(1, std::min<int64_t>(cdiv(E, kTM), num_cus())); }

WsPlan plan_ws(int dtype, int K, int h, int64_t E) {
  WsPlan p;
  const bool bf = dtype == RELNN_BF16;
  p.KP = pick_kp(K);
  const bool h_ok = bf ? (h % 32 == 0 && h <= kHMax) : (h == 32 || h == 64 || h == 96 || h == 128);
  if (!p.KP || !h_ok) {
    p.KP = 0;
    return p;
  }
  p.TM = kTM;
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
  RELNN_REQUIRE(!f.sink.accumulate && !f.sink.out_row && !f.sink.gc.n && !f.sink.gc.bias, RELNN_E_UNSUPPORTED,
                "the fused forward kernels write plain outputs only");
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
      case 64: run_bf16<64>(a, s); break;
      case 128: run_bf16<128>(a, s); break;
      case 256: run_bf16<256>(a, s); break;
      default: run_bf16<384>(a, s); break;
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
