// Forward layer, weight-stationary persistent kernels (the fast path).
//
// Same arithmetic as the tile kernel of layer_fwd.hip (gather -> Linear on
// the matrix cores -> per-group reduce -> act_post), organised for gfx950.
// One block per CU runs a contiguous range of 32-tuple tiles; a group that
// spans tiles is accumulated inside the block (Kahan-compensated sum, or max
// with the earliest maximiser), so a block leaves at most two partials, for
// the groups cut by its range ends; k_fixup combines those in block order.
//
// k_fwd_dma (FP32 and BF16) has two kinds of waves:
//  * h/16 compute waves, 16 output columns each, whose W slice stays in
//    VGPRs for the whole kernel.  They multiply a tile on the matrix cores
//    (f32 16x16x4 or bf16 16x16x32, FP32 accumulation) and reduce it per
//    group straight from the accumulators: a lane holds 8 rows of one
//    column, a run of equal group is summed per lane and across the 4 lanes
//    of the column by two butterfly shuffles, and the group left open at
//    the end of a tile stays in registers for the next one.
//  * 4 DMA waves that move tiles from HBM into an NB-deep LDS ring with
//    16-byte global->LDS loads (no registers in between): while tile t is
//    multiplied, tiles t+1 .. t+NB-2 are in flight and t+NB-1 is issued.
//    The row numbers for a tile are read one tile ahead into VGPRs, before
//    the previous tile's loads are issued, so that waiting for them never
//    waits for tile data (vector memory counts retire in order).
// LDS tile layout: row-major without padding; 16-byte chunk c of row r is
// stored at position c ^ (r & SWM) of its row, so the 16 rows read by one
// MFMA operand load fall into 16 different bank groups.
// One __syncthreads per tile.
//
// k_push (pushdown) keeps the LDS-staged reduce (ws_reduce).
#include "layer_fwd.hpp"

namespace relnn {

constexpr int kDmaWaves = 4;
constexpr int kHMax = 128;
constexpr int kTM = 32;                  // tuples per tile

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

// W for the BF16 kernel, 16-column slices: fragment ks of slice cw, lane l
// holds W[32 ks + 8 (l / 16) + i][16 cw + l % 16], i = 0..7 (one 16x16x32
// B operand).
__global__ void k_ws_swizzle_bf16(const __bf16* __restrict__ W, int K, int KP, int h, __bf16* __restrict__ out) {
  const int nks = KP / 32;
  const int64_t total = (int64_t)(h / 16) * nks * 64 * 8;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(i & 7);
    const int lane = (int)((i >> 3) & 63);
    const int64_t f = i >> 9;
    const int ks = (int)(f % nks);
    const int cw = (int)(f / nks);
    const int k = 32 * ks + 8 * (lane / 16) + e;
    out[i] = k < K ? W[(int64_t)k * h + cw * 16 + lane % 16] : (__bf16)0.0f;
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

// Atom owning Concat column el (j: its index).  Picked with compile-time
// indices: indexing the argument's arrays with a run-time value would move
// the whole argument to scratch memory.
struct AtomSel {
  const void* emb;
  int d, koff, j;
};

__device__ __forceinline__ AtomSel atom_sel(const Atoms& at, int el) {
  AtomSel r{at.emb[0], at.d[0], 0, 0};
  auto pick = [&](auto U) {
    constexpr int u = decltype(U)::value;
    if (u < at.k && el >= at.koff[u]) r = AtomSel{at.emb[u], at.d[u], at.koff[u], u};
  };
  static_assert(kMaxAtoms == 4, "one pick per atom after the first");
  pick(std::integral_constant<int, 1>{});
  pick(std::integral_constant<int, 2>{});
  pick(std::integral_constant<int, 3>{});
  return r;
}

template <class T, int KP, int NB>
struct DmaGeo {
  static constexpr int EPC = 16 / (int)sizeof(T);          // elements per 16-byte chunk
  static constexpr int CPR = KP / EPC;                     // chunks per row
  static constexpr int NI = kTM * CPR / 64;                // wave-wide loads per tile
  static constexpr int NIW = NI / kDmaWaves;               // ... per DMA wave
  static constexpr int SWM = (CPR < 16 ? CPR : 16) - 1;    // chunk swizzle mask
  static constexpr int TILE = kTM * KP * (int)sizeof(T);   // bytes per LDS tile
  static constexpr int NIR = 2 * NB - 1;                   // index slots (tiles t .. t+2NB-2)
  static constexpr int IRB = kDmaWaves * 256;              // bytes per index slot
  // vector-memory operations a DMA wave issues after the loads of tile t+1
  // up to the end of iteration t: NB-2 iterations of (1 + NIW)
  static constexpr int WAIT = (NB - 2) * (1 + NIW);
  static_assert(NI % kDmaWaves == 0, "whole DMA instructions per wave");
  static_assert(kDmaWaves == kMaxAtoms, "one DMA wave per atom moves the row numbers");
  static_assert(WAIT >= 0 && WAIT <= 63, "vmcnt range");
};

// Index slot of tile u (int32): DMA wave j writes 256 bytes at j*64 ints;
// lanes 0..31 carry atom j's row number of tuple r, lanes 32..63 of wave 0
// the tuple's group number and lanes 32, 33 of wave 1 the group numbers of
// the tuples just before and after the tile.  Atoms past k repeat atom 0
// and tuples past the tile repeat its last one, so that every wave issues
// the same operations for every tile.
constexpr int kSlotSeg = 32;          // ints: group numbers of the tile
constexpr int kSlotEdge = 64 + 32;    // ints: groups before and after it

__device__ __forceinline__ void dma_index(const WsArgs& a, int64_t u, char* slot, int dw) {
  const int lane = __lane_id();
  const int64_t e0 = u * kTM;
  const int nv = (int)min<int64_t>(kTM, a.E - e0);
  // compile-time indices only (a chain of selects over the argument's
  // array is turned into a table in scratch memory)
  const int32_t* src = a.at.rows[0];
  auto pick = [&](auto U) {
    constexpr int q = decltype(U)::value;
    if (dw == q && q < a.at.k) src = a.at.rows[q];
  };
  pick(std::integral_constant<int, 1>{});
  pick(std::integral_constant<int, 2>{});
  pick(std::integral_constant<int, 3>{});
  int64_t e = e0 + min(lane & 31, nv - 1);
  if (lane >= 32) {
    src = a.sg.seg_of;
    if (dw == 1) e = lane == 32 ? max<int64_t>(e0 - 1, 0) : min<int64_t>(e0 + nv, a.E - 1);
  }
  const bool on = lane < 32 || dw == 0 || (dw == 1 && lane < 34);
  if (on) __builtin_amdgcn_global_load_lds(src + e, slot + dw * 256, 4, 0, 0);
}

// Issues this DMA wave's share of the loads of tile u into the LDS tile X.
// Chunk slot s (= 64 ins + lane) of the tile is row r = s / CPR, position
// p = s % CPR, holding logical chunk p ^ (r & SWM).  Chunks in the K..KP
// pad are not loaded (their LDS slots were zeroed once).  The row numbers
// come from the tile's LDS slot (an LDS read: no wait on vector memory).
template <class T, int KP, int NB>
__device__ __forceinline__ void dma_tile(const WsArgs& a, const int32_t* rows, char* X, int dw) {
  using G = DmaGeo<T, KP, NB>;
  const int lane = __lane_id();
#pragma unroll
  for (int i = 0; i < G::NIW; ++i) {
    const int ins = dw * G::NIW + i;
    const int sl = ins * 64 + lane;
    const int r = sl / G::CPR;
    const int pos = sl - r * G::CPR;
    const int el = (pos ^ (r & G::SWM)) * G::EPC;
    const int elc = min(el, a.K - G::EPC);
    const AtomSel A = atom_sel(a.at, elc);
    const int32_t row = rows[A.j * 64 + r];
    const T* g = static_cast<const T*>(A.emb) + (int64_t)row * A.d + (elc - A.koff);
    if (el < a.K) __builtin_amdgcn_global_load_lds(g, X + ins * 1024, 16, 0, 0);
  }
}

// Barriers of the DMA ring.  __syncthreads() is a release fence plus
// s_barrier, and a release fence waits for every vector-memory operation,
// LDS-direct loads included: that would drain the ring at every tile.  So
// the waves wait for exactly what the others need and then meet at a bare
// s_barrier; the asm "memory" clobber keeps the compiler from moving memory
// accesses across it.
//   DMA waves:     their loads of tile t+1 have landed in LDS (at most N
//                  newer operations outstanding; vector memory retires in
//                  order).
//   compute waves: their LDS reads of tile t are complete.
template <int N>
__device__ __forceinline__ void dma_barrier() {
  asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(N) : "memory");
}
__device__ __forceinline__ void compute_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Combining the 4 lanes of one output column (lanes c, c+16, c+32, c+48)
// with the gfx950 row swaps (VALU, no LDS): after the 16-lane swap a lane
// holds the values of its row pair, after the 32-lane swap all four.  The
// operands are taken in the same order in every lane, so all four lanes end
// with the same bits.
__device__ __forceinline__ float col_sum4(float v) {
  const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  const float s = __uint_as_float(p[0]) + __uint_as_float(p[1]);
  const auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(s), __float_as_uint(s), false, false);
  return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}

// Max with the earliest maximiser (ties: smaller tuple position).
__device__ __forceinline__ void max_pick(float& v, int32_t& a, float v1, int32_t a1) {
  if (v1 > v || (v1 == v && a1 < a)) {
    v = v1;
    a = a1;
  }
}

__device__ __forceinline__ void col_max4(float& v, int32_t& a) {
  const auto pv = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  const auto pa = __builtin_amdgcn_permlane16_swap((uint32_t)a, (uint32_t)a, false, false);
  v = __uint_as_float(pv[0]);
  a = (int32_t)pa[0];
  max_pick(v, a, __uint_as_float(pv[1]), (int32_t)pa[1]);
  const auto qv = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  const auto qa = __builtin_amdgcn_permlane32_swap((uint32_t)a, (uint32_t)a, false, false);
  v = __uint_as_float(qv[0]);
  a = (int32_t)qa[0];
  max_pick(v, a, __uint_as_float(qv[1]), (int32_t)qa[1]);
}

template <class T>
struct DmaMfma;
template <>
struct DmaMfma<float> {                  // f32 16x16x4, one float4 A read per 4 steps
  typedef float W;
  template <int KP>
  static constexpr int nks() { return KP / 4; }
};
template <>
struct DmaMfma<__bf16> {                 // bf16 16x16x32, one 16-byte A read per step
  typedef bf16x8 W;
  template <int KP>
  static constexpr int nks() { return KP / 32; }
};

template <class T, int KP, int NB>
__global__ void __launch_bounds__((kHMax / 16 + kDmaWaves) * 64) k_fwd_dma(WsArgs a) {
  using G = DmaGeo<T, KP, NB>;
  using WT = typename DmaMfma<T>::W;
  constexpr int NKS = DmaMfma<T>::template nks<KP>();
  constexpr int TM = kTM;
  if (a.E_dev) {                   // run-time size: as many units as tiles, at most the grid
    a.E = *a.E_dev;
    a.ntiles = (a.E + kTM - 1) / kTM;
    a.sg.n = a.E;
    a.nunits = max<int64_t>(1, min<int64_t>(a.nunits, a.ntiles));
    if ((int64_t)blockIdx.x >= a.nunits) return;
  }
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int h = a.h;
  const int ncw = h / 16;
  const int wave = threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  const int64_t bidx = blockIdx.x;
  const int64_t tb = (a.ntiles * bidx) / a.nunits;
  const int64_t te = (a.ntiles * (bidx + 1)) / a.nunits;
  const int64_t range_hi = min<int64_t>(te * TM, a.E);
  if (tb >= te) return;

  // zero the ring once: pad chunks (K..KP) are never written afterwards
  for (int i = threadIdx.x; i < NB * G::TILE / 16; i += blockDim.x)
    reinterpret_cast<uint4*>(smem)[i] = make_uint4(0, 0, 0, 0);
  __syncthreads();
  auto ring = [&](int64_t u) { return smem + (int)((u - tb) % NB) * G::TILE; };
  char* irs = smem + NB * G::TILE;                          // row-number slots
  auto islot = [&](int64_t u) { return irs + (int)((u - tb) % G::NIR) * G::IRB; };

  if (wave >= ncw) {
    // ------------------------------------------------------------ DMA waves
    // Every vector-memory operation of these waves is a global->LDS load;
    // at iteration t a wave issues the index slot of tile t+2NB-2, then its
    // share of tile t+NB-1, then waits until its share of tile t+1 has
    // landed.  The index slot of tile v is issued just before tile v-NB+1,
    // so it has landed (and passed a barrier) before tile v is issued.
    const int dw = wave - ncw;
    const int64_t tl = te - 1;
#pragma unroll
    for (int j = 0; j + 1 < NB; ++j) dma_index(a, min(tb + j, tl), islot(tb + j), dw);
    asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");   // index slots of tb .. tb+NB-2
#pragma unroll
    for (int j = 0; j + 1 < NB; ++j) {
      dma_index(a, min(tb + j + NB - 1, tl), islot(tb + j + NB - 1), dw);
      dma_tile<T, KP, NB>(a, reinterpret_cast<const int32_t*>(islot(tb + j)), ring(tb + j), dw);
    }
    dma_barrier<G::WAIT>();                                   // tile tb has landed
    for (int64_t t = tb; t < te; ++t) {
      dma_index(a, min(t + 2 * NB - 2, tl), islot(t + 2 * NB - 2), dw);
      dma_tile<T, KP, NB>(a, reinterpret_cast<const int32_t*>(islot(t + NB - 1)), ring(t + NB - 1), dw);
      dma_barrier<G::WAIT>();                                 // tile t+1 has landed
    }
    // loads past the range may still be landing: the LDS must not be
    // released to another block before they have
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    return;
  }

  // -------------------------------------------------------------- compute waves
  const int cw = wave;
  const int col = cw * 16 + (lane & 15);
  const float bc = a.b ? a.b[col] : 0.0f;
  const bool maxagg = a.sink.agg == RELNN_MAX;
  WT w[NKS];
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks) w[ks] = reinterpret_cast<const WT*>(a.Wsw)[(cw * NKS + ks) * 64 + lane];
  // W has landed before the loop: otherwise the compiler waits for it (and
  // with it for the group numbers of the next tile) at every tile's MFMAs
  __builtin_amdgcn_s_waitcnt(0);

  // group numbers of tile t from its index slot: lane r < 32 row r
  // (clamped), lane 32 the row before the tile, lane 33 the row after it
  // (clamped; their validity follows from e0 and nv)
  auto seg_read = [&](int64_t t) {
    const int32_t* sl = reinterpret_cast<const int32_t*>(islot(t));
    return sl[lane < 32 ? kSlotSeg + lane : kSlotEdge + min(lane - 32, 1)];
  };

  // state of the group open at the end of the previous tile (per column)
  float oS = 0.0f, oC = 0.0f;
  int32_t oArg = -1, oN = 0;
  bool oCut = false;
  const int q4 = 4 * (lane >> 4);
  const int64_t slot_base = bidx * 2 * h + col;

  compute_barrier();                                         // (index slots staged)
  compute_barrier();                                         // tile tb is in LDS
  for (int64_t t = tb; t < te; ++t) {
    const int32_t gcur = seg_read(t);
    const char* X = ring(t);
    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    const int r0 = lane & 15, r1 = 16 + (lane & 15);
    // A operand of step m: logical chunk 4m + cq of rows r0 / r1, stored at
    // position (4m + cq) ^ sw = 4 (m ^ (sw >> 2)) + ((cq ^ sw) & 3): a
    // per-lane base for m % 4 plus a constant for the rest (four registers
    // per row instead of one address per step)
    const int cq = lane >> 4;
    auto chunk_base = [&](int sw, int j) { return 4 * (j ^ (sw >> 2)) + ((cq ^ sw) & 3); };
    if constexpr (std::is_same<T, float>::value) {
      const float* x0 = reinterpret_cast<const float*>(X) + r0 * KP;
      const float* x1 = reinterpret_cast<const float*>(X) + r1 * KP;
      int b0[4], b1[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        b0[j] = 4 * chunk_base(r0 & G::SWM, j);
        b1[j] = 4 * chunk_base(r1 & G::SWM, j);
      }
      // no read-ahead (the W slice takes most registers): the other compute
      // wave of the SIMD fills the LDS latency
#pragma unroll
      for (int m = 0; m < KP / 16; ++m) {
        const f32x4 c0 = *reinterpret_cast<const f32x4*>(x0 + 16 * (m & ~3) + b0[m & 3]);
        const f32x4 c1 = *reinterpret_cast<const f32x4*>(x1 + 16 * (m & ~3) + b1[m & 3]);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(c0[u], w[4 * m + u], acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(c1[u], w[4 * m + u], acc1, 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      const __bf16* x0 = reinterpret_cast<const __bf16*>(X) + r0 * KP;
      const __bf16* x1 = reinterpret_cast<const __bf16*>(X) + r1 * KP;
      int b0[4], b1[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        b0[j] = 8 * chunk_base(r0 & G::SWM, j);
        b1[j] = 8 * chunk_base(r1 & G::SWM, j);
      }
      bf16x8 c0 = *reinterpret_cast<const bf16x8*>(x0 + b0[0]);
      bf16x8 c1 = *reinterpret_cast<const bf16x8*>(x1 + b1[0]);
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        bf16x8 n0 = c0, n1 = c1;
        if (ks + 1 < NKS) {
          const int kn = ks + 1;
          n0 = *reinterpret_cast<const bf16x8*>(x0 + 32 * (kn & ~3) + b0[kn & 3]);
          n1 = *reinterpret_cast<const bf16x8*>(x1 + 32 * (kn & ~3) + b1[kn & 3]);
        }
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c0, w[ks], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c1, w[ks], acc1, 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        c0 = n0;
        c1 = n1;
      }
    }

    // ---- per-group reduce of the tile (rows of this lane: q4 + i, 16 + q4 + i)
    const int64_t e0 = t * TM;
    const int nv = (int)min<int64_t>(TM, a.E - e0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {                    // tuple values y = act_pre(x W + b), in place
      acc0[i] = act_apply(a.act_pre, acc0[i] + bc);
      acc1[i] = act_apply(a.act_pre, acc1[i] + bc);
    }
    // runs of equal group: lane r starts one if its group differs from
    // lane r-1's (DPP wave shift right by one lane)
    const int32_t gup = __builtin_amdgcn_update_dpp(0, gcur, 0x138, 0xf, 0xf, false);
    const bool start = lane < nv && (lane == 0 || gup != gcur);
    uint64_t runs = __ballot(start);
    const int32_t g_first = __builtin_amdgcn_readlane(gcur, 0);
    const int32_t g_last = __builtin_amdgcn_readlane(gcur, nv - 1);
    const int32_t g_before = __builtin_amdgcn_readlane(gcur, 32);
    const int32_t g_after = __builtin_amdgcn_readlane(gcur, 33);
    const bool prev_same = e0 > 0 && g_before == g_first;
    const bool next_same = e0 + nv < a.E && g_after == g_last;
    bool first_run = true;
    while (runs) {
      const int rs = __builtin_ctzll(runs);
      runs &= runs - 1;
      const int re = runs ? __builtin_ctzll(runs) : nv;
      const bool last_run = runs == 0;
      const int32_t g = __builtin_amdgcn_readlane(gcur, rs);
      // this lane's rows of the run, then the 4 lanes of the column
      float part = maxagg ? -INFINITY : 0.0f;
      int32_t parg = INT32_MAX;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int rw = (i < 4 ? 0 : 16) + q4 + (i & 3);
        const bool in = rw >= rs && rw < re;
        const float yi = i < 4 ? acc0[i & 3] : acc1[i & 3];
        if (maxagg) {
          if (in && yi > part) {
            part = yi;
            parg = (int32_t)(e0 + rw);
          }
        } else {
          part += in ? yi : 0.0f;
        }
      }
      if (maxagg)
        col_max4(part, parg);
      else
        part = col_sum4(part);
      const int32_t cnt = re - rs;
      if (first_run && prev_same) {
        if (t > tb) {                                        // the block's open group
          if (maxagg) {
            if (part > oS) {
              oS = part;
              oArg = parg;
            }
          } else {
            kahan_add(oS, oC, part);
          }
          oN += cnt;
        } else {                                             // began before the range
          oS = part; oC = 0.0f; oArg = parg; oN = cnt; oCut = true;
        }
      } else {
        oS = part; oC = 0.0f; oArg = parg; oN = cnt; oCut = false;
      }
      if (last_run && next_same && e0 + nv < range_hi) {
        // stays open for the next tile
      } else if (lane < 16) {
        const float v = maxagg ? oS : oS - oC;
        if (last_run && next_same) {                         // runs past the range end
          const int64_t o = slot_base + (oCut ? 0 : h);
          a.carry[o] = v;
          if (a.carry_arg) a.carry_arg[o] = oArg;
        } else if (!oCut) {
          sink_write<true>(a.sink, g, col, h, v, oArg, oN);
        } else {                                             // cut by the range start
          a.carry[slot_base] = v;
          if (a.carry_arg) a.carry_arg[slot_base] = oArg;
        }
      }
      first_run = false;
    }
    compute_barrier();
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

// LDS ring depth NB: as many tiles as fit with their 2 NB - 1 index slots,
// at most 6 (tiles t+1 .. t+4 in flight while t is multiplied).
template <class T, int KP>
constexpr int ring_depth() {
  constexpr int TILE = DmaGeo<T, KP, 2>::TILE;
  constexpr int IRB = DmaGeo<T, KP, 2>::IRB;
  constexpr int fit = (160 * 1024 + IRB) / (TILE + 2 * IRB);
  return fit < 6 ? fit : 6;
}

template <class T, int KP>
void run_dma(const WsArgs& a, hipStream_t s) {
  constexpr int NB = ring_depth<T, KP>();
  using G = DmaGeo<T, KP, NB>;
  static_assert(NB >= 2, "two LDS tiles at least");
  const size_t lds = (size_t)NB * G::TILE + (size_t)G::NIR * G::IRB;
  RELNN_REQUIRE(lds <= 160 * 1024, RELNN_E_HIP, "internal: LDS ring of %zu bytes", lds);
  allow_lds(k_fwd_dma<T, KP, NB>, lds);
  KTimer tm("fwd_fused", s);
  k_fwd_dma<T, KP, NB><<<(unsigned)a.nunits, (a.h / 16 + kDmaWaves) * 64, lds, s>>>(a);
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
  const bool h_ok = h % 16 == 0 && h <= kHMax;
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
      case 64: run_dma<__bf16, 64>(a, s); break;
      case 128: run_dma<__bf16, 128>(a, s); break;
      case 256: run_dma<__bf16, 256>(a, s); break;
      default: run_dma<__bf16, 384>(a, s); break;
    }
  } else {
    switch (p.KP) {
      case 64: run_dma<float, 64>(a, s); break;
      case 128: run_dma<float, 128>(a, s); break;
      case 256: run_dma<float, 256>(a, s); break;
      default: run_dma<float, 384>(a, s); break;
    }
  }
  launch_fixup(f.sg, p.TM, f.h, p.ntiles, p.nunits, f.sink, carry, carry_arg, s);
}

}  // namespace relnn
