// Forward layer, weight-stationary persistent kernels (the fast path).
//
// Same arithmetic as the tile kernel of layer_fwd.hip (gather -> Linear on
// the matrix cores -> per-group reduce -> act_post), organised for gfx950.
// One block per CU runs a contiguous range of 32-tuple tiles; a group that
// spans tiles is accumulated inside the block (Kahan-compensated sum, or max
// with the earliest maximiser), so a block leaves at most two partials, for
// the groups cut by its range ends; k_fixup combines those in block order.
//
// k_fwd_dma (FP32 and BF16; SUM/MEAN and MAX instances) has two kinds of
// waves:
//  * compute waves for up to 128 output columns (16 each, or 32 for BF16
//    SUM/MEAN), whose W slice stays in VGPRs for the whole kernel.  They
//    multiply a tile on the matrix cores (f32 16x16x4 or bf16 16x16x32,
//    FP32 accumulation) and reduce it per group straight from the
//    accumulators: SUM/MEAN as one more matrix product per accumulator
//    register with the 0/1 row-in-run matrix, MAX as a segmented max-scan
//    in registers.  The group left open at the end of a tile stays in
//    registers for the next one.  Wider layers run as 128-column chunks.
//  * 4 DMA waves that move tiles from HBM into an NB-deep LDS ring with
//    16-byte global->LDS loads (no registers in between): while tile t is
//    multiplied, tiles t+1 .. t+NB-2 are in flight and t+NB-1 is issued.
//    Each lane's source rows, strides and row-number slots are worked out
//    once per kernel; per tile a wave reads its row numbers from LDS, waits
//    once, and issues its loads.
// LDS tile layout: row-major without padding; 16-byte chunk c of row r is
// stored at position c ^ (r & SWM) of its row, so the 16 rows read by one
// MFMA operand load fall into 16 different bank groups.
// One barrier per tile.
//
// k_push_sum (pushdown) is a segmented gather-sum of node products, one wave
// per range of tuples.
#include <mutex>
#include <vector>

#include "layer_fwd.hpp"

namespace relnn {

constexpr int kDmaWaves = 4;
constexpr int kHMax = 128;
constexpr int kTM = 32;                  // tuples per tile
constexpr int kZeroBytes = 64;           // zero bytes after the re-laid weight

struct WsArgs {
  Atoms at;
  const int32_t* rows;
  int64_t E;
  const int64_t* E_dev;      // if set: E (and the tile count) come from device memory
  int K, h;
  int hc, nch;               // output columns per block, column chunks (h = nch hc)
  int64_t ntiles, nunits;
  const void* Wsw;
  const void* zeros;         // 64 zero bytes (source of the K..KP pad chunks)
  const float* b;
  int act_pre;
  Seg sg;
  Sink sink;
  float* carry;
  int32_t* carry_arg;
};

// Compensated add.  Once the sum is infinite or NaN the compensation
// (t - s) - y would be NaN and turn an infinite sum into NaN, so it is
// dropped: the sum then carries the non-finite value as plain addition does.
__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
  const float y = x - c;
  const float t = s + y;
  c = __builtin_isfinite(t) ? (t - s) - y : 0.0f;
  s = t;
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
  if (blockIdx.x == 0 && threadIdx.x < kZeroBytes / 2) out[total + threadIdx.x] = (__bf16)0.0f;
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
  if (blockIdx.x == 0 && threadIdx.x < kZeroBytes / 4) out[total + threadIdx.x] = 0.0f;
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
// the tuples just before and after the tile.  Every lane of every DMA wave
// loads (atoms past k repeat atom 0, tuples past the tile repeat its last
// one, the remaining lanes fill slot words that the run table below
// overwrites or nobody reads), so the load needs no branch.
// For SUM / MEAN, DMA wave 0 then writes the tile's run table into the
// words the rows of atoms 1..3 do not use: the header (number of runs,
// whether the first run continues a group from before the tile, whether
// the last one runs past it, tuples in the tile), and per run its first
// row and its group.
constexpr int kSlotSeg = 32;          // ints: group numbers of the tile
constexpr int kSlotEdge = 64 + 32;    // ints: groups before and after it
constexpr int kSlotHdr = 98;          // int: runs | prev_same << 8 | next_same << 9 | nv << 16
constexpr int kSlotRunStart = 160;    // ints [32]: first row of run g
constexpr int kSlotRunGroup = 224;    // ints [32]: group of run g

// Per-lane plan of a DMA wave's share of a tile, fixed for the whole kernel:
// load i of the wave moves 16 bytes from src[i] + row * stride[i] into its
// LDS chunk slot, with row read from the tile's index slot at byte roff[i].
// Chunk slot s (= 64 ins + lane) of the tile is row r = s / CPR, position
// p = s % CPR, holding logical chunk p ^ (r & SWM).  Chunks in the K..KP
// pad load 16 zero bytes (stride 0), so every lane loads and no load needs
// a branch.
template <class T, int KP, int NB>
struct DmaPlan {
  using G = DmaGeo<T, KP, NB>;
  const char* src[G::NIW];
  uint32_t stride[G::NIW];
  int roff[G::NIW];
  const int32_t* isrc;       // index slot source of this lane
  int ilane;                 // tuple of the tile this lane's index word names
  bool edge;                 // lanes 32.. of wave 1: the groups around the tile

  __device__ __forceinline__ DmaPlan(const WsArgs& a, int dw) {
    const int lane = __lane_id();
#pragma unroll
    for (int i = 0; i < G::NIW; ++i) {
      const int ins = dw * G::NIW + i;
      const int sl = ins * 64 + lane;
      const int r = sl / G::CPR;
      const int pos = sl - r * G::CPR;
      const int el = (pos ^ (r & G::SWM)) * G::EPC;
      const bool pad = el >= a.K;
      const AtomSel A = atom_sel(a.at, pad ? 0 : el);
      src[i] = pad ? static_cast<const char*>(a.zeros)
                   : static_cast<const char*>(A.emb) + (int64_t)(el - A.koff) * (int)sizeof(T);
      stride[i] = pad ? 0u : (uint32_t)A.d * (uint32_t)sizeof(T);
      roff[i] = (A.j * 64 + r) * 4;
    }
    // compile-time indices only (a chain of selects over the argument's
    // array is turned into a table in scratch memory)
    const int32_t* rs = a.at.rows[0];
    auto pick = [&](auto U) {
      constexpr int q = decltype(U)::value;
      if (dw == q && q < a.at.k) rs = a.at.rows[q];
    };
    pick(std::integral_constant<int, 1>{});
    pick(std::integral_constant<int, 2>{});
    pick(std::integral_constant<int, 3>{});
    isrc = lane < 32 ? rs : a.sg.seg_of;
    ilane = lane & 31;
    edge = dw == 1 && lane >= 32;
  }

  // index slot of tile u (u < ntiles) into slot
  __device__ __forceinline__ void index(const WsArgs& a, int64_t u, char* slot, int dw) const {
    const int64_t e0 = u * kTM;
    const int nv = (int)min<int64_t>(kTM, a.E - e0);
    // offset from e0 in 32 bits (a per-lane choice between 64-bit values
    // costs a conversion sequence)
    int off = min(ilane, nv - 1);
    const int before = e0 > 0 ? -1 : 0;
    const int after = e0 + nv < a.E ? nv : nv - 1;
    if (edge) off = __lane_id() == 32 ? before : after;
    __builtin_amdgcn_global_load_lds(isrc + e0 + off, slot + dw * 256, 4, 0, 0);
  }

  // this wave's loads of a tile whose row numbers are in slot, into X
  __device__ __forceinline__ void tile(const char* slot, char* X, int dw) const {
    int32_t rv[G::NIW];
#pragma unroll
    for (int i = 0; i < G::NIW; ++i) rv[i] = *reinterpret_cast<const int32_t*>(slot + roff[i]);
#pragma unroll
    for (int i = 0; i < G::NIW; ++i) {
      const char* g = src[i] + (uint64_t)(uint32_t)rv[i] * stride[i];
      __builtin_amdgcn_global_load_lds(g, X + (dw * G::NIW + i) * 1024, 16, 0, 0);
    }
  }

  // run table of tile u (wave 0, once its index slot has landed): runs of
  // equal group start where a row's group differs from the row before
  __device__ __forceinline__ static void run_table(const WsArgs& a, int64_t u, char* slot) {
    const int lane = __lane_id();
    int32_t* sw = reinterpret_cast<int32_t*>(slot);
    const int32_t g = sw[lane < 32 ? kSlotSeg + lane : kSlotEdge + min(lane - 32, 1)];
    const int64_t e0 = u * kTM;
    const int nv = (int)min<int64_t>(kTM, a.E - e0);
    const int32_t gup = __builtin_amdgcn_update_dpp(0, g, 0x138, 0xf, 0xf, false);   // row - 1
    const bool start = lane < nv && (lane == 0 || gup != g);
    const uint64_t runs = __ballot(start);
    const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(runs >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)runs, 0u));
    const int nr = __popcll(runs);
    const int32_t g_first = __builtin_amdgcn_readlane(g, 0);
    const int32_t g_last = __builtin_amdgcn_readlane(g, nv - 1);
    const int32_t g_before = __builtin_amdgcn_readlane(g, 32);
    const int32_t g_after = __builtin_amdgcn_readlane(g, 33);
    const int ps = e0 > 0 && g_before == g_first;
    const int ns = e0 + nv < a.E && g_after == g_last;
    if (start) {
      sw[kSlotRunStart + rank] = lane;
      sw[kSlotRunGroup + rank] = g;
    }
    if (lane == 0) sw[kSlotHdr] = nr | (ps << 8) | (ns << 9) | (nv << 16);
  }
};

// Barriers of the DMA ring.  __syncthreads() is a release fence plus
// s_barrier, and a release fence waits for every vector-memory operation,
// LDS-direct loads included: that would drain the ring at every tile.  So
// the waves wait for exactly what the others need and then meet at a bare
// s_barrier; the asm "memory" clobber keeps the compiler from moving memory
// accesses across it.
//   DMA waves:     their loads of tile t+1 have landed in LDS (at most N
//                  newer operations outstanding; vector memory retires in
//                  order), and their LDS writes (run tables) are done.
//   compute waves: their LDS reads of tile t are complete.
template <int N>
__device__ __forceinline__ void dma_barrier() {
  asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}
__device__ __forceinline__ void compute_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Non-finite tuple values in the run sums.  The products that form the
// sums of a tile's runs multiply every value of the tile by 0 or 1, and
// 0 x Inf is NaN, so one infinite value would reach every run of its tile.
// A wave that holds such a value (a wave-uniform test, rare) takes the
// non-finite values out of those products (finite_or_zero) and sums codes
// for them instead (codes: +Inf 1, -Inf 2^12, NaN 2^24; a run of at most
// 32 rows sums them exactly in FP32), from which nf_kind reads the run's
// non-finite part: NaN for a NaN or both infinities, else the infinity
// present, else 0.  Adding it to the finite part gives what plain addition
// gives, so a non-finite value stays in its own group.  The run sums are
// always formed as usual and only redone when the wave holds a non-finite
// value, so the usual path carries none of this work; the code sums are
// packed into two bits per column before the finite part is redone.
// The test is one sum of magnitudes per lane and one ballot: the sum is not
// finite when a value is not (a sum that overflows only takes the slow
// path, which gives the same result); a test per value, each compare
// feeding a scalar OR, cost a tenth of the BF16 kernel's time.
__device__ __forceinline__ float abs_sum(const f32x4& a) {
  return (fabsf(a[0]) + fabsf(a[1])) + (fabsf(a[2]) + fabsf(a[3]));
}
__device__ __forceinline__ bool wave_has_nonfinite(const f32x4& a, const f32x4& b) {
  return __ballot(!__builtin_isfinite(abs_sum(a) + abs_sum(b))) != 0;
}
__device__ __forceinline__ bool wave_has_nonfinite(const f32x4& a, const f32x4& b, const f32x4& c, const f32x4& d) {
  return __ballot(!__builtin_isfinite((abs_sum(a) + abs_sum(b)) + (abs_sum(c) + abs_sum(d)))) != 0;
}
__device__ __forceinline__ float finite_or_zero(float y) { return __builtin_isfinite(y) ? y : 0.0f; }
// kind of one value (0: finite, 1: +Inf, 2: -Inf, 3: NaN) and its code
__device__ __forceinline__ uint32_t nf_val_kind(float y) {
  const uint32_t u = __float_as_uint(y);
  const uint32_t k = (u & 0x7FFFFFu) ? 3u : (u >> 31) ? 2u : 1u;
  return (u & 0x7F800000u) == 0x7F800000u ? k : 0u;
}
__device__ __forceinline__ float nf_kind_code(uint32_t k) {
  k &= 3u;
  return k == 0u ? 0.0f : k == 1u ? 1.0f : k == 2u ? 4096.0f : 16777216.0f;
}
// 0: finite, 1: +Inf, 2: -Inf, 3: NaN
__device__ __forceinline__ uint32_t nf_kind(float code_sum) {
  if (code_sum == 0.0f) return 0u;
  if (code_sum >= 16777216.0f) return 3u;
  const float neg = floorf(code_sum * (1.0f / 4096.0f));
  const float pos = code_sum - 4096.0f * neg;
  return neg > 0.0f ? (pos > 0.0f ? 3u : 2u) : 1u;
}
__device__ __forceinline__ uint32_t nf_pack(const f32x4& n) {
  return nf_kind(n[0]) | (nf_kind(n[1]) << 2) | (nf_kind(n[2]) << 4) | (nf_kind(n[3]) << 6);
}
__device__ __forceinline__ float nf_value(uint32_t packed, int i) {
  const uint32_t k = (packed >> (2 * i)) & 3u;
  return k == 0u ? 0.0f : k == 1u ? INFINITY : k == 2u ? -INFINITY : __builtin_nanf("");
}
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// The same on eight bf16 values, on their bits (exponent all ones: not
// finite; codes 1.0 = 0x3F80, 2^12 = 0x4580, 2^24 = 0x4B80).
__device__ __forceinline__ uint32_t nf_half_code(uint32_t hb) {
  const uint32_t code = (hb & 0x7Fu) ? 0x4B80u : (hb & 0x8000u) ? 0x4580u : 0x3F80u;
  return (hb & 0x7F80u) == 0x7F80u ? code : 0u;
}
__device__ __forceinline__ bf16x8 finite_or_zero8(const bf16x8& v) {
  u32x4 u = __builtin_bit_cast(u32x4, v);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t x = u[i];
    const uint32_t bad = ((x & 0x7F80u) == 0x7F80u ? 0xFFFFu : 0u) |
                         ((x & 0x7F800000u) == 0x7F800000u ? 0xFFFF0000u : 0u);
    u[i] = x & ~bad;
  }
  return __builtin_bit_cast(bf16x8, u);
}
__device__ __forceinline__ bf16x8 nf_code8(const bf16x8& v) {
  u32x4 u = __builtin_bit_cast(u32x4, v);
#pragma unroll
  for (int i = 0; i < 4; ++i) u[i] = nf_half_code(u[i] & 0xFFFFu) | (nf_half_code(u[i] >> 16) << 16);
  return __builtin_bit_cast(bf16x8, u);
}

// A copy the compiler cannot see through: the slow path's work on values
// that do not change across the run passes would otherwise be hoisted out
// of the pass loop, and so out of its branch, into every tile.
__device__ __forceinline__ f32x4 opaque(f32x4 v) {
  asm volatile("" : "+v"(v));
  return v;
}
__device__ __forceinline__ bf16x8 opaque(bf16x8 v) {
  asm volatile("" : "+v"(v));
  return v;
}

// y if bit i of m is set, else +0 (a bit mask, not a multiply: exact for
// every y, infinities included)
__device__ __forceinline__ float keep_bit(float y, uint32_t m, int i) {
  return __int_as_float(__float_as_int(y) & ((int32_t)(m << (31 - i)) >> 31));
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

// Compute waves of the BF16 SUM / MEAN kernel with 32 output columns per
// wave (two 16-column slices of W): each A operand read from LDS feeds two
// products, half the LDS traffic of 16-column waves, which bound the BF16
// kernel.  The per-run sums are bf16 products on a two-term split of the
// FP32 tuple values, y = hi + lo with hi = bf16(y) and lo = bf16(y - hi)
// (about 16 significant bits, FP32 accumulation): one 16x16x32 product per
// term covers all 32 rows of the tile.  Its A operand is the lane's 8
// accumulator values (rows 4 (l/16) + i and 16 + 4 (l/16) + i, column
// l % 16) and its B operand whether each of those rows lies in the run of
// column l % 16, as in the FP32 kernel.
//
// WideMma holds a wave's slice of W in registers and multiplies one LDS
// tile; WideRed reduces the products of one tile into the wave's 32
// columns and carries the group left open at the tile's end.  (Giving each
// compute wave a reducer wave on its SIMD, with the accumulators passed
// through LDS, was slower: 3.7 against 2.8 ms for the ER Item rule.  The
// reducer's dependent chain alone took 3.4 ms, and the extra LDS buffer
// cost a tile of the load ring.)
template <int KP, int NB>
struct WideMma {
  using G = DmaGeo<__bf16, KP, NB>;
  static constexpr int NKS = KP / 32;
  static constexpr int PD = NKS < 4 ? NKS : 4;               // operand reads ahead of the products
  bf16x8 wA[NKS], wB[NKS];
  int b0[4], b1[4];
  int r0, r1;
  float bcA, bcB;

  __device__ __forceinline__ WideMma(const WsArgs& a, int cw, int lane) {
    const int colA = 32 * cw + (lane & 15);
    bcA = a.b ? a.b[colA] : 0.0f;
    bcB = a.b ? a.b[colA + 16] : 0.0f;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      wA[ks] = reinterpret_cast<const bf16x8*>(a.Wsw)[((2 * cw) * NKS + ks) * 64 + lane];
      wB[ks] = reinterpret_cast<const bf16x8*>(a.Wsw)[((2 * cw + 1) * NKS + ks) * 64 + lane];
    }
    __builtin_amdgcn_s_waitcnt(0);
    r0 = lane & 15;
    r1 = 16 + (lane & 15);
    const int cq = lane >> 4;
    auto chunk_base = [&](int sw, int j) { return 4 * (j ^ (sw >> 2)) + ((cq ^ sw) & 3); };
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      b0[j] = G::EPC * chunk_base(r0 & G::SWM, j);
      b1[j] = G::EPC * chunk_base(r1 & G::SWM, j);
    }
  }

  // x W + b of the tile at X: a0 / a1 rows 4 (l/16) + i and 16 + 4 (l/16) + i
  // of column block A (columns 32 cw + l % 16) and B (16 further)
  __device__ __forceinline__ void tile(const char* X, f32x4& a0A, f32x4& a1A, f32x4& a0B, f32x4& a1B) const {
    const __bf16* x0 = reinterpret_cast<const __bf16*>(X) + r0 * KP;
    const __bf16* x1 = reinterpret_cast<const __bf16*>(X) + r1 * KP;
    a0A = f32x4{bcA, bcA, bcA, bcA};
    a1A = a0A;
    a0B = f32x4{bcB, bcB, bcB, bcB};
    a1B = a0B;
    auto rd = [&](const __bf16* x, const int (&b)[4], int k) {
      return *reinterpret_cast<const bf16x8*>(x + 32 * (k & ~3) + b[k & 3]);
    };
    bf16x8 c0[PD], c1[PD];
#pragma unroll
    for (int p = 0; p < PD; ++p) {
      c0[p] = rd(x0, b0, p);
      c1[p] = rd(x1, b1, p);
    }
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const bf16x8 u0 = c0[ks % PD], u1 = c1[ks % PD];
      if (ks + PD < NKS) {
        c0[ks % PD] = rd(x0, b0, ks + PD);
        c1[ks % PD] = rd(x1, b1, ks + PD);
      }
      a0A = __builtin_amdgcn_mfma_f32_16x16x32_bf16(u0, wA[ks], a0A, 0, 0, 0);
      a1A = __builtin_amdgcn_mfma_f32_16x16x32_bf16(u1, wA[ks], a1A, 0, 0, 0);
      a0B = __builtin_amdgcn_mfma_f32_16x16x32_bf16(u0, wB[ks], a0B, 0, 0, 0);
      a1B = __builtin_amdgcn_mfma_f32_16x16x32_bf16(u1, wB[ks], a1B, 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
};

struct WideRed {
  // group open at the end of the previous tile, in the lanes of column off
  f32x4 oSA, oCA, oSB, oCB;
  int oN, off;
  bool oCut;
  int n16, q4, col4;

  __device__ __forceinline__ WideRed(int cw, int lane) {
    oSA = f32x4{0.f, 0.f, 0.f, 0.f};
    oCA = oSA;
    oSB = oSA;
    oCB = oSA;
    oN = 0;
    off = 0;
    oCut = false;
    n16 = lane & 15;
    q4 = 4 * (lane >> 4);
    col4 = 32 * cw + q4;
  }

  // the run-table words of this lane's first-pass run (read early, so the
  // LDS latency hides behind other work)
  struct Run {
    int hdr, rs0, rn0, gid0;
  };
  __device__ __forceinline__ Run run(const int32_t* gsl) const {
    const int gl = (n16 - off) & 15;
    return Run{gsl[kSlotHdr], gsl[kSlotRunStart + gl], gsl[kSlotRunStart + gl + 1], gsl[kSlotRunGroup + gl]};
  }

  // reduce tile t (index slot gsl) of the unit whose tiles are tb .. with
  // tuple values y = act_pre(acc) of this lane's 8 rows in each block
  __device__ __forceinline__ void tile(const WsArgs& a, const int32_t* gsl, const Run& R, int64_t t, int64_t tb,
                                       int64_t range_hi, int64_t bidx, f32x4 a0A, f32x4 a1A, f32x4 a0B,
                                       f32x4 a1B) {
    constexpr int TM = kTM;
    const int h = a.h;
    const int gl = (n16 - off) & 15;
    if (a.act_pre == RELNN_ACT_RELU) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a0A[i] = fmaxf(a0A[i], 0.0f);
        a1A[i] = fmaxf(a1A[i], 0.0f);
        a0B[i] = fmaxf(a0B[i], 0.0f);
        a1B[i] = fmaxf(a1B[i], 0.0f);
      }
    }
    // two-term bf16 split of this lane's 8 values of one column block, in
    // operand order (rows q4 + i, then 16 + q4 + i)
    auto split = [](const f32x4& y0, const f32x4& y1, bf16x8& hi, bf16x8& lo) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const float y = i < 4 ? y0[i] : y1[i - 4];
        const __bf16 hb = (__bf16)y;
        hi[i] = hb;
        lo[i] = (__bf16)(y - (float)hb);
      }
    };
    const bool nonfin = wave_has_nonfinite(a0A, a1A, a0B, a1B);
    bf16x8 hA, lA, hB, lB;
    split(a0A, a1A, hA, lA);
    split(a0B, a1B, hB, lB);

    const int hd = __builtin_amdgcn_readfirstlane(R.hdr);
    const int nr = hd & 63, nv = hd >> 16;
    const bool prev_same = (hd >> 8) & 1, next_same = (hd >> 9) & 1;
    const int64_t e0 = t * TM;
    const bool keep_open = next_same && e0 + nv < range_hi;
    for (int pass = 0; 16 * pass < nr; ++pass) {
      int g = gl, rs = R.rs0, rn = R.rn0, gid = R.gid0;
      if (pass) {                                            // runs 16 .. 31 (rare)
        g = 16 + gl;
        rs = gsl[kSlotRunStart + g];
        rn = gsl[kSlotRunStart + g + 1];
        gid = gsl[kSlotRunGroup + g];
      }
      const bool valid = g < nr;
      const int re = g + 1 < nr ? rn : nv;
      const uint32_t M = valid ? (0xffffffffu >> (32 - (re - rs))) << rs : 0u;   // rows [rs, re)
      const uint32_t bits = ((M >> q4) & 15u) | (((M >> (16 + q4)) & 15u) << 4);
      bf16x8 sel;
#pragma unroll
      for (int i = 0; i < 8; ++i) sel[i] = ((bits >> i) & 1u) ? (__bf16)1.0f : (__bf16)0.0f;
      f32x4 DA = {0.f, 0.f, 0.f, 0.f}, DB = DA;
      DA = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hA, sel, DA, 0, 0, 0);
      DB = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hB, sel, DB, 0, 0, 0);
      DA = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lA, sel, DA, 0, 0, 0);
      DB = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lB, sel, DB, 0, 0, 0);
      if (nonfin) {                // redone; a non-finite y has a non-finite hi term
        const f32x4 z = {0.f, 0.f, 0.f, 0.f};
        const bf16x8 xhA = opaque(hA), xlA = opaque(lA), xhB = opaque(hB), xlB = opaque(lB);
        const uint32_t nfA = nf_pack(__builtin_amdgcn_mfma_f32_16x16x32_bf16(nf_code8(xhA), sel, z, 0, 0, 0));
        const uint32_t nfB = nf_pack(__builtin_amdgcn_mfma_f32_16x16x32_bf16(nf_code8(xhB), sel, z, 0, 0, 0));
        DA = __builtin_amdgcn_mfma_f32_16x16x32_bf16(finite_or_zero8(xhA), sel, z, 0, 0, 0);
        DA = __builtin_amdgcn_mfma_f32_16x16x32_bf16(finite_or_zero8(xlA), sel, DA, 0, 0, 0);
        DB = __builtin_amdgcn_mfma_f32_16x16x32_bf16(finite_or_zero8(xhB), sel, z, 0, 0, 0);
        DB = __builtin_amdgcn_mfma_f32_16x16x32_bf16(finite_or_zero8(xlB), sel, DB, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          DA[i] += nf_value(nfA, i);
          DB[i] += nf_value(nfB, i);
        }
      }
      const int cnt = re - rs;
      const bool first = g == 0 && prev_same;
      const bool last = g == nr - 1 && next_same;
      f32x4 SA = DA, CA = {0.f, 0.f, 0.f, 0.f}, SB = DB, CB = CA;
      int ntot = cnt;
      bool cut = false;
      if (prev_same) {
        if (t > tb) {
          if (first) {                                       // the block's open group
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              float s1 = oSA[i], c1v = oCA[i];
              kahan_add(s1, c1v, DA[i]);
              oSA[i] = s1;
              oCA[i] = c1v;
              float s2 = oSB[i], c2v = oCB[i];
              kahan_add(s2, c2v, DB[i]);
              oSB[i] = s2;
              oCB[i] = c2v;
            }
            SA = oSA;
            CA = oCA;
            SB = oSB;
            CB = oCB;
            ntot = oN + cnt;
            cut = oCut;
          }
        } else {
          cut = first;                                       // began before the block's range
        }
      }
      if (valid) {
        if (last && keep_open) {                             // stays open for the next tile
          oSA = SA;
          oCA = CA;
          oSB = SB;
          oCB = CB;
          oN = ntot;
          oCut = cut;
        } else {
          const f32x4 vA = SA - CA, vB = SB - CB;
          if (last || cut) {                                 // partials for the fix-up
            const int slot = (last && !cut) ? 1 : 0;
            float* cp = a.carry + (bidx * 2 + slot) * h + col4;
            *reinterpret_cast<f32x4*>(cp) = vA;
            *reinterpret_cast<f32x4*>(cp + 16) = vB;
          } else {
            sink_write4(a.sink, gid, col4, h, vA, ntot);
            sink_write4(a.sink, gid, col4 + 16, h, vB, ntot);
          }
        }
      }
    }
    off = (off + nr - 1) & 15;
  }
};

template <int KP, int NB>
__device__ __forceinline__ void fwd_wide_bf16(const WsArgs& a, char* smem, int64_t tb, int64_t te, int64_t range_hi,
                                              int cw, int lane, int64_t bidx) {
  using G = DmaGeo<__bf16, KP, NB>;
  char* irs = smem + NB * G::TILE;
  auto wrap = [](int v, int n) { return v >= n ? v - n : v; };
  const WideMma<KP, NB> M(a, cw, lane);
  WideRed R(cw, lane);
  compute_barrier();                                         // (index slots staged)
  compute_barrier();                                         // tile tb is in LDS
  int rr = 0, ri = 0;
  for (int64_t t = tb; t < te; ++t) {
    const int32_t* gsl = reinterpret_cast<const int32_t*>(irs + ri * G::IRB);
    const WideRed::Run run = R.run(gsl);
    f32x4 a0A, a1A, a0B, a1B;
    M.tile(smem + rr * G::TILE, a0A, a1A, a0B, a1B);
    R.tile(a, gsl, run, t, tb, range_hi, bidx, a0A, a1A, a0B, a1B);
    rr = wrap(rr + 1, NB);
    ri = wrap(ri + 1, G::NIR);
    compute_barrier();
  }
}


// kWide: BF16 SUM / MEAN with h % 32 == 0 (32-column compute waves).
template <class T, int KP, int NB, bool kMax, bool kWide, bool kArg>
__global__ void __launch_bounds__(((kWide ? kHMax / 32 : kHMax / 16) + kDmaWaves) * 64) k_fwd_dma(WsArgs a) {
  static_assert(!kWide || (std::is_same<T, __bf16>::value && !kMax), "wide waves: BF16 SUM / MEAN");
  static_assert(!kArg || kMax, "maximiser positions: MAX only");
  using G = DmaGeo<T, KP, NB>;
  using WT = typename DmaMfma<T>::W;
  constexpr int NKS = DmaMfma<T>::template nks<KP>();
  constexpr int TM = kTM;
  // Block -> (tuple range, column chunk).  Workgroups are dealt to the 8
  // XCDs in turn, so blocks b and b + 8 share an L2: the nch chunks of one
  // range go to blocks 8 apart and start together, and the later gathers of
  // a row find it in that L2.  With one chunk this is the identity.
  const int64_t bid = blockIdx.x;
  const int chunk = (int)((bid >> 3) % a.nch);
  const int64_t bidx = (bid / (8 * a.nch)) * 8 + (bid & 7);
  if (a.E_dev) {                   // run-time size: as many units as tiles, at most the grid
    a.E = *a.E_dev;
    a.ntiles = (a.E + kTM - 1) / kTM;
    a.sg.n = a.E;
    a.nunits = max<int64_t>(1, min<int64_t>(a.nunits, a.ntiles));
  }
  if (bidx >= a.nunits) return;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int h = a.h;
  const int ncw = kWide ? a.hc / 32 : a.hc / 16;             // compute waves of the block
  const int wave = threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  const int64_t tb = (a.ntiles * bidx) / a.nunits;
  const int64_t te = (a.ntiles * (bidx + 1)) / a.nunits;
  const int64_t range_hi = min<int64_t>(te * TM, a.E);
  if (tb >= te) return;

  // zero the ring once (every chunk is rewritten per tile; this only keeps
  // uninitialised LDS out of the first products)
  for (int i = threadIdx.x; i < NB * G::TILE / 16; i += blockDim.x)
    reinterpret_cast<uint4*>(smem)[i] = make_uint4(0, 0, 0, 0);
  __syncthreads();
  char* irs = smem + NB * G::TILE;                          // row-number slots
  // ring position of a tile relative to tb: tile (it % NB), index slot
  // (it % NIR); both kept as wrapping 32-bit counters
  auto wrap = [](int v, int n) { return v >= n ? v - n : v; };

  if (wave >= ncw) {
    // ------------------------------------------------------------ DMA waves
    // At iteration t a wave issues the index slot of tile t+2NB-2, then its
    // share of tile t+NB-1, then waits until its share of tile t+1 has
    // landed.  The index slot of tile v is issued just before tile v-NB+1,
    // so it has landed (and passed a barrier) before tile v is issued.
    const int dw = wave - ncw;
    const DmaPlan<T, KP, NB> P(a, dw);
    const int64_t tl = te - 1;
#pragma unroll
    for (int j = 0; j + 1 < NB; ++j) P.index(a, min(tb + j, tl), irs + j * G::IRB, dw);
    asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");   // index slots of tb .. tb+NB-2
#pragma unroll
    for (int j = 0; j + 1 < NB; ++j) {
      P.index(a, min(tb + j + NB - 1, tl), irs + (j + NB - 1) * G::IRB, dw);
      P.tile(irs + j * G::IRB, smem + j * G::TILE, dw);
      if (!kMax && dw == 0) P.run_table(a, min(tb + j, tl), irs + j * G::IRB);
    }
    dma_barrier<G::WAIT>();                                   // tile tb has landed
    int si = (2 * NB - 2) % G::NIR;                           // index slot of tile t + 2NB - 2
    int sr = NB - 1;                                          // index slot of tile t + NB - 1
    int rr = NB - 1;                                          // ring tile of tile t + NB - 1
    for (int64_t t = tb; t < te; ++t) {
      P.index(a, min(t + 2 * NB - 2, tl), irs + si * G::IRB, dw);
      P.tile(irs + sr * G::IRB, smem + rr * G::TILE, dw);
      if (!kMax && dw == 0) P.run_table(a, min(t + NB - 1, tl), irs + sr * G::IRB);
      dma_barrier<G::WAIT>();                                 // tile t+1 has landed
      si = wrap(si + 1, G::NIR);
      sr = wrap(sr + 1, G::NIR);
      rr = wrap(rr + 1, NB);
    }
    // loads past the range may still be landing: the LDS must not be
    // released to another block before they have
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    return;
  }

  // -------------------------------------------------------------- compute waves
  if constexpr (kWide) {
    fwd_wide_bf16<KP, NB>(a, smem, tb, te, range_hi, chunk * ncw + wave, lane, bidx);
    return;
  }
  const int cw = chunk * ncw + wave;                         // 16-column slice of W and out
  const int col = cw * 16 + (lane & 15);
  const float bc = a.b ? a.b[col] : 0.0f;
  WT w[NKS];
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks) w[ks] = reinterpret_cast<const WT*>(a.Wsw)[(cw * NKS + ks) * 64 + lane];
  // W has landed before the loop: otherwise the compiler waits for it (and
  // with it for the group numbers of the next tile) at every tile's MFMAs
  __builtin_amdgcn_s_waitcnt(0);

  const int q4 = 4 * (lane >> 4);
  const int r0 = lane & 15, r1 = 16 + (lane & 15);
  const int cq = lane >> 4;
  // A operand of step m: logical chunk 4m + cq of rows r0 / r1, stored at
  // position (4m + cq) ^ sw = 4 (m ^ (sw >> 2)) + ((cq ^ sw) & 3): a per-lane
  // base for m % 4 plus a constant for the rest (four registers per row
  // instead of one address per step)
  auto chunk_base = [&](int sw, int j) { return 4 * (j ^ (sw >> 2)) + ((cq ^ sw) & 3); };
  int b0[4], b1[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    b0[j] = G::EPC * chunk_base(r0 & G::SWM, j);
    b1[j] = G::EPC * chunk_base(r1 & G::SWM, j);
  }

  // MAX: state of the group open at the end of the previous tile, per
  // column (the 4 lanes of a column hold the same values)
  float mS = -INFINITY;
  int32_t mArg = -1;
  int mN = 0;
  bool mCut = false;
  const int64_t slot_base = bidx * 2 * h + col;
  // SUM / MEAN: run g of a tile is summed into column (g + off) % 16 of the
  // reduce product, with off the column of the previous tile's last run, so
  // a group that runs on from one tile to the next stays in the same lanes
  // (no data movement).  Lane l of those lanes holds output columns
  // 4 (l / 16) .. + 3 of the open group (sum, Kahan compensation, count).
  f32x4 oS = {0.f, 0.f, 0.f, 0.f}, oC = {0.f, 0.f, 0.f, 0.f};
  int oN = 0;
  bool oCut = false;
  int off = 0;
  const int n16 = lane & 15;
  const int col4 = cw * 16 + q4;                             // first of this lane's 4 reduce columns

  // MAX: reduces tile t from its products (acc0, acc1) and group numbers.
  auto max_tile = [&](int64_t t, f32x4 acc0, f32x4 acc1, int32_t gcur) {
    const int64_t e0 = t * TM;
    // ---- MAX: a segmented max-scan of the tile, whose cost does not
    // depend on the number of runs.  A lane holds rows q4 .. q4+3 (acc0)
    // and 16+q4 .. (acc1) of its column: each 4-row block is scanned in
    // the lane, the block tails across the column's 4 lane rows with two
    // row swaps (whether a block holds a run start follows from the
    // wave-uniform start mask, so only values and positions move), and
    // every row then holds the max of its run up to that row and the
    // run's first maximiser.  The rows that end a run write it.
    const int nv = (int)min<int64_t>(TM, a.E - e0);
    const int32_t gup = __builtin_amdgcn_update_dpp(0, gcur, 0x138, 0xf, 0xf, false);
    const bool start = lane < nv && (lane == 0 || gup != gcur);
    const uint32_t runs = (uint32_t)__ballot(start);
    const int32_t g_first = __builtin_amdgcn_readlane(gcur, 0);
    const int32_t g_last = __builtin_amdgcn_readlane(gcur, nv - 1);
    const int32_t g_before = __builtin_amdgcn_readlane(gcur, 32);
    const int32_t g_after = __builtin_amdgcn_readlane(gcur, 33);
    const bool prev_same = e0 > 0 && g_before == g_first;
    const bool next_same = e0 + nv < a.E && g_after == g_last;
    const bool keep_open = next_same && e0 + nv < range_hi;
    const bool open_in = prev_same && t > tb;            // row 0 continues the block's open group
    const uint32_t sm = open_in ? (runs & ~1u) : runs;   // starts as the scan sees them
    const int qr = lane >> 4;                             // lane row of the column
    // (lv, la) followed by (rv, ra): the later one wins only if strictly
    // greater; (-inf, INT32_MAX) is the empty prefix
    // Without positions (no argmax asked for) only the values are kept:
    // the empty prefix is -inf, which any value replaces or equals.
    auto comb = [](float lv, int32_t la, float rv, int32_t ra, float& ov, int32_t& oa) {
      if constexpr (kArg) {
        const bool take = rv > lv || la == INT32_MAX;
        ov = take ? rv : lv;
        oa = take ? ra : la;
      } else {
        ov = rv > lv ? rv : lv;
        oa = 0;
      }
    };
    auto any_start = [&](int r0s, int n) { return ((sm >> r0s) & ((1u << n) - 1u)) != 0u; };
    // carry into the first row
    float cv = open_in ? mS : -INFINITY;
    int32_t ca = open_in ? mArg : INT32_MAX;
    float fv[8];                                         // per row: run max so far
    int32_t fa[8];                                       // ... and its first maximiser
#pragma unroll
    for (int set = 0; set < 2; ++set) {
      const int base = 16 * set;
      float sv[4];
      int32_t sa[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {                      // in-lane scan of the block
        const int r = base + q4 + i;
        const float y = set ? acc1[i] : acc0[i];
        const int32_t pos = (int32_t)(e0 + r);
        if (i == 0) {
          sv[0] = y;
          sa[0] = pos;
        } else {
          comb(sv[i - 1], sa[i - 1], y, pos, sv[i], sa[i]);
          const bool st = (sm >> r) & 1u;
          sv[i] = st ? y : sv[i];
          sa[i] = st ? pos : sa[i];
        }
      }
      // block tails across the lane rows: pairs (0,1), (2,3), then halves
      const float tv = sv[3];
      const int32_t ta = sa[3];
      const auto p16v = __builtin_amdgcn_permlane16_swap(__float_as_uint(tv), __float_as_uint(tv), false, false);
      const auto p16a = __builtin_amdgcn_permlane16_swap((uint32_t)ta, (uint32_t)ta, false, false);
      const bool odd = qr & 1;
      // the pair partner's tail (rows 0 <-> 1, 2 <-> 3)
      const float xv = __uint_as_float(odd ? p16v[0] : p16v[1]);
      const int32_t xa = (int32_t)(odd ? p16a[0] : p16a[1]);
      const int pr = base + 4 * (qr & 2);                // first row of this lane's pair
      // pair total: the later block's tail if it holds a start
      float pv;
      int32_t pa;
      {
        const float lv = odd ? xv : tv, rv = odd ? tv : xv;
        const int32_t la = odd ? xa : ta, ra = odd ? ta : xa;
        comb(lv, la, rv, ra, pv, pa);
        const bool rf = any_start(pr + 4, 4);
        pv = rf ? rv : pv;
        pa = rf ? ra : pa;
      }
      const auto p32v = __builtin_amdgcn_permlane32_swap(__float_as_uint(pv), __float_as_uint(pv), false, false);
      const auto p32a = __builtin_amdgcn_permlane32_swap((uint32_t)pa, (uint32_t)pa, false, false);
      const bool hi = qr & 2;
      const float ov = __uint_as_float(hi ? p32v[0] : p32v[1]);    // the other pair's total
      const int32_t oa = (int32_t)(hi ? p32a[0] : p32a[1]);
      // prefix of the blocks before this lane's block
      float ev = -INFINITY;
      int32_t ea = INT32_MAX;
      if (qr == 1) {
        ev = xv;
        ea = xa;
      } else if (qr == 2) {
        ev = ov;
        ea = oa;
      } else if (qr == 3) {                              // pair (0,1), then block 2
        comb(ov, oa, xv, xa, ev, ea);
        const bool f2 = any_start(base + 8, 4);
        ev = f2 ? xv : ev;
        ea = f2 ? xa : ea;
      }
      // carry into this block: the set's carry, then that prefix
      float kv;
      int32_t ka;
      comb(cv, ca, ev, ea, kv, ka);
      const bool pf = any_start(base, q4);               // a start in an earlier block of the set
      kv = pf ? ev : kv;
      ka = pf ? ea : ka;
#pragma unroll
      for (int i = 0; i < 4; ++i) {                      // rows before the block's first start
        float v;
        int32_t ag;
        comb(kv, ka, sv[i], sa[i], v, ag);
        const bool own = any_start(base + q4, i + 1);
        fv[4 * set + i] = own ? sv[i] : v;
        fa[4 * set + i] = own ? sa[i] : ag;
      }
      // carry into the next set: the whole set after the current carry
      float tot_v;
      int32_t tot_a;
      {
        const float lv = hi ? ov : pv, rv = hi ? pv : ov;
        const int32_t la = hi ? oa : pa, ra = hi ? pa : oa;
        comb(lv, la, rv, ra, tot_v, tot_a);
        const bool rf = any_start(base + 8, 8);
        tot_v = rf ? rv : tot_v;
        tot_a = rf ? ra : tot_a;
      }
      float nv2;
      int32_t na2;
      comb(cv, ca, tot_v, tot_a, nv2, na2);
      const bool sf = any_start(base, 16);
      cv = sf ? tot_v : nv2;
      ca = sf ? tot_a : na2;
    }
    // outputs: rows that end a run
    const uint32_t first_run_rows = (sm & ~1u) == 0u ? 0xffffffffu : ((sm & ~1u) & (0u - (sm & ~1u))) - 1u;
    const bool cut0 = prev_same && (open_in ? mCut : true);
    // Rows that end a run (a wave-uniform mask).  Row r lives in the lanes
    // of lane row (r % 16) / 4, register (r % 4) + 4 (r / 16).  The ends
    // are visited one by one, so the cost follows the number of runs.
    const uint32_t valid = nv >= 32 ? 0xffffffffu : ((1u << nv) - 1u);
    const uint32_t ends = ((runs >> 1) | (1u << (nv - 1))) & valid;
    const uint32_t last_bit = 1u << (nv - 1);
    const uint32_t first_end = ends & (0u - ends);       // end of the first run
    auto row_val = [&](int r, float& v, int32_t& ag) {
      const int i = (r & 3) + ((r >> 2) & 4);
      v = fv[0];
      ag = fa[0];
#pragma unroll
      for (int k = 1; k < 8; ++k) {
        v = i == k ? fv[k] : v;
        ag = i == k ? fa[k] : ag;
      }
    };
    const bool has_pre = a.sink.pre != nullptr, has_arg = a.sink.argmax != nullptr;
    const bool obf = a.sink.out_bf16;
    // Runs finished inside the tile.  Each lane row of the column writes the
    // run ends among its own rows, one per pass, so a store instruction
    // carries up to four ends (all 64 lanes) instead of one (16 lanes):
    // one end per instruction spent more than half of the BF16 kernel's
    // time in the stores.
    const uint32_t plain = ends & ~(next_same ? last_bit : 0u) & ~(cut0 ? first_end : 0u);
    uint32_t mine = plain & ((0xFu << (4 * qr)) | (0xF0000u << (4 * qr)));   // rows of this lane row
    while (__ballot(mine != 0u)) {                       // wave-uniform: every lane runs each pass
      const bool has = mine != 0u;
      const int r = has ? __builtin_ctz(mine) : 0;
      mine &= mine - 1u;
      float v;
      int32_t ag;
      row_val(r, v, ag);
      // lane r holds the group of row r; read with every lane active (a
      // permute from an inactive lane does not return its value)
      const int32_t gid = __shfl(gcur, r);
      if (has) {
        const int64_t o = (int64_t)gid * h + col;
        if (has_pre) a.sink.pre[o] = v;
        if (kArg && has_arg) a.sink.argmax[o] = ag;
        const float w = act_apply(a.sink.act_post, v);
        if (obf)
          reinterpret_cast<__bf16*>(a.sink.out)[o] = (__bf16)w;
        else
          a.sink.out[o] = w;
      }
    }
    // the first run, cut by the range start, and the last one, running
    // past the range end, leave partials in the block's carry slots
    const bool first_cut = cut0 && !(first_end == last_bit && keep_open);
    const bool last_out = next_same && !keep_open && !(cut0 && first_end == last_bit);
    if (first_cut || last_out) {
      float v;
      int32_t ag;
      if (first_cut) {
        const int r = __builtin_ctz(first_end);
        row_val(r, v, ag);
        if (qr == ((r >> 2) & 3)) {
          a.carry[slot_base] = v;
          if (a.carry_arg) a.carry_arg[slot_base] = kArg ? ag : 0;
        }
      }
      if (last_out) {
        const int r = nv - 1;
        row_val(r, v, ag);
        if (qr == ((r >> 2) & 3)) {
          a.carry[slot_base + h] = v;
          if (a.carry_arg) a.carry_arg[slot_base + h] = kArg ? ag : 0;
        }
      }
    }
    if (keep_open) {                                     // row nv-1 to every lane row of the column
      const int rl = nv - 1, ql = (rl & 15) >> 2, il = (rl & 3) + (rl >= 16 ? 4 : 0);
      float v = fv[0];
      int32_t ag = fa[0];
#pragma unroll
      for (int i = 1; i < 8; ++i) {
        v = il == i ? fv[i] : v;
        ag = il == i ? fa[i] : ag;
      }
      const auto s16v = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
      const auto s16a = __builtin_amdgcn_permlane16_swap((uint32_t)ag, (uint32_t)ag, false, false);
      if ((qr & 1) != (ql & 1)) {
        v = __uint_as_float((qr & 1) ? s16v[0] : s16v[1]);
        ag = (int32_t)((qr & 1) ? s16a[0] : s16a[1]);
      }
      const auto s32v = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
      const auto s32a = __builtin_amdgcn_permlane32_swap((uint32_t)ag, (uint32_t)ag, false, false);
      if ((qr & 2) != (ql & 2)) {
        v = __uint_as_float((qr & 2) ? s32v[0] : s32v[1]);
        ag = (int32_t)((qr & 2) ? s32a[0] : s32a[1]);
      }
      mS = v;
      mArg = ag;
      mCut = ((first_run_rows >> rl) & 1u) && cut0;
    }
  };
  // MAX with more than 4 compute waves: waves 4.. (which share SIMDs with
  // waves 0..3) reduce each tile one iteration late, before the products of
  // the next one, so that on every SIMD one wave runs the scan while the
  // other keeps the matrix core busy.  Only the group numbers are read from
  // the tile's index slot, and they move to the next iteration in a
  // register.
  // (not for FP32 tiles 384 wide, whose W slice leaves no registers for
  // the late tile's products)
  constexpr bool kLag = kMax && !(std::is_same<T, float>::value && KP >= 384);
  const bool lag = kLag && ncw > 4 && wave >= 4;
  f32x4 lacc0 = {0.f, 0.f, 0.f, 0.f}, lacc1 = lacc0;
  int32_t lgcur = 0;

  compute_barrier();                                         // (index slots staged)
  compute_barrier();                                         // tile tb is in LDS
  int rr = 0, ri = 0;                                        // ring tile, index slot of t
  for (int64_t t = tb; t < te; ++t) {
    if constexpr (kMax) {
      if (lag && t > tb) max_tile(t - 1, lacc0, lacc1, lgcur);
    }
    const int32_t* gsl = reinterpret_cast<const int32_t*>(irs + ri * G::IRB);
    // MAX: group numbers of tile t (lane r < 32 row r, clamped; lane 32 the
    // row before the tile, lane 33 the row after it).  SUM / MEAN: the run
    // table, this lane's run of the first pass.
    int32_t gcur = 0, hdr = 0, rs0 = 0, rn0 = 0, gid0 = 0;
    const int gl = (n16 - off) & 15;
    if constexpr (kMax) {
      gcur = gsl[lane < 32 ? kSlotSeg + lane : kSlotEdge + min(lane - 32, 1)];
    } else {
      hdr = gsl[kSlotHdr];
      rs0 = gsl[kSlotRunStart + gl];
      rn0 = gsl[kSlotRunStart + gl + 1];
      gid0 = gsl[kSlotRunGroup + gl];
    }
    const char* X = smem + rr * G::TILE;
    // the bias is the accumulators' initial value
    f32x4 acc0 = {bc, bc, bc, bc}, acc1 = {bc, bc, bc, bc};
    if constexpr (std::is_same<T, float>::value) {
      const float* x0 = reinterpret_cast<const float*>(X) + r0 * KP;
      const float* x1 = reinterpret_cast<const float*>(X) + r1 * KP;
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
      // operand reads run PD steps ahead of the products
      const __bf16* x0 = reinterpret_cast<const __bf16*>(X) + r0 * KP;
      const __bf16* x1 = reinterpret_cast<const __bf16*>(X) + r1 * KP;
      constexpr int PD = NKS < 4 ? NKS : 4;
      auto rd = [&](const __bf16* x, const int (&b)[4], int k) {
        return *reinterpret_cast<const bf16x8*>(x + 32 * (k & ~3) + b[k & 3]);
      };
      bf16x8 c0[PD], c1[PD];
#pragma unroll
      for (int p = 0; p < PD; ++p) {
        c0[p] = rd(x0, b0, p);
        c1[p] = rd(x1, b1, p);
      }
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        const bf16x8 u0 = c0[ks % PD], u1 = c1[ks % PD];
        if (ks + PD < NKS) {
          c0[ks % PD] = rd(x0, b0, ks + PD);
          c1[ks % PD] = rd(x1, b1, ks + PD);
        }
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(u0, w[ks], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(u1, w[ks], acc1, 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // tuple values y = act_pre(x W + b); this lane's rows: q4 + i (acc0)
    // and 16 + q4 + i (acc1)
    if (a.act_pre == RELNN_ACT_RELU) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        acc0[i] = fmaxf(acc0[i], 0.0f);
        acc1[i] = fmaxf(acc1[i], 0.0f);
      }
    }
    const int64_t e0 = t * TM;

    if constexpr (!kMax) {
      const bool nonfin = wave_has_nonfinite(acc0, acc1);
      // ---- SUM / MEAN: per-run sums on the matrix cores.  With S the 0/1
      // matrix [row][run] of the tile, D[c][n] = sum_row y[row][c] S[row][n]
      // is one f32 16x16x4 product per accumulator register: its A operand
      // is the register itself (lane l: row 4 (l/16) + i, column l % 16)
      // and its B operand lane l: whether that row lies in the run of
      // column l % 16.  D lane l holds columns 4 (l/16) .. + 3 of that run.
      const int hd = __builtin_amdgcn_readfirstlane(hdr);
      const int nr = hd & 63, nv = hd >> 16;
      const bool prev_same = (hd >> 8) & 1, next_same = (hd >> 9) & 1;
      const bool keep_open = next_same && e0 + nv < range_hi;
      for (int pass = 0; 16 * pass < nr; ++pass) {
        int g = gl, rs = rs0, rn = rn0, gid = gid0;
        if (pass) {                                          // runs 16 .. 31 (rare)
          g = 16 + gl;
          rs = gsl[kSlotRunStart + g];
          rn = gsl[kSlotRunStart + g + 1];
          gid = gsl[kSlotRunGroup + g];
        }
        const bool valid = g < nr;
        const int re = g + 1 < nr ? rn : nv;
        const uint32_t M = valid ? (0xffffffffu >> (32 - (re - rs))) << rs : 0u;   // rows [rs, re)
        const uint32_t m0 = M >> q4, m1 = M >> (16 + q4);
        f32x4 D = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 4; ++i)
          D = __builtin_amdgcn_mfma_f32_16x16x4f32(acc0[i], keep_bit(1.0f, m0, i), D, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i)
          D = __builtin_amdgcn_mfma_f32_16x16x4f32(acc1[i], keep_bit(1.0f, m1, i), D, 0, 0, 0);
        if (nonfin) {            // redone: the finite part, then the run's non-finite part added
          const f32x4 y0 = opaque(acc0), y1 = opaque(acc1);
          f32x4 N = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            N = __builtin_amdgcn_mfma_f32_16x16x4f32(nf_kind_code(nf_val_kind(y0[i])), keep_bit(1.0f, m0, i), N, 0,
                                                     0, 0);
            N = __builtin_amdgcn_mfma_f32_16x16x4f32(nf_kind_code(nf_val_kind(y1[i])), keep_bit(1.0f, m1, i), N, 0,
                                                     0, 0);
          }
          const uint32_t nfp = nf_pack(N);
          D = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            D = __builtin_amdgcn_mfma_f32_16x16x4f32(finite_or_zero(y0[i]), keep_bit(1.0f, m0, i), D, 0, 0, 0);
            D = __builtin_amdgcn_mfma_f32_16x16x4f32(finite_or_zero(y1[i]), keep_bit(1.0f, m1, i), D, 0, 0, 0);
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) D[i] += nf_value(nfp, i);
        }
        const int cnt = re - rs;
        const bool first = g == 0 && prev_same;              // continues the group open before the tile
        const bool last = g == nr - 1 && next_same;          // runs on past the tile
        f32x4 S = D, C = {0.f, 0.f, 0.f, 0.f};
        int ntot = cnt;
        bool cut = false;
        if (prev_same) {
          if (t > tb) {
            if (first) {                                     // the block's open group
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                float si = oS[i], ci = oC[i];
                kahan_add(si, ci, D[i]);
                oS[i] = si;
                oC[i] = ci;
              }
              S = oS;
              C = oC;
              ntot = oN + cnt;
              cut = oCut;
            }
          } else {
            cut = first;                                     // began before the block's range
          }
        }
        if (valid) {
          if (last && keep_open) {                           // stays open for the next tile
            oS = S;
            oC = C;
            oN = ntot;
            oCut = cut;
          } else {
            const f32x4 v = S - C;
            if (last || cut) {                               // partial for the fix-up
              const int slot = (last && !cut) ? 1 : 0;
              *reinterpret_cast<f32x4*>(a.carry + (bidx * 2 + slot) * h + col4) = v;
            } else {
              sink_write4(a.sink, gid, col4, h, v, ntot);
            }
          }
        }
      }
      off = (off + nr - 1) & 15;
    } else if (lag) {                  // reduced in the next iteration
      lacc0 = acc0;
      lacc1 = acc1;
      lgcur = gcur;
    } else {
      max_tile(t, acc0, acc1, gcur);
    }
    rr = wrap(rr + 1, NB);
    ri = wrap(ri + 1, G::NIR);
    compute_barrier();
  }
  if constexpr (kMax) {
    if (lag) max_tile(te - 1, lacc0, lacc1, lgcur);
  }
}

// ---------------------------------------------------------------- pushdown
// Transform pushed below the join (affine tau only): with P_j = Z_j W_j
// computed once per row of atom j, the tuple value is sum_j P_j[r_j] + b.
// The P rows of the atoms that vary inside a group are summed per tuple and
// aggregated per group; the others, and b, are one constant per group that
// the sink adds.  This is a segmented gather-sum over the sorted tuple list:
// one wave per contiguous range of positions (boundaries on multiples of
// kPsTM), lane l owning columns 2 l, 2 l + 1 of each 128-column block, rows
// of kPsBatch tuples loaded together.  SUM / MEAN accumulate with Kahan
// compensation, MAX keeps the value and its first maximiser; a group cut by
// a range end leaves its partial in carry slot 0 (cut by the start) or 1
// (runs past the end), which k_fixup combines in range order.
struct PushArgs {
  int n;                                  // atoms gathered per tuple
  const void* P[RELNN_MAX_ATOMS];         // [n_rows_j][h]: FP32 node products, or the embeddings (product)
  const int32_t* rows[RELNN_MAX_ATOMS];   // [E] joined row per tuple
  int act_pre;                            // product transform: activation per tuple
};

// Gather-combine modes: the sum of FP32 node products (pushdown), or the
// product of the atoms' embeddings, FP32 or bf16 (product transform).
enum { PS_SUM = 0, PS_PROD_F32 = 1, PS_PROD_BF16 = 2 };

// Second pass of the pushdown: V holds each group's aggregate of the varying
// atoms (MEAN already divided by the count); the group constant is added
// (count times for SUM) and the result written through the sink.  One
// thread per (group, column): the constant's loads are independent here,
// where in the gather-sum they would stall a wave at every group end.
__global__ void k_push_finish(const float* V, int64_t G, int h, Sink k) {
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  const int C4 = h / 4;                                     // h % 4 == 0 for the pushdown
  const GroupConst& gc = k.gc;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < G * C4;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = i / C4;
    const int c = 4 * (int)(i - s * C4);
    const int64_t e0 = gc.offsets[s];
    f32x4 g = gc.bias ? *reinterpret_cast<const f32x4*>(gc.bias + c) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < RELNN_MAX_ATOMS; ++j)    // constant trip count: no run-time index into the argument
      if (j < gc.n) g += *reinterpret_cast<const f32x4*>(gc.P[j] + (int64_t)gc.rows[j][e0] * h + c);
    const float cnt = (float)(gc.offsets[s + 1] - e0);
    f32x4 v = *reinterpret_cast<const f32x4*>(V + s * h + c);
    v += k.agg == RELNN_SUM ? cnt * g : g;
    const int64_t o = (k.out_row ? (int64_t)k.out_row[s] : s) * h + c;
    if (k.pre) *reinterpret_cast<f32x4*>(k.pre + o) = v;
    if (k.accumulate) {
      *reinterpret_cast<f32x4*>(k.out + o) += v;
    } else {
      f32x4 w;
#pragma unroll
      for (int q = 0; q < 4; ++q) w[q] = act_apply(k.act_post, v[q]);
      if (k.out_bf16) {
        bf16x4 b;
#pragma unroll
        for (int q = 0; q < 4; ++q) b[q] = (__bf16)w[q];
        *reinterpret_cast<bf16x4*>(reinterpret_cast<__bf16*>(k.out) + o) = b;
      } else {
        *reinterpret_cast<f32x4*>(k.out + o) = w;
      }
    }
  }
}

constexpr int kPsTM = 64;       // range boundaries on multiples of 64 positions
constexpr int kPsWaves = 4;     // waves per block
constexpr int kPsBatch = 8;     // tuples whose rows are loaded together

// kNA: the number of atoms gathered per tuple, fixed at compile time (no
// run-time atom loop around a batch's loads); with the rows read through
// buffer resources this took the ER pushdown gather-sum from 2.80 to 1.69
// ms a launch.
template <int kMode, int kNA>
__global__ void __launch_bounds__(kPsWaves * 64) k_push_sum(WsArgs a, PushArgs pa) {
  const int lane = threadIdx.x % 64;
  const int64_t u = (int64_t)blockIdx.x * kPsWaves + threadIdx.x / 64;
  if (u >= a.nunits) return;
  const int64_t r0 = ((a.ntiles * u) / a.nunits) * kPsTM;
  const int64_t r1 = min<int64_t>(((a.ntiles * (u + 1)) / a.nunits) * kPsTM, a.E);
  if (r0 >= r1) return;
  const int h = a.h;
  const bool is_max = a.sink.agg == RELNN_MAX;
  for (int cb = 0; cb < h; cb += 128) {
    const int col = cb + 2 * lane;
    const bool on = col < h;
    const int cc = on ? col : 0;
    const float s_init = is_max ? -INFINITY : 0.0f;
    float s0 = s_init, s1 = s_init, c0 = 0.0f, c1 = 0.0f;
    int32_t m0 = -1, m1 = -1;                              // MAX: first maximiser, -1 before any tuple
    int32_t g = a.sg.seg_of[r0];
    // only the range's first group can have begun before r0, and only its
    // last one can run past r1 (one list read at each end); a group wholly
    // inside the range has the count of tuples seen here
    const bool lo_cont = r0 > 0 && a.sg.seg_of[r0 - 1] == g;
    bool first = true;
    int32_t cnt = 0;
    auto flush = [&](bool last_seg) {
      const bool cut_lo = first && lo_cont;
      const bool cut_hi = last_seg && r1 < a.E && a.sg.seg_of[r1] == g;
      if (on) {
        const float v0 = is_max ? s0 : s0 - c0, v1 = is_max ? s1 : s1 - c1;
        if (cut_lo || cut_hi) {
          const int64_t o = (u * 2 + (cut_lo ? 0 : 1)) * h + col;
          a.carry[o] = v0;
          a.carry[o + 1] = v1;
          if (a.carry_arg) {
            a.carry_arg[o] = m0;
            a.carry_arg[o + 1] = m1;
          }
        } else {
          sink_write(a.sink, g, col, h, v0, m0, cnt);
          sink_write(a.sink, g, col + 1, h, v1, m1, cnt);
        }
      }
      first = false;
      cnt = 0;
      s0 = s_init;
      s1 = s_init;
      c0 = 0.0f;
      c1 = 0.0f;
      m0 = -1;
      m1 = -1;
    };
    for (int64_t base = r0; base < r1; base += 64) {
      const int n = (int)min<int64_t>(64, r1 - base);
      const int64_t e = base + min(lane, n - 1);
      const int32_t gl = a.sg.seg_of[e];
      // row numbers of the 64 positions, one vector per atom (compile-time
      // atom indices: a run-time index into the argument would put it in
      // scratch memory)
      int32_t R[kNA];
#pragma unroll
      for (int j = 0; j < kNA; ++j) R[j] = pa.rows[j][e];
      for (int bt = 0; bt < n; bt += kPsBatch) {
        float2 v[kPsBatch];
#pragma unroll
        for (int i = 0; i < kPsBatch; ++i) {
          const int q = min(bt + i, n - 1);                 // clamped: every load is valid
          v[i] = kMode == PS_SUM ? make_float2(0.0f, 0.0f) : make_float2(1.0f, 1.0f);
#pragma unroll
          for (int j = 0; j < kNA; ++j) {
            {
              const int32_t row = __builtin_amdgcn_readlane(R[j], q);
              // the row as a buffer resource (scalar registers) read at a
              // 32-bit lane offset: a batch of loads holds no per-lane
              // 64-bit addresses
              constexpr int esz = kMode == PS_PROD_BF16 ? 2 : 4;
              const __amdgpu_buffer_rsrc_t rs = row_rsrc(static_cast<const char*>(pa.P[j]) + (int64_t)row * h * esz,
                                                         (uint32_t)(h * esz));
              float2 p;
              if constexpr (kMode == PS_PROD_BF16) {
                const uint32_t u = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, 2u * (uint32_t)cc, 0, 0);
                p = make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
              } else {
                p = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, 4u * (uint32_t)cc, 0, 0));
              }
              if constexpr (kMode == PS_SUM) {
                v[i].x += p.x;
                v[i].y += p.y;
              } else {
                v[i].x *= p.x;
                v[i].y *= p.y;
              }
            }
          }
          if (kMode != PS_SUM && pa.act_pre == RELNN_ACT_RELU) {
            v[i].x = fmaxf(v[i].x, 0.0f);
            v[i].y = fmaxf(v[i].y, 0.0f);
          }
        }
#pragma unroll
        for (int i = 0; i < kPsBatch; ++i) {
          const int q = bt + i;
          if (q >= n) break;
          const int32_t gq = __builtin_amdgcn_readlane(gl, q);
          if (gq != g) {                                     // a group ends
            flush(false);
            g = gq;
          }
          ++cnt;
          if (is_max) {
            const int32_t pos = (int32_t)(base + q);
            if (v[i].x > s0 || m0 < 0) {
              s0 = v[i].x;
              m0 = pos;
            }
            if (v[i].y > s1 || m1 < 0) {
              s1 = v[i].y;
              m1 = pos;
            }
          } else {
            kahan_add(s0, c0, v[i].x);
            kahan_add(s1, c1, v[i].y);
          }
        }
      }
    }
    flush(true);
  }
}

namespace {

template <class KernelT>
void allow_lds(KernelT k, size_t bytes) {
  RELNN_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

// LDS ring depth NB: as many tiles as fit with their 2 NB - 1 index slots,
// at most 6 (tiles t+1 .. t+4 in flight while t is multiplied).
template <class T, int KP>
constexpr int ring_depth() {
  constexpr int TILE = DmaGeo<T, KP, 2>::TILE;
  constexpr int IRB = DmaGeo<T, KP, 2>::IRB;
  constexpr int fit = (160 * 1024 + IRB) / (TILE + 2 * IRB);
  return fit < 6 ? fit : 6;
}

template <class T, int KP, int NB, bool kMax, bool kWide, bool kArg>
void launch_dma(const WsArgs& a, size_t lds, hipStream_t s) {
  allow_lds(k_fwd_dma<T, KP, NB, kMax, kWide, kArg>, lds);
  KTimer tm("fwd_fused", s);
  const int64_t grid = a.nch == 1 ? a.nunits : round_up(a.nunits, 8) * a.nch;
  k_fwd_dma<T, KP, NB, kMax, kWide, kArg><<<(unsigned)grid, (a.hc / (kWide ? 32 : 16) + kDmaWaves) * 64, lds, s>>>(a);
  RELNN_LAUNCHED();
}

template <class T, int KP>
void run_dma(const WsArgs& a, hipStream_t s) {
  constexpr int NB = ring_depth<T, KP>();
  using G = DmaGeo<T, KP, NB>;
  static_assert(NB >= 2, "two LDS tiles at least");
  const size_t lds = (size_t)NB * G::TILE + (size_t)G::NIR * G::IRB;
  RELNN_REQUIRE(lds <= 160 * 1024, RELNN_E_HIP, "internal: LDS ring of %zu bytes", lds);
  if (a.sink.agg == RELNN_MAX) {
    if (a.sink.argmax)
      launch_dma<T, KP, NB, true, false, true>(a, lds, s);
    else                           // values only (the carry positions are written as 0)
      launch_dma<T, KP, NB, true, false, false>(a, lds, s);
  } else if (std::is_same<T, __bf16>::value && a.hc % 32 == 0) {
    launch_dma<T, KP, NB, false, std::is_same<T, __bf16>::value, false>(a, lds, s);
  } else {
    launch_dma<T, KP, NB, false, false, false>(a, lds, s);
  }
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


// Tile width: K rounded up to 64, 128, 256 or 384, and 512 for BF16 (an
// FP32 tile that wide leaves room for two LDS tiles only, no loads ahead).
int pick_kp(int K, bool bf) {
  for (int kp : {64, 128, 256, 384})
    if (K <= kp) return kp;
  return bf && K <= 512 ? 512 : 0;
}

// Output columns per block: all of h up to 128, else chunks of 128.
int pick_hc(int h) {
  if (h % 16 == 0 && h <= kHMax) return h;
  return h % kHMax == 0 ? kHMax : 0;
}

}  // namespace

int64_t resident_waves(const void* kernel, int threads) {
  static std::mutex mu;
  static std::vector<std::pair<const void*, int64_t>> cache;
  std::lock_guard<std::mutex> lock(mu);
  for (const auto& e : cache)
    if (e.first == kernel) return e.second;
  int blocks = 0;
  RELNN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, threads, 0));
  const int64_t w = (int64_t)std::max(blocks, 1) * num_cus() * (threads / 64);
  cache.emplace_back(kernel, w);
  return w;
}

template <int kMode>
auto push_sum_kernel(int n) {
  return n <= 1 ? k_push_sum<kMode, 1> : n == 2 ? k_push_sum<kMode, 2> : n == 3 ? k_push_sum<kMode, 3>
                                                                                : k_push_sum<kMode, 4>;
}

template <int kMode>
void launch_push_sum(int n, const WsArgs& a, const PushArgs& pa, hipStream_t s) {
  push_sum_kernel<kMode>(n)<<<(unsigned)cdiv(a.nunits, kPsWaves), kPsWaves * 64, 0, s>>>(a, pa);
}

void launch_push(const FwdArgs& f, int64_t nunits, int n, const float* const* P, const int32_t* const* rows,
                 float* carry, int32_t* carry_arg, int64_t G, float* V, hipStream_t s) {
  RELNN_REQUIRE(f.h % 4 == 0 && f.h <= kHMax, RELNN_E_UNSUPPORTED, "pushdown needs h %% 4 == 0 and h <= %d", kHMax);
  WsArgs a{};
  a.at = f.at;
  a.E = f.E;
  a.h = f.h;
  a.ntiles = cdiv(f.E, kPsTM);
  a.nunits = one_round_units(push_sum_kernel<PS_SUM>(n), kPsWaves * 64, std::min<int64_t>(a.ntiles, nunits));
  a.b = nullptr;                      // the bias is part of the group constant
  a.act_pre = RELNN_ACT_NONE;
  a.sg = f.sg;
  // the gather-sum and its fix-up write the aggregate of the varying atoms
  // into V (MEAN divided, maximisers to argmax); k_push_finish adds the
  // group constant and applies the rest of the sink
  Sink raw{};
  raw.agg = f.sink.agg;
  raw.act_post = RELNN_ACT_NONE;
  raw.out = V;
  raw.argmax = f.sink.argmax;
  a.sink = raw;
  a.carry = carry;
  a.carry_arg = carry_arg;
  PushArgs pa{};
  pa.n = n;
  for (int j = 0; j < n; ++j) {
    pa.P[j] = P[j];
    pa.rows[j] = rows[j];
  }
  KTimer tm("fwd_push", s);                // gather-sum, fix-up and finish
  launch_push_sum<PS_SUM>(n, a, pa, s);
  RELNN_LAUNCHED();
  launch_fixup(f.sg, kPsTM, f.h, a.ntiles, a.nunits, raw, carry, carry_arg, s);
  Sink fin = f.sink;
  fin.argmax = nullptr;
  fin.gc.offsets = f.sg.offsets;
  const int64_t n4 = G * (f.h / 4);
  if (n4 > 0) {
    k_push_finish<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n4, 256), 1 << 16)), 256, 0, s>>>(
        V, G, f.h, fin);
    RELNN_LAUNCHED();
  }
}

void launch_product(const FwdArgs& f, bool bf16, int64_t nunits, float* carry, int32_t* carry_arg, hipStream_t s) {
  RELNN_REQUIRE(f.h % 4 == 0, RELNN_E_UNSUPPORTED, "the product transform needs h %% 4 == 0");
  WsArgs a{};
  a.at = f.at;
  a.E = f.E;
  a.h = f.h;
  a.ntiles = cdiv(f.E, kPsTM);
  a.nunits = one_round_units(bf16 ? push_sum_kernel<PS_PROD_BF16>(f.at.k) : push_sum_kernel<PS_PROD_F32>(f.at.k),
                             kPsWaves * 64, std::min<int64_t>(a.ntiles, nunits));
  a.act_pre = f.act_pre;
  a.sg = f.sg;
  a.sink = f.sink;
  a.carry = carry;
  a.carry_arg = carry_arg;
  PushArgs pa{};
  pa.n = f.at.k;
  pa.act_pre = f.act_pre;
  for (int j = 0; j < f.at.k; ++j) {
    pa.P[j] = f.at.emb[j];
    pa.rows[j] = f.at.rows[j];
  }
  KTimer tm("fwd_product", s);
  if (bf16)
    launch_push_sum<PS_PROD_BF16>(f.at.k, a, pa, s);
  else
    launch_push_sum<PS_PROD_F32>(f.at.k, a, pa, s);
  RELNN_LAUNCHED();
  launch_fixup(f.sg, kPsTM, f.h, a.ntiles, a.nunits, f.sink, carry, carry_arg, s);
}

// ranges of the pushdown gather-sum (and carry pairs): up to 8192 waves
int64_t push_units(int64_t E) { return std::max<int64_t>(1, std::min<int64_t>(cdiv(E, kPsTM), 8192)); }

WsPlan plan_ws(int dtype, int K, int h, int64_t E) {
  WsPlan p;
  const bool bf = dtype == RELNN_BF16;
  p.KP = pick_kp(K, bf);
  p.hc = pick_hc(h);
  if (!p.KP || !p.hc) {
    p.KP = 0;
    return p;
  }
  p.nch = h / p.hc;
  p.TM = kTM;
  p.ntiles = cdiv(E, p.TM);
  // one block per CU: the column chunks of a range share the CUs
  p.nunits = std::max<int64_t>(1, std::min<int64_t>(p.ntiles, std::max(1, num_cus() / p.nch)));
  p.wsw_bytes = (size_t)p.KP * h * (bf ? 2 : 4) + kZeroBytes;
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
  a.hc = p.hc;
  a.nch = p.nch;
  a.ntiles = p.ntiles;
  a.nunits = p.nunits;
  a.Wsw = Wsw;
  a.zeros = static_cast<const char*>(Wsw) + (size_t)p.KP * f.h * (dtype == RELNN_BF16 ? 2 : 4);
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
      case 384: run_dma<__bf16, 384>(a, s); break;
      default: run_dma<__bf16, 512>(a, s); break;
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

// Explicit instantiations of the fused kernel: with implicit ones alone the
// host pass left the launch stubs of some instances undefined.
#define RELNN_DMA_INST(T, KP)                                                                    \
  template __global__ void k_fwd_dma<T, KP, ring_depth<T, KP>(), false, false, false>(WsArgs); \
  template __global__ void k_fwd_dma<T, KP, ring_depth<T, KP>(), true, false, true>(WsArgs);   \
  template __global__ void k_fwd_dma<T, KP, ring_depth<T, KP>(), true, false, false>(WsArgs);
RELNN_DMA_INST(float, 64)
RELNN_DMA_INST(float, 128)
RELNN_DMA_INST(float, 256)
RELNN_DMA_INST(float, 384)
RELNN_DMA_INST(__bf16, 64)
RELNN_DMA_INST(__bf16, 128)
RELNN_DMA_INST(__bf16, 256)
RELNN_DMA_INST(__bf16, 384)
RELNN_DMA_INST(__bf16, 512)
template __global__ void k_fwd_dma<__bf16, 64, ring_depth<__bf16, 64>(), false, true, false>(WsArgs);
template __global__ void k_fwd_dma<__bf16, 128, ring_depth<__bf16, 128>(), false, true, false>(WsArgs);
template __global__ void k_fwd_dma<__bf16, 256, ring_depth<__bf16, 256>(), false, true, false>(WsArgs);
template __global__ void k_fwd_dma<__bf16, 384, ring_depth<__bf16, 384>(), false, true, false>(WsArgs);
template __global__ void k_fwd_dma<__bf16, 512, ring_depth<__bf16, 512>(), false, true, false>(WsArgs);
#undef RELNN_DMA_INST

}  // namespace relnn
