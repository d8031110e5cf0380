// Tile machinery shared by the forward and backward layer kernels.
//
// A tile is TM consecutive tuples of a sorted tuple list.  The operand rows
// of a tile are staged in LDS (row-major, padded), multiplied on the matrix
// cores with a pre-swizzled weight in global memory (L2-resident), and the
// FP32 result tile is reduced per segment (runs of equal segment number)
// straight from LDS.  Segments that cross a tile edge leave one partial per
// tile in a carry buffer; a fix-up kernel combines those partials in tile
// order, so every result is deterministic and no float atomics are used.
#pragma once

#include "common.hpp"
#include "index.hpp"

namespace relnn {

constexpr int kThreads = 256;            // 4 waves
constexpr int kMaxQ = 16;                // 16x16 accumulator blocks per wave
constexpr int kMaxAtoms = RELNN_MAX_ATOMS;

template <class T>
struct Mfma;

// bf16: v_mfma_f32_16x16x32_bf16.  A lane holds 8 consecutive k of one row
// (row = lane % 16, k = 8 * (lane / 16) + i); B likewise for one column.
template <>
struct Mfma<__bf16> {
  static constexpr int KS = 32;        // k per instruction
  static constexpr int EPC = 8;        // elements per 16-byte chunk
  static constexpr int XPAD = 8;       // LDS row padding (elements)
};
// f32: v_mfma_f32_16x16x4_f32.  A lane holds A[lane % 16][lane / 16].
template <>
struct Mfma<float> {
  static constexpr int KS = 4;
  static constexpr int EPC = 4;
  static constexpr int XPAD = 4;
};

// Output of a 16x16 block: lane holds C[4 * (lane / 16) + i][lane % 16].

struct Seg {                 // segment structure of a sorted tuple list
  const int32_t* seg_of;     // [n] segment number of each list position
  const int32_t* offsets;    // [nseg+1]
  int64_t n;
  const int64_t* n_dev;      // if set: n is read from device memory at run time
};

__device__ __forceinline__ float act_apply(int act, float v) {
  return act == RELNN_ACT_RELU ? fmaxf(v, 0.0f) : v;
}

// Swizzled weight: fragment (ks, cb) occupies 64 lanes x one operand each.
template <class T>
__device__ __forceinline__ int64_t wsw_index(int ks, int cb, int ncb, int lane) {
  return ((int64_t)ks * ncb + cb) * 64 + lane;
}

// acc[qi] += Xs(rows of block rb) * Wsw(cols of block cb), all k.
// Xs: LDS [TM][XS] of T, Kp columns used.  Wave w owns blocks q = w + 4 qi.
template <class T>
__device__ __forceinline__ void mfma_tile(const T* __restrict__ Xs, int XS, int Kp, int nblk, int ncb,
                                          const T* __restrict__ Wsw, f32x4 (&acc)[kMaxQ]) {
  const int lane = __lane_id();
  const int w = threadIdx.x / 64;
#pragma unroll
  for (int qi = 0; qi < kMaxQ; ++qi) acc[qi] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int nks = Kp / Mfma<T>::KS;
  for (int ks = 0; ks < nks; ++ks) {
#pragma unroll
    for (int qi = 0; qi < kMaxQ; ++qi) {
      const int q = w + 4 * qi;
      if (q < nblk) {
        const int rb = q / ncb, cb = q - (q / ncb) * ncb;
        if constexpr (sizeof(T) == 2) {
          const bf16x8 a = *reinterpret_cast<const bf16x8*>(
              Xs + (rb * 16 + (lane & 15)) * XS + ks * 32 + (lane >> 4) * 8);
          const bf16x8 b = reinterpret_cast<const bf16x8*>(Wsw)[wsw_index<T>(ks, cb, ncb, lane)];
          acc[qi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[qi], 0, 0, 0);
        } else {
          const float a = Xs[(rb * 16 + (lane & 15)) * XS + ks * 4 + (lane >> 4)];
          const float b = Wsw[wsw_index<T>(ks, cb, ncb, lane)];
          acc[qi] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[qi], 0, 0, 0);
        }
      }
    }
  }
}

// Adds the bias, applies act, and stores the accumulators into Ys [TM][YS].
__device__ __forceinline__ void store_acc(const f32x4 (&acc)[kMaxQ], int nblk, int ncb,
                                          const float* __restrict__ bias, int act, float* Ys,
                                          int YS) {
  const int lane = __lane_id();
  const int w = threadIdx.x / 64;
#pragma unroll
  for (int qi = 0; qi < kMaxQ; ++qi) {
    const int q = w + 4 * qi;
    if (q < nblk) {
      const int rb = q / ncb, cb = q - (q / ncb) * ncb;
      const int col = cb * 16 + (lane & 15);
      const float bv = bias ? bias[col] : 0.0f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rb * 16 + (lane >> 4) * 4 + i;
        Ys[row * YS + col] = act_apply(act, acc[qi][i] + bv);
      }
    }
  }
}

// Per-group constant of the pushed-down transform: sum over the atoms
// whose key is a function of the group of P_j[row of the group] (+ bias).
struct GroupConst {
  int n;                          // such atoms (0: none)
  const float* P[RELNN_MAX_ATOMS];      // [n_rows_j][h] node products
  const int32_t* rows[RELNN_MAX_ATOMS]; // joined rows of the atom per tuple
  const int32_t* offsets;         // group offsets (any tuple names the row)
  const float* bias;              // [h] or null
};

// How a finished segment value is written.
struct Sink {
  int agg;          // relnn_agg
  int act_post;
  float* out;       // [nseg][h]
  float* pre;       // [nseg][h] or null
  int32_t* argmax;  // [nseg][h] or null
  bool accumulate;  // out += value (backward scatter into embeddings)
  const int32_t* out_row;   // optional remap: segment -> output row
  bool out_bf16;    // out holds bf16 (round to nearest even)
  GroupConst gc;    // pushed-down transform: per-group constant term
};

__device__ __forceinline__ float group_const(const GroupConst& g, int64_t s, int c, int h) {
  float v = g.bias ? g.bias[c] : 0.0f;
  if (g.n) {
    const int64_t e = g.offsets[s];
#pragma unroll
    for (int j = 0; j < RELNN_MAX_ATOMS; ++j)    // constant trip count: no run-time index into the argument
      if (j < g.n) v += g.P[j][(int64_t)g.rows[j][e] * h + c];
  }
  return v;
}

// kStoreOnly: the sink has no group constant, no row remap and no
// accumulation, so writing issues no global load (a kernel that keeps
// gathers in flight must not wait on them to write a result).
template <bool kStoreOnly = false>
__device__ __forceinline__ void sink_write(const Sink& k, int64_t s, int c, int h, float v, int32_t am,
                                           int32_t cnt) {
  if (k.agg == RELNN_MEAN) v = v / (float)cnt;
  if (!kStoreOnly && (k.gc.n || k.gc.bias)) {   // pushed-down transform: add the group's constant term
    const float g = group_const(k.gc, s, c, h);
    v = (k.agg == RELNN_SUM) ? v + (float)cnt * g : v + g;
  }
  const int64_t row = (!kStoreOnly && k.out_row) ? (int64_t)k.out_row[s] : s;
  const int64_t o = row * h + c;
  if (k.pre) k.pre[o] = v;
  if (k.argmax && k.agg == RELNN_MAX) k.argmax[o] = am;
  if (!kStoreOnly && k.accumulate)
    k.out[o] += v;
  else if (k.out_bf16)
    reinterpret_cast<__bf16*>(k.out)[o] = (__bf16)act_apply(k.act_post, v);
  else
    k.out[o] = act_apply(k.act_post, v);
}

// Columns c4 .. c4 + 3 of a finished SUM / MEAN group, for kernels whose
// sink has no group constant, no row remap and no accumulation (c4 and h
// multiples of 4).  MEAN scales by the reciprocal of the count.
__device__ __forceinline__ void sink_write4(const Sink& k, int64_t s, int c4, int h, f32x4 v, int32_t cnt) {
  if (k.agg == RELNN_MEAN) v *= __builtin_amdgcn_rcpf((float)cnt);
  const int64_t o = s * h + c4;
  if (k.pre) *reinterpret_cast<f32x4*>(k.pre + o) = v;
  f32x4 w;
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = act_apply(k.act_post, v[i]);
  if (k.out_bf16) {
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    bf16x4 b;
#pragma unroll
    for (int i = 0; i < 4; ++i) b[i] = (__bf16)w[i];
    *reinterpret_cast<bf16x4*>(reinterpret_cast<__bf16*>(k.out) + o) = b;
  } else {
    *reinterpret_cast<f32x4*>(k.out + o) = w;
  }
}

// Reduces the rows [0, nv) of the LDS tile Ys (list positions e0..) per
// segment.  Segments wholly inside the tile are finished and written; a
// segment cut by the tile start leaves its partial in carry slot 0, one
// that starts in the tile and runs past its end in slot 1.
__device__ inline void reduce_tile(const float* Ys, int YS, int h, int64_t e0, int nv, int64_t tile,
                            const Seg& sg, const Sink& sink, float* carry, int32_t* carry_arg) {
  const int64_t s_first = sg.seg_of[e0];
  const int64_t s_last = sg.seg_of[e0 + nv - 1];
  const int64_t ns = s_last - s_first + 1;
  const int64_t work = ns * h;
  for (int64_t p = threadIdx.x; p < work; p += blockDim.x) {
    const int64_t s = s_first + p / h;
    const int c = (int)(p - (p / h) * h);
    const int64_t g0 = sg.offsets[s], g1 = sg.offsets[s + 1];
    const int r0 = (int)(max(g0, e0) - e0);
    const int r1 = (int)(min(g1, e0 + nv) - e0);
    float v;
    int32_t am = -1;
    if (sink.agg == RELNN_MAX) {
      v = Ys[r0 * YS + c];
      am = (int32_t)(e0 + r0);
      for (int r = r0 + 1; r < r1; ++r) {
        const float y = Ys[r * YS + c];
        if (y > v) {
          v = y;
          am = (int32_t)(e0 + r);
        }
      }
    } else {
      v = 0.0f;
      for (int r = r0; r < r1; ++r) v += Ys[r * YS + c];
    }
    if (g0 >= e0 && g1 <= e0 + nv) {
      sink_write(sink, s, c, h, v, am, (int32_t)(g1 - g0));
    } else {
      const int slot = (g0 < e0) ? 0 : 1;      // cut by the tile start : by its end
      carry[(tile * 2 + slot) * h + c] = v;
      if (carry_arg) carry_arg[(tile * 2 + slot) * h + c] = am;
    }
  }
}

}  // namespace relnn
