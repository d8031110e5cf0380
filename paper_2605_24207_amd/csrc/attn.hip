// Segmented softmax attention over the joined tuples of an index whose body
// atoms are (Q, K, V): the paper's attention as rules (Section 1's Score
// rule q*k and Attention rule sum(a*v), Section 5.2's HGT head with a
// softmax over each target's tuples).
//
// Forward: one wave per contiguous range of tuples in canonical order.  A
// lane holds two columns of the q, k and v rows; the score of a head is the
// butterfly sum of the q*k products over the head's lanes, times the scale.
// Each lane keeps the running maximum, the running sum of exponentials and
// its two output columns of its head (the online form of max-subtract-exp-
// sum), rescaling both when the maximum grows.  A group that ends inside
// the range is finished there (out = acc / l, lse = m + log l); a group cut
// by a range edge leaves its state (m, l, acc) in a carry slot, and a
// fix-up merges the states of a group in range order, so results are
// deterministic and no float atomics are used.
//
// Backward: per tuple the softmax weight a = exp(s - lse) and the score
// gradient ds = a (dp - D), dp = <dout_h, v_h>, D = <dout_h, out_h>, are
// written out; then each of dQ, dK and dV is a weighted gather-sum in the
// transpose order of its atom (rows of K weighted by scale ds into dQ, rows
// of Q by scale ds into dK, rows of dout by a into dV), added into the
// embedding gradients.
#include "index.hpp"
#include "layer_fwd.hpp"

namespace relnn {
namespace {

constexpr int kAtTM = 64;       // range boundaries on multiples of 64 tuples
constexpr int kAtWaves = 4;
constexpr int kAtBatch = 8;     // tuples whose rows are loaded together

struct AttnArgs {
  const void* q;
  const void* k;
  const void* v;
  const int32_t* rq;
  const int32_t* rk;
  const int32_t* rv;
  int bf16;
  int d, dv, heads, hd, hdv;
  float scale;
  int64_t E;
  Seg sg;
  float* out;             // [G][dv]
  float* lse;             // [G][heads] or null
  float* carry;           // [nunits][2][dv + 2 heads]: acc, m, l
  int64_t ntiles, nunits;
};

template <bool kBF16>
__device__ __forceinline__ float2 ld2(const void* base, int64_t row, int ld, int col) {
  if constexpr (kBF16) {
    const uint32_t u = *reinterpret_cast<const uint32_t*>(static_cast<const __bf16*>(base) + row * ld + col);
    return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
  } else {
    return *reinterpret_cast<const float2*>(static_cast<const float*>(base) + row * ld + col);
  }
}

template <bool kBF16>
__global__ void __launch_bounds__(kAtWaves * 64) k_attn_fwd(AttnArgs a) {
  const int lane = threadIdx.x % 64;
  const int64_t u = (int64_t)blockIdx.x * kAtWaves + threadIdx.x / 64;
  if (u >= a.nunits) return;
  const int64_t r0 = ((a.ntiles * u) / a.nunits) * kAtTM;
  const int64_t r1 = min<int64_t>(((a.ntiles * (u + 1)) / a.nunits) * kAtTM, a.E);
  if (r0 >= r1) return;
  const int cq = 2 * lane, cv = 2 * lane;
  const bool on_q = cq < a.d, on_v = cv < a.dv;
  const int cqc = on_q ? cq : 0, cvc = on_v ? cv : 0;
  const int hq_lanes = a.hd / 2;                          // lanes of one head in the q / k layout
  const int hv = cvc / a.hdv;                             // head of this lane's value columns
  const int src_lane = hv * hq_lanes;                     // a lane holding that head's score
  const bool head_lead = on_v && cv % a.hdv == 0;         // writes the head's m, l, lse
  const int slot = a.dv + 2 * a.heads;

  float m = -INFINITY, l = 0.0f, acc0 = 0.0f, acc1 = 0.0f;
  int32_t g = a.sg.seg_of[r0];
  const bool lo_cont = r0 > 0 && a.sg.seg_of[r0 - 1] == g;
  bool first = true;
  auto flush = [&](bool last_seg) {
    const bool cut_lo = first && lo_cont;
    const bool cut_hi = last_seg && r1 < a.E && a.sg.seg_of[r1] == g;
    if (cut_lo || cut_hi) {
      float* c = a.carry + (u * 2 + (cut_lo ? 0 : 1)) * slot;
      if (on_v) {
        c[cv] = acc0;
        c[cv + 1] = acc1;
      }
      if (head_lead) {
        c[a.dv + hv] = m;
        c[a.dv + a.heads + hv] = l;
      }
    } else {
      const float inv = 1.0f / l;
      if (on_v) *reinterpret_cast<float2*>(a.out + (int64_t)g * a.dv + cv) = make_float2(acc0 * inv, acc1 * inv);
      if (head_lead && a.lse) a.lse[(int64_t)g * a.heads + hv] = m + logf(l);
    }
    first = false;
    m = -INFINITY;
    l = 0.0f;
    acc0 = acc1 = 0.0f;
  };
  for (int64_t base = r0; base < r1; base += 64) {
    const int n = (int)min<int64_t>(64, r1 - base);
    const int64_t e = base + min(lane, n - 1);
    const int32_t gl = a.sg.seg_of[e];
    const int32_t Rq = a.rq[e], Rk = a.rk[e], Rv = a.rv[e];
    for (int bt = 0; bt < n; bt += kAtBatch) {
      float2 qv[kAtBatch], kv[kAtBatch], vv[kAtBatch];
#pragma unroll
      for (int i = 0; i < kAtBatch; ++i) {
        const int q = min(bt + i, n - 1);                 // clamped: every load is valid
        qv[i] = ld2<kBF16>(a.q, __builtin_amdgcn_readlane(Rq, q), a.d, cqc);
        kv[i] = ld2<kBF16>(a.k, __builtin_amdgcn_readlane(Rk, q), a.d, cqc);
        vv[i] = ld2<kBF16>(a.v, __builtin_amdgcn_readlane(Rv, q), a.dv, cvc);
      }
#pragma unroll
      for (int i = 0; i < kAtBatch; ++i) {
        const int q = bt + i;
        if (q >= n) break;
        const int32_t gq = __builtin_amdgcn_readlane(gl, q);
        if (gq != g) {                                    // a group ends
          flush(false);
          g = gq;
        }
        float p = on_q ? qv[i].x * kv[i].x + qv[i].y * kv[i].y : 0.0f;
        for (int off = 1; off < hq_lanes; off <<= 1) p += __shfl_xor(p, off);
        const float sc = a.scale * __shfl(p, src_lane);  // this lane's value head
        const float mn = fmaxf(m, sc);
        const float fa = expf(m - mn), fb = expf(sc - mn);
        l = l * fa + fb;
        acc0 = acc0 * fa + fb * vv[i].x;
        acc1 = acc1 * fa + fb * vv[i].y;
        m = mn;
      }
    }
  }
  flush(true);
}

// Merges the carried states of a group cut by range edges, in range order
// (block b handles the group running across the start of range b, as the
// layer's fix-up does), then writes out and lse.
__global__ void k_attn_fixup(AttnArgs a) {
  const int64_t b = (int64_t)blockIdx.x + 1;
  auto pos = [&](int64_t uu) { return ((a.ntiles * uu) / a.nunits) * kAtTM; };
  const int64_t e = pos(b);
  if (e <= 0 || e >= a.E) return;
  const int64_t s = a.sg.seg_of[e];
  if (a.sg.seg_of[e - 1] != s) return;
  const int64_t g0 = a.sg.offsets[s], g1 = a.sg.offsets[s + 1];
  if (g0 < pos(b - 1)) return;
  int64_t lo = b, hi = a.nunits - 1;                      // last range holding part of s
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (pos(mid) < g1) lo = mid; else hi = mid - 1;
  }
  const int64_t P = lo - (b - 1) + 1;                     // range b-1 (slot 1), ranges b..lo (slot 0)
  const int slot = a.dv + 2 * a.heads;
  auto at = [&](int64_t i) { return a.carry + ((b - 1 + i) * 2 + (i == 0 ? 1 : 0)) * slot; };
  for (int c = threadIdx.x; c < a.dv; c += blockDim.x) {
    const int h = c / a.hdv;
    float m = -INFINITY, l = 0.0f, acc = 0.0f;
    // a hot group spans many ranges: the partials are loaded eight at a
    // time, then merged in range order
    constexpr int kFB = 8;
    for (int64_t i0 = 0; i0 < P; i0 += kFB) {
      float m2[kFB], l2[kFB], a2[kFB];
#pragma unroll
      for (int j = 0; j < kFB; ++j) {
        const float* st = at(min<int64_t>(i0 + j, P - 1));   // clamped: every load is valid
        m2[j] = st[a.dv + h];
        l2[j] = st[a.dv + a.heads + h];
        a2[j] = st[c];
      }
#pragma unroll
      for (int j = 0; j < kFB; ++j) {
        if (i0 + j >= P) break;
        const float mn = fmaxf(m, m2[j]);
        if (mn == -INFINITY) continue;                    // nothing seen yet on either side
        const float fa = expf(m - mn), fb = expf(m2[j] - mn);
        l = l * fa + l2[j] * fb;
        acc = acc * fa + a2[j] * fb;
        m = mn;
      }
    }
    a.out[s * a.dv + c] = acc / l;
    if (a.lse && c % a.hdv == 0) a.lse[s * a.heads + h] = m + logf(l);
  }
}

// ---------------------------------------------------------------- backward
// D[g][h] = <dout_g,h, out_g,h>
__global__ void k_attn_delta(const float* dout, const float* out, int64_t G, int dv, int heads, float* D) {
  const int hdv = dv / heads;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < G * heads;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = i / heads;
    const int h = (int)(i - g * heads);
    float s = 0.0f;
    for (int c = h * hdv; c < (h + 1) * hdv; ++c) s += dout[g * dv + c] * out[g * dv + c];
    D[i] = s;
  }
}

// Per tuple and head: A = exp(s - lse) and DS = scale A (dp - D), dp =
// <dout_g,h, v_h>.  Lanes over columns, as the forward; a wave takes 64
// consecutive tuples, reads their row numbers as one vector each, and
// loads the rows of kTupB tuples before using any of them, so that the
// random K and V rows of several tuples are in flight at once (one tuple
// at a time left the kernel waiting on one row fetch after another).
constexpr int kTupB = 4;
template <bool kBF16>
__global__ void __launch_bounds__(256) k_attn_tuple(AttnArgs a, const int32_t* tuple_group, const float* dout,
                                                    const float* lse, const float* D, float* A, float* DS) {
  const int lane = threadIdx.x % 64;
  const int cq = 2 * lane, cv = 2 * lane;
  const bool on_q = cq < a.d, on_v = cv < a.dv;
  const int cqc = on_q ? cq : 0, cvc = on_v ? cv : 0;
  const int hq_lanes = a.hd / 2, hv_lanes = a.hdv / 2;
  const int h = on_v ? cv / a.hdv : 0;                 // the head this lane's columns belong to
  const int64_t stride = (int64_t)gridDim.x * 4 * 64;
  for (int64_t base = ((int64_t)blockIdx.x * 4 + threadIdx.x / 64) * 64; base < a.E; base += stride) {
    const int n = (int)min<int64_t>(64, a.E - base);
    const int64_t e = base + min(lane, n - 1);
    const int32_t Rq = a.rq[e], Rk = a.rk[e], Rv = a.rv[e], Rg = tuple_group[e];
    for (int bt = 0; bt < n; bt += kTupB) {
      // every load of the batch first (the group's lse and D included),
      // so that the arithmetic waits once for all of them
      float2 qv[kTupB], kv[kTupB], vv[kTupB], dv[kTupB];
      float lw[kTupB], dw[kTupB];
#pragma unroll
      for (int i = 0; i < kTupB; ++i) {               // clamped: every load is valid
        const int q = min(bt + i, n - 1);
        const int64_t gi = __builtin_amdgcn_readlane(Rg, q);
        qv[i] = ld2<kBF16>(a.q, __builtin_amdgcn_readlane(Rq, q), a.d, cqc);
        kv[i] = ld2<kBF16>(a.k, __builtin_amdgcn_readlane(Rk, q), a.d, cqc);
        vv[i] = ld2<kBF16>(a.v, __builtin_amdgcn_readlane(Rv, q), a.dv, cvc);
        dv[i] = *reinterpret_cast<const float2*>(dout + gi * a.dv + cvc);
        lw[i] = lse[gi * a.heads + h];
        dw[i] = D[gi * a.heads + h];
      }
#pragma unroll
      for (int i = 0; i < kTupB; ++i) {
        if (bt + i >= n) break;
        const int64_t t = base + bt + i;
        float p = on_q ? qv[i].x * kv[i].x + qv[i].y * kv[i].y : 0.0f;
        for (int off = 1; off < hq_lanes; off <<= 1) p += __shfl_xor(p, off);
        float dp = on_v ? dv[i].x * vv[i].x + dv[i].y * vv[i].y : 0.0f;
        for (int off = 1; off < hv_lanes; off <<= 1) dp += __shfl_xor(dp, off);
        // lane h * hv_lanes writes head h; its score sits on lane h * hq_lanes
        const float sc = a.scale * __shfl(p, h * hq_lanes);
        if (on_v && cv % a.hdv == 0) {
          const float w = expf(sc - lw[i]);
          A[t * a.heads + h] = w;
          DS[t * a.heads + h] = a.scale * w * (dp - dw[i]);
        }
      }
    }
  }
}

// When Q's key is the group column (one Q row per group, distinct across
// groups, as in the HGT head), the weights pass also forms dQ: dQ_g = sum
// over the group's tuples of DS_tau,h k_tau (the columns of head h), in
// canonical order with Kahan compensation, added into the group's Q row
// once; groups cut by range edges leave partials for the fix-up.  This
// saves the gather-sum over Q's rows, which read every K row a second
// time.  One wave per contiguous tuple range, as the forward.
// compensated add; the compensation is dropped once the sum is not finite
__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
  const float y = x - c;
  const float t = s + y;
  c = __builtin_isfinite(t) ? (t - s) - y : 0.0f;
  s = t;
}

template <bool kBF16>
__global__ void __launch_bounds__(kAtWaves * 64) k_attn_tuple_q(AttnArgs a, const float* dout, const float* lse,
                                                               const float* D, float* A, float* DS,
                                                               const int32_t* qrow, float* dq, float* carry) {
  const int lane = threadIdx.x % 64;
  const int64_t u = (int64_t)blockIdx.x * kAtWaves + threadIdx.x / 64;
  if (u >= a.nunits) return;
  const int64_t r0 = ((a.ntiles * u) / a.nunits) * kAtTM;
  const int64_t r1 = min<int64_t>(((a.ntiles * (u + 1)) / a.nunits) * kAtTM, a.E);
  if (r0 >= r1) return;
  const int cq = 2 * lane, cv = 2 * lane;
  const bool on_q = cq < a.d, on_v = cv < a.dv;
  const int cqc = on_q ? cq : 0, cvc = on_v ? cv : 0;
  const int hq_lanes = a.hd / 2, hv_lanes = a.hdv / 2;
  const int h = on_v ? cv / a.hdv : 0;                    // head of this lane's value columns
  const int hq = cqc / a.hd;                              // head of this lane's q / k columns
  const bool head_lead = on_v && cv % a.hdv == 0;

  float s0 = 0.f, s1 = 0.f, c0 = 0.f, c1 = 0.f;           // dQ of the open group, this lane's columns
  int32_t g = a.sg.seg_of[r0];
  const bool lo_cont = r0 > 0 && a.sg.seg_of[r0 - 1] == g;
  bool first = true;
  // the open group's Q row and that row's dQ so far, fetched when the group
  // opens (each row is written by one wave only), so that closing it waits
  // for neither
  int32_t grow = qrow[g];
  float2 gold = on_q ? *reinterpret_cast<const float2*>(dq + (int64_t)grow * a.d + cq) : make_float2(0.f, 0.f);
  auto flush = [&](bool last_seg) {
    const bool cut_lo = first && lo_cont;
    const bool cut_hi = last_seg && r1 < a.E && a.sg.seg_of[r1] == g;
    if (on_q) {
      const float v0 = s0 - c0, v1 = s1 - c1;
      if (cut_lo || cut_hi) {
        *reinterpret_cast<float2*>(carry + (u * 2 + (cut_lo ? 0 : 1)) * a.d + cq) = make_float2(v0, v1);
      } else {                                            // the group's row is written by this wave alone
        *reinterpret_cast<float2*>(dq + (int64_t)grow * a.d + cq) = make_float2(gold.x + v0, gold.y + v1);
      }
    }
    first = false;
    s0 = s1 = c0 = c1 = 0.f;
  };
  for (int64_t base = r0; base < r1; base += 64) {
    const int n = (int)min<int64_t>(64, r1 - base);
    const int64_t e = base + min(lane, n - 1);
    const int32_t gl = a.sg.seg_of[e];
    const int32_t Rq = a.rq[e], Rk = a.rk[e], Rv = a.rv[e];
    const int32_t QR = qrow[gl];                          // Q row of each position's group
    for (int bt = 0; bt < n; bt += kTupB) {
      // every load of the batch first (the group's lse and D included),
      // so that the arithmetic waits once for all of them
      float2 qv[kTupB], kv[kTupB], vv[kTupB], dv[kTupB];
      float lw[kTupB], dw[kTupB];
#pragma unroll
      for (int i = 0; i < kTupB; ++i) {                  // clamped: every load is valid
        const int q = min(bt + i, n - 1);
        const int64_t gi = __builtin_amdgcn_readlane(gl, q);
        qv[i] = ld2<kBF16>(a.q, __builtin_amdgcn_readlane(Rq, q), a.d, cqc);
        kv[i] = ld2<kBF16>(a.k, __builtin_amdgcn_readlane(Rk, q), a.d, cqc);
        vv[i] = ld2<kBF16>(a.v, __builtin_amdgcn_readlane(Rv, q), a.dv, cvc);
        dv[i] = *reinterpret_cast<const float2*>(dout + gi * a.dv + cvc);
        lw[i] = lse[gi * a.heads + h];
        dw[i] = D[gi * a.heads + h];
      }
#pragma unroll
      for (int i = 0; i < kTupB; ++i) {
        const int q = bt + i;
        if (q >= n) break;
        const int32_t gq = __builtin_amdgcn_readlane(gl, q);
        if (gq != g) {                                    // a group ends
          flush(false);
          g = gq;
          grow = __builtin_amdgcn_readlane(QR, q);
          if (on_q) gold = *reinterpret_cast<const float2*>(dq + (int64_t)grow * a.d + cq);
        }
        const int64_t t = base + q;
        float p = on_q ? qv[i].x * kv[i].x + qv[i].y * kv[i].y : 0.0f;
        for (int off = 1; off < hq_lanes; off <<= 1) p += __shfl_xor(p, off);
        float dp = on_v ? dv[i].x * vv[i].x + dv[i].y * vv[i].y : 0.0f;
        for (int off = 1; off < hv_lanes; off <<= 1) dp += __shfl_xor(dp, off);
        const float sc = a.scale * __shfl(p, h * hq_lanes);
        const float w = expf(sc - lw[i]);
        const float ds = a.scale * w * (dp - dw[i]);
        if (head_lead) {
          A[t * a.heads + h] = w;
          DS[t * a.heads + h] = ds;
        }
        const float dsq = __shfl(ds, hq * hv_lanes);     // DS of the head of this lane's k columns
        kahan_add(s0, c0, dsq * kv[i].x);
        kahan_add(s1, c1, dsq * kv[i].y);
      }
    }
  }
  flush(true);
}

// qrow[g] = row of atom 0 joined to the first tuple of group g
__global__ void k_group_rows(const int32_t* offsets, const int32_t* rq, int64_t G, int32_t* qrow) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G; g += (int64_t)gridDim.x * blockDim.x)
    qrow[g] = rq[offsets[g]];
}

// out[i] = y[ord[i]]
__global__ void k_gather_rows_idx(const int32_t* ord, const int32_t* y, int64_t n, int32_t* out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = y[ord[i]];
}

unsigned grid_n(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 1 << 16)); }

int64_t attn_units(int64_t E) { return std::max<int64_t>(1, std::min<int64_t>(cdiv(std::max<int64_t>(E, 1), kAtTM), 8192)); }

void check_attn(const relnn_index* idx, const relnn_attn_desc* A) {
  RELNN_REQUIRE(idx != nullptr && A != nullptr, RELNN_E_INVALID, "index or descriptor is NULL");
  RELNN_REQUIRE(idx->k == 3, RELNN_E_INVALID, "attention needs an index with three atoms (Q, K, V), not %d", idx->k);
  RELNN_REQUIRE(A->dtype == RELNN_F32 || A->dtype == RELNN_BF16, RELNN_E_INVALID, "unknown dtype");
  RELNN_REQUIRE(A->heads >= 1 && A->d > 0 && A->dv > 0 && A->d % A->heads == 0 && A->dv % A->heads == 0,
                RELNN_E_INVALID, "d and dv must be multiples of heads");
  const int hd = A->d / A->heads, hdv = A->dv / A->heads;
  auto pow2 = [](int x) { return x > 0 && (x & (x - 1)) == 0; };
  RELNN_REQUIRE(A->d <= 128 && A->dv <= 128 && A->d % 4 == 0 && A->dv % 4 == 0 && pow2(hd) && pow2(hdv) &&
                    hd >= 2 && hdv >= 2,
                RELNN_E_UNSUPPORTED, "attention needs d, dv <= 128, multiples of 4, with power-of-two head widths");
}

AttnArgs make_args(const relnn_index* idx, const relnn_attn_desc* A, const void* q, const void* k, const void* v) {
  AttnArgs a{};
  a.q = q;
  a.k = k;
  a.v = v;
  a.rq = idx->rows;
  a.rk = idx->rows + idx->E;
  a.rv = idx->rows + 2 * idx->E;
  a.bf16 = A->dtype == RELNN_BF16;
  a.d = A->d;
  a.dv = A->dv;
  a.heads = A->heads;
  a.hd = A->d / A->heads;
  a.hdv = A->dv / A->heads;
  a.scale = A->scale;
  a.E = idx->E;
  a.sg = Seg{idx->tuple_group, idx->offsets, idx->E, nullptr};
  a.ntiles = cdiv(std::max<int64_t>(idx->E, 1), kAtTM);
  a.nunits = attn_units(idx->E);
  return a;
}

struct AttnPlan {
  size_t carry = 0, lse = 0, D = 0, A = 0, DS = 0, yrow = 0, gcarry = 0, qrow = 0, qcarry = 0, total = 0;
};

AttnPlan plan_attn(const relnn_index* idx, const relnn_attn_desc* A, bool bwd) {
  AttnPlan p;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += round_up(std::max<size_t>(bytes, 1), 256);
    return o;
  };
  const int64_t E = std::max<int64_t>(idx->E, 1), G = std::max<int64_t>(idx->G, 1);
  p.carry = take((size_t)attn_units(idx->E) * 2 * (A->dv + 2 * A->heads) * 4);
  if (bwd) {
    const int w = std::max(A->d, A->dv);
    p.lse = take((size_t)G * A->heads * 4);
    p.D = take((size_t)G * A->heads * 4);
    p.A = take((size_t)E * A->heads * 4);
    p.DS = take((size_t)E * A->heads * 4);
    p.yrow = take((size_t)E * 4);
    p.gcarry = take((size_t)gs_units(E) * 2 * w * 4);
    p.qrow = take((size_t)G * 4);
    p.qcarry = take((size_t)attn_units(idx->E) * 2 * A->d * 4);
  }
  p.total = off;
  return p;
}

template <class K>
void launch_fwd_k(K kern, const AttnArgs& a, hipStream_t s) {
  kern<<<(unsigned)cdiv(a.nunits, kAtWaves), kAtWaves * 64, 0, s>>>(a);
  RELNN_LAUNCHED();
}

void run_attn_fwd(const AttnArgs& args, hipStream_t s) {
  KTimer tm("attn_fwd", s);
  AttnArgs a = args;
  a.nunits = one_round_units(a.bf16 ? k_attn_fwd<true> : k_attn_fwd<false>, kAtWaves * 64, a.nunits);
  if (a.bf16)
    launch_fwd_k(k_attn_fwd<true>, a, s);
  else
    launch_fwd_k(k_attn_fwd<false>, a, s);
  if (a.nunits > 1) {
    k_attn_fixup<<<(unsigned)(a.nunits - 1), 256, 0, s>>>(a);
    RELNN_LAUNCHED();
  }
}

}  // namespace
}  // namespace relnn

using namespace relnn;

extern "C" relnn_status relnn_attn_workspace_size(const relnn_index* idx, const relnn_attn_desc* A, int bwd,
                                                  size_t* bytes) {
  return guard([&] {
    RELNN_REQUIRE(bytes != nullptr, RELNN_E_INVALID, "bytes is NULL");
    check_attn(idx, A);
    *bytes = plan_attn(idx, A, bwd != 0).total;
  });
}

extern "C" relnn_status relnn_attn_fwd(const relnn_index* idx, const relnn_attn_desc* A, const void* q,
                                       const void* k, const void* v, float* out, float* lse, void* ws,
                                       size_t ws_bytes, relnn_stream_t stream) {
  return guard([&] {
    check_attn(idx, A);
    RELNN_REQUIRE(idx->E == 0 || (q && k && v && out), RELNN_E_INVALID, "q, k, v and out are required");
    const AttnPlan P = plan_attn(idx, A, false);
    RELNN_REQUIRE(ws != nullptr && ws_bytes >= P.total, RELNN_E_INVALID, "workspace of %zu bytes given, %zu needed",
                  ws_bytes, P.total);
    if (idx->E == 0) return;
    hipStream_t s = (hipStream_t)stream;
    AttnArgs a = make_args(idx, A, q, k, v);
    a.out = out;
    a.lse = lse;
    a.carry = reinterpret_cast<float*>(static_cast<char*>(ws) + P.carry);
    run_attn_fwd(a, s);
  });
}

extern "C" relnn_status relnn_attn_bwd(const relnn_index* idx, const relnn_attn_desc* A, const void* q,
                                       const void* k, const void* v, const float* out, const float* lse,
                                       const float* dout, float* dq, float* dk, float* dv, void* ws,
                                       size_t ws_bytes, relnn_stream_t stream) {
  return guard([&] {
    check_attn(idx, A);
    RELNN_REQUIRE(idx->has_bwd, RELNN_E_INVALID, "the index was built without RELNN_IDX_BWD");
    RELNN_REQUIRE(idx->E == 0 || (q && k && v && out && lse && dout && dq && dk && dv), RELNN_E_INVALID,
                  "q, k, v, out, lse, dout, dq, dk and dv are required");
    const AttnPlan P = plan_attn(idx, A, true);
    RELNN_REQUIRE(ws != nullptr && ws_bytes >= P.total, RELNN_E_INVALID, "workspace of %zu bytes given, %zu needed",
                  ws_bytes, P.total);
    if (idx->E == 0) return;
    hipStream_t s = (hipStream_t)stream;
    char* w = static_cast<char*>(ws);
    const int64_t E = idx->E, G = idx->G;
    AttnArgs a = make_args(idx, A, q, k, v);
    float* D = reinterpret_cast<float*>(w + P.D);
    float* Aw = reinterpret_cast<float*>(w + P.A);
    float* DS = reinterpret_cast<float*>(w + P.DS);
    KTimer tm("attn_bwd", s);
    k_attn_delta<<<grid_n(G * A->heads), 256, 0, s>>>(dout, out, G, A->dv, A->heads, D);
    RELNN_LAUNCHED();
    // Q keyed by the group column: dQ is formed by the weights pass
    const bool q_fused = idx->atom_gk[0];
    if (q_fused) {
      int32_t* qrow = reinterpret_cast<int32_t*>(w + P.qrow);
      float* qcarry = reinterpret_cast<float*>(w + P.qcarry);
      k_group_rows<<<grid_n(G), 256, 0, s>>>(idx->offsets, a.rq, G, qrow);
      RELNN_LAUNCHED();
      a.ntiles = cdiv(E, kAtTM);
      a.nunits = one_round_units(a.bf16 ? k_attn_tuple_q<true> : k_attn_tuple_q<false>, kAtWaves * 64,
                                 attn_units(E));
      const unsigned gu = (unsigned)cdiv(a.nunits, kAtWaves);
      if (a.bf16)
        k_attn_tuple_q<true><<<gu, kAtWaves * 64, 0, s>>>(a, dout, lse, D, Aw, DS, qrow, dq, qcarry);
      else
        k_attn_tuple_q<false><<<gu, kAtWaves * 64, 0, s>>>(a, dout, lse, D, Aw, DS, qrow, dq, qcarry);
      RELNN_LAUNCHED();
      Sink sk{};
      sk.agg = RELNN_SUM;
      sk.act_post = RELNN_ACT_NONE;
      sk.out = dq;
      sk.out_row = qrow;
      sk.accumulate = true;
      launch_fixup(a.sg, kAtTM, A->d, a.ntiles, a.nunits, sk, qcarry, nullptr, s);
    } else {
      const unsigned gt = (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(E, 4 * 64), 1 << 16));
      if (a.bf16)
        k_attn_tuple<true><<<gt, 256, 0, s>>>(a, idx->tuple_group, dout, lse, D, Aw, DS);
      else
        k_attn_tuple<false><<<gt, 256, 0, s>>>(a, idx->tuple_group, dout, lse, D, Aw, DS);
      RELNN_LAUNCHED();
    }
    // dX_j[r] += sum over the tuples joined to row r of atom j of the
    // weighted rows: dQ <- scale ds K rows, dK <- scale ds Q rows, dV <- a dout rows
    struct Part {
      int j;
      const void* y;
      bool y_bf16;
      const int32_t* yrow;     // [E] row of y for each tuple (canonical order)
      int width;
      const float* wgt;
      int whd;
      float* dst;
    } parts[3] = {
        {0, k, a.bf16 != 0, a.rk, A->d, DS, A->d / A->heads, dq},
        {1, q, a.bf16 != 0, a.rq, A->d, DS, A->d / A->heads, dk},
        {2, dout, false, idx->tuple_group, A->dv, Aw, A->dv / A->heads, dv},
    };
    int32_t* yrow_t = reinterpret_cast<int32_t*>(w + P.yrow);
    for (const Part& pt : parts) {
      const int j = pt.j;
      if (j == 0 && q_fused) continue;
      const int64_t nseg = idx->t_nseg[j];
      if (nseg == 0) continue;
      k_gather_rows_idx<<<grid_n(E), 256, 0, s>>>(idx->t_pos[j], pt.yrow, E, yrow_t);
      RELNN_LAUNCHED();
      GsArgs g{};
      g.emb[0] = pt.y;
      g.rows[0] = yrow_t;                      // row of y at each transpose position
      g.rows[1] = idx->t_pos[j];               // its canonical tuple
      g.d[0] = pt.width;
      g.k = 1;
      g.K = pt.width;
      g.bf16 = pt.y_bf16;
      g.n = E;
      g.sg = Seg{idx->t_seg[j], idx->t_segoff[j], E, nullptr};
      g.out = pt.dst;                          // each segment's sum added into its row of dX_j
      g.out_row = idx->t_segrow[j];
      g.accumulate = true;
      g.ldo = pt.width;
      g.carry = reinterpret_cast<float*>(w + P.gcarry);
      g.wgt = pt.wgt;
      g.wh = A->heads;
      g.whd = pt.whd;
      seg_gather_sum(g, gs_units(E), s);
    }
  });
}
