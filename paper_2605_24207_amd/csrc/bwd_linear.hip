// Backward of a relational layer through sums over groups and over joined
// rows.  With dY_tau the gradient of tuple tau's transformed value
// (dA_g = dout_g * act_post'(pre_g), divided by |g| for MEAN; routed to the
// maximiser tuple per column for MAX; masked by act_pre' when act_pre is
// ReLU), the map from x_tau to y_tau is affine, so for every layer
//
//   dz_j[r] += (sum_{tau joined to row r} dY_tau) W_j^T  =  DS_j[r] W_j^T
//
// and, when dY_tau = dA_g for every tuple of g (SUM or MEAN with an affine
// transform: the transformation commutes with the union, Section 2.2),
//
//   dW = sum_g (sum_{tau in g} x_tau)^T dA_g = XS^T dA,   db = sum_g |g| dA_g.
//
// XS [G, K] and DS_j [rows of j, h] are segmented gather-sums over sorted
// lists (k_seg_gather_sum: atomic-free, deterministic); the products on them
// (gemm.hip: FP32 or, for bf16 layers, bf16 matrix-core products with FP32
// accumulation) are far smaller than the per-tuple ones.  dW of the other
// layers is the per-tuple product of layer_bwd.hip.
#include "gemm.hpp"
#include "layer_fwd.hpp"
#include "prims.hpp"

namespace relnn {

namespace {

constexpr int kGsTM = 64;          // unit boundaries on multiples of 64 positions
constexpr int kGsWaves = 4;        // waves per block
constexpr int kGsBatch = 8;        // positions loaded together

// Compensated add; the compensation is dropped once the sum is not finite
// (an infinite sum stays infinite instead of turning NaN).
__device__ __forceinline__ void kahan_add1(float& s, float& c, float x) {
  const float y = x - c;
  const float t = s + y;
  c = __builtin_isfinite(t) ? (t - s) - y : 0.0f;
  s = t;
}

// Four consecutive elements of column block cq of the joined row at list
// position e, as FP32.  The atom of the block is picked with compile-time
// indices (a run-time index into the argument's arrays would put it in
// scratch memory).
struct GsAtom {
  const void* emb;
  int d, koff, j;
};

__device__ __forceinline__ GsAtom gs_atom(const GsArgs& a, int col) {
  GsAtom r{a.emb[0], a.d[0], 0, 0};
  auto pick = [&](auto U) {
    constexpr int u = decltype(U)::value;
    if (u < a.k && col >= a.koff[u]) r = GsAtom{a.emb[u], a.d[u], a.koff[u], u};
  };
  pick(std::integral_constant<int, 1>{});
  pick(std::integral_constant<int, 2>{});
  pick(std::integral_constant<int, 3>{});
  return r;
}

// The words holding VW (4 or 2) consecutive elements of the joined row at
// list position e (bf16: VW/2 words, FP32: VW words; the rest zero).  The
// conversion to FP32 is kept apart (gs_cvt) so that it is done where the
// value is added: a use right after the load would make the wave wait for
// each row before it asks for the next.
template <int VW, bool kBF16>
__device__ __forceinline__ uint4 gs_load_raw(const GsAtom& A, int32_t row, int col) {
  const int64_t o = (int64_t)row * A.d + (col - A.koff);
  uint4 r{0u, 0u, 0u, 0u};
  if constexpr (kBF16) {
    const __bf16* p = static_cast<const __bf16*>(A.emb) + o;
    if constexpr (VW == 4) {
      const uint2 v = *reinterpret_cast<const uint2*>(p);
      r.x = v.x;
      r.y = v.y;
    } else {
      r.x = *reinterpret_cast<const uint32_t*>(p);
    }
  } else {
    const float* p = static_cast<const float*>(A.emb) + o;
    if constexpr (VW == 4) {
      r = *reinterpret_cast<const uint4*>(p);
    } else {
      const uint2 v = *reinterpret_cast<const uint2*>(p);
      r.x = v.x;
      r.y = v.y;
    }
  }
  return r;
}

// The VW elements of gs_load_raw's words as FP32 (the unused lanes of the
// f32x4 are zero).
template <bool kBF16>
__device__ __forceinline__ f32x4 gs_cvt(uint4 r) {
  if constexpr (kBF16)
    return f32x4{__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xffff0000u), __uint_as_float(r.y << 16),
                 __uint_as_float(r.y & 0xffff0000u)};
  return f32x4{__uint_as_float(r.x), __uint_as_float(r.y), __uint_as_float(r.z), __uint_as_float(r.w)};
}

// out[s] = sum over the positions e of segment s of the joined row at e.
// One wavefront per unit of positions [pos(u), pos(u+1)), pos(u) = (ntiles
// u / nunits) 64; lane l owns the VW columns VW (64 p + l) .. of pass p.  A
// segment cut by a unit end leaves its partial in carry slot 0 (cut by the
// start) or 1 (runs past the end); k_fixup combines them in unit order.
// VW columns per lane: 4, or 2 for rows of at most 128 elements (all 64
// lanes busy; a wave instruction costs the same with 32 or 64 lanes on).
// kMode 0: plain sums written to out[s]; 1: rows may be scaled by a
// per-tuple weight (wgt) or masked by per-tuple ownership bits (own); 2: as
// 1, and the sums may go to remapped rows (out_row) and be added to what
// they hold (accumulate).
template <int VW, bool kBF16, int kMode>
__global__ void __launch_bounds__(kGsWaves * 64) k_seg_gather_sum(GsArgs a) {
  const int lane = threadIdx.x % 64;
  const int64_t u = (int64_t)blockIdx.x * kGsWaves + threadIdx.x / 64;
  if (u >= a.nunits) return;
  const int64_t r0 = ((a.ntiles * u) / a.nunits) * kGsTM;
  const int64_t r1 = min<int64_t>(((a.ntiles * (u + 1)) / a.nunits) * kGsTM, a.n);
  if (r0 >= r1) return;
  const int K = a.K;
  constexpr bool kTw = kMode >= 1;
  constexpr bool kRmw = kMode == 2;

  for (int cb = 0; cb < K; cb += 64 * VW) {
    const int col = cb + VW * lane;
    const bool on = col < K;
    const GsAtom A = gs_atom(a, on ? col : 0);
    f32x4 s = {0.f, 0.f, 0.f, 0.f}, c = {0.f, 0.f, 0.f, 0.f};
    int32_t g = a.sg.seg_of[r0];
    // only the range's first segment can have begun before r0, and only its
    // last one can run past r1: one list read at each end instead of two
    // dependent offset reads at every segment end
    const bool lo_cont = r0 > 0 && a.sg.seg_of[r0 - 1] == g;
    bool first = true;
    // the open segment's output row and (accumulate) that row's values so
    // far, fetched when the segment opens, so that closing it waits for
    // neither: a segment's row is written by its wave alone
    auto old_vals = [&](int32_t orow) {
      f32x4 o = {0.f, 0.f, 0.f, 0.f};
      if (kRmw && a.accumulate && on) {
        const float* p = a.out + (int64_t)orow * a.ldo + col;
        if constexpr (VW == 4) {
          o = *reinterpret_cast<const f32x4*>(p);
        } else {
          const float2 t = *reinterpret_cast<const float2*>(p);
          o[0] = t.x;
          o[1] = t.y;
        }
      }
      return o;
    };
    int32_t grow = (kRmw && a.out_row) ? a.out_row[g] : g;
    f32x4 gold = old_vals(grow);
    auto flush = [&](bool last_seg) {
      const bool cut_lo = first && lo_cont;
      const bool cut_hi = last_seg && r1 < a.n && a.sg.seg_of[r1] == g;
      if (on) {
        f32x4 v = s - c;
        const bool cut = cut_lo || cut_hi;
        float* dst = cut ? a.carry + (u * 2 + (cut_lo ? 0 : 1)) * a.ldo + col : a.out + (int64_t)grow * a.ldo + col;
        if (kRmw && a.accumulate && !cut) {
          if constexpr (VW == 4) {
            v += gold;
          } else {
            v[0] += gold[0];
            v[1] += gold[1];
          }
        }
        if constexpr (VW == 4)
          *reinterpret_cast<f32x4*>(dst) = v;
        else
          *reinterpret_cast<float2*>(dst) = make_float2(v[0], v[1]);
      }
      first = false;
      s = f32x4{0.f, 0.f, 0.f, 0.f};
      c = s;
    };
    for (int64_t base = r0; base < r1; base += 64) {
      const int n = (int)min<int64_t>(64, r1 - base);
      const int64_t e = base + min(lane, n - 1);
      const int32_t gl = a.sg.seg_of[e];
      const int32_t orl = (kRmw && a.out_row) ? a.out_row[gl] : gl;   // output row of each position's segment
      // row numbers of the 64 positions, one vector per atom (absent ones
      // repeat atom 0)
      int32_t R[kMaxAtoms];
#pragma unroll
      for (int j = 0; j < kMaxAtoms; ++j) R[j] = (a.rows[j] ? a.rows[j] : a.rows[0])[e];
      for (int bt = 0; bt < n; bt += kGsBatch) {
        // all loads of the batch first (rows, and the weight or ownership
        // word of each tuple), then the conversions and the adds in order
        uint4 raw[kGsBatch];
        float wv[kGsBatch];
        uint32_t ob[kGsBatch];
        const int cc = on ? col : 0;
#pragma unroll
        for (int i = 0; i < kGsBatch; ++i) {
          const int q = min(bt + i, n - 1);           // clamped: every load is valid
          int32_t row = __builtin_amdgcn_readlane(R[0], q);
#pragma unroll
          for (int j = 1; j < kMaxAtoms; ++j) {
            const int32_t rj = __builtin_amdgcn_readlane(R[j], q);
            row = A.j == j ? rj : row;
          }
          raw[i] = gs_load_raw<VW, kBF16>(A, row, cc);
          if constexpr (kTw) {
            const int32_t tau = __builtin_amdgcn_readlane(R[1], q);
            wv[i] = a.wgt ? a.wgt[(int64_t)tau * a.wh + cc / a.whd] : 1.0f;   // one weight per tuple and column block
            ob[i] = a.own ? a.own[(int64_t)tau * a.own_w + (cc >> 5)] : ~0u;   // VW columns of one 32-column word
          }
        }
#pragma unroll
        for (int i = 0; i < kGsBatch; ++i) {
          const int q = bt + i;
          if (q >= n) break;
          const int32_t gq = __builtin_amdgcn_readlane(gl, q);
          if (__builtin_expect(gq != g, 0)) {         // a segment ends
            flush(false);
            g = gq;
            grow = __builtin_amdgcn_readlane(orl, q);
            gold = old_vals(grow);
          }
          f32x4 v = gs_cvt<kBF16>(raw[i]);
          if (kTw && a.wgt) {
#pragma unroll
            for (int x = 0; x < VW; ++x) v[x] *= wv[i];
          }
          if (kTw && a.own) {                           // route the gradient row of this tuple
#pragma unroll
            for (int x = 0; x < VW; ++x) v[x] = ((ob[i] >> ((cc & 31) + x)) & 1u) ? v[x] : 0.0f;
          }
#pragma unroll
          for (int x = 0; x < VW; ++x) {
            float sx = s[x], cx = c[x];
            kahan_add1(sx, cx, v[x]);
            s[x] = sx;
            c[x] = cx;
          }
        }
      }
    }
    flush(true);
  }
}

}  // namespace

int64_t gs_units(int64_t n) {
  const int64_t nt = cdiv(std::max<int64_t>(n, 1), kGsTM);
  return std::max<int64_t>(1, std::min<int64_t>(nt, 8192));
}

void seg_gather_sum(GsArgs a, int64_t nseg_units_cap, hipStream_t s) {
  a.ntiles = cdiv(a.n, kGsTM);
  // Up to 8192 waves, more than the GPU holds at once: the ranges differ in
  // cost (each row that ends is a read-modify-write), and the waves of a
  // second round even that out; one round of fewer, longer ranges measured
  // about 5 % slower.
  a.nunits = gs_units(a.n);
  RELNN_REQUIRE(a.nunits <= nseg_units_cap, RELNN_E_HIP, "internal: carry region too small");
  RELNN_REQUIRE(a.K % 4 == 0, RELNN_E_UNSUPPORTED, "row width %d is not a multiple of 4", a.K);
  const unsigned g = (unsigned)cdiv(a.nunits, kGsWaves);
  // the per-tuple words and the read-modify-write of output rows cost
  // registers in every variant that may use them; plain sums use one that
  // does not
  const int mode = (a.out_row || a.accumulate) ? 2 : (a.wgt || a.own) ? 1 : 0;
  auto go = [&](auto kern) { kern<<<g, kGsWaves * 64, 0, s>>>(a); };
  auto pick = [&](auto VWc, auto Bc) {
    constexpr int kVW = decltype(VWc)::value;
    constexpr bool kB = decltype(Bc)::value;
    if (mode == 2)
      go(k_seg_gather_sum<kVW, kB, 2>);
    else if (mode == 1)
      go(k_seg_gather_sum<kVW, kB, 1>);
    else
      go(k_seg_gather_sum<kVW, kB, 0>);
  };
  if (a.K <= 128) {
    if (a.bf16)
      pick(std::integral_constant<int, 2>{}, std::true_type{});
    else
      pick(std::integral_constant<int, 2>{}, std::false_type{});
  } else {
    if (a.bf16)
      pick(std::integral_constant<int, 4>{}, std::true_type{});
    else
      pick(std::integral_constant<int, 4>{}, std::false_type{});
  }
  RELNN_LAUNCHED();
  // the fix-up reads carry slots and writes out rows with stride ldo
  Sink sk{};
  sk.agg = RELNN_SUM;
  sk.act_post = RELNN_ACT_NONE;
  sk.out = a.out;
  sk.out_row = a.out_row;
  sk.accumulate = a.accumulate;
  launch_fixup(a.sg, kGsTM, a.ldo, a.ntiles, a.nunits, sk, a.carry, nullptr, s);
}


// Workspace of the aggregated backward, after `base` bytes.
LinBwdPlan plan_lin_bwd(const relnn_index* idx, const relnn_layer_desc* L, size_t base, bool xs_dw) {
  LinBwdPlan p;
  int K = 0;
  for (int j = 0; j < L->k; ++j) K += L->d[j];
  int64_t nseg = 1;
  for (int j = 0; j < L->k; ++j) nseg = std::max<int64_t>(nseg, idx->t_nseg[j]);
  const int64_t G = std::max<int64_t>(idx->G, 1), E = std::max<int64_t>(idx->E, 1);
  const int h = L->h;
  size_t off = base;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += round_up(bytes, 256);
    return o;
  };
  p.units = gs_units(E);
  p.ldx = K;
  if (xs_dw) {
    p.ws_xs = take((size_t)G * p.ldx * 4);
    p.ws_part = take((size_t)gemm_tn_ws_floats(G, K, h) * 4);
  }
  p.ws_ds = take((size_t)nseg * h * 4);
  p.ws_carry = take((size_t)p.units * 2 * std::max(p.ldx, h) * 4);
  p.total = off;
  return p;
}

void lin_bwd_dw(const relnn_index* idx, const relnn_layer_desc* L, const LinBwdPlan& P, const void* const* emb,
                const float* dA, float* dW, float* db, bool accum, char* w, hipStream_t s) {
  const int h = L->h;
  const int64_t G = idx->G, E = idx->E;
  int K = 0;
  for (int j = 0; j < L->k; ++j) K += L->d[j];
  float* xs = reinterpret_cast<float*>(w + P.ws_xs);
  KTimer tm("bwd_dw", s);
  // XS: per-group sums of the joined rows (canonical order, groups as
  // segments)
  {
    GsArgs a{};
    int koff = 0;
    for (int j = 0; j < L->k; ++j) {
      a.emb[j] = emb[j];
      a.rows[j] = idx->rows + (int64_t)j * E;
      a.d[j] = L->d[j];
      a.koff[j] = koff;
      koff += L->d[j];
    }
    a.k = L->k;
    a.K = K;
    a.bf16 = L->dtype == RELNN_BF16;
    a.n = E;
    a.sg = Seg{idx->tuple_group, idx->offsets, E, nullptr};
    a.out = xs;
    a.ldo = P.ldx;
    a.carry = reinterpret_cast<float*>(w + P.ws_carry);
    seg_gather_sum(a, P.units, s);
  }
  // dW = XS^T dA and db = sum_g |g| dA_g, split over chunks of groups whose
  // partials are added in chunk order
  TnB B;
  B.B = dA;
  B.ldb = h;
  gemm_tn(L->dtype == RELNN_BF16, xs, false, P.ldx, nullptr, nullptr, B, G, K, h, idx->offsets, dW, db, accum,
          reinterpret_cast<float*>(w + P.ws_part), s);
}

int64_t gk_dw_ws_floats(int64_t G, int d, int h) { return gemm_tn_ws_floats(G, d, h); }

// dW rows of atom j = sum_g x_j(g)^T dA_g, x_j(g) the row group g joins
// (rows[offsets[g]]), gathered by the product itself.
void gk_dw(const relnn_index* idx, int j, const void* emb, bool bf16, int d, int h, const float* dA, float* dW_rows,
           bool accum, float* part, hipStream_t s) {
  const int64_t G = idx->G, E = idx->E;
  TnB B;
  B.B = dA;
  B.ldb = h;
  gemm_tn(bf16, emb, bf16, d, idx->rows + (int64_t)j * E, idx->offsets, B, G, d, h, nullptr, dW_rows, nullptr,
          accum, part, s);
}

void lin_bwd_dx(const relnn_index* idx, const relnn_layer_desc* L, const LinBwdPlan& P, const void* W,
                const float* dA, const uint32_t* route, int route_w, bool per_tuple, float* const* demb, char* w,
                hipStream_t s) {
  const int h = L->h;
  const int64_t E = idx->E;
  const bool bf16 = L->dtype == RELNN_BF16;
  const size_t esz = bf16 ? 2 : 4;
  const bool routed = route != nullptr;
  // dz_j = DS_j W_j^T, added into the rows of atom j.  W_j = rows koff.. of
  // W ([d][h]), so the product's B[k][n] = W[koff + n][k] (k < h, n < d).
  for (int j = 0, koff = 0; j < L->k; koff += L->d[j], ++j) {
    const int d = L->d[j];
    const int64_t nseg = idx->t_nseg[j];
    if (nseg == 0) continue;
    RELNN_REQUIRE(d % 4 == 0, RELNN_E_UNSUPPORTED, "backward needs d %% 4 == 0");
    const void* Wj = static_cast<const char*>(W) + (size_t)koff * h * esz;
    if (idx->atom_gk[j] && !per_tuple) {
      // one row per group: DS_j[row of g] = w_g dA_g, w_g = |g| (SUM, MEAN)
      // or 1 (MAX: each column goes to exactly one tuple of the group)
      KTimer tm("bwd_dx", s);
      RowsEpi epi;
      epi.orow = idx->rows + (int64_t)j * E;
      epi.oidx = idx->offsets;
      epi.wcnt = L->agg == RELNN_MAX ? nullptr : idx->offsets;
      epi.accumulate = true;
      gemm_rows(bf16, dA, false, h, idx->G, h, Wj, bf16, true, h, d, demb[j], d, epi, s);
      continue;
    }
    const int32_t* tg = idx->t_grp[j];                               // group of each transposed tuple
    float* ds = reinterpret_cast<float*>(w + P.ws_ds);
    KTimer tm("bwd_dx", s);
    GsArgs a{};
    a.emb[0] = dA;
    a.rows[0] = tg;
    a.rows[1] = routed ? idx->t_pos[j] : tg;                         // canonical position of each tuple
    a.d[0] = h;
    a.koff[0] = 0;
    a.k = 1;
    a.K = h;
    a.bf16 = false;
    a.n = E;
    a.sg = Seg{idx->t_seg[j], idx->t_segoff[j], E, nullptr};
    a.out = ds;
    a.ldo = h;
    a.carry = reinterpret_cast<float*>(w + P.ws_carry);
    a.own = route;
    a.own_w = route_w;
    seg_gather_sum(a, P.units, s);
    RowsEpi epi;
    epi.orow = idx->t_segrow[j];
    epi.accumulate = true;
    gemm_rows(bf16, ds, false, h, nseg, h, Wj, bf16, true, h, d, demb[j], d, epi, s);
  }
}

}  // namespace relnn
