// Backward of the product transform tau = act_pre(z_1 * ... * z_k) (the
// Score rule's q*k and the Attention rule's a*v of Section 1, the gated
// mean z_e*z_w of Section 5.4): the gradient of atom j's row r is
//
//   dz_j[r] = sum over the tuples joined to r of
//             dY_tau * act_pre'(z_1 * ... * z_k) * prod_{i != j} z_i[r_i(tau)]
//
// with dY_tau the routed gradient of the tuple (dA of its group; MEAN
// divided by the group's count; MAX only in the columns the tuple
// maximises).
//
// Atoms whose row is a function of the group (the head key's own relation,
// and relations reached from it by foreign keys) contribute one factor per
// group, Q_g = product of their rows.  The passes use that:
//
// * no such atom: one pass per atom over its transpose order (tuples sorted
//   by joined row), each term dA * act' * the other atoms' rows;
// * otherwise, with F the group-constant atoms and N the others:
//   - per group, R_g = dA_g * Q_g and the signs of Q_g;
//   - each atom j of N: a pass over its transpose order with terms
//     R_g * act' * the rows of N other than j (act' from the signs of the
//     rows of N and of Q_g);
//   - S_g = sum over the group's tuples of dA_g * act' * the rows of N, one
//     pass in canonical order; each atom j of F then receives S_g * the
//     other F rows of g, added straight into its row when j is keyed by the
//     group column (one group per row), else once per group in a pass over
//     j's transpose order.
//
// Every pass is a segmented sum: a wave takes a contiguous range of
// positions, sums each segment's terms with Kahan compensation and adds the
// sum into its row once; segments cut by range edges leave partials for the
// fix-up, which adds them in range order.  Atomic-free and deterministic.
#include "layer_fwd.hpp"

namespace relnn {
namespace {

constexpr int kPbTM = 64;        // range boundaries on multiples of 64 positions
constexpr int kPbWaves = 4;      // waves per block
constexpr int kPbBatch = 4;      // positions whose rows are loaded together (4: 8.3 ms a
                                 // three-atom backward over 20M tuples; 2, 6, 8 and 12:
                                 // 9.6, 8.8, 8.7 and 10.3 ms, fewer waves or fewer loads)

struct ProdBwdArgs {
  const void* emb[RELNN_MAX_ATOMS];          // [n_i][h], FP32 or bf16
  const int32_t* rows_t[RELNN_MAX_ATOMS];    // row of atom i at each position (atoms read only)
  uint32_t mult;                             // atoms whose rows multiply the term
  uint32_t sgn;                              // atoms whose signs enter act_pre'
  // the atoms a pass reads (mult, and sgn under ReLU), in atom order:
  // table, rows in the pass's order, and whether each multiplies (bit k of
  // lmult) or gives its sign (bit k of lsgn); filled at launch
  const void* lemb[RELNN_MAX_ATOMS];
  const int32_t* lrows[RELNN_MAX_ATOMS];
  uint32_t lmult, lsgn;
  const uint32_t* qsign;                     // [G][2][own_w]: Q_g > 0, Q_g < 0 bits, or null (Q = 1)
  const int32_t* grp_t;                      // group of the tuple at each position
  const int32_t* tau_t;                      // its canonical position, or null (the position itself)
  const float* B;                            // [G][h] per-group factor of the term
  const uint32_t* own;                       // MAX: maximiser bits [E][own_w], or null
  int own_w;
  int relu;                                  // apply act_pre' = [product > 0]
  int first_only;                            // add a group's term at its first position of the segment only
  int h;
  int64_t n;                                 // positions
  Seg sg;                                    // the rows (or groups) as segments of the order
  const int32_t* out_row;                    // segment -> output row, or null (the segment itself)
  float* out;                                // [.][h], accumulated
  float* carry;                              // [nunits][2][h]
  int64_t ntiles, nunits;
};

__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
  const float y = x - c;
  const float t = s + y;
  c = __builtin_isfinite(t) ? (t - s) - y : 0.0f;
  s = t;
}

template <bool kBF16>
__device__ __forceinline__ float2 row2(const void* base, int32_t row, int h, int col) {
  if constexpr (kBF16) {
    const uint32_t u = *reinterpret_cast<const uint32_t*>(static_cast<const __bf16*>(base) + (int64_t)row * h + col);
    return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
  } else {
    return *reinterpret_cast<const float2*>(static_cast<const float*>(base) + (int64_t)row * h + col);
  }
}

// The words of row2's two elements, loaded as they are (bf16: one word,
// FP32: two); row2_cvt turns them into FP32 where they are used, so that a
// batch's loads are all in flight before the first use waits for them.
template <bool kBF16>
__device__ __forceinline__ uint2 row2_raw(const void* base, int32_t row, int h, int col) {
  if constexpr (kBF16)
    return make_uint2(*reinterpret_cast<const uint32_t*>(static_cast<const __bf16*>(base) + (int64_t)row * h + col), 0u);
  else
    return *reinterpret_cast<const uint2*>(static_cast<const float*>(base) + (int64_t)row * h + col);
}

template <bool kBF16>
__device__ __forceinline__ float2 row2_cvt(uint2 u) {
  if constexpr (kBF16) return make_float2(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u));
  return make_float2(__uint_as_float(u.x), __uint_as_float(u.y));
}

// kNL: the number of atoms whose rows the pass reads (lemb, lrows).
template <bool kBF16, int kNL>
__global__ void __launch_bounds__(kPbWaves * 64) k_prod_bwd(ProdBwdArgs a) {
  const int lane = threadIdx.x % 64;
  const int64_t u = (int64_t)blockIdx.x * kPbWaves + threadIdx.x / 64;
  if (u >= a.nunits) return;
  const int64_t r0 = ((a.ntiles * u) / a.nunits) * kPbTM;
  const int64_t r1 = min<int64_t>(((a.ntiles * (u + 1)) / a.nunits) * kPbTM, a.n);
  if (r0 >= r1) return;
  const int h = a.h;
  constexpr int kNA = kNL > 0 ? kNL : 1;
  for (int cb = 0; cb < h; cb += 128) {
    const int col = cb + 2 * lane;
    const bool on = col < h;
    const int cc = on ? col : 0;
    float s0 = 0.f, s1 = 0.f, c0 = 0.f, c1 = 0.f;
    int32_t g = a.sg.seg_of[r0];
    const bool lo_cont = r0 > 0 && a.sg.seg_of[r0 - 1] == g;
    bool first = true;
    // the open segment's output row and that row's values so far, fetched
    // when the segment opens (the row is written by this wave alone), so
    // that closing it waits for neither
    int32_t grow = a.out_row ? a.out_row[g] : g;
    float2 gold = on ? *reinterpret_cast<const float2*>(a.out + (int64_t)grow * h + col) : make_float2(0.f, 0.f);
    auto flush = [&](bool last_seg) {
      const bool cut_lo = first && lo_cont;
      const bool cut_hi = last_seg && r1 < a.n && a.sg.seg_of[r1] == g;
      if (on) {
        const float v0 = s0 - c0, v1 = s1 - c1;
        if (cut_lo || cut_hi)
          *reinterpret_cast<float2*>(a.carry + (u * 2 + (cut_lo ? 0 : 1)) * h + col) = make_float2(v0, v1);
        else
          *reinterpret_cast<float2*>(a.out + (int64_t)grow * h + col) = make_float2(gold.x + v0, gold.y + v1);
      }
      first = false;
      s0 = s1 = c0 = c1 = 0.f;
    };
    for (int64_t base = r0; base < r1; base += 64) {
      const int n = (int)min<int64_t>(64, r1 - base);
      const int64_t e = base + min(lane, n - 1);
      const int32_t gl = a.sg.seg_of[e];
      const int32_t orl = a.out_row ? a.out_row[gl] : gl;   // output row of each position's segment
      const int32_t G = a.grp_t[e];
      const int32_t T = a.own ? (a.tau_t ? a.tau_t[e] : (int32_t)e) : 0;
      // the group of the position before the block (first_only)
      const int32_t gprev = (a.first_only && base > 0) ? a.grp_t[base - 1] : -1;
      // rows of the 64 positions, one vector per read atom
      int32_t R[kNA];
#pragma unroll
      for (int i = 0; i < kNL; ++i) R[i] = a.lrows[i][e];
      for (int bt = 0; bt < n; bt += kPbBatch) {
        // the batch's group, position and row numbers first (one wait for
        // the vectors they come from), then its loads (factor rows,
        // maximiser and sign words, atom rows), then its arithmetic
        int32_t sgrp[kPbBatch], sprev[kPbBatch], stau[kPbBatch], srow[kPbBatch][kNA];
#pragma unroll
        for (int b = 0; b < kPbBatch; ++b) {
          const int q = min(bt + b, n - 1);         // clamped: every load is valid
          sgrp[b] = __builtin_amdgcn_readlane(G, q);
          sprev[b] = q > 0 ? __builtin_amdgcn_readlane(G, q - 1) : gprev;
          stau[b] = __builtin_amdgcn_readlane(T, q);
#pragma unroll
          for (int i = 0; i < kNL; ++i) srow[b][i] = __builtin_amdgcn_readlane(R[i], q);
        }
        float2 dr[kPbBatch];
        uint32_t ow[kPbBatch], qp[kPbBatch], qn[kPbBatch];
        uint2 zr[kPbBatch][kNA];
        uint32_t skip = 0u;                         // positions whose term is zero (first_only)
#pragma unroll
        for (int b = 0; b < kPbBatch; ++b) {
          const int32_t grp = sgrp[b];
          if (a.first_only && sprev[b] == grp) {    // a group's term once per segment: no loads for the rest
            skip |= 1u << b;
            continue;
          }
          dr[b] = *reinterpret_cast<const float2*>(a.B + (int64_t)grp * h + cc);
          if (a.own)                                // MAX: the columns this tuple maximises
            ow[b] = a.own[(int64_t)stau[b] * a.own_w + (cc >> 5)];
#pragma unroll
          for (int i = 0; i < kNL; ++i) zr[b][i] = row2_raw<kBF16>(a.lemb[i], srow[b][i], h, cc);
          if (a.relu && a.qsign) {                  // the signs of the group's factor Q_g
            const uint32_t* qs = a.qsign + (int64_t)grp * 2 * a.own_w + (cc >> 5);
            qp[b] = qs[0];
            qn[b] = qs[a.own_w];
          }
        }
#pragma unroll
        for (int b = 0; b < kPbBatch; ++b) {
          const int q = bt + b;
          if (q >= n) break;
          const int32_t gq = __builtin_amdgcn_readlane(gl, q);
          if (gq != g) {                            // a segment ends
            flush(false);
            g = gq;
            grow = __builtin_amdgcn_readlane(orl, q);
            if (on) gold = *reinterpret_cast<const float2*>(a.out + (int64_t)grow * h + col);
          }
          float2 v = make_float2(0.0f, 0.0f);
          if (!((skip >> b) & 1u)) {
            float2 d = dr[b];
            if (a.own) {
              const uint32_t bits = ow[b] >> (cc & 31);
              d.x = (bits & 1u) ? d.x : 0.0f;
              d.y = (bits & 2u) ? d.y : 0.0f;
            }
            float2 m = make_float2(1.0f, 1.0f), ps = make_float2(1.0f, 1.0f);
#pragma unroll
            for (int i = 0; i < kNL; ++i) {
              const float2 z = row2_cvt<kBF16>(zr[b][i]);
              if ((a.lmult >> i) & 1u) {
                m.x *= z.x;
                m.y *= z.y;
              }
              if ((a.lsgn >> i) & 1u) {
                ps.x *= z.x;
                ps.y *= z.y;
              }
            }
            if (a.relu) {                           // act_pre'(product) = [product > 0], ReLU'(0) = 0
              if (a.qsign) {                        // times the sign of the group's factor Q_g
                const uint32_t pos = qp[b] >> (cc & 31), neg = qn[b] >> (cc & 31);
                ps.x = (pos & 1u) ? ps.x : ((neg & 1u) ? -ps.x : 0.0f);
                ps.y = (pos & 2u) ? ps.y : ((neg & 2u) ? -ps.y : 0.0f);
              }
              d.x = ps.x > 0.0f ? d.x : 0.0f;
              d.y = ps.y > 0.0f ? d.y : 0.0f;
            }
            v = make_float2(d.x * m.x, d.y * m.y);
          }
          kahan_add(s0, c0, v.x);
          kahan_add(s1, c1, v.y);
        }
      }
    }
    flush(true);
  }
}

// out[i] = y[ord[i]]
__global__ void k_gather_idx(const int32_t* ord, const int32_t* y, int64_t n, int32_t* out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = y[ord[i]];
}

__global__ void k_zero(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

// The group-constant atoms (bit set in fmask) of group g: the product of
// their rows at the group's first tuple, columns c, c + 1.
template <bool kBF16>
__device__ __forceinline__ float2 group_prod(const ProdBwdArgs& a, const int32_t* rows, int64_t E, uint32_t fmask,
                                             int64_t e0, int c) {
  float2 q = make_float2(1.0f, 1.0f);
#pragma unroll
  for (int i = 0; i < RELNN_MAX_ATOMS; ++i)
    if ((fmask >> i) & 1u) {
      const float2 z = row2<kBF16>(a.emb[i], rows[(int64_t)i * E + e0], a.h, c);
      q.x *= z.x;
      q.y *= z.y;
    }
  return q;
}

// Spreads the 16 bits of x to the even bit positions of a word.
__device__ __forceinline__ uint32_t spread16(uint32_t x) {
  x &= 0xffffu;
  x = (x | (x << 8)) & 0x00ff00ffu;
  x = (x | (x << 4)) & 0x0f0f0f0fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}

// Per group g: R_g = dA_g * Q_g and the sign bits of Q_g (Q_g the product
// of the group-constant atoms' rows).  One wave per group and 128 columns,
// lane l owning columns 2 l and 2 l + 1; the sign words are assembled from
// ballots (word w: lanes 16 w .. 16 w + 15, their two columns interleaved).
template <bool kBF16>
__global__ void k_pb_group(ProdBwdArgs a, const int32_t* rows, const int32_t* offsets, int64_t E, int64_t G,
                           uint32_t fmask, const float* dA, float* Rg, uint32_t* qsign) {
  const int lane = threadIdx.x % 64;
  const int nw = a.own_w, h = a.h;
  const int ncb = (h + 127) / 128;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t wv = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; wv < G * ncb; wv += waves) {
    const int64_t g = wv / ncb;
    const int cb = 128 * (int)(wv - g * ncb);
    const int c = cb + 2 * lane;
    const bool on = c < h;
    const int cc = on ? c : 0;
    const int64_t e0 = offsets[g];
    const float2 q = group_prod<kBF16>(a, rows, E, fmask, e0, cc);
    if (on) {
      const float2 d = *reinterpret_cast<const float2*>(dA + g * h + c);
      *reinterpret_cast<float2*>(Rg + g * h + c) = make_float2(d.x * q.x, d.y * q.y);
    }
    const uint64_t px = __ballot(on && q.x > 0.0f), py = __ballot(on && q.y > 0.0f);
    const uint64_t nx = __ballot(on && q.x < 0.0f), ny = __ballot(on && q.y < 0.0f);
    if (lane < 4) {                                // word cb / 32 + lane: lanes 16 lane .. + 15
      const int w = cb / 32 + lane;
      if (w < nw) {
        const int sh = 16 * lane;
        const uint32_t pos = spread16((uint32_t)(px >> sh)) | (spread16((uint32_t)(py >> sh)) << 1);
        const uint32_t neg = spread16((uint32_t)(nx >> sh)) | (spread16((uint32_t)(ny >> sh)) << 1);
        qsign[g * 2 * nw + w] = pos;
        qsign[g * 2 * nw + nw + w] = neg;
      }
    }
  }
}

// Atom j of the group-constant atoms: V_g = S_g * the rows of the other
// group-constant atoms (omask).  direct: added into row r_j(g) of out (j
// keyed by the group column: one group per row); else stored in V.
template <bool kBF16>
__global__ void k_pb_fatom(ProdBwdArgs a, const int32_t* rows, const int32_t* offsets, int64_t E, int64_t G,
                           uint32_t omask, int j, const float* S, int direct, float* out, float* V) {
  const int C2 = a.h / 2;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < G * C2; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = i / C2;
    const int c = 2 * (int)(i - g * C2);
    const int64_t e0 = offsets[g];
    const float2 q = group_prod<kBF16>(a, rows, E, omask, e0, c);
    const float2 s = *reinterpret_cast<const float2*>(S + g * a.h + c);
    const float2 v = make_float2(s.x * q.x, s.y * q.y);
    if (direct) {
      float2* dst = reinterpret_cast<float2*>(out + (int64_t)rows[(int64_t)j * E + e0] * a.h + c);
      const float2 o = *dst;
      *dst = make_float2(o.x + v.x, o.y + v.y);
    } else {
      *reinterpret_cast<float2*>(V + g * a.h + c) = v;
    }
  }
}

int64_t pb_units(int64_t E) { return std::max<int64_t>(1, std::min<int64_t>(cdiv(std::max<int64_t>(E, 1), kPbTM), 8192)); }

unsigned grid_n(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 1 << 16)); }

struct PbLayout {
  size_t other_rows = 0, carry = 0, Rg = 0, qsign = 0, S = 0, V = 0, total = 0;
};

PbLayout pb_layout(const relnn_index* idx, const relnn_layer_desc* L) {
  PbLayout p;
  const int64_t E = std::max<int64_t>(idx->E, 1), G = std::max<int64_t>(idx->G, 1);
  const int h = L->h, nw = (int)cdiv(h, 32);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += round_up(std::max<size_t>(bytes, 1), 256);
    return o;
  };
  p.other_rows = take((size_t)E * 4 * RELNN_MAX_ATOMS);
  p.carry = take((size_t)pb_units(idx->E) * 2 * h * 4);
  p.Rg = take((size_t)G * h * 4);
  p.qsign = take((size_t)G * 2 * nw * 4);
  p.S = take((size_t)G * h * 4);
  p.V = take((size_t)G * h * 4);
  p.total = off;
  return p;
}

}  // namespace

size_t prod_bwd_ws_bytes(const relnn_index* idx, const relnn_layer_desc* L) { return pb_layout(idx, L).total; }

void prod_bwd(const relnn_index* idx, const relnn_layer_desc* L, const void* const* emb, const float* dA,
              const uint32_t* own, int own_w, float* const* demb, char* ws, hipStream_t s) {
  const int64_t E = idx->E, G = idx->G;
  const int h = L->h, k = L->k;
  RELNN_REQUIRE(h % 2 == 0, RELNN_E_UNSUPPORTED, "the product backward needs an even h");
  if (E == 0) return;
  const PbLayout P = pb_layout(idx, L);
  int32_t* other_rows = reinterpret_cast<int32_t*>(ws + P.other_rows);   // [atom][E] rows in one atom's order
  float* carry = reinterpret_cast<float*>(ws + P.carry);
  const bool bf16 = L->dtype == RELNN_BF16;
  const bool relu = L->act_pre == RELNN_ACT_RELU;
  const unsigned gE = grid_n(E);
  const int qw = (int)cdiv(h, 32);                     // words of a row's column bits
  const uint32_t all = (1u << k) - 1u;
  uint32_t fmask = 0u;
  for (int j = 0; j < k; ++j)
    if (idx->atom_fd[j]) fmask |= 1u << j;
  const uint32_t nmask = all & ~fmask;

  ProdBwdArgs base{};
  for (int i = 0; i < k; ++i) base.emb[i] = emb[i];
  base.own = own;
  base.own_w = own ? own_w : qw;
  base.h = h;
  base.n = E;
  base.carry = carry;
  base.ntiles = cdiv(E, kPbTM);
  auto run = [&](ProdBwdArgs a, float* out, const int32_t* out_row) {
    a.out = out;
    a.out_row = out_row;
    // the atoms the pass reads, in atom order (their rows in rows_t)
    const uint32_t loads = a.mult | (a.relu ? a.sgn : 0u);
    int nl = 0;
    a.lmult = a.lsgn = 0u;
    for (int i = 0; i < RELNN_MAX_ATOMS; ++i) {
      if (!((loads >> i) & 1u)) continue;
      a.lemb[nl] = a.emb[i];
      a.lrows[nl] = a.rows_t[i];
      if ((a.mult >> i) & 1u) a.lmult |= 1u << nl;
      if ((a.sgn >> i) & 1u) a.lsgn |= 1u << nl;
      ++nl;
    }
    {
      KTimer tm("bwd_dx", s);
      auto go = [&](auto kern) {
        a.nunits = one_round_units(kern, kPbWaves * 64, pb_units(E));
        kern<<<(unsigned)cdiv(a.nunits, kPbWaves), kPbWaves * 64, 0, s>>>(a);
      };
      auto pick = [&](auto B) {
        constexpr bool kB = decltype(B)::value;
        switch (nl) {
          case 0: go(k_prod_bwd<kB, 0>); break;
          case 1: go(k_prod_bwd<kB, 1>); break;
          case 2: go(k_prod_bwd<kB, 2>); break;
          case 3: go(k_prod_bwd<kB, 3>); break;
          default: go(k_prod_bwd<kB, 4>); break;
        }
      };
      if (bf16)
        pick(std::true_type{});
      else
        pick(std::false_type{});
      RELNN_LAUNCHED();
    }
    Sink sk{};
    sk.agg = RELNN_SUM;
    sk.act_post = RELNN_ACT_NONE;
    sk.out = out;
    sk.out_row = out_row;
    sk.accumulate = true;
    launch_fixup(a.sg, kPbTM, h, a.ntiles, a.nunits, sk, carry, nullptr, s);
  };
  // a pass over atom j's transpose order, with the rows of the atoms in
  // `need` gathered into that order
  auto transposed = [&](int j, uint32_t need, ProdBwdArgs a) {
    for (int i = 0; i < k; ++i) {
      if (!((need >> i) & 1u)) continue;
      if (i == j) {
        a.rows_t[i] = idx->t_row[j];
      } else {
        int32_t* dst = other_rows + (int64_t)i * E;
        k_gather_idx<<<gE, 256, 0, s>>>(idx->t_pos[j], idx->rows + (int64_t)i * E, E, dst);
        RELNN_LAUNCHED();
        a.rows_t[i] = dst;
      }
    }
    a.grp_t = idx->t_grp[j];
    a.tau_t = idx->t_pos[j];
    a.sg = Seg{idx->t_seg[j], idx->t_segoff[j], E, nullptr};
    run(a, demb[j], idx->t_segrow[j]);
  };

  if (fmask == 0u) {                                   // every atom varies inside a group
    for (int j = 0; j < k; ++j) {
      if (idx->t_nseg[j] == 0) continue;
      ProdBwdArgs a = base;
      a.B = dA;
      a.mult = all & ~(1u << j);
      a.sgn = all;
      a.relu = relu;
      transposed(j, a.mult | (relu ? a.sgn : 0u), a);
    }
    return;
  }

  // per group: R_g = dA_g * Q_g, the signs of Q_g
  float* Rg = reinterpret_cast<float*>(ws + P.Rg);
  uint32_t* qsign = reinterpret_cast<uint32_t*>(ws + P.qsign);
  {
    ProdBwdArgs a = base;
    a.own_w = qw;
    if (bf16)
      k_pb_group<true><<<grid_n(G * cdiv(h, 128) * 64), 256, 0, s>>>(a, idx->rows, idx->offsets, E, G, fmask, dA,
                                                                       Rg, qsign);
    else
      k_pb_group<false><<<grid_n(G * cdiv(h, 128) * 64), 256, 0, s>>>(a, idx->rows, idx->offsets, E, G, fmask, dA,
                                                                        Rg, qsign);
    RELNN_LAUNCHED();
  }
  // the sign words are read with the stride of the ownership words
  RELNN_REQUIRE(!own || own_w == qw, RELNN_E_HIP, "internal: ownership words %d, column words %d", own_w, qw);
  // the atoms varying inside a group
  for (int j = 0; j < k; ++j) {
    if (!((nmask >> j) & 1u) || idx->t_nseg[j] == 0) continue;
    ProdBwdArgs a = base;
    a.B = Rg;
    a.mult = nmask & ~(1u << j);
    a.sgn = nmask;
    a.relu = relu;
    a.qsign = relu ? qsign : nullptr;
    transposed(j, a.mult | (relu ? a.sgn : 0u), a);
  }
  // S_g over each group's tuples, in canonical order
  float* S = reinterpret_cast<float*>(ws + P.S);
  k_zero<<<grid_n(G * h), 256, 0, s>>>(S, G * h);
  RELNN_LAUNCHED();
  {
    ProdBwdArgs a = base;
    a.B = dA;
    a.mult = nmask;
    a.sgn = nmask;
    a.relu = relu;
    a.qsign = relu ? qsign : nullptr;
    for (int i = 0; i < k; ++i) a.rows_t[i] = idx->rows + (int64_t)i * E;
    a.grp_t = idx->tuple_group;
    a.tau_t = nullptr;
    a.sg = Seg{idx->tuple_group, idx->offsets, E, nullptr};
    run(a, S, nullptr);
  }
  // the group-constant atoms
  float* V = reinterpret_cast<float*>(ws + P.V);
  for (int j = 0; j < k; ++j) {
    if (!((fmask >> j) & 1u)) continue;
    const bool direct = idx->atom_gk[j];
    {
      KTimer tm("bwd_dx", s);
      const unsigned gg = grid_n(G * (h / 2));
      if (bf16)
        k_pb_fatom<true><<<gg, 256, 0, s>>>(base, idx->rows, idx->offsets, E, G, fmask & ~(1u << j), j, S,
                                            direct ? 1 : 0, demb[j], V);
      else
        k_pb_fatom<false><<<gg, 256, 0, s>>>(base, idx->rows, idx->offsets, E, G, fmask & ~(1u << j), j, S,
                                             direct ? 1 : 0, demb[j], V);
      RELNN_LAUNCHED();
    }
    if (!direct && idx->t_nseg[j] > 0) {                 // V_g added once per group into row r_j(g)
      ProdBwdArgs a = base;
      a.B = V;
      a.mult = 0u;
      a.sgn = 0u;
      a.relu = 0;
      a.own = nullptr;
      a.first_only = 1;
      transposed(j, 0u, a);
    }
  }
}

}  // namespace relnn
