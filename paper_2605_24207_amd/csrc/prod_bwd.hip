// Backward of the product transform tau = act_pre(z_1 * ... * z_k) (the
// Score rule's q*k and the Attention rule's a*v of Section 1, the gated
// mean z_e*z_w of Section 5.4): the gradient of atom j's row r is
//
//   dz_j[r] = sum over the tuples joined to r of
//             dY_tau * act_pre'(z_1 * ... * z_k) * prod_{i != j} z_i[r_i(tau)]
//
// with dY_tau the routed gradient of the tuple (dA of its group; MEAN
// divided by the group's count; MAX only in the columns the tuple
// maximises).  One pass per atom over its transpose order (tuples sorted by
// joined row): a wave takes a contiguous range of positions, sums each
// row's terms with Kahan compensation and adds the sum into the row of
// dz_j once; rows cut by range edges leave partials for the fix-up, which
// adds them in range order.  Atomic-free and deterministic.
#include "layer_fwd.hpp"

namespace relnn {
namespace {

constexpr int kPbTM = 64;        // range boundaries on multiples of 64 positions
constexpr int kPbWaves = 4;      // waves per block
constexpr int kPbBatch = 8;      // positions whose rows are loaded together

struct ProdBwdArgs {
  int k, j;                                  // atoms; the one differentiated
  const void* emb[RELNN_MAX_ATOMS];          // [n_i][h], FP32 or bf16
  const int32_t* rows_t[RELNN_MAX_ATOMS];    // row of atom i at each position of j's transpose order
  const int32_t* grp_t;                      // group of the tuple at each position
  const int32_t* tau_t;                      // canonical position of that tuple
  const float* dA;                           // [G][h] routed gradient per group (MEAN divided)
  const uint32_t* own;                       // MAX: maximiser bits [E][own_w], or null
  int own_w;
  int act_pre;
  int h;
  int64_t n;                                 // positions (E)
  Seg sg;                                    // rows of atom j as segments of its transpose order
  const int32_t* out_row;                    // segment -> row of dz_j
  float* out;                                // dz_j [n_j][h], accumulated
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

template <bool kBF16>
__global__ void __launch_bounds__(kPbWaves * 64) k_prod_bwd(ProdBwdArgs a) {
  const int lane = threadIdx.x % 64;
  const int64_t u = (int64_t)blockIdx.x * kPbWaves + threadIdx.x / 64;
  if (u >= a.nunits) return;
  const int64_t r0 = ((a.ntiles * u) / a.nunits) * kPbTM;
  const int64_t r1 = min<int64_t>(((a.ntiles * (u + 1)) / a.nunits) * kPbTM, a.n);
  if (r0 >= r1) return;
  const int h = a.h;
  for (int cb = 0; cb < h; cb += 128) {
    const int col = cb + 2 * lane;
    const bool on = col < h;
    const int cc = on ? col : 0;
    float s0 = 0.f, s1 = 0.f, c0 = 0.f, c1 = 0.f;
    int32_t g = a.sg.seg_of[r0];
    const bool lo_cont = r0 > 0 && a.sg.seg_of[r0 - 1] == g;
    bool first = true;
    auto flush = [&](bool last_seg) {
      const bool cut_lo = first && lo_cont;
      const bool cut_hi = last_seg && r1 < a.n && a.sg.seg_of[r1] == g;
      if (on) {
        const float v0 = s0 - c0, v1 = s1 - c1;
        if (cut_lo || cut_hi) {
          *reinterpret_cast<float2*>(a.carry + (u * 2 + (cut_lo ? 0 : 1)) * h + col) = make_float2(v0, v1);
        } else {                                  // the row is written by this wave alone
          float2* dst = reinterpret_cast<float2*>(a.out + (int64_t)a.out_row[g] * h + col);
          const float2 o = *dst;
          *dst = make_float2(o.x + v0, o.y + v1);
        }
      }
      first = false;
      s0 = s1 = c0 = c1 = 0.f;
    };
    for (int64_t base = r0; base < r1; base += 64) {
      const int n = (int)min<int64_t>(64, r1 - base);
      const int64_t e = base + min(lane, n - 1);
      const int32_t gl = a.sg.seg_of[e];
      const int32_t G = a.grp_t[e];
      const int32_t T = a.own ? a.tau_t[e] : 0;
      // rows of the 64 positions, one vector per atom (compile-time atom
      // indices: a run-time index into the argument would go to scratch)
      int32_t R[RELNN_MAX_ATOMS];
#pragma unroll
      for (int i = 0; i < RELNN_MAX_ATOMS; ++i) R[i] = i < a.k ? a.rows_t[i][e] : 0;
      int32_t Rj = 0;                               // atom j's own row, read only for ReLU'
      const void* ej = a.emb[0];
#pragma unroll
      for (int i = 0; i < RELNN_MAX_ATOMS; ++i)
        if (i == a.j) {
          Rj = R[i];
          ej = a.emb[i];
        }
      for (int bt = 0; bt < n; bt += kPbBatch) {
        float2 v[kPbBatch];
#pragma unroll
        for (int b = 0; b < kPbBatch; ++b) {
          const int q = min(bt + b, n - 1);         // clamped: every load is valid
          const int32_t grp = __builtin_amdgcn_readlane(G, q);
          float2 d = *reinterpret_cast<const float2*>(a.dA + (int64_t)grp * h + cc);
          if (a.own) {                              // MAX: the columns this tuple maximises
            const int32_t tau = __builtin_amdgcn_readlane(T, q);
            const uint32_t bits = a.own[(int64_t)tau * a.own_w + (cc >> 5)] >> (cc & 31);
            d.x = (bits & 1u) ? d.x : 0.0f;
            d.y = (bits & 2u) ? d.y : 0.0f;
          }
          float2 others = make_float2(1.0f, 1.0f), mine = make_float2(1.0f, 1.0f);
#pragma unroll
          for (int i = 0; i < RELNN_MAX_ATOMS; ++i) {
            if (i < a.k && i != a.j) {
              const float2 z = row2<kBF16>(a.emb[i], __builtin_amdgcn_readlane(R[i], q), h, cc);
              others.x *= z.x;
              others.y *= z.y;
            }
          }
          if (a.act_pre == RELNN_ACT_RELU) {        // act_pre'(z_1 * ... * z_k), ReLU'(0) = 0
            mine = row2<kBF16>(ej, __builtin_amdgcn_readlane(Rj, q), h, cc);
            d.x = others.x * mine.x > 0.0f ? d.x : 0.0f;
            d.y = others.y * mine.y > 0.0f ? d.y : 0.0f;
          }
          v[b] = make_float2(d.x * others.x, d.y * others.y);
        }
#pragma unroll
        for (int b = 0; b < kPbBatch; ++b) {
          const int q = bt + b;
          if (q >= n) break;
          const int32_t gq = __builtin_amdgcn_readlane(gl, q);
          if (gq != g) {                            // a row ends
            flush(false);
            g = gq;
          }
          kahan_add(s0, c0, v[b].x);
          kahan_add(s1, c1, v[b].y);
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

int64_t pb_units(int64_t E) { return std::max<int64_t>(1, std::min<int64_t>(cdiv(std::max<int64_t>(E, 1), kPbTM), 8192)); }

}  // namespace

size_t prod_bwd_ws_bytes(const relnn_index* idx, const relnn_layer_desc* L) {
  const int64_t E = std::max<int64_t>(idx->E, 1);
  return round_up((size_t)E * 4 * (RELNN_MAX_ATOMS - 1), 256) + round_up((size_t)pb_units(idx->E) * 2 * L->h * 4, 256);
}

void prod_bwd(const relnn_index* idx, const relnn_layer_desc* L, const void* const* emb, const float* dA,
              const uint32_t* own, int own_w, float* const* demb, char* ws, hipStream_t s) {
  const int64_t E = idx->E;
  const int h = L->h;
  RELNN_REQUIRE(h % 2 == 0, RELNN_E_UNSUPPORTED, "the product backward needs an even h");
  int32_t* other_rows = reinterpret_cast<int32_t*>(ws);                 // [k - 1][E]
  float* carry = reinterpret_cast<float*>(ws + round_up((size_t)std::max<int64_t>(E, 1) * 4 * (RELNN_MAX_ATOMS - 1),
                                                        256));
  const unsigned gE = (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(E, 256), 1 << 16));
  for (int j = 0; j < L->k; ++j) {
    if (idx->t_nseg[j] == 0) continue;
    ProdBwdArgs a{};
    a.k = L->k;
    a.j = j;
    for (int i = 0, slot = 0; i < L->k; ++i) {
      a.emb[i] = emb[i];
      if (i == j) {
        a.rows_t[i] = idx->t_row[j];                                    // the row itself
      } else {                                                          // atom i's row of each tuple, in j's order
        int32_t* dst = other_rows + (int64_t)(slot++) * E;
        k_gather_idx<<<gE, 256, 0, s>>>(idx->t_pos[j], idx->rows + (int64_t)i * E, E, dst);
        RELNN_LAUNCHED();
        a.rows_t[i] = dst;
      }
    }
    a.grp_t = idx->t_grp[j];
    a.tau_t = idx->t_pos[j];
    a.dA = dA;
    a.own = own;
    a.own_w = own_w;
    a.act_pre = L->act_pre;
    a.h = h;
    a.n = E;
    a.sg = Seg{idx->t_seg[j], idx->t_segoff[j], E, nullptr};
    a.out_row = idx->t_segrow[j];
    a.out = demb[j];
    a.carry = carry;
    a.ntiles = cdiv(E, kPbTM);
    a.nunits = pb_units(E);
    KTimer tm("bwd_dx", s);
    if (L->dtype == RELNN_BF16)
      k_prod_bwd<true><<<(unsigned)cdiv(a.nunits, kPbWaves), kPbWaves * 64, 0, s>>>(a);
    else
      k_prod_bwd<false><<<(unsigned)cdiv(a.nunits, kPbWaves), kPbWaves * 64, 0, s>>>(a);
    RELNN_LAUNCHED();
    Sink sk{};
    sk.agg = RELNN_SUM;
    sk.act_post = RELNN_ACT_NONE;
    sk.out = demb[j];
    sk.out_row = idx->t_segrow[j];
    sk.accumulate = true;
    launch_fixup(a.sg, kPbTM, h, a.ntiles, a.nunits, sk, carry, nullptr, s);
  }
}

}  // namespace relnn
