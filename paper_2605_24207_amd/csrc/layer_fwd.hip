// Forward of one relational layer: join -> transformation -> projected union.
//
//   y_tau = act_pre(x_tau W + b),  x_tau = z_1[r_1] (+) ... (+) z_k[r_k]
//   pre_g = alpha over the tuples of group g of y_tau,  out_g = act_post(pre_g)
//
// (join and its concatenated embedding, transformation applied per tuple,
// projected union with SUM / MEAN / MAX applied once: Section 2.2; their
// composition by a join rule: Section 3.1.)
//
// Fused path: one kernel per tile of TM tuples gathers the joined rows
// into LDS with 16-byte coalesced loads, multiplies them on the matrix cores
// (bf16 16x16x32 or f32 16x16x4, FP32 accumulation), keeps the FP32 result
// tile in LDS and reduces it per group; nothing of size [E, .] reaches HBM.
// Plain path (plain.hip): the same steps as a gather kernel, a library
// GEMM and a segmented-reduce kernel that materialise X = [E, K] and
// Y = [E, h] in HBM, the shape of a library pipeline (index_select + cat
// -> Linear -> scatter).
#include "layer_common.hpp"
#include "gemm.hpp"
#include "layer_fwd.hpp"

namespace relnn {

__global__ void k_swizzle_bf16(const __bf16* __restrict__ W, int K, int Kp, int h, __bf16* __restrict__ Wsw) {
  const int ncb = h / 16;
  const int64_t total = (int64_t)Kp * h;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    // i enumerates (ks, cb, lane, e) in Wsw order
    const int e = (int)(i & 7);
    const int64_t f = i >> 3;
    const int lane = (int)(f & 63);
    const int64_t kc = f >> 6;
    const int cb = (int)(kc % ncb);
    const int ks = (int)(kc / ncb);
    const int k = ks * 32 + (lane >> 4) * 8 + e;
    const int n = cb * 16 + (lane & 15);
    Wsw[i] = k < K ? W[(int64_t)k * h + n] : (__bf16)0.0f;
  }
}

__global__ void k_swizzle_f32(const float* __restrict__ W, int K, int Kp, int h, float* __restrict__ Wsw) {
  const int ncb = h / 16;
  const int64_t total = (int64_t)Kp * h;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int lane = (int)(i & 63);
    const int64_t kc = i >> 6;
    const int cb = (int)(kc % ncb);
    const int ks = (int)(kc / ncb);
    const int k = ks * 4 + (lane >> 4);
    const int n = cb * 16 + (lane & 15);
    Wsw[i] = k < K ? W[(int64_t)k * h + n] : 0.0f;
  }
}

// Copies the joined rows of tuples e0..e0+nv-1 into Xs [TM][XS] (T), in
// Concat order, zero-filling the K..Kp pad and rows past nv.
template <class T>
__device__ __forceinline__ void gather_rows(const Atoms& at, const int32_t* __restrict__ rows, int64_t E,
                                            int64_t e0, int nv, int TM, int K, int Kp, T* Xs, int XS,
                                            const int32_t* rowidx) {
  constexpr int EPC = Mfma<T>::EPC;
  const int cpr = Kp / EPC;
  for (int i = threadIdx.x; i < TM * cpr; i += blockDim.x) {
    const int r = i / cpr;
    const int c = i - r * cpr;
    const int el = c * EPC;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (r < nv && el < K) {
      int j = 0;
#pragma unroll
      for (int q = 1; q < kMaxAtoms; ++q)
        if (q < at.k && el >= at.koff[q]) j = q;
      const int64_t row = rowidx[j * TM + r];
      const T* src = static_cast<const T*>(at.emb[j]) + row * at.d[j] + (el - at.koff[j]);
      v = *reinterpret_cast<const uint4*>(src);
    }
    *reinterpret_cast<uint4*>(Xs + r * XS + el) = v;
  }
}

// Combines the carry partials of segments cut by unit boundaries.  A unit
// is a run of tiles: unit u covers list positions [pos(u), pos(u+1)) with
// pos(u) = ((ntiles * u) / nunits) * TM (one tile per unit when nunits =
// ntiles).  A unit leaves, per column, a partial in slot 0 for the segment
// cut by its start and in slot 1 for the segment that starts inside it and
// runs past its end.  Block b (b >= 1) handles the segment containing
// pos(b) if it also contains pos(b) - 1 and starts at or after pos(b - 1):
// its partials are slot 1 of unit b-1 followed by slot 0 of the units that
// follow, summed in unit order (runs of 64 per strand, Kahan-compensated
// across runs, strands in order) so the result is deterministic.
__global__ void __launch_bounds__(kThreads) k_fixup(Seg sg, int64_t ntiles, int64_t nunits, int TM, int h,
                                                    Sink sink, const float* carry, const int32_t* carry_arg) {
  const int64_t b = (int64_t)blockIdx.x + 1;
  if (sg.n_dev) {                  // run-time size: the forward kernels used min(units, tiles) units
    sg.n = *sg.n_dev;
    ntiles = (sg.n + TM - 1) / TM;
    nunits = max<int64_t>(1, min<int64_t>(nunits, ntiles));
    if (b >= nunits) return;
  }
  auto pos = [&](int64_t u) { return ((ntiles * u) / nunits) * TM; };
  const int64_t e = pos(b);
  if (e <= 0 || e >= sg.n) return;
  const int64_t s = sg.seg_of[e];
  if (sg.seg_of[e - 1] != s) return;
  const int64_t g0 = sg.offsets[s], g1 = sg.offsets[s + 1];
  if (g0 < pos(b - 1)) return;
  int64_t ulast = b;                       // last unit holding part of s
  {
    int64_t lo = b, hi = nunits - 1;       // largest u with pos(u) < g1
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (pos(mid) < g1) lo = mid; else hi = mid - 1;
    }
    ulast = lo;
  }
  const int64_t P = ulast - (b - 1) + 1;   // partials: unit b-1 (slot 1), units b..ulast (slot 0)
  auto at = [&](int64_t i) { return ((b - 1 + i) * 2 + (i == 0 ? 1 : 0)) * h; };
  const int CG = min(h, kThreads);
  const int S = kThreads / CG;
  const int strand = threadIdx.x / CG;
  __shared__ float red_v[kThreads];
  __shared__ int32_t red_a[kThreads];
  for (int cbase = 0; cbase < h; cbase += CG) {
    const int c = cbase + (threadIdx.x % CG);
    const bool active = strand < S && c < h;
    float v = 0.0f, comp = 0.0f;
    int32_t am = -1;
    if (active) {
      const int64_t lo = (P * strand) / S, hi = (P * (strand + 1)) / S;
      // a hot segment spans many units: the partials are loaded eight at a
      // time (clamped to the strand's last), then combined in unit order
      constexpr int kFB = 8;
      if (sink.agg == RELNN_MAX) {
        v = -INFINITY;
        for (int64_t i0 = lo; i0 < hi; i0 += kFB) {
          float x[kFB];
          int32_t xa[kFB];
#pragma unroll
          for (int j = 0; j < kFB; ++j) {
            const int64_t i = min(i0 + j, hi - 1);
            x[j] = carry[at(i) + c];
            xa[j] = carry_arg[at(i) + c];
          }
#pragma unroll
          for (int j = 0; j < kFB; ++j) {
            if (i0 + j >= hi) break;
            if (x[j] > v || am < 0) {
              v = x[j];
              am = xa[j];
            }
          }
        }
      } else {
        for (int64_t i0 = lo; i0 < hi; i0 += 64) {
          float inner = 0.0f;
          const int64_t i1 = min(hi, i0 + 64);
          for (int64_t ib = i0; ib < i1; ib += kFB) {
            float x[kFB];
#pragma unroll
            for (int j = 0; j < kFB; ++j) x[j] = carry[at(min(ib + j, i1 - 1)) + c];
#pragma unroll
            for (int j = 0; j < kFB; ++j)
              if (ib + j < i1) inner += x[j];
          }
          const float y = inner - comp;
          const float tt = v + y;
          comp = __builtin_isfinite(tt) ? (tt - v) - y : 0.0f;   // an infinite sum stays infinite
          v = tt;
        }
      }
    }
    red_v[threadIdx.x] = v - comp;
    red_a[threadIdx.x] = am;
    __syncthreads();
    if (strand == 0 && c < h) {
      float acc = red_v[threadIdx.x];
      int32_t aa = red_a[threadIdx.x];
      for (int q = 1; q < S; ++q) {
        const float x = red_v[q * CG + threadIdx.x];
        const int32_t xa = red_a[q * CG + threadIdx.x];
        if (sink.agg == RELNN_MAX) {
          if (xa >= 0 && (aa < 0 || x > acc)) {
            acc = x;
            aa = xa;
          }
        } else {
          acc += x;
        }
      }
      sink_write(sink, s, c, h, acc, aa, (int32_t)(g1 - g0));
    }
    __syncthreads();
  }
}


enum { MODE_FUSED = 0, MODE_MASK = 3 };

// One tile of TM tuples per block.
template <class T, int MODE>
__global__ void __launch_bounds__(kThreads) k_layer_fwd(FwdArgs a) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int TM = a.TM;
  const int64_t tile = blockIdx.x;
  const int64_t e0 = tile * TM;
  const int nv = (int)min<int64_t>(TM, a.E - e0);
  const int XS = a.Kp + Mfma<T>::XPAD;
  const int YS = a.h + 4;
  int32_t* rowidx = reinterpret_cast<int32_t*>(smem);
  T* Xs = reinterpret_cast<T*>(smem + a.off_x);
  float* Ys = reinterpret_cast<float*>(smem + a.off_y);
  const int ncb = a.h / 16;
  const int nblk = (TM / 16) * ncb;

  if constexpr (MODE == MODE_FUSED || MODE == MODE_MASK) {
    for (int i = threadIdx.x; i < a.at.k * TM; i += blockDim.x) {
      const int j = i / TM, r = i - (i / TM) * TM;
      rowidx[i] = r < nv ? a.at.rows[j][e0 + r] : 0;
    }
    __syncthreads();
    gather_rows<T>(a.at, a.rows, a.E, e0, nv, TM, a.K, a.Kp, Xs, XS, rowidx);
  }
  {
    __syncthreads();
    f32x4 acc[kMaxQ];
    mfma_tile<T>(Xs, XS, a.Kp, nblk, ncb, static_cast<const T*>(a.Wsw), acc);
    if constexpr (MODE == MODE_MASK) {
      // one bit per tuple and column: lanes 16 g .. 16 g + 15 hold the 16
      // columns of column block cb for row 4 g + i of the row block, so one
      // ballot gives four 16-bit halves of the rows' bit words
      const int lane = __lane_id();
      const int w = threadIdx.x / 64;
      const int nhalf = 2 * (int)((a.h + 31) / 32);
      uint16_t* bits = reinterpret_cast<uint16_t*>(a.mask);
#pragma unroll
      for (int qi = 0; qi < kMaxQ; ++qi) {
        const int q = w + 4 * qi;
        if (q < nblk) {
          const int rb = q / ncb, cb = q - (q / ncb) * ncb;
          const int col = cb * 16 + (lane & 15);
          const float bv = a.b ? a.b[col] : 0.0f;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const uint64_t bal = __ballot((acc[qi][i] + bv) > 0.0f);
            const int row = rb * 16 + (lane >> 4) * 4 + i;
            if ((lane & 15) == 0 && row < nv)
              bits[(e0 + row) * nhalf + cb] = (uint16_t)(bal >> (lane & 48));
          }
        }
      }
      return;
    } else {
      store_acc(acc, nblk, ncb, a.b, a.act_pre, Ys, YS);
    }
  }
  __syncthreads();
  reduce_tile(Ys, YS, a.h, e0, nv, tile, a.sg, a.sink, a.carry, a.carry_arg);
}

// Plain gather: X[e] = concat of the joined rows, Kp columns (pad zero).
// A block moves 8 rows per pass, 32 threads per row, each thread the
// 16-byte chunks c, c + 32, .. of its row: 512 contiguous bytes per row and
// instruction, and no per-chunk 64-bit division (which made a one-chunk-
// per-thread mapping spend a quarter of its time on index arithmetic).
template <class T>
__global__ void __launch_bounds__(256) k_gather_plain(Atoms at, const int32_t* __restrict__ rows, int64_t E, int K,
                                                      int Kp, T* __restrict__ X) {
  constexpr int EPC = Mfma<T>::EPC;
  const int cpr = Kp / EPC;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  for (int64_t e = (int64_t)blockIdx.x * 8 + ty; e < E; e += (int64_t)gridDim.x * 8) {
    int32_t r[kMaxAtoms];
#pragma unroll
    for (int j = 0; j < kMaxAtoms; ++j) r[j] = j < at.k ? at.rows[j][e] : 0;
    for (int c = tx; c < cpr; c += 32) {
      const int el = c * EPC;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (el < K) {
        int j = 0;
#pragma unroll
        for (int q = 1; q < kMaxAtoms; ++q)
          if (q < at.k && el >= at.koff[q]) j = q;
        int32_t row = r[0];
#pragma unroll
        for (int q = 1; q < kMaxAtoms; ++q) row = j == q ? r[q] : row;
        v = *reinterpret_cast<const uint4*>(static_cast<const T*>(at.emb[j]) + (int64_t)row * at.d[j] +
                                            (el - at.koff[j]));
      }
      // X is written once and read back by the GEMM from HBM: non-temporal
      // stores keep it from evicting the cached embedding rows
      const u32x4 w = {v.x, v.y, v.z, v.w};
      __builtin_nontemporal_store(w, reinterpret_cast<u32x4*>(X + e * Kp + el));
    }
  }
}

// ---------------------------------------------------------------- host
namespace {

unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 1 << 20));
}

template <class KernelT>
void allow_lds(KernelT k, size_t bytes) {
  RELNN_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

template <class T>
void launch_fwd_t(const FwdPlan& P, FwdArgs a, bool plain, hipStream_t s) {
  const int64_t ntiles = P.ntiles;
  if (plain) {
    {
      KTimer t("fwd_gather", s);
      k_gather_plain<T><<<grid_for(a.E * 32), 256, 0, s>>>(
          a.at, a.rows, a.E, a.K, a.Kp, static_cast<T*>(const_cast<void*>(a.X)));
      RELNN_LAUNCHED();
    }
    {
      KTimer t("fwd_gemm", s);
      plain_gemm(std::is_same<T, __bf16>::value ? RELNN_BF16 : RELNN_F32, a.X, a.E, a.K, a.Kp, a.W, a.h, a.Y, s);
    }
    launch_seg_reduce(a.Y, a.E, a.h, a.sg, a.b, a.act_pre, a.sink, a.carry, a.carry_arg, P.carry_units, s);
    return;
  }
  allow_lds(k_layer_fwd<T, MODE_FUSED>, P.lds);
  {
    KTimer t("fwd_fused", s);
    k_layer_fwd<T, MODE_FUSED><<<(unsigned)ntiles, kThreads, P.lds, s>>>(a);
    RELNN_LAUNCHED();
  }
  launch_fixup(a.sg, a.TM, a.h, ntiles, ntiles, a.sink, a.carry, a.carry_arg, s);
}

}  // namespace

void launch_fixup(const Seg& sg, int TM, int h, int64_t ntiles, int64_t nunits, const Sink& sink,
                  const float* carry, const int32_t* carry_arg, hipStream_t s) {
  if (nunits <= 1) return;
  k_fixup<<<(unsigned)(nunits - 1), kThreads, 0, s>>>(sg, ntiles, nunits, TM, h, sink, carry, carry_arg);
  RELNN_LAUNCHED();
}

FwdPlan plan_fwd(const relnn_index* idx, const relnn_layer_desc* L) {
  FwdPlan P;
  const bool bf = L->dtype == RELNN_BF16;
  const int esz = bf ? 2 : 4;
  const int KS = bf ? 32 : 4;
  const int XPAD = bf ? 8 : 4;
  int K = 0;
  for (int j = 0; j < L->k; ++j) K += L->d[j];
  P.K = K;
  P.Kp = (int)round_up(K, KS);
  const int h = L->h;
  P.TM = 0;
  for (int TM : {64, 32, 16}) {
    if ((TM / 16) * (h / 16) > 4 * kMaxQ) continue;
    const size_t rowidx = (size_t)kMaxAtoms * TM * 4;
    const size_t xs = (size_t)TM * (P.Kp + XPAD) * esz;
    const size_t ys = (size_t)TM * (h + 4) * 4;
    const size_t lds = round_up(rowidx, 16) + round_up(xs, 16) + ys;
    if (lds <= 160 * 1024) {
      P.TM = TM;
      P.off_x = round_up(rowidx, 16);
      P.off_y = P.off_x + round_up(xs, 16);
      P.lds = lds;
      break;
    }
  }
  const int64_t E = idx->E;
  P.ntiles = P.TM ? cdiv(E, P.TM) : 0;
  // carry partials: one pair per unit of the forward kernel that runs (the
  // plain path's segmented reduce; else the persistent fused kernel where it
  // covers the shape, the tile kernel otherwise)
  const WsPlan wp = plan_ws(L->dtype, K, h, E);
  const bool plain = (L->flags & RELNN_PLAIN) != 0;
  const bool prod = (L->flags & RELNN_TF_PRODUCT) != 0;
  P.carry_units = std::max<int64_t>(1, prod ? push_units(E) : plain ? seg_reduce_units(E) : wp.KP ? wp.nunits
                                                                                               : P.ntiles);
  // the weight as the kernel that runs reads it (the plain path reads W as
  // given, the product transform has none)
  const size_t wsw = (plain || prod) ? 0 : wp.KP ? wp.wsw_bytes : (size_t)P.Kp * h * esz;
  size_t off = 0;
  P.ws_wsw = off;
  off += round_up(wsw, 256);
  P.ws_carry = off;
  off += round_up(P.carry_units * 2 * h * 4, 256);
  P.ws_carry_arg = off;
  if (L->agg == RELNN_MAX) off += round_up(P.carry_units * 2 * h * 4, 256);
  P.ws_fused = off;
  P.ws_x = off;
  off += round_up(std::max<int64_t>(E, 1) * P.Kp * esz, 256);
  P.ws_y = off;
  off += round_up(std::max<int64_t>(E, 1) * h * 4, 256);
  P.ws_plain = off;
  if (L->flags & RELNN_PUSHDOWN) {        // node products, W slices, carry of the gather-reduce
    size_t o = 0;
    for (int j = 0; j < L->k; ++j) {
      P.ws_push_p[j] = o;
      o += round_up(std::max<int64_t>(idx->n_rows[j], 1) * h * 4, 256);
    }
    P.carry_units = std::max<int64_t>(P.carry_units, push_units(E));
    P.ws_carry = o;
    o += round_up(P.carry_units * 2 * h * 4, 256);
    P.ws_carry_arg = o;
    if (L->agg == RELNN_MAX) o += round_up(P.carry_units * 2 * h * 4, 256);
    P.ws_push_v = o;
    o += round_up(std::max<int64_t>(idx->G, 1) * h * 4, 256);
    P.ws_push = o;
  }
  return P;
}

void check_layer_args(const relnn_index* idx, const relnn_layer_desc* L) {
  RELNN_REQUIRE(idx != nullptr && L != nullptr, RELNN_E_INVALID, "index or layer descriptor is NULL");
  RELNN_REQUIRE(L->k == idx->k, RELNN_E_INVALID, "layer has %d atoms, index has %d", L->k, idx->k);
  RELNN_REQUIRE(L->d != nullptr, RELNN_E_INVALID, "layer widths are NULL");
  RELNN_REQUIRE(L->dtype == RELNN_F32 || L->dtype == RELNN_BF16, RELNN_E_INVALID, "unknown dtype");
  RELNN_REQUIRE(L->agg >= RELNN_SUM && L->agg <= RELNN_MAX, RELNN_E_INVALID, "unknown aggregate");
  RELNN_REQUIRE((L->act_pre == RELNN_ACT_NONE || L->act_pre == RELNN_ACT_RELU) &&
                    (L->act_post == RELNN_ACT_NONE || L->act_post == RELNN_ACT_RELU),
                RELNN_E_INVALID, "unknown activation");
  RELNN_REQUIRE((L->flags & ~(RELNN_PLAIN | RELNN_DW_ACCUM | RELNN_OUT_BF16 | RELNN_PUSHDOWN | RELNN_TF_PRODUCT)) == 0,
                RELNN_E_INVALID, "unknown layer flags");
  if (L->flags & RELNN_TF_PRODUCT) {
    RELNN_REQUIRE(!(L->flags & (RELNN_PLAIN | RELNN_PUSHDOWN)), RELNN_E_INVALID,
                  "RELNN_TF_PRODUCT excludes RELNN_PLAIN and RELNN_PUSHDOWN");
    for (int j = 0; j < L->k; ++j)
      RELNN_REQUIRE(L->d[j] == L->h, RELNN_E_INVALID, "the product transform needs d[%d] == h", j);
  }
  RELNN_REQUIRE(L->h > 0, RELNN_E_INVALID, "h must be positive");
  const int epc = L->dtype == RELNN_BF16 ? 8 : 4;
  for (int j = 0; j < L->k; ++j) {
    RELNN_REQUIRE(L->d[j] > 0, RELNN_E_INVALID, "d[%d] must be positive", j);
    RELNN_REQUIRE(L->d[j] % epc == 0, RELNN_E_UNSUPPORTED,
                  "d[%d] = %d: rows must be a multiple of 16 bytes", j, L->d[j]);
  }
  RELNN_REQUIRE(L->h % 16 == 0, RELNN_E_UNSUPPORTED, "h = %d must be a multiple of 16", L->h);
}

FwdPlan checked_plan(const relnn_index* idx, const relnn_layer_desc* L) {
  check_layer_args(idx, L);
  FwdPlan P = plan_fwd(idx, L);
  RELNN_REQUIRE(P.TM > 0 || (L->flags & RELNN_TF_PRODUCT), RELNN_E_UNSUPPORTED,
                "K = %d, h = %d does not fit the LDS tile", P.K, L->h);
  return P;
}

Atoms make_atoms(const relnn_layer_desc* L, const void* const* emb, const relnn_index* idx) {
  Atoms at{};
  at.k = L->k;
  int off = 0;
  for (int j = 0; j < L->k; ++j) {
    at.emb[j] = emb[j];
    at.rows[j] = idx ? idx->rows + (int64_t)j * idx->E : nullptr;
    at.d[j] = L->d[j];
    at.koff[j] = off;
    off += L->d[j];
  }
  return at;
}

void swizzle_w(const void* W, int dtype, int K, int Kp, int h, void* Wsw, hipStream_t s) {
  if (dtype == RELNN_BF16)
    k_swizzle_bf16<<<grid_for((int64_t)Kp * h), 256, 0, s>>>(static_cast<const __bf16*>(W), K, Kp, h,
                                                              static_cast<__bf16*>(Wsw));
  else
    k_swizzle_f32<<<grid_for((int64_t)Kp * h), 256, 0, s>>>(static_cast<const float*>(W), K, Kp, h,
                                                             static_cast<float*>(Wsw));
  RELNN_LAUNCHED();
}

template <class T>
void launch_mask_t(const FwdPlan& P, const FwdArgs& a, hipStream_t s) {
  allow_lds(k_layer_fwd<T, MODE_MASK>, P.lds);
  k_layer_fwd<T, MODE_MASK><<<(unsigned)P.ntiles, kThreads, P.lds, s>>>(a);
  RELNN_LAUNCHED();
}

void launch_mask(const FwdPlan& P, const FwdArgs& a, int dtype, hipStream_t s) {
  if (dtype == RELNN_BF16)
    launch_mask_t<__bf16>(P, a, s);
  else
    launch_mask_t<float>(P, a, s);
}

void launch_fwd(const FwdPlan& P, const FwdArgs& a, int dtype, bool plain, hipStream_t s) {
  if (dtype == RELNN_BF16)
    launch_fwd_t<__bf16>(P, a, plain, s);
  else
    launch_fwd_t<float>(P, a, plain, s);
}

}  // namespace relnn

using namespace relnn;

extern "C" relnn_status relnn_workspace_size(const relnn_index* idx, const relnn_layer_desc* L, int bwd,
                                             size_t* bytes) {
  return guard([&] {
    RELNN_REQUIRE(bytes != nullptr, RELNN_E_INVALID, "bytes is NULL");
    FwdPlan P = checked_plan(idx, L);
    if (bwd) {
      *bytes = bwd_workspace(idx, L, P);
    } else {
      *bytes = (L->flags & RELNN_PUSHDOWN) ? P.ws_push : (L->flags & RELNN_PLAIN) ? P.ws_plain : P.ws_fused;
    }
  });
}

namespace relnn {

size_t layer_fwd_ws_bytes(const relnn_index* idx, const relnn_layer_desc* L) {
  const FwdPlan P = checked_plan(idx, L);
  return (L->flags & RELNN_PUSHDOWN) ? P.ws_push : (L->flags & RELNN_PLAIN) ? P.ws_plain : P.ws_fused;
}

void layer_fwd_run(const relnn_index* idx, const relnn_layer_desc* L, const void* const* emb, const void* W,
                   const float* b, float* out, float* pre, int32_t* argmax, void* ws, size_t ws_bytes,
                   hipStream_t stream) {
  {
    FwdPlan P = checked_plan(idx, L);
    const bool plain = (L->flags & RELNN_PLAIN) != 0;
    const bool push = (L->flags & RELNN_PUSHDOWN) != 0;
    RELNN_REQUIRE(!(plain && push), RELNN_E_INVALID, "RELNN_PLAIN and RELNN_PUSHDOWN exclude each other");
    if (push) {
      RELNN_REQUIRE(L->act_pre == RELNN_ACT_NONE, RELNN_E_INVALID,
                    "RELNN_PUSHDOWN needs an affine transform (act_pre = NONE)");
      const int ks = L->dtype == RELNN_BF16 ? 32 : 4;
      for (int j = 0; j < L->k; ++j)
        RELNN_REQUIRE(L->d[j] % ks == 0, RELNN_E_UNSUPPORTED, "RELNN_PUSHDOWN needs d[%d] %% %d == 0", j, ks);
      RELNN_REQUIRE(L->h % 4 == 0 && L->h <= 128, RELNN_E_UNSUPPORTED, "RELNN_PUSHDOWN needs h %% 4 == 0, h <= 128");
    }
    const size_t need = push ? P.ws_push : plain ? P.ws_plain : P.ws_fused;
    RELNN_REQUIRE(emb != nullptr, RELNN_E_INVALID, "emb is NULL");
    for (int j = 0; j < L->k; ++j) {
      RELNN_REQUIRE(emb[j] != nullptr || idx->n_rows[j] == 0, RELNN_E_INVALID, "emb[%d] is NULL", j);
      RELNN_REQUIRE(((uintptr_t)emb[j] & 15) == 0, RELNN_E_UNSUPPORTED, "emb[%d] is not 16-byte aligned", j);
    }
    const bool prod = (L->flags & RELNN_TF_PRODUCT) != 0;
    RELNN_REQUIRE(W != nullptr || prod, RELNN_E_INVALID, "W is NULL");
    RELNN_REQUIRE(out != nullptr || idx->G == 0, RELNN_E_INVALID, "out is NULL");
    RELNN_REQUIRE(ws != nullptr && ws_bytes >= need, RELNN_E_INVALID,
                  "workspace of %zu bytes given, %zu needed", ws_bytes, need);
    RELNN_REQUIRE(((uintptr_t)ws & 255) == 0, RELNN_E_INVALID, "workspace must be 256-byte aligned");
    if (idx->E == 0) return;
    hipStream_t s = (hipStream_t)stream;
    char* w = static_cast<char*>(ws);
    FwdArgs a{};
    a.at = make_atoms(L, emb, idx);
    a.rows = idx->rows;
    a.E = idx->E;
    a.K = P.K;
    a.Kp = P.Kp;
    a.h = L->h;
    a.TM = P.TM;
    a.off_x = (int)P.off_x;
    a.off_y = (int)P.off_y;
    a.Wsw = w + P.ws_wsw;
    a.W = W;
    a.b = b;
    a.act_pre = L->act_pre;
    a.sg = Seg{idx->tuple_group, idx->offsets, idx->E, nullptr};
    a.sink = Sink{L->agg, L->act_post, out, pre, argmax, false, nullptr, (L->flags & RELNN_OUT_BF16) != 0};
    a.carry = reinterpret_cast<float*>(w + P.ws_carry);
    a.carry_arg = L->agg == RELNN_MAX ? reinterpret_cast<int32_t*>(w + P.ws_carry_arg) : nullptr;
    a.X = w + P.ws_x;
    a.Y = reinterpret_cast<float*>(w + P.ws_y);
    if (prod) {                         // tau = z_1 * ... * z_k, elementwise
      launch_product(a, L->dtype == RELNN_BF16, P.carry_units, a.carry, a.carry_arg, s);
      return;
    }
    if (push) {
      // node products P_j = Z_j W_j, once per atom row
      const int esz = L->dtype == RELNN_BF16 ? 2 : 4;
      const float* Pj[kMaxAtoms];
      for (int j = 0, koff = 0; j < L->k; koff += L->d[j], ++j) {
        Pj[j] = reinterpret_cast<const float*>(w + P.ws_push_p[j]);
        KTimer t("node_gemm", s);
        const bool bf16 = L->dtype == RELNN_BF16;
        gemm_rows(bf16, emb[j], bf16, L->d[j], idx->n_rows[j], L->d[j],
                  static_cast<const char*>(W) + (size_t)koff * L->h * esz, bf16, false, L->h, L->h,
                  const_cast<float*>(Pj[j]), L->h, RowsEpi{}, s);
      }
      // atoms varying inside a group are gathered per tuple; the others
      // (and the bias) are one constant per group
      const float* gp[kMaxAtoms];
      const int32_t* gr[kMaxAtoms];
      int n = 0;
      Sink sk = a.sink;
      sk.gc = GroupConst{};
      sk.gc.offsets = idx->offsets;
      sk.gc.bias = b;
      for (int j = 0; j < L->k; ++j) {
        const int32_t* rj = idx->rows + (int64_t)j * idx->E;
        if (idx->atom_fd[j]) {
          sk.gc.P[sk.gc.n] = Pj[j];
          sk.gc.rows[sk.gc.n] = rj;
          ++sk.gc.n;
        } else {
          gp[n] = Pj[j];
          gr[n] = rj;
          ++n;
        }
      }
      a.sink = sk;
      a.carry = reinterpret_cast<float*>(w + P.ws_carry);
      a.carry_arg = L->agg == RELNN_MAX ? reinterpret_cast<int32_t*>(w + P.ws_carry_arg) : nullptr;
      launch_push(a, push_units(idx->E), n, gp, gr, a.carry, a.carry_arg, idx->G,
                  reinterpret_cast<float*>(w + P.ws_push_v), s);
      return;
    }
    const WsPlan wp = plan_ws(L->dtype, P.K, L->h, idx->E);
    if (!plain && wp.KP) {
      RELNN_REQUIRE(wp.nunits <= P.carry_units && wp.wsw_bytes <= P.ws_carry - P.ws_wsw, RELNN_E_HIP,
                    "internal: workspace plan does not cover the launch");
      swizzle_ws(W, L->dtype, P.K, wp.KP, L->h, w + P.ws_wsw, s);
      launch_ws(wp, L->dtype, a, w + P.ws_wsw, a.carry, a.carry_arg, s);
      return;
    }
    if (!plain) {
      RELNN_REQUIRE(P.ntiles <= P.carry_units && (size_t)P.Kp * L->h * (L->dtype == RELNN_BF16 ? 2 : 4) <=
                                                     P.ws_carry - P.ws_wsw,
                    RELNN_E_HIP, "internal: workspace plan does not cover the launch");
      swizzle_w(W, L->dtype, P.K, P.Kp, L->h, w + P.ws_wsw, s);
    }
    launch_fwd(P, a, L->dtype, plain, s);
  }
}

}  // namespace relnn

extern "C" relnn_status relnn_layer_fwd(const relnn_index* idx, const relnn_layer_desc* L,
                                        const void* const* emb, const void* W, const float* b, float* out,
                                        float* pre, int32_t* argmax, void* ws, size_t ws_bytes,
                                        relnn_stream_t stream) {
  return guard([&] { layer_fwd_run(idx, L, emb, W, b, out, pre, argmax, ws, ws_bytes, (hipStream_t)stream); });
}
