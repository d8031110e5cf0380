// Hand-written matrix-core products of the backward and of the pushed-down
// transform (gfx950).
//
//   gemm_rows  C[dst(m)] (+)= s_m A[m] B over many rows m, with a small B (a
//              slice of a layer's W, or its transpose) that every block lays
//              into LDS once, in MFMA fragment order, and keeps for all of its
//              row tiles.  Each wave multiplies 16 rows: their A values come
//              straight from global memory into registers (16 bytes per lane,
//              the next 64-wide k chunk in flight while the current one is
//              multiplied), B fragments are read from LDS.  The epilogue adds
//              the result into the rows the caller names (the joined
//              embedding rows of a transpose segment, or the one row a group
//              joins, scaled by the group's size) or stores it.
//   gemm_tn    D = sum_m A(m)^T B[m] over many rows m (A rows optionally
//              gathered through a row list), split over contiguous chunks of
//              m.  A block stages 32 (FP32) or 64 (bf16) rows of A and B
//              transposed in LDS (double-buffered, the loads of the next tile
//              in flight during the products), multiplies a 128 x 128 output
//              block (8 waves x 16 rows x 8 column blocks), and writes its
//              partial; the partials are then added in chunk order.
//
// FP32 products use v_mfma_f32_16x16x4_f32.  bf16 products use
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation; FP32 operands are rounded
// to nearest even when they are loaded.  Operand layouts: a lane of the
// 16x16x4 instruction holds A[l % 16][l / 16] and B[l / 16][l % 16]; of the
// 16x16x32 one, A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16],
// e = 0..7; the result lane holds C[4 (l / 16) + r][l % 16], r = 0..3.
#include <type_traits>

#include "gemm.hpp"

namespace relnn {

namespace {

constexpr int kRowsWaves = 8;
constexpr int kRowsTM = 16 * kRowsWaves;     // rows per tile of gemm_rows
constexpr int kKC = 64;                      // k per register chunk
constexpr int kSlabBytes = 64 * 1024;        // B fragments per block (two blocks per CU)

constexpr int kTnThreads = 512;              // gemm_tn: 8 waves, a 128 x 128 output block
constexpr int kTnTarget = 512;               // blocks gemm_tn aims for (two per CU)

__device__ __forceinline__ f32x4 bf4_f32(uint32_t x, uint32_t y) {
  return f32x4{__uint_as_float(x << 16), __uint_as_float(x & 0xffff0000u), __uint_as_float(y << 16),
               __uint_as_float(y & 0xffff0000u)};
}

__device__ __forceinline__ bf16x8 f32_bf8(const f32x4& lo, const f32x4& hi) {
  bf16x8 r;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    r[e] = (__bf16)lo[e];
    r[e + 4] = (__bf16)hi[e];
  }
  return r;
}

int cu_count() {
  static int cache[64] = {};
  int dev = 0;
  RELNN_HIP(hipGetDevice(&dev));
  int& n = cache[dev & 63];
  if (!n) RELNN_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
  return n;
}

template <class KernelT>
void allow_lds(KernelT k, size_t bytes) {
  RELNN_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)bytes));
}

// ------------------------------------------------------------- gemm_rows
struct RowsArgs {
  const void* A;
  int64_t lda, M;
  int Kd, KP, N;
  const void* B;
  int64_t ldb;
  int b_bf16, b_trans;
  float* C;
  int64_t ldc;
  RowsEpi epi;
  int64_t ntiles;
};

__device__ __forceinline__ float b_elem(const RowsArgs& a, int k, int n) {
  if (k >= a.Kd || n >= a.N) return 0.0f;
  const int64_t o = a.b_trans ? (int64_t)n * a.ldb + k : (int64_t)k * a.ldb + n;
  return a.b_bf16 ? (float)static_cast<const __bf16*>(a.B)[o] : static_cast<const float*>(a.B)[o];
}

// B slab in LDS, column blocks n0 / 16 .. n0 / 16 + NCB - 1, all KP rows:
//   FP32: f32x4 unit (cb nq + q) 64 + l holds B[16 q + 4 (l / 16) + u][n0 + 16 cb + l % 16], u = 0..3
//         (the four k-steps of one 16-row group, one read per lane);
//   bf16: bf16x8 unit (cb nks + ks) 64 + l holds B[32 ks + 8 (l / 16) + e][n0 + 16 cb + l % 16].
// A chunk c of a lane (row m, k from 64 c): FP32 products read A[m][64 c +
// 16 q + 4 (l / 16) .. + 3] for q = 0..3; bf16 products read A[m][64 c + 32 s
// + 8 (l / 16) .. + 7] for s = 0, 1.
template <class TA, bool kB16, int NCB>
__global__ void __launch_bounds__(kRowsWaves * 64) k_gemm_rows(RowsArgs a) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int lane = __lane_id();
  const int w = threadIdx.x / 64;
  const int lg = lane >> 4, lm = lane & 15;
  const int n0 = blockIdx.y * 16 * NCB;
  const int KP = a.KP;
  const int nch = KP / kKC;
  if constexpr (!kB16) {
    const int nq = KP / 16;
    float* S = reinterpret_cast<float*>(smem);
    const int total = NCB * nq * 256;
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
      const int u = i & 3, l = (i >> 2) & 63, f = i >> 8;
      const int q = f % nq, cb = f / nq;
      S[i] = b_elem(a, 16 * q + 4 * (l >> 4) + u, n0 + 16 * cb + (l & 15));
    }
  } else {
    const int nks = KP / 32;
    __bf16* S = reinterpret_cast<__bf16*>(smem);
    const int total = NCB * nks * 512;
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
      const int e = i & 7, l = (i >> 3) & 63, f = i >> 9;
      const int ks = f % nks, cb = f / nks;
      S[i] = (__bf16)b_elem(a, 32 * ks + 8 * (l >> 4) + e, n0 + 16 * cb + (l & 15));
    }
  }
  __syncthreads();
  int64_t t = blockIdx.x;
  if (t >= a.ntiles) return;

  constexpr bool kA16 = std::is_same<TA, __bf16>::value;
  // k offset (within a chunk) and width of register q of the chunk
  auto koff = [&](int q) {
    if constexpr (!kB16) return 16 * q + 4 * lg;
    else if constexpr (kA16) return 32 * q + 8 * lg;
    else return 32 * (q >> 1) + 8 * lg + 4 * (q & 1);
  };
  constexpr int NR = (kB16 && kA16) ? 2 : 4;        // 16- or 8-byte loads per chunk
  constexpr int WID = (kB16 && kA16) ? 8 : 4;       // elements per load
  // every load is issued from a valid (clamped) address and zeroed after
  // where it lies past Kd or M
  auto load_chunk = [&](int64_t tt, int c, uint4 (&v)[4]) {
    const int64_t m = min<int64_t>(tt * kRowsTM + 16 * w + lm, a.M - 1);
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int k = kKC * c + koff(q);
      const int kc = min(k, a.Kd - WID);
      if constexpr (kA16) {
        const __bf16* p = static_cast<const __bf16*>(a.A) + m * a.lda + kc;
        if constexpr (WID == 8) {
          v[q] = *reinterpret_cast<const uint4*>(p);
        } else {
          const uint2 x = *reinterpret_cast<const uint2*>(p);
          v[q] = uint4{x.x, x.y, 0u, 0u};
        }
      } else {
        v[q] = *reinterpret_cast<const uint4*>(static_cast<const float*>(a.A) + m * a.lda + kc);
      }
      if (k + WID > a.Kd) v[q] = uint4{0u, 0u, 0u, 0u};
    }
  };
  f32x4 acc[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto compute = [&](const uint4 (&v)[4], int c) {
    if constexpr (!kB16) {
      const f32x4* S4 = reinterpret_cast<const f32x4*>(smem);
      const int nq = KP / 16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 av = kA16 ? bf4_f32(v[q].x, v[q].y) : __builtin_bit_cast(f32x4, v[q]);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          if (n0 + 16 * cb >= a.N) break;
          const f32x4 bq = S4[(cb * nq + 4 * c + q) * 64 + lane];
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], bq[u], acc[cb], 0, 0, 0);
        }
      }
    } else {
      const bf16x8* S8 = reinterpret_cast<const bf16x8*>(smem);
      const int nks = KP / 32;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        bf16x8 av;
        if constexpr (kA16)
          av = __builtin_bit_cast(bf16x8, v[s]);
        else
          av = f32_bf8(__builtin_bit_cast(f32x4, v[2 * s]), __builtin_bit_cast(f32x4, v[2 * s + 1]));
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          if (n0 + 16 * cb >= a.N) break;
          const bf16x8 bf = S8[(cb * nks + 2 * c + s) * 64 + lane];
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bf, acc[cb], 0, 0, 0);
        }
      }
    }
  };
  // Epilogue of a tile: destination rows and scales are looked up one tile
  // ahead (they depend on index loads), and the values a tile adds into are
  // loaded before its products, so neither wait sits in front of the stores.
  int64_t dst_cur[4], dst_nxt[4];
  float sc_cur[4], sc_nxt[4];
  float cv[4][NCB];
  auto epi_rows = [&](int64_t tt, int64_t (&dst)[4], float (&sc)[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = min<int64_t>(tt * kRowsTM + 16 * w + 4 * lg + r, a.M - 1);
      dst[r] = a.epi.orow ? (int64_t)a.epi.orow[a.epi.oidx ? a.epi.oidx[m] : m] : m;
      sc[r] = a.epi.wcnt ? (float)(a.epi.wcnt[m + 1] - a.epi.wcnt[m]) : 1.0f;
    }
  };
  auto epi_load = [&](int64_t tt) {
    if (!a.epi.accumulate) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool on = tt * kRowsTM + 16 * w + 4 * lg + r < a.M;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int n = min(n0 + 16 * cb + lm, a.N - 1);
        cv[r][cb] = on ? a.C[dst_cur[r] * a.ldc + n] : 0.0f;
      }
    }
  };
  auto epilogue = [&](int64_t tt) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = tt * kRowsTM + 16 * w + 4 * lg + r;
      if (m < a.M) {
        float* crow = a.C + dst_cur[r] * a.ldc;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const int n = n0 + 16 * cb + lm;
          if (n < a.N) {
            const float v = sc_cur[r] * acc[cb][r];
            if (a.epi.accumulate) {
              crow[n] = cv[r][cb] + v;
            } else {
              const float u = a.epi.bias ? v + a.epi.bias[n] : v;
              crow[n] = a.epi.act == RELNN_ACT_RELU ? fmaxf(u, 0.0f) : u;
            }
          }
        }
      }
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
  };

  uint4 cur[4], nxt[4];
  load_chunk(t, 0, cur);
  epi_rows(t, dst_cur, sc_cur);
  epi_rows(min<int64_t>(t + gridDim.x, a.ntiles - 1), dst_nxt, sc_nxt);
  epi_load(t);
  int c = 0;
  for (;;) {
    int64_t tn = t;
    int cn = c + 1;
    if (cn == nch) {
      cn = 0;
      tn = t + gridDim.x;
    }
    load_chunk(min<int64_t>(tn, a.ntiles - 1), cn, nxt);   // the next chunk is in flight meanwhile
    compute(cur, c);
    if (cn == 0) {
      epilogue(t);
      if (tn >= a.ntiles) break;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        dst_cur[r] = dst_nxt[r];
        sc_cur[r] = sc_nxt[r];
      }
      epi_load(tn);
      epi_rows(min<int64_t>(tn + gridDim.x, a.ntiles - 1), dst_nxt, sc_nxt);
    }
    t = tn;
    c = cn;
#pragma unroll
    for (int q = 0; q < 4; ++q) cur[q] = nxt[q];
  }
}

template <class TA, bool kB16, int NCB>
void launch_rows_n(const RowsArgs& a, int64_t slab, hipStream_t s) {
  const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(a.ntiles, 2 * (int64_t)cu_count()));
  const unsigned gy = (unsigned)cdiv(a.N, 16 * NCB);
  allow_lds(k_gemm_rows<TA, kB16, NCB>, (size_t)slab);
  k_gemm_rows<TA, kB16, NCB><<<dim3(gx, gy), kRowsWaves * 64, (size_t)slab, s>>>(a);
  RELNN_LAUNCHED();
}

template <class TA, bool kB16>
void launch_rows(const RowsArgs& a, hipStream_t s) {
  const int64_t per_cb = (int64_t)a.KP * 16 * (kB16 ? 2 : 4);       // slab bytes per column block
  int ncb = 8;
  while (ncb > 1 && (16 * (ncb / 2) >= a.N || per_cb * ncb > kSlabBytes)) ncb /= 2;
  RELNN_REQUIRE(per_cb * ncb <= kSlabBytes, RELNN_E_UNSUPPORTED, "product depth %d too large", a.Kd);
  const int64_t slab = per_cb * ncb;
  switch (ncb) {
    case 8: launch_rows_n<TA, kB16, 8>(a, slab, s); break;
    case 4: launch_rows_n<TA, kB16, 4>(a, slab, s); break;
    case 2: launch_rows_n<TA, kB16, 2>(a, slab, s); break;
    default: launch_rows_n<TA, kB16, 1>(a, slab, s); break;
  }
}

// --------------------------------------------------------------- gemm_tn
struct TnArgs {
  const void* A;
  int64_t lda;
  const int32_t* arow;
  const int32_t* aidx;
  TnB b;
  int64_t M;
  int Ka, N;
  const int32_t* wcnt;   // db weights (null: 1)
  int do_db;
  float* part;     // [nchunk][Ka][N]
  float* dbpart;   // [nchunk][N]
  int64_t ntiles, nchunk;
};

// Tile of MT rows m: AT[i][m] (128 columns i of A from i0) and BT[n][m] (128
// columns n of B from n0), row stride TS elements, in FP32 or bf16.  Staging
// unit: 4 rows x 4 columns of one matrix (four 16-byte loads, written as four
// 4-element column vectors).
template <class TA, bool kB16>
__global__ void __launch_bounds__(kTnThreads) k_gemm_tn(TnArgs a) {
  constexpr int MT = kB16 ? 64 : 32;
  constexpr int TS = MT + (kB16 ? 8 : 4);
  using LT = typename std::conditional<kB16, __bf16, float>::type;
  constexpr int NB = (MT / 4) * 32;                // staging units per matrix and tile
  constexpr int PER = 2 * NB / kTnThreads;         // units per thread: 1 (FP32) or 2 (bf16)
  constexpr int BUF = 2 * 128 * TS;                // elements per buffer
  constexpr bool kA16 = std::is_same<TA, __bf16>::value;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  LT* lds = reinterpret_cast<LT*>(smem);
  const int tid = threadIdx.x, lane = __lane_id(), w = tid / 64, lg = lane >> 4, lm = lane & 15;
  const int i0 = blockIdx.y * 128, n0 = blockIdx.z * 128;
  const int64_t ch = blockIdx.x;
  const int64_t tb = a.ntiles * ch / a.nchunk, te = a.ntiles * (ch + 1) / a.nchunk;
  const bool do_db = a.do_db && blockIdx.y == 0;
  const bool route = a.b.own != nullptr;
  const bool wave_on = i0 + 16 * w < a.Ka;

  int unit_mat[PER], unit_mg[PER], unit_cg[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int bi = tid + kTnThreads * p;
    unit_mat[p] = bi / NB;
    const int idx = bi % NB;
    unit_mg[p] = idx / 32;
    unit_cg[p] = idx % 32;
  }
  int32_t rn0[PER][4], rn1[PER][4];                // source rows of the units, two tiles
  // bf16 A into bf16 tiles moves the raw 16-bit values (no conversion)
  constexpr bool kRawA = kA16 && kB16;
  struct Stage {                                   // one tile's loads, in registers
    f32x4 x[PER][4];                               // one f32x4 per unit row
    uint2 raw[PER][4];                             // kRawA: the A unit rows as loaded
    int32_t cnt[PER][4];                           // db weights of the B unit rows
    uint32_t keep[PER][4];                         // routing of the B unit rows: one bit per column
  };
  Stage st0, st1;
  auto fetch_idx = [&](int64_t t, int32_t (&rn)[PER][4]) {
#pragma unroll
    for (int p = 0; p < PER; ++p)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = min<int64_t>(t * MT + 4 * unit_mg[p] + r, a.M - 1);
        if (unit_mat[p] == 0 && a.arow)
          rn[p][r] = a.arow[a.aidx ? a.aidx[m] : m];
        else if (unit_mat[p] == 1 && a.b.brow)
          rn[p][r] = a.b.brow[m];
        else
          rn[p][r] = (int32_t)m;
      }
  };
  auto fetch_data = [&](int64_t t, Stage& S, const int32_t (&rn)[PER][4]) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      if (unit_mat[p] == 0) {
        const int col = min(i0 + 4 * unit_cg[p], a.Ka - 4);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if constexpr (kRawA) {
            S.raw[p][r] =
                *reinterpret_cast<const uint2*>(static_cast<const __bf16*>(a.A) + (int64_t)rn[p][r] * a.lda + col);
          } else if constexpr (kA16) {
            const uint2 v =
                *reinterpret_cast<const uint2*>(static_cast<const __bf16*>(a.A) + (int64_t)rn[p][r] * a.lda + col);
            S.x[p][r] = bf4_f32(v.x, v.y);
          } else {
            S.x[p][r] = *reinterpret_cast<const f32x4*>(static_cast<const float*>(a.A) + (int64_t)rn[p][r] * a.lda + col);
          }
        }
      } else {
        const int col = min(n0 + 4 * unit_cg[p], a.N - 4);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t m = min<int64_t>(t * MT + 4 * unit_mg[p] + r, a.M - 1);
          S.x[p][r] = *reinterpret_cast<const f32x4*>(a.b.B + (int64_t)rn[p][r] * a.b.ldb + col);
          if (do_db && a.wcnt) S.cnt[p][r] = a.wcnt[m + 1] - a.wcnt[m];
          if (route)                                // the four columns col .. col + 3 of row m
            S.keep[p][r] = 15u & (a.b.own[m * a.b.own_w + (col >> 5)] >> (col & 31));
        }
      }
    }
  };
  f32x4 dbacc = {0.f, 0.f, 0.f, 0.f};              // db of this thread's B unit columns (do_db)
  auto stash = [&](int b, int64_t t, const Stage& S) {
    LT* base = lds + b * BUF;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int mat = unit_mat[p], mg = unit_mg[p], cg = unit_cg[p];
      const bool col_on = mat == 0 ? i0 + 4 * cg + 4 <= a.Ka : n0 + 4 * cg + 4 <= a.N;
      LT* dst = base + (mat * 128 + 4 * cg) * TS + 4 * mg;
      if constexpr (kRawA) {
        if (mat == 0) {                            // rows r of column cc: 16-bit half cc % 2 of word cc / 2
          uint2 u[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const bool on = col_on && t * MT + 4 * mg + r < a.M;
            u[r] = on ? S.raw[p][r] : make_uint2(0u, 0u);
          }
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            const uint32_t w0 = cc < 2 ? u[0].x : u[0].y, w1 = cc < 2 ? u[1].x : u[1].y;
            const uint32_t w2 = cc < 2 ? u[2].x : u[2].y, w3 = cc < 2 ? u[3].x : u[3].y;
            const uint32_t sel = (cc & 1) ? 0x07060302u : 0x05040100u;
            *reinterpret_cast<uint2*>(dst + cc * TS) =
                make_uint2(__builtin_amdgcn_perm(w1, w0, sel), __builtin_amdgcn_perm(w3, w2, sel));
          }
          continue;
        }
      }
      f32x4 v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool on = col_on && t * MT + 4 * mg + r < a.M;
        v[r] = on ? S.x[p][r] : f32x4{0.f, 0.f, 0.f, 0.f};
        if (mat == 1 && route) {
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) v[r][cc] = ((S.keep[p][r] >> cc) & 1u) ? v[r][cc] : 0.0f;
        }
        if (mat == 1 && do_db) dbacc += (on ? (a.wcnt ? (float)S.cnt[p][r] : 1.0f) : 0.0f) * v[r];
      }
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        if constexpr (kB16) {
          typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
          bf16x4 q;
#pragma unroll
          for (int r = 0; r < 4; ++r) q[r] = (__bf16)v[r][cc];
          *reinterpret_cast<bf16x4*>(dst + cc * TS) = q;
        } else {
          *reinterpret_cast<f32x4*>(dst + cc * TS) = f32x4{v[0][cc], v[1][cc], v[2][cc], v[3][cc]};
        }
      }
    }
  };
  f32x4 acc[8];
#pragma unroll
  for (int cb = 0; cb < 8; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto compute = [&](int b) {
    if (!wave_on) return;
    const LT* AT = lds + b * BUF;
    const LT* BT = AT + 128 * TS;
    if constexpr (!kB16) {
#pragma unroll
      for (int grp = 0; grp < 2; ++grp) {
        const int to = 8 * lg + 4 * grp;
        const f32x4 aa = *reinterpret_cast<const f32x4*>(AT + (16 * w + lm) * TS + to);
#pragma unroll
        for (int cb = 0; cb < 8; ++cb) {
          if (n0 + 16 * cb >= a.N) break;
          const f32x4 bb = *reinterpret_cast<const f32x4*>(BT + (16 * cb + lm) * TS + to);
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aa[u], bb[u], acc[cb], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const int off = 32 * ks + 8 * lg;
        const bf16x8 aa = *reinterpret_cast<const bf16x8*>(AT + (16 * w + lm) * TS + off);
#pragma unroll
        for (int cb = 0; cb < 8; ++cb) {
          if (n0 + 16 * cb >= a.N) break;
          const bf16x8 bb = *reinterpret_cast<const bf16x8*>(BT + (16 * cb + lm) * TS + off);
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aa, bb, acc[cb], 0, 0, 0);
        }
      }
    }
  };

  // Tile t is multiplied from LDS buffer (t - tb) & 1 while tile t + 1 is
  // stashed into the other.  Values are loaded two tiles ahead into two
  // register stages and row numbers three tiles ahead into two row buffers,
  // all at indices known at compile time (the loop runs two tiles a pass).
  // Each tile's row numbers are loaded before the previous tile's values,
  // so waiting for them never waits for values still in flight.  Prefetches
  // past the chunk's last tile repeat it (valid, unused).
  const int64_t tl = te - 1;
  fetch_idx(tb, rn0);
  fetch_idx(min(tb + 1, tl), rn1);
  fetch_data(tb, st0, rn0);
  fetch_idx(min(tb + 2, tl), rn0);
  fetch_data(min(tb + 1, tl), st1, rn1);
  fetch_idx(min(tb + 3, tl), rn1);
  stash(0, tb, st0);
  __syncthreads();
  for (int64_t t = tb; t < te; t += 2) {
    fetch_data(min(t + 2, tl), st0, rn0);
    fetch_idx(min(t + 4, tl), rn0);
    compute(0);
    if (t + 1 < te) stash(1, t + 1, st1);
    __syncthreads();
    if (t + 1 >= te) break;
    fetch_data(min(t + 3, tl), st1, rn1);
    fetch_idx(min(t + 5, tl), rn1);
    compute(1);
    if (t + 2 < te) stash(0, t + 2, st0);
    __syncthreads();
  }
  if (wave_on) {
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) {
      const int n = n0 + 16 * cb + lm;
      if (n < a.N) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + 16 * w + 4 * lg + r;
          if (i < a.Ka) a.part[(ch * a.Ka + i) * a.N + n] = acc[cb][r];
        }
      }
    }
  }
  if (do_db) {                                      // uniform over the block
    float* dbs = reinterpret_cast<float*>(smem);    // [MT / 4][128], the tiles are no longer read
#pragma unroll
    for (int p = 0; p < PER; ++p)
      if (unit_mat[p] == 1)
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) dbs[unit_mg[p] * 128 + 4 * unit_cg[p] + cc] = dbacc[cc];
    __syncthreads();
    if (tid < 128 && n0 + tid < a.N) {
      float sdb = 0.0f;
      for (int mg = 0; mg < MT / 4; ++mg) sdb += dbs[mg * 128 + tid];
      a.dbpart[ch * a.N + n0 + tid] = sdb;
    }
  }
}

// D[i][n] (+)= sum over chunks c of part[c][i][n] (and db from dbpart), in
// chunk order, Kahan-compensated.
__global__ void k_tn_sum(const float* part, const float* dbpart, int64_t nchunk, int Ka, int N, float* D, float* db,
                         int accumulate) {
  const int64_t nd = (int64_t)Ka * N;
  const int64_t total = nd + (db ? N : 0);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const bool is_d = i < nd;
    const float* src = is_d ? part + i : dbpart + (i - nd);
    const int64_t stride = is_d ? nd : N;
    float s = 0.0f, c = 0.0f;
    for (int64_t k = 0; k < nchunk; ++k) {
      const float y = src[k * stride] - c;
      const float t = s + y;
      c = __builtin_isfinite(t) ? (t - s) - y : 0.0f;    // no NaN compensation of an infinite sum
      s = t;
    }
    float* o = is_d ? D + i : db + (i - nd);
    *o = accumulate ? *o + s : s;
  }
}

__global__ void k_zero_or_keep(float* p, int64_t n, int accumulate) {
  if (accumulate) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

int64_t tn_chunks(int64_t M, int Ka, int N) {
  const int64_t blocks_per_chunk = cdiv(Ka, 128) * cdiv(N, 128);
  return std::max<int64_t>(1, std::min<int64_t>(cdiv(std::max<int64_t>(M, 1), 64),
                                                std::max<int64_t>(1, kTnTarget / blocks_per_chunk)));
}

template <class TA, bool kB16>
void launch_tn(TnArgs a, hipStream_t s) {
  constexpr int MT = kB16 ? 64 : 32;
  constexpr int TS = MT + (kB16 ? 8 : 4);
  const size_t lds = (size_t)2 * 2 * 128 * TS * (kB16 ? 2 : 4);
  a.ntiles = cdiv(a.M, MT);
  dim3 grid((unsigned)a.nchunk, (unsigned)cdiv(a.Ka, 128), (unsigned)cdiv(a.N, 128));
  allow_lds(k_gemm_tn<TA, kB16>, lds);
  k_gemm_tn<TA, kB16><<<grid, kTnThreads, lds, s>>>(a);
  RELNN_LAUNCHED();
}

unsigned grid_1d(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 1 << 16)); }

}  // namespace

void gemm_rows(bool mfma_bf16, const void* A, bool a_bf16, int64_t lda, int64_t M, int Kd, const void* Bsrc,
               bool b_bf16, bool b_trans, int64_t ldb, int N, float* C, int64_t ldc, const RowsEpi& epi,
               hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  RELNN_REQUIRE(Kd > 0 && Kd <= 1024 && Kd % (a_bf16 && mfma_bf16 ? 8 : 4) == 0, RELNN_E_UNSUPPORTED,
                "product depth %d not supported", Kd);
  RELNN_REQUIRE(((uintptr_t)A & 15) == 0 && (lda * (a_bf16 ? 2 : 4)) % 16 == 0, RELNN_E_UNSUPPORTED,
                "product operand rows are not 16-byte aligned");
  RowsArgs a{};
  a.A = A;
  a.lda = lda;
  a.M = M;
  a.Kd = Kd;
  a.KP = (int)round_up(Kd, kKC);
  a.N = N;
  a.B = Bsrc;
  a.ldb = ldb;
  a.b_bf16 = b_bf16 ? 1 : 0;
  a.b_trans = b_trans ? 1 : 0;
  a.C = C;
  a.ldc = ldc;
  a.epi = epi;
  a.ntiles = cdiv(M, kRowsTM);
  if (mfma_bf16) {
    if (a_bf16)
      launch_rows<__bf16, true>(a, s);
    else
      launch_rows<float, true>(a, s);
  } else {
    if (a_bf16)
      launch_rows<__bf16, false>(a, s);
    else
      launch_rows<float, false>(a, s);
  }
}

int64_t gemm_tn_ws_floats(int64_t M, int Ka, int N) {
  const int64_t nc = tn_chunks(M, Ka, N);
  return nc * Ka * N + nc * N;
}

void gemm_tn(bool mfma_bf16, const void* Asrc, bool a_bf16, int64_t lda, const int32_t* arow, const int32_t* aidx,
             const TnB& B, int64_t M, int Ka, int N, const int32_t* wcnt, float* D, float* db, bool accumulate,
             float* ws, hipStream_t s) {
  if (Ka <= 0 || N <= 0) return;
  RELNN_REQUIRE(Ka % 4 == 0 && N % 4 == 0 && lda % 4 == 0 && B.ldb % 4 == 0, RELNN_E_UNSUPPORTED,
                "product widths %d x %d not supported", Ka, N);
  RELNN_REQUIRE(M < (int64_t)INT32_MAX, RELNN_E_RANGE, "product over %lld rows", (long long)M);
  if (M <= 0) {
    k_zero_or_keep<<<grid_1d((int64_t)Ka * N), 256, 0, s>>>(D, (int64_t)Ka * N, accumulate ? 1 : 0);
    RELNN_LAUNCHED();
    if (db) {
      k_zero_or_keep<<<1, 256, 0, s>>>(db, N, accumulate ? 1 : 0);
      RELNN_LAUNCHED();
    }
    return;
  }
  TnArgs a{};
  a.A = Asrc;
  a.lda = lda;
  a.arow = arow;
  a.aidx = aidx;
  a.b = B;
  a.M = M;
  a.Ka = Ka;
  a.N = N;
  a.wcnt = wcnt;
  a.do_db = db != nullptr;
  a.nchunk = tn_chunks(M, Ka, N);
  a.part = ws;
  a.dbpart = ws + a.nchunk * Ka * N;
  if (mfma_bf16) {
    if (a_bf16)
      launch_tn<__bf16, true>(a, s);
    else
      launch_tn<float, true>(a, s);
  } else {
    if (a_bf16)
      launch_tn<__bf16, false>(a, s);
    else
      launch_tn<float, false>(a, s);
  }
  k_tn_sum<<<grid_1d((int64_t)Ka * N + N), 256, 0, s>>>(a.part, a.dbpart, a.nchunk, Ka, N, D, db,
                                                         accumulate ? 1 : 0);
  RELNN_LAUNCHED();
}

}  // namespace relnn
