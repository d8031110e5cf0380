// Unfused ("plain") layer: the three steps of a library pipeline, each its
// own pass over HBM, with [E, K] and [E, h] materialised in between:
//
//   gather     X[e] = z_1[r_1(e)] (+) ... (+) z_k[r_k(e)]        (k_gather_plain)
//   transform  Y = X W                                          (rocBLAS GEMM)
//   aggregate  out_g = act_post(alpha_{e in g} act_pre(Y[e] + b)) (k_seg_reduce)
//
// (join with concatenated embedding, per-tuple transformation and projected
// union: Section 2.2.)  The aggregate is a segmented reduction over the
// group-sorted rows, written atomic-free: one wavefront streams a unit of
// consecutive rows, finishes the groups that lie inside it, and leaves a
// partial for a group cut by either unit end; k_fixup combines the
// partials in unit order.
#include <rocblas/rocblas.h>

#include <map>
#include <mutex>

#include "layer_fwd.hpp"

namespace relnn {

namespace {

constexpr int kRedTM = 64;            // unit boundaries fall on multiples of 64 rows
constexpr int kRedWaves = 4;          // waves per block
constexpr int kRedBatch = 16;         // rows loaded together per wave
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Compensated add; the compensation is dropped once the sum is not finite
// (an infinite sum stays infinite instead of turning NaN).
__device__ __forceinline__ void kahan(float& s, float& c, float x) {
  const float y = x - c;
  const float t = s + y;
  c = __builtin_isfinite(t) ? (t - s) - y : 0.0f;
  s = t;
}

struct RedArgs {
  const float* Y;            // [E][h]
  int64_t E;
  int h;
  const float* b;            // [h] or null
  int act_pre;
  Seg sg;
  Sink sink;
  float* carry;
  int32_t* carry_arg;
  int64_t ntiles, nunits;
};

// Unit u (one wavefront) covers rows [pos(u), pos(u+1)), pos(u) = (ntiles u
// / nunits) 64; lane l owns columns cb + 2l, cb + 2l + 1 of column pass cb.
// Rows are read 16 at a time with clamped (always valid) addresses so that
// no load sits behind a branch; rows past the unit are skipped after the
// load.  Group numbers come from one coalesced load per 64 rows and are
// read out lane by lane (wave-uniform).
__global__ void __launch_bounds__(kRedWaves * 64) k_seg_reduce(RedArgs a) {
  const int lane = threadIdx.x % 64;
  const int64_t u = (int64_t)blockIdx.x * kRedWaves + threadIdx.x / 64;
  if (u >= a.nunits) return;
  const int64_t r0 = ((a.ntiles * u) / a.nunits) * kRedTM;
  const int64_t r1 = min<int64_t>(((a.ntiles * (u + 1)) / a.nunits) * kRedTM, a.E);
  if (r0 >= r1) return;
  const bool maxagg = a.sink.agg == RELNN_MAX;
  const int h = a.h;

  for (int cb = 0; cb < h; cb += 128) {
    const int c = cb + 2 * lane;
    const bool on = c < h;
    const int cc = on ? c : 0;                     // inactive lanes read column 0
    const float b0 = a.b && on ? a.b[c] : 0.0f;
    const float b1 = a.b && on ? a.b[c + 1] : 0.0f;
    float s0 = 0.0f, s1 = 0.0f, k0 = 0.0f, k1 = 0.0f;   // sum / max, Kahan term
    int32_t a0 = -1, a1 = -1;                            // argmax
    if (maxagg) s0 = s1 = -INFINITY;
    int32_t g = a.sg.seg_of[r0];                         // group being accumulated
    bool first = true;                                   // g is the unit's first group

    auto flush = [&]() {
      const int64_t g0 = a.sg.offsets[g], g1 = a.sg.offsets[g + 1];
      const bool cut_lo = first && g0 < r0;     // began before the unit
      const bool cut_hi = g1 > r1;              // runs past the unit
      if (on) {
        const float v0 = maxagg ? s0 : s0 - k0, v1 = maxagg ? s1 : s1 - k1;
        if (cut_lo || cut_hi) {
          const int64_t o = (u * 2 + (cut_lo ? 0 : 1)) * h + c;
          a.carry[o] = v0;
          a.carry[o + 1] = v1;
          if (a.carry_arg) {
            a.carry_arg[o] = a0;
            a.carry_arg[o + 1] = a1;
          }
        } else {
          sink_write<true>(a.sink, g, c, h, v0, a0, (int32_t)(g1 - g0));
          sink_write<true>(a.sink, g, c + 1, h, v1, a1, (int32_t)(g1 - g0));
        }
      }
      first = false;
      s0 = s1 = maxagg ? -INFINITY : 0.0f;
      k0 = k1 = 0.0f;
      a0 = a1 = -1;
    };

    for (int64_t base = r0; base < r1; base += 64) {
      const int n = (int)min<int64_t>(64, r1 - base);
      const int32_t gl = a.sg.seg_of[base + min(lane, n - 1)];
#pragma unroll
      for (int bt = 0; bt < 64 / kRedBatch; ++bt) {
        if (bt * kRedBatch >= n) break;
        float2 y[kRedBatch];
#pragma unroll
        for (int i = 0; i < kRedBatch; ++i) {
          const int64_t r = base + min(bt * kRedBatch + i, n - 1);
          // Y is read once: non-temporal loads keep it from displacing
          // cached lines
          const f32x2 t2 = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(a.Y + r * h + cc));
          y[i] = make_float2(t2.x, t2.y);
        }
#pragma unroll
        for (int i = 0; i < kRedBatch; ++i) {
          const int q = bt * kRedBatch + i;
          if (q >= n) break;
          const int32_t gq = __builtin_amdgcn_readlane(gl, q);
          if (__builtin_expect(gq != g, 0)) {      // a group ends (cold: keeps the row path compact)
            flush();
            g = gq;
          }
          const float x0 = act_apply(a.act_pre, y[i].x + b0);
          const float x1 = act_apply(a.act_pre, y[i].y + b1);
          if (maxagg) {
            if (x0 > s0) { s0 = x0; a0 = (int32_t)(base + q); }
            if (x1 > s1) { s1 = x1; a1 = (int32_t)(base + q); }
          } else {
            kahan(s0, k0, x0);
            kahan(s1, k1, x1);
          }
        }
      }
    }
    flush();
  }
}

// One rocBLAS handle per device, created on first use.
std::mutex g_blas_mu;
std::map<int, rocblas_handle> g_blas;

rocblas_handle blas_for_current_device() {
  int dev = 0;
  RELNN_HIP(hipGetDevice(&dev));
  auto it = g_blas.find(dev);
  if (it != g_blas.end()) return it->second;
  rocblas_handle h = nullptr;
  RELNN_REQUIRE(rocblas_create_handle(&h) == rocblas_status_success, RELNN_E_HIP, "rocblas_create_handle failed");
  g_blas[dev] = h;
  return h;
}

}  // namespace

void plain_gemm(int dtype, const void* X, int64_t n, int K, int ldx, const void* W, int h, float* Y,
                hipStream_t s) {
  if (n <= 0) return;
  std::lock_guard<std::mutex> lk(g_blas_mu);
  rocblas_handle hb = blas_for_current_device();
  RELNN_REQUIRE(rocblas_set_stream(hb, s) == rocblas_status_success, RELNN_E_HIP, "rocblas_set_stream failed");
  const float one = 1.0f, zero = 0.0f;
  // Row-major Y[n][h] = X[n][K] W[K][h] is, column-major, Y^T = W^T X^T:
  // m = h, n = rows, k = K, A = W (lda h), B = X (ldb ldx), C = Y (ldc h).
  const int64_t step = int64_t(1) << 30;          // rocblas_int row counts
  const size_t esz = dtype == RELNN_BF16 ? 2 : 4;
  for (int64_t r = 0; r < n; r += step) {
    const rocblas_int m = (rocblas_int)std::min<int64_t>(step, n - r);
    const void* Xr = static_cast<const char*>(X) + (size_t)r * ldx * esz;
    float* Yr = Y + r * h;
    rocblas_status st;
    if (dtype == RELNN_BF16)
      st = rocblas_gemm_ex(hb, rocblas_operation_none, rocblas_operation_none, h, m, K, &one, W,
                           rocblas_datatype_bf16_r, h, Xr, rocblas_datatype_bf16_r, ldx, &zero, Yr,
                           rocblas_datatype_f32_r, h, Yr, rocblas_datatype_f32_r, h, rocblas_datatype_f32_r,
                           rocblas_gemm_algo_standard, 0, 0);
    else
      st = rocblas_sgemm(hb, rocblas_operation_none, rocblas_operation_none, h, m, K, &one,
                         static_cast<const float*>(W), h, static_cast<const float*>(Xr), ldx, &zero, Yr, h);
    RELNN_REQUIRE(st == rocblas_status_success, RELNN_E_HIP, "rocBLAS GEMM failed (status %d)", (int)st);
  }
}

int64_t seg_reduce_units(int64_t E) {
  const int64_t ntiles = cdiv(std::max<int64_t>(E, 1), kRedTM);
  return std::max<int64_t>(1, std::min<int64_t>(ntiles, 32768));   // 128 waves per CU
}

void launch_seg_reduce(const float* Y, int64_t E, int h, const Seg& sg, const float* b, int act_pre,
                       const Sink& sink, float* carry, int32_t* carry_arg, int64_t carry_units, hipStream_t s) {
  if (E <= 0) return;
  RELNN_REQUIRE(!sink.accumulate && !sink.out_row && !sink.gc.n && !sink.gc.bias, RELNN_E_UNSUPPORTED,
                "the plain aggregate writes plain outputs only");
  RedArgs a{};
  a.Y = Y;
  a.E = E;
  a.h = h;
  a.b = b;
  a.act_pre = act_pre;
  a.sg = sg;
  a.sink = sink;
  a.carry = carry;
  a.carry_arg = carry_arg;
  a.ntiles = cdiv(E, kRedTM);
  a.nunits = seg_reduce_units(E);
  RELNN_REQUIRE(a.nunits <= carry_units, RELNN_E_HIP, "internal: carry region holds %lld units, %lld needed",
                (long long)carry_units, (long long)a.nunits);
  {
    KTimer t("fwd_reduce", s);
    k_seg_reduce<<<(unsigned)cdiv(a.nunits, kRedWaves), kRedWaves * 64, 0, s>>>(a);
    RELNN_LAUNCHED();
  }
  launch_fixup(sg, kRedTM, h, a.ntiles, a.nunits, sink, carry, carry_arg, s);
}

}  // namespace relnn
