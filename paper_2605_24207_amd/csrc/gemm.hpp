// Matrix-core products of the backward and of the pushed-down transform
// (gemm.hip).  No library GEMM: FP32 products on v_mfma_f32_16x16x4_f32, or
// bf16 products with FP32 accumulation on v_mfma_f32_16x16x32_bf16 (FP32
// operands are rounded to nearest even as they are loaded).
#pragma once

#include "common.hpp"

namespace relnn {

// Where a row of gemm_rows' result goes: C row orow[oidx[m]] (oidx null:
// orow[m]; orow null: m), scaled by wcnt[m+1] - wcnt[m] (wcnt null: 1), added
// into C (accumulate) or stored (plus bias, then the activation act).
// Destination rows must be distinct.
struct RowsEpi {
  const int32_t* orow = nullptr;
  const int32_t* oidx = nullptr;
  const int32_t* wcnt = nullptr;
  bool accumulate = false;
  const float* bias = nullptr;    // stored rows only: + bias[n], then act
  int act = RELNN_ACT_NONE;
};

// C[dst(m)][n] (+)= s_m sum_{k < Kd} A[m][k] B[k][n] for m < M, n < N.
// A: device [M][lda], FP32 or bf16 (a_bf16), Kd % 4 == 0 (FP32 A) or
// Kd % 8 == 0 (bf16 A), rows 16-byte aligned.  B[k][n] = Bsrc[k ldb + n], or
// Bsrc[n ldb + k] when b_trans, FP32 or bf16 (b_bf16).  C: device FP32 with
// row stride ldc.  Kd <= 1024.
void gemm_rows(bool mfma_bf16, const void* A, bool a_bf16, int64_t lda, int64_t M, int Kd, const void* Bsrc,
               bool b_bf16, bool b_trans, int64_t ldb, int N, float* C, int64_t ldc, const RowsEpi& epi,
               hipStream_t s);

// The B side of gemm_tn: row m is B[brow[m]] (brow null: B[m]), [.][ldb]
// FP32, with column n kept only where bit n % 32 of own[m own_w + n / 32] is
// set (own non-null), zero elsewhere: the routed gradient rows of the
// backward.
struct TnB {
  const float* B = nullptr;
  int64_t ldb = 0;
  const int32_t* brow = nullptr;
  const uint32_t* own = nullptr;
  int own_w = 0;
};

// D[i][n] (+)= sum_{m < M} A(m)[i] B(m)[n] for i < Ka, n < N, and, when db
// is given, db[n] (+)= sum_m w_m B(m)[n] with w_m = wcnt[m+1] - wcnt[m]
// (wcnt null: 1).  A(m) is row arow[aidx[m]] (aidx null: arow[m]; arow
// null: m) of Asrc [.][lda], FP32 or bf16.  Ka % 4 == 0, N % 4 == 0, lda,
// ldb multiples of 4.  The sum over m is split over contiguous
// chunks whose partials (ws: gemm_tn_ws_floats(M, Ka, N) floats) are added
// in chunk order, so results are deterministic.
int64_t gemm_tn_ws_floats(int64_t M, int Ka, int N);
void gemm_tn(bool mfma_bf16, const void* Asrc, bool a_bf16, int64_t lda, const int32_t* arow, const int32_t* aidx,
             const TnB& B, int64_t M, int Ka, int N, const int32_t* wcnt, float* D, float* db, bool accumulate,
             float* ws, hipStream_t s);

}  // namespace relnn
