// Internal interface between the forward and backward layer sources.
#pragma once

#include "layer_common.hpp"

namespace relnn {

struct Atoms {
  const void* emb[kMaxAtoms];
  const int32_t* rows[kMaxAtoms];   // [E] joined row of atom j per tuple
  int32_t d[kMaxAtoms];
  int32_t koff[kMaxAtoms];   // first Concat column of atom j
  int32_t k;
};

struct FwdArgs {
  Atoms at;
  const int32_t* rows;       // [k*E]
  int64_t E;
  const int64_t* E_dev;      // if set: E read from device memory at run time
  int K, Kp, h, TM;
  int off_x, off_y;          // LDS byte offsets of Xs / Ys
  const void* Wsw;
  const float* b;
  int act_pre;
  Seg sg;
  Sink sink;
  float* carry;
  int32_t* carry_arg;
  const void* W;             // plain: W as given, row-major [K][h]
  const void* X;             // plain: [E][Kp]
  float* Y;                  // plain: [E][h]
  uint32_t* mask;            // act_pre mask: [E][ceil(h / 32)] words, bit c % 32 of word c / 32 set where x W + b > 0
};

struct FwdPlan {
  int K = 0, Kp = 0, TM = 0;
  size_t off_x = 0, off_y = 0, lds = 0;
  int64_t ntiles = 0;
  int64_t carry_units = 0;   // units the carry region holds (max over kernels)
  size_t ws_push_p[RELNN_MAX_ATOMS] = {};   // pushdown: node products of atom j
  size_t ws_push_v = 0;                     // pushdown: per-group aggregates before the group constant
  size_t ws_push = 0;                       // pushdown total
  size_t ws_wsw = 0, ws_carry = 0, ws_carry_arg = 0, ws_x = 0, ws_y = 0;
  size_t ws_fused = 0, ws_plain = 0;
};

FwdPlan plan_fwd(const relnn_index* idx, const relnn_layer_desc* L);
// relnn_layer_fwd without the status mapping (throws Fail), and the
// workspace bytes it needs for this index and layer.
void layer_fwd_run(const relnn_index* idx, const relnn_layer_desc* L, const void* const* emb, const void* W,
                   const float* b, float* out, float* pre, int32_t* argmax, void* ws, size_t ws_bytes,
                   hipStream_t stream);
size_t layer_fwd_ws_bytes(const relnn_index* idx, const relnn_layer_desc* L);
// relnn_layer_bwd without the status mapping (throws Fail), and its
// workspace bytes.
void layer_bwd_run(const relnn_index* idx, const relnn_layer_desc* L, const void* const* emb, const void* W,
                   const float* b, const float* pre, const int32_t* argmax, const float* dout, float* const* demb,
                   float* dW, float* db, void* ws, size_t ws_bytes, hipStream_t stream);
size_t layer_bwd_ws_bytes(const relnn_index* idx, const relnn_layer_desc* L);
// Validates the index / layer pair, then plans (RELNN_E_* on failure).
FwdPlan checked_plan(const relnn_index* idx, const relnn_layer_desc* L);
Atoms make_atoms(const relnn_layer_desc* L, const void* const* emb, const relnn_index* idx);
void swizzle_w(const void* W, int dtype, int K, int Kp, int h, void* Wsw, hipStream_t s);
void launch_fwd(const FwdPlan& P, const FwdArgs& a, int dtype, bool plain, hipStream_t s);

// Plain path (plain.hip).  plain_gemm: row-major Y[n][h] = X[n][K] W[K][h]
// (X with leading dimension ldx) on rocBLAS, FP32 or BF16 inputs with FP32
// accumulation.  launch_seg_reduce: out_g = act_post(alpha over the rows of
// group g of act_pre(Y + b)), then the carry fix-up; seg_reduce_units is
// the number of carry units it uses for E rows.
void plain_gemm(int dtype, const void* X, int64_t n, int K, int ldx, const void* W, int h, float* Y,
                hipStream_t s);
int64_t seg_reduce_units(int64_t E);
void launch_seg_reduce(const float* Y, int64_t E, int h, const Seg& sg, const float* b, int act_pre,
                       const Sink& sink, float* carry, int32_t* carry_arg, int64_t carry_units, hipStream_t s);
// Recomputes y = x W + b per tuple and writes the bits (y > 0) (tile kernel).
void launch_mask(const FwdPlan& P, const FwdArgs& a, int dtype, hipStream_t s);
void launch_fixup(const Seg& sg, int TM, int h, int64_t ntiles, int64_t nunits, const Sink& sink,
                  const float* carry, const int32_t* carry_arg, hipStream_t s);

// Weight-stationary persistent forward (layer_ws.hip).  KP == 0: the shape
// is not covered and the tile kernel runs instead.
struct WsPlan {
  int KP = 0, TM = 0;
  int hc = 0, nch = 0;       // output columns per block, column chunks
  int64_t ntiles = 0, nunits = 0;
  size_t wsw_bytes = 0, carry_elems = 0;
};
WsPlan plan_ws(int dtype, int K, int h, int64_t E);
void swizzle_ws(const void* W, int dtype, int K, int KP, int h, void* out, hipStream_t s);
void launch_ws(const WsPlan& p, int dtype, const FwdArgs& f, const void* Wsw, float* carry,
               int32_t* carry_arg, hipStream_t s);

// Pushed-down transform: gather-sum of the node products P (n atoms per
// tuple) and per-group reduce (layer_ws.hip); the sink carries the group
// constant, which a second pass over the G groups adds (V: [G][h] FP32
// workspace for the aggregates before it).  push_units: waves (and carry
// units) it uses for E tuples.
void launch_push(const FwdArgs& f, int64_t nunits, int n, const float* const* P, const int32_t* const* rows,
                 float* carry, int32_t* carry_arg, int64_t G, float* V, hipStream_t s);
int64_t push_units(int64_t E);
// Product transform (RELNN_TF_PRODUCT): the same gather over the atoms'
// embeddings, multiplied elementwise per tuple (act_pre applied), then
// aggregated through the sink.
void launch_product(const FwdArgs& f, bool bf16, int64_t nunits, float* carry, int32_t* carry_arg, hipStream_t s);

// Segmented gather-sum over a sorted list (bwd_linear.hip): out[s] = sum
// over the positions e of segment s of the joined row at e (the atoms' rows
// concatenated), optionally routed (MAX ownership bits, act_pre mask) and
// weighted (one weight per tuple and block of whd columns); atomic-free,
// Kahan within a wave's range, carries combined in order.
struct GsArgs {
  const void* emb[kMaxAtoms];      // [n_j][d_j], FP32 or BF16
  const int32_t* rows[kMaxAtoms];  // [n] row of atom j at each list position
  int d[kMaxAtoms];
  int koff[kMaxAtoms];
  int k;
  int K;                           // sum of d_j, a multiple of 4
  bool bf16;
  int64_t n;                       // list positions
  Seg sg;                          // segments of the sorted list
  float* out;                      // [nseg][ldo], or rows out_row[seg] of it
  int ldo;                         // row stride of out and carry (>= K)
  const int32_t* out_row;          // optional remap: segment -> row of out
  bool accumulate;                 // out row += sum (rows distinct) instead of ==
  float* carry;                    // [nunits][2][ldo]
  int64_t ntiles, nunits;
  // routing of a gathered gradient row (one atom, dA of width h; rows[0] is
  // the group of the tuple at each position, rows[1] its canonical position):
  // keep column c only where bit c % 32 of word c / 32 of the tuple is set
  // (MAX: the tuple is its group's maximiser; act_pre: x W + b > 0)
  const uint32_t* own;             // [E][own_w] or null
  int own_w;
  // weights: column c of the row at position e times wgt[tau wh + c / whd],
  // tau = rows[1][e] (whd a multiple of the columns a lane holds)
  const float* wgt;
  int wh, whd;
};
int64_t gs_units(int64_t n);
void seg_gather_sum(GsArgs a, int64_t nseg_units_cap, hipStream_t s);

// Backward through sums over groups and joined rows (bwd_linear.hip).
// lin_bwd_dx: dz_j of every atom, for any layer (routed by argmax for MAX,
// masked by act_pre'); lin_bwd_dw: dW and db when the transform is affine
// and the aggregate SUM or MEAN (xs_dw).
struct LinBwdPlan {
  int64_t units = 0;
  int ldx = 0;
  size_t ws_xs = 0, ws_part = 0, ws_ds = 0, ws_carry = 0, total = 0;
};
LinBwdPlan plan_lin_bwd(const relnn_index* idx, const relnn_layer_desc* L, size_t base, bool xs_dw);
void lin_bwd_dw(const relnn_index* idx, const relnn_layer_desc* L, const LinBwdPlan& P, const void* const* emb,
                const float* dA, float* dW, float* db, bool accum, char* ws, hipStream_t s);
// route: routing bits [E][route_w] (bit c % 32 of word c / 32: the tuple's
// gradient reaches column c: it is its group's maximiser (MAX) and x W + b >
// 0 there (act_pre)), or null; per_tuple: act_pre, so a group-keyed atom
// cannot take its rows from the group sums
void lin_bwd_dx(const relnn_index* idx, const relnn_layer_desc* L, const LinBwdPlan& P, const void* W,
                const float* dA, const uint32_t* route, int route_w, bool per_tuple, float* const* demb, char* ws,
                hipStream_t s);
size_t bwd_workspace(const relnn_index* idx, const relnn_layer_desc* L, const FwdPlan& P);
// Backward of the product transform (prod_bwd.hip): dz_j of every atom from
// the routed gradient dA [G][h] (MEAN divided) and, for MAX, the maximiser
// bits; act_pre' is taken from the full product inside the pass.
size_t prod_bwd_ws_bytes(const relnn_index* idx, const relnn_layer_desc* L);
void prod_bwd(const relnn_index* idx, const relnn_layer_desc* L, const void* const* emb, const float* dA,
              const uint32_t* own, int own_w, float* const* demb, char* ws, hipStream_t s);
// dW rows [d][h] of atom j when its FK is the group column, for MAX without
// act_pre: sum_g x_j(g)^T dA_g over the groups (part: gk_dw_ws_floats(G, d,
// h) FP32 workspace).
int64_t gk_dw_ws_floats(int64_t G, int d, int h);
void gk_dw(const relnn_index* idx, int j, const void* emb, bool bf16, int d, int h, const float* dA, float* dW_rows,
           bool accum, float* part, hipStream_t s);

}  // namespace relnn
