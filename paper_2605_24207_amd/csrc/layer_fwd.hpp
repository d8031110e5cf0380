// Internal interface between the forward and backward layer sources.
#pragma once

#include "layer_common.hpp"

namespace relnn {

struct Atoms {
  const void* emb[kMaxAtoms];
  int32_t d[kMaxAtoms];
  int32_t koff[kMaxAtoms];   // first Concat column of atom j
  int32_t k;
};

struct FwdArgs {
  Atoms at;
  const int32_t* rows;       // [k*E]
  int64_t E;
  int K, Kp, h, TM;
  int off_x, off_y;          // LDS byte offsets of Xs / Ys
  const void* Wsw;
  const float* b;
  int act_pre;
  Seg sg;
  Sink sink;
  float* carry;
  int32_t* carry_arg;
  const void* X;             // plain: [E][Kp]
  float* Y;                  // plain: [E][h]
};

struct FwdPlan {
  int K = 0, Kp = 0, TM = 0;
  size_t off_x = 0, off_y = 0, lds = 0;
  int64_t ntiles = 0;
  size_t ws_wsw = 0, ws_carry = 0, ws_carry_arg = 0, ws_x = 0, ws_y = 0;
  size_t ws_fused = 0, ws_plain = 0;
};

FwdPlan plan_fwd(const relnn_index* idx, const relnn_layer_desc* L);
void check_layer(const relnn_index* idx, const relnn_layer_desc* L, const FwdPlan& P);
Atoms make_atoms(const relnn_layer_desc* L, const void* const* emb);
void swizzle_w(const void* W, int dtype, int K, int Kp, int h, void* Wsw, hipStream_t s);
void launch_fwd(const FwdPlan& P, const FwdArgs& a, int dtype, bool plain, hipStream_t s);
void launch_fixup(const Seg& sg, int TM, int h, int64_t ntiles, const Sink& sink, const float* carry,
                  const int32_t* carry_arg, hipStream_t s);
size_t bwd_workspace(const relnn_index* idx, const relnn_layer_desc* L, const FwdPlan& P);

}  // namespace relnn
