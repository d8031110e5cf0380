/*
 * relnn.h -- C ABI of librelnn, an MI355X (gfx950) library for one
 * relational layer of Neuro-Relational Algebra:
 *
 *     Out(g; act_post(alpha(act_pre(Linear(z_1 (+) ... (+) z_k)))))
 *         :- Link(...), R_1(c_1; z_1), ..., R_k(c_k; z_k)
 *
 * i.e. the join rule of Section 3.1 compiled to projected-union(T(join)):
 *   - join (Section 2.2): natural join of a link relation with body atoms on
 *     foreign-key -> primary-key equality; a joined tuple's embedding is the
 *     concatenation of the atoms' embeddings in body order;
 *   - transformation (Section 2.2): tau = act_pre(x W + b) per joined tuple;
 *   - projected union, k = 1 (Section 2.2): group the joined tuples by the
 *     head key (a set of keys) and aggregate each multiset with SUM, MEAN or
 *     MAX exactly once; act_post follows the union-rule form (Section 3.1),
 *     where the transform comes after the union.
 * Parameters include both the embeddings and the weights (Section 2.3), so
 * the backward returns gradients for both.
 *
 * Conventions for every entry point:
 *   - Return a relnn_status; nothing throws across the ABI.  On an error
 *     relnn_last_error() holds a message (thread-local).
 *   - Arguments are validated before any launch; on a validation error
 *     nothing is written.
 *   - "device" pointers are HIP device memory of the current device;
 *     "host" pointers are ordinary host memory.  Arrays of device pointers
 *     (emb, demb, cols) are themselves host arrays.
 *   - The caller owns every embedding, weight, output and workspace buffer
 *     and keeps them alive until the stream work completes.  The library
 *     owns relnn_index and relnn_server and all memory inside them.
 *   - Layer calls are asynchronous on the given stream.  relnn_build_index
 *     synchronises the stream (the sizes E and G become known there).
 *   - Ids and keys are int32; a tuple count must stay below 2^31.
 */
#ifndef RELNN_H
#define RELNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Same type as hipStream_t; NULL is the default stream. */
typedef struct ihipStream_t* relnn_stream_t;

typedef enum {
  RELNN_OK = 0,
  RELNN_E_INVALID = 1,      /* bad argument or descriptor */
  RELNN_E_RANGE = 2,        /* a size or count out of the supported range */
  RELNN_E_NOT_UNIQUE = 3,   /* duplicate primary key in a keyed relation */
  RELNN_E_OOM = 4,          /* device allocation failed / budget exceeded */
  RELNN_E_HIP = 5,          /* a HIP runtime call failed */
  RELNN_E_BUSY = 6,         /* server: no slot or budget free right now */
  RELNN_E_NOT_READY = 7,    /* server: request not finished yet */
  RELNN_E_UNSUPPORTED = 8   /* valid, but a shape the library does not run */
} relnn_status;

typedef enum { RELNN_F32 = 0, RELNN_BF16 = 1 } relnn_dtype;
typedef enum { RELNN_SUM = 0, RELNN_MEAN = 1, RELNN_MAX = 2 } relnn_agg;
typedef enum { RELNN_ACT_NONE = 0, RELNN_ACT_RELU = 1 } relnn_act;

/* ---------------------------------------------------------------- index */

/* A body atom R_j(key; z_j) (Section 2.1: content plus embedding).  Its
 * rows are matched to the link tuples whose column `col` equals the key. */
typedef struct {
  int64_t n_rows;          /* |R_j| */
  const int32_t* keys;     /* device [n_rows] primary key; NULL => dense ids
                              0..n_rows-1 (row = key) */
  int32_t col;             /* column of the joined link tuples holding the
                              FK (see relnn_join_desc for the numbering) */
} relnn_atom;

/* A derived column: for every link tuple, the value vals[r] of the row r of
 * a lookup relation whose key equals column src_col (an FK chain such as
 * Buys.item -> BelongsTo.cat).  A missing key drops the tuple. */
typedef struct {
  int32_t src_col;         /* link column or an earlier derived column */
  int64_t n_rows;
  const int32_t* keys;     /* device [n_rows]; NULL => dense */
  const int32_t* vals;     /* device [n_rows] */
} relnn_chain;

#define RELNN_IDX_BWD 1u   /* also build per-atom transpose CSRs (backward) */

/* A further link relation S joined into the link tuples built so far: the
 * natural join of Section 2.2 on one or two column pairs, bag semantics.
 * Every pair of a tuple and a row r of S with col[on[q]] == S.cols[key[q]][r]
 * for all q < n_on is a tuple, with S's columns appended after the columns
 * so far.  Chained steps give many-to-many joins; a step whose second pair
 * closes a cycle gives cyclic joins (the triangle Edge(n,v), Edge(v,w),
 * Edge(w,n) of the paper's DHN encoding, Section 5.2). */
typedef struct {
  int64_t n_rows;
  int32_t n_cols;
  const int32_t* const* cols;     /* host [n_cols] of device [n_rows] */
  int32_t n_on;                   /* 1 or 2 column pairs */
  int32_t on[2];                  /* columns of the tuples so far */
  int32_t key[2];                 /* columns of S */
} relnn_join_step;

typedef enum { RELNN_CMP_EQ = 0, RELNN_CMP_NE = 1, RELNN_CMP_LT = 2, RELNN_CMP_LE = 3,
               RELNN_CMP_GT = 4, RELNN_CMP_GE = 5 } relnn_cmp;

/* One atomic predicate e1 theta e2 of a filter expression (Section 3.1),
 * over the content variables of the joined tuples and constants, written as
 *     mul_a * col[a] + mul_b * col[b] + add   theta   0
 * in 64-bit two's-complement integer arithmetic (a or b = -1 leaves that
 * term out).  A filter is the conjunction of its predicates; the selection
 * (Section 2.2) keeps the tuples that satisfy it. */
typedef struct {
  int32_t a, b;
  int64_t mul_a, mul_b, add;
  int32_t op;                     /* relnn_cmp */
} relnn_pred;

/* The join of one rule: the link relation (bag semantics: every stored row
 * is a tuple), further link relations joined into it, its FK chains, its
 * body atoms in Concat order, a filter, and the head key (the projection
 * attribute of the projected union).
 *
 * Column numbering of the joined link tuples: the link relation's columns
 * 0..n_cols-1 (with two_hop: 0..2 n_cols-1, see relnn_build_index), then the
 * columns of each step in step order, then one derived column per chain in
 * chain order.  Chains may read any earlier column; atoms, the head key and
 * predicates any column. */
typedef struct {
  int64_t n_link;                 /* rows of the link relation */
  int32_t n_cols;                 /* its columns */
  const int32_t* const* cols;     /* host [n_cols] of device [n_link] */
  int32_t n_chains;
  const relnn_chain* chains;      /* host [n_chains] */
  int32_t n_atoms;                /* k, 1..RELNN_MAX_ATOMS */
  const relnn_atom* atoms;        /* host [k] */
  int32_t group_col;              /* column holding the head key */
  int32_t two_hop_mid;            /* -1, or the column on which the link
                                     relation is self-joined first */
  int32_t two_hop_cap;            /* paths kept per mid key (two-hop only) */
  uint32_t flags;                 /* RELNN_IDX_BWD */
  int32_t n_steps;                /* further link relations, joined in order */
  const relnn_join_step* steps;   /* host [n_steps] */
  int32_t n_preds;                /* filter expression: conjunction of */
  const relnn_pred* preds;        /* host [n_preds] predicates */
} relnn_join_desc;

#define RELNN_MAX_ATOMS 4

typedef struct relnn_index relnn_index;   /* opaque, device-resident */

/* Builds the join result in canonical order -- tuples sorted by (head key,
 * FK values of the atoms in body order, link row) -- and its group CSR:
 * group_keys[G] ascending, offsets[G+1], and per tuple the joined row of
 * every atom.  Dangling foreign keys drop the tuple (inner join); groups
 * with no tuple are absent (the output content is the set of head keys that
 * occur).  A duplicate key in a keyed atom or chain: RELNN_E_NOT_UNIQUE.
 *
 * Two-hop (two_hop_mid >= 0): the link relation is first self-joined on
 * column two_hop_mid.  For each mid key, its link rows are ordered by their
 * other columns then by link row (b_0..b_{n-1}), and path p < min(cap, n*n)
 * pairs b_i with b_j, i = p mod n, j = (i + 1 + p div n) mod n.  The path
 * relation has 2*n_cols columns: 0..n_cols-1 from b_i, n_cols.. from b_j;
 * atoms, chains and group_col refer to those.  "link row" then means the
 * path number (mid keys ascending, then p).
 *
 * Steps: each joined tuple extends one tuple so far by one row of S; the
 * joined link tuples are numbered in the order (link row or path number,
 * row of step 1's relation, row of step 2's ...), and "link row" means that
 * number.  The filter applies after the chains; a tuple that fails it is
 * dropped before the atoms are matched.  More than 2^31 - 1 joined link
 * tuples: RELNN_E_RANGE.
 *
 * Synchronises `stream`.  *out is owned by the caller through
 * relnn_index_free. */
relnn_status relnn_build_index(const relnn_join_desc* desc, relnn_stream_t stream,
                               relnn_index** out);

/* Sizes: joined tuples E, groups G, device bytes held by the index. */
relnn_status relnn_index_query(const relnn_index* idx, int64_t* n_tuples,
                               int64_t* n_groups, int64_t* dev_bytes);

/* Copies the canonical index into caller device buffers (any may be NULL):
 * group_keys[G], offsets[G+1], link_rows[E], tuple_rows[k*E] (atom-major:
 * tuple_rows[j*E + e] is the row of atom j joined to tuple e).  Async. */
relnn_status relnn_index_export(const relnn_index* idx, int32_t* group_keys,
                                int32_t* offsets, int32_t* link_rows,
                                int32_t* tuple_rows, relnn_stream_t stream);

relnn_status relnn_index_free(relnn_index* idx);

/* ---------------------------------------------------------------- layer */

#define RELNN_FUSED    0u  /* default: gather -> MFMA -> segmented reduce in
                              one pass, nothing [E, .] in HBM */
#define RELNN_PLAIN    1u  /* unfused pipeline: materialise X = [E, K], then
                              Y = [E, h], then reduce (comparison path) */
#define RELNN_DW_ACCUM 2u  /* backward adds into dW / db instead of writing */
#define RELNN_OUT_BF16 4u  /* forward writes `out` as bf16 (round to nearest
                              even) so it can feed a bf16 layer; `pre` stays
                              FP32 */
#define RELNN_PUSHDOWN 8u  /* forward with the transform pushed below the join
                              (Section 6's future-work rewrite: the transform
                              evaluated per node rather than per edge):
                              for act_pre = NONE, Linear(z_1 (+) ... (+) z_k)
                              = sum_j z_j W_j + b, so P_j = Z_j W_j is formed
                              once per atom row and each tuple sums P rows;
                              atoms whose key is a function of the head key,
                              and b, enter once per group.  Same results up
                              to rounding; needs act_pre = NONE (else
                              RELNN_E_INVALID), d_j a multiple of 4 (FP32) or
                              32 (BF16) and h <= 128 with h % 4 == 0 (else
                              RELNN_E_UNSUPPORTED); not with RELNN_PLAIN */

#define RELNN_TF_PRODUCT 16u /* transform tau = act_pre(z_1 * ... * z_k), the
                              elementwise product of the atoms' embeddings
                              (Section 1's Score rule q*k, Attention's a*v,
                              Section 5.4's gated mean z_e*z_w); every d_j
                              must equal h; W and b are not read (may be
                              NULL); relnn_layer_bwd gives the embedding
                              gradients only (W, b, dW, db not used; h even);
                              not with RELNN_PLAIN or RELNN_PUSHDOWN */

typedef struct {
  int32_t k;               /* body atoms, equal to the index's */
  const int32_t* d;        /* host [k] embedding widths, Concat order */
  int32_t h;               /* output width */
  int32_t dtype;           /* relnn_dtype of embeddings and W; accumulation,
                              bias, outputs and gradients are FP32 */
  int32_t agg;             /* relnn_agg */
  int32_t act_pre;         /* relnn_act inside tau, per joined tuple */
  int32_t act_post;        /* relnn_act after the aggregate */
  uint32_t flags;          /* RELNN_FUSED | RELNN_PLAIN | RELNN_PUSHDOWN,
                              RELNN_TF_PRODUCT, RELNN_DW_ACCUM,
                              RELNN_OUT_BF16 */
} relnn_layer_desc;

/* Workspace bytes relnn_layer_fwd (bwd = 0) or relnn_layer_bwd (bwd = 1)
 * needs for this index and layer. */
relnn_status relnn_workspace_size(const relnn_index* idx, const relnn_layer_desc* L,
                                  int bwd, size_t* bytes);

/* Forward.  emb: host [k] of device [n_j, d_j] row-major (dtype), 16-byte
 * aligned rows.  W: device [K, h] row-major (dtype), y = x W + b, K = sum
 * d_j (the transpose of nn.Linear.weight).  b: device [h] FP32 or NULL.
 * out: device [G, h] FP32 (bf16 with RELNN_OUT_BF16), row q is group
 * group_keys[q].  pre: device
 * [G, h] FP32 aggregate before act_post, or NULL (needed by the backward
 * when act_post != NONE).  argmax: device [G, h] int32 canonical tuple
 * position of the first maximiser, MAX only, or NULL (then the fused
 * kernels track values only; out and pre are the same bit for bit).  ws:
 * device workspace of relnn_workspace_size(.., 0) bytes. */
relnn_status relnn_layer_fwd(const relnn_index* idx, const relnn_layer_desc* L,
                             const void* const* emb, const void* W, const float* b,
                             float* out, float* pre, int32_t* argmax,
                             void* ws, size_t ws_bytes, relnn_stream_t stream);

/* Backward of sum(out * dout) through the forward above.  Needs an index
 * built with RELNN_IDX_BWD.  pre: the forward's pre (required when
 * act_post != NONE); argmax: the forward's argmax (required for MAX).
 * demb: host [k] of device [n_j, d_j] FP32, ACCUMULATED (+=); entries may
 * alias (a self-join adds both roles).  dW: device [K, h] FP32, written
 * (or added with RELNN_DW_ACCUM).  db: device [h] FP32 or NULL, same rule.
 * The joined tuples are re-gathered, not stored. */
relnn_status relnn_layer_bwd(const relnn_index* idx, const relnn_layer_desc* L,
                             const void* const* emb, const void* W, const float* b,
                             const float* pre, const int32_t* argmax, const float* dout,
                             float* const* demb, float* dW, float* db,
                             void* ws, size_t ws_bytes, relnn_stream_t stream);

/* Dense layout of an output (Section 2.2: the output content is the set of
 * head keys that occur, one compact row per group in key order).  dense
 * row key = compact row g for the group g with that key; the rows of keys
 * that do not occur are 0 and their present byte 0 (1 for the others).
 * keys: device [G] ascending distinct, e.g. relnn_index_export's
 * group_keys or relnn_union_export's keys; compact: device [G, h] FP32 (a
 * layer's or union's out or pre); dense: device [n_out, h] FP32; present:
 * device [n_out] uint8 or NULL.  Keys outside [0, n_out): RELNN_E_RANGE,
 * nothing written.  Reads the first and last key to the host, so it
 * synchronises `stream`. */
relnn_status relnn_out_dense(const int32_t* keys, int64_t G, const float* compact, int32_t h, int64_t n_out,
                             float* dense, uint8_t* present, relnn_stream_t stream);

/* ------------------------------------------------------------ attention */

/* Segmented softmax attention: the paper's attention as rules (Section 1,
 * Score(p,t; q*k) and Attention(p; sum(a*v)); Section 5.2, the HGT head with
 * a softmax over each target's tuples).  The index's three body atoms are
 * (Q, K, V); for every group g (head key) and head h:
 *
 *   s_tau   = scale * <q_h[r_Q(tau)], k_h[r_K(tau)]>     (q*k summed per head)
 *   a_tau   = exp(s_tau - max s) / sum exp(s - max s)    over the tuples of g
 *   out_g,h = sum_tau a_tau v_h[r_V(tau)]
 *   lse_g,h = log sum_tau exp(s_tau)
 *
 * d and dv <= 128, multiples of 4, split into `heads` blocks of a power of
 * two columns each. */
typedef struct {
  int32_t heads;
  int32_t d;          /* width of the Q and K rows */
  int32_t dv;         /* width of the V rows */
  float scale;        /* 1 / sqrt(d / heads) in the HGT head */
  int32_t dtype;      /* relnn_dtype of q, k, v; arithmetic and outputs FP32 */
} relnn_attn_desc;

relnn_status relnn_attn_workspace_size(const relnn_index* idx, const relnn_attn_desc* A, int bwd,
                                       size_t* bytes);

/* q: device [n_Q, d], k: [n_K, d], v: [n_V, dv] (dtype), rows of the
 * index's atoms 0, 1, 2.  out: device [G, dv] FP32; lse: device [G, heads]
 * FP32 or NULL (the backward needs it).  Async. */
relnn_status relnn_attn_fwd(const relnn_index* idx, const relnn_attn_desc* A, const void* q, const void* k,
                            const void* v, float* out, float* lse, void* ws, size_t ws_bytes,
                            relnn_stream_t stream);

/* Backward of sum(out * dout): dq, dk, dv device FP32 shaped as q, k, v,
 * ACCUMULATED (+=), may alias (K and V from one relation).  Needs an index
 * built with RELNN_IDX_BWD and the forward's out and lse. */
relnn_status relnn_attn_bwd(const relnn_index* idx, const relnn_attn_desc* A, const void* q, const void* k,
                            const void* v, const float* out, const float* lse, const float* dout, float* dq,
                            float* dk, float* dv, void* ws, size_t ws_bytes, relnn_stream_t stream);

/* ---------------------------------------------------------------- union */

/* The k-ary projected union (Section 2.2) of the join results of k rules
 * with one head, e.g. the several bodies of one head relation:
 *
 *     Out(g; act_post(tau_post(alpha(...))))  over  T_1(join_1) | ... | T_k(join_k)
 *
 * The output content is the set of head keys of all k indices (ascending);
 * the multiset of a key holds every joined tuple of every branch with that
 * key, each with its own branch's transform tau_i; alpha is applied once
 * over the whole multiset (MEAN is the sum over all members divided by
 * their number, not a mean of the branches' means).  A union rule
 * (Section 3.1) applies its transform after the union: tau_post(v) =
 * v W_post + b_post on each key's aggregate. */
#define RELNN_MAX_UNION 8

typedef struct relnn_union relnn_union;   /* opaque, device-resident */

/* Builds the union's keys and maps every branch group to its union row.
 * The branch indices stay caller-owned and must outlive the union.
 * Synchronises `stream`. */
relnn_status relnn_union_build(const relnn_index* const* branches, int32_t k, relnn_stream_t stream,
                               relnn_union** out);
relnn_status relnn_union_query(const relnn_union* u, int64_t* n_groups);
/* keys [G] ascending and counts [G] (members over all branches), device,
 * either may be NULL.  Async. */
relnn_status relnn_union_export(const relnn_union* u, int32_t* keys, int32_t* counts, relnn_stream_t stream);
relnn_status relnn_union_free(relnn_union* u);

/* Workspace bytes of relnn_union_fwd for these branch layers. */
relnn_status relnn_union_workspace_size(const relnn_union* u, const relnn_layer_desc* const* L, int32_t agg,
                                        size_t* bytes);

/* Forward.  L: host [k] layer descriptors of the branches (widths, dtype,
 * act_pre; all the same h; their agg and act_post are not used; flags may
 * hold RELNN_FUSED and RELNN_DW_ACCUM, the latter used by the backward
 * only).  agg: the union's aggregate (SUM, MEAN, MAX).  emb: host [k] of
 * the branch's host [k_i] device embedding pointers; W: host [k] device
 * [K_i, h]; b: host [k] of device [h] or NULL (or b NULL).  W_post: device
 * [h, h_out] FP32 row-major or NULL (then h_out = h); b_post: device
 * [h_out] or NULL.  out: device [G, h_out] FP32 =
 * act_post(tau_post(aggregate)); pre: device [G, h] FP32 aggregate or NULL.
 * argmax: MAX only, device [G, h] int32 or NULL: the first maximiser of
 * each column in (branch, position) order, as a position in the
 * concatenation of the branches' canonical tuple orders (branch i's
 * positions start at E_0 + ... + E_{i-1}); -1 where no value is larger
 * than -Inf.  Row u is the union's key u. */
relnn_status relnn_union_fwd(const relnn_union* u, const relnn_layer_desc* const* L, int32_t agg,
                             int32_t act_post, const void* const* const* emb, const void* const* W,
                             const float* const* b, const float* W_post, const float* b_post, int32_t h_out,
                             float* out, float* pre, int32_t* argmax, void* ws, size_t ws_bytes,
                             relnn_stream_t stream);

/* Workspace bytes of relnn_union_bwd for these branch layers and h_out. */
relnn_status relnn_union_bwd_workspace_size(const relnn_union* u, const relnn_layer_desc* const* L, int32_t agg,
                                            int32_t h_out, size_t* bytes);

/* Backward of sum(out * dout) through relnn_union_fwd (chain rule,
 * Sections 2.2-2.3 and 3.1): with u = v W_post + b_post, dU = dout *
 * act_post'(u), dW_post = v^T dU, db_post = sum over keys of dU, dV = dU
 * W_post^T (without W_post, dV = dout * act_post'(v)).  Each tuple of
 * branch i with key t then receives dV[t] (SUM), dV[t] / members(t)
 * (MEAN), or the columns of dV[t] it maximises (MAX, from argmax), and
 * branch i's layer backward takes it to the branch's weights and
 * embeddings.  Arguments as in the forward, plus: pre, the forward's
 * aggregate (required with W_post or act_post); argmax, the forward's
 * (required for MAX); dout device [G, h_out] FP32; demb: host [k] of host
 * [k_i] device FP32 gradients shaped as emb, ACCUMULATED (+=), may alias;
 * dW: host [k] of device [K_i, h] FP32, written (added with RELNN_DW_ACCUM
 * in L[i]->flags, so branches sharing one W can share one dW); db: host
 * [k] of device [h] or NULL (or db NULL), same rule; dW_post device [h,
 * h_out] FP32, written (required with W_post); db_post device [h_out] or
 * NULL.  Every branch index needs RELNN_IDX_BWD.  With W_post, h and h_out
 * must be multiples of 4, at most 1024 (RELNN_E_UNSUPPORTED). */
relnn_status relnn_union_bwd(const relnn_union* u, const relnn_layer_desc* const* L, int32_t agg,
                             int32_t act_post, const void* const* const* emb, const void* const* W,
                             const float* const* b, const float* W_post, const float* b_post, int32_t h_out,
                             const float* pre, const int32_t* argmax, const float* dout,
                             float* const* const* demb, float* const* dW, float* const* db, float* dW_post,
                             float* db_post, void* ws, size_t ws_bytes, relnn_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * forward of relnn_layer_fwd with the same arguments except the workspace.
 * Its workspace is a static device array of relnn_static_scratch_bytes()
 * bytes (32 MiB) on each GPU the library runs on, held until the process
 * ends; no call allocates or frees anything.  A layer whose workspace
 * (relnn_workspace_size(.., 0)) exceeds the array: RELNN_E_RANGE, nothing
 * launched.  RELNN_PLAIN (a library GEMM, which may allocate):
 * RELNN_E_UNSUPPORTED.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other threads) race and
 * must be serialised by the caller.  Nothing in the array has to start
 * at zero; it keeps the last call's contents.  Results equal those of
 * relnn_layer_fwd bit for bit. */
relnn_status relnn_static_scratch_bytes(size_t* bytes);
relnn_status relnn_layer_fwd_static(const relnn_index* idx, const relnn_layer_desc* L,
                                    const void* const* emb, const void* W, const float* b,
                                    float* out, float* pre, int32_t* argmax, relnn_stream_t stream);

/* ---------------------------------------------------------------- serve */

/* Serving of the two-layer ER network on sampled neighbourhoods.  The
 * paper trains whole graphs; sampling and mini-batches are its stated
 * future work (Section 6).  A request is a set of seed Items and a seed for
 * the sampler; its result is one h-wide embedding per seed:
 *
 *   hop 1: for each seed item s, up to fanout1 of its buyers (Buys rows
 *          with item = s, ordered by user then row), without replacement;
 *   hop 2: for each sampled buyer u, up to fanout2 of u's Buys rows
 *          (ordered by item then row);
 *   layer 1: User'(u)  = ReLU(MEAN over u's hop-2 rows of Lin_U(z_u (+) z_i)),
 *            Item'(s)  = ReLU(SUM over s's hop-1 rows of Lin_I1(z_u (+) z_s (+) z_c(s)));
 *   layer 2: out(s)    = ReLU(SUM over s's hop-1 rows of
 *                             Lin_I2(User'(u) (+) Item'(s) (+) z_c(s))).
 *
 * Each join above is the layer of relnn_layer_fwd on the sampled link
 * rows; a User' value is computed for every hop-1 row that samples u (the
 * sampler is keyed by (request seed, hop, node), so copies agree).
 * Sampling: k of n positions by Floyd's algorithm; draw number q of the
 * stream for (req_seed, hop, node) is SplitMix64's output function applied
 * to base + (q + 1) * 0x9E3779B97F4A7C15, base = mix(req_seed +
 * (2 * node + hop + 1) * 0x9E3779B97F4A7C15); a draw r in [0, j] is
 * ((r >> 32) * (j + 1)) >> 32.  The sampled positions are sorted.
 *
 * Continuous batching: a scheduler thread runs steps back to back; each
 * step admits waiting requests in arrival order while their seeds fit the
 * step's capacity (sized from budget_bytes) and max_slots, runs one
 * captured hipGraph over all of them, and completes them together.
 * Requests that arrive during a step join a later step. */
typedef struct {
  int64_t n_user, n_item, n_cat, n_buys;
  const int32_t* buys_user;        /* device [n_buys] Buys.user (dense ids) */
  const int32_t* buys_item;        /* device [n_buys] Buys.item */
  const int32_t* item_cat;         /* device [n_item] BelongsTo.cat */
  const void* user_emb;            /* device [n_user, d] (dtype) */
  const void* item_emb;            /* device [n_item, d] */
  const void* cat_emb;             /* device [n_cat, d] */
  int32_t d, h;                    /* input and hidden width (d == h) */
  const void* W_user;              /* device [2d, h] layer-1 User rule */
  const void* W_item1;             /* device [3d, h] layer-1 Item rule */
  const void* W_item2;             /* device [2h + d, h] layer-2 Item rule */
  const float* b_user;             /* device [h] or NULL (each bias) */
  const float* b_item1;
  const float* b_item2;
  int32_t fanout1, fanout2;        /* 1..32 each (15 and 10) */
  int32_t dtype;                   /* relnn_dtype of embeddings and weights */
  int32_t max_seeds;               /* largest request (seeds) */
  int32_t max_slots;               /* requests per step */
  size_t budget_bytes;             /* device bytes for in-flight work */
} relnn_serve_desc;

typedef struct {
  int64_t t_arrive_ns;             /* submit (steady clock) */
  int64_t t_admit_ns;              /* its step started */
  int64_t t_done_ns;               /* its step's results were on the host */
  int64_t tuples;                  /* joined tuples evaluated for it */
  int64_t step;                    /* step number it ran in */
  int32_t n_seeds;
} relnn_req_stats;

typedef struct relnn_server relnn_server;

/* Builds the item and user adjacency (CSR) of Buys on the device, swizzles
 * the weights and allocates the step buffers (library-owned, counted
 * against budget_bytes), then starts the scheduler thread.  The resident
 * relations and weights stay caller-owned and must outlive the server.
 * RELNN_E_OOM if budget_bytes cannot hold one largest request. */
relnn_status relnn_serve_create(const relnn_serve_desc* desc, relnn_server** out);

/* Queues a request: seeds host [n] distinct item ids (an id outside
 * 0..n_item-1 has no neighbourhood and no output), 1 <= n <= max_seeds.
 * Returns a ticket at once.  RELNN_E_RANGE if n is out of range,
 * RELNN_E_BUSY if the queue is full. */
relnn_status relnn_serve_submit(relnn_server* srv, const int32_t* seeds, int32_t n, uint64_t req_seed,
                                uint64_t* ticket);

/* Non-blocking.  RELNN_E_NOT_READY until the request's step is done; then
 * fills out host [n, h] FP32, present host [n] (0 for a seed with no
 * buyer: its row is zero) and stats (any may be NULL) and forgets the
 * ticket.  RELNN_E_INVALID for an unknown ticket. */
relnn_status relnn_serve_poll(relnn_server* srv, uint64_t ticket, float* out, uint8_t* present,
                              relnn_req_stats* stats);

/* Cancels a request: a request still queued is removed and never runs; one
 * already taken into the running step finishes there and its result is
 * dropped; a finished one not yet polled is forgotten.  Either way the
 * ticket is unknown afterwards (poll and cancel: RELNN_E_INVALID).
 * was_admitted (may be NULL) receives 1 if the request had been taken into
 * a step (its work was spent), else 0.  RELNN_E_INVALID for an unknown
 * ticket. */
relnn_status relnn_serve_cancel(relnn_server* srv, uint64_t ticket, int32_t* was_admitted);

/* Stops the scheduler after the step in flight and frees everything the
 * server owns.  Requests not yet polled are dropped. */
relnn_status relnn_serve_destroy(relnn_server* srv);

/* ---------------------------------------------------------------- timing */

/* Measurement hooks.  While enabled, each main kernel launch of the layer
 * calls is bracketed by HIP events on its own stream, under a class name:
 * "fwd_fused", "fwd_gather", "fwd_gemm", "fwd_reduce", "bwd_dx", "bwd_dw".
 * relnn_timing_read waits for the recorded launches of one class and
 * returns their summed milliseconds and count; relnn_timing_reset drops
 * the records.  Process-wide; not for use inside graph capture. */
relnn_status relnn_timing_enable(int on);
relnn_status relnn_timing_reset(void);
relnn_status relnn_timing_read(const char* kernel, double* total_ms, int64_t* launches);

const char* relnn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RELNN_H */
