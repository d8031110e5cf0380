// Index build: the join of a rule in canonical order plus its group CSR.
//
// Join (Section 2.2): every link tuple is matched to one row of each body
// atom by FK -> PK equality; FK chains add derived columns first.  A
// missing key drops the tuple (inner join).  The projected union (Section
// 2.2) groups the joined tuples by the head key; its content is the set of
// keys that occur, so empty groups never appear.
//
// Further link relations (general, many-to-many and cyclic joins) are joined
// by sort-and-probe: the relation's rows are radix-sorted by their key
// columns, every tuple so far finds its range of matches by binary search on
// the key pair, the counts are scanned, and one pass writes for every output
// tuple the tuple it extends and the matching row.  A filter (the selection
// of Section 3.1) clears the valid flag of the tuples that fail it, before
// the compaction.
//
// GPU plan: key tables of keyed relations are radix-sorted and probed by
// binary search; dense relations are direct-addressed.  Valid tuples are
// compacted by a scan, then put in canonical order by a stable LSD radix
// sort over (FK values of the atoms in reverse body order, then the head
// key), starting from link-row order so ties keep it.  Columns that are
// functions of the head key (the head column itself, or a chain off it) and
// repeated columns cannot change the order and are skipped.
#include <memory>
#include <vector>

#include "index.hpp"
#include "prims.hpp"

using namespace relnn;

namespace {

struct KeyTable {
  bool dense = true;
  int64_t n = 0;
  DevBuf ukeys;   // sorted (key ^ 0x80000000)
  DevBuf rows;    // row of each sorted key
};

__global__ void k_check_dup(const uint32_t* sk, int64_t n, int32_t* flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (sk[i] == sk[i - 1]) *flag = 1;
}

unsigned grid_for(int64_t n) {
  int64_t g = cdiv(n, 256);
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

void make_table(const int32_t* keys, int64_t n_rows, KeyTable& t, hipStream_t s, const char* what) {
  t.n = n_rows;
  t.dense = keys == nullptr;
  if (t.dense || n_rows == 0) return;
  t.ukeys.alloc(n_rows * sizeof(uint32_t));
  t.rows.alloc(n_rows * sizeof(int32_t));
  prim::make_keys(keys, nullptr, n_rows, 0u, t.ukeys.as<uint32_t>(), s);
  prim::iota_i32(t.rows.as<int32_t>(), n_rows, s);
  DevBuf tk(n_rows * sizeof(uint32_t)), tv(n_rows * sizeof(int32_t));
  prim::radix_sort_pairs(t.ukeys.as<uint32_t>(), t.rows.as<int32_t>(), tk.as<uint32_t>(),
                         tv.as<int32_t>(), n_rows, 32, s);
  DevBuf flag(sizeof(int32_t));
  RELNN_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
  k_check_dup<<<grid_for(n_rows), 256, 0, s>>>(t.ukeys.as<uint32_t>(), n_rows, flag.as<int32_t>());
  RELNN_LAUNCHED();
  int32_t dup = 0;
  RELNN_HIP(hipMemcpyAsync(&dup, flag.p, sizeof(dup), hipMemcpyDeviceToHost, s));
  RELNN_HIP(hipStreamSynchronize(s));
  RELNN_REQUIRE(!dup, RELNN_E_NOT_UNIQUE, "%s has a duplicate primary key", what);
}

// out[i] = row (or vals[row]) of the relation row whose key equals v[i];
// a missing key clears valid[i].
__global__ void k_lookup(const int32_t* v, int64_t n, int64_t n_rows, const uint32_t* sk,
                         const int32_t* srows, const int32_t* vals, int32_t* out, uint8_t* valid) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t key = v[i];
    int64_t r = -1;
    if (sk == nullptr) {
      if (key >= 0 && (int64_t)key < n_rows) r = key;
    } else {
      const uint32_t u = (uint32_t)key ^ 0x80000000u;
      int64_t lo = 0, hi = n_rows;
      while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (sk[mid] < u) lo = mid + 1; else hi = mid;
      }
      if (lo < n_rows && sk[lo] == u) r = srows[lo];
    }
    if (r < 0) {
      valid[i] = 0;
      out[i] = 0;
    } else {
      out[i] = vals ? vals[r] : (int32_t)r;
    }
  }
}

void lookup(const int32_t* v, int64_t n, const KeyTable& t, const int32_t* vals, int32_t* out,
            uint8_t* valid, hipStream_t s) {
  if (n <= 0) return;
  k_lookup<<<grid_for(n), 256, 0, s>>>(v, n, t.n, t.dense ? nullptr : t.ukeys.as<uint32_t>(),
                                       t.dense ? nullptr : t.rows.as<int32_t>(), vals, out, valid);
  RELNN_LAUNCHED();
}

__global__ void k_compact(const uint8_t* valid, const int32_t* pos, int64_t n, int32_t* perm) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (valid[i]) perm[pos[i]] = (int32_t)i;
}

// Stable sort of perm by column col (values gathered through perm).
void sort_by_column(const int32_t* col, int32_t* perm, int64_t n, hipStream_t s) {
  if (n <= 1) return;
  uint32_t kmin, kmax;
  prim::key_range(col, perm, n, &kmin, &kmax, s);
  const int bits = prim::bits_for((uint64_t)(kmax - kmin));
  if (bits == 0) return;
  DevBuf keys(n * sizeof(uint32_t)), tk(n * sizeof(uint32_t)), tv(n * sizeof(int32_t));
  prim::make_keys(col, perm, n, kmin, keys.as<uint32_t>(), s);
  prim::radix_sort_pairs(keys.as<uint32_t>(), perm, tk.as<uint32_t>(), tv.as<int32_t>(), n, bits, s);
}

__global__ void k_path_counts(const int32_t* offs, int64_t nseg, int64_t cap, int64_t* cnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nseg;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = offs[i + 1] - offs[i];
    cnt[i] = std::min<int64_t>(cap, m * m);
  }
}

// Path p of mid segment s: rows b_i, b_j of the segment with
// i = q mod m, j = (i + 1 + q div m) mod m, q = p - poff[s].
__global__ void k_paths(const int32_t* offs, const int64_t* poff, int64_t nseg, const int32_t* perm,
                        int64_t P, int32_t* la, int32_t* lb) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = nseg;          // last s with poff[s] <= p
    while (hi - lo > 1) {
      int64_t mid = (lo + hi) >> 1;
      if (poff[mid] <= p) lo = mid; else hi = mid;
    }
    const int64_t q = p - poff[lo];
    const int64_t m = offs[lo + 1] - offs[lo];
    const int64_t i = q % m;
    const int64_t j = (i + 1 + q / m) % m;
    la[p] = perm[offs[lo] + i];
    lb[p] = perm[offs[lo] + j];
  }
}

__global__ void k_fill_u8(uint8_t* p, int64_t n, uint8_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

using BufList = std::vector<std::unique_ptr<DevBuf>>;

int32_t* new_buf(BufList& owned, int64_t n) {
  owned.emplace_back(new DevBuf((size_t)std::max<int64_t>(n, 1) * sizeof(int32_t)));
  return owned.back()->as<int32_t>();
}

// Self-join of the link relation on column `mid` (two-hop paths).
int64_t expand_two_hop(std::vector<const int32_t*>& col, int64_t n_link, int mid, int64_t cap,
                       BufList& owned, hipStream_t s) {
  const int nc = (int)col.size();
  DevBuf perm(std::max<int64_t>(n_link, 1) * sizeof(int32_t));
  prim::iota_i32(perm.as<int32_t>(), n_link, s);
  for (int c = nc - 1; c >= 0; --c)
    if (c != mid) sort_by_column(col[c], perm.as<int32_t>(), n_link, s);
  sort_by_column(col[mid], perm.as<int32_t>(), n_link, s);
  DevBuf smid(std::max<int64_t>(n_link, 1) * sizeof(int32_t));
  DevBuf seg_of(std::max<int64_t>(n_link, 1) * sizeof(int32_t));
  DevBuf offs((n_link + 1) * sizeof(int32_t));
  prim::gather_i32(col[mid], perm.as<int32_t>(), n_link, smid.as<int32_t>(), s);
  const int64_t nseg = prim::segments(smid.as<int32_t>(), n_link, seg_of.as<int32_t>(),
                                      offs.as<int32_t>(), nullptr, s);
  DevBuf cnt(std::max<int64_t>(nseg, 1) * sizeof(int64_t)), poff(std::max<int64_t>(nseg, 1) * sizeof(int64_t));
  int64_t P = 0;
  if (nseg > 0) {
    k_path_counts<<<grid_for(nseg), 256, 0, s>>>(offs.as<int32_t>(), nseg, cap, cnt.as<int64_t>());
    RELNN_LAUNCHED();
    prim::scan_i64(cnt.as<int64_t>(), nseg, poff.as<int64_t>(), &P, s);
  }
  RELNN_REQUIRE(P < (int64_t)INT32_MAX, RELNN_E_RANGE, "two-hop path count %lld exceeds 2^31",
                (long long)P);
  int32_t* la = new_buf(owned, P);
  int32_t* lb = new_buf(owned, P);
  if (P > 0) {
    k_paths<<<grid_for(P), 256, 0, s>>>(offs.as<int32_t>(), poff.as<int64_t>(), nseg,
                                         perm.as<int32_t>(), P, la, lb);
    RELNN_LAUNCHED();
  }
  std::vector<const int32_t*> out(2 * nc);
  for (int c = 0; c < nc; ++c) {
    int32_t* a = new_buf(owned, P);
    int32_t* b = new_buf(owned, P);
    prim::gather_i32(col[c], la, P, a, s);
    prim::gather_i32(col[c], lb, P, b, s);
    out[c] = a;
    out[nc + c] = b;
  }
  RELNN_HIP(hipStreamSynchronize(s));
  col = out;
  return P;
}

// Range [lo, lo + cnt) of the rows of S (sorted by (k0, k1)) whose key pair
// equals (v0[i], v1[i]) (k1 / v1 null: one column).
__global__ void k_probe(const int32_t* v0, const int32_t* v1, int64_t n, const int32_t* k0, const int32_t* k1,
                        int64_t ns, int32_t* lo_out, int64_t* cnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = v0[i];
    const int32_t b = v1 ? v1[i] : 0;
    auto less = [&](int64_t m, bool upper) {      // key[m] < (a, b), or <= for the upper bound
      const int32_t x = k0[m];
      if (x != a) return x < a;
      if (!k1) return upper;
      const int32_t y = k1[m];
      return upper ? y <= b : y < b;
    };
    int64_t lo = 0, hi = ns;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (less(mid, false)) lo = mid + 1; else hi = mid;
    }
    int64_t lo2 = lo, hi2 = ns;
    while (lo2 < hi2) {
      const int64_t mid = (lo2 + hi2) >> 1;
      if (less(mid, true)) lo2 = mid + 1; else hi2 = mid;
    }
    lo_out[i] = (int32_t)lo;
    cnt[i] = lo2 - lo;
  }
}

// Output tuple p extends tuple i (the last i with off[i] <= p) with row
// perm[lo[i] + p - off[i]] of S.
__global__ void k_expand(const int64_t* off, const int32_t* lo, int64_t n, const int32_t* perm, int64_t P,
                         int32_t* src, int32_t* srow) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    int64_t a = 0, b = n;
    while (b - a > 1) {
      const int64_t mid = (a + b) >> 1;
      if (off[mid] <= p) a = mid; else b = mid;
    }
    src[p] = (int32_t)a;
    srow[p] = perm[lo[a] + (p - off[a])];
  }
}

// Joins further link relation st into the tuples so far (n of them, columns
// col); col and n are replaced by the joined tuples.
int64_t expand_step(std::vector<const int32_t*>& col, int64_t n, const relnn_join_step& st, BufList& owned,
                    hipStream_t s) {
  const int64_t ns = st.n_rows;
  std::vector<const int32_t*> out;
  if (n == 0 || ns == 0) {
    for (size_t c = 0; c < col.size() + (size_t)st.n_cols; ++c) out.push_back(new_buf(owned, 0));
    col = out;
    return 0;
  }
  // rows of S sorted by (key0, key1, row): stable passes, least significant first
  DevBuf perm(ns * sizeof(int32_t));
  prim::iota_i32(perm.as<int32_t>(), ns, s);
  if (st.n_on == 2) sort_by_column(st.cols[st.key[1]], perm.as<int32_t>(), ns, s);
  sort_by_column(st.cols[st.key[0]], perm.as<int32_t>(), ns, s);
  DevBuf k0(ns * sizeof(int32_t)), k1(st.n_on == 2 ? ns * sizeof(int32_t) : 0);
  prim::gather_i32(st.cols[st.key[0]], perm.as<int32_t>(), ns, k0.as<int32_t>(), s);
  if (st.n_on == 2) prim::gather_i32(st.cols[st.key[1]], perm.as<int32_t>(), ns, k1.as<int32_t>(), s);
  DevBuf lo(n * sizeof(int32_t)), cnt(n * sizeof(int64_t)), off(n * sizeof(int64_t));
  k_probe<<<grid_for(n), 256, 0, s>>>(col[st.on[0]], st.n_on == 2 ? col[st.on[1]] : nullptr, n, k0.as<int32_t>(),
                                      st.n_on == 2 ? k1.as<int32_t>() : nullptr, ns, lo.as<int32_t>(),
                                      cnt.as<int64_t>());
  RELNN_LAUNCHED();
  int64_t P = 0;
  prim::scan_i64(cnt.as<int64_t>(), n, off.as<int64_t>(), &P, s);
  RELNN_REQUIRE(P < (int64_t)INT32_MAX, RELNN_E_RANGE, "joined link tuples %lld exceed 2^31 - 1", (long long)P);
  DevBuf src(std::max<int64_t>(P, 1) * sizeof(int32_t)), srow(std::max<int64_t>(P, 1) * sizeof(int32_t));
  if (P > 0) {
    k_expand<<<grid_for(P), 256, 0, s>>>(off.as<int64_t>(), lo.as<int32_t>(), n, perm.as<int32_t>(), P,
                                         src.as<int32_t>(), srow.as<int32_t>());
    RELNN_LAUNCHED();
  }
  for (const int32_t* c : col) {
    int32_t* a = new_buf(owned, P);
    prim::gather_i32(c, src.as<int32_t>(), P, a, s);
    out.push_back(a);
  }
  for (int c = 0; c < st.n_cols; ++c) {
    int32_t* a = new_buf(owned, P);
    prim::gather_i32(st.cols[c], srow.as<int32_t>(), P, a, s);
    out.push_back(a);
  }
  RELNN_HIP(hipStreamSynchronize(s));
  col = out;
  return P;
}

// valid[i] &= (mul_a ca[i] + mul_b cb[i] + add) op 0, in int64 arithmetic
// (wrapping as two's complement).
__global__ void k_pred(const int32_t* ca, const int32_t* cb, int64_t mul_a, int64_t mul_b, int64_t add, int op,
                       int64_t n, uint8_t* valid) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t v = (uint64_t)add;
    if (ca) v += (uint64_t)mul_a * (uint64_t)(int64_t)ca[i];
    if (cb) v += (uint64_t)mul_b * (uint64_t)(int64_t)cb[i];
    const int64_t x = (int64_t)v;
    bool ok;
    switch (op) {
      case RELNN_CMP_EQ: ok = x == 0; break;
      case RELNN_CMP_NE: ok = x != 0; break;
      case RELNN_CMP_LT: ok = x < 0; break;
      case RELNN_CMP_LE: ok = x <= 0; break;
      case RELNN_CMP_GT: ok = x > 0; break;
      default: ok = x >= 0; break;
    }
    if (!ok) valid[i] = 0;
  }
}

void validate(const relnn_join_desc* D) {
  RELNN_REQUIRE(D != nullptr, RELNN_E_INVALID, "join descriptor is NULL");
  RELNN_REQUIRE(D->n_link >= 0 && D->n_link < (int64_t)INT32_MAX, RELNN_E_RANGE,
                "n_link %lld out of range", (long long)D->n_link);
  RELNN_REQUIRE(D->n_cols >= 1 && D->cols != nullptr, RELNN_E_INVALID, "link relation has no columns");
  for (int c = 0; c < D->n_cols; ++c)
    RELNN_REQUIRE(D->cols[c] != nullptr || D->n_link == 0, RELNN_E_INVALID, "link column %d is NULL", c);
  const bool two = D->two_hop_mid >= 0;
  if (two) {
    RELNN_REQUIRE(D->two_hop_mid < D->n_cols, RELNN_E_INVALID, "two_hop_mid out of range");
    RELNN_REQUIRE(D->two_hop_cap >= 1, RELNN_E_INVALID, "two_hop_cap must be >= 1");
  }
  int base = two ? 2 * D->n_cols : D->n_cols;
  RELNN_REQUIRE(D->n_steps >= 0 && (D->n_steps == 0 || D->steps != nullptr), RELNN_E_INVALID, "steps NULL");
  for (int i = 0; i < D->n_steps; ++i) {
    const relnn_join_step& st = D->steps[i];
    RELNN_REQUIRE(st.n_rows >= 0 && st.n_rows < (int64_t)INT32_MAX, RELNN_E_RANGE, "step %d n_rows", i);
    RELNN_REQUIRE(st.n_cols >= 1 && st.cols != nullptr, RELNN_E_INVALID, "step %d has no columns", i);
    for (int c = 0; c < st.n_cols; ++c)
      RELNN_REQUIRE(st.cols[c] != nullptr || st.n_rows == 0, RELNN_E_INVALID, "step %d column %d is NULL", i, c);
    RELNN_REQUIRE(st.n_on == 1 || st.n_on == 2, RELNN_E_INVALID, "step %d: n_on must be 1 or 2", i);
    for (int q = 0; q < st.n_on; ++q) {
      RELNN_REQUIRE(st.on[q] >= 0 && st.on[q] < base, RELNN_E_INVALID, "step %d on[%d] out of range", i, q);
      RELNN_REQUIRE(st.key[q] >= 0 && st.key[q] < st.n_cols, RELNN_E_INVALID, "step %d key[%d] out of range", i, q);
    }
    base += st.n_cols;
  }
  RELNN_REQUIRE(D->n_chains >= 0 && (D->n_chains == 0 || D->chains != nullptr), RELNN_E_INVALID,
                "chains NULL");
  for (int i = 0; i < D->n_chains; ++i) {
    const relnn_chain& ch = D->chains[i];
    RELNN_REQUIRE(ch.src_col >= 0 && ch.src_col < base + i, RELNN_E_INVALID,
                  "chain %d src_col %d out of range", i, ch.src_col);
    RELNN_REQUIRE(ch.n_rows >= 0 && ch.n_rows < (int64_t)INT32_MAX, RELNN_E_RANGE, "chain %d n_rows", i);
    RELNN_REQUIRE(ch.vals != nullptr || ch.n_rows == 0, RELNN_E_INVALID, "chain %d vals NULL", i);
  }
  const int ncol = base + D->n_chains;
  RELNN_REQUIRE(D->n_atoms >= 1 && D->n_atoms <= RELNN_MAX_ATOMS && D->atoms != nullptr,
                RELNN_E_INVALID, "n_atoms must be 1..%d", RELNN_MAX_ATOMS);
  for (int j = 0; j < D->n_atoms; ++j) {
    const relnn_atom& a = D->atoms[j];
    RELNN_REQUIRE(a.col >= 0 && a.col < ncol, RELNN_E_INVALID, "atom %d col %d out of range", j, a.col);
    RELNN_REQUIRE(a.n_rows >= 0 && a.n_rows < (int64_t)INT32_MAX, RELNN_E_RANGE, "atom %d n_rows", j);
  }
  RELNN_REQUIRE(D->group_col >= 0 && D->group_col < ncol, RELNN_E_INVALID, "group_col out of range");
  RELNN_REQUIRE(D->n_preds >= 0 && (D->n_preds == 0 || D->preds != nullptr), RELNN_E_INVALID, "preds NULL");
  for (int i = 0; i < D->n_preds; ++i) {
    const relnn_pred& p = D->preds[i];
    RELNN_REQUIRE(p.a >= -1 && p.a < ncol && p.b >= -1 && p.b < ncol, RELNN_E_INVALID,
                  "predicate %d column out of range", i);
    RELNN_REQUIRE(p.op >= RELNN_CMP_EQ && p.op <= RELNN_CMP_GE, RELNN_E_INVALID, "predicate %d: unknown op", i);
  }
  RELNN_REQUIRE((D->flags & ~RELNN_IDX_BWD) == 0, RELNN_E_INVALID, "unknown index flags");
}

}  // namespace

extern "C" relnn_status relnn_build_index(const relnn_join_desc* D, relnn_stream_t stream,
                                          relnn_index** out) {
  return guard([&] {
    RELNN_REQUIRE(out != nullptr, RELNN_E_INVALID, "out is NULL");
    *out = nullptr;
    validate(D);
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<relnn_index> idx(new relnn_index());
    RELNN_HIP(hipGetDevice(&idx->device));
    idx->k = D->n_atoms;
    BufList owned;

    std::vector<const int32_t*> col(D->cols, D->cols + D->n_cols);
    int64_t n = D->n_link;
    if (D->two_hop_mid >= 0 && n > 0)
      n = expand_two_hop(col, n, D->two_hop_mid, D->two_hop_cap, owned, s);
    else if (D->two_hop_mid >= 0)
      col.resize(2 * D->n_cols, nullptr);
    for (int i = 0; i < D->n_steps; ++i) {
      if (n > 0) {
        n = expand_step(col, n, D->steps[i], owned, s);
      } else {
        for (int c = 0; c < D->steps[i].n_cols; ++c) col.push_back(nullptr);
      }
    }
    const int base = (int)col.size();
    std::vector<bool> fd(base + D->n_chains, false);   // functionally dependent on the head key

    DevBuf valid(std::max<int64_t>(n, 1));
    if (n > 0) {
      k_fill_u8<<<grid_for(n), 256, 0, s>>>(valid.as<uint8_t>(), n, 1);
      RELNN_LAUNCHED();
    }
    for (int i = 0; i < D->n_chains; ++i) {
      const relnn_chain& ch = D->chains[i];
      KeyTable t;
      make_table(ch.keys, ch.n_rows, t, s, "a chain relation");
      int32_t* dcol = new_buf(owned, n);
      lookup(col[ch.src_col], n, t, ch.vals, dcol, valid.as<uint8_t>(), s);
      RELNN_HIP(hipStreamSynchronize(s));
      col.push_back(dcol);
    }
    for (int i = 0; i < D->n_preds && n > 0; ++i) {      // the filter: a conjunction
      const relnn_pred& p = D->preds[i];
      k_pred<<<grid_for(n), 256, 0, s>>>(p.a >= 0 ? col[p.a] : nullptr, p.b >= 0 ? col[p.b] : nullptr, p.mul_a,
                                         p.mul_b, p.add, p.op, n, valid.as<uint8_t>());
      RELNN_LAUNCHED();
    }
    for (int c = 0; c < (int)fd.size(); ++c) {
      fd[c] = (c == D->group_col);
      if (c >= base) fd[c] = fd[c] || fd[D->chains[c - base].src_col];
    }
    std::vector<int32_t*> rowsL(D->n_atoms);
    for (int j = 0; j < D->n_atoms; ++j) {
      const relnn_atom& a = D->atoms[j];
      idx->n_rows[j] = a.n_rows;
      KeyTable t;
      make_table(a.keys, a.n_rows, t, s, "a body atom");
      rowsL[j] = new_buf(owned, n);
      lookup(col[a.col], n, t, nullptr, rowsL[j], valid.as<uint8_t>(), s);
      RELNN_HIP(hipStreamSynchronize(s));
    }

    // compact the surviving tuples in link-row order
    DevBuf pos(std::max<int64_t>(n, 1) * sizeof(int32_t));
    int64_t E = 0;
    prim::scan_u8(valid.as<uint8_t>(), n, pos.as<int32_t>(), &E, s);
    idx->E = E;
    int32_t* perm = idx->alloc<int32_t>(E);
    if (n > 0) {
      k_compact<<<grid_for(n), 256, 0, s>>>(valid.as<uint8_t>(), pos.as<int32_t>(), n, perm);
      RELNN_LAUNCHED();
    }

    // canonical order: LSD over atom FK columns (reverse body order), then head key
    for (int j = 0; j < D->n_atoms; ++j) {
      idx->atom_fd[j] = fd[D->atoms[j].col];
      idx->atom_gk[j] = D->atoms[j].col == D->group_col;
    }
    std::vector<int> order;
    for (int j = 0; j < D->n_atoms; ++j) {
      const int c = D->atoms[j].col;
      if (fd[c] || std::find(order.begin(), order.end(), c) != order.end()) continue;
      order.push_back(c);
    }
    for (auto it = order.rbegin(); it != order.rend(); ++it) sort_by_column(col[*it], perm, E, s);
    sort_by_column(col[D->group_col], perm, E, s);
    idx->link_row = perm;

    idx->rows = idx->alloc<int32_t>((int64_t)D->n_atoms * E);
    for (int j = 0; j < D->n_atoms; ++j) prim::gather_i32(rowsL[j], perm, E, idx->rows + (int64_t)j * E, s);
    DevBuf gk(std::max<int64_t>(E, 1) * sizeof(int32_t)), offs((E + 1) * sizeof(int32_t)),
        keys(std::max<int64_t>(E, 1) * sizeof(int32_t));
    prim::gather_i32(col[D->group_col], perm, E, gk.as<int32_t>(), s);
    idx->tuple_group = idx->alloc<int32_t>(E);
    const int64_t G = prim::segments(gk.as<int32_t>(), E, idx->tuple_group, offs.as<int32_t>(),
                                     keys.as<int32_t>(), s);
    idx->G = G;
    idx->offsets = idx->alloc<int32_t>(G + 1);
    idx->group_keys = idx->alloc<int32_t>(G);
    RELNN_HIP(hipMemcpyAsync(idx->offsets, offs.p, (G + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (G > 0)
      RELNN_HIP(hipMemcpyAsync(idx->group_keys, keys.p, G * sizeof(int32_t), hipMemcpyDeviceToDevice, s));

    if (D->flags & RELNN_IDX_BWD) {
      idx->has_bwd = true;
      for (int j = 0; j < D->n_atoms; ++j) {
        const int64_t nr = D->atoms[j].n_rows;
        idx->t_row[j] = idx->alloc<int32_t>(E);
        idx->t_pos[j] = idx->alloc<int32_t>(E);
        idx->t_off[j] = idx->alloc<int32_t>(nr + 1);
        RELNN_HIP(hipMemcpyAsync(idx->t_row[j], idx->rows + (int64_t)j * E, E * sizeof(int32_t),
                                 hipMemcpyDeviceToDevice, s));
        prim::iota_i32(idx->t_pos[j], E, s);
        DevBuf tk(std::max<int64_t>(E, 1) * sizeof(uint32_t)), tv(std::max<int64_t>(E, 1) * sizeof(int32_t));
        prim::radix_sort_pairs(reinterpret_cast<uint32_t*>(idx->t_row[j]), idx->t_pos[j],
                               tk.as<uint32_t>(), tv.as<int32_t>(), E,
                               prim::bits_for((uint64_t)std::max<int64_t>(nr - 1, 0)), s);
        prim::csr_from_sorted(reinterpret_cast<uint32_t*>(idx->t_row[j]), E, nr, idx->t_off[j], s);
        idx->t_grp[j] = idx->alloc<int32_t>(E);
        prim::gather_i32(idx->tuple_group, idx->t_pos[j], E, idx->t_grp[j], s);
        DevBuf so((E + 1) * sizeof(int32_t)), sr(std::max<int64_t>(E, 1) * sizeof(int32_t));
        idx->t_seg[j] = idx->alloc<int32_t>(E);
        const int64_t ns = prim::segments(idx->t_row[j], E, idx->t_seg[j], so.as<int32_t>(), sr.as<int32_t>(), s);
        idx->t_nseg[j] = ns;
        idx->t_segoff[j] = idx->alloc<int32_t>(ns + 1);
        idx->t_segrow[j] = idx->alloc<int32_t>(ns);
        RELNN_HIP(hipMemcpyAsync(idx->t_segoff[j], so.p, (ns + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        if (ns > 0)
          RELNN_HIP(hipMemcpyAsync(idx->t_segrow[j], sr.p, ns * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        RELNN_HIP(hipStreamSynchronize(s));
      }
    }
    RELNN_HIP(hipStreamSynchronize(s));
    *out = idx.release();
  });
}

extern "C" relnn_status relnn_index_query(const relnn_index* idx, int64_t* n_tuples, int64_t* n_groups,
                                          int64_t* dev_bytes) {
  return guard([&] {
    RELNN_REQUIRE(idx != nullptr, RELNN_E_INVALID, "index is NULL");
    if (n_tuples) *n_tuples = idx->E;
    if (n_groups) *n_groups = idx->G;
    if (dev_bytes) *dev_bytes = idx->dev_bytes;
  });
}

extern "C" relnn_status relnn_index_export(const relnn_index* idx, int32_t* group_keys, int32_t* offsets,
                                           int32_t* link_rows, int32_t* tuple_rows, relnn_stream_t stream) {
  return guard([&] {
    RELNN_REQUIRE(idx != nullptr, RELNN_E_INVALID, "index is NULL");
    hipStream_t s = (hipStream_t)stream;
    const auto cp = [&](void* dst, const void* src, int64_t n) {
      if (dst && n > 0) RELNN_HIP(hipMemcpyAsync(dst, src, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    };
    cp(group_keys, idx->group_keys, idx->G);
    cp(offsets, idx->offsets, idx->G + 1);
    cp(link_rows, idx->link_row, idx->E);
    cp(tuple_rows, idx->rows, (int64_t)idx->k * idx->E);
  });
}

extern "C" relnn_status relnn_index_free(relnn_index* idx) {
  return guard([&] { delete idx; });
}
