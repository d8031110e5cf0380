// Device primitives for the index build: exclusive scan, stable LSD radix
// sort of (key, value) pairs, key range, sorted-segment CSR.  All integer
// work, deterministic, no library sort.
#pragma once

#include "common.hpp"

namespace relnn {
namespace prim {

// out[i] = sum of in[0..i) for i in [0, n); *total_host = sum of all (if
// non-null; synchronises the stream).
void scan_u8(const uint8_t* in, int64_t n, int32_t* out, int64_t* total_host, hipStream_t s);
void scan_i32(const int32_t* in, int64_t n, int32_t* out, int64_t* total_host, hipStream_t s);
void scan_i64(const int64_t* in, int64_t n, int64_t* out, int64_t* total_host, hipStream_t s);

// Stable sort of (keys, vals) by the low `bits` bits of keys (bits <= 32).
// Uses keys_tmp / vals_tmp as ping-pong buffers; on return the sorted data
// is in keys / vals (copied back if the pass count is odd).
void radix_sort_pairs(uint32_t* keys, int32_t* vals, uint32_t* keys_tmp, int32_t* vals_tmp,
                      int64_t n, int bits, hipStream_t s);

// Minimum and maximum of (uint32)(v[idx[i]] ^ 0x80000000) over i < n (idx
// NULL => identity).  Synchronises.  n > 0.
void key_range(const int32_t* v, const int32_t* idx, int64_t n, uint32_t* kmin, uint32_t* kmax,
               hipStream_t s);

// keys[i] = ((uint32)(v[idx[i]] ^ 0x80000000)) - kmin  (idx NULL => identity)
void make_keys(const int32_t* v, const int32_t* idx, int64_t n, uint32_t kmin, uint32_t* keys,
               hipStream_t s);

// Segments of a sorted int32 array: seg_of[i] = segment number of element
// i, offsets[0..nseg] (device, capacity n+1), first_vals[nseg] (optional).
// Returns nseg (synchronises).
int64_t segments(const int32_t* sorted, int64_t n, int32_t* seg_of, int32_t* offsets,
                 int32_t* first_vals, hipStream_t s);

// off[r] = lower_bound(sorted_keys, r) for r in [0, n_rows]  (CSR over dense rows)
void csr_from_sorted(const uint32_t* sorted_keys, int64_t n, int64_t n_rows, int32_t* off,
                     hipStream_t s);

// out[i] = v[idx[i]]
void gather_i32(const int32_t* v, const int32_t* idx, int64_t n, int32_t* out, hipStream_t s);
void iota_i32(int32_t* out, int64_t n, hipStream_t s);

int bits_for(uint64_t range_max);   // bits needed to hold 0..range_max

}  // namespace prim
}  // namespace relnn
