// Integer device primitives of the index build (see prims.hpp).
#include "prims.hpp"

namespace relnn {
namespace prim {

namespace {

constexpr int kT = 256;        // threads per block
constexpr int kIPT = 16;       // items per thread
constexpr int kChunk = kT * kIPT;

// ------------------------------------------------------------------ scan
template <class V>
__device__ __forceinline__ V wave_incl_scan_t(V v) {
  const int l = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    V t = __shfl_up(v, o, 64);
    if (l >= o) v += t;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread; returns the exclusive
// prefix and writes the block total to *total.
template <class V>
__device__ V block_excl_scan(V v, V* total) {
  __shared__ V wsum[kT / 64];
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  V inc = wave_incl_scan_t(v);
  if (l == 63) wsum[w] = inc;
  __syncthreads();
  V before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kT / 64; ++i) {
    if (i < w) before += wsum[i];
    all += wsum[i];
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

template <class In, class V>
__global__ void k_scan_reduce(const In* in, int64_t n, V* block_sums) {
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  V s = 0;
#pragma unroll
  for (int i = 0; i < kIPT; ++i) {
    int64_t j = base + (int64_t)i * kT + threadIdx.x;
    if (j < n) s += (V)in[j];
  }
  V tot;
  (void)block_excl_scan<V>(s, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// Each thread owns kIPT consecutive items (staged through LDS so the global
// accesses stay coalesced).
template <class In, class V>
__global__ void k_scan_apply(const In* in, int64_t n, const V* block_prefix, V* out, V* total) {
  __shared__ V buf[kChunk + kChunk / 64];
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  auto slot = [](int i) { return i + i / 64; };     // pad against bank conflicts
#pragma unroll
  for (int i = 0; i < kIPT; ++i) {
    int li = i * kT + threadIdx.x;
    int64_t j = base + li;
    buf[slot(li)] = j < n ? (V)in[j] : (V)0;
  }
  __syncthreads();
  V loc[kIPT];
  V s = 0;
#pragma unroll
  for (int i = 0; i < kIPT; ++i) {
    loc[i] = buf[slot(threadIdx.x * kIPT + i)];
    s += loc[i];
  }
  V tot;
  V pre = block_excl_scan<V>(s, &tot) + (block_prefix ? block_prefix[blockIdx.x] : (V)0);
#pragma unroll
  for (int i = 0; i < kIPT; ++i) {
    buf[slot(threadIdx.x * kIPT + i)] = pre;
    pre += loc[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kIPT; ++i) {
    int li = i * kT + threadIdx.x;
    int64_t j = base + li;
    if (j < n) out[j] = buf[slot(li)];
  }
  if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kT - 1) *total = pre;
}

template <class In, class V>
void scan_impl(const In* in, int64_t n, V* out, V* total_dev, hipStream_t s) {
  if (n <= 0) {
    if (total_dev) RELNN_HIP(hipMemsetAsync(total_dev, 0, sizeof(V), s));
    return;
  }
  const int64_t nb = cdiv(n, kChunk);
  if (nb == 1) {
    k_scan_apply<In, V><<<1, kT, 0, s>>>(in, n, (const V*)nullptr, out, total_dev);
    RELNN_LAUNCHED();
    return;
  }
  DevBuf sums(nb * sizeof(V)), pref(nb * sizeof(V));
  k_scan_reduce<In, V><<<(unsigned)nb, kT, 0, s>>>(in, n, sums.as<V>());
  RELNN_LAUNCHED();
  scan_impl<V, V>(sums.as<V>(), nb, pref.as<V>(), (V*)nullptr, s);
  k_scan_apply<In, V><<<(unsigned)nb, kT, 0, s>>>(in, n, pref.as<V>(), out, total_dev);
  RELNN_LAUNCHED();
  RELNN_HIP(hipStreamSynchronize(s));   // sums / pref are freed on return
}

template <class In, class V>
void scan_host(const In* in, int64_t n, V* out, int64_t* total_host, hipStream_t s) {
  DevBuf tot(sizeof(V));
  scan_impl<In, V>(in, n, out, tot.as<V>(), s);
  if (total_host) {
    V t = 0;
    RELNN_HIP(hipMemcpyAsync(&t, tot.p, sizeof(V), hipMemcpyDeviceToHost, s));
    RELNN_HIP(hipStreamSynchronize(s));
    *total_host = (int64_t)t;
  }
}

// ------------------------------------------------------------------ radix sort
__global__ void k_hist(const uint32_t* keys, int64_t n, int shift, int ndig, int64_t ntiles,
                       int32_t* hist) {
  __shared__ int cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  const uint32_t mask = (uint32_t)ndig - 1;
#pragma unroll 4
  for (int i = 0; i < kIPT; ++i) {
    int64_t j = base + (int64_t)i * kT + threadIdx.x;
    if (j < n) atomicAdd(&cnt[(keys[j] >> shift) & mask], 1);
  }
  __syncthreads();
  if (threadIdx.x < ndig) hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: items of a tile are ranked in (round, wave, lane) order,
// which is their input order.
__global__ void k_scatter(const uint32_t* keys, const int32_t* vals, int64_t n, int shift, int db,
                          int64_t ntiles, const int32_t* hist_scanned, uint32_t* keys_out,
                          int32_t* vals_out) {
  __shared__ int gofs[256];
  __shared__ int run[256];
  __shared__ int wcount[kT / 64][256];
  __shared__ int wpre[kT / 64][256];
  const int ndig = 1 << db;
  const uint32_t mask = (uint32_t)ndig - 1;
  const int tid = threadIdx.x, w = tid / 64, l = tid % 64;
  if (tid < ndig) gofs[tid] = hist_scanned[(int64_t)tid * ntiles + blockIdx.x];
  run[tid] = 0;
  const uint64_t lt = (l == 0) ? 0ull : (~0ull >> (64 - l));
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  for (int r = 0; r < kIPT; ++r) {
    const int64_t j = base + (int64_t)r * kT + tid;
    const bool valid = j < n;
    const uint32_t key = valid ? keys[j] : 0u;
    const int32_t val = valid ? vals[j] : 0;
    const int dg = (int)((key >> shift) & mask);
#pragma unroll
    for (int q = 0; q < kT / 64; ++q) wcount[q][tid] = 0;
    __syncthreads();
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < db; ++b) {
      const bool bit = (dg >> b) & 1;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const int rank = __popcll(peers & lt);
    if (valid && rank == 0) wcount[w][dg] = __popcll(peers);
    __syncthreads();
    if (tid < ndig) {
      int sacc = run[tid];
#pragma unroll
      for (int q = 0; q < kT / 64; ++q) {
        wpre[q][tid] = sacc;
        sacc += wcount[q][tid];
      }
      run[tid] = sacc;
    }
    __syncthreads();
    if (valid) {
      const int pos = gofs[dg] + wpre[w][dg] + rank;
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
  }
}

// Smallest and largest key (order-preserving unsigned form).  One atomic
// pair per block: atomics from every wave to one address serialise in L2.
constexpr int kRangeThreads = 256;
constexpr unsigned kRangeBlocks = 1024;
__global__ void __launch_bounds__(kRangeThreads) k_key_range(const int32_t* v, const int32_t* idx, int64_t n,
                                                             uint32_t* mm) {
  uint32_t lo = 0xFFFFFFFFu, hi = 0u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t k = (uint32_t)(idx ? v[idx[i]] : v[i]) ^ 0x80000000u;
    lo = min(lo, k);
    hi = max(hi, k);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, 64));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, 64));
  }
  __shared__ uint32_t wlo[kRangeThreads / 64], whi[kRangeThreads / 64];
  const int w = threadIdx.x / 64;
  if (__lane_id() == 0) {
    wlo[w] = lo;
    whi[w] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = 1; j < kRangeThreads / 64; ++j) {
      lo = min(lo, wlo[j]);
      hi = max(hi, whi[j]);
    }
    atomicMin(&mm[0], lo);
    atomicMax(&mm[1], hi);
  }
}

__global__ void k_make_keys(const int32_t* v, const int32_t* idx, int64_t n, uint32_t kmin,
                            uint32_t* keys) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    keys[i] = ((uint32_t)(idx ? v[idx[i]] : v[i]) ^ 0x80000000u) - kmin;
  }
}

__global__ void k_heads(const int32_t* sorted, int64_t n, int32_t* head) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    head[i] = (i == 0 || sorted[i] != sorted[i - 1]) ? 1 : 0;
}

// head holds the exclusive scan of the head flags on input.
__global__ void k_segs(const int32_t* sorted, int64_t n, const int32_t* excl, int32_t* seg_of,
                       int32_t* offsets, int32_t* first_vals) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const bool h = (i == 0 || sorted[i] != sorted[i - 1]);
    const int32_t sg = excl[i] + (h ? 1 : 0) - 1;
    seg_of[i] = sg;
    if (h) {
      offsets[sg] = (int32_t)i;
      if (first_vals) first_vals[sg] = sorted[i];
    }
  }
}

__global__ void k_csr_lb(const uint32_t* sk, int64_t n, int64_t n_rows, int32_t* off) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n_rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if ((int64_t)sk[mid] < r) lo = mid + 1; else hi = mid;
    }
    off[r] = (int32_t)lo;
  }
}

__global__ void k_gather_i32(const int32_t* v, const int32_t* idx, int64_t n, int32_t* out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = v[idx[i]];
}

__global__ void k_iota(int32_t* out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (int32_t)i;
}

inline unsigned grid_for(int64_t n) {
  int64_t g = cdiv(n, 256);
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

void scan_u8(const uint8_t* in, int64_t n, int32_t* out, int64_t* total_host, hipStream_t s) {
  scan_host<uint8_t, int32_t>(in, n, out, total_host, s);
}
void scan_i32(const int32_t* in, int64_t n, int32_t* out, int64_t* total_host, hipStream_t s) {
  scan_host<int32_t, int32_t>(in, n, out, total_host, s);
}
void scan_i64(const int64_t* in, int64_t n, int64_t* out, int64_t* total_host, hipStream_t s) {
  scan_host<int64_t, int64_t>(in, n, out, total_host, s);
}

int bits_for(uint64_t range_max) {
  int b = 0;
  while (b < 64 && (range_max >> b) != 0) ++b;
  return b;
}

void radix_sort_pairs(uint32_t* keys, int32_t* vals, uint32_t* keys_tmp, int32_t* vals_tmp,
                      int64_t n, int bits, hipStream_t s) {
  if (n <= 1 || bits <= 0) return;
  const int passes = (int)cdiv(bits, 8);
  const int db = (int)cdiv(bits, passes);
  const int64_t ntiles = cdiv(n, kChunk);
  const int ndig = 1 << db;
  DevBuf hist(ndig * ntiles * sizeof(int32_t)), hsc(ndig * ntiles * sizeof(int32_t));
  uint32_t *ki = keys, *ko = keys_tmp;
  int32_t *vi = vals, *vo = vals_tmp;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * db;
    const int dbp = std::min(db, bits - shift);
    k_hist<<<(unsigned)ntiles, kT, 0, s>>>(ki, n, shift, 1 << dbp, ntiles, hist.as<int32_t>());
    RELNN_LAUNCHED();
    scan_impl<int32_t, int32_t>(hist.as<int32_t>(), (int64_t)(1 << dbp) * ntiles, hsc.as<int32_t>(),
                                (int32_t*)nullptr, s);
    k_scatter<<<(unsigned)ntiles, kT, 0, s>>>(ki, vi, n, shift, dbp, ntiles, hsc.as<int32_t>(), ko, vo);
    RELNN_LAUNCHED();
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  if (ki != keys) {
    RELNN_HIP(hipMemcpyAsync(keys, ki, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    RELNN_HIP(hipMemcpyAsync(vals, vi, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  }
  RELNN_HIP(hipStreamSynchronize(s));   // hist buffers are freed on return
}

void key_range(const int32_t* v, const int32_t* idx, int64_t n, uint32_t* kmin, uint32_t* kmax,
               hipStream_t s) {
  DevBuf mm(2 * sizeof(uint32_t));
  uint32_t init[2] = {0xFFFFFFFFu, 0u};
  RELNN_HIP(hipMemcpyAsync(mm.p, init, sizeof(init), hipMemcpyHostToDevice, s));
  k_key_range<<<std::min(grid_for(n), kRangeBlocks), kRangeThreads, 0, s>>>(v, idx, n, mm.as<uint32_t>());
  RELNN_LAUNCHED();
  uint32_t res[2];
  RELNN_HIP(hipMemcpyAsync(res, mm.p, sizeof(res), hipMemcpyDeviceToHost, s));
  RELNN_HIP(hipStreamSynchronize(s));
  *kmin = res[0];
  *kmax = res[1];
}

void make_keys(const int32_t* v, const int32_t* idx, int64_t n, uint32_t kmin, uint32_t* keys,
               hipStream_t s) {
  if (n <= 0) return;
  k_make_keys<<<grid_for(n), 256, 0, s>>>(v, idx, n, kmin, keys);
  RELNN_LAUNCHED();
}

int64_t segments(const int32_t* sorted, int64_t n, int32_t* seg_of, int32_t* offsets,
                 int32_t* first_vals, hipStream_t s) {
  if (n <= 0) {
    int32_t z = 0;
    RELNN_HIP(hipMemcpyAsync(offsets, &z, sizeof(z), hipMemcpyHostToDevice, s));
    RELNN_HIP(hipStreamSynchronize(s));
    return 0;
  }
  DevBuf head(n * sizeof(int32_t)), excl(n * sizeof(int32_t));
  k_heads<<<grid_for(n), 256, 0, s>>>(sorted, n, head.as<int32_t>());
  RELNN_LAUNCHED();
  int64_t nseg = 0;
  scan_i32(head.as<int32_t>(), n, excl.as<int32_t>(), &nseg, s);
  k_segs<<<grid_for(n), 256, 0, s>>>(sorted, n, excl.as<int32_t>(), seg_of, offsets, first_vals);
  RELNN_LAUNCHED();
  int32_t end = (int32_t)n;
  RELNN_HIP(hipMemcpyAsync(offsets + nseg, &end, sizeof(end), hipMemcpyHostToDevice, s));
  RELNN_HIP(hipStreamSynchronize(s));
  return nseg;
}

void csr_from_sorted(const uint32_t* sorted_keys, int64_t n, int64_t n_rows, int32_t* off,
                     hipStream_t s) {
  k_csr_lb<<<grid_for(n_rows + 1), 256, 0, s>>>(sorted_keys, n, n_rows, off);
  RELNN_LAUNCHED();
}

void gather_i32(const int32_t* v, const int32_t* idx, int64_t n, int32_t* out, hipStream_t s) {
  if (n <= 0) return;
  k_gather_i32<<<grid_for(n), 256, 0, s>>>(v, idx, n, out);
  RELNN_LAUNCHED();
}

void iota_i32(int32_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_iota<<<grid_for(n), 256, 0, s>>>(out, n);
  RELNN_LAUNCHED();
}

}  // namespace prim
}  // namespace relnn
