// Serving: continuous batching of sampled two-hop neighbourhood requests on
// the resident ER graph (request semantics in relnn.h).
//
// A step is one hipGraph over fixed device buffers: count hop-1 -> scan ->
// sample hop-1 -> count hop-2 -> scan -> sample hop-2 -> three persistent
// layer launches (+ their fix-ups).  Every size inside the graph (seeds,
// hop-1 rows, hop-2 rows) is read from device memory, so one captured graph
// serves every batch shape.  The samplers write their tuples grouped by
// seed (hop 1) and by hop-1 row (hop 2) with positions ascending, which is
// the canonical order of those joins, so the layer kernels consume them
// directly as an index.  A host scheduler thread admits requests, fills
// the pinned input buffers, launches the graph and hands results back.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "layer_fwd.hpp"
#include "prims.hpp"

namespace relnn {
namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr int kMaxFan = 32;

// SplitMix64 output function (Steele, Lea and Flood, 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t stream_base(uint64_t req_seed, int hop, int64_t node) {
  return mix64(req_seed + (uint64_t)(2 * node + hop + 1) * kGolden);
}

// k distinct positions of [0, n) (Floyd's algorithm), sorted ascending.
__device__ __forceinline__ void floyd(uint64_t base, int64_t n, int k, int32_t* pos) {
  int m = 0;
  for (int64_t j = n - k; j < n; ++j) {
    const uint64_t r = mix64(base + (uint64_t)(m + 1) * kGolden);
    const int64_t t = (int64_t)(((r >> 32) * (uint64_t)(j + 1)) >> 32);
    bool seen = false;
    for (int q = 0; q < m; ++q) seen |= (pos[q] == t);
    pos[m++] = (int32_t)(seen ? j : t);
  }
  for (int a = 1; a < k; ++a) {            // insertion sort, k <= 32
    const int32_t v = pos[a];
    int b = a - 1;
    while (b >= 0 && pos[b] > v) {
      pos[b + 1] = pos[b];
      --b;
    }
    pos[b + 1] = v;
  }
}

__global__ void k_count1(const int32_t* seeds, const int64_t* n_dev, const int32_t* i_off, int64_t n_item, int f1,
                         int32_t* cnt) {
  const int64_t n = *n_dev;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = seeds[i];
    const int64_t deg = (s >= 0 && s < n_item) ? (int64_t)(i_off[s + 1] - i_off[s]) : 0;
    cnt[i] = (int32_t)min<int64_t>(f1, deg);
  }
}

__global__ void k_sample1(const int32_t* seeds, const uint64_t* rseed, const int64_t* n_dev, const int32_t* i_off,
                          const int32_t* i_user, const int32_t* item_cat, int64_t n_item, int f1, const int32_t* off1,
                          int32_t* t1_user, int32_t* t1_seed, int32_t* t1_item, int32_t* t1_cat) {
  const int64_t n = *n_dev;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = seeds[i];
    if (s < 0 || s >= n_item) continue;
    const int64_t deg = i_off[s + 1] - i_off[s];
    const int k = (int)min<int64_t>(f1, deg);
    int32_t pos[kMaxFan];
    floyd(stream_base(rseed[i], 1, s), deg, k, pos);
    const int64_t base = off1[i];
    for (int q = 0; q < k; ++q) {
      t1_user[base + q] = i_user[i_off[s] + pos[q]];
      t1_seed[base + q] = (int32_t)i;
      t1_item[base + q] = s;
      t1_cat[base + q] = item_cat[s];
    }
  }
}

__global__ void k_count2(const int32_t* t1_user, const int64_t* e1_dev, const int32_t* u_off, int f2, int32_t* cnt) {
  const int64_t n = *e1_dev;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = t1_user[e];
    cnt[e] = (int32_t)min<int64_t>(f2, (int64_t)(u_off[u + 1] - u_off[u]));
  }
}

__global__ void k_sample2(const int32_t* t1_user, const int32_t* t1_seed, const uint64_t* rseed, const int64_t* e1_dev,
                          const int32_t* u_off, const int32_t* u_item, int f2, const int32_t* off2, int32_t* t2_user,
                          int32_t* t2_item, int32_t* t2_grp) {
  const int64_t n = *e1_dev;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = t1_user[e];
    const int64_t deg = u_off[u + 1] - u_off[u];
    const int k = (int)min<int64_t>(f2, deg);
    int32_t pos[kMaxFan];
    floyd(stream_base(rseed[t1_seed[e]], 2, u), deg, k, pos);
    const int64_t base = off2[e];
    for (int q = 0; q < k; ++q) {
      t2_user[base + q] = u;
      t2_item[base + q] = u_item[u_off[u] + pos[q]];
      t2_grp[base + q] = (int32_t)e;
    }
  }
}

// One-block exclusive scan of in[0..n) (n read from device): out[0..n],
// out[n] = *total = sum.
__global__ void __launch_bounds__(1024) k_scan_one(const int32_t* in, const int64_t* n_dev, int32_t* out,
                                                   int64_t* total) {
  __shared__ int64_t part[1024];
  const int64_t n = *n_dev;
  const int64_t chunk = (n + 1023) / 1024;
  const int64_t lo = min<int64_t>(n, threadIdx.x * chunk), hi = min<int64_t>(n, lo + chunk);
  int64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += in[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {      // inclusive Hillis-Steele scan
    const int64_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t run = part[threadIdx.x] - s;
  for (int64_t i = lo; i < hi; ++i) {
    out[i] = (int32_t)run;
    run += in[i];
  }
  if (threadIdx.x == 1023) {
    out[n] = (int32_t)part[1023];
    *total = part[1023];
  }
}

__global__ void k_iota32(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (int32_t)i;
}

int num_cus_serve() {
  int dev = 0, n = 0;
  RELNN_HIP(hipGetDevice(&dev));
  RELNN_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
  return n;
}

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  uint64_t ticket;
  std::vector<int32_t> seeds;
  uint64_t req_seed;
  relnn_req_stats st{};
  std::vector<float> out;
  std::vector<uint8_t> present;
  bool admitted = false;             // taken into a step
  bool cancelled = false;            // admitted, then cancelled: dropped when its step ends
  bool done = false;
};

// A layer launch of the step: kernel plan + arguments.
struct LayerCall {
  WsPlan plan;
  FwdArgs f;
  void* Wsw;
};

}  // namespace
}  // namespace relnn

using namespace relnn;

struct relnn_server {
  relnn_serve_desc D{};
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t cap_seeds = 0, cap_t1 = 0, cap_t2 = 0;
  std::vector<void*> allocs;
  int64_t dev_bytes = 0;
  // resident adjacency
  int32_t *i_off = nullptr, *i_user = nullptr, *u_off = nullptr, *u_item = nullptr;
  // step buffers
  int32_t* seeds_d = nullptr;
  uint64_t* rseed_d = nullptr;
  int64_t* counts_d = nullptr;            // [0] seeds, [1] hop-1 rows, [2] hop-2 rows
  int32_t *cnt1 = nullptr, *off1 = nullptr, *t1_user = nullptr, *t1_seed = nullptr, *t1_item = nullptr,
          *t1_cat = nullptr, *t1_iota = nullptr, *cnt2 = nullptr, *off2 = nullptr;
  int32_t *t2_user = nullptr, *t2_item = nullptr, *t2_grp = nullptr;
  void *U1 = nullptr, *I1 = nullptr;
  float* OUT = nullptr;
  float* carry = nullptr;
  // pinned host staging
  int32_t* seeds_h = nullptr;
  uint64_t* rseed_h = nullptr;
  int64_t* counts_h = nullptr;
  float* out_h = nullptr;
  int32_t* off1_h = nullptr;
  int32_t* off2_h = nullptr;
  LayerCall calls[3];
  hipGraphExec_t graph = nullptr;
  hipEvent_t done_ev = nullptr;
  // requests
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_ticket = 1;
  int64_t steps = 0;
  bool stop = false;
  std::thread worker;
  std::string worker_error;

  template <class T>
  T* dalloc(int64_t n) {
    void* p = nullptr;
    const size_t bytes = (size_t)std::max<int64_t>(n, 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      relnn::set_error("server allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
      throw relnn::Fail{RELNN_E_OOM};
    }
    allocs.push_back(p);
    dev_bytes += bytes;
    return static_cast<T*>(p);
  }

  ~relnn_server() {
    if (graph) (void)hipGraphExecDestroy(graph);
    if (done_ev) (void)hipEventDestroy(done_ev);
    if (stream) (void)hipStreamSynchronize(stream);
    for (void* p : allocs) (void)hipFree(p);
    for (void* p : {(void*)seeds_h, (void*)rseed_h, (void*)counts_h, (void*)out_h, (void*)off1_h, (void*)off2_h})
      if (p) (void)hipHostFree(p);
    if (stream) (void)hipStreamDestroy(stream);
  }

  void run_step_kernels(hipStream_t s);
  void run_step(std::vector<Request*>& batch);
  void loop();
};

static unsigned grid_n(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 4096)); }

// Device bytes per seed of step capacity.
static int64_t bytes_per_seed(const relnn_serve_desc& D) {
  const int64_t esz = D.dtype == RELNN_BF16 ? 2 : 4;
  const int64_t t1 = D.fanout1, t2 = (int64_t)D.fanout1 * D.fanout2;
  return 4 * 4 + 8 + t1 * (7 * 4) + t2 * (3 * 4) + t1 * D.h * esz + D.h * esz + D.h * 4 + 4 * D.h;
}

void relnn_server::run_step_kernels(hipStream_t s) {
  const int f1 = D.fanout1, f2 = D.fanout2;
  k_count1<<<grid_n(cap_seeds), 256, 0, s>>>(seeds_d, counts_d, i_off, D.n_item, f1, cnt1);
  k_scan_one<<<1, 1024, 0, s>>>(cnt1, counts_d, off1, counts_d + 1);
  k_sample1<<<grid_n(cap_seeds), 256, 0, s>>>(seeds_d, rseed_d, counts_d, i_off, i_user, D.item_cat, D.n_item, f1,
                                               off1, t1_user, t1_seed, t1_item, t1_cat);
  k_count2<<<grid_n(cap_t1), 256, 0, s>>>(t1_user, counts_d + 1, u_off, f2, cnt2);
  k_scan_one<<<1, 1024, 0, s>>>(cnt2, counts_d + 1, off2, counts_d + 2);
  k_sample2<<<grid_n(cap_t1), 256, 0, s>>>(t1_user, t1_seed, rseed_d, counts_d + 1, u_off, u_item, f2, off2, t2_user,
                                           t2_item, t2_grp);
  RELNN_LAUNCHED();
  for (LayerCall& c : calls) launch_ws(c.plan, D.dtype, c.f, c.Wsw, carry, nullptr, s);
}

void relnn_server::run_step(std::vector<Request*>& batch) {
  int64_t n = 0;
  for (Request* r : batch) {
    for (size_t q = 0; q < r->seeds.size(); ++q) {
      seeds_h[n + q] = r->seeds[q];
      rseed_h[n + q] = r->req_seed;
    }
    n += (int64_t)r->seeds.size();
  }
  counts_h[0] = n;
  const int64_t t_admit = now_ns();
  hipStream_t s = stream;
  RELNN_HIP(hipMemcpyAsync(seeds_d, seeds_h, n * sizeof(int32_t), hipMemcpyHostToDevice, s));
  RELNN_HIP(hipMemcpyAsync(rseed_d, rseed_h, n * sizeof(uint64_t), hipMemcpyHostToDevice, s));
  RELNN_HIP(hipMemcpyAsync(counts_d, counts_h, sizeof(int64_t), hipMemcpyHostToDevice, s));
  if (!graph) {
    run_step_kernels(s);            // first step eager (sets kernel attributes), then capture
    RELNN_HIP(hipStreamSynchronize(s));
    hipGraph_t g = nullptr;
    RELNN_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    run_step_kernels(s);
    RELNN_HIP(hipStreamEndCapture(s, &g));
    RELNN_HIP(hipGraphInstantiate(&graph, g, nullptr, nullptr, 0));
    RELNN_HIP(hipGraphDestroy(g));
  } else {
    RELNN_HIP(hipGraphLaunch(graph, s));
  }
  RELNN_HIP(hipMemcpyAsync(counts_h, counts_d, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  RELNN_HIP(hipMemcpyAsync(out_h, OUT, n * D.h * sizeof(float), hipMemcpyDeviceToHost, s));
  RELNN_HIP(hipMemcpyAsync(off1_h, off1, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  RELNN_HIP(hipStreamSynchronize(s));
  const int64_t e1 = counts_h[1];
  RELNN_HIP(hipMemcpyAsync(off2_h, off2, (e1 + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  RELNN_HIP(hipStreamSynchronize(s));
  const int64_t t_done = now_ns();
  int64_t base = 0;
  std::lock_guard<std::mutex> lk(mu);
  for (Request* r : batch) {
    const int64_t m = (int64_t)r->seeds.size();
    if (r->cancelled) {              // its caller no longer wants it
      base += m;
      reqs.erase(r->ticket);
      continue;
    }
    r->out.assign(out_h + base * D.h, out_h + (base + m) * D.h);
    r->present.resize(m);
    for (int64_t q = 0; q < m; ++q) {
      const bool pr = off1_h[base + q + 1] > off1_h[base + q];
      r->present[q] = pr ? 1 : 0;
      if (!pr) std::fill(r->out.begin() + q * D.h, r->out.begin() + (q + 1) * D.h, 0.0f);
    }
    const int64_t a1 = off1_h[base], b1 = off1_h[base + m];
    r->st.tuples = 2 * (b1 - a1) + (off2_h[b1] - off2_h[a1]);
    r->st.t_admit_ns = t_admit;
    r->st.t_done_ns = t_done;
    r->st.step = steps;
    r->done = true;
    base += m;
  }
  ++steps;
}

void relnn_server::loop() {
  RELNN_HIP(hipSetDevice(device));
  for (;;) {
    std::vector<Request*> batch;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || !pending.empty(); });
      if (stop) return;
      int64_t seeds = 0;
      while (!pending.empty() && (int)batch.size() < D.max_slots) {
        Request* r = pending.front();
        if (seeds + (int64_t)r->seeds.size() > cap_seeds) break;   // waits for the next step
        seeds += (int64_t)r->seeds.size();
        r->admitted = true;
        batch.push_back(r);
        pending.pop_front();
      }
    }
    run_step(batch);
  }
}

extern "C" relnn_status relnn_serve_create(const relnn_serve_desc* D, relnn_server** out) {
  return guard([&] {
    RELNN_REQUIRE(D && out, RELNN_E_INVALID, "NULL argument");
    *out = nullptr;
    RELNN_REQUIRE(D->n_user > 0 && D->n_item > 0 && D->n_cat > 0 && D->n_buys >= 0, RELNN_E_INVALID, "bad sizes");
    RELNN_REQUIRE(D->buys_user && D->buys_item && D->item_cat && D->user_emb && D->item_emb && D->cat_emb &&
                      D->W_user && D->W_item1 && D->W_item2,
                  RELNN_E_INVALID, "a resident relation or weight is NULL");
    RELNN_REQUIRE(D->d == D->h && D->h > 0, RELNN_E_UNSUPPORTED, "serving needs d == h");
    RELNN_REQUIRE(D->fanout1 >= 1 && D->fanout1 <= kMaxFan && D->fanout2 >= 1 && D->fanout2 <= kMaxFan,
                  RELNN_E_RANGE, "fanouts must be 1..%d", kMaxFan);
    RELNN_REQUIRE(D->dtype == RELNN_F32 || D->dtype == RELNN_BF16, RELNN_E_INVALID, "unknown dtype");
    RELNN_REQUIRE(D->max_seeds >= 1 && D->max_slots >= 1, RELNN_E_INVALID, "max_seeds and max_slots must be >= 1");
    std::unique_ptr<relnn_server> S(new relnn_server());
    S->D = *D;
    RELNN_HIP(hipGetDevice(&S->device));
    RELNN_HIP(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
    hipStream_t s = S->stream;

    // step capacity from the budget
    const int64_t bps = bytes_per_seed(*D);
    const int64_t fixed = (int64_t)num_cus_serve() * 2 * D->h * 4 + (1 << 20);
    const int64_t by_budget = ((int64_t)D->budget_bytes - fixed) / bps;
    RELNN_REQUIRE(by_budget >= D->max_seeds, RELNN_E_OOM,
                  "budget of %zu bytes holds %lld seeds per step, less than max_seeds = %d", D->budget_bytes,
                  (long long)std::max<int64_t>(by_budget, 0), D->max_seeds);
    S->cap_seeds = std::min<int64_t>(by_budget, (int64_t)D->max_seeds * D->max_slots);
    S->cap_seeds = std::min<int64_t>(S->cap_seeds, (int64_t)INT32_MAX / ((int64_t)D->fanout1 * D->fanout2 + 1));
    S->cap_t1 = S->cap_seeds * D->fanout1;
    S->cap_t2 = S->cap_t1 * D->fanout2;

    // resident adjacency: buyers of each item ordered by (user, row); Buys
    // rows of each user ordered by (item, row)
    const int64_t nb = D->n_buys;
    {
      DevBuf perm(std::max<int64_t>(nb, 1) * 4), keys(std::max<int64_t>(nb, 1) * 4),
          tk(std::max<int64_t>(nb, 1) * 4), tv(std::max<int64_t>(nb, 1) * 4);
      auto build = [&](const int32_t* major, const int32_t* minor, int64_t n_major, int32_t*& off, int32_t*& val) {
        off = S->dalloc<int32_t>(n_major + 1);
        val = S->dalloc<int32_t>(nb);
        prim::iota_i32(perm.as<int32_t>(), nb, s);
        for (const int32_t* col : {minor, major}) {
          uint32_t kmin, kmax;
          if (nb == 0) break;
          prim::key_range(col, perm.as<int32_t>(), nb, &kmin, &kmax, s);
          const int bits = prim::bits_for((uint64_t)(kmax - kmin));
          prim::make_keys(col, perm.as<int32_t>(), nb, kmin, keys.as<uint32_t>(), s);
          prim::radix_sort_pairs(keys.as<uint32_t>(), perm.as<int32_t>(), tk.as<uint32_t>(), tv.as<int32_t>(), nb,
                                 bits, s);
        }
        prim::make_keys(major, perm.as<int32_t>(), nb, 0x80000000u, keys.as<uint32_t>(), s);
        prim::csr_from_sorted(keys.as<uint32_t>(), nb, n_major, off, s);
        prim::gather_i32(minor, perm.as<int32_t>(), nb, val, s);
        RELNN_HIP(hipStreamSynchronize(s));
      };
      build(D->buys_item, D->buys_user, D->n_item, S->i_off, S->i_user);
      build(D->buys_user, D->buys_item, D->n_user, S->u_off, S->u_item);
    }

    // step buffers
    const int64_t cs = S->cap_seeds, c1 = S->cap_t1, c2 = S->cap_t2, h = D->h;
    const int esz = D->dtype == RELNN_BF16 ? 2 : 4;
    S->seeds_d = S->dalloc<int32_t>(cs);
    S->rseed_d = S->dalloc<uint64_t>(cs);
    S->counts_d = S->dalloc<int64_t>(4);
    S->cnt1 = S->dalloc<int32_t>(cs);
    S->off1 = S->dalloc<int32_t>(cs + 1);
    S->t1_user = S->dalloc<int32_t>(c1);
    S->t1_seed = S->dalloc<int32_t>(c1);
    S->t1_item = S->dalloc<int32_t>(c1);
    S->t1_cat = S->dalloc<int32_t>(c1);
    S->t1_iota = S->dalloc<int32_t>(c1);
    S->cnt2 = S->dalloc<int32_t>(c1);
    S->off2 = S->dalloc<int32_t>(c1 + 1);
    S->t2_user = S->dalloc<int32_t>(c2);
    S->t2_item = S->dalloc<int32_t>(c2);
    S->t2_grp = S->dalloc<int32_t>(c2);
    S->U1 = S->dalloc<char>(c1 * h * esz);
    S->I1 = S->dalloc<char>(cs * h * esz);
    S->OUT = S->dalloc<float>(cs * h);
    k_iota32<<<grid_n(c1), 256, 0, s>>>(S->t1_iota, c1);
    RELNN_LAUNCHED();
    RELNN_HIP(hipHostMalloc((void**)&S->seeds_h, cs * sizeof(int32_t), hipHostMallocDefault));
    RELNN_HIP(hipHostMalloc((void**)&S->rseed_h, cs * sizeof(uint64_t), hipHostMallocDefault));
    RELNN_HIP(hipHostMalloc((void**)&S->counts_h, 4 * sizeof(int64_t), hipHostMallocDefault));
    RELNN_HIP(hipHostMalloc((void**)&S->out_h, cs * h * sizeof(float), hipHostMallocDefault));
    RELNN_HIP(hipHostMalloc((void**)&S->off1_h, (cs + 1) * sizeof(int32_t), hipHostMallocDefault));
    RELNN_HIP(hipHostMalloc((void**)&S->off2_h, (c1 + 1) * sizeof(int32_t), hipHostMallocDefault));

    // the three layer calls
    const int d = D->d;
    struct Spec {
      int k;
      int dims[3];
      const void* emb[3];
      const int32_t* rows[3];
      const void* W;
      const float* b;
      int agg;
      const int32_t* seg_of;
      const int32_t* offsets;
      int64_t cap;
      const int64_t* n_dev;
      void* out;
      bool out_bf16;
    } spec[3] = {
        {2, {d, d, 0}, {D->user_emb, D->item_emb, nullptr}, {S->t2_user, S->t2_item, nullptr}, D->W_user, D->b_user,
         RELNN_MEAN, S->t2_grp, S->off2, c2, S->counts_d + 2, S->U1, D->dtype == RELNN_BF16},
        {3, {d, d, d}, {D->user_emb, D->item_emb, D->cat_emb}, {S->t1_user, S->t1_item, S->t1_cat}, D->W_item1,
         D->b_item1, RELNN_SUM, S->t1_seed, S->off1, c1, S->counts_d + 1, S->I1, D->dtype == RELNN_BF16},
        {3, {(int)h, (int)h, d}, {S->U1, S->I1, D->cat_emb}, {S->t1_iota, S->t1_seed, S->t1_cat}, D->W_item2,
         D->b_item2, RELNN_SUM, S->t1_seed, S->off1, c1, S->counts_d + 1, S->OUT, false},
    };
    int64_t max_units = 1;
    for (int q = 0; q < 3; ++q) {
      const Spec& p = spec[q];
      relnn_layer_desc L{};
      L.k = p.k;
      L.d = p.dims;
      L.h = (int)h;
      L.dtype = D->dtype;
      L.agg = p.agg;
      L.act_pre = RELNN_ACT_NONE;
      L.act_post = RELNN_ACT_RELU;
      int K = 0;
      for (int j = 0; j < p.k; ++j) K += p.dims[j];
      LayerCall& c = S->calls[q];
      c.plan = plan_ws(D->dtype, K, (int)h, p.cap);
      RELNN_REQUIRE(c.plan.KP != 0, RELNN_E_UNSUPPORTED, "serving layer shape K=%d h=%d not supported", K, (int)h);
      c.Wsw = S->dalloc<char>(c.plan.wsw_bytes);
      swizzle_ws(p.W, D->dtype, K, c.plan.KP, (int)h, c.Wsw, s);
      FwdArgs& f = c.f;
      f = FwdArgs{};
      f.at = make_atoms(&L, p.emb, nullptr);
      for (int j = 0; j < p.k; ++j) f.at.rows[j] = p.rows[j];
      f.E = p.cap;
      f.E_dev = p.n_dev;
      f.K = K;
      f.h = (int)h;
      f.b = p.b;
      f.act_pre = RELNN_ACT_NONE;
      f.sg = Seg{p.seg_of, p.offsets, p.cap, p.n_dev};
      f.sink = Sink{p.agg, RELNN_ACT_RELU, static_cast<float*>(p.out), nullptr, nullptr, false, nullptr, p.out_bf16};
      max_units = std::max(max_units, c.plan.nunits);
    }
    S->carry = S->dalloc<float>(max_units * 2 * h);
    RELNN_HIP(hipEventCreateWithFlags(&S->done_ev, hipEventDisableTiming));
    RELNN_HIP(hipStreamSynchronize(s));
    relnn_server* raw = S.get();
    S->worker = std::thread([raw] {
      try {
        raw->loop();
      } catch (const Fail&) {
        std::lock_guard<std::mutex> lk(raw->mu);
        raw->worker_error = relnn_last_error();
        raw->stop = true;
      } catch (...) {
        std::lock_guard<std::mutex> lk(raw->mu);
        raw->worker_error = "unexpected exception in the scheduler";
        raw->stop = true;
      }
    });
    *out = S.release();
  });
}

extern "C" relnn_status relnn_serve_submit(relnn_server* S, const int32_t* seeds, int32_t n, uint64_t req_seed,
                                           uint64_t* ticket) {
  return guard([&] {
    RELNN_REQUIRE(S && seeds && ticket, RELNN_E_INVALID, "NULL argument");
    RELNN_REQUIRE(n >= 1 && n <= S->D.max_seeds, RELNN_E_RANGE, "request of %d seeds (max %d)", n, S->D.max_seeds);
    std::unique_ptr<Request> r(new Request());
    r->seeds.assign(seeds, seeds + n);
    r->req_seed = req_seed;
    r->st.n_seeds = n;
    r->st.t_arrive_ns = now_ns();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      RELNN_REQUIRE(!S->stop, RELNN_E_HIP, "server stopped: %s", S->worker_error.c_str());
      RELNN_REQUIRE(S->pending.size() < 1u << 20, RELNN_E_BUSY, "request queue is full");
      r->ticket = S->next_ticket++;
      *ticket = r->ticket;
      S->pending.push_back(r.get());
      S->reqs.emplace(r->ticket, std::move(r));
    }
    S->cv.notify_one();
  });
}

extern "C" relnn_status relnn_serve_poll(relnn_server* S, uint64_t ticket, float* out, uint8_t* present,
                                         relnn_req_stats* stats) {
  relnn_status st = RELNN_OK;
  relnn_status g = guard([&] {
    RELNN_REQUIRE(S != nullptr, RELNN_E_INVALID, "NULL server");
    std::unique_ptr<Request> r;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      auto it = S->reqs.find(ticket);
      RELNN_REQUIRE(it != S->reqs.end() && !it->second->cancelled, RELNN_E_INVALID, "unknown ticket %llu",
                    (unsigned long long)ticket);
      if (!it->second->done) {
        RELNN_REQUIRE(!S->stop, RELNN_E_HIP, "server stopped: %s", S->worker_error.c_str());
        st = RELNN_E_NOT_READY;
        return;
      }
      r = std::move(it->second);
      S->reqs.erase(it);
    }
    if (out) std::copy(r->out.begin(), r->out.end(), out);
    if (present) std::copy(r->present.begin(), r->present.end(), present);
    if (stats) *stats = r->st;
  });
  return g != RELNN_OK ? g : st;
}

extern "C" relnn_status relnn_serve_cancel(relnn_server* S, uint64_t ticket, int32_t* was_admitted) {
  return guard([&] {
    RELNN_REQUIRE(S != nullptr, RELNN_E_INVALID, "NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    RELNN_REQUIRE(it != S->reqs.end() && !it->second->cancelled, RELNN_E_INVALID, "unknown ticket %llu",
                  (unsigned long long)ticket);
    Request* r = it->second.get();
    if (was_admitted) *was_admitted = r->admitted ? 1 : 0;
    if (!r->admitted) {              // still queued: it never runs
      auto q = std::find(S->pending.begin(), S->pending.end(), r);
      if (q != S->pending.end()) S->pending.erase(q);
      S->reqs.erase(it);
    } else if (r->done) {            // finished, not yet polled
      S->reqs.erase(it);
    } else {                         // in the running step: its result is dropped at the step's end
      r->cancelled = true;
    }
  });
}

extern "C" relnn_status relnn_serve_destroy(relnn_server* S) {
  return guard([&] {
    if (!S) return;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stop = true;
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    delete S;
  });
}
