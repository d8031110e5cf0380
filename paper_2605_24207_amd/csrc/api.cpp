// Error reporting and kernel timing of the C ABI.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace relnn {

static thread_local std::string g_error;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
}

// ------------------------------------------------------------------ timing
namespace {
struct Timed {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Timed> g_done;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  RELNN_HIP(hipEventCreate(&e));
  return e;
}
}  // namespace

KTimer::KTimer(const char* name, hipStream_t s) : name_(name), s_(s) {
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_on) return;
  a_ = take_event();
  b_ = take_event();
  RELNN_HIP(hipEventRecord((hipEvent_t)a_, s_));
}

KTimer::~KTimer() {
  if (!a_) return;
  std::lock_guard<std::mutex> g(g_mu);
  if (hipEventRecord((hipEvent_t)b_, s_) == hipSuccess)
    g_done.push_back(Timed{name_, (hipEvent_t)a_, (hipEvent_t)b_});
}

}  // namespace relnn

using namespace relnn;

extern "C" const char* relnn_last_error(void) { return relnn::g_error.c_str(); }

extern "C" relnn_status relnn_timing_enable(int on) {
  return guard([&] {
    std::lock_guard<std::mutex> g(g_mu);
    g_on = on != 0;
  });
}

extern "C" relnn_status relnn_timing_reset(void) {
  return guard([&] {
    std::lock_guard<std::mutex> g(g_mu);
    for (auto& t : g_done) {
      RELNN_HIP(hipEventSynchronize(t.b));
      g_pool.push_back(t.a);
      g_pool.push_back(t.b);
    }
    g_done.clear();
  });
}

extern "C" relnn_status relnn_timing_read(const char* kernel, double* total_ms, int64_t* launches) {
  return guard([&] {
    RELNN_REQUIRE(kernel && total_ms && launches, RELNN_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> g(g_mu);
    double ms = 0.0;
    int64_t n = 0;
    for (auto& t : g_done) {
      if (strcmp(t.name, kernel) != 0) continue;
      RELNN_HIP(hipEventSynchronize(t.b));
      float x = 0.f;
      RELNN_HIP(hipEventElapsedTime(&x, t.a, t.b));
      ms += x;
      ++n;
    }
    *total_ms = ms;
    *launches = n;
  });
}
