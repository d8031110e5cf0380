// Error reporting of the C ABI.
#include <stdarg.h>
#include <stdio.h>

#include <string>

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

}  // namespace relnn

extern "C" const char* relnn_last_error(void) { return relnn::g_error.c_str(); }
