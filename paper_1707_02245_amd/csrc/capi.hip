// Error reporting of the C ABI: status names and the per-thread last message.
#include <cstdarg>
#include <cstdio>

#include "pat_internal.hpp"

namespace pat {

namespace {
thread_local char g_last_error[1024] = "";
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
}

void clear_error() { g_last_error[0] = '\0'; }

}  // namespace pat

extern "C" const char* pat_status_string(pat_status s) {
  switch (s) {
    case PAT_OK: return "PAT_OK";
    case PAT_NOT_CONVERGED: return "PAT_NOT_CONVERGED";
    case PAT_ERR_INVALID_ARG: return "PAT_ERR_INVALID_ARG";
    case PAT_ERR_OOM: return "PAT_ERR_OOM";
    case PAT_ERR_DEVICE: return "PAT_ERR_DEVICE";
    case PAT_ERR_NUMERIC: return "PAT_ERR_NUMERIC";
    case PAT_ERR_UNSUPPORTED: return "PAT_ERR_UNSUPPORTED";
  }
  return "PAT_UNKNOWN_STATUS";
}

extern "C" const char* pat_last_error(void) { return pat::g_last_error; }
