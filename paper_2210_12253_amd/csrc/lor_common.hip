// Error state and small ABI entry points of the LOR library.
#include "lor_common.hpp"

namespace lor {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

}  // namespace lor

extern "C" const char* lor_last_error(void) { return lor::g_last_error.c_str(); }

extern "C" int lor_abi_version(void) { return 3; }

extern "C" size_t lor_sched_bytes(void) { return sizeof(lor_sched); }
