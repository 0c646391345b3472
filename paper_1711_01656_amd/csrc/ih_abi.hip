// Host-side plumbing of the C ABI: error reporting, version, stream cast.
#include <stdarg.h>
#include <stdio.h>

#include "ih_internal.h"

namespace ih {

static thread_local char g_err[512] = "no error";

int set_error(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

int hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return IH_OK;
  return set_error(IH_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace ih

extern "C" int ih_version(void) { return 102; }

extern "C" const char *ih_last_error(void) { return ih::g_err; }
