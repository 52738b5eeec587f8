// Error reporting and small queries of the C ABI.
#include <cstdarg>
#include <cstdio>
#include <string>

#include "common.h"

namespace lrvr {

static thread_local std::string g_last_error;

lr_status fail(lr_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

}  // namespace lrvr

LR_API const char* lr_last_error(void) { return lrvr::g_last_error.c_str(); }

LR_API int32_t lr_version(void) { return 200; }

#ifndef LR_BUILD_ID
#define LR_BUILD_ID "unknown"
#endif
LR_API const char* lr_build_id(void) { return LR_BUILD_ID; }

LR_API int64_t lr_bezier_stride(const int32_t p[3], int32_t ncomp, int32_t dtype) {
  if (!p || ncomp < 1) return -1;
  int64_t n = ncomp;
  for (int d = 0; d < 3; ++d) {
    if (p[d] < 1 || p[d] > 3) return -1;
    n *= p[d] + 1;
  }
  const int64_t per16 = dtype == LR_F16 ? 8 : dtype == LR_F32 ? 4 : dtype == LR_F64 ? 2 : 0;
  if (!per16) return -1;
  return (n + per16 - 1) / per16 * per16;
}
