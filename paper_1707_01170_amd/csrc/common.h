// Internal helpers shared by the library's translation units.
#pragma once

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/lrvr.h"

#define LR_API extern "C" __attribute__((visibility("default")))

namespace lrvr {

// Records the message for lr_last_error() and returns the status.
lr_status fail(lr_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

inline bool is_pow2(int32_t v) { return v > 0 && (v & (v - 1)) == 0; }

inline bool fp32_exact(double v) { return (double)(float)v == v; }

}  // namespace lrvr
