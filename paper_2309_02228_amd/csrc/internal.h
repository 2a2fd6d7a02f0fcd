// Declarations shared by the library's source files (not part of the C ABI).
#pragma once

#include "../../include/mpk.h"

#define MPK_API extern "C" __attribute__((visibility("default")))

namespace mpk {
// Sets the calling thread's message for mpk_last_error and returns `s`.
mpk_status set_error(mpk_status s, const char* fmt, ...);
}  // namespace mpk
