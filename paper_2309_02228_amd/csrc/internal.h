// Declarations shared by the library's source files (not part of the C ABI).
#pragma once

#include "../../include/mpk.h"

#define MPK_API extern "C" __attribute__((visibility("default")))

namespace mpk {
// Sets the calling thread's message for mpk_last_error and returns `s`.
mpk_status set_error(mpk_status s, const char* fmt, ...);
// True when the plan stores FP64 matrix values on the device.
bool plan_is_f64(mpk_plan_t p);
// MPK_OK when the plan has been uploaded, else MPK_ERR_STATE (message set).
mpk_status plan_uploaded(mpk_plan_t p);
// MPK_SCALE_NONE or MPK_SCALE_JACOBI: whether the plan holds A or A D^{-1}.
int plan_column_scaling(mpk_plan_t p);
// out (device, n, level order) = the stored diagonal of the plan's matrix, on `stream`.
mpk_status plan_diagonal(mpk_plan_t p, double* out, void* stream);
// True when the two plans hold the same matrix size, pattern size and level order.
bool plans_match(mpk_plan_t a, mpk_plan_t b);
}  // namespace mpk
