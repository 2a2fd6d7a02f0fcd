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
// Whether the plan records the lower-triangle masks of the GS2 chain (split_lower).
bool plan_split_lower(mpk_plan_t p);
// The plan's powers per blocked launch (p_block).
int plan_p_block(mpk_plan_t p);
// MPK_SCALE_NONE or MPK_SCALE_JACOBI: whether the plan holds A or A D^{-1}.
int plan_column_scaling(mpk_plan_t p);
// out (device, n, level order) = the stored diagonal of the plan's matrix, on `stream`.
mpk_status plan_diagonal(mpk_plan_t p, double* out, void* stream);
// The Jacobi chain in level order (plan holding A D^{-1}): Y[(q-1) ldy + i] receives power
// q = 1..p of x under A P^{-1} = I - (I - B)^k, each link closing with (A P^{-1} w - lam_q w)
// / sig_q (lam, sig: host arrays of p, or NULL for 0 and 1).  work: the ring of p_block + 2
// vectors of n doubles.
mpk_status jacobi_chain(mpk_plan_t p, int k, const double* x, double* Y, int64_t ldy, int pw, const double* lam,
                        const double* sig, uint32_t flags, void* work, size_t work_bytes, void* stream);
// The GS2 chain in level order (plan built with split_lower): Y[(q-1) ldy + i] receives
// power q = 1..p of x, each power gamma + 2 sub-powers closing with (A g_gamma - lam_q w)
// / sig_q (lam, sig: host arrays of p, or NULL for 0 and 1), or, with pinv, gamma + 1
// sub-powers closing with g_gamma = P^{-1} w.  work: the ring of p_block + gamma + 2
// vectors of (n + 31) / 32 * 32 doubles.  No argument checks beyond the ring size.
mpk_status gs2_chain(mpk_plan_t p, int gamma, const double* x, double* Y, int64_t ldy, int pw, const double* lam,
                     const double* sig, int pinv, uint32_t flags, void* work, size_t work_bytes, void* stream);
// True when the two plans hold the same matrix size, pattern size and level order.
bool plans_match(mpk_plan_t a, mpk_plan_t b);
}  // namespace mpk
