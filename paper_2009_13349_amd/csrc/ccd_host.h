// Host-side internals shared by the runtime and the serving loop.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ccd.h"
#include "ccd_internal.h"

namespace ccd {

// Plans scratch for a launch of a.n queries (largest m_I = mi_max), grows the
// context's buffers and enqueues the kernel sequence on stream s.
int run_args(ccd_context* ctx, BatchArgs a, int64_t mi_max, hipStream_t s);

// Grows the context's scratch for launches of up to n queries with m_I up to
// mi_max, so that later launches of that size allocate nothing.
int reserve(ccd_context* ctx, int64_t n, int64_t mi_max);

// The validation rule of a query (same as the kernels').
bool host_valid(const double X[24], int kind, double delta, int64_t max_iter, double min_sep);

// Records a failed HIP call for ccd_last_error(); returns e == hipSuccess.
bool record_hip(hipError_t e, const char* what);
void set_last_error(const char* msg);

}  // namespace ccd
