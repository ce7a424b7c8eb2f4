// Host-side helpers shared by the libdop C ABI and the serving engine.
#ifndef DOP_HOST_H_
#define DOP_HOST_H_

#include <hip/hip_runtime.h>

#include "../../include/dop.h"

namespace dop {

// Record `fmt` as the calling thread's last error and return `s`.
dop_status fail(dop_status s, const char *fmt, ...);
void clear_error();

// Full validation of a problem description (no device access).
dop_status validate_problem(const dop_problem *prob);

// Workspace bytes of any operation on `prob` (one M x M complex64 field).
size_t workspace_bytes(const dop_problem *prob);

// Enqueue the whole PSF of `prob` (all wavelengths) on `stream`.
dop_status enqueue_psf(const dop_context *ctx, const dop_problem *prob, const float *h,
                       const float *amp, float *psf, void *saved_u, void *ws, hipStream_t stream);

int context_device(const dop_context *ctx);

}  // namespace dop

#endif  // DOP_HOST_H_
