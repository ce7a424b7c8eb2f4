// Host-side helpers shared by the libdop C ABI and the serving engine.
#ifndef DOP_HOST_H_
#define DOP_HOST_H_

#include <hip/hip_runtime_api.h>

#include "../../include/dop.h"

namespace dop {

// Record `fmt` as the calling thread's last error and return `s`.
dop_status fail(dop_status s, const char *fmt, ...);
void clear_error();

// Grid and DOE extents of a problem: columns are m and n, rows my and ny
// (0 there means square).
inline int grid_cols(const dop_problem *p) { return p->m; }
inline int grid_rows(const dop_problem *p) { return p->my > 0 ? p->my : p->m; }
inline int doe_cols(const dop_problem *p) { return p->n; }
inline int doe_rows(const dop_problem *p) { return p->ny > 0 ? p->ny : p->n; }

// Full validation of a problem description (no device access).
dop_status validate_problem(const dop_problem *prob);

// Workspace bytes of any operation on `prob` (one My x Mx complex64 field).
size_t workspace_bytes(const dop_problem *prob);

// Enqueue the whole PSF of `prob` (all wavelengths) on `stream`.  A workspace
// of g >= 2 fields (ws_bytes) lets wavelengths run in groups of up to g (see
// psf_group).  With `timed` false the passes are never bracketed by timing
// events, even while profiling is on (so the call creates no events).
dop_status enqueue_psf(const dop_context *ctx, const dop_problem *prob, const float *h,
                       const float *amp, float *psf, void *saved_u, void *ws, size_t ws_bytes,
                       hipStream_t stream, bool timed = true);

// The same for wavelengths kbeg..kend-1 only (0 <= kbeg < kend <= K): their
// terms are added to the PSF (wavelength 0 overwrites it), in the order and
// rounding of the whole call, so consecutive ranges that cover 0..K-1, run in
// order, give the whole call's PSF bitwise.
dop_status enqueue_psf_range(const dop_context *ctx, const dop_problem *prob, int kbeg, int kend,
                             const float *h, const float *amp, float *psf, void *saved_u, void *ws,
                             size_t ws_bytes, hipStream_t stream, bool timed = true);

// Wavelengths per group that dop_psf uses for `prob` with a workspace of
// ws_bytes: as many whole fields as fit, at most the plan's limit and the
// wavelength count, and 1 when the fields are saved.
int psf_group(const dop_problem *prob, const void *saved_u, size_t ws_bytes);

int context_device(const dop_context *ctx);

}  // namespace dop

#endif  // DOP_HOST_H_
