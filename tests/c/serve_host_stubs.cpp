// Host-only stand-ins for what the serving engine (csrc/dop_serve.cpp) links
// against, so that the scheduler, its arena and its condition variables can
// be built with GCC's thread, address and undefined-behaviour sanitizers and
// driven through the mock executor without a GPU or the HIP runtime.
//
// Only the mock executor runs in these builds: the HIP entry points below
// report "not supported" and the GPU enqueue reports a device error, so a
// stray GPU path fails loudly instead of touching a device.
#include <hip/hip_runtime_api.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/dop.h"
#include "../../paper_2505_22313_amd/csrc/dop_host.h"

namespace dop {

static thread_local std::string g_err;

dop_status fail(dop_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

void clear_error() { g_err.clear(); }

// The checks the scheduler relies on (sizes and the wavelength arrays); the
// full validation lives in the library and is tested there.
dop_status validate_problem(const dop_problem *p) {
  if (!p) return fail(DOP_ERR_INVALID_ARG, "problem is NULL");
  if (p->n < 1 || p->m < p->n || grid_rows(p) < doe_rows(p))
    return fail(DOP_ERR_INVALID_ARG, "bad sizes");
  if (p->n_lambda < 1 || p->n_lambda > DOP_MAX_LAMBDA || !p->lambda || !p->n_index)
    return fail(DOP_ERR_INVALID_ARG, "bad wavelengths");
  return DOP_OK;
}

// One My x Mx complex64 field with a row pitch of Mx + 16, as the library.
size_t workspace_bytes(const dop_problem *p) {
  return (size_t)grid_rows(p) * ((size_t)grid_cols(p) + 16) * 8;
}

dop_status enqueue_psf(const dop_context *, const dop_problem *, const float *, const float *,
                       float *, void *, void *, size_t, hipStream_t, bool) {
  return fail(DOP_ERR_DEVICE, "no GPU in the host sanitizer build");
}

dop_status enqueue_psf_range(const dop_context *, const dop_problem *, int, int, const float *,
                             const float *, float *, void *, void *, size_t, hipStream_t, bool) {
  return fail(DOP_ERR_DEVICE, "no GPU in the host sanitizer build");
}

// Wavelength groups as the library forms them: up to four, as many as fit.
int psf_group(const dop_problem *p, const void *saved_u, size_t ws_bytes) {
  if (saved_u) return 1;
  const size_t fit = ws_bytes / workspace_bytes(p);
  int g = p->n_lambda < 4 ? p->n_lambda : 4;
  if (fit < (size_t)g) g = (int)fit;
  return g < 1 ? 1 : g;
}

int context_device(const dop_context *) { return 0; }

}  // namespace dop

extern "C" {
hipError_t hipSetDevice(int) { return hipErrorNotSupported; }
hipError_t hipStreamCreateWithFlags(hipStream_t *, unsigned int) { return hipErrorNotSupported; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipErrorNotSupported; }
hipError_t hipStreamDestroy(hipStream_t) { return hipErrorNotSupported; }
hipError_t hipEventCreateWithFlags(hipEvent_t *, unsigned) { return hipErrorNotSupported; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipEventQuery(hipEvent_t) { return hipErrorNotSupported; }
hipError_t hipEventDestroy(hipEvent_t) { return hipErrorNotSupported; }
}

extern "C" const char *dop_last_error(void) { return dop::g_err.c_str(); }
