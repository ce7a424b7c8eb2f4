// libdop C ABI: argument validation, context (twiddle table), workspace query
// and the per-wavelength orchestration of the propagation passes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dop.h"
#include "dop_internal.h"
#include "dop_host.h"

// Scratch memory of the no-allocation entry point dop_psf_noalloc: the
// workspace fields of problems up to DOP_NOALLOC_MAX_BYTES.  Each device the
// library runs on holds its own copy until the process ends.  In host code
// `scratch` names a host-side stand-in, not device memory: its address on
// each device is looked up once (scratch_on_device) and only that address is
// handed to kernels.
static __device__ __align__(256) unsigned char scratch[DOP_NOALLOC_MAX_BYTES];

struct dop_context {
  int device = 0;
  float2 *tw = nullptr;  // kTwN complex64 twiddles exp(-2 pi i j / kTwN)
  void *scratch = nullptr;  // device address of `scratch` on this device
  // per-pass timing (off unless enabled)
  std::mutex prof_mu;
  bool prof_on = false;
  std::vector<hipEvent_t> prof_pool;            // idle events
  // marks around launched passes: interval i (ev[i] -> ev[i + 1]) is pass
  // slot[i] (one more event than passes)
  struct Pending {
    std::vector<hipEvent_t> ev;
    std::vector<int> slot;
  };
  std::vector<Pending> pending;
  double prof_ms[dop::kNumPasses] = {0, 0, 0, 0, 0};
  uint64_t prof_n[dop::kNumPasses] = {0, 0, 0, 0, 0};
};

namespace dop {

static thread_local std::string g_last_error;

dop_status fail(dop_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

void clear_error() { g_last_error.clear(); }

// Device address of `scratch` on `device`, which must be the current device:
// looked up once per device and kept; NULL if the lookup failed.
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices];

static void *scratch_on_device(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess && ptr)
      g_scratch_dev[device] = ptr;
    else
      (void)hipGetLastError();  // leave no sticky error behind
  }
  return g_scratch_dev[device];
}

static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
static bool aligned(const void *p, size_t a) { return reinterpret_cast<uintptr_t>(p) % a == 0; }
static int upsample_factor(const dop_problem *prob) {
  return prob->upsample <= 1 ? 1 : prob->upsample;
}
static int ilog2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

dop_status validate_problem(const dop_problem *prob) {
  if (!prob) return fail(DOP_ERR_INVALID_ARG, "problem is NULL");
  if (prob->n < 1) return fail(DOP_ERR_INVALID_ARG, "n must be >= 1 (got %d)", prob->n);
  if (prob->m < 1) return fail(DOP_ERR_INVALID_ARG, "m must be >= 1 (got %d)", prob->m);
  if (prob->ny < 0) return fail(DOP_ERR_INVALID_ARG, "ny must be >= 0 (got %d)", prob->ny);
  if (prob->my < 0) return fail(DOP_ERR_INVALID_ARG, "my must be >= 0 (got %d)", prob->my);
  const int mx = grid_cols(prob), my = grid_rows(prob);
  if (plan_id(mx, my) < 0) {
    int gr[32], gc[32];
    const int ng = table_grids(gr, gc, 32);
    std::string list;
    for (int i = 0; i < ng && i < 32; ++i)
      list += (i ? ", " : "") + (gr[i] == gc[i] ? std::to_string(gc[i]) + "^2"
                                                : std::to_string(gr[i]) + "x" + std::to_string(gc[i]));
    return fail(DOP_ERR_UNSUPPORTED,
                "grid %d rows x %d columns has no plan: square powers of two in [%d, %d] and "
                "%s (rows x columns)", my, mx, DOP_MIN_M, DOP_MAX_M, list.c_str());
  }
  if (prob->n > mx) return fail(DOP_ERR_INVALID_ARG, "n (%d) exceeds m (%d)", prob->n, mx);
  if (doe_rows(prob) > my)
    return fail(DOP_ERR_INVALID_ARG, "ny (%d) exceeds my (%d)", doe_rows(prob), my);
  if (!(prob->dx > 0.0) || !std::isfinite(prob->dx))
    return fail(DOP_ERR_INVALID_ARG, "dx must be finite and > 0");
  if (!std::isfinite(prob->z)) return fail(DOP_ERR_INVALID_ARG, "z must be finite");
  if (prob->n_lambda < 1 || prob->n_lambda > DOP_MAX_LAMBDA)
    return fail(DOP_ERR_INVALID_ARG, "n_lambda must be in [1, %d] (got %d)", DOP_MAX_LAMBDA,
                prob->n_lambda);
  if (!prob->lambda) return fail(DOP_ERR_INVALID_ARG, "lambda array is NULL");
  if (!prob->n_index) return fail(DOP_ERR_INVALID_ARG, "n_index array is NULL");
  for (int k = 0; k < prob->n_lambda; ++k) {
    if (!(prob->lambda[k] > 0.0) || !std::isfinite(prob->lambda[k]))
      return fail(DOP_ERR_INVALID_ARG, "lambda[%d] must be finite and > 0", k);
    if (!std::isfinite(prob->n_index[k]))
      return fail(DOP_ERR_INVALID_ARG, "n_index[%d] must be finite", k);
    if (prob->weight && !std::isfinite(prob->weight[k]))
      return fail(DOP_ERR_INVALID_ARG, "weight[%d] must be finite", k);
  }
  if (prob->out_mode != DOP_OUT_CROP && prob->out_mode != DOP_OUT_FULL)
    return fail(DOP_ERR_INVALID_ARG, "out_mode must be DOP_OUT_CROP or DOP_OUT_FULL");
  if (prob->flags & ~DOP_BANDLIMIT)
    return fail(DOP_ERR_UNSUPPORTED, "unknown flags 0x%x", (unsigned)prob->flags);
  if (prob->upsample < 0 || prob->upsample > DOP_MAX_UPSAMPLE || !is_pow2(upsample_factor(prob)))
    return fail(DOP_ERR_UNSUPPORTED, "upsample must be 0, 1, 2, 4, 8 or 16 (got %d)",
                prob->upsample);
  if (prob->n % upsample_factor(prob) != 0 || doe_rows(prob) % upsample_factor(prob) != 0)
    return fail(DOP_ERR_INVALID_ARG, "upsample factor %d does not divide n = %d and ny = %d",
                prob->upsample, prob->n, doe_rows(prob));
  // The phase and transfer arguments are reduced in FP64; beyond ~2^40 turns
  // their fractional part would carry no bits.
  for (int k = 0; k < prob->n_lambda; ++k) {
    if (std::fabs(prob->z / prob->lambda[k]) > 1e12)
      return fail(DOP_ERR_UNSUPPORTED, "|z / lambda[%d]| exceeds 1e12 turns", k);
  }
  return DOP_OK;
}

size_t workspace_bytes(const dop_problem *prob) {
  return (size_t)grid_rows(prob) * ((size_t)grid_cols(prob) + kRowPad) * sizeof(float2);
}

// Byte offset of the fine-grid gradient in a DOP_OP_PSF_BACKWARD workspace
// (present when the design is upsampled): after the field, 256-byte aligned.
static size_t fine_grad_offset(const dop_problem *prob) {
  return (workspace_bytes(prob) + 255) & ~(size_t)255;
}

static size_t workspace_bytes_op(const dop_problem *prob, int op) {
  if (op == DOP_OP_PSF_BACKWARD && upsample_factor(prob) > 1)
    return fine_grad_offset(prob) + (size_t)doe_rows(prob) * prob->n * sizeof(float);
  return workspace_bytes(prob);
}

// Band limit of the sampled transfer function (see DOP_BANDLIMIT), formed
// exactly as 1 / (lambda sqrt(t t + 1)), t = 2 |z| / (M dx), without FMA
// contraction, so the mask matches a plain FP64 evaluation bin for bin.  m is
// the length of the axis the limit applies to.
static double band_limit(double lam, double z, int m, double dx) {
#pragma clang fp contract(off)
  const double t = 2.0 * std::fabs(z) / ((double)m * dx);
  return 1.0 / (lam * std::sqrt(t * t + 1.0));
}

// Fill the per-wavelength kernel parameters shared by every operation.
void fill_common(KParams &kp, const dop_context *ctx, const dop_problem *prob, int k, void *ws) {
  std::memset(&kp, 0, sizeof(kp));
  kp.ws = static_cast<float2 *>(ws);
  kp.tw = ctx->tw;
  const int mx = grid_cols(prob), my = grid_rows(prob);
  kp.n = prob->n;
  kp.plan = plan_id(mx, my);
  kp.nrows_in = doe_rows(prob);
  kp.p0x = (mx - prob->n) / 2;
  kp.p0y = (my - doe_rows(prob)) / 2;
  kp.up_log2 = ilog2i(upsample_factor(prob));
  kp.nh = prob->n >> kp.up_log2;
  const double lam = prob->lambda[k];
  kp.lam = lam;
  kp.zl = prob->z / lam;
  kp.inv_mdx = 1.0 / ((double)mx * prob->dx);
  kp.inv_mdy = 1.0 / ((double)my * prob->dx);
  const bool bl = (prob->flags & DOP_BANDLIMIT) != 0;
  kp.flim_x = bl ? band_limit(lam, prob->z, mx, prob->dx) : HUGE_VAL;
  kp.flim_y = bl ? band_limit(lam, prob->z, my, prob->dx) : HUGE_VAL;
  kp.phase_turns = (prob->n_index[k] - 1.0) / lam;
  const float w = prob->weight ? prob->weight[k] : 1.0f;
  const double m2 = (double)mx * (double)my;
  kp.wk_m4 = (float)((double)w / (m2 * m2));
  kp.two_wk = 2.0f * w;
  kp.ck_m2 = (float)(2.0 * M_PI * (prob->n_index[k] - 1.0) / lam / m2);
  kp.inv_m2 = (float)(1.0 / m2);
  kp.group = 1;
  kp.field_elems = workspace_bytes(prob) / sizeof(float2);
}

// Timing events for `n` consecutive passes while profiling is on (empty
// otherwise, or when `timed` is false).
static dop_status take_events(dop_context *ctx, int n, bool timed, std::vector<hipEvent_t> *ev) {
  if (!timed) return DOP_OK;
  std::lock_guard<std::mutex> lk(ctx->prof_mu);
  if (!ctx->prof_on) return DOP_OK;
  while ((int)ev->size() < n + 1) {
    hipEvent_t e = nullptr;
    if (!ctx->prof_pool.empty()) {
      e = ctx->prof_pool.back();
      ctx->prof_pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      return fail(DOP_ERR_DEVICE, "hipEventCreate failed");
    }
    ev->push_back(e);
  }
  return DOP_OK;
}

static void keep_events(dop_context *ctx, std::vector<hipEvent_t> &ev, std::vector<int> slot) {
  if (ev.empty()) return;
  std::lock_guard<std::mutex> lk(ctx->prof_mu);
  ctx->pending.push_back({std::move(ev), std::move(slot)});
}

// Enqueue passes first..last of kp (0 = A ... 4 = A'), bracketed by timing
// events while profiling is on.
dop_status launch_range(const dop_context *cctx, const KParams &kp, int first, int last,
                        hipStream_t stream, bool timed = true) {
  dop_context *ctx = const_cast<dop_context *>(cctx);
  std::vector<hipEvent_t> ev;
  dop_status s = take_events(ctx, last - first + 1, timed, &ev);
  if (s != DOP_OK) return s;
  const hipError_t e = launch_passes(kp, first, last, stream, ev.empty() ? nullptr : ev.data());
  std::vector<int> slot;
  for (int i = first; i <= last; ++i) slot.push_back(i);
  keep_events(ctx, ev, std::move(slot));
  if (e != hipSuccess) return fail(DOP_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return DOP_OK;
}

// One wavelength of the small-grid path (rows, columns with H, rows); its
// passes are timed as pass_a_fwd, pass_c and pass_a_inv.
static dop_status launch_small_wavelength(const dop_context *cctx, const KParams &kp,
                                          hipStream_t stream, bool timed) {
  dop_context *ctx = const_cast<dop_context *>(cctx);
  std::vector<hipEvent_t> ev;
  dop_status s = take_events(ctx, 3, timed, &ev);
  if (s != DOP_OK) return s;
  const hipError_t e = launch_small(kp, stream, ev.empty() ? nullptr : ev.data());
  keep_events(ctx, ev, {0, 2, 4});
  if (e != hipSuccess)
    return fail(DOP_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return DOP_OK;
}

dop_status launch(const dop_context *ctx, const KParams &kp, hipStream_t stream) {
  return launch_range(ctx, kp, 0, kNumPasses - 1, stream);
}

dop_status check_ctx_device(const dop_context *ctx) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(DOP_ERR_DEVICE, "hipGetDevice failed");
  if (cur != ctx->device)
    return fail(DOP_ERR_INVALID_ARG, "current HIP device %d differs from the context's device %d",
                cur, ctx->device);
  return DOP_OK;
}

int psf_group(const dop_problem *prob, const void *saved_u, size_t ws_bytes) {
  if (saved_u || small_path(plan_id(grid_cols(prob), grid_rows(prob)))) return 1;
  const size_t field = workspace_bytes(prob);
  const int g = plan_max_group(plan_id(grid_cols(prob), grid_rows(prob)));
  const size_t fit = ws_bytes / field;
  int r = prob->n_lambda < g ? prob->n_lambda : g;
  if (fit < (size_t)r) r = (int)fit;
  return r < 1 ? 1 : r;
}

dop_status enqueue_psf(const dop_context *ctx, const dop_problem *prob, const float *h,
                       const float *amp, float *psf, void *saved_u, void *ws, size_t ws_bytes,
                       hipStream_t stream, bool timed) {
  return enqueue_psf_range(ctx, prob, 0, prob->n_lambda, h, amp, psf, saved_u, ws, ws_bytes,
                           stream, timed);
}

dop_status enqueue_psf_range(const dop_context *ctx, const dop_problem *prob, int kbeg, int kend,
                             const float *h, const float *amp, float *psf, void *saved_u, void *ws,
                             size_t ws_bytes, hipStream_t stream, bool timed) {
  const size_t nn = (size_t)doe_rows(prob) * prob->n;
  const int g = psf_group(prob, saved_u, ws_bytes);
  auto setup = [&](KParams &kp, int k, void *field) {
    fill_common(kp, ctx, prob, k, field);
    kp.in_mode = IN_PHASE;
    kp.out_mode = OUT_PSF;
    kp.full = prob->out_mode == DOP_OUT_FULL;
    kp.nrows_out = kp.full ? grid_rows(prob) : doe_rows(prob);
    kp.h = h;
    kp.amp = amp;
    kp.psf = psf;
  };
  for (int k0 = kbeg; k0 < kend;) {
    const int gk = kend - k0 < g ? kend - k0 : g;
    if (gk == 1) {
      KParams kp;
      setup(kp, k0, ws);
      kp.first = (k0 == 0);
      kp.saved_out = saved_u ? static_cast<float2 *>(saved_u) + (size_t)k0 * nn : nullptr;
      const dop_status s = small_path(kp.plan)
                               ? launch_small_wavelength(ctx, kp, stream, timed)
                               : launch_range(ctx, kp, 0, kNumPasses - 1, stream, timed);
      if (s != DOP_OK) return s;
    } else {
      // a group: pass A forms the gk fields from one read of the heights,
      // passes B, C, B' run per field, pass A' adds the gk intensities to
      // the PSF in one read-modify-write (the same sums in the same order
      // as one wavelength at a time)
      KParams g0;
      setup(g0, k0, ws);
      g0.first = (k0 == 0);
      g0.group = gk;
      for (int q = 0; q < gk; ++q) {
        KParams kq;
        setup(kq, k0 + q, ws);
        g0.phase_turns_g[q] = kq.phase_turns;
        g0.wk_m4_g[q] = kq.wk_m4;
      }
      dop_status s = launch_range(ctx, g0, 0, 0, stream, timed);
      if (s != DOP_OK) return s;
      for (int q = 0; q < gk; ++q) {
        KParams kq;
        setup(kq, k0 + q, static_cast<float2 *>(ws) + (size_t)q * g0.field_elems);
        s = launch_range(ctx, kq, 1, 3, stream, timed);
        if (s != DOP_OK) return s;
      }
      s = launch_range(ctx, g0, kNumPasses - 1, kNumPasses - 1, stream, timed);
      if (s != DOP_OK) return s;
    }
    k0 += gk;
  }
  return DOP_OK;
}

}  // namespace dop

using namespace dop;

extern "C" {

const char *dop_status_string(dop_status s) {
  switch (s) {
    case DOP_OK: return "DOP_OK";
    case DOP_NOT_READY: return "DOP_NOT_READY";
    case DOP_ERR_INVALID_ARG: return "DOP_ERR_INVALID_ARG";
    case DOP_ERR_UNSUPPORTED: return "DOP_ERR_UNSUPPORTED";
    case DOP_ERR_WORKSPACE: return "DOP_ERR_WORKSPACE";
    case DOP_ERR_DEVICE: return "DOP_ERR_DEVICE";
    case DOP_ERR_BUDGET: return "DOP_ERR_BUDGET";
    case DOP_ERR_NOT_FOUND: return "DOP_ERR_NOT_FOUND";
    case DOP_ERR_SHUTDOWN: return "DOP_ERR_SHUTDOWN";
    case DOP_ERR_TIMEOUT: return "DOP_ERR_TIMEOUT";
  }
  return "DOP_UNKNOWN_STATUS";
}

const char *dop_last_error(void) { return g_last_error.c_str(); }

dop_status dop_context_create(int device, dop_context **out) {
  clear_error();
  if (!out) return fail(DOP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
    return fail(DOP_ERR_DEVICE, "no HIP device available");
  if (device < 0 || device >= count)
    return fail(DOP_ERR_INVALID_ARG, "device %d out of range [0, %d)", device, count);
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(device) != hipSuccess) return fail(DOP_ERR_DEVICE, "hipSetDevice(%d) failed", device);
  // FP64-generated twiddles, rounded once to complex64.
  std::vector<float2> host(kTwN);
  for (int j = 0; j < kTwN; ++j) {
    const double a = -2.0 * M_PI * (double)j / (double)kTwN;
    host[j] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  dop_context *ctx = new dop_context();
  ctx->device = device;
  hipError_t e = hipMalloc(reinterpret_cast<void **>(&ctx->tw), sizeof(float2) * kTwN);
  if (e == hipSuccess)
    e = hipMemcpy(ctx->tw, host.data(), sizeof(float2) * kTwN, hipMemcpyHostToDevice);
  // the no-allocation entry point's scratch on this device (NULL: that entry
  // point reports the failure; everything else works without it)
  if (e == hipSuccess) ctx->scratch = scratch_on_device(device);
  (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    if (ctx->tw) (void)hipFree(ctx->tw);
    delete ctx;
    return fail(DOP_ERR_DEVICE, "twiddle upload failed: %s", hipGetErrorString(e));
  }
  *out = ctx;
  return DOP_OK;
}

dop_status dop_context_destroy(dop_context *ctx) {
  clear_error();
  if (!ctx) return fail(DOP_ERR_INVALID_ARG, "context is NULL");
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  for (auto &pl : ctx->pending)
    for (hipEvent_t e : pl.ev) {
      (void)hipEventSynchronize(e);
      (void)hipEventDestroy(e);
    }
  for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
  if (ctx->tw) (void)hipFree(ctx->tw);
  (void)hipSetDevice(prev);
  delete ctx;
  return DOP_OK;
}

static const char *kPassNames[kNumPasses] = {"pass_a_fwd", "pass_b_fwd", "pass_c", "pass_b_inv",
                                             "pass_a_inv"};

// Wait for the pending events and fold their intervals into the totals.
static dop_status collect(dop_context *ctx) {
  for (auto &pl : ctx->pending) {
    const std::vector<hipEvent_t> &v = pl.ev;
    if (hipEventSynchronize(v.back()) != hipSuccess)
      return fail(DOP_ERR_DEVICE, "hipEventSynchronize failed");
    for (size_t i = 0; i + 1 < v.size(); ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, v[i], v[i + 1]) != hipSuccess)
        return fail(DOP_ERR_DEVICE, "hipEventElapsedTime failed");
      ctx->prof_ms[pl.slot[i]] += ms;
      ctx->prof_n[pl.slot[i]] += 1;
    }
    for (hipEvent_t e : v) ctx->prof_pool.push_back(e);
  }
  ctx->pending.clear();
  return DOP_OK;
}

dop_status dop_profile_enable(dop_context *ctx, int enable) {
  clear_error();
  if (!ctx) return fail(DOP_ERR_INVALID_ARG, "context is NULL");
  std::lock_guard<std::mutex> lk(ctx->prof_mu);
  const dop_status s = collect(ctx);
  if (s != DOP_OK) return s;
  if (enable) {
    for (int i = 0; i < kNumPasses; ++i) {
      ctx->prof_ms[i] = 0;
      ctx->prof_n[i] = 0;
    }
  }
  ctx->prof_on = enable != 0;
  return DOP_OK;
}

dop_status dop_profile_read(dop_context *ctx, dop_pass_profile *out, int max, int *count) {
  clear_error();
  if (!ctx || !out || !count) return fail(DOP_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(ctx->prof_mu);
  const dop_status s = collect(ctx);
  if (s != DOP_OK) return s;
  const int n = max < kNumPasses ? max : kNumPasses;
  for (int i = 0; i < n; ++i) {
    std::memset(&out[i], 0, sizeof(out[i]));
    std::strncpy(out[i].name, kPassNames[i], sizeof(out[i].name) - 1);
    out[i].launches = ctx->prof_n[i];
    out[i].total_ms = ctx->prof_ms[i];
  }
  *count = n;
  return DOP_OK;
}

dop_status dop_probe_bandwidth(dop_context *ctx, int kind, void *buf, size_t bytes, int m,
                               size_t *moved, void *stream) {
  clear_error();
  if (!ctx) return fail(DOP_ERR_INVALID_ARG, "context is NULL");
  if (!buf || !moved) return fail(DOP_ERR_INVALID_ARG, "buf / moved must not be NULL");
  if (!aligned(buf, 256)) return fail(DOP_ERR_INVALID_ARG, "buf must be 256-byte aligned");
  if (bytes < 64 || bytes % 64 != 0)
    return fail(DOP_ERR_INVALID_ARG, "bytes must be a positive multiple of 64 (got %zu)", bytes);
  if (kind < DOP_PROBE_READ || kind > DOP_PROBE_PASSC)
    return fail(DOP_ERR_INVALID_ARG, "unknown probe kind %d", kind);
  size_t mv = 0;
  if (kind == DOP_PROBE_PASSC) {
    if (m < 16384 || m > DOP_MAX_M || !is_pow2(m))
      return fail(DOP_ERR_UNSUPPORTED, "the pass-C probe needs m = 16384 .. %d, a power of two "
                  "(got %d)", DOP_MAX_M, m);
    const size_t need = (size_t)m * ((size_t)m + kRowPad) * sizeof(float2);
    if (bytes < need)
      return fail(DOP_ERR_WORKSPACE, "buf has %zu bytes, the %d^2 field needs %zu", bytes, m, need);
    mv = 2 * sizeof(float2) * (size_t)m * (size_t)m;
  } else {
    mv = kind == DOP_PROBE_INPLACE ? 2 * bytes : bytes;
  }
  dop_status s = check_ctx_device(ctx);
  if (s != DOP_OK) return s;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const hipError_t e = kind == DOP_PROBE_PASSC
                           ? launch_probe_passc(ilog2i(m), static_cast<float2 *>(buf), 1.0f, st)
                           : launch_probe_stream(kind, buf, bytes / 16, 1.0f, st);
  if (e != hipSuccess) return fail(DOP_ERR_DEVICE, "probe launch failed: %s", hipGetErrorString(e));
  *moved = mv;
  return DOP_OK;
}

dop_status dop_workspace_size(const dop_context *ctx, const dop_problem *prob, int op,
                              size_t *bytes) {
  clear_error();
  (void)ctx;
  if (!bytes) return fail(DOP_ERR_INVALID_ARG, "bytes is NULL");
  if (op != DOP_OP_PROPAGATE && op != DOP_OP_PSF && op != DOP_OP_PSF_BACKWARD)
    return fail(DOP_ERR_INVALID_ARG, "unknown op %d", op);
  const dop_status s = validate_problem(prob);
  if (s != DOP_OK) return s;
  *bytes = workspace_bytes_op(prob, op);
  return DOP_OK;
}

static dop_status check_ws(const dop_problem *prob, int op, void *ws, size_t ws_bytes) {
  if (!ws) return fail(DOP_ERR_WORKSPACE, "workspace is NULL");
  if (ws_bytes < workspace_bytes_op(prob, op))
    return fail(DOP_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes,
                workspace_bytes_op(prob, op));
  if (reinterpret_cast<uintptr_t>(ws) % 16 != 0)
    return fail(DOP_ERR_WORKSPACE, "workspace must be 16-byte aligned");
  return DOP_OK;
}


dop_status dop_propagate(dop_context *ctx, const dop_problem *prob, int k, const void *u_in,
                         void *u_out, void *ws, size_t ws_bytes, void *stream) {
  clear_error();
  if (!ctx) return fail(DOP_ERR_INVALID_ARG, "context is NULL");
  dop_status s = validate_problem(prob);
  if (s != DOP_OK) return s;
  if (k < 0 || k >= prob->n_lambda)
    return fail(DOP_ERR_INVALID_ARG, "k=%d out of range [0, %d)", k, prob->n_lambda);
  if (!u_in || !u_out) return fail(DOP_ERR_INVALID_ARG, "u_in / u_out must not be NULL");
  if (!aligned(u_in, 8) || !aligned(u_out, 8))
    return fail(DOP_ERR_INVALID_ARG, "complex arrays must be 8-byte aligned");
  if (upsample_factor(prob) != 1)
    return fail(DOP_ERR_INVALID_ARG, "upsample applies to height maps; dop_propagate needs 0 or 1");
  if ((s = check_ws(prob, DOP_OP_PROPAGATE, ws, ws_bytes)) != DOP_OK) return s;
  if ((s = check_ctx_device(ctx)) != DOP_OK) return s;
  KParams kp;
  fill_common(kp, ctx, prob, k, ws);
  kp.in_mode = IN_FIELD;
  kp.out_mode = OUT_FIELD;
  kp.full = prob->out_mode == DOP_OUT_FULL;
  kp.nrows_out = kp.full ? grid_rows(prob) : doe_rows(prob);
  kp.first = 1;
  kp.u_in = static_cast<const float2 *>(u_in);
  kp.u_out = static_cast<float2 *>(u_out);
  return launch(ctx, kp, static_cast<hipStream_t>(stream));
}

// Checks of dop_psf's arguments other than the workspace.
static dop_status check_psf_args(const dop_context *ctx, const dop_problem *prob, const float *h,
                                 const float *amp, const float *psf, const void *saved_u) {
  if (!ctx) return fail(DOP_ERR_INVALID_ARG, "context is NULL");
  const dop_status s = validate_problem(prob);
  if (s != DOP_OK) return s;
  if (!h || !psf) return fail(DOP_ERR_INVALID_ARG, "h / psf must not be NULL");
  if (!aligned(h, 4) || !aligned(psf, 4) || (amp && !aligned(amp, 4)))
    return fail(DOP_ERR_INVALID_ARG, "float arrays must be 4-byte aligned");
  if (saved_u && prob->out_mode != DOP_OUT_CROP)
    return fail(DOP_ERR_UNSUPPORTED, "saved_u requires DOP_OUT_CROP");
  if (saved_u && !aligned(saved_u, 8))
    return fail(DOP_ERR_INVALID_ARG, "saved_u must be 8-byte aligned");
  return DOP_OK;
}

dop_status dop_psf(dop_context *ctx, const dop_problem *prob, const float *h, const float *amp,
                   float *psf, void *saved_u, void *ws, size_t ws_bytes, void *stream) {
  clear_error();
  dop_status s = check_psf_args(ctx, prob, h, amp, psf, saved_u);
  if (s != DOP_OK) return s;
  if ((s = check_ws(prob, DOP_OP_PSF, ws, ws_bytes)) != DOP_OK) return s;
  if ((s = check_ctx_device(ctx)) != DOP_OK) return s;
  return enqueue_psf(ctx, prob, h, amp, psf, saved_u, ws, ws_bytes,
                     static_cast<hipStream_t>(stream));
}

dop_status dop_psf_noalloc(dop_context *ctx, const dop_problem *prob, const float *h,
                           const float *amp, float *psf, void *saved_u, void *stream) {
  clear_error();
  dop_status s = check_psf_args(ctx, prob, h, amp, psf, saved_u);
  if (s != DOP_OK) return s;
  const size_t need = workspace_bytes_op(prob, DOP_OP_PSF);
  if (need > (size_t)DOP_NOALLOC_MAX_BYTES)
    return fail(DOP_ERR_WORKSPACE,
                "grid %d x %d needs %zu bytes of workspace; the scratch of dop_psf_noalloc holds "
                "%zu bytes (grids up to 4096 x 4096)",
                grid_rows(prob), grid_cols(prob), need, (size_t)DOP_NOALLOC_MAX_BYTES);
  if (!ctx->scratch)
    return fail(DOP_ERR_DEVICE, "the device scratch of dop_psf_noalloc is not available on "
                "device %d", ctx->device);
  if ((s = check_ctx_device(ctx)) != DOP_OK) return s;
  // every workspace element a pass reads has been written earlier in the same
  // call (pass A writes the input rows, pass B every row), so the scratch
  // left by an earlier call needs no clearing; no timing events are created
  return enqueue_psf(ctx, prob, h, amp, psf, saved_u, ctx->scratch, DOP_NOALLOC_MAX_BYTES,
                     static_cast<hipStream_t>(stream), false);
}

dop_status dop_psf_backward(dop_context *ctx, const dop_problem *prob, const float *h,
                            const float *amp, const void *saved_u, const float *grad_psf,
                            float *grad_h, void *ws, size_t ws_bytes, void *stream) {
  clear_error();
  if (!ctx) return fail(DOP_ERR_INVALID_ARG, "context is NULL");
  dop_status s = validate_problem(prob);
  if (s != DOP_OK) return s;
  if (prob->out_mode != DOP_OUT_CROP)
    return fail(DOP_ERR_UNSUPPORTED, "dop_psf_backward supports DOP_OUT_CROP only");
  if (!h || !saved_u || !grad_psf || !grad_h)
    return fail(DOP_ERR_INVALID_ARG, "h / saved_u / grad_psf / grad_h must not be NULL");
  if (!aligned(h, 4) || !aligned(grad_psf, 4) || !aligned(grad_h, 4) || !aligned(saved_u, 8) ||
      (amp && !aligned(amp, 4)))
    return fail(DOP_ERR_INVALID_ARG, "misaligned array");
  if ((s = check_ws(prob, DOP_OP_PSF_BACKWARD, ws, ws_bytes)) != DOP_OK) return s;
  if ((s = check_ctx_device(ctx)) != DOP_OK) return s;
  const size_t nn = (size_t)doe_rows(prob) * prob->n;
  const int up = upsample_factor(prob);
  // with an upsampled design the passes accumulate the n x n fine gradient in
  // the workspace tail; its s x s block sums are the coarse gradient
  float *grad_fine =
      up > 1 ? reinterpret_cast<float *>(static_cast<char *>(ws) + fine_grad_offset(prob)) : grad_h;
  for (int k = 0; k < prob->n_lambda; ++k) {
    KParams kp;
    fill_common(kp, ctx, prob, k, ws);
    kp.in_mode = IN_GRAD;
    kp.out_mode = OUT_GRADH;
    kp.full = 0;
    kp.nrows_out = doe_rows(prob);
    kp.first = (k == 0);
    kp.adjoint = 1;
    kp.zl = -kp.zl;  // conj(H) = H at -z (the band limit depends on |z| only)
    kp.h = h;
    kp.amp = amp;
    kp.gpsf = grad_psf;
    kp.saved_in = static_cast<const float2 *>(saved_u) + (size_t)k * nn;
    kp.grad_h = grad_fine;
    s = launch(ctx, kp, static_cast<hipStream_t>(stream));
    if (s != DOP_OK) return s;
  }
  if (up > 1) {
    const hipError_t e = launch_upsample_adjoint(DOP_UPSAMPLE_NEAREST, doe_rows(prob) / up,
                                                 prob->n / up, up, grad_fine, grad_h,
                                                 static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
      return fail(DOP_ERR_DEVICE, "upsample adjoint launch failed: %s", hipGetErrorString(e));
  }
  return DOP_OK;
}

static dop_status check_upsample_args(const dop_context *ctx, int kind, int ncy, int ncx, int s,
                                      const void *in, const void *out) {
  if (!ctx) return fail(DOP_ERR_INVALID_ARG, "context is NULL");
  if (kind != DOP_UPSAMPLE_NEAREST && kind != DOP_UPSAMPLE_LANCZOS3)
    return fail(DOP_ERR_INVALID_ARG, "unknown upsample kind %d", kind);
  if (ncy < 1 || ncx < 1)
    return fail(DOP_ERR_INVALID_ARG, "coarse grid must be at least 1 x 1 (got %d x %d)", ncy, ncx);
  if (s < 1 || s > DOP_MAX_UPSAMPLE)
    return fail(DOP_ERR_UNSUPPORTED, "factor must be in [1, %d] (got %d)", DOP_MAX_UPSAMPLE, s);
  if ((long long)ncy * s > DOP_MAX_M || (long long)ncx * s > DOP_MAX_M)
    return fail(DOP_ERR_UNSUPPORTED, "fine grid %lld x %lld exceeds %d", (long long)ncy * s,
                (long long)ncx * s, DOP_MAX_M);
  if (!in || !out) return fail(DOP_ERR_INVALID_ARG, "arrays must not be NULL");
  if (!aligned(in, 4) || !aligned(out, 4))
    return fail(DOP_ERR_INVALID_ARG, "float arrays must be 4-byte aligned");
  const char *a = static_cast<const char *>(in), *b = static_cast<const char *>(out);
  const size_t na = (size_t)ncy * ncx * sizeof(float);
  const size_t nb = (size_t)ncy * s * ((size_t)ncx * s) * sizeof(float);
  if (a < b + nb && b < a + na) return fail(DOP_ERR_INVALID_ARG, "input and output overlap");
  return check_ctx_device(ctx);
}

dop_status dop_upsample_rect(dop_context *ctx, int kind, int ncy, int ncx, int s,
                             const float *coarse, float *fine, void *stream) {
  clear_error();
  const dop_status st = check_upsample_args(ctx, kind, ncy, ncx, s, coarse, fine);
  if (st != DOP_OK) return st;
  const hipError_t e =
      launch_upsample(kind, ncy, ncx, s, coarse, fine, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(DOP_ERR_DEVICE, "upsample launch failed: %s", hipGetErrorString(e));
  return DOP_OK;
}

dop_status dop_upsample_adjoint_rect(dop_context *ctx, int kind, int ncy, int ncx, int s,
                                     const float *grad_fine, float *grad_coarse, void *stream) {
  clear_error();
  const dop_status st = check_upsample_args(ctx, kind, ncy, ncx, s, grad_coarse, grad_fine);
  if (st != DOP_OK) return st;
  const hipError_t e = launch_upsample_adjoint(kind, ncy, ncx, s, grad_fine, grad_coarse,
                                               static_cast<hipStream_t>(stream));
  if (e != hipSuccess)
    return fail(DOP_ERR_DEVICE, "upsample adjoint launch failed: %s", hipGetErrorString(e));
  return DOP_OK;
}

dop_status dop_upsample(dop_context *ctx, int kind, int nc, int s, const float *coarse, float *fine,
                        void *stream) {
  return dop_upsample_rect(ctx, kind, nc, nc, s, coarse, fine, stream);
}

dop_status dop_upsample_adjoint(dop_context *ctx, int kind, int nc, int s, const float *grad_fine,
                                float *grad_coarse, void *stream) {
  return dop_upsample_adjoint_rect(ctx, kind, nc, nc, s, grad_fine, grad_coarse, stream);
}

}  // extern "C"

int dop::context_device(const dop_context *ctx) { return ctx->device; }
