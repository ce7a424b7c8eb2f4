/*
 * dop.h - C ABI of libdop, an MI355X (gfx950) engine for FFT-based
 * angular-spectrum propagation of large diffractive optical elements.
 *
 * What is computed (Wei et al., "Large-Area Fabrication-Aware Computational
 * Diffractive Optics", ACM TOG 2025, Sec. 3.1):
 *   Eq. (1)  Phi_k(x,y) = 2 pi / lambda_k * (n_k - 1) * h(x,y)
 *   Eq. (2)  E_k = amp * exp(i Phi_k)        (normal plane wave times an
 *                                              optional real aperture)
 *   Eq. (3)  U_k = F^-1{ F{E_k padded} * H_k }
 *            H_k(fx,fy) = exp(i 2 pi z sqrt(1/lambda_k^2 - fx^2 - fy^2))
 *                         when s = (lambda_k fx)^2 + (lambda_k fy)^2 < 1,
 *                         0 otherwise (evanescent cutoff)
 *   Eq. (4)  PSF = sum_k w_k |U_k|^2            (fixed k order)
 * The N x N DOE is zero-padded into an M x M grid at offset
 * p0 = (M - N) / 2 (integer division) on both axes; frequencies are
 * f = k_signed / (M dx) with k_signed = k for k < M/2, k - M otherwise.
 * The backward pass uses the adjoint of Eq. (3), which the paper notes is
 * again a 2-D FFT chain (Sec. 4.1): the same passes with conj(H).
 *
 * Conventions common to every entry point:
 *  - Lengths (dx, z, lambda) share one unit of the caller's choosing.
 *  - Device arrays are row-major, x fastest, caller-owned, and must stay
 *    alive until the work enqueued on `stream` has completed.  Complex
 *    arrays are interleaved float pairs (re, im) ("c64").
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls
 *    enqueue work and return without synchronising.
 *  - Every argument is validated before anything is enqueued.  On any error
 *    nothing is launched and no output is touched; the return value says
 *    why and dop_last_error() (thread-local) gives the detail.
 *  - Results are deterministic: no floating-point atomics, fixed wavelength
 *    order, so the same inputs give bitwise-identical outputs.
 *  - A context may be used from several host threads at once on different
 *    streams, provided each call has its own workspace.
 */
#ifndef DOP_H_
#define DOP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DOP_OK = 0,
  DOP_NOT_READY = 1,            /* serve: ticket still queued or running   */
  DOP_ERR_INVALID_ARG = -1,     /* malformed argument                      */
  DOP_ERR_UNSUPPORTED = -2,     /* valid but not supported (e.g. an M with
                                   no plan, M > 131072)                     */
  DOP_ERR_WORKSPACE = -3,       /* workspace missing or too small          */
  DOP_ERR_DEVICE = -4,          /* HIP runtime or launch failure           */
  DOP_ERR_BUDGET = -5,          /* serve: request can never fit the arena  */
  DOP_ERR_NOT_FOUND = -6,       /* serve: unknown ticket                   */
  DOP_ERR_SHUTDOWN = -7,        /* serve: server is shutting down          */
  DOP_ERR_TIMEOUT = -8          /* serve: wait timed out                   */
} dop_status;

/* Output region of a field or PSF. */
enum {
  DOP_OUT_CROP = 0,  /* N x N window [p0, p0+N)^2 of the propagated plane  */
  DOP_OUT_FULL = 1   /* the whole M x M plane, in centred coordinates      */
};

/* Problem flags. */
enum {
  /* Band-limited ASM (Matsushima & Shimobaba, Opt. Express 17, 19662,
   * 2009; one of the ASM variants the paper cites for Eq. (3)): H is also
   * zero where |fx| >= f_lim or |fy| >= f_lim with
   * f_lim = 1 / (lambda sqrt((2 |z| / (M dx))^2 + 1)), the frequency beyond
   * which the sampled transfer function aliases on the M-point grid. */
  DOP_BANDLIMIT = 1
};

/* Interpolation kernels of the super-resolved front end (dop_upsample). */
enum {
  DOP_UPSAMPLE_NEAREST = 0,  /* fine sample j takes coarse sample j / s      */
  DOP_UPSAMPLE_LANCZOS3 = 1  /* separable Lanczos-3, pixel centres aligned  */
};

/* Operation selector for dop_workspace_size. */
enum { DOP_OP_PROPAGATE = 0, DOP_OP_PSF = 1, DOP_OP_PSF_BACKWARD = 2 };

/* Limits. */
#define DOP_MAX_M 131072
#define DOP_MIN_M 16
#define DOP_MAX_LAMBDA 64
#define DOP_MAX_UPSAMPLE 16

/*
 * Problem description (paper Sec. 3.1: grid, pitch, wavelengths, index,
 * distance, padding).  Host arrays are read during the call only.  In the
 * calls below, "N x N" stands for the DOE's ny rows x n columns and "M x M"
 * for the grid's my rows x m columns.
 */
typedef struct {
  int32_t n;             /* DOE columns (n x n when ny = 0), 1 <= n <= m     */
  int32_t m;             /* padded FFT grid columns (m x m when my = 0).
                            Square grids: a power of two in 16..131072
                            (137 GB of workspace at 131072), or 240, 720,
                            1440, 3072, 3600, 28800 (= 2^7 3^2 5^2), 40000
                            (= 2^6 5^4) and 2144 (= 2^5 67).
                            Rectangular grids (my rows x m columns):
                            720 x 240, 512 x 2048, 240 x 2144, 5360 x 240,
                            16080 x 10720 and 128640 x 85760 (the paper's
                            largest, Table 2: 2^7 3 5 67 x 2^8 5 67, an
                            88 GB workspace).                             */
  double dx;             /* sampling pitch (> 0)                              */
  double z;              /* propagation distance (any sign, 0 allowed)        */
  int32_t n_lambda;      /* K, 1..DOP_MAX_LAMBDA                              */
  const double *lambda;  /* host[K], > 0, same unit as dx                     */
  const double *n_index; /* host[K], refractive index n(lambda_k), finite     */
  const float *weight;   /* host[K] PSF weights w_k, or NULL for all 1        */
  int32_t out_mode;      /* DOP_OUT_CROP or DOP_OUT_FULL                      */
  int32_t flags;         /* 0 or DOP_BANDLIMIT                                */
  int32_t upsample;      /* 0 or 1: h is the n x n map.  2, 4, 8 or 16 (must
                            divide n): h is a coarse design of
                            (n/upsample)^2 samples, nearest-neighbour
                            upsampled to n x n inside the first pass (paper
                            Sec. 3.2, Table 2: 8x nearest upsampling).  amp
                            stays n x n; dop_psf_backward returns the
                            gradient on the coarse grid.  dop_propagate
                            requires 0 or 1.                               */
  int32_t ny;            /* DOE rows; 0 means ny = n.  1 <= ny <= my        */
  int32_t my;            /* padded grid rows; 0 means my = m.  Arrays are
                            row-major (x fastest): the DOE is ny x n, a full
                            plane my x m, and every axis is padded by
                            p0 = (M - N) / 2 on its own (Sec. 3.1 with the
                            rectangular grid of Table 2).                  */
} dop_problem;

typedef struct dop_context dop_context;
typedef struct dop_server dop_server;

/* Human-readable name of a status code (static string). */
const char *dop_status_string(dop_status s);

/* Detail of the last error raised on the calling thread ("" if none). */
const char *dop_last_error(void);

/*
 * Create a context on HIP device `device`: uploads the twiddle table
 * (exp(-2 pi i j / 131072), generated in FP64 and rounded to c64, 1 MiB).
 * The context owns only that table.  Synchronous.
 */
dop_status dop_context_create(int device, dop_context **out);
dop_status dop_context_destroy(dop_context *ctx);

/*
 * Workspace bytes an operation needs for `prob` (op = DOP_OP_*): one M x M
 * c64 field stored with a row pitch of m + 16 elements (8 my (m + 16)
 * bytes), plus, for DOP_OP_PSF_BACKWARD with upsample >= 2, an ny x n
 * float32 fine-grid gradient (starting at the next 256-byte boundary).  Pure
 * host call.
 */
dop_status dop_workspace_size(const dop_context *ctx, const dop_problem *prob,
                              int op, size_t *bytes);

/*
 * Eq. (3) for one wavelength index k (0 <= k < K; lambda[k] is used, n_index
 * and weight are ignored): propagates the N x N c64 field `u_in` (zero-padded
 * to M x M at p0) by z.  `u_out` receives N x N c64 (CROP) or M x M c64
 * (FULL, centred coordinates).  `u_in` and `u_out` must not overlap.
 */
dop_status dop_propagate(dop_context *ctx, const dop_problem *prob, int k,
                         const void *u_in, void *u_out, void *ws,
                         size_t ws_bytes, void *stream);

/*
 * Eq. (1)-(4): PSF = sum_k w_k |U_k|^2 for height map `h` (N x N float32,
 * or the coarse (N/upsample)^2 design when prob->upsample >= 2)
 * and optional aperture `amp` (N x N float32, NULL = 1).  `psf` is
 * overwritten: N x N float32 (CROP) or M x M float32 (FULL).  If `saved_u`
 * is not NULL (CROP only) it receives the fields U_k as K x N x N c64, the
 * state dop_psf_backward needs.
 */
dop_status dop_psf(dop_context *ctx, const dop_problem *prob, const float *h,
                   const float *amp, float *psf, void *saved_u, void *ws,
                   size_t ws_bytes, void *stream);
/* Wavelength groups: when saved_u is NULL and ws_bytes holds g >= 2 whole
 * workspaces of dop_workspace_size(DOP_OP_PSF) bytes, dop_psf runs up to
 * min(g, 4) wavelengths per group (consecutive k): the first pass forms the
 * group's fields from one read of h, and the last pass adds their
 * intensities to the PSF in one read-modify-write.  The result is bitwise
 * the same as one wavelength at a time.  Grids whose x digit has the factor
 * 67 run one wavelength at a time. */

/*
 * dop_psf for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation, arguments and result as dop_psf, bitwise, but the
 * workspace is the library's own device scratch, a static array of
 * DOP_NOALLOC_MAX_BYTES that each device holds until the process ends (its
 * address is looked up once per device when a context is created).  The
 * call allocates nothing and creates no events (it is not timed by
 * dop_profile_*).  Problems whose workspace (dop_workspace_size with
 * DOP_OP_PSF) exceeds DOP_NOALLOC_MAX_BYTES, i.e. grids larger than
 * 4096 x 4096, are rejected with DOP_ERR_WORKSPACE before anything is
 * enqueued; up to four wavelengths run as one group when their fields fit.
 * All calls on one device share its scratch and leave their last contents
 * in it: calls whose work overlaps on one device (different streams, or
 * host threads without ordering) race and give wrong results.  Nothing in
 * the scratch needs clearing between calls.
 */
#define DOP_NOALLOC_MAX_BYTES ((size_t)167772160) /* 160 MiB */

dop_status dop_psf_noalloc(dop_context *ctx, const dop_problem *prob, const float *h,
                           const float *amp, float *psf, void *saved_u, void *stream);

/*
 * Gradient of a real loss L with respect to h, given grad_psf = dL/dPSF
 * (N x N float32, CROP only) and the fields saved by dop_psf (K x N x N c64).
 * Per wavelength: g_U = 2 w_k G U_k, g_E = adjoint of Eq. (3) applied to g_U
 * (conj(H_k)), dL/dh += c_k Im(g_E conj(E_k)) with c_k = 2 pi (n_k - 1) /
 * lambda_k and E_k recomputed from h and amp.  `grad_h` (N x N float32,
 * or (N/upsample)^2 when prob->upsample >= 2: the fine gradient summed over
 * each upsample x upsample block) is overwritten.
 */
dop_status dop_psf_backward(dop_context *ctx, const dop_problem *prob,
                            const float *h, const float *amp,
                            const void *saved_u, const float *grad_psf,
                            float *grad_h, void *ws, size_t ws_bytes,
                            void *stream);

/* ------------------------------------------------------------------------
 * Super-resolved front end (paper Sec. 3.2 and Table 2: designs on a coarse
 * feature grid simulated on an s-times finer grid, filled by nearest
 * neighbour, or by a smooth Lanczos-3 kernel, the interpolation kernels of
 * its Fig. 4 comparison).  Both maps are separable: fine = W coarse W^T with
 * a one-axis matrix W of shape (nc s, nc).
 *   NEAREST:  W[j][i] = 1 iff i = floor(j / s).
 *   LANCZOS3: fine sample j sits at coarse coordinate u = (j + 0.5)/s - 0.5;
 *             W[j][i] = L(u - i) for |u - i| < 3 and 0 <= i < nc, with
 *             L(x) = sinc(x) sinc(x/3), each row divided by its sum
 *             (weights in FP64, rounded to float32; sums in float32).
 * Arguments: kind = DOP_UPSAMPLE_*, coarse grid nc x nc (nc >= 1), factor
 * s in 1..DOP_MAX_UPSAMPLE, nc * s <= DOP_MAX_M.  All arrays are device
 * float32, row-major, caller-owned and must not overlap.  Asynchronous on
 * `stream`; arguments are validated before anything is enqueued.
 * ---------------------------------------------------------------------- */

/* fine ((nc s) x (nc s)) = W coarse (nc x nc) W^T. */
dop_status dop_upsample(dop_context *ctx, int kind, int nc, int s,
                        const float *coarse, float *fine, void *stream);

/* grad_coarse (nc x nc) = W^T grad_fine ((nc s) x (nc s)) W: the adjoint,
 * which carries a fine-grid gradient back to the coarse design (for NEAREST,
 * the sum over each s x s block). */
dop_status dop_upsample_adjoint(dop_context *ctx, int kind, int nc, int s,
                                const float *grad_fine, float *grad_coarse,
                                void *stream);

/* The same two maps for a rectangular design of ncy rows and ncx columns
 * (each axis has its own W, fine = Wy coarse Wx^T, grad_coarse = Wy^T
 * grad_fine Wx; the paper's large-area design is 16,080 x 10,720 samples):
 * coarse ncy x ncx, fine (ncy s) x (ncx s), the same limits per axis.
 * dop_upsample and dop_upsample_adjoint are these with ncy = ncx = nc. */
dop_status dop_upsample_rect(dop_context *ctx, int kind, int ncy, int ncx, int s,
                             const float *coarse, float *fine, void *stream);
dop_status dop_upsample_adjoint_rect(dop_context *ctx, int kind, int ncy, int ncx,
                                     int s, const float *grad_fine,
                                     float *grad_coarse, void *stream);

/* ------------------------------------------------------------------------
 * Per-pass timing.  While enabled, every wavelength's five passes are
 * bracketed by HIP events on the stream they run on; dop_profile_read waits
 * for the recorded events and returns, per pass, the launch count and the
 * summed event-to-event time.  Enabling clears the accumulators.  Timing
 * adds one event record between consecutive passes and is off by default.
 * Pass names: "pass_a_fwd", "pass_b_fwd", "pass_c", "pass_b_inv",
 * "pass_a_inv" (the kernels dop::k_pass_*<log2 M>).
 * ---------------------------------------------------------------------- */

#define DOP_NUM_PASSES 5

typedef struct {
  char name[32];
  uint64_t launches;
  double total_ms;
} dop_pass_profile;

dop_status dop_profile_enable(dop_context *ctx, int enable);
dop_status dop_profile_read(dop_context *ctx, dop_pass_profile *out, int max, int *count);

/* ------------------------------------------------------------------------
 * Bandwidth probes: the HBM ceilings the passes are measured against (the
 * paper notes that memory, not arithmetic, limits the FFT propagation,
 * Sec. 4).  Each call enqueues one kernel on `stream` over the caller's
 * device buffer `buf` (`bytes`, 256-byte aligned, a multiple of 64; its
 * contents are overwritten) and reports the bytes the kernel moves in
 * *moved:
 *   DOP_PROBE_READ     reads every byte of buf              (moved = bytes)
 *   DOP_PROBE_WRITE    writes every byte                    (moved = bytes)
 *   DOP_PROBE_COPY     copies the first half onto the second (moved = bytes)
 *   DOP_PROBE_INPLACE  reads and writes back every byte     (moved = 2 bytes)
 * with 16-byte accesses and non-temporal hints, and
 *   DOP_PROBE_PASSC    pass C's access pattern without its arithmetic, on
 *                      the field of the square power-of-two grid m (16384
 *                      .. 131072; buf holds 8 m (m + 16) bytes): the same
 *                      tiles, tile order, grid, prefetch, register layout and
 *                      LDS footprint, each element read and written back in
 *                      place                            (moved = 16 m^2).
 * m is ignored by the stream kinds.  Validated before anything is enqueued.
 * ---------------------------------------------------------------------- */
enum {
  DOP_PROBE_READ = 0,
  DOP_PROBE_WRITE = 1,
  DOP_PROBE_COPY = 2,
  DOP_PROBE_INPLACE = 3,
  DOP_PROBE_PASSC = 4
};

dop_status dop_probe_bandwidth(dop_context *ctx, int kind, void *buf, size_t bytes, int m,
                               size_t *moved, void *stream);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of PSF requests (dop_psf, CROP or FULL) of
 * mixed sizes and wavelength counts.  The server sub-allocates workspaces
 * from a caller-provided device arena (it never calls hipMalloc per request),
 * admits queued requests as request slots and arena memory free up, and runs
 * their work on streams of its own while others are still running (see the
 * policies below).  Each request's result is bitwise the same as dop_psf on
 * its own.  Thread-safe.
 * ---------------------------------------------------------------------- */

typedef struct {
  uint64_t submitted;     /* requests accepted by dop_serve_submit           */
  uint64_t completed;     /* requests finished (ok or failed)                */
  uint64_t failed;        /* requests that finished with an error            */
  uint32_t queued;        /* waiting for admission                           */
  uint32_t running;       /* admitted and not yet finished                   */
  uint64_t arena_bytes;   /* arena size                                      */
  uint64_t arena_peak;    /* peak bytes sub-allocated                        */
  double p50_ms;          /* latency (submit -> done) percentiles over all   */
  double p99_ms;          /*   completed requests                            */
  double mean_ms;
} dop_serve_stats;

/*
 * Create a server on `ctx` with `max_slots` (1..64) concurrent requests,
 * sub-allocating from `arena` (device memory, `arena_bytes`, caller-owned,
 * alive until dop_serve_destroy returns).  Starts one scheduler thread.
 */
dop_status dop_serve_create(dop_context *ctx, void *arena, size_t arena_bytes,
                            int max_slots, dop_server **out);

/*
 * Queue a PSF request.  `prob` and its host arrays are copied.  `h` (N x N
 * float32, or the coarse design when prob->upsample >= 2), `amp` (N x N
 * float32 or NULL; an addition to the serving calls of the paper-derived
 * boundary, so that aperture-masked requests can be served) and `psf`
 * (output, as dop_psf) are device buffers that must stay alive until the
 * ticket completes.  The server runs the request on streams of its own that
 * are not ordered after any stream of the caller: `h` and `amp` must already
 * hold their final values when dop_serve_submit is called (complete, e.g.
 * synchronise, the work that produces them first), and nothing may read or
 * write `psf` until the ticket is done.
 * DOP_ERR_BUDGET if the request could never fit the arena.
 */
dop_status dop_serve_submit(dop_server *srv, const dop_problem *prob,
                            const float *h, const float *amp, float *psf,
                            uint64_t *ticket);

/* Scheduling policies.
 *   DOP_SERVE_CHUNKED (default): a request runs in chunks of one wavelength
 *     group (up to four wavelengths; its workspace holds that many fields,
 *     at most half the arena, or as many fields as fit at admission).
 *     All chunks go through one in-order stream, two enqueued at a time
 *     (up to eight while those hold under 1e8 padded pixels x wavelengths,
 *     about a millisecond of work); each time a chunk completes, the next
 *     is taken from the admitted request with the least work left
 *     (n_lambda not yet enqueued x my x m), except that requests older than
 *     the age bound (seconds since submit) go first, oldest first.  A
 *     request arriving while a large one runs waits only for the chunks
 *     already enqueued (two of a large grid's); the large one pauses but
 *     never shares the GPU.  Admission takes the head of the queue first; while the head
 *     does not fit and is younger than the age bound, later requests that
 *     fit (among the next 32) may be admitted ahead of it.
 *   DOP_SERVE_FIFO: admission in submission order; a request's whole PSF is
 *     enqueued at admission on its slot's stream, beside whatever runs.
 *   DOP_SERVE_SIZE_AWARE: as FIFO, but while requests run the head starts
 *     only if its work (n_lambda * my * m) is at most share_ratio times the
 *     largest running request's; otherwise it waits for the GPU to drain. */
enum { DOP_SERVE_FIFO = 0, DOP_SERVE_SIZE_AWARE = 1, DOP_SERVE_CHUNKED = 2 };

/* Set the policy for requests not yet admitted (admitted ones finish under
 * the policy they were admitted with).  `param` (finite, >= 0) is the age
 * bound in seconds for DOP_SERVE_CHUNKED (default 0.25; 0 serves chunks
 * oldest request first), share_ratio for DOP_SERVE_SIZE_AWARE (default
 * 0.25), and ignored for DOP_SERVE_FIFO. */
dop_status dop_serve_set_policy(dop_server *srv, int policy, double param);

/* DOP_OK when done, DOP_NOT_READY while queued/running, or the request's
 * error.  A finished ticket can be polled any number of times. */
dop_status dop_serve_poll(dop_server *srv, uint64_t ticket);

/* Block until the ticket is done (DOP_OK or its error) or `timeout_s`
 * (< 0: forever) elapses (DOP_ERR_TIMEOUT). */
dop_status dop_serve_wait(dop_server *srv, uint64_t ticket, double timeout_s);

/* Latency (ms, submit -> done) of a finished ticket. */
dop_status dop_serve_latency(dop_server *srv, uint64_t ticket, double *ms);

dop_status dop_serve_stats_get(dop_server *srv, dop_serve_stats *out);

/* Stop admitting, cancel queued requests (DOP_ERR_SHUTDOWN), wait for
 * running ones, free everything.  No other call on `srv` may be in progress
 * or follow (tickets die with the server). */
dop_status dop_serve_destroy(dop_server *srv);

/*
 * Test hook: a server whose executor is a host-side mock instead of the GPU.
 * Its streams are in-order queues of wall time: a chunk of k wavelengths
 * (a whole request under FIFO / SIZE_AWARE) occupies its stream for
 * service_us_per_mpix * (k * my * m / 1e6) microseconds and writes nothing.
 * `arena` is only used as an address range (may be any non-NULL value).
 * For CPU tests of admission, scheduling, budget, order and shutdown; needs
 * no GPU.
 */
dop_status dop_serve_create_mock(void *arena, size_t arena_bytes,
                                 int max_slots, double service_us_per_mpix,
                                 dop_server **out);

#ifdef __cplusplus
}
#endif

#endif /* DOP_H_ */
