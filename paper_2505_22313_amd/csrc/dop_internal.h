// Internal declarations shared by the libdop host code and its HIP kernels.
#ifndef DOP_INTERNAL_H_
#define DOP_INTERNAL_H_

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dop {

// Size of the shared twiddle table: W[j] = exp(-2 pi i j / kTwN).
constexpr int kTwLog = 17;
constexpr int kTwN = 1 << kTwLog;

// Wavelengths per group: pass A forms, and pass A' accumulates, up to this
// many fields (one workspace field each) per launch.
constexpr int kMaxGroup = 4;

// Row pitch of the M x M workspace, in elements: M + kRowPad.  The pad keeps
// rows that are a power of two apart from landing on the same HBM channels
// (column passes read hundreds of rows at one column offset).
constexpr int kRowPad = 16;

// Pass-A input modes.
enum InMode : int {
  IN_PHASE = 0,  // E = amp * exp(i 2 pi (n-1)/lambda h)        (Eq. 1-2)
  IN_FIELD = 1,  // caller's complex field
  IN_GRAD = 2    // g_U = 2 w_k G * U_k (adjoint seed)
};

// Last-pass output modes.
enum OutMode : int {
  OUT_PSF = 0,    // psf (+)= w_k |U|^2                          (Eq. 4)
  OUT_FIELD = 1,  // complex U
  OUT_GRADH = 2   // grad_h (+)= c_k Im(g_E conj(E_k))
};

// Everything one wavelength's five passes need.  Passed by value.
struct KParams {
  float2 *ws;            // My x Mx c64 workspace (row pitch Mx + kRowPad)
  const float2 *tw;      // twiddle table, kTwN entries
  int n;                 // DOE columns Nx (row length of every N-wide array)
  int plan;              // plan id of the grid (plan_id)
  int nrows_in;          // rows of the padded input that may be nonzero
  int nrows_out;         // rows of the output plane that are needed
  int p0x, p0y;          // (Mx - Nx) / 2, (My - Ny) / 2
  int in_mode, out_mode;
  int full;              // 1: output the whole M x M plane (centred)
  int first;             // 1: overwrite the accumulator, 0: add to it
  int adjoint;           // 1: adjoint pass (H conjugated through zl < 0)
  const float *h;        // heights (IN_PHASE, OUT_GRADH): row y, column x of
                         // the Ny x Nx map is h[(y >> up_log2) * nh + (x >> up_log2)]
  int up_log2;           // log2 of the nearest-neighbour upsampling factor
  int nh;                // row length of h: Nx >> up_log2
  const float *amp;      // N x N amplitude or NULL
  const float2 *u_in;    // N x N field (IN_FIELD)
  const float2 *saved_in;// N x N field U_k (IN_GRAD)
  const float *gpsf;     // N x N dL/dPSF (IN_GRAD)
  float *psf;            // OUT_PSF destination
  float2 *u_out;         // OUT_FIELD destination
  float2 *saved_out;     // optional N x N copy of U_k (OUT_PSF, crop)
  float *grad_h;         // OUT_GRADH destination
  double phase_turns;    // (n_k - 1) / lambda_k  (turns of phase per unit h)
  double zl;             // z / lambda_k (turns at normal incidence); -z / lambda_k
                         // for the adjoint, whose transfer function is conj(H)
  double lam;            // lambda_k
  double inv_mdx;        // 1 / (Mx dx)
  double inv_mdy;        // 1 / (My dx)
  double flim_x;         // band limit on |fx| (infinity: none)
  double flim_y;         // band limit on |fy| (infinity: none)
  float wk_m4;           // w_k / (My Mx)^2: PSF weight times the squared
                         // 1/(My Mx) of the inverse DFT, which the passes
                         // leave to the output
  float two_wk;          // 2 w_k
  float ck_m2;           // 2 pi (n_k - 1) / lambda_k / (My Mx)
  float inv_m2;          // 1 / (My Mx) (inverse-DFT normalisation of output fields)
  int group;             // wavelengths in this launch of pass A (IN_PHASE) or A'
                         // (OUT_PSF, no saved fields): 1, or 2..kMaxGroup with
                         // their fields field_elems apart and the per-wavelength
                         // constants below
  size_t field_elems;    // elements from one field of a group to the next
  double phase_turns_g[kMaxGroup];
  float wk_m4_g[kMaxGroup];
};

constexpr int kNumPasses = 5;

// Enqueue the five passes of one wavelength on `stream`.  If `ev` is not
// NULL, ev[0..5] are recorded before the first pass, between passes and
// after the last one.
hipError_t launch_wavelength(const KParams &p, hipStream_t stream, hipEvent_t *ev);

// Enqueue passes first..last (0 = A, 1 = B, 2 = C, 3 = B', 4 = A') of `p`;
// ev (if not NULL) gets last - first + 2 marks around them.
hipError_t launch_passes(const KParams &p, int first, int last, hipStream_t stream,
                         hipEvent_t *ev);

// Small-grid path: square power-of-two grids of 2^kSmallMinLM .. 2^kSmallMaxLM
// points per side run the PSF (IN_PHASE / OUT_PSF only) as three passes:
// rows, columns with H, rows.  small_path(plan) says whether a plan id is
// one of them; launch_small enqueues one wavelength's three passes, with
// ev[0..3] (if not NULL) recorded before, between and after them.
constexpr int kSmallMinLM = 4;
constexpr int kSmallMaxLM = 11;
bool small_path(int plan);
hipError_t launch_small(const KParams &p, hipStream_t stream, hipEvent_t *ev);

// Largest wavelength group the plan supports (1 if pass A' ends in a
// radix-67 stage), 0 for an unknown plan.
int plan_max_group(int plan);

// Plan id of the My x Mx grid (mx columns, my rows): log2(M) for a square
// power of two M in [16, 131072], a larger id for each grid of the plan
// table, -1 if the grid has no plan.
int plan_id(int mx, int my);

// The grids of the plan table (square grids that are not powers of two,
// and rectangular grids): writes up to `max` (rows, columns) pairs and
// returns how many there are.
int table_grids(int *rows, int *cols, int max);

// Tile geometry of a pass plan (host-side copy of the compile-time plan,
// used for reporting and tests).
struct PlanInfo {
  int ax, bx, ay, by, ra, rc;
  int threads_a, threads_b, threads_c;
};
bool plan_info(int plan, PlanInfo *out);

// Bandwidth probes (dop_probe_bandwidth): pass C's access pattern without its
// arithmetic on the power-of-two grid of plan id `plan` (14..17), and plain
// 16-byte stream kernels over n16 16-byte vectors.  Arguments already
// validated.
hipError_t launch_probe_passc(int plan, float2 *ws, float scale, hipStream_t stream);
hipError_t launch_probe_stream(int kind, void *buf, size_t n16, float scale, hipStream_t stream);

// Super-resolved front end: fine = Wy coarse Wx^T and its adjoint for a
// coarse design of ncy rows and ncx columns (kind 0: nearest, 1: Lanczos-3;
// see dop_upsample).  Arguments already validated.
hipError_t launch_upsample(int kind, int ncy, int ncx, int s, const float *coarse, float *fine,
                           hipStream_t stream);
hipError_t launch_upsample_adjoint(int kind, int ncy, int ncx, int s, const float *grad_fine,
                                   float *grad_coarse, hipStream_t stream);

}  // namespace dop

#endif  // DOP_INTERNAL_H_
