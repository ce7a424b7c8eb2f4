// Super-resolved front end: the coarse design is filled onto the simulation
// grid by a separable interpolation kernel (paper Sec. 3.2, Table 2), and the
// design gradient is carried back by the adjoint map.
//
//   fine = Wy coarse Wx^T,   grad_coarse = Wy^T grad_fine Wx,   W: (nc s) x nc
//
// for a coarse design of ncy rows and ncx columns (each axis has its own W).
//
// Nearest: W[j][i] = [i == j / s].  Lanczos-3: fine sample j sits at coarse
// coordinate u_j = (j + 0.5)/s - 0.5 and takes the six coarse samples
// i0 .. i0+5, i0 = floor(u_j) - 2, weighted by L(u_j - i) with
// L(x) = sinc(x) sinc(x/3) (zero for |x| >= 3 and for i outside [0, nc)),
// each row divided by its sum.  Weights are formed in FP64 and rounded to
// float32; the sums run in float32.
//
// These maps run once per call, not once per wavelength, so they are plain
// LDS-tiled kernels: the coarse patch a fine tile needs is staged in LDS,
// interpolated along y, then along x.

#include <hip/hip_runtime.h>
#include <math.h>

#include "dop_internal.h"

namespace dop {
namespace {

#define DEV __device__ __forceinline__

constexpr int kUpMaxS = 16;

// Lanczos-3 kernel L(x) = sinc(x) sinc(x/3), |x| < 3.
DEV double lanczos3(double x) {
  const double ax = fabs(x);
  if (ax >= 3.0) return 0.0;
  if (ax == 0.0) return 1.0;
  return 3.0 * sinpi(x) * sinpi(x / 3.0) / (M_PI * M_PI * x * x);
}

// Fine sample j = q s + r sits at coarse coordinate u = q + f_r with
// f_r = (r + 0.5)/s - 0.5 in (-1/2, 1/2), so its first tap i0 = floor(u) - 2
// = q + shift_r and its offsets u - i depend on the residue r only.  A block
// tabulates, per residue, the raw kernel values L(u - i0 - t) (FP64) and the
// normalised weights of an interior sample; a sample whose taps leave
// [0, nc) renormalises over the taps inside.
struct TapTable {
  double raw[kUpMaxS][6];
  float wint[kUpMaxS][6];
  int shift[kUpMaxS];
};

DEV void tap_table_fill(TapTable &tt, int s) {
  for (int r = threadIdx.x; r < s; r += blockDim.x) {
    const double f = ((double)r + 0.5) / (double)s - 0.5;
    const int fl = f < 0.0 ? -1 : 0;
    double sum = 0.0;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      tt.raw[r][t] = lanczos3(f - (double)(fl - 2 + t));
      sum += tt.raw[r][t];
    }
#pragma unroll
    for (int t = 0; t < 6; ++t) tt.wint[r][t] = (float)(tt.raw[r][t] / sum);
    tt.shift[r] = fl - 2;
  }
}

// Taps of fine sample j: returns i0 and writes the six normalised weights of
// coarse samples i0 .. i0+5 (zero outside [0, nc)).
DEV int lanczos_taps(int j, int s, int nc, const TapTable &tt, float *w) {
  const int q = j / s, r = j - q * s;
  const int i0 = q + tt.shift[r];
  if (i0 >= 0 && i0 + 5 < nc) {
#pragma unroll
    for (int t = 0; t < 6; ++t) w[t] = tt.wint[r][t];
  } else {
    double v[6];
    double sum = 0.0;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      v[t] = (i0 + t >= 0 && i0 + t < nc) ? tt.raw[r][t] : 0.0;
      sum += v[t];
    }
#pragma unroll
    for (int t = 0; t < 6; ++t) w[t] = (float)(v[t] / sum);
  }
  return i0;
}

// ---------------------------------------------------------------------------
// Nearest neighbour.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_up_nearest(int ncy, int ncx, int s,
                                                    const float *__restrict__ in,
                                                    float *__restrict__ out) {
  const int nfy = ncy * s, nfx = ncx * s;
  for (int y = blockIdx.y; y < nfy; y += gridDim.y) {
    const float *src = in + (size_t)(y / s) * ncx;
    float *dst = out + (size_t)y * nfx;
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < nfx; x += gridDim.x * blockDim.x)
      dst[x] = src[x / s];
  }
}

// Sum of each s x s block of a (ncy s) x (ncx s) map, rows in order, columns
// in order within a row.
__global__ __launch_bounds__(256) void k_up_nearest_adj(int ncy, int ncx, int s,
                                                        const float *__restrict__ g,
                                                        float *__restrict__ out) {
  const int nfx = ncx * s;
  for (int i = blockIdx.y; i < ncy; i += gridDim.y) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < ncx; k += gridDim.x * blockDim.x) {
      float a = 0.f;
      for (int dy = 0; dy < s; ++dy) {
        const float *row = g + (size_t)(i * s + dy) * nfx + (size_t)k * s;
        for (int dx = 0; dx < s; ++dx) a += row[dx];
      }
      out[(size_t)i * ncx + k] = a;
    }
  }
}

// ---------------------------------------------------------------------------
// Lanczos-3, forward: one 64 x 64 fine tile per block.  The taps of the
// tile's first and last rows bound the coarse patch: at most 63/s + 1 + 6
// <= 70 coarse rows (and columns) for s >= 1.
// ---------------------------------------------------------------------------
constexpr int kUpTile = 64;
constexpr int kUpPatch = kUpTile + 6;

__global__ __launch_bounds__(256) void k_up_lanczos(int ncy, int ncx, int s,
                                                    const float *__restrict__ in,
                                                    float *__restrict__ out) {
  const int nfy = ncy * s, nfx = ncx * s;
  __shared__ float rw[kUpTile][6], cw[kUpTile][6];
  __shared__ int rs[kUpTile], cs[kUpTile];
  __shared__ float patch[kUpPatch][kUpPatch + 1];
  __shared__ float vert[kUpTile][kUpPatch + 1];
  __shared__ TapTable tt;
  const int fy0 = blockIdx.y * kUpTile, fx0 = blockIdx.x * kUpTile;
  const int tid = threadIdx.x;
  tap_table_fill(tt, s);
  __syncthreads();
  // taps of every row and column of the tile (clamped to the grid: rows past
  // the edge repeat the last one and are not written)
  if (tid < kUpTile) {
    rs[tid] = lanczos_taps(min(fy0 + tid, nfy - 1), s, ncy, tt, rw[tid]);
  } else if (tid < 2 * kUpTile) {
    const int c = tid - kUpTile;
    cs[c] = lanczos_taps(min(fx0 + c, nfx - 1), s, ncx, tt, cw[c]);
  }
  __syncthreads();
  const int cy0 = rs[0], cx0 = cs[0];
  const int pr = rs[kUpTile - 1] + 6 - cy0;
  const int pc = cs[kUpTile - 1] + 6 - cx0;
  for (int e = tid; e < pr * pc; e += blockDim.x) {
    const int r = e / pc, c = e - (e / pc) * pc;
    const int gy = cy0 + r, gx = cx0 + c;
    patch[r][c] = (gy >= 0 && gy < ncy && gx >= 0 && gx < ncx) ? in[(size_t)gy * ncx + gx] : 0.f;
  }
  __syncthreads();
  // along y: vert[r][c] = sum_t rw[r][t] patch[rs[r] - cy0 + t][c]
  for (int e = tid; e < kUpTile * pc; e += blockDim.x) {
    const int r = e / pc, c = e - (e / pc) * pc;
    const int o = rs[r] - cy0;
    float a = 0.f;
#pragma unroll
    for (int t = 0; t < 6; ++t) a += rw[r][t] * patch[o + t][c];
    vert[r][c] = a;
  }
  __syncthreads();
  // along x
  for (int e = tid; e < kUpTile * kUpTile; e += blockDim.x) {
    const int r = e / kUpTile, c = e % kUpTile;
    const int fy = fy0 + r, fx = fx0 + c;
    if (fy >= nfy || fx >= nfx) continue;
    const int o = cs[c] - cx0;
    float a = 0.f;
#pragma unroll
    for (int t = 0; t < 6; ++t) a += cw[c][t] * vert[r][o + t];
    out[(size_t)fy * nfx + fx] = a;
  }
}

// ---------------------------------------------------------------------------
// Lanczos-3, adjoint: one 16 x 16 coarse tile per block.  Coarse sample i is
// a tap of fine sample j only if floor(u_j) is in [i-3, i+2], i.e. j in
// [s(i-3) - 1, s(i+3) + s]; a tile therefore gathers from at most
// s (16 + 6) + 2 fine rows and as many columns (SPAN for s <= SMAX).  Fine
// rows are staged through LDS 16 at a time, the next chunk loaded into
// registers while the current one is reduced along x into
// hsum[row][coarse col]; the reduction along y follows.
// ---------------------------------------------------------------------------
constexpr int kAdjTile = 16;
constexpr int kAdjChunk = 16;
constexpr int kAdjThreads = 256;

DEV int fine_lo(int i, int s) { return s * (i - 3) - 1; }
DEV int fine_hi(int i, int s) { return s * (i + 3) + s; }

template <int SMAX>
__global__ __launch_bounds__(kAdjThreads) void k_up_lanczos_adj(int ncy, int ncx, int s,
                                                                const float *__restrict__ g,
                                                                float *__restrict__ out) {
  constexpr int SPAN = SMAX * (kAdjTile + 6) + 2;
  constexpr int PF = (kAdjChunk * SPAN + kAdjThreads - 1) / kAdjThreads;
  const int nfy = ncy * s, nfx = ncx * s;
  __shared__ TapTable tt;
  __shared__ float rw[SPAN][6], cw[SPAN][6];
  __shared__ int rs[SPAN], cs[SPAN];
  __shared__ float hsum[SPAN][kAdjTile + 1];
  __shared__ float chunk[kAdjChunk][SPAN + 1];
  const int i0 = blockIdx.y * kAdjTile, k0 = blockIdx.x * kAdjTile;
  const int tid = threadIdx.x;
  const int jlo = max(0, fine_lo(i0, s)), jhi = min(nfy - 1, fine_hi(i0 + kAdjTile - 1, s));
  const int llo = max(0, fine_lo(k0, s)), lhi = min(nfx - 1, fine_hi(k0 + kAdjTile - 1, s));
  const int nj = jhi - jlo + 1, nl = lhi - llo + 1;
  tap_table_fill(tt, s);
  __syncthreads();
  for (int e = tid; e < nj; e += kAdjThreads) rs[e] = lanczos_taps(jlo + e, s, ncy, tt, rw[e]);
  for (int e = tid; e < nl; e += kAdjThreads) cs[e] = lanczos_taps(llo + e, s, ncx, tt, cw[e]);
  float nxt[PF];
  auto load_chunk = [&](int c0) {
    const int rows = min(kAdjChunk, nj - c0);
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = tid + q * kAdjThreads;
      const int r = e / nl, c = e - (e / nl) * nl;
      nxt[q] = r < rows ? g[(size_t)(jlo + c0 + r) * nfx + llo + c] : 0.f;
    }
  };
  const int kk = tid % kAdjTile;  // coarse column of this thread
  const int k = k0 + kk;
  const int clo = max(0, fine_lo(k, s) - llo), chi = min(nl - 1, fine_hi(k, s) - llo);
  load_chunk(0);
  for (int c0 = 0; c0 < nj; c0 += kAdjChunk) {
    const int rows = min(kAdjChunk, nj - c0);
    __syncthreads();  // the previous chunk has been consumed
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = tid + q * kAdjThreads;
      const int r = e / nl, c = e - (e / nl) * nl;
      if (r < rows) chunk[r][c] = nxt[q];
    }
    __syncthreads();
    if (c0 + kAdjChunk < nj) load_chunk(c0 + kAdjChunk);
    const int r = tid / kAdjTile;
    if (r < rows) {
      float a = 0.f;
      for (int c = clo; c <= chi; ++c) {
        const int t = k - cs[c];
        if (t >= 0 && t < 6) a += cw[c][t] * chunk[r][c];
      }
      hsum[c0 + r][kk] = a;
    }
  }
  __syncthreads();
  const int i = i0 + tid / kAdjTile;
  if (i < ncy && k < ncx) {
    const int rlo = max(0, fine_lo(i, s) - jlo), rhi = min(nj - 1, fine_hi(i, s) - jlo);
    float a = 0.f;
    for (int r = rlo; r <= rhi; ++r) {
      const int t = i - rs[r];
      if (t >= 0 && t < 6) a += rw[r][t] * hsum[r][kk];
    }
    out[(size_t)i * ncx + k] = a;
  }
}

unsigned cdiv(int a, int b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

hipError_t launch_upsample(int kind, int ncy, int ncx, int s, const float *coarse, float *fine,
                           hipStream_t stream) {
  const int nfy = ncy * s, nfx = ncx * s;
  if (kind == 0) {
    const dim3 grid(cdiv(nfx, 256) < 64 ? cdiv(nfx, 256) : 64, nfy < 4096 ? nfy : 4096);
    hipLaunchKernelGGL(k_up_nearest, grid, dim3(256), 0, stream, ncy, ncx, s, coarse, fine);
  } else {
    const dim3 grid(cdiv(nfx, kUpTile), cdiv(nfy, kUpTile));
    hipLaunchKernelGGL(k_up_lanczos, grid, dim3(256), 0, stream, ncy, ncx, s, coarse, fine);
  }
  return hipGetLastError();
}

hipError_t launch_upsample_adjoint(int kind, int ncy, int ncx, int s, const float *grad_fine,
                                   float *grad_coarse, hipStream_t stream) {
  if (kind == 0) {
    const dim3 grid(cdiv(ncx, 256) < 64 ? cdiv(ncx, 256) : 64, ncy < 4096 ? ncy : 4096);
    hipLaunchKernelGGL(k_up_nearest_adj, grid, dim3(256), 0, stream, ncy, ncx, s, grad_fine,
                       grad_coarse);
  } else {
    const dim3 grid(cdiv(ncx, kAdjTile), cdiv(ncy, kAdjTile));
    if (s <= 8)
      hipLaunchKernelGGL(k_up_lanczos_adj<8>, grid, dim3(kAdjThreads), 0, stream, ncy, ncx, s,
                         grad_fine, grad_coarse);
    else
      hipLaunchKernelGGL(k_up_lanczos_adj<kUpMaxS>, grid, dim3(kAdjThreads), 0, stream, ncy, ncx,
                         s, grad_fine, grad_coarse);
  }
  return hipGetLastError();
}

}  // namespace dop
