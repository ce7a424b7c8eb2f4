// HIP kernels for CDNA4 (gfx950): FFT-based angular-spectrum propagation of a
// DOE, Eq. (1)-(4) of Wei et al., "Large-Area Fabrication-Aware Computational
// Diffractive Optics" (Sec. 3.1).
//
// One wavelength = five passes over an M x M complex64 field held in HBM.
// Each axis index is split into two digits,
//     x = BX * xa + xb,   y = BY * ya + yb      (M = AX * BX = AY * BY),
// and the 2-D FFT is the row-column decomposition of the paper's Sec. 4.1
// carried one step further: the 1-D transforms along x and y are themselves
// four-step (digit) transforms.  Forward transforms work in place and leave
// the spectrum in digit-transposed order (position BX*kxa + kxb holds
// frequency kxa + AX*kxb), the single-GPU analogue of the paper keeping the
// spectrum in swapped sharding; the transfer function is evaluated at that
// order and the inverse transforms undo it.
//
//   A  : DFT over xa (stride BX) of the N input rows.  Forms the DOE field
//        from h on the fly (Eq. 1-2); columns >= N are implicit zeros.
//   B  : DFT over xb (contiguous) and over ya (stride BY rows), one tile.
//        Rows >= N are implicit zeros.
//   C  : DFT over yb, multiply by H (Eq. 3, evaluated per element with an
//        FP64 argument, never stored), inverse DFT over yb.  Fused.
//   B' : inverse of B; only the rows that are needed are written.
//   A' : inverse of A, then |U|^2 with the wavelength weight accumulated into
//        the PSF (Eq. 4), or the field, or the height gradient.
//
// The DOE sits at the corner of the padded grid internally; propagation is a
// circular convolution, so the centred placement of the paper's grids is the
// same result shifted by p0 = (M - N)/2, applied when writing a full plane.
//
// Within a pass each tile lives in LDS and its DFTs run as Stockham radix
// 16/8/4 stages in registers.  Inner twiddles and four-step twiddles come
// from one FP64-generated complex64 table of exp(-2 pi i j / 65536).

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dop_internal.h"

namespace dop {

#define DEV __device__ __forceinline__

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
DEV float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
DEV float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
DEV float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
DEV float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
DEV float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }   // -i a
DEV float2 mul_pi(float2 a) { return make_float2(-a.y, a.x); }   // +i a
DEV float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// v * w16^q with w16 = exp(-2 pi i / 16) (forward) or its conjugate (INV).
// q is a compile-time constant after unrolling, so the switch folds away.
template <bool INV>
DEV float2 mulw16(float2 v, int q) {
  q &= 15;
  if (q == 0) return v;
  if (q == 4) return INV ? mul_pi(v) : mul_mi(v);
  if (q == 8) return make_float2(-v.x, -v.y);
  if (q == 12) return INV ? mul_mi(v) : mul_pi(v);
  // cos(2 pi q/16), sin(2 pi q/16)
  constexpr float C1 = 0.923879532511286756128f;  // cos(pi/8)
  constexpr float S1 = 0.382683432365089771728f;  // sin(pi/8)
  constexpr float RT = 0.707106781186547524401f;  // cos(pi/4)
  float c = 0.f, s = 0.f;
  switch (q) {
    case 1: c = C1; s = S1; break;
    case 2: c = RT; s = RT; break;
    case 3: c = S1; s = C1; break;
    case 5: c = -S1; s = C1; break;
    case 6: c = -RT; s = RT; break;
    case 7: c = -C1; s = S1; break;
    case 9: c = -C1; s = -S1; break;
    case 10: c = -RT; s = -RT; break;
    case 11: c = -S1; s = -C1; break;
    case 13: c = S1; s = -C1; break;
    case 14: c = RT; s = -RT; break;
    case 15: c = C1; s = -S1; break;
    default: break;
  }
  const float sn = INV ? s : -s;  // w = c + i*sn
  return make_float2(v.x * c - v.y * sn, v.x * sn + v.y * c);
}

// ---------------------------------------------------------------------------
// In-register DFTs of length 2, 4, 8, 16 (natural order in and out).
// Forward: X[k] = sum_n a[n] exp(-2 pi i n k / R); INV flips the sign.
// ---------------------------------------------------------------------------
template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<1, INV> {
  DEV static void run(float2 *) {}
};

template <bool INV>
struct Dft<2, INV> {
  DEV static void run(float2 *a) {
    const float2 t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  }
};

template <bool INV>
struct Dft<4, INV> {
  DEV static void run(float2 *a) {
    const float2 t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    const float2 t2 = cadd(a[1], a[3]), t3 = csub(a[1], a[3]);
    const float2 it3 = INV ? mul_pi(t3) : mul_mi(t3);
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, it3);
    a[3] = csub(t1, it3);
  }
};

// R = 4 * R2 (R = 8, 16): four-step split n = n1*R2 + n2, k = k1 + 4*k2.
template <int R, bool INV>
struct Dft {
  static_assert(R == 8 || R == 16, "radix");
  static constexpr int R2 = R / 4;
  DEV static void run(float2 *a) {
    float2 t[R];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      float2 b[4];
#pragma unroll
      for (int n1 = 0; n1 < 4; ++n1) b[n1] = a[n1 * R2 + n2];
      Dft<4, INV>::run(b);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1)
        t[k1 * R2 + n2] = mulw16<INV>(b[k1], n2 * k1 * (16 / R));
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 c[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) c[n2] = t[k1 * R2 + n2];
      Dft<R2, INV>::run(c);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) a[k1 + 4 * k2] = c[k2];
    }
  }
};

// ---------------------------------------------------------------------------
// Stockham stage plan for an L-point DFT (L = 2..1024).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

__host__ __device__ constexpr int num_stages(int L) { return L <= 16 ? 1 : (L <= 256 ? 2 : 3); }

__host__ __device__ constexpr int fwd_radix(int L, int s) {
  return L <= 16 ? L
       : L == 32 ? (s == 0 ? 8 : 4)
       : L == 64 ? 8
       : L == 128 ? (s == 0 ? 16 : 8)
       : L == 256 ? 16
       : L == 512 ? (s == 0 ? 16 : (s == 1 ? 8 : 4))
       : (s == 0 ? 16 : 8);  // 1024
}

// REV reverses the radix order (used by the inverse half of the fused middle
// pass so that it starts with the radix the forward half ended with).
__host__ __device__ constexpr int stage_radix(int L, int s, bool rev) {
  return rev ? fwd_radix(L, num_stages(L) - 1 - s) : fwd_radix(L, s);
}

__host__ __device__ constexpr int stage_ns(int L, int s, bool rev) {
  return s == 0 ? 1 : stage_ns(L, s - 1, rev) * stage_radix(L, s - 1, rev);
}

// Tile geometry: element (j, b) of the tile (j = transform index in [0, L),
// b = batch index in [0, NB)) lives at LDS offset j*SJ + b*SB.  JFAST chooses
// whether consecutive threads walk j or b.
template <int L_, int NB_, int SJ_, int SB_, int T_, bool JFAST_>
struct Geo {
  static constexpr int L = L_, NB = NB_, SJ = SJ_, SB = SB_, T = T_;
  static constexpr bool JFAST = JFAST_;
};

enum { SRC_LDS = 0, SRC_FN = 1, SRC_REG = 2 };
enum { SNK_LDS = 0, SNK_FN = 1, SNK_REG = 2 };

template <class G, int R>
struct StageShape {
  static constexpr int LR = G::L / R;
  static constexpr int ITEMS = LR * G::NB;
  static constexpr int PER = (ITEMS + G::T - 1) / G::T;
  static constexpr bool EXACT = (ITEMS % G::T) == 0;
};

template <class G, int R>
DEV void decode_item(int it, int &j, int &b) {
  constexpr int LR = G::L / R;
  if constexpr (G::JFAST) {
    j = it & (LR - 1);
    b = it / LR;
  } else {
    b = it & (G::NB - 1);
    j = it / G::NB;
  }
}

// Register block handed between the forward and inverse halves of pass C.
template <class G, bool REV>
struct LastRegs {
  static constexpr int R = stage_radix(G::L, num_stages(G::L) - 1, REV);
  static constexpr int PER = StageShape<G, R>::PER;
};

// One Stockham stage S of the L-point DFT along j for every b, followed by the
// remaining stages.  The first stage reads from SRC (LDS, a load functor
// ld(j, b), or the register block), every later stage from LDS.  The last
// stage writes natural-order results to SNK (LDS, a store functor
// st(j, b, v), or the register block).  All threads of the block must call.
template <class G, bool INV, bool REV, int S, int SRC, int SNK, class LoadF, class StoreF,
          int PERR, int RR>
DEV void stages(float2 *lds, const float2 *__restrict__ tw, const LoadF &ld, const StoreF &st,
                float2 (&regs)[PERR][RR]) {
  constexpr int NSTG = num_stages(G::L);
  constexpr int R = stage_radix(G::L, S, REV);
  constexpr int NS = stage_ns(G::L, S, REV);
  constexpr bool FIRST = (S == 0), LAST = (S == NSTG - 1);
  using SS = StageShape<G, R>;
  constexpr int LR = SS::LR, PER = SS::PER, ITEMS = SS::ITEMS;
  constexpr int TWSH = kTwLog - ilog2c(NS * R);
  const int tid = threadIdx.x;

  float2 v[PER][R];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int it = tid + i * G::T;
    if (SS::EXACT || it < ITEMS) {
      int j, b;
      decode_item<G, R>(it, j, b);
      if constexpr (FIRST && SRC == SRC_REG) {
        static_assert(PERR == PER && RR == R, "register hand-off shape");
#pragma unroll
        for (int t = 0; t < R; ++t) v[i][t] = regs[i][t];
      } else if constexpr (FIRST && SRC == SRC_FN) {
#pragma unroll
        for (int t = 0; t < R; ++t) v[i][t] = ld(j + t * LR, b);
      } else {
#pragma unroll
        for (int t = 0; t < R; ++t) v[i][t] = lds[(j + t * LR) * G::SJ + b * G::SB];
      }
    }
  }

#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int it = tid + i * G::T;
    if (SS::EXACT || it < ITEMS) {
      if constexpr (!FIRST) {
        int j, b;
        decode_item<G, R>(it, j, b);
        const int k = j & (NS - 1);
#pragma unroll
        for (int t = 1; t < R; ++t) {
          const float2 w = tw[(t * k) << TWSH];
          v[i][t] = INV ? cmulc(v[i][t], w) : cmul(v[i][t], w);
        }
      }
      Dft<R, INV>::run(v[i]);
    }
  }

  if constexpr (LAST) {
    if constexpr (SNK == SNK_LDS) __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int it = tid + i * G::T;
      if (SS::EXACT || it < ITEMS) {
        int j, b;
        decode_item<G, R>(it, j, b);
#pragma unroll
        for (int t = 0; t < R; ++t) {
          if constexpr (SNK == SNK_REG) {
            static_assert(PERR == PER && RR == R, "register hand-off shape");
            regs[i][t] = v[i][t];
          } else if constexpr (SNK == SNK_FN) {
            st(j + t * LR, b, v[i][t]);
          } else {
            lds[(j + t * LR) * G::SJ + b * G::SB] = v[i][t];
          }
        }
      }
    }
    if constexpr (SNK == SNK_LDS) __syncthreads();
  } else {
    __syncthreads();  // every read of this stage is done before LDS is reused
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int it = tid + i * G::T;
      if (SS::EXACT || it < ITEMS) {
        int j, b;
        decode_item<G, R>(it, j, b);
        const int k = j & (NS - 1);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int t = 0; t < R; ++t) lds[(base + t * NS) * G::SJ + b * G::SB] = v[i][t];
      }
    }
    __syncthreads();
    stages<G, INV, REV, S + 1, SRC_LDS, SNK>(lds, tw, ld, st, regs);
  }
}

template <class G, bool INV, bool REV, int SRC, int SNK, class LoadF, class StoreF, int PERR,
          int RR>
DEV void dft_tile(float2 *lds, const float2 *__restrict__ tw, const LoadF &ld, const StoreF &st,
                  float2 (&regs)[PERR][RR]) {
  stages<G, INV, REV, 0, SRC, SNK>(lds, tw, ld, st, regs);
}

struct NoLoad {
  DEV float2 operator()(int, int) const { return make_float2(0.f, 0.f); }
};
struct NoStore {
  DEV void operator()(int, int, float2) const {}
};

// ---------------------------------------------------------------------------
// Pass plan per log2(M).  Tiles hold at most 8192 points (64 KiB + padding),
// so two blocks fit in one CU's 160 KiB LDS.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }
__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }
__host__ __device__ constexpr int plan_bx(int lm) { return cmin(lm / 2, 6); }
__host__ __device__ constexpr int plan_ay(int lm) {
  return cmin(cmin(lm / 2, 7), 13 - plan_bx(lm));
}
__host__ __device__ constexpr int threads_for(int pts) { return cmin(512, cmax(64, pts / 16)); }

template <int LOGM>
struct Plan {
  static constexpr int M = 1 << LOGM;
  static constexpr int BX = 1 << plan_bx(LOGM);
  static constexpr int AX = M / BX;
  static constexpr int AY = 1 << plan_ay(LOGM);
  static constexpr int BY = M / AY;
  static constexpr int RA = cmin(8, BX);   // contiguous run in passes A / A'
  static constexpr int RC = cmin(16, M);   // contiguous run in pass C
  static constexpr int TA = threads_for(AX * RA);
  static constexpr int TB = threads_for(BX * AY);
  static constexpr int TC = threads_for(BY * RC);
};

// ---------------------------------------------------------------------------
// Element-wise physics.
// ---------------------------------------------------------------------------

// exp(i 2 pi q), q = turns_per_h * h formed in FP64 and reduced to
// [-1/2, 1/2] turn before the cast to FP32 (Eq. 1-2).
DEV float2 doe_phase(float hv, double turns_per_h) {
  const double q = turns_per_h * (double)hv;
  const double fr = q - rint(q);
  float s, c;
  sincospif((float)(2.0 * fr), &s, &c);
  return make_float2(c, s);
}

// (lambda * f)^2 for DFT bin k of M, f = k_signed / (M dx), each product
// rounded once in FP64 (no contraction), as the evanescent test needs.
DEV double lam_f_sq(int k, int m, const KParams &p) {
#pragma clang fp contract(off)
  const int ks = k < (m >> 1) ? k : k - m;
  const double f = (double)ks * p.inv_mdx;
  const double a = p.lam * f;
  return a * a;
}

// H(ky, kx) / M^2 (conjugated when p.adjoint): zero unless
// s = a2y + a2x < 1; else exp(i 2 pi (z/lambda) sqrt(1 - s)) with the
// argument formed and reduced mod one turn in FP64.
DEV float2 transfer(double a2y, double a2x, const KParams &p) {
#pragma clang fp contract(off)
  const double s = a2y + a2x;
  if (!(s < 1.0)) return make_float2(0.f, 0.f);
  const double root = sqrt(1.0 - s);
  const double t = p.zl * root;
  const double fr = t - rint(t);
  float sn, cs;
  sincospif((float)(2.0 * fr), &sn, &cs);
  if (p.adjoint) sn = -sn;
  return make_float2(cs * p.inv_m2, sn * p.inv_m2);
}

DEV float2 twiddle(const float2 *__restrict__ tw, int q, int logm) {
  return tw[(q & ((1 << logm) - 1)) << (kTwLog - logm)];
}

// ---------------------------------------------------------------------------
// Pass A: DFT over xa for the N input rows, input formed on the fly.
// Block = one row y and a run of RA consecutive xb.
// ---------------------------------------------------------------------------
template <int LOGM>
__global__ __launch_bounds__(Plan<LOGM>::TA) void k_pass_a_fwd(KParams p) {
  using P = Plan<LOGM>;
  constexpr int AX = P::AX, BX = P::BX, RA = P::RA, M = P::M;
  using G = Geo<AX, RA, RA + 1, 1, P::TA, false>;
  __shared__ float2 lds[AX * (RA + 1)];
  constexpr int RUNS = BX / RA;
  const int y = blockIdx.x / RUNS;
  const int xb0 = (blockIdx.x % RUNS) * RA;
  const int n = p.n;
  const size_t rowin = (size_t)y * n;

  auto ld = [&](int xa, int b) -> float2 {
    const int x = BX * xa + xb0 + b;
    if (x >= n) return make_float2(0.f, 0.f);
    const size_t idx = rowin + x;
    if (p.in_mode == IN_PHASE) {
      float2 e = doe_phase(p.h[idx], p.phase_turns);
      if (p.amp) e = cscale(e, p.amp[idx]);
      return e;
    } else if (p.in_mode == IN_FIELD) {
      return p.u_in[idx];
    } else {
      return cscale(p.saved_in[idx], p.two_wk * p.gpsf[idx]);
    }
  };
  float2 *out = p.ws + (size_t)y * M;
  auto st = [&](int kxa, int b, float2 v) {
    const int xb = xb0 + b;
    out[BX * kxa + xb] = cmul(v, twiddle(p.tw, xb * kxa, LOGM));
  };
  float2 dummy[1][1];
  dft_tile<G, false, false, SRC_FN, SNK_FN>(lds, p.tw, ld, st, dummy);
}

// ---------------------------------------------------------------------------
// Pass B: DFT over xb then over ya on a BX x AY tile (block = (kxa, yb)).
// ---------------------------------------------------------------------------
template <int LOGM>
__global__ __launch_bounds__(Plan<LOGM>::TB) void k_pass_b_fwd(KParams p) {
  using P = Plan<LOGM>;
  constexpr int AX = P::AX, BX = P::BX, AY = P::AY, BY = P::BY, M = P::M, T = P::TB;
  constexpr int SR = BX + 1;
  __shared__ float2 lds[AY * SR];
  const int kxa = blockIdx.x % AX;
  const int yb = blockIdx.x / AX;
  const float2 *__restrict__ ws = p.ws;
  const size_t col0 = (size_t)BX * kxa;

  for (int e = threadIdx.x; e < AY * BX; e += T) {
    const int ya = e / BX, xb = e % BX;
    const int y = BY * ya + yb;
    lds[ya * SR + xb] = (y < p.nrows_in) ? ws[(size_t)y * M + col0 + xb] : make_float2(0.f, 0.f);
  }
  __syncthreads();

  float2 dummy[1][1];
  using GX = Geo<BX, AY, 1, SR, T, true>;
  dft_tile<GX, false, false, SRC_LDS, SNK_LDS>(lds, p.tw, NoLoad{}, NoStore{}, dummy);

  float2 *wsw = p.ws;
  auto st = [&](int kya, int kxb, float2 v) {
    wsw[(size_t)(BY * kya + yb) * M + col0 + kxb] = cmul(v, twiddle(p.tw, yb * kya, LOGM));
  };
  using GY = Geo<AY, BX, SR, 1, T, false>;
  dft_tile<GY, false, false, SRC_LDS, SNK_FN>(lds, p.tw, NoLoad{}, st, dummy);
}

// ---------------------------------------------------------------------------
// Pass C: DFT over yb, times H, inverse DFT over yb (block = (kya, run of RC
// columns)).
// ---------------------------------------------------------------------------
template <int LOGM>
__global__ __launch_bounds__(Plan<LOGM>::TC) void k_pass_c(KParams p) {
  using P = Plan<LOGM>;
  constexpr int AX = P::AX, BX = P::BX, AY = P::AY, BY = P::BY, M = P::M, RC = P::RC, T = P::TC;
  using G = Geo<BY, RC, RC + 1, 1, T, false>;
  __shared__ float2 lds[BY * (RC + 1)];
  constexpr int RUNS = M / RC;
  const int px0 = (blockIdx.x % RUNS) * RC;
  const int kya = blockIdx.x / RUNS;
  float2 *base = p.ws + (size_t)(BY * kya) * M + px0;

  auto ld = [&](int yb, int b) -> float2 { return base[(size_t)yb * M + b]; };
  auto st = [&](int yb, int b, float2 v) { base[(size_t)yb * M + b] = v; };

  using LR_ = LastRegs<G, false>;
  float2 regs[LR_::PER][LR_::R];
  dft_tile<G, false, false, SRC_FN, SNK_REG>(lds, p.tw, ld, NoStore{}, regs);

  {
    constexpr int R = LR_::R;
    constexpr int LRn = BY / R;
    using SS = StageShape<G, R>;
#pragma unroll
    for (int i = 0; i < LR_::PER; ++i) {
      const int it = threadIdx.x + i * T;
      if (SS::EXACT || it < SS::ITEMS) {
        int j, b;
        decode_item<G, R>(it, j, b);
        const int px = px0 + b;
        const int kx = (px / BX) + AX * (px % BX);
        const double a2x = lam_f_sq(kx, M, p);
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int kyb = j + t * LRn;
          const int ky = kya + AY * kyb;
          regs[i][t] = cmul(regs[i][t], transfer(lam_f_sq(ky, M, p), a2x, p));
        }
      }
    }
  }

  dft_tile<G, true, true, SRC_REG, SNK_FN>(lds, p.tw, NoLoad{}, st, regs);
}

// ---------------------------------------------------------------------------
// Pass B': inverse DFT over kya then over kxb (block = (kxa, yb)); writes the
// rows y < nrows_out.
// ---------------------------------------------------------------------------
template <int LOGM>
__global__ __launch_bounds__(Plan<LOGM>::TB) void k_pass_b_inv(KParams p) {
  using P = Plan<LOGM>;
  constexpr int AX = P::AX, BX = P::BX, AY = P::AY, BY = P::BY, M = P::M, T = P::TB;
  constexpr int SR = BX + 1;
  __shared__ float2 lds[AY * SR];
  const int kxa = blockIdx.x % AX;
  const int yb = blockIdx.x / AX;
  const size_t col0 = (size_t)BX * kxa;
  const float2 *__restrict__ ws = p.ws;

  auto ld = [&](int kya, int kxb) -> float2 {
    const float2 v = ws[(size_t)(BY * kya + yb) * M + col0 + kxb];
    return cmulc(v, twiddle(p.tw, yb * kya, LOGM));
  };
  float2 dummy[1][1];
  using GY = Geo<AY, BX, SR, 1, T, false>;
  dft_tile<GY, true, false, SRC_FN, SNK_LDS>(lds, p.tw, ld, NoStore{}, dummy);
  using GX = Geo<BX, AY, 1, SR, T, true>;
  dft_tile<GX, true, false, SRC_LDS, SNK_LDS>(lds, p.tw, NoLoad{}, NoStore{}, dummy);

  float2 *wsw = p.ws;
  for (int e = threadIdx.x; e < AY * BX; e += T) {
    const int ya = e / BX, xb = e % BX;
    const int y = BY * ya + yb;
    if (y < p.nrows_out) wsw[(size_t)y * M + col0 + xb] = lds[ya * SR + xb];
  }
}

// ---------------------------------------------------------------------------
// Pass A': inverse DFT over kxa for the rows y < nrows_out, then the output
// stage: PSF accumulation (Eq. 4), field, or height gradient.
// ---------------------------------------------------------------------------
template <int LOGM>
__global__ __launch_bounds__(Plan<LOGM>::TA) void k_pass_a_inv(KParams p) {
  using P = Plan<LOGM>;
  constexpr int AX = P::AX, BX = P::BX, RA = P::RA, M = P::M;
  using G = Geo<AX, RA, RA + 1, 1, P::TA, false>;
  __shared__ float2 lds[AX * (RA + 1)];
  constexpr int RUNS = BX / RA;
  const int y = blockIdx.x / RUNS;
  const int xb0 = (blockIdx.x % RUNS) * RA;
  const int n = p.n;
  const float2 *__restrict__ row = p.ws + (size_t)y * M;

  auto ld = [&](int kxa, int b) -> float2 {
    const int xb = xb0 + b;
    return cmulc(row[BX * kxa + xb], twiddle(p.tw, xb * kxa, LOGM));
  };
  auto st = [&](int xa, int b, float2 u) {
    const int x = BX * xa + xb0 + b;
    size_t idx;
    if (p.full) {
      const int yo = (y + p.p0) & (M - 1), xo = (x + p.p0) & (M - 1);
      idx = (size_t)yo * M + xo;
    } else {
      if (x >= n) return;
      idx = (size_t)y * n + x;
    }
    if (p.out_mode == OUT_PSF) {
      const float v = p.wk * (u.x * u.x + u.y * u.y);
      p.psf[idx] = p.first ? v : p.psf[idx] + v;
      if (p.saved_out) p.saved_out[idx] = u;
    } else if (p.out_mode == OUT_FIELD) {
      p.u_out[idx] = u;
    } else {
      float2 e = doe_phase(p.h[idx], p.phase_turns);
      if (p.amp) e = cscale(e, p.amp[idx]);
      const float v = p.ck * (u.y * e.x - u.x * e.y);  // c_k Im(g_E conj(E))
      p.grad_h[idx] = p.first ? v : p.grad_h[idx] + v;
    }
  };
  float2 dummy[1][1];
  dft_tile<G, true, false, SRC_FN, SNK_FN>(lds, p.tw, ld, st, dummy);
}

// ---------------------------------------------------------------------------
// Host-side launch of the five passes.
// ---------------------------------------------------------------------------
static inline void mark(hipEvent_t *ev, int i, hipStream_t s) {
  if (ev) (void)hipEventRecord(ev[i], s);
}

template <int LOGM>
static hipError_t launch_impl(const KParams &p, hipStream_t s, hipEvent_t *ev) {
  using P = Plan<LOGM>;
  const unsigned ga = (unsigned)p.nrows_in * (P::BX / P::RA);
  const unsigned gb = (unsigned)(P::AX * P::BY);
  const unsigned gc = (unsigned)(P::AY * (P::M / P::RC));
  const unsigned gai = (unsigned)p.nrows_out * (P::BX / P::RA);
  mark(ev, 0, s);
  hipLaunchKernelGGL(k_pass_a_fwd<LOGM>, dim3(ga), dim3(P::TA), 0, s, p);
  mark(ev, 1, s);
  hipLaunchKernelGGL(k_pass_b_fwd<LOGM>, dim3(gb), dim3(P::TB), 0, s, p);
  mark(ev, 2, s);
  hipLaunchKernelGGL(k_pass_c<LOGM>, dim3(gc), dim3(P::TC), 0, s, p);
  mark(ev, 3, s);
  hipLaunchKernelGGL(k_pass_b_inv<LOGM>, dim3(gb), dim3(P::TB), 0, s, p);
  mark(ev, 4, s);
  hipLaunchKernelGGL(k_pass_a_inv<LOGM>, dim3(gai), dim3(P::TA), 0, s, p);
  mark(ev, 5, s);
  return hipGetLastError();
}

hipError_t launch_wavelength(const KParams &p, hipStream_t s, hipEvent_t *ev) {
  switch (p.logm) {
    case 4: return launch_impl<4>(p, s, ev);
    case 5: return launch_impl<5>(p, s, ev);
    case 6: return launch_impl<6>(p, s, ev);
    case 7: return launch_impl<7>(p, s, ev);
    case 8: return launch_impl<8>(p, s, ev);
    case 9: return launch_impl<9>(p, s, ev);
    case 10: return launch_impl<10>(p, s, ev);
    case 11: return launch_impl<11>(p, s, ev);
    case 12: return launch_impl<12>(p, s, ev);
    case 13: return launch_impl<13>(p, s, ev);
    case 14: return launch_impl<14>(p, s, ev);
    case 15: return launch_impl<15>(p, s, ev);
    case 16: return launch_impl<16>(p, s, ev);
    default: return hipErrorInvalidValue;
  }
}

template <int LOGM>
static void fill_plan(PlanInfo *o) {
  using P = Plan<LOGM>;
  o->ax = P::AX; o->bx = P::BX; o->ay = P::AY; o->by = P::BY; o->ra = P::RA; o->rc = P::RC;
  o->threads_a = P::TA; o->threads_b = P::TB; o->threads_c = P::TC;
}

bool plan_info(int logm, PlanInfo *o) {
  switch (logm) {
    case 4: fill_plan<4>(o); return true;
    case 5: fill_plan<5>(o); return true;
    case 6: fill_plan<6>(o); return true;
    case 7: fill_plan<7>(o); return true;
    case 8: fill_plan<8>(o); return true;
    case 9: fill_plan<9>(o); return true;
    case 10: fill_plan<10>(o); return true;
    case 11: fill_plan<11>(o); return true;
    case 12: fill_plan<12>(o); return true;
    case 13: fill_plan<13>(o); return true;
    case 14: fill_plan<14>(o); return true;
    case 15: fill_plan<15>(o); return true;
    case 16: fill_plan<16>(o); return true;
    default: return false;
  }
}

}  // namespace dop
