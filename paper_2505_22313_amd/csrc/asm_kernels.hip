// HIP kernels for CDNA4 (gfx950): FFT-based angular-spectrum propagation of a
// DOE, Eq. (1)-(4) of Wei et al., "Large-Area Fabrication-Aware Computational
// Diffractive Optics" (Sec. 3.1).
//
// One wavelength = five passes over an My x Mx complex64 field held in HBM
// (square, or rectangular as the paper's 128,640 x 85,760 grid).  Each axis
// index is split into two digits,
//     x = BX * xa + xb,   y = BY * ya + yb      (Mx = AX * BX, My = AY * BY),
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
// 16/8/4 (and 3, 5, 9, 15) stages in registers, or a radix-67 stage through
// LDS.  Inner twiddles and four-step twiddles come from one FP64-generated
// complex64 table of exp(-2 pi i j / 2^17) on power-of-two grids, and are
// generated per block in FP64 on the others.

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

template <bool INV>
struct Dft<3, INV> {
  // X1,2 = a0 - (a1 + a2)/2 -/+ i (sqrt(3)/2) (a1 - a2)   (forward sign)
  DEV static void run(float2 *a) {
    constexpr float H = 0.866025403784438646764f;  // sin(2 pi / 3)
    const float2 t1 = cadd(a[1], a[2]);
    const float2 t2 = make_float2(a[0].x - 0.5f * t1.x, a[0].y - 0.5f * t1.y);
    const float2 d = cscale(csub(a[1], a[2]), H);
    const float2 t3 = INV ? mul_pi(d) : mul_mi(d);
    a[0] = cadd(a[0], t1);
    a[1] = cadd(t2, t3);
    a[2] = csub(t2, t3);
  }
};

template <bool INV>
struct Dft<5, INV> {
  // with t1 = a1 + a4, t2 = a2 + a3, t3 = a1 - a4, t4 = a2 - a3 (forward sign):
  // X1,4 = a0 + c1 t1 + c2 t2 -/+ i (s1 t3 + s2 t4)
  // X2,3 = a0 + c2 t1 + c1 t2 -/+ i (s2 t3 - s1 t4)
  DEV static void run(float2 *a) {
    constexpr float C1 = 0.309016994374947424102f;   // cos(2 pi / 5)
    constexpr float C2 = -0.809016994374947424102f;  // cos(4 pi / 5)
    constexpr float S1 = 0.951056516295153572116f;   // sin(2 pi / 5)
    constexpr float S2 = 0.587785252292473129169f;   // sin(4 pi / 5)
    const float2 t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
    const float2 t3 = csub(a[1], a[4]), t4 = csub(a[2], a[3]);
    const float2 r1 = make_float2(a[0].x + C1 * t1.x + C2 * t2.x, a[0].y + C1 * t1.y + C2 * t2.y);
    const float2 r2 = make_float2(a[0].x + C2 * t1.x + C1 * t2.x, a[0].y + C2 * t1.y + C1 * t2.y);
    const float2 q1 = make_float2(S1 * t3.x + S2 * t4.x, S1 * t3.y + S2 * t4.y);
    const float2 q2 = make_float2(S2 * t3.x - S1 * t4.x, S2 * t3.y - S1 * t4.y);
    const float2 i1 = INV ? mul_pi(q1) : mul_mi(q1);
    const float2 i2 = INV ? mul_pi(q2) : mul_mi(q2);
    a[0] = cadd(a[0], cadd(t1, t2));
    a[1] = cadd(r1, i1);
    a[4] = csub(r1, i1);
    a[2] = cadd(r2, i2);
    a[3] = csub(r2, i2);
  }
};

// cos(2 pi q / R) and sin(2 pi q / R), q < R, for the composite radices
// (values of the unit circle rounded to float).
template <int R>
struct UnitRoots;
template <>
struct UnitRoots<9> {
  static constexpr float c[9] = {
      1.000000000e+00f, 7.660444431e-01f, 1.736481777e-01f, -5.000000000e-01f,
      -9.396926208e-01f, -9.396926208e-01f, -5.000000000e-01f, 1.736481777e-01f,
      7.660444431e-01f};
  static constexpr float s[9] = {
      0.000000000e+00f, 6.427876097e-01f, 9.848077530e-01f, 8.660254038e-01f,
      3.420201433e-01f, -3.420201433e-01f, -8.660254038e-01f, -9.848077530e-01f,
      -6.427876097e-01f};
};
template <>
struct UnitRoots<15> {
  static constexpr float c[15] = {
      1.000000000e+00f, 9.135454576e-01f, 6.691306064e-01f, 3.090169944e-01f,
      -1.045284633e-01f, -5.000000000e-01f, -8.090169944e-01f, -9.781476007e-01f,
      -9.781476007e-01f, -8.090169944e-01f, -5.000000000e-01f, -1.045284633e-01f,
      3.090169944e-01f, 6.691306064e-01f, 9.135454576e-01f};
  static constexpr float s[15] = {
      0.000000000e+00f, 4.067366431e-01f, 7.431448255e-01f, 9.510565163e-01f,
      9.945218954e-01f, 8.660254038e-01f, 5.877852523e-01f, 2.079116908e-01f,
      -2.079116908e-01f, -5.877852523e-01f, -8.660254038e-01f, -9.945218954e-01f,
      -9.510565163e-01f, -7.431448255e-01f, -4.067366431e-01f};
};

template <>
struct UnitRoots<67> {
  static constexpr float c[67] = {
      1.000000000e+00f, 9.956059820e-01f, 9.824625429e-01f, 9.606851876e-01f,
      9.304652963e-01f, 8.920684426e-01f, 8.458320593e-01f, 7.921624734e-01f,
      7.315313353e-01f, 6.644714734e-01f, 5.915722124e-01f, 5.134741935e-01f,
      4.308637449e-01f, 3.444668503e-01f, 2.550427686e-01f, 1.633773618e-01f,
      7.027618895e-02f, -2.344257360e-02f, -1.169553220e-01f, -2.094402628e-01f,
      -3.000846350e-01f, -3.880918527e-01f, -4.726885052e-01f, -5.531311541e-01f,
      -6.287128666e-01f, -6.987694278e-01f, -7.626851781e-01f, -8.198984237e-01f,
      -8.699063724e-01f, -9.122695527e-01f, -9.466156753e-01f, -9.726429053e-01f,
      -9.901225145e-01f, -9.989008915e-01f, -9.989008915e-01f, -9.901225145e-01f,
      -9.726429053e-01f, -9.466156753e-01f, -9.122695527e-01f, -8.699063724e-01f,
      -8.198984237e-01f, -7.626851781e-01f, -6.987694278e-01f, -6.287128666e-01f,
      -5.531311541e-01f, -4.726885052e-01f, -3.880918527e-01f, -3.000846350e-01f,
      -2.094402628e-01f, -1.169553220e-01f, -2.344257360e-02f, 7.027618895e-02f,
      1.633773618e-01f, 2.550427686e-01f, 3.444668503e-01f, 4.308637449e-01f,
      5.134741935e-01f, 5.915722124e-01f, 6.644714734e-01f, 7.315313353e-01f,
      7.921624734e-01f, 8.458320593e-01f, 8.920684426e-01f, 9.304652963e-01f,
      9.606851876e-01f, 9.824625429e-01f, 9.956059820e-01f};
  static constexpr float s[67] = {
      0.000000000e+00f, 9.364148953e-02f, 1.864600543e-01f, 2.776400014e-01f,
      3.663800382e-01f, 4.519003140e-01f, 5.334492736e-01f, 6.103102618e-01f,
      6.818078216e-01f, 7.473136296e-01f, 8.062520186e-01f, 8.581050359e-01f,
      9.024169952e-01f, 9.387984816e-01f, 9.669297732e-01f, 9.865636511e-01f,
      9.975275722e-01f, 9.997251851e-01f, 9.931371772e-01f, 9.778214440e-01f,
      9.539125808e-01f, 9.216206996e-01f, 8.812295825e-01f, 8.330941882e-01f,
      7.776375321e-01f, 7.153469695e-01f, 6.467699120e-01f, 5.725090173e-01f,
      4.932168927e-01f, 4.095903603e-01f, 3.223643332e-01f, 2.323053566e-01f,
      1.402048723e-01f, 4.687226247e-02f, -4.687226247e-02f, -1.402048723e-01f,
      -2.323053566e-01f, -3.223643332e-01f, -4.095903603e-01f, -4.932168927e-01f,
      -5.725090173e-01f, -6.467699120e-01f, -7.153469695e-01f, -7.776375321e-01f,
      -8.330941882e-01f, -8.812295825e-01f, -9.216206996e-01f, -9.539125808e-01f,
      -9.778214440e-01f, -9.931371772e-01f, -9.997251851e-01f, -9.975275722e-01f,
      -9.865636511e-01f, -9.669297732e-01f, -9.387984816e-01f, -9.024169952e-01f,
      -8.581050359e-01f, -8.062520186e-01f, -7.473136296e-01f, -6.818078216e-01f,
      -6.103102618e-01f, -5.334492736e-01f, -4.519003140e-01f, -3.663800382e-01f,
      -2.776400014e-01f, -1.864600543e-01f, -9.364148953e-02f};
};

// R = R1 * R2 from two in-register DFTs (four-step split n = n1 R2 + n2,
// k = k1 + R1 k2, twiddles omega_R^(n2 k1) from UnitRoots<R>).
template <int R1, int R2, bool INV>
struct DftComposite {
  static constexpr int R = R1 * R2;
  DEV static void run(float2 *a) {
    float2 t[R];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      float2 b[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) b[n1] = a[n1 * R2 + n2];
      Dft<R1, INV>::run(b);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) {
        const int q = (n2 * k1) % R;
        if (q == 0) {
          t[k1 * R2 + n2] = b[k1];
        } else {
          const float c = UnitRoots<R>::c[q];
          const float sn = INV ? UnitRoots<R>::s[q] : -UnitRoots<R>::s[q];
          t[k1 * R2 + n2] = make_float2(b[k1].x * c - b[k1].y * sn, b[k1].x * sn + b[k1].y * c);
        }
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      float2 c[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) c[n2] = t[k1 * R2 + n2];
      Dft<R2, INV>::run(c);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) a[k1 + R1 * k2] = c[k2];
    }
  }
};

template <bool INV>
struct Dft<9, INV> : DftComposite<3, 3, INV> {};
template <bool INV>
struct Dft<15, INV> : DftComposite<3, 5, INV> {};

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
// Stockham stage plan for an L-point DFT, L = 2^a 3^b 5^c 67^d <= 1024: the
// power-of-two factor in radix 16/8/4 stages (as for a power-of-two L), then
// the odd factor: a radix-15 stage per (3, 5) pair, radix 9 per pair of the
// remaining threes, radix 5 per remaining five, a last radix 3, and last of
// all a radix-67 stage (the prime factor of the paper's 128,640 x 85,760
// grid; see stage_prime).  (Radix 25 would save more stages, but 25 points
// per item plus the prefetched inputs overflow the 128 registers a thread
// has at this occupancy.)
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }
__host__ __device__ constexpr bool is_pow2c(int v) { return v > 0 && (v & (v - 1)) == 0; }
__host__ __device__ constexpr int pow2_part(int v) { return v % 2 ? 1 : 2 * pow2_part(v / 2); }
__host__ __device__ constexpr int cmin_(int a, int b) { return a < b ? a : b; }
__host__ __device__ constexpr int count_factor(int v, int f) {
  return v % f ? 0 : 1 + count_factor(v / f, f);
}

__host__ __device__ constexpr int num_stages_p2(int L) {
  return L <= 1 ? 0 : L <= 16 ? 1 : (L <= 256 ? 2 : 3);
}

__host__ __device__ constexpr int fwd_radix_p2(int L, int s) {
  return L <= 16 ? L
       : L == 32 ? (s == 0 ? 8 : 4)
       : L == 64 ? 8
       : L == 128 ? (s == 0 ? 16 : 8)
       : L == 256 ? 16
       : L == 512 ? (s == 0 ? 16 : (s == 1 ? 8 : 4))
       : L == 1024 ? (s == 0 ? 16 : 8)
       : L == 2048 ? (s < 2 ? 16 : 8)
       : 16;  // 4096 (whole rows and columns of the small-grid path)
}

__host__ __device__ constexpr int n15(int L) {
  return cmin_(count_factor(L, 3), count_factor(L, 5));
}
__host__ __device__ constexpr int n9(int L) { return (count_factor(L, 3) - n15(L)) / 2; }
__host__ __device__ constexpr int n5(int L) { return count_factor(L, 5) - n15(L); }
__host__ __device__ constexpr int n3(int L) { return (count_factor(L, 3) - n15(L)) % 2; }
constexpr int kP = 67;  // the prime radix
__host__ __device__ constexpr int n67(int L) { return count_factor(L, kP); }

__host__ __device__ constexpr int num_stages(int L) {
  return L <= 1 ? 1 : num_stages_p2(pow2_part(L)) + n15(L) + n9(L) + n5(L) + n3(L) + n67(L);
}

// radix of odd-factor stage s (s counted from the first odd stage)
__host__ __device__ constexpr int odd_radix(int L, int s) {
  return s < n15(L)                         ? 15
         : s < n15(L) + n9(L)               ? 9
         : s < n15(L) + n9(L) + n5(L)       ? 5
         : s < n15(L) + n9(L) + n5(L) + n3(L) ? 3
                                            : kP;
}

__host__ __device__ constexpr int fwd_radix(int L, int s) {
  return L <= 1 ? 1
       : s < num_stages_p2(pow2_part(L)) ? fwd_radix_p2(pow2_part(L), s)
                                         : odd_radix(L, s - num_stages_p2(pow2_part(L)));
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
    j = is_pow2c(LR) ? it & (LR - 1) : (int)((unsigned)it % LR);
    b = it / LR;
  } else {
    b = is_pow2c(G::NB) ? it & (G::NB - 1) : (int)((unsigned)it % G::NB);
    j = it / G::NB;
  }
}

// Register block handed between the forward and inverse halves of pass C.
template <class G, bool REV>
struct LastRegs {
  static constexpr int R = stage_radix(G::L, num_stages(G::L) - 1, REV);
  static constexpr int PER = StageShape<G, R>::PER;
};

// ---------------------------------------------------------------------------
// Radix-67 Stockham stage.  67 points per item do not fit in registers, so
// the stage works through the tile in LDS, in place:
//  1. fold: for every item and t = 1..33 (one thread per pair), read v_t and
//     v_{67-t} (after the stage twiddles) and write v_t + v_{67-t} to slot t
//     and v_t - v_{67-t} to slot 67 - t (slot 0 keeps v_0);
//  2. three or four threads per item (whichever spreads the tile's
//     wavefronts evenly over the four SIMDs) each form a share of the 33
//     output pairs from the folded values, X_k, X_{67-k} = v_0 + sum_t s_t cos(2 pi t k / 67)
//     -/+ i sum_t d_t sin(2 pi t k / 67) (forward sign; the symmetric form of
//     the direct DFT, 2 real multiply-adds per input pair and output), with
//     the constants folded in at compile time; a share is uniform across a
//     wavefront so that the code paths of the shares do not diverge;
//  3. the outputs go to the stage's Stockham positions, in LDS or through the
//     store functor.
// Inputs come from LDS or the load functor, never from registers, and
// outputs never go to registers.
// ---------------------------------------------------------------------------
constexpr int kPH = (kP - 1) / 2;  // folded input pairs
// With NSH shares per item, share rb covers output pairs k = share_k0 ..
// share_k0 + share_np - 1: 11 + 11 + 11 or 9 + 8 + 8 + 8.
__host__ __device__ constexpr int share_np(int nsh, int rb) {
  return nsh == 3 ? 11 : (rb == 0 ? 9 : 8);
}
__host__ __device__ constexpr int share_k0(int nsh, int rb) {
  return nsh == 3 ? 1 + 11 * rb : (rb == 0 ? 1 : 10 + 8 * (rb - 1));
}
constexpr int kPBMax = 11;
static_assert(share_k0(3, 2) + share_np(3, 2) == kPH + 1, "three shares cover 1..33");
static_assert(share_k0(4, 3) + share_np(4, 3) == kPH + 1, "four shares cover 1..33");

template <class G, int NSH, int RB, bool INV>
DEV void prime_outputs(const float2 *lds, const int e0, float2 (&o)[2 * kPBMax + 1]) {
  constexpr int STEP = (G::L / kP) * G::SJ;
  constexpr int K0 = share_k0(NSH, RB), NP = share_np(NSH, RB);
  const float2 x0 = lds[e0];
  float2 a[NP], q[NP];
  float2 sum = x0;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    a[i] = x0;
    q[i] = make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int t = 1; t <= kPH; ++t) {
    const float2 sv = lds[e0 + t * STEP], dv = lds[e0 + (kP - t) * STEP];
    if constexpr (RB == 0) sum = cadd(sum, sv);
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int e = (t * (K0 + i)) % kP;
      const float c = UnitRoots<kP>::c[e], sn_ = UnitRoots<kP>::s[e];
      a[i].x += sv.x * c;
      a[i].y += sv.y * c;
      q[i].x += dv.x * sn_;
      q[i].y += dv.y * sn_;
    }
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const float2 iq = INV ? mul_pi(q[i]) : mul_mi(q[i]);
    o[2 * i] = cadd(a[i], iq);      // X_{K0 + i}
    o[2 * i + 1] = csub(a[i], iq);  // X_{67 - K0 - i}
  }
  o[2 * kPBMax] = sum;              // X_0 (share 0)
}

template <class G, bool INV, bool FIRST, bool LAST, int NS, int TWMUL, int SRC, int SNK,
          class LoadF, class StoreF, class Hook>
DEV void stage_prime(float2 *lds, const float2 *twl, const LoadF &ld, const StoreF &st,
                     const Hook &hook, const int tid, const int nb_act) {
  static_assert(SRC != SRC_REG && SNK != SNK_REG,
                "a radix-67 stage reads and writes LDS or functors, not registers");
  constexpr int LR = G::L / kP, ITEMS = LR * G::NB;
  auto at = [](int j, int b) { return j * G::SJ + b * G::SB; };
  // 1. fold, one thread per (item, pair), in place; item fastest so that
  // neighbouring threads touch neighbouring LDS words
  for (int u = tid; u < ITEMS * (kPH + 1); u += G::T) {
    const int it = u % ITEMS, t = u / ITEMS;
    int j, b;
    decode_item<G, kP>(it, j, b);
    if (b >= nb_act) continue;
    if (t == 0) {
      if constexpr (SRC == SRC_FN) lds[at(j, b)] = ld(j, b);
      continue;
    }
    const int k = FIRST ? 0 : (is_pow2c(NS) ? j & (NS - 1) : (int)((unsigned)j % NS));
    auto in = [&](int tt) {
      float2 x;
      if constexpr (SRC == SRC_FN) x = ld(j + tt * LR, b);
      else x = lds[at(j + tt * LR, b)];
      if constexpr (!FIRST) {
        const float2 w = twl[(tt * k) * TWMUL];
        x = INV ? cmulc(x, w) : cmul(x, w);
      }
      return x;
    };
    const float2 v1 = in(t), v2 = in(kP - t);
    lds[at(j + t * LR, b)] = cadd(v1, v2);
    lds[at(j + (kP - t) * LR, b)] = csub(v1, v2);
  }
  if constexpr (FIRST) hook();
  __syncthreads();
  // 2. outputs: wavefront w takes share w / IW of items (w % IW) * 64 + lane
  constexpr int IW = (ITEMS + 63) / 64;
  constexpr int NSH = (3 * IW) % 4 == 0 || 4 * IW * 64 > G::T ? 3 : 4;
  static_assert(NSH * IW * 64 <= G::T, "one output share per thread");
  const int wv = tid >> 6, rb = wv / IW, it = (wv % IW) * 64 + (tid & 63);
  int j = 0, b = 0;
  bool act = rb < NSH && it < ITEMS;
  if (act) {
    decode_item<G, kP>(it, j, b);
    act = b < nb_act;
  }
  float2 o[2 * kPBMax + 1];
  if (act) {
    const int e0 = at(j, b);
    if (rb == 0) prime_outputs<G, NSH, 0, INV>(lds, e0, o);
    else if (rb == 1) prime_outputs<G, NSH, 1, INV>(lds, e0, o);
    else if (NSH == 3 || rb == 2) prime_outputs<G, NSH, 2, INV>(lds, e0, o);
    else prime_outputs<G, NSH, NSH == 3 ? 2 : 3, INV>(lds, e0, o);
  }
  // 3. output t of item (j, b) goes to (j - k) * 67 + k + t * NS, k = j mod NS
  constexpr bool TO_LDS = !LAST || SNK == SNK_LDS;
  if constexpr (TO_LDS) __syncthreads();  // every fold slot has been read
  if (act) {
    const int k = is_pow2c(NS) ? j & (NS - 1) : (int)((unsigned)j % NS);
    const int base = (j - k) * kP + k;
    auto put = [&](int t, float2 val) {
      if constexpr (TO_LDS) lds[at(base + t * NS, b)] = val;
      else st(base + t * NS, b, val);
    };
    const int k0 = share_k0(NSH, rb), np = share_np(NSH, rb);
#pragma unroll
    for (int i = 0; i < kPBMax; ++i) {
      if (i < np) {
        put(k0 + i, o[2 * i]);
        put(kP - k0 - i, o[2 * i + 1]);
      }
    }
    if (rb == 0) put(0, o[2 * kPBMax]);
  }
  if constexpr (TO_LDS) __syncthreads();
}

// One Stockham stage S of the L-point DFT along j for every b, followed by the
// remaining stages.  The first stage reads from SRC (LDS, a load functor
// ld(j, b), or the register block rin), every later stage from LDS.  The last
// stage writes natural-order results to SNK (LDS, a store functor
// st(j, b, v), or the register block rout).  hook() runs once, right after
// the first stage has consumed its inputs (so prefetches issued there do not
// overlap the first stage's registers).  All threads of the block must call.
template <class G, bool INV, bool REV, int S, int SRC, int SNK, int THI, class LoadF, class StoreF,
          class Hook, int PI, int RI, int PO, int RO>
DEV void stages(float2 *lds, const float2 *twl, const LoadF &ld, const StoreF &st,
                const Hook &hook, float2 (&rin)[PI][RI], float2 (&rout)[PO][RO], const int tid,
                const int nb_act) {
  constexpr int NSTG = num_stages(G::L);
  constexpr int R = stage_radix(G::L, S, REV);
  constexpr int NS = stage_ns(G::L, S, REV);
  constexpr bool FIRST = (S == 0), LAST = (S == NSTG - 1);
  using SS = StageShape<G, R>;
  constexpr int LR = SS::LR, PER = SS::PER, ITEMS = SS::ITEMS;
  static_assert(NS * R <= THI, "twiddle table too small");
  constexpr int TWMUL = THI / (NS * R);  // omega_{NS R}^e = twl[e * TWMUL]
  if constexpr (R == kP) {
    stage_prime<G, INV, FIRST, LAST, NS, TWMUL, SRC, SNK>(lds, twl, ld, st, hook, tid, nb_act);
    if constexpr (!LAST)
      stages<G, INV, REV, S + 1, SRC_LDS, SNK, THI>(lds, twl, ld, st, hook, rin, rout, tid, nb_act);
  } else {
  float2 v[PER][R];
  // an item is live if it exists and its batch column is below nb_act (the
  // columns at or beyond nb_act are known to be zero, or are not needed)
  auto live = [&](int it, int &j, int &b) {
    if (!(SS::EXACT || it < ITEMS)) return false;
    decode_item<G, R>(it, j, b);
    return b < nb_act;
  };
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int it = tid + i * G::T;
    int j, b;
    if (live(it, j, b)) {
      if constexpr (FIRST && SRC == SRC_REG) {
        static_assert(PI == PER && RI == R, "register input shape");
#pragma unroll
        for (int t = 0; t < R; ++t) v[i][t] = rin[i][t];
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
    int j, b;
    if (live(it, j, b)) {
      if constexpr (!FIRST) {
        const int k = is_pow2c(NS) ? j & (NS - 1) : (int)((unsigned)j % NS);
#pragma unroll
        for (int t = 1; t < R; ++t) {
          const float2 w = twl[(t * k) * TWMUL];
          v[i][t] = INV ? cmulc(v[i][t], w) : cmul(v[i][t], w);
        }
      }
      Dft<R, INV>::run(v[i]);
    }
  }

  if constexpr (LAST) {
    if constexpr (FIRST) hook();
    if constexpr (SNK == SNK_LDS) __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int it = tid + i * G::T;
      int j, b;
      if (live(it, j, b)) {
#pragma unroll
        for (int t = 0; t < R; ++t) {
          if constexpr (SNK == SNK_REG) {
            static_assert(PO == PER && RO == R, "register output shape");
            rout[i][t] = v[i][t];
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
      int j, b;
      if (live(it, j, b)) {
        const int k = is_pow2c(NS) ? j & (NS - 1) : (int)((unsigned)j % NS);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int t = 0; t < R; ++t) lds[(base + t * NS) * G::SJ + b * G::SB] = v[i][t];
      }
    }
    if constexpr (FIRST) hook();
    __syncthreads();
    stages<G, INV, REV, S + 1, SRC_LDS, SNK, THI>(lds, twl, ld, st, hook, rin, rout, tid, nb_act);
  }
  }
}

struct NoHook {
  DEV void operator()() const {}
};

// L-point DFT of every batch column of a tile; twl is the LDS table
// omega_THI^i, i < THI (THI a multiple of L).  One register block serves as
// input (SRC_REG) and output (SNK_REG).
template <class G, bool INV, bool REV, int SRC, int SNK, int THI, class LoadF, class StoreF,
          int PERR, int RR>
DEV void dft_tile(float2 *lds, const float2 *twl, const LoadF &ld, const StoreF &st,
                  float2 (&regs)[PERR][RR], const int tid, const int nb_act = G::NB) {
  stages<G, INV, REV, 0, SRC, SNK, THI>(lds, twl, ld, st, NoHook{}, regs, regs, tid, nb_act);
}

// As dft_tile, with separate input and output register blocks and a hook run
// after the first stage.
template <class G, bool INV, bool REV, int SRC, int SNK, int THI, class LoadF, class StoreF,
          class Hook, int PI, int RI, int PO, int RO>
DEV void dft_tile_hooked(float2 *lds, const float2 *twl, const LoadF &ld, const StoreF &st,
                         const Hook &hook, float2 (&rin)[PI][RI], float2 (&rout)[PO][RO],
                         const int tid, const int nb_act = G::NB) {
  stages<G, INV, REV, 0, SRC, SNK, THI>(lds, twl, ld, st, hook, rin, rout, tid, nb_act);
}

// Thread index re-read in every tile iteration through an empty asm
// statement, so per-thread LDS addresses are recomputed inside the tile loop
// instead of being hoisted out of it and spilled.
DEV int loop_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Shape of the first Stockham stage of a tile (what a prefetch must gather);
// REV: of the reversed radix order.
template <class G, bool REV = false>
struct FirstStage {
  static constexpr int R = stage_radix(G::L, 0, REV);
  using SS = StageShape<G, R>;
  static constexpr int PER = SS::PER, LR = SS::LR, ITEMS = SS::ITEMS;
  static constexpr bool EXACT = SS::EXACT;
};

struct NoLoad {
  DEV float2 operator()(int, int) const { return make_float2(0.f, 0.f); }
};
struct NoStore {
  DEV void operator()(int, int, float2) const {}
};

// ---------------------------------------------------------------------------
// Pass plans.  Tiles of passes B and C hold at most 8192 points (64 KiB +
// padding), so two blocks fit in one CU's 160 KiB LDS; tiles of passes A and
// A' hold up to 16384 (one block per CU) so that every row run they move is a
// whole 128-byte line.
//
// Plan id PID < kTabBase: the square grid M = 2^PID.  PID = kTabBase + i:
// the i-th grid of table_plan, My x Mx with Mx = AX * BX and My = AY * BY
// from a hand-chosen digit split: BX a power of two >= 16, every tile within
// the limits above, and every digit length a product of the radices
// 16/8/4/2, 3, 5 and 67.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }
__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }
__host__ __device__ constexpr int round64(int v) { return (v + 63) / 64 * 64; }
// M = 2^17 splits both axes 1024 x 128: its B tiles hold 16384 points (one
// 1024-thread block per CU), the only way to keep every digit <= 1024; its
// pass-C tiles are 1024 rows by 8 columns (see RC below).
__host__ __device__ constexpr int plan_bx(int lm) { return lm == 17 ? 7 : cmin(lm / 2, 6); }
__host__ __device__ constexpr int plan_ay(int lm) {
  return lm == 17 ? 7 : cmin(cmin(lm / 2, 7), 13 - plan_bx(lm));
}
__host__ __device__ constexpr int threads_for(int pts) {
  return round64(cmin(512, cmax(64, pts / 16)));
}

struct TablePlan {
  int ax, bx, ay, by;  // Mx = ax * bx columns, My = ay * by rows
  // pass-C run and threads (0: 16 columns, about 8 points per thread); the
  // 1005-row tiles of the paper's grid take 8 columns and 512 threads, so two
  // blocks share a CU and one block's ALU work overlaps the other's traffic
  int rc = 0, tc = 0;
  // pass-A / A' run and threads (0: 16 columns, about 8 points per thread);
  // the 28,800 grid's 450 x 16 tiles take 512 threads, so two blocks share a CU
  int ra = 0, ta = 0;
  // pass-B / B' threads (0: about 8 points per thread); the 40,000 grid's
  // B, B' and C tiles take 512 threads, so two blocks share a CU
  int tb = 0;
};
constexpr int kTabBase = 100;
constexpr int kNumTab = 14;
__host__ __device__ constexpr TablePlan table_plan(int i) {
  return i == 0    ? TablePlan{15, 16, 15, 16}        // 240^2
         : i == 1  ? TablePlan{45, 16, 45, 16}        // 720^2
         : i == 2  ? TablePlan{45, 32, 45, 32}        // 1440^2
         : i == 3  ? TablePlan{48, 64, 48, 64}        // 3072^2
         : i == 4  ? TablePlan{225, 16, 15, 240}      // 3600^2
         : i == 5  ? TablePlan{450, 64, 120, 240, 0, 0, 0, 512}         // 28800^2, 2^7 3^2 5^2
         : i == 6  ? TablePlan{625, 64, 100, 400, 0, 512, 0, 0, 512}    // 40000^2, 2^6 5^4
         : i == 7  ? TablePlan{134, 16, 16, 134}      // 2144^2, 2^5 67
         : i == 8  ? TablePlan{15, 16, 45, 16}        // 720 rows x 240 columns
         : i == 9  ? TablePlan{128, 16, 16, 32}       // 512 x 2048
         : i == 10 ? TablePlan{134, 16, 15, 16}       // 240 x 2144
         : i == 11 ? TablePlan{15, 16, 16, 335}       // 5360 x 240
         : i == 12 ? TablePlan{670, 16, 16, 1005}     // 16080 x 10720
         : i == 13 ? TablePlan{670, 128, 128, 1005, 8, 512}  // 128640 x 85760: 2^7 3 5 67 x 2^8 5 67
                   : TablePlan{0, 0, 0, 0};
}

// Two 512-thread blocks per CU = 4 waves per SIMD: caps registers at 128.
#define DOP_KERNEL(T) __global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(4)))

template <int PID>
struct Plan {
  static constexpr bool POW2 = PID < kTabBase;  // square power-of-two grid
  static constexpr TablePlan TP = table_plan(POW2 ? -1 : PID - kTabBase);
  static constexpr int MX = POW2 ? 1 << PID : TP.ax * TP.bx;  // columns
  static constexpr int MY = POW2 ? 1 << PID : TP.ay * TP.by;  // rows
  static constexpr size_t PITCH = (size_t)MX + kRowPad;  // workspace row pitch
  static constexpr int BX = POW2 ? 1 << plan_bx(PID) : TP.bx;
  static constexpr int AX = MX / BX;
  static constexpr int AY = POW2 ? 1 << plan_ay(PID) : TP.ay;
  static constexpr int BY = MY / AY;
  static constexpr int RA = TP.ra ? TP.ra : cmin(16, BX);  // run in passes A / A': a 128-byte line
  // contiguous run in pass C: 16 columns (128-byte lines); 8 on the 2^17
  // grid, whose 1024-row tiles would otherwise hold one block per CU (two
  // 80 KB blocks share a CU instead: pass C 75.7 -> 71.9 ms per wavelength)
  static constexpr int RC = TP.rc ? TP.rc : PID == 17 ? 8 : cmin(16, MX);
  // A / A' tiles (up to 1024 x 16 points, 128 KiB of LDS) run one block of
  // up to 1024 threads per CU
  // (other M: about 8 points per thread, since their mixed-radix stage
  // shapes do not divide evenly among threads and need more registers each)
  static constexpr int TA = TP.ta ? TP.ta : round64(cmin(1024, cmax(64, AX * RA / (POW2 ? 16 : 8))));
  // pass-B / B' threads: about 16 points each, 8 on the 2048 and 4096 grids
  // (passes B and B' at 4096^2: 61 -> 58 and 52 -> 48 us per wavelength)
  static constexpr int TB = TP.tb ? TP.tb : !POW2 ? round64(cmin(1024, cmax(64, BX * AY / 8)))
                            : BX * AY > 8192 ? 1024
                            : (PID == 11 || PID == 12) ? 2 * threads_for(BX * AY)
                                                       : threads_for(BX * AY);
  // pass-C threads: about 16 points each, except 8 on the 2048, 4096 and
  // 32768 grids, whose 64-, 64- and 256-row transforms spilled registers at
  // 16 (pass C at 4096^2: 71 -> 53 us per wavelength; at 32768^2: 3.84 ->
  // 3.69 ms)
  static constexpr int TC = TP.tc ? TP.tc : !POW2 ? round64(cmin(1024, cmax(64, BY * RC / 8)))
                            : BY * RC > 8192 ? 1024
                            : (PID == 11 || PID == 12 || PID == 15) ? 2 * threads_for(BY * RC)
                                                                     : threads_for(BY * RC);
  // Twiddles in LDS: omega_M^q = HI[q / S] * LO[q % S] with HI[i] = omega_M^(i S)
  // (= omega_THI^i) and LO[i] = omega_M^i.  Power-of-two M: THI = min(M, 1024),
  // which also serves every inner DFT length.  Table grids: THI = AX (S = BX),
  // the inner table of passes A and A'; passes B, B' and C keep their own.
  static constexpr int THI = POW2 ? (MX < 1024 ? MX : 1024) : AX;
  static constexpr int S = MX / THI;
  static_assert(AX * BX == MX && AY * BY == MY, "digit split");
  static_assert(MX % 2 == 0 && MY % 2 == 0, "even axes (signed frequency split at M / 2)");
  static_assert(is_pow2c(BX) && BX % RA == 0 && MX % RC == 0, "runs");
  static_assert(AX * RA <= 16384 && BX * AY <= 16384 && BY * RC <= 16384, "tile sizes");
  static_assert(AX <= 1024 && BX <= 1024 && AY <= 1024 && BY <= 1024, "digit lengths");
};

// Four-step twiddles of one axis (x: passes A and A'; y: passes B and B').
// The y axis shares the x tables on a square grid; on a rectangular one it
// has its own, HI over AY and LO over BY (q = yb * kya < My).
template <int PID, bool Y>
struct TwAxis {
  using P = Plan<PID>;
  static constexpr bool OWN = Y && P::MX != P::MY;
  static constexpr int M = Y ? P::MY : P::MX;
  static constexpr int THI = OWN ? P::AY : P::THI;
  static constexpr int S = M / THI;
};

template <int PID, bool Y = false>
struct TwLds {
  float2 hi[TwAxis<PID, Y>::THI];
  float2 lo[TwAxis<PID, Y>::S];
};

// exp(-2 pi i num / den), 0 <= num < den, formed in FP64 and rounded once.
DEV float2 omega_fp64(int num, int den) {
  double sn, cs;
  sincospi(-2.0 * (double)num / (double)den, &sn, &cs);
  return make_float2((float)cs, (float)sn);
}

// This plan's twiddles in LDS: from the FP64-generated global table
// (power-of-two M), or generated in FP64 (table grids).
template <int PID, int T, bool Y = false>
DEV void tw_fill(TwLds<PID, Y> &t, const float2 *__restrict__ g) {
  using P = Plan<PID>;
  using A = TwAxis<PID, Y>;
  if constexpr (P::POW2) {
    for (int i = threadIdx.x; i < A::THI; i += T) t.hi[i] = g[(i * A::S) << (kTwLog - PID)];
    for (int i = threadIdx.x; i < A::S; i += T) t.lo[i] = g[i << (kTwLog - PID)];
  } else {
    for (int i = threadIdx.x; i < A::THI; i += T) t.hi[i] = omega_fp64(i * A::S, A::M);
    for (int i = threadIdx.x; i < A::S; i += T) t.lo[i] = omega_fp64(i, A::M);
  }
}

// Table of omega_L^i, i < L (the inner twiddles of an L-point DFT).
template <int L, int T>
DEV void omega_fill(float2 *t) {
  for (int i = threadIdx.x; i < L; i += T) t[i] = omega_fp64(i, L);
}

// omega_M^q (forward sign) of the axis, q >= 0.
template <int PID, bool Y = false>
DEV float2 tw_q(const TwLds<PID, Y> &t, int q) {
  using A = TwAxis<PID, Y>;
  const unsigned u = (unsigned)q % (unsigned)A::M;
  if constexpr (A::S == 1) {
    return t.hi[u];
  } else {
    return cmul(t.hi[u / A::S], t.lo[u % A::S]);
  }
}

// Tiles per launch are walked by a grid of resident blocks.  Blocks are
// handed to the eight XCDs round-robin, so tile ids are permuted within each
// run of 64 to give every XCD eight consecutive tiles at a time (neighbouring
// tiles share cache lines and DRAM pages).
__host__ __device__ constexpr int kMaxBlocks = 4096;
DEV int xcd_tile(int p, int ntiles) {
  if (p >= (ntiles & ~63)) return p;
  return (p & ~63) | ((p & 7) << 3) | ((p >> 3) & 7);
}

// Passes A and A' read heights and read-modify-write the PSF in float runs
// shorter than a cache line, shared by CH sibling tiles of one row.  A block walks the siblings of a chunk back to back (the
// chunks themselves in the XCD-aware order), so each line is consumed by one
// block while it is still in L2 even with the next tile's loads in flight.
template <int CH>
struct ChunkSeq {
  int ntiles, nchunks;
  DEV explicit ChunkSeq(int n) : ntiles(n), nchunks((n + CH - 1) / CH) {}
  // k-th tile of this block (k counts the block's own tiles), or -1
  DEV int tile(int k) const {
    const int q = (int)blockIdx.x + (k / CH) * (int)gridDim.x;
    if (q >= nchunks) return -1;
    const int t = CH * xcd_tile(q, nchunks) + k % CH;
    return t < ntiles ? t : -2;  // -2: past the end of a short last chunk
  }
};

// ---------------------------------------------------------------------------
// Element-wise physics.
// ---------------------------------------------------------------------------

// exp(i 2 pi f) for f in [-1/2, 1/2] turn: the hardware sine and cosine take
// their argument in turns (max abs error 1.3e-7 over [-1/2, 1/2], measured
// against FP64 on gfx950).
DEV float2 cis_turns(float f) {
  return make_float2(__builtin_amdgcn_cosf(f), __builtin_amdgcn_sinf(f));
}

// exp(i 2 pi q), q = turns_per_h * h formed in FP64 and reduced to
// [-1/2, 1/2] turn before the cast to FP32 (Eq. 1-2).
DEV float2 doe_phase(float hv, double turns_per_h) {
  const double q = turns_per_h * (double)hv;
  return cis_turns((float)(q - rint(q)));
}

// sqrt(q) for q in (0, 1] in FP64: FP32 reciprocal-square-root seed (relative
// error below 2^-22) and one Goldschmidt iteration, which squares the error:
// below 3e-14 relative.  Times z/lambda <= 2^17 turns that is under 4e-9 turn
// of phase, far below the 1.3e-7 turn error of the FP32 sin/cos that follows.
DEV double sqrt_unit(double q) {
  const double r = (double)__builtin_amdgcn_rsqf((float)q);
  const double g = q * r, h = 0.5 * r;
  const double e = fma(-g, h, 0.5);
  return fma(g, e, g);
}

// Per-axis frequency data of DFT bin k of an M-point axis: f = k_signed / (M dx), the
// square (lambda f)^2 with each product rounded once in FP64 (no
// contraction), as the evanescent test needs, and whether |f| is inside the
// band limit (always, unless DOP_BANDLIMIT).
struct AxisFreq {
  double a2;
  bool inband;
};
DEV AxisFreq axis_freq(int k, int m, double inv_md, double flim, const KParams &p) {
#pragma clang fp contract(off)
  const int ks = k < (m >> 1) ? k : k - m;
  const double f = (double)ks * inv_md;
  const double a = p.lam * f;
  return AxisFreq{a * a, fabs(f) < flim};
}

// (lambda f)^2 of one axis with the band limit folded in: a frequency outside
// the band gets 2, so that s >= 1 below whatever the other axis holds (an
// in-band s is unchanged).
DEV double a2_eff(AxisFreq f) { return f.inband ? f.a2 : 2.0; }

// H(ky, kx) from the two axes' a2_eff: zero unless s = a2y + a2x < 1; else
// exp(i 2 pi zl sqrt(1 - s)) with the argument formed and reduced mod one
// turn in FP64.  zl = z / lambda, negated for the adjoint (conj(H) is H at
// -z).  The inverse DFT's 1/M^2 is left to the last pass's output constants.
// Branch-free: cut bins evaluate a harmless dummy root (1 - s is floored at
// 2^-60, below any propagating 1 - s >= 2^-53) and are replaced by zero.
DEV float2 transfer(double a2y, double a2x, const KParams &p) {
#pragma clang fp contract(off)
  const double s = a2y + a2x;
  const double t = p.zl * sqrt_unit(fmax(1.0 - s, 0x1p-60));
  const float2 w = cis_turns((float)(t - rint(t)));
  return s < 1.0 ? w : make_float2(0.f, 0.f);
}

// Entry q of a per-group constant, selected with constant indices: indexing
// a kernel-argument array with a run-time value would copy the whole
// parameter block to scratch memory.
template <class T>
DEV T group_value(const T (&a)[kMaxGroup], int q) {
  static_assert(kMaxGroup == 4, "one select per entry");
  return q == 0 ? a[0] : q == 1 ? a[1] : q == 2 ? a[2] : a[3];
}

// One wavelength's term of the PSF (Eq. 4) added to an accumulator: acc +
// w_k |U|^2 with U = w / (My Mx) folded into wk.  Shared by the per-wavelength
// and the grouped output stages, so that both round alike.
DEV float psf_add(float acc, float wk, float2 w) { return acc + wk * (w.x * w.x + w.y * w.y); }

// Element at a 32-bit byte offset from a block-uniform base: the offset is
// formed in 32-bit arithmetic so the access can take a scalar base plus one
// 32-bit vector offset instead of a 64-bit address per lane.
template <class T>
DEV T *at_byte(T *base, unsigned off) {
  return reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off);
}
template <class T>
DEV const T *at_byte(const T *base, unsigned off) {
  return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}

// ---------------------------------------------------------------------------
// Pass A: DFT over xa for the N input rows, input formed on the fly.
// Tile = one row y and a run of RA consecutive xb.
// ---------------------------------------------------------------------------
template <int PID, int INM>
DOP_KERNEL(Plan<PID>::TA) void k_pass_a_fwd(KParams p) {
  using P = Plan<PID>;
  constexpr int AX = P::AX, BX = P::BX, RA = P::RA, T = P::TA;
  using G = Geo<AX, RA, RA, 1, T, false>;
  using FS = FirstStage<G>;
  __shared__ float2 lds[AX * RA];
  __shared__ TwLds<PID> tw;
  tw_fill<PID, T>(tw, p.tw);
  constexpr int RUNS = BX / RA;
  const int ntiles = p.nrows_in * RUNS;
  const int n = p.n;
  // Raw inputs of one tile's first DFT stage, loaded one tile ahead:
  // (h, amp) for IN_PHASE, the field for IN_FIELD, the saved field for
  // IN_GRAD; columns x >= n are zero.
  float2 pre[FS::PER][FS::R];
  // A tile is one input row: its arrays are addressed as a tile-uniform row
  // base plus a 32-bit byte offset per element.
  auto fetch = [&](int tile, int tid) {
    const int y = tile / RUNS;
    const size_t rowin = (size_t)y * n;
    const float *hrow = p.h + (size_t)(y >> p.up_log2) * p.nh;
    const float *arow = p.amp ? p.amp + rowin : nullptr;
    const float2 *frow = INM == IN_FIELD ? p.u_in + rowin : INM == IN_GRAD ? p.saved_in + rowin
                                                                          : nullptr;
    const int xb0 = (tile % RUNS) * RA;
#pragma unroll
    for (int i = 0; i < FS::PER; ++i) {
      const int it = tid + i * T;
      if (FS::EXACT || it < FS::ITEMS) {
        int j, b;
        decode_item<G, FS::R>(it, j, b);
#pragma unroll
        for (int t = 0; t < FS::R; ++t) {
          const int x = BX * (j + t * FS::LR) + xb0 + b;
          float2 v = make_float2(0.f, 0.f);
          if (x < n) {
            const unsigned ux = (unsigned)x;
            if constexpr (INM == IN_PHASE)
              v = make_float2(*at_byte(hrow, (ux >> p.up_log2) * 4u),
                              arow ? *at_byte(arow, ux * 4u) : 1.f);
            else v = *at_byte(frow, ux * 8u);
          }
          pre[i][t] = v;
        }
      }
    }
  };
  constexpr int CH = RUNS < 4 ? RUNS : 4;
  const ChunkSeq<CH> seq(ntiles);
  const int ngroup = INM == IN_PHASE ? p.group : 1;
  if (seq.tile(0) >= 0) fetch(seq.tile(0), threadIdx.x);
  for (int k = 0;; ++k) {
    const int tile = seq.tile(k);
    if (tile == -1) break;
    if (tile < 0) continue;
    const int y = tile / RUNS;
    const int xb0 = (tile % RUNS) * RA;
    // a group of wavelengths shares the tile's heights.  On grids of 2^28
    // points and more the prefetched values stay in registers for every
    // member of the group (each forms its field from them and writes its own
    // workspace field) and the next tile's loads are issued during the last
    // member's transform, so h crosses the fabric once per group.  Smaller
    // grids re-read the tile (an L2 hit) for each member: keeping the values
    // live there made the compiler spill.  (Grids with the factor 67 in x
    // run one wavelength at a time.)
    constexpr bool KEEP_H = (size_t)P::MX * P::MY >= (1ull << 28) && n67(AX) == 0;
    for (int q = 0; q < ngroup; ++q) {
      const int tid = loop_tid();
      __syncthreads();
      const double turns = ngroup > 1 ? group_value(p.phase_turns_g, q) : p.phase_turns;
      // the DOE field (Eq. 1-2) or the caller's field, from the prefetched values
      float2 v[FS::PER][FS::R];
#pragma unroll
      for (int i = 0; i < FS::PER; ++i) {
        const int it = tid + i * T;
        if (FS::EXACT || it < FS::ITEMS) {
          int j, b;
          decode_item<G, FS::R>(it, j, b);
#pragma unroll
          for (int t = 0; t < FS::R; ++t) {
            const float2 r = pre[i][t];
            if constexpr (INM == IN_PHASE) {
              v[i][t] = cscale(doe_phase(r.x, turns), r.y);  // r.y = 0 past column n
            } else if constexpr (INM == IN_FIELD) {
              v[i][t] = r;
            } else {
              const int x = BX * (j + t * FS::LR) + xb0 + b;
              v[i][t] = x < n ? cscale(r, p.two_wk * p.gpsf[(size_t)y * n + x]) : r;
            }
          }
        }
      }
      if (q + 1 < ngroup) {
        if constexpr (!KEEP_H) fetch(tile, tid);
      } else {
        const int nt = seq.tile(k + 1) >= 0 ? seq.tile(k + 1) : seq.tile(k + 2);
        if (nt >= 0) fetch(nt, tid);
      }
      float2 *out = p.ws + (size_t)q * p.field_elems + (size_t)y * P::PITCH;
      auto st = [&](int kxa, int b, float2 w) {
        const int xb = xb0 + b;
        out[BX * kxa + xb] = cmul(w, tw_q<PID>(tw, xb * kxa));
      };
      dft_tile<G, false, false, SRC_REG, SNK_FN, P::THI>(lds, tw.hi, NoLoad{}, st, v, tid);
    }
  }
}

// ---------------------------------------------------------------------------
// Pass B: DFT over xb then over ya on a BX x AY tile (tile = (kxa, yb)).
// Rows are moved between HBM and LDS as 16-byte (two-element) vectors.
// ---------------------------------------------------------------------------
typedef float f4v __attribute__((ext_vector_type(4)));

DEV f4v ld_pair(const float2 *p) { return *reinterpret_cast<const f4v *>(p); }
DEV void st_pair(float2 *p, float2 a, float2 b) {
  *reinterpret_cast<f4v *>(p) = f4v{a.x, a.y, b.x, b.y};
}

template <int PID>
DOP_KERNEL(Plan<PID>::TB) void k_pass_b_fwd(KParams p) {
  using P = Plan<PID>;
  constexpr int AX = P::AX, BX = P::BX, AY = P::AY, BY = P::BY, T = P::TB;
  constexpr int SR = BX + 1;  // odd row stride: conflict-free for both DFT directions
  constexpr int HB = BX / 2;  // 16-byte pairs per row segment
  constexpr int PF = (AY * HB + T - 1) / T;  // pairs each thread moves per tile
  __shared__ float2 lds[AY * SR];
  __shared__ TwLds<PID, true> tw;  // y four-step twiddles omega_My
  __shared__ float2 rowtw[AY];
  // inner twiddles: the shared power-of-two table, else tables of their own
  __shared__ float2 wbx[P::POW2 ? 1 : BX], way[P::POW2 ? 1 : AY];
  tw_fill<PID, T, true>(tw, p.tw);
  if constexpr (!P::POW2) {
    omega_fill<BX, T>(wbx);
    omega_fill<AY, T>(way);
  }
  constexpr int THX = P::POW2 ? P::THI : BX, THY = P::POW2 ? P::THI : AY;
  const float2 *twx = P::POW2 ? tw.hi : wbx;
  const float2 *twy = P::POW2 ? tw.hi : way;
  constexpr int NT = AX * BY;
  float2 dummy[1][1];
  // rows ya with BY*ya + yb >= nrows_in hold zeros: not read, x-DFT skipped
  auto nzrows = [&](int yb) {
    return p.nrows_in > yb ? cmin(AY, (p.nrows_in - yb + BY - 1) / BY) : 0;
  };
  // Loads of one tile's nonzero rows into registers; issued one tile ahead so
  // that they are in flight while the current tile is transformed.
  f4v pre[PF];
  auto fetch = [&](int pt, int tid) {
    const int tile = xcd_tile(pt, NT);
    const int kxa = tile % AX, yb = tile / AX, nz = nzrows(yb);
    const float2 *src = p.ws + (size_t)yb * P::PITCH + (size_t)BX * kxa;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = tid + i * T, ya = e / HB, c = e % HB;
      pre[i] = f4v{0.f, 0.f, 0.f, 0.f};
      if ((PF * T == AY * HB || e < AY * HB) && ya < nz)
        pre[i] = ld_pair(src + (size_t)(BY * ya) * P::PITCH + 2 * c);
    }
  };
  if (blockIdx.x < NT) fetch(blockIdx.x, threadIdx.x);
  for (int pt = blockIdx.x; pt < NT; pt += gridDim.x) {
    const int tid = loop_tid();
    const int tile = xcd_tile(pt, NT);
    const int kxa = tile % AX;
    const int yb = tile / AX;
    const size_t col0 = (size_t)BX * kxa;
    const int nz = nzrows(yb);
    __syncthreads();
    for (int r = tid; r < AY; r += T) rowtw[r] = tw_q<PID, true>(tw, yb * r);  // omega_My^(yb kya)
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = tid + i * T, ya = e / HB, c = e % HB;
      if (PF * T == AY * HB || e < AY * HB) {
        lds[ya * SR + 2 * c] = make_float2(pre[i].x, pre[i].y);
        lds[ya * SR + 2 * c + 1] = make_float2(pre[i].z, pre[i].w);
      }
    }
    if (pt + (int)gridDim.x < NT) fetch(pt + gridDim.x, tid);
    __syncthreads();
    using GX = Geo<BX, AY, 1, SR, T, false>;
    dft_tile<GX, false, false, SRC_LDS, SNK_LDS, THX>(lds, twx, NoLoad{}, NoStore{}, dummy, tid, nz);
    using GY = Geo<AY, BX, SR, 1, T, false>;
    dft_tile<GY, false, false, SRC_LDS, SNK_LDS, THY>(lds, twy, NoLoad{}, NoStore{}, dummy, tid);
    for (int e = tid; e < AY * HB; e += T) {
      const int kya = e / HB, c = e % HB;
      const float2 w = rowtw[kya];
      st_pair(p.ws + (size_t)(BY * kya + yb) * P::PITCH + col0 + 2 * c,
              cmul(lds[kya * SR + 2 * c], w), cmul(lds[kya * SR + 2 * c + 1], w));
    }
  }
}

// ---------------------------------------------------------------------------
// Pass C: DFT over yb, times H, inverse DFT over yb (tile = (kya, run of RC
// columns)).
// ---------------------------------------------------------------------------
template <int PID>
DOP_KERNEL(Plan<PID>::TC) void k_pass_c(KParams p) {
  using P = Plan<PID>;
  constexpr int AX = P::AX, BX = P::BX, AY = P::AY, BY = P::BY, RC = P::RC, T = P::TC;
  // LDS row stride: one pad element for 16-column tiles; an 8-column tile
  // goes unpadded so that two blocks fit in a CU's LDS
  constexpr int SJ = RC >= 16 ? RC + 1 : RC;
  using G = Geo<BY, RC, SJ, 1, T, false>;
  using FS = FirstStage<G>;
  // A radix-67 stage cannot hand its outputs over in registers: with one, the
  // forward DFT ends in LDS (natural order) and the inverse DFT reads it
  // through a load functor that applies H.
  constexpr bool VIA_LDS = n67(BY) > 0;
  static_assert((size_t)BY * P::PITCH * sizeof(float2) <= 0xFFFFFFFFull,
                "tile byte offsets are 32-bit");
  __shared__ float2 lds[BY * SJ];
  // only BY-point DFTs run here: their twiddles omega_BY^i, i < BY
  __shared__ float2 twc[BY];
  // a2_eff of the tile's BY frequency rows (and, via LDS, of its RC columns)
  __shared__ double a2row[BY];
  __shared__ double a2col[VIA_LDS ? RC : 1];
  if constexpr (P::POW2) {
    for (int i = threadIdx.x; i < BY; i += T) twc[i] = p.tw[i << (kTwLog - ilog2c(BY))];
  } else {
    omega_fill<BY, T>(twc);
  }
  constexpr int RUNS = P::MX / RC;
  constexpr int NT = AY * RUNS;
  auto tile_base = [&](int pt) {
    const int tile = xcd_tile(pt, NT);
    return p.ws + (size_t)(BY * (tile / RUNS)) * P::PITCH + (tile % RUNS) * RC;
  };
  // frequency-x data of padded column px (spectrum position BX kxa + kxb
  // holds kx = kxa + AX kxb)
  auto col_a2 = [&](int px) {
    const int kx = (px / BX) + AX * (px % BX);
    return a2_eff(axis_freq(kx, P::MX, p.inv_mdx, p.flim_x, p));
  };
  // one tile's first-stage inputs, loaded one tile ahead
  float2 pre[FS::PER][FS::R];
  auto fetch = [&](int pt, int tid) {
    const float2 *base = tile_base(pt);
#pragma unroll
    for (int i = 0; i < FS::PER; ++i) {
      const int it = tid + i * T;
      if (FS::EXACT || it < FS::ITEMS) {
        int j, b;
        decode_item<G, FS::R>(it, j, b);
#pragma unroll
        for (int t = 0; t < FS::R; ++t)
          pre[i][t] = *at_byte(base, ((unsigned)(j + t * FS::LR) * (unsigned)P::PITCH + b) * 8u);
      }
    }
  };
  if ((int)blockIdx.x < NT) fetch(blockIdx.x, threadIdx.x);
  for (int pt = blockIdx.x; pt < NT; pt += gridDim.x) {
    const int tid = loop_tid();
    const int tile = xcd_tile(pt, NT);
    const int px0 = (tile % RUNS) * RC;
    const int kya = tile / RUNS;
    float2 *base = p.ws + (size_t)(BY * kya) * P::PITCH + px0;
    __syncthreads();
    // frequency rows of this tile: position kyb holds ky = kya + AY kyb; read
    // after the forward DFT, whose stage barriers order this write before them
    for (int r = tid; r < BY; r += T)
      a2row[r] = a2_eff(axis_freq(kya + AY * r, P::MY, p.inv_mdy, p.flim_y, p));
    if constexpr (VIA_LDS)
      for (int c = tid; c < RC; c += T) a2col[c] = col_a2(px0 + c);
    float2 v[FS::PER][FS::R];
#pragma unroll
    for (int i = 0; i < FS::PER; ++i)
#pragma unroll
      for (int t = 0; t < FS::R; ++t) v[i][t] = pre[i][t];
    auto hook = [&]() {
      if (pt + (int)gridDim.x < NT) fetch(pt + gridDim.x, tid);
    };
    auto st = [&](int yb, int b, float2 w) {
      *at_byte(base, ((unsigned)yb * (unsigned)P::PITCH + b) * 8u) = w;
    };
    if constexpr (VIA_LDS) {
      float2 dummy[1][1];
      dft_tile_hooked<G, false, false, SRC_REG, SNK_LDS, BY>(lds, twc, NoLoad{}, NoStore{}, hook,
                                                            v, dummy, tid);
      auto ld_h = [&](int kyb, int b) {
        return cmul(lds[kyb * SJ + b], transfer(a2row[kyb], a2col[b], p));
      };
      dft_tile<G, true, true, SRC_FN, SNK_FN, BY>(lds, twc, ld_h, st, dummy, tid);
    } else {
      using LR_ = LastRegs<G, false>;
      float2 regs[LR_::PER][LR_::R];
      dft_tile_hooked<G, false, false, SRC_REG, SNK_REG, BY>(lds, twc, NoLoad{}, NoStore{}, hook,
                                                            v, regs, tid);
      {
        constexpr int R = LR_::R;
        constexpr int LRn = BY / R;
        using SS = StageShape<G, R>;
#pragma unroll
        for (int i = 0; i < LR_::PER; ++i) {
          const int it = tid + i * T;
          if (SS::EXACT || it < SS::ITEMS) {
            int j, b;
            decode_item<G, R>(it, j, b);
            const double a2x = col_a2(px0 + b);
#pragma unroll
            for (int t = 0; t < R; ++t)
              regs[i][t] = cmul(regs[i][t], transfer(a2row[j + t * LRn], a2x, p));
          }
        }
      }
      dft_tile<G, true, true, SRC_REG, SNK_FN, BY>(lds, twc, NoLoad{}, st, regs, tid);
    }
  }
}

// ---------------------------------------------------------------------------
// Pass B': inverse DFT over kya then over kxb (tile = (kxa, yb)); writes the
// rows y < nrows_out.
// ---------------------------------------------------------------------------
template <int PID>
DOP_KERNEL(Plan<PID>::TB) void k_pass_b_inv(KParams p) {
  using P = Plan<PID>;
  constexpr int AX = P::AX, BX = P::BX, AY = P::AY, BY = P::BY, T = P::TB;
  constexpr int SR = BX + 1;
  constexpr int HB = BX / 2;
  constexpr int PF = (AY * HB + T - 1) / T;
  __shared__ float2 lds[AY * SR];
  __shared__ TwLds<PID, true> tw;
  __shared__ float2 rowtw[AY];
  __shared__ float2 wbx[P::POW2 ? 1 : BX], way[P::POW2 ? 1 : AY];
  tw_fill<PID, T, true>(tw, p.tw);
  if constexpr (!P::POW2) {
    omega_fill<BX, T>(wbx);
    omega_fill<AY, T>(way);
  }
  constexpr int THX = P::POW2 ? P::THI : BX, THY = P::POW2 ? P::THI : AY;
  const float2 *twx = P::POW2 ? tw.hi : wbx;
  const float2 *twy = P::POW2 ? tw.hi : way;
  constexpr int NT = AX * BY;
  float2 dummy[1][1];
  f4v pre[PF];
  auto fetch = [&](int pt, int tid) {
    const int tile = xcd_tile(pt, NT);
    const int kxa = tile % AX, yb = tile / AX;
    const float2 *src = p.ws + (size_t)yb * P::PITCH + (size_t)BX * kxa;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = tid + i * T, kya = e / HB, c = e % HB;
      if (PF * T == AY * HB || e < AY * HB) pre[i] = ld_pair(src + (size_t)(BY * kya) * P::PITCH + 2 * c);
    }
  };
  if (blockIdx.x < NT) fetch(blockIdx.x, threadIdx.x);
  for (int pt = blockIdx.x; pt < NT; pt += gridDim.x) {
    const int tid = loop_tid();
    const int tile = xcd_tile(pt, NT);
    const int kxa = tile % AX;
    const int yb = tile / AX;
    const size_t col0 = (size_t)BX * kxa;
    // only the rows ya with BY*ya + yb < nrows_out are needed
    const int nz = p.nrows_out > yb ? cmin(AY, (p.nrows_out - yb + BY - 1) / BY) : 0;
    __syncthreads();
    for (int r = tid; r < AY; r += T) rowtw[r] = tw_q<PID, true>(tw, yb * r);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = tid + i * T, kya = e / HB, c = e % HB;
      if (PF * T == AY * HB || e < AY * HB) {
        const float2 w = rowtw[kya];
        lds[kya * SR + 2 * c] = cmulc(make_float2(pre[i].x, pre[i].y), w);
        lds[kya * SR + 2 * c + 1] = cmulc(make_float2(pre[i].z, pre[i].w), w);
      }
    }
    if (pt + (int)gridDim.x < NT) fetch(pt + gridDim.x, tid);
    __syncthreads();
    using GY = Geo<AY, BX, SR, 1, T, false>;
    dft_tile<GY, true, false, SRC_LDS, SNK_LDS, THY>(lds, twy, NoLoad{}, NoStore{}, dummy, tid);
    using GX = Geo<BX, AY, 1, SR, T, false>;
    dft_tile<GX, true, false, SRC_LDS, SNK_LDS, THX>(lds, twx, NoLoad{}, NoStore{}, dummy, tid, nz);
    for (int e = tid; e < nz * HB; e += T) {
      const int ya = e / HB, c = e % HB;
      st_pair(p.ws + (size_t)(BY * ya + yb) * P::PITCH + col0 + 2 * c, lds[ya * SR + 2 * c],
              lds[ya * SR + 2 * c + 1]);
    }
  }
}

// ---------------------------------------------------------------------------
// Pass A': inverse DFT over kxa for the rows y < nrows_out, then the output
// stage: PSF accumulation (Eq. 4), field, or height gradient.
// ---------------------------------------------------------------------------
template <int PID, int OUTM>
DOP_KERNEL(Plan<PID>::TA) void k_pass_a_inv(KParams p) {
  using P = Plan<PID>;
  constexpr int AX = P::AX, BX = P::BX, RA = P::RA, MX = P::MX, MY = P::MY, T = P::TA;
  using G = Geo<AX, RA, RA, 1, T, false>;
  using FS = FirstStage<G>;
  // A radix-67 last stage writes through a store functor that does the
  // output stage; otherwise the last stage's registers are finished here.
  constexpr bool VIA_FN = n67(AX) > 0;
  using LS = LastRegs<G, false>;
  constexpr int LRL = AX / LS::R;
  using SSL = StageShape<G, LS::R>;
  constexpr int APER = VIA_FN ? 1 : LS::PER, AR = VIA_FN ? 1 : LS::R;
  __shared__ float2 lds[AX * RA];
  __shared__ TwLds<PID> tw;
  tw_fill<PID, T>(tw, p.tw);
  constexpr int RUNS = BX / RA;
  const int ntiles = p.nrows_out * RUNS;
  const int n = p.n;
  const bool accumulate = (OUTM == OUT_PSF || OUTM == OUT_GRADH) && !p.first;
  // a group of wavelengths (PSF output, no saved fields) adds all its
  // intensities to one read-modify-write of the PSF; field q of the group
  // sits q * field_elems after the first
  const int ngroup = (OUTM == OUT_PSF && !VIA_FN) ? p.group : 1;
  // spectrum values of one tile's first inverse stage, loaded one tile ahead
  float2 pre[FS::PER][FS::R];
  auto fetch = [&](int tile, int tid, int q) {
    const float2 *row = p.ws + (size_t)q * p.field_elems + (size_t)(tile / RUNS) * P::PITCH +
                        (tile % RUNS) * RA;
#pragma unroll
    for (int i = 0; i < FS::PER; ++i) {
      const int it = tid + i * T;
      if (FS::EXACT || it < FS::ITEMS) {
        int j, b;
        decode_item<G, FS::R>(it, j, b);
#pragma unroll
        for (int t = 0; t < FS::R; ++t) pre[i][t] = row[BX * (j + t * FS::LR) + b];
      }
    }
  };
  // A tile is one row y, so every output array is addressed as a
  // tile-uniform row base plus a 32-bit column offset.  Element offset of
  // the output row of row y (full plane: centred, wrapped):
  auto out_row = [&](int y) -> size_t {
    if (p.full) {
      const int ys = y + p.p0y;  // < 2 My
      return (size_t)(ys >= MY ? ys - MY : ys) * MX;
    }
    return (size_t)y * n;
  };
  // output column of element (xa, b) of the current tile; false if outside
  auto out_col = [&](int xb0, int xa, int b, unsigned &c) {
    const int x = BX * xa + xb0 + b;
    if (p.full) {
      const int xs = x + p.p0x;  // < 2 Mx
      c = (unsigned)(xs >= MX ? xs - MX : xs);
      return true;
    }
    c = (unsigned)x;
    return x < n;
  };
  // Row bases of the outputs (and, for the gradient, of h and amp).
  struct Rows {
    float *acc;         // PSF or gradient row
    float2 *field;      // saved or output field row (NULL if none)
    const float *h;     // height row (gradient)
    const float *amp;   // aperture row (gradient, NULL if none)
  };
  auto rows_of = [&](int y) {
    const size_t r = out_row(y);
    Rows o{nullptr, nullptr, nullptr, nullptr};
    if constexpr (OUTM == OUT_PSF) {
      o.acc = p.psf + r;
      if (p.saved_out) o.field = p.saved_out + r;
    } else if constexpr (OUTM == OUT_FIELD) {
      o.field = p.u_out + r;
    } else {
      o.acc = p.grad_h + r;
      o.h = p.h + (size_t)(y >> p.up_log2) * p.nh;
      if (p.amp) o.amp = p.amp + r;
    }
    return o;
  };
  // output stage of one element at column c: w is My Mx U (the inverse DFT's
  // 1/(My Mx) is applied here), accv the accumulator value it adds to, wk
  // the PSF weight
  auto finish = [&](const Rows &o, unsigned c, float2 w, float accv, float wk) {
    if constexpr (OUTM == OUT_PSF) {
      *at_byte(o.acc, c * 4u) = psf_add(accv, wk, w);
      if (o.field) *at_byte(o.field, c * 8u) = cscale(w, p.inv_m2);
    } else if constexpr (OUTM == OUT_FIELD) {
      *at_byte(o.field, c * 8u) = cscale(w, p.inv_m2);
    } else {
      // crop only: the column is x < n
      float2 e = doe_phase(o.h[c >> p.up_log2], p.phase_turns);
      if (o.amp) e = cscale(e, *at_byte(o.amp, c * 4u));
      // c_k Im(g_E conj(E)), g_E = w / (My Mx)
      *at_byte(o.acc, c * 4u) = accv + p.ck_m2 * (w.y * e.x - w.x * e.y);
    }
  };
  constexpr int CH = RUNS < 4 ? RUNS : 4;
  const ChunkSeq<CH> seq(ntiles);
  if (seq.tile(0) >= 0) fetch(seq.tile(0), threadIdx.x, 0);
  for (int k = 0;; ++k) {
    const int tile = seq.tile(k);
    if (tile == -1) break;
    if (tile < 0) continue;
    const int y = tile / RUNS;
    const int xb0 = (tile % RUNS) * RA;
    const Rows orow = rows_of(y);
    float acc[APER][AR];
    for (int q = 0; q < ngroup; ++q) {
      const int tid = loop_tid();
      __syncthreads();
      const float wk = ngroup > 1 ? group_value(p.wk_m4_g, q) : p.wk_m4;
      float2 v[FS::PER][FS::R];
#pragma unroll
      for (int i = 0; i < FS::PER; ++i) {
        const int it = tid + i * T;
        if (FS::EXACT || it < FS::ITEMS) {
          int j, b;
          decode_item<G, FS::R>(it, j, b);
#pragma unroll
          for (int t = 0; t < FS::R; ++t)
            v[i][t] = cmulc(pre[i][t], tw_q<PID>(tw, (xb0 + b) * (j + t * FS::LR)));
        }
      }
      // After the first stage: read the accumulator values this tile will
      // add to (once per group), then start the next loads (the group's next
      // field of this tile, else the next tile).  Loads complete in issue
      // order, so the accumulator reads go first: waiting for them at the end
      // of this tile must not also wait for the prefetch.
      auto hook = [&]() {
        if constexpr (!VIA_FN) {
          if (q == 0) {
#pragma unroll
            for (int i = 0; i < LS::PER; ++i) {
              const int it = tid + i * T;
              int j = 0, b = 0;
              if (SSL::EXACT || it < SSL::ITEMS) decode_item<G, LS::R>(it, j, b);
#pragma unroll
              for (int t = 0; t < LS::R; ++t) {
                acc[i][t] = 0.f;
                unsigned c;
                if (accumulate && (SSL::EXACT || it < SSL::ITEMS) &&
                    out_col(xb0, j + t * LRL, b, c))
                  acc[i][t] = *at_byte(orow.acc, c * 4u);
              }
            }
          }
        }
        if (q + 1 < ngroup) {
          fetch(tile, tid, q + 1);
        } else {
          const int nt = seq.tile(k + 1) >= 0 ? seq.tile(k + 1) : seq.tile(k + 2);
          if (nt >= 0) fetch(nt, tid, 0);
        }
      };
      if constexpr (VIA_FN) {
        float2 dummy[1][1];
        auto st = [&](int xa, int b, float2 w) {
          unsigned c;
          if (!out_col(xb0, xa, b, c)) return;
          const float accv = accumulate ? *at_byte(orow.acc, c * 4u) : 0.f;
          finish(orow, c, w, accv, wk);
        };
        dft_tile_hooked<G, true, false, SRC_REG, SNK_FN, P::THI>(lds, tw.hi, NoLoad{}, st, hook, v,
                                                                dummy, tid);
      } else {
        float2 u[LS::PER][LS::R];
        dft_tile_hooked<G, true, false, SRC_REG, SNK_REG, P::THI>(lds, tw.hi, NoLoad{}, NoStore{},
                                                                 hook, v, u, tid);
        const bool last = q + 1 == ngroup;
#pragma unroll
        for (int i = 0; i < LS::PER; ++i) {
          const int it = tid + i * T;
          if (SSL::EXACT || it < SSL::ITEMS) {
            int j, b;
            decode_item<G, LS::R>(it, j, b);
#pragma unroll
            for (int t = 0; t < LS::R; ++t) {
              unsigned c;
              if (!out_col(xb0, j + t * LRL, b, c)) continue;
              if (last) finish(orow, c, u[i][t], acc[i][t], wk);
              else acc[i][t] = psf_add(acc[i][t], wk, u[i][t]);
            }
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Small-grid path (square power-of-two M up to 2048), three passes:
//   S1: M-point DFT over x of each of the N input rows (field formed from h
//       on the fly, Eq. 1-2), written in natural frequency order;
//   S2: for a run of columns, M-point DFT over y (rows >= N are zeros and not
//       read), times H (Eq. 3), inverse DFT over y; only the rows the output
//       needs are written back;
//   S3: inverse M-point DFT over kx of those rows, then the output stage
//       (|U|^2 accumulated into the PSF with the wavelength weight, Eq. 4,
//       and the optional saved field).
// A whole row or column fits in a block, so the 2-D FFT takes two sweeps
// instead of the large path's digit passes, and the column pass touches
// only the N rows that hold data.  At these sizes the field (<= 32 MiB)
// stays in the Infinity Cache between passes, and the five large-path
// launches were latency-bound.  At 4096 the column pass, limited to two
// columns (16-byte runs) by the LDS, was twice as slow as the large path.
// ---------------------------------------------------------------------------
template <int LM>
struct SmallPlan {
  static constexpr int M = 1 << LM;
  static constexpr size_t PITCH = (size_t)M + kRowPad;
  // points per thread: 8 below 2048 (more waves to hide the latency chain of
  // these small tiles), 16 at 2048 (measured equal or better there)
  static constexpr int PPT = M >= 2048 ? 16 : 8;
  // rows per S1/S3 tile (at least 512 points; two at 1024, measured 2 %
  // faster than one) and threads; at these sizes the passes are
  // latency-bound, so tiles are kept small and numerous
  static constexpr int RB = M == 1024 ? 2 : M >= 512 ? 1 : 512 / M;
  static constexpr int TR = cmax(64, RB * M / PPT);
  // columns per S2 tile: M / 256 (so that there are 256 tiles), at least 1
  // and at most 4
  static constexpr int C = cmin(4, cmax(1, M / 256));
  static constexpr int SJ = C + 1;  // LDS row stride: conflict-free column walks
  static constexpr int TC = cmax(64, M * C / PPT);
};

// The twiddle table omega_M^i, i < M, read into registers (loads issued, not
// yet waited for) and then written to LDS.
template <int LM, int T>
struct SmallTw {
  static constexpr int M = 1 << LM, N = (M + T - 1) / T;
  float2 r[N];
  DEV void load(const float2 *g) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      const int i = (int)threadIdx.x + q * T;
      if (M % T == 0 || i < M) r[q] = g[i << (kTwLog - LM)];
    }
  }
  DEV void put(float2 *tw) const {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      const int i = (int)threadIdx.x + q * T;
      if (M % T == 0 || i < M) tw[i] = r[q];
    }
  }
};

// The first Stockham stage's inputs of a tile gathered into registers, in
// the layout a register-fed first stage consumes (only the items it will
// use: b < nb_act).  Issued together with the twiddle loads, so the two
// memory latencies overlap instead of following each other; ld must not
// branch around its loads (clamp the address and select instead), so that
// all of an item's loads are in flight before the first is waited for.
// The register block a first stage of that shape consumes.
template <class G, bool REV>
using FirstRegs = float2[FirstStage<G, REV>::PER][FirstStage<G, REV>::R];
template <class G, bool REV, class LoadF>
DEV void gather_first(FirstRegs<G, REV> &pre, const LoadF &ld, const int tid, const int nb_act) {
  using FS = FirstStage<G, REV>;
#pragma unroll
  for (int i = 0; i < FS::PER; ++i) {
    const int it = tid + i * G::T;
    if (FS::EXACT || it < FS::ITEMS) {
      int j, b;
      decode_item<G, FS::R>(it, j, b);
      if (b < nb_act) {
#pragma unroll
        for (int t = 0; t < FS::R; ++t) pre[i][t] = ld(j + t * FS::LR, b);
      }
    }
  }
}

// S1 / S3: one tile = RB rows of M points; the row DFT runs along x.
// IN_PHASE forward (S1) or OUT_PSF inverse (S3, OUTM = OUT_PSF).  S1 (and S2)
// take the radices smallest first, so that every thread has items in the
// first stage, where the inputs' loads and the phase arithmetic sit (2 %
// faster at 1024^2 and 2048^2); S3 was faster in the natural order.
template <int LM, bool INV>
__global__ __launch_bounds__(SmallPlan<LM>::TR) void k_small_rows(KParams p) {
  using S = SmallPlan<LM>;
  constexpr int M = S::M, RB = S::RB, T = S::TR;
  // element (x, r) of the tile at LDS x * RB + r: x fastest across threads
  using G = Geo<M, RB, RB, 1, T, true>;
  using FS = FirstStage<G, !INV>;
  __shared__ float2 lds[M * RB];
  __shared__ float2 tw[M];
  const int nrows = INV ? p.nrows_out : p.nrows_in;
  const int ntiles = (nrows + RB - 1) / RB;
  const int n = p.n;
  // forward (S1): the DOE field (Eq. 1-2), zero past column n.  Branch-free:
  // columns past n read column 0 and are replaced by zero; without an
  // amplitude the amplitude load reads h[0] and is replaced by one.
  const float *amp_src = p.amp ? p.amp : p.h;
  auto ld_doe = [&](int y0, int x, int r) {
    const bool in = x < n;
    const int xc = in ? x : 0;
    const int y = y0 + r;
    const float hv = p.h[(size_t)(y >> p.up_log2) * p.nh + (xc >> p.up_log2)];
    const float av = amp_src[p.amp ? (size_t)y * n + xc : 0];
    const float a = p.amp ? av : 1.f;
    const float2 v = cscale(doe_phase(hv, p.phase_turns), a);
    return in ? v : make_float2(0.f, 0.f);
  };
  // inverse (S3): the spectrum rows left by S2
  auto ld_ws = [&](int y0, int kx, int r) { return p.ws[(size_t)(y0 + r) * S::PITCH + kx]; };
  auto gather = [&](int tile, float2 (&pre)[FS::PER][FS::R], int tid) {
    const int y0 = tile * RB, nb = cmin(RB, nrows - y0);
    if constexpr (!INV)
      gather_first<G, true>(pre, [&](int x, int r) { return ld_doe(y0, x, r); }, tid, nb);
    else
      gather_first<G, false>(pre, [&](int kx, int r) { return ld_ws(y0, kx, r); }, tid, nb);
  };
  SmallTw<LM, T> twr;
  twr.load(p.tw);
  float2 pre[FS::PER][FS::R];
  if ((int)blockIdx.x < ntiles) gather(blockIdx.x, pre, threadIdx.x);
  twr.put(tw);  // read from the second stage on, after the first's barriers
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int tid = loop_tid();
    const int y0 = tile * RB;
    const int nb = cmin(RB, nrows - y0);
    if (tile != (int)blockIdx.x) {
      __syncthreads();
      gather(tile, pre, tid);
    }
    if constexpr (!INV) {
      auto st = [&](int kx, int r, float2 v) { p.ws[(size_t)(y0 + r) * S::PITCH + kx] = v; };
      dft_tile<G, false, true, SRC_REG, SNK_FN, M>(lds, tw, NoLoad{}, st, pre, tid, nb);
    } else {
      // output stage: w is M^2 U (the inverse DFT's 1/M^2 is in the constants)
      auto st = [&](int x, int r, float2 w) {
        const int y = y0 + r;
        long long idx;
        if (p.full) {
          const int ys = y + p.p0y, xs = x + p.p0x;
          idx = (long long)(ys >= M ? ys - M : ys) * M + (xs >= M ? xs - M : xs);
        } else {
          if (x >= n) return;
          idx = (long long)y * n + x;
        }
        const float accv = p.first ? 0.f : p.psf[idx];
        p.psf[idx] = psf_add(accv, p.wk_m4, w);
        if (p.saved_out) p.saved_out[idx] = cscale(w, p.inv_m2);
      };
      dft_tile<G, true, false, SRC_REG, SNK_FN, M>(lds, tw, NoLoad{}, st, pre, tid, nb);
    }
  }
}

// S2: one tile = C consecutive columns of M points; DFT over y, times H,
// inverse DFT over y, rows < nrows_out written back.  A tile's rows are
// C * 8 bytes wide, so 128 / (C * 8) neighbouring tiles share each cache
// line: tiles go to blocks in the XCD-aware order, which puts neighbours on
// one XCD and its L2 (at 1024^2 this took the pass from 18.7 to 14.1 us).
template <int LM>
__global__ __launch_bounds__(SmallPlan<LM>::TC) void k_small_cols(KParams p) {
  using S = SmallPlan<LM>;
  constexpr int M = S::M, C = S::C, SJ = S::SJ, T = S::TC;
  using G = Geo<M, C, SJ, 1, T, false>;
  using FS = FirstStage<G, true>;
  __shared__ float2 lds[M * SJ];
  __shared__ float2 tw[M];
  __shared__ double a2col[C];
  constexpr int NT = M / C;
  auto gather = [&](int tile, float2 (&pre)[FS::PER][FS::R], int tid) {
    const int x0 = xcd_tile(tile, NT) * C;
    // rows at or past nrows_in are zero: read row 0 and replace (branch-free)
    auto ld = [&](int y, int c) {
      const bool in = y < p.nrows_in;
      const float2 v = p.ws[(size_t)(in ? y : 0) * S::PITCH + x0 + c];
      return in ? v : make_float2(0.f, 0.f);
    };
    gather_first<G, true>(pre, ld, tid, C);
  };
  SmallTw<LM, T> twr;
  twr.load(p.tw);
  float2 pre[FS::PER][FS::R];
  if ((int)blockIdx.x < NT) gather(blockIdx.x, pre, threadIdx.x);
  twr.put(tw);  // read from the second stage on, after the first's barriers
  for (int tile = blockIdx.x; tile < NT; tile += gridDim.x) {
    const int tid = loop_tid();
    const int x0 = xcd_tile(tile, NT) * C;
    if (tile != (int)blockIdx.x) {
      __syncthreads();
      gather(tile, pre, tid);
    }
    // frequency-x data of the tile's columns; read after the forward DFT,
    // whose stage barriers order this write before them
    for (int c = tid; c < C; c += T) a2col[c] = a2_eff(axis_freq(x0 + c, M, p.inv_mdx, p.flim_x, p));
    dft_tile<G, false, true, SRC_REG, SNK_LDS, M>(lds, tw, NoLoad{}, NoStore{}, pre, tid);
    auto ld_h = [&](int ky, int c) {
      const double a2y = a2_eff(axis_freq(ky, M, p.inv_mdy, p.flim_y, p));
      return cmul(lds[ky * SJ + c], transfer(a2y, a2col[c], p));
    };
    auto st = [&](int y, int c, float2 v) {
      if (y < p.nrows_out) p.ws[(size_t)y * S::PITCH + x0 + c] = v;
    };
    float2 dummy[1][1];
    dft_tile<G, true, true, SRC_FN, SNK_FN, M>(lds, tw, ld_h, st, dummy, tid);
  }
}

static inline void mark(hipEvent_t *ev, int i, hipStream_t s);

template <int LM>
static hipError_t launch_small_lm(const KParams &p, hipStream_t s, hipEvent_t *ev) {
  using S = SmallPlan<LM>;
  auto grid = [](long long tiles) {
    return (unsigned)(tiles < 1 ? 1 : tiles < kMaxBlocks ? tiles : kMaxBlocks);
  };
  mark(ev, 0, s);
  hipLaunchKernelGGL((k_small_rows<LM, false>), dim3(grid((p.nrows_in + S::RB - 1) / S::RB)),
                     dim3(S::TR), 0, s, p);
  mark(ev, 1, s);
  hipLaunchKernelGGL(k_small_cols<LM>, dim3(grid(S::M / S::C)), dim3(S::TC), 0, s, p);
  mark(ev, 2, s);
  hipLaunchKernelGGL((k_small_rows<LM, true>), dim3(grid((p.nrows_out + S::RB - 1) / S::RB)),
                     dim3(S::TR), 0, s, p);
  mark(ev, 3, s);
  return hipGetLastError();
}

bool small_path(int plan) { return plan >= kSmallMinLM && plan <= kSmallMaxLM; }

hipError_t launch_small(const KParams &p, hipStream_t s, hipEvent_t *ev) {
  if (p.in_mode != IN_PHASE || p.out_mode != OUT_PSF) return hipErrorInvalidValue;
  switch (p.plan) {
    case 4: return launch_small_lm<4>(p, s, ev);
    case 5: return launch_small_lm<5>(p, s, ev);
    case 6: return launch_small_lm<6>(p, s, ev);
    case 7: return launch_small_lm<7>(p, s, ev);
    case 8: return launch_small_lm<8>(p, s, ev);
    case 9: return launch_small_lm<9>(p, s, ev);
    case 10: return launch_small_lm<10>(p, s, ev);
    case 11: return launch_small_lm<11>(p, s, ev);
    default: return hipErrorInvalidValue;
  }
}
static_assert(kSmallMinLM == 4 && kSmallMaxLM == 11, "one launch case per small grid");

// ---------------------------------------------------------------------------
// Ceiling probe with pass C's memory access pattern and none of its
// arithmetic: the same tiles (BY rows x RC columns of the padded-pitch
// field), the same persistent grid and XCD-aware tile order, the same
// one-tile-ahead prefetch into the first stage's register layout (which is
// also the last inverse stage's store layout), the same LDS footprint (so as
// many blocks share a CU), and each element written back in place times
// `scale`.  What pass C achieves against this is the share of the pattern's
// bandwidth its arithmetic leaves.
// ---------------------------------------------------------------------------
template <int PID>
DOP_KERNEL(Plan<PID>::TC) void k_probe_passc(float2 *ws, float scale) {
  using P = Plan<PID>;
  constexpr int AY = P::AY, BY = P::BY, RC = P::RC, T = P::TC;
  constexpr int SJ = RC >= 16 ? RC + 1 : RC;
  using G = Geo<BY, RC, SJ, 1, T, false>;
  using FS = FirstStage<G>;
  static_assert((size_t)BY * P::PITCH * sizeof(float2) <= 0xFFFFFFFFull,
                "tile byte offsets are 32-bit");
  constexpr int RUNS = P::MX / RC;
  constexpr int NT = AY * RUNS;
  auto tile_base = [&](int pt) {
    const int tile = xcd_tile(pt, NT);
    return ws + (size_t)(BY * (tile / RUNS)) * P::PITCH + (tile % RUNS) * RC;
  };
  auto off = [&](int j, int b) { return ((unsigned)j * (unsigned)P::PITCH + b) * 8u; };
  float2 pre[FS::PER][FS::R];
  auto fetch = [&](int pt, int tid) {
    const float2 *base = tile_base(pt);
#pragma unroll
    for (int i = 0; i < FS::PER; ++i) {
      const int it = tid + i * T;
      if (FS::EXACT || it < FS::ITEMS) {
        int j, b;
        decode_item<G, FS::R>(it, j, b);
#pragma unroll
        for (int t = 0; t < FS::R; ++t) pre[i][t] = *at_byte(base, off(j + t * FS::LR, b));
      }
    }
  };
  if ((int)blockIdx.x < NT) fetch(blockIdx.x, threadIdx.x);
  for (int pt = blockIdx.x; pt < NT; pt += gridDim.x) {
    const int tid = loop_tid();
    float2 v[FS::PER][FS::R];
#pragma unroll
    for (int i = 0; i < FS::PER; ++i)
#pragma unroll
      for (int t = 0; t < FS::R; ++t) v[i][t] = pre[i][t];
    if (pt + (int)gridDim.x < NT) fetch(pt + gridDim.x, tid);
    float2 *base = tile_base(pt);
#pragma unroll
    for (int i = 0; i < FS::PER; ++i) {
      const int it = tid + i * T;
      if (FS::EXACT || it < FS::ITEMS) {
        int j, b;
        decode_item<G, FS::R>(it, j, b);
#pragma unroll
        for (int t = 0; t < FS::R; ++t) *at_byte(base, off(j + t * FS::LR, b)) = cscale(v[i][t], scale);
      }
    }
  }
}

// LDS bytes of pass C of plan PID (the probe reserves as much, dynamically).
template <int PID>
constexpr size_t pass_c_lds_bytes() {
  using P = Plan<PID>;
  constexpr int SJ = P::RC >= 16 ? P::RC + 1 : P::RC;
  constexpr bool VIA_LDS = n67(P::BY) > 0;
  return sizeof(float2) * (P::BY * SJ + P::BY) + sizeof(double) * (P::BY + (VIA_LDS ? P::RC : 1));
}

template <int PID>
static hipError_t launch_probe(float2 *ws, float scale, hipStream_t s) {
  using P = Plan<PID>;
  const long long tiles = (long long)P::AY * (P::MX / P::RC);
  const unsigned grid = (unsigned)(tiles < kMaxBlocks ? tiles : kMaxBlocks);
  hipLaunchKernelGGL(k_probe_passc<PID>, dim3(grid), dim3(P::TC), pass_c_lds_bytes<PID>(), s, ws,
                     scale);
  return hipGetLastError();
}

hipError_t launch_probe_passc(int plan, float2 *ws, float scale, hipStream_t s) {
  switch (plan) {
    case 14: return launch_probe<14>(ws, scale, s);
    case 15: return launch_probe<15>(ws, scale, s);
    case 16: return launch_probe<16>(ws, scale, s);
    case 17: return launch_probe<17>(ws, scale, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Host-side launch of the five passes.
// ---------------------------------------------------------------------------
static inline void mark(hipEvent_t *ev, int i, hipStream_t s) {
  if (ev) (void)hipEventRecord(ev[i], s);
}

template <int PID>
static hipError_t launch_range(const KParams &p, int first, int last, hipStream_t s,
                               hipEvent_t *ev) {
  using P = Plan<PID>;
  auto grid = [](long long tiles) {
    return (unsigned)(tiles < kMaxBlocks ? tiles : kMaxBlocks);
  };
  const unsigned ga = grid((long long)p.nrows_in * (P::BX / P::RA));
  const unsigned gb = grid((long long)P::AX * P::BY);
  const unsigned gc = grid((long long)P::AY * (P::MX / P::RC));
  const unsigned gai = grid((long long)p.nrows_out * (P::BX / P::RA));
  for (int pass = first; pass <= last; ++pass) {
    mark(ev, pass - first, s);
    switch (pass) {
      case 0:
        if (p.in_mode == IN_PHASE)
          hipLaunchKernelGGL((k_pass_a_fwd<PID, IN_PHASE>), dim3(ga), dim3(P::TA), 0, s, p);
        else if (p.in_mode == IN_FIELD)
          hipLaunchKernelGGL((k_pass_a_fwd<PID, IN_FIELD>), dim3(ga), dim3(P::TA), 0, s, p);
        else
          hipLaunchKernelGGL((k_pass_a_fwd<PID, IN_GRAD>), dim3(ga), dim3(P::TA), 0, s, p);
        break;
      case 1: hipLaunchKernelGGL(k_pass_b_fwd<PID>, dim3(gb), dim3(P::TB), 0, s, p); break;
      case 2: hipLaunchKernelGGL(k_pass_c<PID>, dim3(gc), dim3(P::TC), 0, s, p); break;
      case 3: hipLaunchKernelGGL(k_pass_b_inv<PID>, dim3(gb), dim3(P::TB), 0, s, p); break;
      default:
        if (p.out_mode == OUT_PSF)
          hipLaunchKernelGGL((k_pass_a_inv<PID, OUT_PSF>), dim3(gai), dim3(P::TA), 0, s, p);
        else if (p.out_mode == OUT_FIELD)
          hipLaunchKernelGGL((k_pass_a_inv<PID, OUT_FIELD>), dim3(gai), dim3(P::TA), 0, s, p);
        else
          hipLaunchKernelGGL((k_pass_a_inv<PID, OUT_GRADH>), dim3(gai), dim3(P::TA), 0, s, p);
        break;
    }
  }
  mark(ev, last - first + 1, s);
  return hipGetLastError();
}

hipError_t launch_passes(const KParams &p, int first, int last, hipStream_t s, hipEvent_t *ev) {
  if (first < 0 || last >= kNumPasses || first > last) return hipErrorInvalidValue;
  switch (p.plan) {
    case 4: return launch_range<4>(p, first, last, s, ev);
    case 5: return launch_range<5>(p, first, last, s, ev);
    case 6: return launch_range<6>(p, first, last, s, ev);
    case 7: return launch_range<7>(p, first, last, s, ev);
    case 8: return launch_range<8>(p, first, last, s, ev);
    case 9: return launch_range<9>(p, first, last, s, ev);
    case 10: return launch_range<10>(p, first, last, s, ev);
    case 11: return launch_range<11>(p, first, last, s, ev);
    case 12: return launch_range<12>(p, first, last, s, ev);
    case 13: return launch_range<13>(p, first, last, s, ev);
    case 14: return launch_range<14>(p, first, last, s, ev);
    case 15: return launch_range<15>(p, first, last, s, ev);
    case 16: return launch_range<16>(p, first, last, s, ev);
    case 17: return launch_range<17>(p, first, last, s, ev);
    case kTabBase + 0: return launch_range<kTabBase + 0>(p, first, last, s, ev);
    case kTabBase + 1: return launch_range<kTabBase + 1>(p, first, last, s, ev);
    case kTabBase + 2: return launch_range<kTabBase + 2>(p, first, last, s, ev);
    case kTabBase + 3: return launch_range<kTabBase + 3>(p, first, last, s, ev);
    case kTabBase + 4: return launch_range<kTabBase + 4>(p, first, last, s, ev);
    case kTabBase + 5: return launch_range<kTabBase + 5>(p, first, last, s, ev);
    case kTabBase + 6: return launch_range<kTabBase + 6>(p, first, last, s, ev);
    case kTabBase + 7: return launch_range<kTabBase + 7>(p, first, last, s, ev);
    case kTabBase + 8: return launch_range<kTabBase + 8>(p, first, last, s, ev);
    case kTabBase + 9: return launch_range<kTabBase + 9>(p, first, last, s, ev);
    case kTabBase + 10: return launch_range<kTabBase + 10>(p, first, last, s, ev);
    case kTabBase + 11: return launch_range<kTabBase + 11>(p, first, last, s, ev);
    case kTabBase + 12: return launch_range<kTabBase + 12>(p, first, last, s, ev);
    case kTabBase + 13: return launch_range<kTabBase + 13>(p, first, last, s, ev);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_wavelength(const KParams &p, hipStream_t s, hipEvent_t *ev) {
  return launch_passes(p, 0, kNumPasses - 1, s, ev);
}
static_assert(kNumTab == 14, "one launch case per grid of table_plan");

int plan_id(int mx, int my) {
  if (mx == my && mx >= 16 && mx <= (1 << 17) && is_pow2c(mx)) return ilog2c(mx);
  for (int i = 0; i < kNumTab; ++i) {
    const TablePlan t = table_plan(i);
    if (t.ax * t.bx == mx && t.ay * t.by == my) return kTabBase + i;
  }
  return -1;
}

int table_grids(int *rows, int *cols, int max) {
  for (int i = 0; i < kNumTab && i < max; ++i) {
    const TablePlan t = table_plan(i);
    rows[i] = t.ay * t.by;
    cols[i] = t.ax * t.bx;
  }
  return kNumTab;
}

template <int PID>
static void fill_plan(PlanInfo *o) {
  using P = Plan<PID>;
  o->ax = P::AX; o->bx = P::BX; o->ay = P::AY; o->by = P::BY; o->ra = P::RA; o->rc = P::RC;
  o->threads_a = P::TA; o->threads_b = P::TB; o->threads_c = P::TC;
}

// A group of wavelengths needs pass A' to hold the accumulator in registers,
// which a radix-67 last stage (writing through a store functor) does not.
int plan_max_group(int plan) {
  PlanInfo o;
  if (!plan_info(plan, &o)) return 0;
  return o.ax % kP == 0 ? 1 : kMaxGroup;
}

bool plan_info(int plan, PlanInfo *o) {
  switch (plan) {
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
    case 17: fill_plan<17>(o); return true;
    case kTabBase + 0: fill_plan<kTabBase + 0>(o); return true;
    case kTabBase + 1: fill_plan<kTabBase + 1>(o); return true;
    case kTabBase + 2: fill_plan<kTabBase + 2>(o); return true;
    case kTabBase + 3: fill_plan<kTabBase + 3>(o); return true;
    case kTabBase + 4: fill_plan<kTabBase + 4>(o); return true;
    case kTabBase + 5: fill_plan<kTabBase + 5>(o); return true;
    case kTabBase + 6: fill_plan<kTabBase + 6>(o); return true;
    case kTabBase + 7: fill_plan<kTabBase + 7>(o); return true;
    case kTabBase + 8: fill_plan<kTabBase + 8>(o); return true;
    case kTabBase + 9: fill_plan<kTabBase + 9>(o); return true;
    case kTabBase + 10: fill_plan<kTabBase + 10>(o); return true;
    case kTabBase + 11: fill_plan<kTabBase + 11>(o); return true;
    case kTabBase + 12: fill_plan<kTabBase + 12>(o); return true;
    case kTabBase + 13: fill_plan<kTabBase + 13>(o); return true;
    default: return false;
  }
}

}  // namespace dop
