// Device-side geometry of the polar-stroking tessellator (gfx950).
//
// Method: Kilgard, "Polar Stroking", ACM TOG 2020.  Every segment form is
// written through one hodograph: g'(t) is a positive multiple of
//     H(t) = (1-t)^2 E0 + 2(1-t)t E1 + t^2 E2
// with (a = P1-P0, b = P2-P1, c = P3-P2)
//     cubic      E0 = a,      E1 = b,          E2 = c        (factor 3)
//     quadratic  E0 = a,      E1 = (P2-P0)/2,  E2 = b        (factor 2)
//     conic      E0 = w a,    E1 = (P2-P0)/2,  E2 = w b      (factor 2/den^2)
//     line       E0 = E1 = E2 = P1-P0                        (factor 1)
// so the tangent-angle solve g'(t).N = 0 (Eq. angle2t) is the same quadratic
// for every kind and a wavefront never diverges on the segment form there.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ps.h"

namespace psd {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr double kCountEps = 1e-9;     // step count = ceil(|delta|/q - eps)
constexpr double kUnwrapGuard = 1e-12; // |short-way turn| below this is never unwrapped
constexpr int kMaxIv = 5;              // intervals per segment (collinear: 3 flat + 2 folds)

enum Role : uint8_t { ROLE_SEG = 0, ROLE_JOIN = 1, ROLE_SCAP = 2, ROLE_ECAP = 3, ROLE_EMPTY = 255 };

// Per-link record, written by the count kernel and read by emit: everything
// a rib of the link needs, as the emit kernels hold it (in LDS or registers).
// In memory it is kept in two parts, so that most links cost 64 bytes to
// write and to read instead of 144: a head that every link has (header,
// control points or pivot, the first two angles: the 16-byte pieces 0, 2, 3
// and 4 of the record) and a tail (pieces 1, 5, 6, 7, 8: the further interval
// ends, angles and parameters of a segment with several intervals, a miter
// join's normals) that only links flagged kHasTail have.  A reader without
// the tail takes dsum[1..4] = INT_MAX and never reads psi[2..5] or p.
struct alignas(16) LinkRec {
  uint8_t role;           // Role
  uint8_t n_iv;           // intervals (segments); 1 for pivots
  uint8_t kind;           // segment form (segments)
  uint8_t flags;          // kFirstInPath, kFirstSegInPath, kHasTail; bits 4..7: cap or join style
  float r;                // half the stroke width
  float w;                // conic weight (conics)
  int32_t dsum[kMaxIv];   // cumulative steps Delta_Sigma(1..n_iv), INT_MAX past the last; pivots: dsum[0] = J
  float x[4], y[4];       // control points (segments); x[0], y[0]: pivot (joins, caps)
  double psi[kMaxIv + 1]; // unwrapped Psi_0..Psi_{n_iv}; pivots psi[0], psi[1] = psi[0] + delta
  double p[kMaxIv - 1];   // interior interval boundaries p_1..p_{n_iv-1}; miter joins: unit normals
};
static_assert(sizeof(LinkRec) == 144, "LinkRec must stay 144 bytes");
static_assert(__builtin_offsetof(LinkRec, dsum) == 12 && __builtin_offsetof(LinkRec, x) == 32 &&
                  __builtin_offsetof(LinkRec, psi) == 64 && __builtin_offsetof(LinkRec, p) == 112,
              "the head and tail pieces of LinkRec assume this layout");

typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));
constexpr int kRecPieces = 9, kHeadPieces = 4, kTailPieces = 5;
// the record piece held by head piece k, and by tail piece k
__host__ __device__ constexpr int head_piece(int k) { return k == 0 ? 0 : k + 1; }
__host__ __device__ constexpr int tail_piece(int k) { return k == 0 ? 1 : k + 4; }

constexpr uint8_t kFirstInPath = 1;     // first link with ribs of its path
constexpr uint8_t kFirstSegInPath = 2;  // first segment with ribs of its path
constexpr uint8_t kHasTail = 4;         // the link's record has a tail

// A segment of two or three intervals needs only tail pieces 0, 1 and 3
// (dsum[1..4], psi[2..3], p[0..1]); a longer one, or a miter join, all five.
__host__ __device__ inline bool tail_whole(const LinkRec& r) { return r.n_iv > 3 || r.role != ROLE_SEG; }

// Device status word kept at the start of the workspace.
struct DevStatus {
  unsigned int flags;
  unsigned int pad;
  unsigned long long total_ribs;
  unsigned long long fixups;
  unsigned long long dash_ribs;
  unsigned long long dash_count;
  unsigned long long tile_counter;
  unsigned long long dash_tile_counter;
  unsigned long long scan_ticket;   // block order of the one-pass link scan
};

// ---------------------------------------------------------------------------
// Segments in FP64 (inputs are FP32 and taken as exact)
// ---------------------------------------------------------------------------
template <typename F>
struct SegT {
  int kind;
  int npts;
  F x[4], y[4];
  F w;
};
using Seg = SegT<double>;

__device__ __forceinline__ int npts_of(int kind) {
  return kind == PS_KIND_CUBIC ? 4 : (kind == PS_KIND_LINE ? 2 : 3);
}

// Segment i in the arithmetic F of the setup (the FP32 inputs convert exactly
// to either).
template <typename F = double>
__device__ inline SegT<F> load_seg(const ps_batch& B, int i) {
  SegT<F> s;
  s.kind = B.kind[i];
  s.npts = npts_of(s.kind);
  const int64_t S = B.n_segs;
  // points past the last one repeat it (constant indices only)
  s.x[0] = (F)B.cx[i];         s.y[0] = (F)B.cy[i];
  s.x[1] = (F)B.cx[S + i];     s.y[1] = (F)B.cy[S + i];
  s.x[2] = s.npts > 2 ? (F)B.cx[2 * S + i] : s.x[1];
  s.y[2] = s.npts > 2 ? (F)B.cy[2 * S + i] : s.y[1];
  s.x[3] = s.npts > 3 ? (F)B.cx[3 * S + i] : s.x[2];
  s.y[3] = s.npts > 3 ? (F)B.cy[3 * S + i] : s.y[2];
  s.w = (s.kind == PS_KIND_CONIC) ? (F)B.conic_w[i] : (F)1;
  return s;
}

// (the padded points repeat the last one, so all four can be tested)
__device__ __forceinline__ bool seg_is_point(const Seg& s) {
  // a conic of weight 0 is its chord P0 P2, whatever P1 is
  if (s.kind == PS_KIND_CONIC && s.w == 0.0) return s.x[2] == s.x[0] && s.y[2] == s.y[0];
  bool same = true;
#pragma unroll
  for (int k = 1; k < 4; ++k) same = same && s.x[k] == s.x[0] && s.y[k] == s.y[0];
  return same;
}

__device__ __forceinline__ bool seg_finite(const Seg& s) {
  bool ok = isfinite(s.w);
#pragma unroll
  for (int k = 0; k < 4; ++k) ok = ok && isfinite(s.x[k]) && isfinite(s.y[k]);
  return ok;
}

template <typename F>
__device__ __forceinline__ F sgn(F v) { return (F)((v > 0) - (v < 0)); }
__device__ __forceinline__ double sgn_d(double v) { return sgn(v); }

// ===========================================================================
// Setup arithmetic (count kernel), in FP64 (F = double) or, for the
// single-precision study mode, in FP32.  FMA contraction is off so the step
// counts come out of plain IEEE operations.
// ===========================================================================
#pragma clang fp contract(off)

template <typename F>
__device__ __forceinline__ F crs(F ax, F ay, F bx, F by) {
  return ax * by - ay * bx;
}

// Start / end gradient directions (unnormalised) by the fallbacks of the table
// of segment forms: difference successive control points until nonzero.
template <typename F>
__device__ inline void start_dir(const SegT<F>& s, F& dx, F& dy) {
  dx = s.x[1] - s.x[0]; dy = s.y[1] - s.y[0];
  if (s.kind == PS_KIND_CUBIC) {
    if (dx == 0 && dy == 0) { dx = s.x[2] - s.x[0]; dy = s.y[2] - s.y[0]; }
    if (dx == 0 && dy == 0) { dx = s.x[3] - s.x[0]; dy = s.y[3] - s.y[0]; }
  } else if (s.kind == PS_KIND_QUAD) {
    if (dx == 0 && dy == 0) { dx = s.x[2] - s.x[0]; dy = s.y[2] - s.y[0]; }
  } else if (s.kind == PS_KIND_CONIC) {
    // g'(0) = 2 w_B (P1 - P0): a negative weight starts backwards
    if ((dx == 0 && dy == 0) || s.w == 0) { dx = s.x[2] - s.x[0]; dy = s.y[2] - s.y[0]; }
    else if (s.w < 0) { dx = -dx; dy = -dy; }
  }
}

template <typename F>
__device__ inline void end_dir(const SegT<F>& s, F& dx, F& dy) {
  if (s.kind == PS_KIND_LINE) { dx = s.x[1] - s.x[0]; dy = s.y[1] - s.y[0]; return; }
  // last point minus the one before it (x[3] repeats the last point)
  const bool cub = s.kind == PS_KIND_CUBIC;
  dx = s.x[3] - (cub ? s.x[2] : s.x[1]); dy = s.y[3] - (cub ? s.y[2] : s.y[1]);
  if (s.kind == PS_KIND_CUBIC) {
    if (dx == 0 && dy == 0) { dx = s.x[3] - s.x[1]; dy = s.y[3] - s.y[1]; }
    if (dx == 0 && dy == 0) { dx = s.x[3] - s.x[0]; dy = s.y[3] - s.y[0]; }
  } else if (s.kind == PS_KIND_CONIC) {
    // g'(1) = 2 w_B (P2 - P1)
    if ((dx == 0 && dy == 0) || s.w == 0) { dx = s.x[2] - s.x[0]; dy = s.y[2] - s.y[0]; }
    else if (s.w < 0) { dx = -dx; dy = -dy; }
  } else {
    if (dx == 0 && dy == 0) { dx = s.x[2] - s.x[0]; dy = s.y[2] - s.y[0]; }
  }
}

template <typename F>
__device__ __forceinline__ F unit_angle(F dx, F dy) {
  // the direction of (dx,dy) after normalisation (Eq. Psi uses tan^-1 of the
  // normalised gradient)
  const F inv = (F)1 / sqrt(dx * dx + dy * dy);
  return atan2(inv * dy, inv * dx);
}

// relative angle difference (-)
template <typename F>
__device__ __forceinline__ F adiff(F a, F b) {
  F d = a - b;
  if (d > (F)kPi) return d - (F)kTwoPi;
  if (d < -(F)kPi) return d + (F)kTwoPi;
  return d;
}

template <typename F>
__device__ __forceinline__ int steps_of(F abs_turn, F q) {
  F x = ceil(abs_turn / q - (F)kCountEps);
  return x < (F)1 ? 1 : (int)x;
}

// Simple real roots in (0,1) of A t^2 + B1 t + C, sorted, distinct.  A double
// root is not returned (it is no sign change).
template <typename F>
__device__ inline int simple_roots01(F A, F B1, F C, F r[2]) {
  int n = 0;
  F t0 = 0, t1 = 0;
  if (A == (F)0) {
    if (B1 != (F)0) { t0 = -C / B1; n = 1; }
  } else {
    F disc = B1 * B1 - 4 * A * C;
    if (disc > 0) {
      F sq = sqrt(disc);
      F qq = (F)-0.5 * (B1 + (B1 >= 0 ? sq : -sq));
      t0 = qq / A;
      t1 = C / qq;
      n = 2;
    }
  }
  // the roots inside (0,1), ascending, a repeated one once (selections only,
  // with constant indices, so the array stays in registers)
  const bool ok0 = n >= 1 && t0 > 0 && t0 < 1;
  const bool ok1 = n >= 2 && t1 > 0 && t1 < 1;
  if (ok0 && ok1) {
    r[0] = t0 < t1 ? t0 : t1;
    r[1] = t0 < t1 ? t1 : t0;
    return t0 == t1 ? 1 : 2;
  }
  r[0] = ok0 ? t0 : t1;
  return (ok0 || ok1) ? 1 : 0;
}

// a[n] = v for a run-time n, as a chain of selections over constant indices
// (a dynamically indexed private array would live in scratch memory)
template <int NMAX, typename T, typename V>
__device__ __forceinline__ void put_at(T (&a)[NMAX], int n, V v) {
#pragma unroll
  for (int m = 0; m < NMAX; ++m)
    if (m == n) a[m] = (T)v;
}

// Cubic curvature sign: g' x g'' ~ (1-t)^2 X + (1-t) t Y + t^2 Z.
template <typename F>
__device__ __forceinline__ F cubic_curv(F X, F Y, F Z, F t) {
  F u = 1 - t;
  return u * u * X + u * t * Y + t * t * Z;
}

#pragma clang fp contract(on)

// 1/x in FP64 for normal, finite x: the hardware estimate refined by two
// Newton steps (each squares the relative error), so within an ulp or two.
__device__ __forceinline__ double rcp64(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

// sqrt(x) in FP64 for x >= 0: from the hardware 1/sqrt estimate (relative
// error about 2^-23), one coupled Newton step on (sqrt x, 1/(2 sqrt x)),
// which squares it to about 2^-46, and one residual correction x - g^2,
// which leaves an error of an ulp or so.  x below 2^-960 (and 0, and
// negative x) gives 0: the uses here (squared chords in px^2, discriminants
// of tangent equations) cannot tell roots below 2^-480 from 0, and a select
// costs less than a branch to the library routine.
__device__ __forceinline__ double sqrt64(double x) {
  const bool tiny = !(x >= 0x1p-960);
  x = tiny ? 1.0 : x;
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  return tiny ? 0.0 : fma(d, h, g);
}

// sin and cos in FP64 of y + q pi/2 for |y| <= pi/4: the Taylor series of
// sin (to y^17) and cos (to y^16), whose truncation errors there are below
// 3e-18, then the quadrant q (mod 4).
__device__ __forceinline__ void sincos_quadrant(double y, int q, double* s, double* c) {
  const double z = y * y;
  double ps = 2.8114572543455206e-15;       //  1/17!
  ps = ps * z - 7.647163731819816e-13;      // -1/15!
  ps = ps * z + 1.6059043836821613e-10;     //  1/13!
  ps = ps * z - 2.505210838544172e-08;      // -1/11!
  ps = ps * z + 2.7557319223985893e-06;     //  1/9!
  ps = ps * z - 1.984126984126984e-04;      // -1/7!
  ps = ps * z + 8.333333333333333e-03;      //  1/5!
  ps = ps * z - 1.6666666666666666e-01;     // -1/3!
  const double sn = y + y * z * ps;
  double pc = 4.779477332387385e-14;        //  1/16!
  pc = pc * z - 1.1470745597729725e-11;     // -1/14!
  pc = pc * z + 2.08767569878681e-09;       //  1/12!
  pc = pc * z - 2.755731922398589e-07;      // -1/10!
  pc = pc * z + 2.48015873015873e-05;       //  1/8!
  pc = pc * z - 1.388888888888889e-03;      // -1/6!
  pc = pc * z + 4.1666666666666664e-02;     //  1/4!
  pc = pc * z - 0.5;                        // -1/2!
  const double cs = 1.0 + z * pc;
  q &= 3;
  const double s0 = (q & 1) ? cs : sn, c0 = (q & 1) ? sn : cs;
  *s = (q & 2) ? -s0 : s0;
  *c = ((q + 1) & 2) ? -c0 : c0;
}

// pi/2 in three parts, the first two of 33 significant bits, so that k P1 and
// k P2 are exact for |k| < 2^20
constexpr double kHalfPi1 = 1.5707963267341256, kHalfPi2 = 6.077100506303966e-11,
                 kHalfPi3 = 2.0222662487959506e-21;

// sin and cos of an unwrapped tangent angle in FP64 (|x| < 2^20; the angles
// here stay within a few turns): x = k pi/2 + y, |y| <= pi/4, by Cody-Waite
// reduction with the three parts of pi/2.
__device__ __forceinline__ void sincos_rd(double x, double* s, double* c) {
  const double k = rint(x * 0.6366197723675814);
  const double y = ((x - k * kHalfPi1) - k * kHalfPi2) - k * kHalfPi3;
  sincos_quadrant(y, (int)k, s, c);
}

// Table-driven sin and cos for the per-rib directions.  The table holds
// (sin, cos) of k 2pi/kSinTab, k = 0..kSinTab-1, and lives in LDS (filled once
// per workgroup by fill_sincos_tab).  x = k 2pi/kSinTab + y with 2pi/kSinTab
// split in three parts (those of pi/2 divided by kSinTab/4, a power of two),
// so |y| <= pi/kSinTab; then sin y to y^7 and cos y - 1 to y^8, whose truncation
// errors there are below 4e-19 relative, and the angle-sum identities.  Few
// coefficients, none of them large in register count, instead of the two
// degree-17 series with quadrant selection.
constexpr int kSinTab = 128;

__device__ __forceinline__ void fill_sincos_tab(double2* tab) {
  // entry k is the angle q pi/2 + m 2pi/kSinTab with q the nearest quadrant
  // and |m| <= kSinTab/8, the residual formed from the same three parts
  constexpr int kQ = kSinTab / 4;
  for (int k = threadIdx.x; k < kSinTab; k += blockDim.x) {
    const int q = (k + kQ / 2) / kQ;
    const double m = (double)(k - q * kQ);
    const double y = (m * (kHalfPi1 / kQ) + m * (kHalfPi2 / kQ)) + m * (kHalfPi3 / kQ);
    double s, c;
    sincos_quadrant(y, q, &s, &c);
    tab[k] = make_double2(s, c);
  }
}

__device__ __forceinline__ void sincos_tab(const double2* tab, double x, double* s, double* c) {
  constexpr double P1 = kHalfPi1 / (kSinTab / 4), P2 = kHalfPi2 / (kSinTab / 4),
                   P3 = kHalfPi3 / (kSinTab / 4);
  const double k = rint(x * (kSinTab / kTwoPi));
  const double y = ((x - k * P1) - k * P2) - k * P3;
  const double z = y * y;
  const double ps = (z * (1.0 / 120) - 1.0 / 6) - z * z * (1.0 / 5040);   // (sin y - y) / y^3
  const double sy = y + y * z * ps;
  const double pc = (z * (1.0 / 24) - 0.5) + z * z * (z * (1.0 / 40320) - 1.0 / 720);
  const double cm1 = z * pc;                                              // cos y - 1
  const double2 t = tab[(int)k & (kSinTab - 1)];
  *s = fma(t.y, sy, fma(t.x, cm1, t.x));
  *c = fma(-t.x, sy, fma(t.y, cm1, t.y));
}

// ===========================================================================
// Hodograph and the tangent-angle solve (Eq. angle2t), FP32 or FP64
// ===========================================================================
template <typename F>
struct Hodo {
  F e0x, e0y, e1x, e1y, e2x, e2y;
};

template <typename F, typename P>
__device__ __forceinline__ Hodo<F> hodo_of(int kind, const P* X, const P* Y, F w) {
  Hodo<F> h;
  const F ax = (F)X[1] - (F)X[0], ay = (F)Y[1] - (F)Y[0];
  if (kind == PS_KIND_CUBIC) {
    h.e0x = ax; h.e0y = ay;
    h.e1x = (F)X[2] - (F)X[1]; h.e1y = (F)Y[2] - (F)Y[1];
    h.e2x = (F)X[3] - (F)X[2]; h.e2y = (F)Y[3] - (F)Y[2];
  } else if (kind == PS_KIND_LINE) {
    h.e0x = h.e1x = h.e2x = ax; h.e0y = h.e1y = h.e2y = ay;
  } else {
    const F bx = (F)X[2] - (F)X[1], by = (F)Y[2] - (F)Y[1];
    const F ww = (kind == PS_KIND_CONIC) ? w : (F)1;
    h.e0x = ww * ax; h.e0y = ww * ay;
    h.e1x = (F)0.5 * ((F)X[2] - (F)X[0]); h.e1y = (F)0.5 * ((F)Y[2] - (F)Y[0]);
    h.e2x = ww * bx; h.e2y = ww * by;
  }
  return h;
}

template <typename F>
__device__ __forceinline__ void hodo_eval(const Hodo<F>& h, F t, F& gx, F& gy) {
  const F u = (F)1 - t;
  const F a = u * u, b = (F)2 * u * t, c = t * t;
  gx = a * h.e0x + b * h.e1x + c * h.e2x;
  gy = a * h.e0y + b * h.e1y + c * h.e2y;
}

template <typename F>
struct SolveOut {
  F t;
  bool found;   // a root inside [lo, hi] was taken (else the endpoint rule)
  F hx, hy;     // H(t)
  F dh;         // |d/dt (H(t).N)|
};

// Roots of (1-t)^2 al + 2(1-t)t be + t^2 ga = 0 inside [lo, hi]; the one whose
// gradient points along T wins (a cusp root scores 0, a reversed one < 0).
// With none inside, the paper's endpoint rule: the end with smaller |g'.N|.
template <typename F>
__device__ __forceinline__ SolveOut<F> solve_t(const Hodo<F>& h, F nx, F ny, F tx, F ty, F lo,
                                               F hi) {
  const F al = h.e0x * nx + h.e0y * ny;
  const F be = h.e1x * nx + h.e1y * ny;
  const F ga = h.e2x * nx + h.e2y * ny;
  const F A = al - (F)2 * be + ga, B1 = (F)2 * (be - al), C = al;
  F r0 = (F)-1, r1 = (F)-1;
  if (A != (F)0) {
    const F disc = B1 * B1 - (F)4 * A * C;
    if (disc >= (F)0) {
      // one reciprocal for both roots: qq/A = qq^2/(A qq), C/qq = C A/(A qq)
      // (FP32: the hardware square root and reciprocal, about 1 ulp each)
      F sq;
      if constexpr (sizeof(F) == 8) sq = sqrt64(disc);
      else sq = __builtin_amdgcn_sqrtf(disc);
      const F qq = (F)-0.5 * (B1 + (B1 >= (F)0 ? sq : -sq));
      const F aq = A * qq;
      if (aq != (F)0) {
        F inv;
        if constexpr (sizeof(F) == 8) inv = rcp64(aq);
        else inv = __builtin_amdgcn_rcpf(aq);
        r0 = qq * qq * inv;
        r1 = C * A * inv;
      } else {
        r0 = r1 = (F)0;   // qq = 0 only when B1 = C = 0: the double root t = 0
      }
    }
  } else if (B1 != (F)0) {
    r0 = r1 = -C / B1;
  }
  SolveOut<F> o;
  const bool in0 = r0 >= lo && r0 <= hi;
  const bool in1 = r1 >= lo && r1 <= hi && r1 != r0;
  o.found = in0 || in1;
  o.t = in0 ? r0 : (in1 ? r1 : hi);
  // (a wavefront skips these unless one of its lanes needs them)
  if (__ballot(in0 && in1)) {
    if (in0 && in1) {
      // two candidates: the larger score g'(t).T (r0 on a tie)
      F gx, gy;
      hodo_eval(h, r0, gx, gy);
      const F s0 = gx * tx + gy * ty;
      hodo_eval(h, r1, gx, gy);
      if (gx * tx + gy * ty > s0) o.t = r1;
    }
  }
  if (__ballot(!o.found)) {
    if (!o.found) {
      const F ul = (F)1 - lo, uh = (F)1 - hi;
      const F hl = ul * ul * al + (F)2 * ul * lo * be + lo * lo * ga;
      const F hh = uh * uh * al + (F)2 * uh * hi * be + hi * hi * ga;
      o.t = (fabs(hl) < fabs(hh)) ? lo : hi;
    }
  }
  hodo_eval(h, o.t, o.hx, o.hy);
  o.dh = fabs((F)2 * A * o.t + B1);
  return o;
}

// g(t) in FP64: cubic Bernstein, or a rational quadratic (quadratic: w = 1,
// line: middle point at the chord midpoint).
__device__ __forceinline__ void eval_point(int kind, const double* X, const double* Y, double w,
                                           double t, double& gx, double& gy) {
  const double u = 1.0 - t;
  if (kind == PS_KIND_CUBIC) {
    const double b0 = u * u * u, b1 = 3.0 * u * u * t, b2 = 3.0 * u * t * t, b3 = t * t * t;
    gx = b0 * X[0] + b1 * X[1] + b2 * X[2] + b3 * X[3];
    gy = b0 * Y[0] + b1 * Y[1] + b2 * Y[2] + b3 * Y[3];
  } else if (kind == PS_KIND_LINE) {
    gx = u * X[0] + t * X[1];
    gy = u * Y[0] + t * Y[1];
  } else {
    const double ww = (kind == PS_KIND_CONIC) ? w : 1.0;
    const double b0 = u * u, b1 = 2.0 * u * t * ww, b2 = t * t;
    const double inv = rcp64(b0 + b1 + b2);   // >= (1 + w)/2 > 0 on [0,1] for w > -1
    gx = (b0 * X[0] + b1 * X[1] + b2 * X[2]) * inv;
    gy = (b0 * Y[0] + b1 * Y[1] + b2 * Y[2]) * inv;
  }
}

}  // namespace psd
