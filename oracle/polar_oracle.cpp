// Polar stroking -- plain FP64 CPU oracle.
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
// that the GPU tessellator is checked against.  Only the test-suite, the smoke
// check and the benchmark's CPU-baseline leg may load it; the product library
// never links, calls or falls back to it, and it shares no code, header or
// table with the GPU path.
//
// Source: M. J. Kilgard, "Polar Stroking: New Theory and Methods for Stroking
// Paths", ACM TOG 39(4) art. 145, 2020.  Citations below name the paper's
// sections, equations and tables.  Every computation is FP64 on FP32 inputs,
// which are taken as exact.  No FMA contraction (build with -ffp-contract=off).
//
// Readings where the paper is silent or inconsistent (each is listed, with its
// reason, in the design notes of the repository):
//   * control points are P0..P_last in order (4 for cubic, 3 for quadratic and
//     conic, 2 for line); gradients are differences of successive points;
//   * the rib normal is n(psi) = (-sin psi, cos psi) (Sec. "Switching from Normal
//     Angle to Tangent Angle"); P = G + r_P n, N = G - r_N n;
//   * interval k spans [p_{k-1}, p_k] and turns delta_k = Psi_k (-) Psi_{k-1};
//     the short-way difference is unwrapped with the sign of curvature sigma_k
//     (a monotone interval can turn more than pi: loops and cusps);
//   * an exact cusp is not an interval boundary; the interval containing it
//     turns >= pi and is split at the half angle (Sec. "Bounding Total Curvature
//     Within Tangent Angle Intervals"); the cusp fan comes out of the root choice;
//   * every interval gets at least one step (a line is one quad, Sec.
//     "Building a Discrete Interval Range"); counts use ceil(x - 1e-9);
//   * exactly collinear segments: direction reversals ("folds") are cusps and
//     become +pi pivots at fixed t;
//   * joins/caps: the radius on the inner side of the pivot is zero; the start
//     cap pivots +pi from the reversed start tangent, the end cap pivots -pi
//     from the end tangent; an exactly antiparallel join turns +pi;
//   * arc length accumulates along the whole path, is zero across joins and
//     caps, and a step whose t decreases adds nothing (Sec. "Limitations").

#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>
#include <algorithm>

namespace {

const double kPi = 3.14159265358979323846;
const double kCountEps = 1e-9;   // ceil(x - eps): knife-edge guard for exact k*q turns
const double kUnwrapGuard = 1e-12;

enum { KIND_L = 0, KIND_Q = 1, KIND_K = 2, KIND_C = 3 };
enum { JOIN_NONE = 0, JOIN_BEVEL = 1, JOIN_ROUND = 2, JOIN_TRIANGLE = 3, JOIN_MITER = 4,
       JOIN_MITER_CLIP = 5 };
enum { CAP_BUTT = 0, CAP_ROUND = 1, CAP_SQUARE = 2, CAP_TRIANGLE = 3 };
enum { ROLE_SEGMENT = 0, ROLE_JOIN = 1, ROLE_START_CAP = 2, ROLE_END_CAP = 3 };

struct V2 { double x, y; };
V2 add(V2 a, V2 b) { return {a.x + b.x, a.y + b.y}; }
V2 sub(V2 a, V2 b) { return {a.x - b.x, a.y - b.y}; }
V2 mul(double s, V2 a) { return {s * a.x, s * a.y}; }
double dot(V2 a, V2 b) { return a.x * b.x + a.y * b.y; }
double cross(V2 a, V2 b) { return a.x * b.y - a.y * b.x; }
double len(V2 a) { return std::sqrt(a.x * a.x + a.y * a.y); }
double angle_of(V2 a) { return std::atan2(a.y, a.x); }
V2 normal_of(double psi) { return {-std::sin(psi), std::cos(psi)}; }   // n(psi)
V2 tangent_of(double psi) { return {std::cos(psi), std::sin(psi)}; }
bool nonzero(V2 a) { return a.x != 0.0 || a.y != 0.0; }
int sgn(double v) { return (v > 0) - (v < 0); }

// theta1 (-) theta2: relative angle difference (Eq. ConventionalStroking)
double angle_diff(double t1, double t2) {
  double d = t1 - t2;
  if (d > kPi) return d - 2 * kPi;
  if (d < -kPi) return d + 2 * kPi;
  return d;
}

// ---------------------------------------------------------------------------
// Segment forms and their end gradients (Table tab:path-segments)
// ---------------------------------------------------------------------------
struct Seg {
  int kind;
  int npts;
  V2 P[4];
  double w;   // conic weight w_B (K only)
};

int npts_of(int kind) { return kind == KIND_C ? 4 : (kind == KIND_L ? 2 : 3); }

// g_f(t)
V2 seg_point(const Seg& s, double t) {
  double u = 1 - t;
  switch (s.kind) {
    case KIND_L: return add(mul(u, s.P[0]), mul(t, s.P[1]));
    case KIND_Q: return add(add(mul(u * u, s.P[0]), mul(2 * u * t, s.P[1])), mul(t * t, s.P[2]));
    case KIND_K: {
      V2 num = add(add(mul(u * u, s.P[0]), mul(2 * u * t * s.w, s.P[1])), mul(t * t, s.P[2]));
      double den = u * u + 2 * u * t * s.w + t * t;
      return mul(1.0 / den, num);
    }
    default:
      return add(add(mul(u * u * u, s.P[0]), mul(3 * u * u * t, s.P[1])),
                 add(mul(3 * u * t * t, s.P[2]), mul(t * t * t, s.P[3])));
  }
}

// g'_f(t).  Bezier forms: textbook derivative.  Conic: quotient rule on the
// rational form of the table (num/den), so g' = (num' den - num den') / den^2.
V2 seg_deriv(const Seg& s, double t) {
  double u = 1 - t;
  switch (s.kind) {
    case KIND_L: return sub(s.P[1], s.P[0]);
    case KIND_Q:
      return mul(2.0, add(mul(u, sub(s.P[1], s.P[0])), mul(t, sub(s.P[2], s.P[1]))));
    case KIND_K: {
      V2 num = add(add(mul(u * u, s.P[0]), mul(2 * u * t * s.w, s.P[1])), mul(t * t, s.P[2]));
      double den = u * u + 2 * u * t * s.w + t * t;
      V2 dnum = add(add(mul(-2 * u, s.P[0]), mul(2 * s.w * (u - t), s.P[1])), mul(2 * t, s.P[2]));
      double dden = -2 * u + 2 * s.w * (u - t) + 2 * t;
      return mul(1.0 / (den * den), sub(mul(den, dnum), mul(dden, num)));
    }
    default: {
      V2 a = sub(s.P[1], s.P[0]), b = sub(s.P[2], s.P[1]), c = sub(s.P[3], s.P[2]);
      return mul(3.0, add(add(mul(u * u, a), mul(2 * u * t, b)), mul(t * t, c)));
    }
  }
}

// A segment whose control points coincide has zero length.  A conic with
// w_B = 0 reduces to the chord P0 P2 whatever P1 is (the middle term of the
// numerator and the denominator vanish together), so it has zero length when
// its end points coincide.
bool zero_length(const Seg& s) {
  if (s.kind == KIND_K && s.w == 0) return s.P[2].x == s.P[0].x && s.P[2].y == s.P[0].y;
  for (int i = 1; i < s.npts; ++i)
    if (s.P[i].x != s.P[0].x || s.P[i].y != s.P[0].y) return false;
  return true;
}

// Initial normalized gradient, by the fallbacks of the table: successive
// control points are differenced until a nonzero vector is found.
V2 grad_start(const Seg& s) {
  V2 d{0, 0};
  switch (s.kind) {
    case KIND_L: d = sub(s.P[1], s.P[0]); break;
    case KIND_Q: d = sub(s.P[1], s.P[0]); if (!nonzero(d)) d = sub(s.P[2], s.P[0]); break;
    case KIND_K:
      d = sub(s.P[1], s.P[0]);
      if (nonzero(d) && s.w != 0) d = mul(sgn(s.w), d); else d = sub(s.P[2], s.P[0]);
      break;
    default:
      d = sub(s.P[1], s.P[0]);
      if (!nonzero(d)) d = sub(s.P[2], s.P[0]);
      if (!nonzero(d)) d = sub(s.P[3], s.P[0]);
  }
  return mul(1.0 / len(d), d);
}

// Terminal normalized gradient (same table).
V2 grad_end(const Seg& s) {
  V2 d{0, 0};
  switch (s.kind) {
    case KIND_L: d = sub(s.P[1], s.P[0]); break;
    case KIND_Q: d = sub(s.P[2], s.P[1]); if (!nonzero(d)) d = sub(s.P[2], s.P[0]); break;
    case KIND_K:
      d = sub(s.P[2], s.P[1]);
      if (nonzero(d) && s.w != 0) d = mul(sgn(s.w), d); else d = sub(s.P[2], s.P[0]);
      break;
    default:
      d = sub(s.P[3], s.P[2]);
      if (!nonzero(d)) d = sub(s.P[3], s.P[1]);
      if (!nonzero(d)) d = sub(s.P[3], s.P[0]);
  }
  return mul(1.0 / len(d), d);
}

V2 end_point(const Seg& s) { return s.P[s.npts - 1]; }

// ---------------------------------------------------------------------------
// Real roots of A t^2 + B1 t + C = 0, by the numerically stable form of the
// quadratic formula (the larger-magnitude root first, the other from the
// product of roots).  Returns the number of roots written to r[].
// ---------------------------------------------------------------------------
int quad_roots(double A, double B1, double C, double r[2]) {
  if (A == 0.0) {
    if (B1 == 0.0) return 0;
    r[0] = -C / B1;
    return 1;
  }
  double disc = B1 * B1 - 4 * A * C;
  if (disc < 0) return 0;
  double sq = std::sqrt(disc);
  double qq = -0.5 * (B1 + (B1 >= 0 ? sq : -sq));
  r[0] = qq / A;
  if (qq == 0.0) return 1;   // B1 == 0 and C == 0: double root at 0
  r[1] = C / qq;
  return 2;
}

// h(t) = g'(t) . N as a power-basis quadratic A t^2 + B1 t + C (up to a
// positive factor).  Eq. angle2t: quadratic for cubics and conics (the conic
// denominator is dropped), linear for quadratics, nothing to solve for lines.
void hodo_coeffs(const Seg& s, V2 N, double* A, double* B1, double* C) {
  if (s.kind == KIND_C) {
    V2 a = sub(s.P[1], s.P[0]), b = sub(s.P[2], s.P[1]), c = sub(s.P[3], s.P[2]);
    double al = dot(a, N), be = dot(b, N), ga = dot(c, N);
    // (1-t)^2 al + 2(1-t)t be + t^2 ga
    *A = al - 2 * be + ga; *B1 = 2 * (be - al); *C = al;
  } else if (s.kind == KIND_Q) {
    V2 a = sub(s.P[1], s.P[0]), b = sub(s.P[2], s.P[1]);
    double al = dot(a, N), be = dot(b, N);
    // (1-t) al + t be
    *A = 0; *B1 = be - al; *C = al;
  } else if (s.kind == KIND_K) {
    // numerator of the conic derivative: w(1-t)^2 a + (1-t)t (P2-P0) + w t^2 b
    V2 a = sub(s.P[1], s.P[0]), b = sub(s.P[2], s.P[1]);
    double al = dot(a, N), be = dot(b, N), w = s.w;
    *A = w * al - (al + be) + w * be; *B1 = (al + be) - 2 * w * al; *C = w * al;
  } else {
    *A = 0; *B1 = 0; *C = dot(sub(s.P[1], s.P[0]), N);
  }
}

// t_[Psi_{k-1},Psi_k](psi): Eq. angle2t plus the endpoint rule that follows it.
// Among the real roots inside [lo, hi] the one whose gradient points along the
// tangent (cos psi, sin psi) is taken -- a true root scores > 0, a cusp root 0,
// a root of the reverse direction < 0.  With no root inside, the endpoint with
// the smaller |g'(t).N| is used, ties going to hi.
double solve_t(const Seg& s, double psi, double lo, double hi) {
  if (lo == hi) return lo;   // pivot at fixed t
  V2 N = normal_of(psi), T = tangent_of(psi);
  double A, B1, C;
  hodo_coeffs(s, N, &A, &B1, &C);
  double r[2];
  int n = quad_roots(A, B1, C, r);
  double best_t = 0, best_score = 0;
  bool found = false;
  for (int i = 0; i < n; ++i) {
    if (!(r[i] >= lo && r[i] <= hi)) continue;
    double score = dot(seg_deriv(s, r[i]), T);
    if (!found || score > best_score) { found = true; best_t = r[i]; best_score = score; }
  }
  if (found) return best_t;
  double hl = std::fabs(dot(seg_deriv(s, lo), N)), hh = std::fabs(dot(seg_deriv(s, hi), N));
  return hl < hh ? lo : hi;
}

// ---------------------------------------------------------------------------
// Intervals of one segment: Eqs. p-value, Psi, continuous-delta, the split of
// intervals turning >= pi, and the step counts of Eq. Delta_i.
// ---------------------------------------------------------------------------
struct Interval {
  double t0, t1;    // [p_{k-1}, p_k]; t0 == t1 for a pivot at fixed t
  double psi0;      // Psi_{k-1} (unwrapped)
  double delta;     // delta_k
  int steps;        // Delta_k
};

int step_count(double abs_delta, double q) {
  int n = (int)std::ceil(abs_delta / q - kCountEps);
  return n < 1 ? 1 : n;
}

// Rotation sense of a monotone interval: sign of g' x g'' inside it.
// For a cubic, g' x g'' is proportional to (1-t)^2 (a x b) + (1-t) t (a x c) + t^2 (b x c),
// whose sign is constant between reversal parameters except at a double root
// (an exact cusp); it is sampled at the midpoint, then the quarter points.
int rotation_sense(const Seg& s, double t0, double t1) {
  if (s.kind == KIND_C) {
    V2 a = sub(s.P[1], s.P[0]), b = sub(s.P[2], s.P[1]), c = sub(s.P[3], s.P[2]);
    const double fr[3] = {0.5, 0.25, 0.75};
    for (double f : fr) {
      double t = t0 + f * (t1 - t0), u = 1 - t;
      int sg = sgn(u * u * cross(a, b) + u * t * cross(a, c) + t * t * cross(b, c));
      if (sg != 0) return sg;
    }
    return 0;
  }
  if (s.kind == KIND_Q)
    return sgn(cross(sub(s.P[1], s.P[0]), sub(s.P[2], s.P[1])));
  if (s.kind == KIND_K) {
    // g' x g'' = 4 w_B ((P1-P0) x (P2-P1)) / D(t)^3 with D(t) > 0 for w_B > -1:
    // a negative weight turns the tangent the other way, so an external
    // ellipse runs the long way round (Sec. "Bounding Total Curvature Within
    // Tangent Angle Intervals")
    return sgn(s.w) * sgn(cross(sub(s.P[1], s.P[0]), sub(s.P[2], s.P[1])));
  }
  return 0;
}

bool exactly_collinear(const Seg& s) {
  if (s.kind == KIND_L) return true;
  if (s.kind == KIND_K && s.w == 0) return true;   // the chord P0 P2
  V2 a = sub(s.P[1], s.P[0]), b = sub(s.P[2], s.P[1]);
  if (s.kind == KIND_C) {
    V2 c = sub(s.P[3], s.P[2]);
    return cross(a, b) == 0 && cross(a, c) == 0 && cross(b, c) == 0;
  }
  return cross(a, b) == 0;
}

// Reversal parameters: simple roots in (0,1) of the curvature sign.  For a
// cubic that is the quadratic above (Loop-Blinn); quadratics, lines and conics
// with w_B > 0 have none (Sec. "The Need for Limited Tangent Angle Ranges").
std::vector<double> reversal_params(const Seg& s) {
  std::vector<double> out;
  if (s.kind != KIND_C) return out;
  V2 a = sub(s.P[1], s.P[0]), b = sub(s.P[2], s.P[1]), c = sub(s.P[3], s.P[2]);
  double X = cross(a, b), Y = cross(a, c), Z = cross(b, c);
  // X (1-t)^2 + Y (1-t) t + Z t^2 in power basis
  double A = X - Y + Z, B1 = Y - 2 * X, C = X;
  double r[2];
  int n = 0;
  if (A == 0.0) {
    if (B1 != 0.0) { r[0] = -C / B1; n = 1; }
  } else {
    double disc = B1 * B1 - 4 * A * C;
    if (disc > 0) n = quad_roots(A, B1, C, r);   // a double root is no reversal
  }
  for (int i = 0; i < n; ++i)
    if (r[i] > 0 && r[i] < 1) out.push_back(r[i]);
  std::sort(out.begin(), out.end());
  out.erase(std::unique(out.begin(), out.end()), out.end());
  return out;
}

// Simple roots in (0,1) of g'(t).d for an exactly collinear segment: the
// parameters where the segment reverses along its line (a cusp).
std::vector<double> fold_params(const Seg& s, V2 d) {
  std::vector<double> out;
  double A = 0, B1 = 0, C = 0;
  if (s.kind == KIND_C) {
    V2 a = sub(s.P[1], s.P[0]), b = sub(s.P[2], s.P[1]), c = sub(s.P[3], s.P[2]);
    double al = dot(a, d), be = dot(b, d), ga = dot(c, d);
    A = al - 2 * be + ga; B1 = 2 * (be - al); C = al;
  } else if (s.kind == KIND_Q) {
    double al = dot(sub(s.P[1], s.P[0]), d), be = dot(sub(s.P[2], s.P[1]), d);
    B1 = be - al; C = al;
  } else if (s.kind == KIND_K) {
    double al = dot(sub(s.P[1], s.P[0]), d), be = dot(sub(s.P[2], s.P[1]), d), w = s.w;
    A = w * al - (al + be) + w * be; B1 = (al + be) - 2 * w * al; C = w * al;
  } else {
    return out;
  }
  double r[2];
  int n = 0;
  if (A == 0.0) {
    if (B1 != 0.0) { r[0] = -C / B1; n = 1; }
  } else {
    double disc = B1 * B1 - 4 * A * C;
    if (disc > 0) n = quad_roots(A, B1, C, r);
  }
  for (int i = 0; i < n; ++i)
    if (r[i] > 0 && r[i] < 1) out.push_back(r[i]);
  std::sort(out.begin(), out.end());
  out.erase(std::unique(out.begin(), out.end()), out.end());
  return out;
}

std::vector<Interval> segment_intervals(const Seg& s, double q) {
  std::vector<Interval> iv;
  double psi_start = angle_of(grad_start(s));
  if (exactly_collinear(s)) {
    // Flat pieces of one step each, separated by +pi pivots at the folds.
    std::vector<double> f = fold_params(s, grad_start(s));
    double t_prev = 0, psi = psi_start;
    for (double tf : f) {
      iv.push_back({t_prev, tf, psi, 0.0, step_count(0.0, q)});
      iv.push_back({tf, tf, psi, kPi, step_count(kPi, q)});
      psi += kPi;
      t_prev = tf;
    }
    iv.push_back({t_prev, 1.0, psi, 0.0, step_count(0.0, q)});
    return iv;
  }
  // Sequences p and Psi (Eqs. p-value, Psi)
  std::vector<double> p;
  p.push_back(0.0);
  for (double r : reversal_params(s)) p.push_back(r);
  p.push_back(1.0);
  size_t M = p.size() - 1;
  std::vector<double> Psi(M + 1);
  Psi[0] = psi_start;
  for (size_t i = 1; i < M; ++i) Psi[i] = angle_of(seg_deriv(s, p[i]));
  Psi[M] = angle_of(grad_end(s));
  double psi_unwrapped = Psi[0];
  for (size_t k = 1; k <= M; ++k) {
    double d = angle_diff(Psi[k], Psi[k - 1]);   // short way
    int sigma = rotation_sense(s, p[k - 1], p[k]);
    if (sigma != 0 && d != 0 && sgn(d) != sigma && std::fabs(d) > kUnwrapGuard)
      d += 2 * kPi * sigma;                       // the long way round
    if (std::fabs(d) >= kPi) {
      // split(theta_a, theta_b): halve at the middle angle, solved for t
      double psi_s = psi_unwrapped + 0.5 * d;
      double ts = solve_t(s, psi_s, p[k - 1], p[k]);
      iv.push_back({p[k - 1], ts, psi_unwrapped, 0.5 * d, step_count(std::fabs(0.5 * d), q)});
      iv.push_back({ts, p[k], psi_s, 0.5 * d, step_count(std::fabs(0.5 * d), q)});
    } else {
      iv.push_back({p[k - 1], p[k], psi_unwrapped, d, step_count(std::fabs(d), q)});
    }
    psi_unwrapped += d;
  }
  return iv;
}

// ---------------------------------------------------------------------------
// Paths, links and the fixed link-slot layout.
//   path p with segments [b, e):  slot 2b+p      start cap
//                                 slot 2i+p+1    segment i
//                                 slot 2i+p+2    join after i (end cap if last)
// A zero-length segment has no ribs and is transparent to joins; the join slot
// after segment i joins it to the next segment with nonzero length, or holds
// the end cap when there is none.
// ---------------------------------------------------------------------------
struct Batch {
  int n_paths, n_segs;
  const int32_t* seg_begin;
  const uint8_t* kind;
  const float* cx;
  const float* cy;
  const float* conic_w;
  const float* width;
  const uint8_t* join;
  const uint8_t* cap;
  const uint8_t* closed;   // NULL: every path open
  double miter_limit;
};

bool path_closed(const Batch& B, int p) { return B.closed && B.closed[p]; }

Seg load_seg(const Batch& B, int i) {
  Seg s;
  s.kind = B.kind[i];
  s.npts = npts_of(s.kind);
  for (int k = 0; k < 4; ++k) {
    s.P[k].x = k < s.npts ? (double)B.cx[(int64_t)k * B.n_segs + i] : 0.0;
    s.P[k].y = k < s.npts ? (double)B.cy[(int64_t)k * B.n_segs + i] : 0.0;
  }
  s.w = s.kind == KIND_K ? (double)B.conic_w[i] : 1.0;
  return s;
}

// A pivot link (join or cap): ribs j = 0..J at psi0 + delta*j/J around c.
struct Pivot {
  V2 c;
  double psi0, delta;
  int J;           // 0 => no ribs
  int role;
  int cap_style;   // square caps enlarge the corner ribs
  int join_style;  // miter joins move the outer vertices of ribs 1 and 2
};

int join_steps(int style, double delta, double q) {
  if (delta == 0.0) return 0;
  switch (style) {
    case JOIN_BEVEL: return 1;
    case JOIN_TRIANGLE: return 2;
    case JOIN_ROUND: return (int)std::ceil(std::fabs(delta) / q - kCountEps);
    case JOIN_MITER:
    case JOIN_MITER_CLIP: return 3;   // Sec. "Harder Joins: Miter Truncate and Revert"
    default: return 0;
  }
}

int cap_steps(int style, double q) {
  switch (style) {
    case CAP_TRIANGLE: return 2;
    case CAP_SQUARE: return 4;
    case CAP_ROUND: return (int)std::ceil(kPi / q - kCountEps);
    default: return 0;
  }
}

// Everything one link slot contributes.
struct Link {
  int role;
  bool empty;
  int seg;                       // segment index for ROLE_SEGMENT
  std::vector<Interval> iv;      // ROLE_SEGMENT
  Pivot pv;                      // joins and caps
  double r;                      // w/2
  int ribs;
};

Link make_link(const Batch& B, int p, int slot, double q) {
  int b = B.seg_begin[p], e = B.seg_begin[p + 1];
  Link L;
  L.empty = true; L.ribs = 0; L.seg = -1; L.r = 0.5 * (double)B.width[p];
  L.role = ROLE_SEGMENT;
  int rel = slot - (2 * b + p);
  if (rel == 0) {
    // start cap of the first segment with nonzero length (closed contours
    // have none)
    L.role = ROLE_START_CAP;
    for (int i = b; i < e && !path_closed(B, p); ++i) {
      Seg s = load_seg(B, i);
      if (zero_length(s)) continue;
      int J = cap_steps(B.cap[p], q);
      double psi_s = angle_of(grad_start(s));
      L.pv = {s.P[0], psi_s - kPi, kPi, J, ROLE_START_CAP, B.cap[p], 0};
      if (J > 0) { L.empty = false; L.ribs = J + 1; }
      break;
    }
    return L;
  }
  int i = b + (rel - 1) / 2;
  Seg s = load_seg(B, i);
  if ((rel - 1) % 2 == 0) {
    L.role = ROLE_SEGMENT; L.seg = i;
    if (zero_length(s)) return L;
    L.iv = segment_intervals(s, q);
    int N = 0;
    for (const Interval& v : L.iv) N += v.steps;
    L.empty = false; L.ribs = N + 1;
    return L;
  }
  // join after segment i, or the end cap
  if (zero_length(s)) { L.role = ROLE_JOIN; return L; }
  double psi_e = angle_of(grad_end(s));
  // the next segment with nonzero length; after the last one, a closed
  // contour joins back to its first
  int next = -1;
  for (int k = i + 1; k < e && next < 0; ++k)
    if (!zero_length(load_seg(B, k))) next = k;
  for (int k = b; k <= i && next < 0 && path_closed(B, p); ++k)
    if (!zero_length(load_seg(B, k))) next = k;
  if (next >= 0) {
    double d = angle_diff(angle_of(grad_start(load_seg(B, next))), psi_e);
    if (d == -kPi) d = kPi;                   // antiparallel: turn +pi
    int J = join_steps(B.join[p], d, q);
    L.role = ROLE_JOIN;
    L.pv = {end_point(s), psi_e, d, J, ROLE_JOIN, 0, B.join[p]};
    if (J > 0) { L.empty = false; L.ribs = J + 1; }
    return L;
  }
  L.role = ROLE_END_CAP;
  int J = cap_steps(B.cap[p], q);
  L.pv = {end_point(s), psi_e, -kPi, J, ROLE_END_CAP, B.cap[p], 0};
  if (J > 0) { L.empty = false; L.ribs = J + 1; }
  return L;
}

// Miter vertex of rib j (1 or 2) of a miter join; the paper leaves its
// construction to standard stroking practice, taken here as: o0, o3 the outer
// unit normals at the two ends of the join, M = c + r (o0 + o3) / (1 + o0.o3)
// the meeting point of the two outer offset lines, miter ratio 1/cos(|delta|/2)
// (miter length over stroke width).  Within the limit both ribs take M; beyond
// it the miter either reverts to the bevel (rib 1 at c + r o0, rib 2 at
// c + r o3) or is cut square to the bisector b at distance limit * r from c
// (rib 1 on the incoming offset line, rib 2 on the outgoing one).
V2 miter_vertex(const Pivot& pv, double r, double limit, int j) {
  double sgn = pv.delta > 0 ? -1.0 : 1.0;   // outer side: -n for a left turn
  V2 o0 = {sgn * -std::sin(pv.psi0), sgn * std::cos(pv.psi0)};
  double psi3 = pv.psi0 + pv.delta;
  V2 o3 = {sgn * -std::sin(psi3), sgn * std::cos(psi3)};
  V2 sum = {o0.x + o3.x, o0.y + o3.y};
  double half_len = 0.5 * std::sqrt(sum.x * sum.x + sum.y * sum.y);   // cos(|delta| / 2)
  if (half_len * limit >= 1.0) {
    double f = r / (1.0 + (o0.x * o3.x + o0.y * o3.y));
    return {pv.c.x + f * sum.x, pv.c.y + f * sum.y};
  }
  if (pv.join_style == JOIN_MITER) {
    V2 o = j == 1 ? o0 : o3;
    return {pv.c.x + r * o.x, pv.c.y + r * o.y};
  }
  V2 t0 = {std::cos(pv.psi0), std::sin(pv.psi0)}, t3 = {std::cos(psi3), std::sin(psi3)};
  V2 bis = half_len > 0 ? V2{sum.x / (2 * half_len), sum.y / (2 * half_len)} : t0;
  double u = (limit * r - r * (o0.x * bis.x + o0.y * bis.y)) / (t0.x * bis.x + t0.y * bis.y);
  if (j == 1) return {pv.c.x + r * o0.x + u * t0.x, pv.c.y + r * o0.y + u * t0.y};
  return {pv.c.x + r * o3.x - u * t3.x, pv.c.y + r * o3.y - u * t3.y};
}

struct Out {
  double* vx; double* vy;   // [2R]: vertex 2r = N side, 2r+1 = P side
  double* vs;               // [R]  cumulative arc length per rib
  double* rib_t;            // [R]  parameter (segments) or -1 (pivots)
  double* rib_psi;          // [R]  tangent angle psi_j
  uint8_t* rib_role;        // [R]  ROLE_*
};

// Direction of g'(t) for the uniform baseline; where g' vanishes (a cusp hit
// exactly) it is taken a step of 2^-20 / N further into the segment.
V2 uniform_tangent(const Seg& s, double t, int N) {
  V2 d = seg_deriv(s, t);
  if (d.x == 0 && d.y == 0) {
    double h = std::ldexp(1.0, -20) / N;
    d = seg_deriv(s, t < 0.5 ? t + h : t - h);
  }
  return d;
}

// Emit the ribs of one path (Sec. "Complete Algorithm") with its arc length.
// uniform: the baseline of Eq. NaiveStroking sampled at t_j = j/N with the
// same rib count per segment (joins and caps unchanged).
void emit_path(const Batch& B, int p, double q, const int64_t* off, const Out& o, bool uniform) {
  int b = B.seg_begin[p], e = B.seg_begin[p + 1];
  int first = 2 * b + p, last = 2 * e + p;   // inclusive slot range
  double s_acc = 0.0;
  for (int slot = first; slot <= last; ++slot) {
    Link L = make_link(B, p, slot, q);
    if (L.empty) continue;
    int64_t r0 = off[slot];
    if (L.role == ROLE_SEGMENT) {
      Seg s = load_seg(B, L.seg);
      int j = 0;
      V2 G_prev{0, 0};
      double t_prev = 0;
      for (size_t k = 0; k < L.iv.size(); ++k) {
        const Interval& v = L.iv[k];
        int jstart = (k == 0) ? 0 : 1;   // boundary ribs are shared
        for (int i = jstart; i <= v.steps; ++i, ++j) {
          double psi, t;
          if (uniform) {
            int N = L.ribs - 1;
            t = (double)j / (double)N;
            psi = angle_of(uniform_tangent(s, t, N));
          } else if (i == 0) { psi = v.psi0; t = v.t0; }
          else if (i == v.steps) { psi = v.psi0 + v.delta; t = v.t1; }
          else {
            psi = v.psi0 + v.delta * (double)i / (double)v.steps;
            t = solve_t(s, psi, v.t0, v.t1);
          }
          V2 G = seg_point(s, t), n = normal_of(psi);
          int64_t r = r0 + j;
          o.vx[2 * r] = G.x - L.r * n.x; o.vy[2 * r] = G.y - L.r * n.y;
          o.vx[2 * r + 1] = G.x + L.r * n.x; o.vy[2 * r + 1] = G.y + L.r * n.y;
          if (j > 0 && t >= t_prev) s_acc += len(sub(G, G_prev));   // Eq. arc-length-approximation
          o.vs[r] = s_acc; o.rib_t[r] = t; o.rib_psi[r] = psi; o.rib_role[r] = ROLE_SEGMENT;
          G_prev = G; t_prev = t;
        }
      }
    } else {
      const Pivot& pv = L.pv;
      for (int j = 0; j <= pv.J; ++j) {
        double psi = pv.psi0 + pv.delta * (double)j / (double)pv.J;
        V2 n = normal_of(psi);
        double rout = L.r;
        if (pv.cap_style == CAP_SQUARE && (j == 1 || j == 3)) rout = L.r * std::sqrt(2.0);
        // only the side away from the turn keeps its radius
        double rN = pv.delta > 0 ? rout : 0.0, rP = pv.delta > 0 ? 0.0 : rout;
        int64_t r = r0 + j;
        o.vx[2 * r] = pv.c.x - rN * n.x; o.vy[2 * r] = pv.c.y - rN * n.y;
        o.vx[2 * r + 1] = pv.c.x + rP * n.x; o.vy[2 * r + 1] = pv.c.y + rP * n.y;
        if (pv.role == ROLE_JOIN && (pv.join_style == JOIN_MITER || pv.join_style == JOIN_MITER_CLIP) &&
            (j == 1 || j == 2)) {
          // the outer vertex of ribs 1 and 2 (N side of a left turn, P side
          // of a right turn) becomes the miter vertex
          V2 m = miter_vertex(pv, L.r, B.miter_limit, j);
          int k = pv.delta > 0 ? 2 * r : 2 * r + 1;
          o.vx[k] = m.x; o.vy[k] = m.y;
        }
        o.vs[r] = s_acc; o.rib_t[r] = -1.0; o.rib_psi[r] = psi; o.rib_role[r] = (uint8_t)pv.role;
      }
    }
  }
}

template <class F>
void parallel_paths(int n_paths, int nthreads, F fn) {
  if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
  if (nthreads > n_paths) nthreads = n_paths < 1 ? 1 : n_paths;
  if (nthreads <= 1) { for (int p = 0; p < n_paths; ++p) fn(p); return; }
  std::vector<std::thread> th;
  for (int w = 0; w < nthreads; ++w)
    th.emplace_back([=]() { for (int p = w; p < n_paths; p += nthreads) fn(p); });
  for (auto& t : th) t.join();
}


// ---------------------------------------------------------------------------
// Coverage of the quad strip (Sec. "Stroked Paths Tessellated to Quad
// Strips"; the support predicate, Eq. polar-stroking-predicate, taken over the
// tessellation).  A path covers a sample when any of its quads does, and a
// quad covers it when its winding number is nonzero, so both lobes of a
// bow-tie quad count and nothing between them (the quad rasterized as such,
// not as two overlapping triangles).
// ---------------------------------------------------------------------------
enum { COVER_QUAD = 0, COVER_TRIANGLES = 1 };

// Winding number of the closed polygon (x[k], y[k]), k < n, about (px, py):
// an edge going up with the point strictly to its left counts +1, an edge
// going down with the point strictly to its right counts -1; an edge counts as
// going up when it starts at or below py and ends above it (half-open).
int winding_number(const double* x, const double* y, int n, double px, double py) {
  int wn = 0;
  for (int k = 0; k < n; ++k) {
    double ux = x[k], uy = y[k], vx = x[(k + 1) % n], vy = y[(k + 1) % n];
    double side = (vx - ux) * (py - uy) - (px - ux) * (vy - uy);
    if (uy <= py) {
      if (vy > py && side > 0) ++wn;
    } else {
      if (vy <= py && side < 0) --wn;
    }
  }
  return wn;
}

// The quad between ribs r and r+1: a = N_r, b = P_r, c = P_{r+1}, d = N_{r+1}.
// COVER_TRIANGLES takes the two triangles (a, b, c) and (a, c, d) that a
// triangle rasterizer would draw instead.
bool quad_covers(const double* x, const double* y, int mode, double px, double py) {
  if (mode == COVER_QUAD) return winding_number(x, y, 4, px, py) != 0;
  double tx[3] = {x[0], x[2], x[3]}, ty[3] = {y[0], y[2], y[3]};
  return winding_number(x, y, 3, px, py) != 0 || winding_number(tx, ty, 3, px, py) != 0;
}

// Calls fn(r, p) for every quad (ribs r, r+1) of path p: consecutive ribs of
// one link, and the quad from a link's last rib to the next link's first rib
// unless both links are segments (two segments meet with no join ribs between
// them; the quad would draw a bevel where the join style asks for none).  A
// link's role follows from its slot: the start cap first, then segment, join,
// segment, ..., join or end cap.
template <class F>
void for_each_quad(const int32_t* seg_begin, const int64_t* offsets, int p, F fn) {
  int64_t first = 2 * (int64_t)seg_begin[p] + p, last = 2 * (int64_t)seg_begin[p + 1] + p;
  int64_t prev_rib = -1, prev_slot = -1;
  for (int64_t l = first; l <= last; ++l) {
    bool seg = ((l - first) & 1) == 1;
    for (int64_t r = offsets[l]; r < offsets[l + 1]; ++r) {
      if (prev_rib >= 0) {
        bool prev_seg = ((prev_slot - first) & 1) == 1;
        if (prev_slot == l || !(prev_seg && seg)) fn(prev_rib, p);
      }
      prev_rib = r; prev_slot = l;
    }
  }
}

void quad_corners(const float* vx, const float* vy, int64_t r, double* x, double* y) {
  x[0] = vx[2 * r];           y[0] = vy[2 * r];            // N_r
  x[1] = vx[2 * r + 1];       y[1] = vy[2 * r + 1];        // P_r
  x[2] = vx[2 * (r + 1) + 1]; y[2] = vy[2 * (r + 1) + 1];  // P_{r+1}
  x[3] = vx[2 * (r + 1)];     y[3] = vy[2 * (r + 1)];      // N_{r+1}
}

// Range of sample indices k (sample at o + k + 1/2, k in [0, n)) whose sample
// lies in [lo, hi]; empty when k0 > k1, and for non-finite bounds (a quad with
// a non-finite corner covers nothing).
void sample_range(double lo, double hi, double o, int n, int64_t* k0, int64_t* k1) {
  if (!std::isfinite(lo) || !std::isfinite(hi)) { *k0 = 0; *k1 = -1; return; }
  double a = std::ceil(lo - o - 0.5), b = std::floor(hi - o - 0.5);
  *k0 = (int64_t)std::max(a, 0.0);
  *k1 = (int64_t)std::min(b, (double)n - 1);
}


// A conic with w_B <= -1 has a root of its denominator in [0, 1] (at
// t = 1/2 +- sqrt((-1 - w_B) / (1 - w_B)) / 2): the curve runs through a point
// at infinity and its stroke is unbounded, so no batch may hold one.
bool weights_bounded(int n_segs, const uint8_t* kind, const float* conic_w) {
  for (int i = 0; i < n_segs; ++i)
    if (kind[i] == KIND_K && !((double)conic_w[i] > -1.0)) return false;
  return true;
}

}  // namespace

extern "C" {

int oracle_num_threads(void) { return (int)std::max(1u, std::thread::hardware_concurrency()); }

// Ribs of every link slot (Eqs. Delta_i, DeltaSigmaK; joins and caps).
int oracle_count(int n_paths, int n_segs, const int32_t* seg_begin, const uint8_t* kind,
                 const float* cx, const float* cy, const float* conic_w, const float* width,
                 const uint8_t* join, const uint8_t* cap, const uint8_t* closed, double q,
                 int32_t* link_ribs, int nthreads) {
  if (n_paths < 0 || n_segs < 0 || !(q > 0 && q <= kPi)) return -1;
  if (!weights_bounded(n_segs, kind, conic_w)) return -2;
  Batch B{n_paths, n_segs, seg_begin, kind, cx, cy, conic_w, width, join, cap, closed, 4.0};
  parallel_paths(n_paths, nthreads, [&](int p) {
    int b = seg_begin[p], e = seg_begin[p + 1];
    for (int slot = 2 * b + p; slot <= 2 * e + p; ++slot)
      link_ribs[slot] = make_link(B, p, slot, q).ribs;
  });
  return 0;
}

// Vertices, arc length and per-rib diagnostics at the offsets given
// (the exclusive prefix sum of oracle_count's output).
int oracle_emit(int n_paths, int n_segs, const int32_t* seg_begin, const uint8_t* kind,
                const float* cx, const float* cy, const float* conic_w, const float* width,
                const uint8_t* join, const uint8_t* cap, const uint8_t* closed, double miter_limit,
                double q, const int64_t* offsets, double* vx, double* vy, double* vs,
                double* rib_t, double* rib_psi, uint8_t* rib_role, int uniform, int nthreads) {
  if (n_paths < 0 || n_segs < 0 || !(q > 0 && q <= kPi) || !(miter_limit >= 1.0)) return -1;
  if (!weights_bounded(n_segs, kind, conic_w)) return -2;
  Batch B{n_paths, n_segs, seg_begin, kind, cx, cy, conic_w, width, join, cap, closed, miter_limit};
  Out o{vx, vy, vs, rib_t, rib_psi, rib_role};
  parallel_paths(n_paths, nthreads, [&](int p) { emit_path(B, p, q, offsets, o, uniform != 0); });
  return 0;
}

// Facet angles of the segment ribs of a rib stream (Sec. "Uniform Tangent
// Angle Step Tessellation": the angle where one quad meets the next).  On each
// side of a segment's strip, the facet at interior rib j (0 < j < N) is the
// angle between the boundary edges E_{j-1} = V_{j-1}V_j and E_j = V_jV_{j+1}.
// An edge E_k is regular when it is not empty and runs with the generator's
// direction of travel at both of its ribs; that direction at rib k is
// n rotated by -90 degrees, n = P_k - N_k (a rib of zero width has none).  The
// boundary inside an offset cusp reverses, so its edges are not regular; the
// paper leaves out the few facets beside such cusps, and here a facet is
// ordinary when every edge of the segment within one rib of it (E_{j-2} ..
// E_{j+1}) is regular.  Writes the count, the maximum, the sum and the sum of
// squares of the ordinary facet angles (radians) into stats[0..3].
static bool facet_edge_regular(const float* vx, const float* vy, int64_t k, int side) {
  double ex = (double)vx[2 * (k + 1) + side] - vx[2 * k + side];
  double ey = (double)vy[2 * (k + 1) + side] - vy[2 * k + side];
  if (ex == 0 && ey == 0) return false;
  for (int64_t r = k; r <= k + 1; ++r) {
    double nx = (double)vx[2 * r + 1] - vx[2 * r], ny = (double)vy[2 * r + 1] - vy[2 * r];
    if (nx == 0 && ny == 0) return false;
    // E . (n.y, -n.x) >= 0, scaled by |n|
    if (ex * ny - ey * nx < 0) return false;
  }
  return true;
}

void oracle_facet_stats(int n_paths, const int32_t* seg_begin, const int64_t* offsets,
                        const float* vx, const float* vy, double* stats) {
  double cnt = 0, mx = 0, sum = 0, sq = 0;
  for (int p = 0; p < n_paths; ++p) {
    for (int i = seg_begin[p]; i < seg_begin[p + 1]; ++i) {
      int64_t slot = 2 * (int64_t)i + p + 1;
      int64_t r0 = offsets[slot], r1 = offsets[slot + 1];
      for (int side = 0; side < 2; ++side) {
        for (int64_t r = r0 + 1; r + 1 < r1; ++r) {
          bool ordinary = true;
          for (int64_t k = std::max(r0, r - 2); k <= std::min(r1 - 2, r + 1); ++k)
            ordinary = ordinary && facet_edge_regular(vx, vy, k, side);
          if (!ordinary) continue;
          V2 a = {vx[2 * (r - 1) + side], vy[2 * (r - 1) + side]};
          V2 b = {vx[2 * r + side], vy[2 * r + side]};
          V2 c = {vx[2 * (r + 1) + side], vy[2 * (r + 1) + side]};
          V2 e1 = sub(b, a), e2 = sub(c, b);
          double ang = std::atan2(std::fabs(e1.x * e2.y - e1.y * e2.x), e1.x * e2.x + e1.y * e2.y);
          cnt += 1; sum += ang; sq += ang * ang; mx = std::max(mx, ang);
        }
      }
    }
  }
  stats[0] = cnt; stats[1] = mx; stats[2] = sum; stats[3] = sq;
}

// Per-segment intervals for inspection: writes up to cap entries of
// (t0, t1, psi0, delta, steps) and returns the interval count (0 if empty).
int oracle_segment_intervals(int kind, const double* px, const double* py, double w, double q,
                             double* t0, double* t1, double* psi0, double* delta, int32_t* steps,
                             int cap) {
  Seg s;
  s.kind = kind; s.npts = npts_of(kind); s.w = kind == KIND_K ? w : 1.0;
  if (!(s.w > -1.0)) return -1;
  for (int k = 0; k < 4; ++k) { s.P[k].x = k < s.npts ? px[k] : 0; s.P[k].y = k < s.npts ? py[k] : 0; }
  if (zero_length(s)) return 0;
  std::vector<Interval> iv = segment_intervals(s, q);
  for (size_t k = 0; k < iv.size() && (int)k < cap; ++k) {
    t0[k] = iv[k].t0; t1[k] = iv[k].t1; psi0[k] = iv[k].psi0; delta[k] = iv[k].delta;
    steps[k] = iv[k].steps;
  }
  return (int)iv.size();
}

// Dashing (Sec. "Dashing").  The rib stream of each path is split into "on"
// runs of the pattern (on0, off0, on1, off1, ...), which starts at pattern
// position `phase` at s = 0 of every path.  A pattern boundary at arc length
// s_b with s_{j-1} < s_b <= s_j inserts a rib interpolated linearly in s
// between ribs j-1 and j; steps of zero length contain no boundary.  Output
// ribs: dx/dy [2*cap_ribs] (N then P vertex), ds [cap_ribs]; dash d spans
// output ribs [range[2d], range[2d+1]).  Returns the number of output ribs
// (negative on capacity overflow); *n_dashes receives the dash count.
const int64_t kDashOutOfRange = INT64_MIN;

int64_t oracle_dash(int n_paths, const int64_t* path_rib_begin, const float* vx, const float* vy,
                    const float* vs, const double* pattern, int n_pattern, double phase,
                    double* dx, double* dy, double* ds, int64_t* range, int64_t cap_ribs,
                    int64_t cap_dashes, int64_t* n_dashes) {
  double period = 0;
  for (int i = 0; i < n_pattern; ++i) period += pattern[i];
  if (n_pattern < 2 || (n_pattern & 1) || !(period > 0)) return -1;
  // the phase is at most 2^40 periods, and a step may not end 2^50 periods or
  // more into the pattern or span more than 2^20 periods: within these bounds
  // the period count m below is exact and every boundary loop ends
  if (!(phase >= 0 && phase <= std::ldexp(period, 40))) return -1;
  std::vector<double> cum(n_pattern + 1, 0.0);
  for (int i = 0; i < n_pattern; ++i) cum[i + 1] = cum[i] + pattern[i];
  int64_t out = 0, nd = 0;
  bool overflow = false;
  auto put = [&](double nx, double ny, double px, double py, double s) {
    if (out < cap_ribs) {
      dx[2 * out] = nx; dy[2 * out] = ny; dx[2 * out + 1] = px; dy[2 * out + 1] = py; ds[out] = s;
    } else overflow = true;
    ++out;
  };
  auto open = [&]() { if (nd < cap_dashes) range[2 * nd] = out; else overflow = true; };
  auto close = [&]() { if (nd < cap_dashes) range[2 * nd + 1] = out; ++nd; };
  // pattern state at position u: "on" iff u mod period lies in an even entry
  auto state_on = [&](double u) {
    double m = std::floor(u / period);
    double x = u - m * period;
    int idx = 0;
    while (idx + 1 < n_pattern && cum[idx + 1] <= x) ++idx;
    return (idx & 1) == 0;
  };
  for (int p = 0; p < n_paths; ++p) {
    int64_t rb = path_rib_begin[p], re = path_rib_begin[p + 1];
    if (rb >= re) continue;
    bool on = state_on((double)vs[rb] + phase);
    if (on) open();
    if (on) put(vx[2 * rb], vy[2 * rb], vx[2 * rb + 1], vy[2 * rb + 1], vs[rb]);
    for (int64_t j = rb + 1; j < re; ++j) {
      double u0 = (double)vs[j - 1] + phase, u1 = (double)vs[j] + phase;
      if (u1 > u0 && !(u1 < std::ldexp(period, 50) && u1 - u0 <= std::ldexp(period, 20)))
        return kDashOutOfRange;
      if (u1 > u0) {
        // boundaries u_b = m*period + cum[i] with u0 < u_b <= u1, in order
        double m = std::floor(u0 / period);
        for (;; m += 1.0) {
          bool done = false;
          for (int i = 0; i < n_pattern; ++i) {
            double ub = m * period + cum[i];
            if (ub <= u0) continue;
            if (ub > u1) { done = true; break; }
            double lam = (ub - u0) / (u1 - u0);
            double nx = vx[2 * (j - 1)] + lam * ((double)vx[2 * j] - vx[2 * (j - 1)]);
            double ny = vy[2 * (j - 1)] + lam * ((double)vy[2 * j] - vy[2 * (j - 1)]);
            double px = vx[2 * (j - 1) + 1] + lam * ((double)vx[2 * j + 1] - vx[2 * (j - 1) + 1]);
            double py = vy[2 * (j - 1) + 1] + lam * ((double)vy[2 * j + 1] - vy[2 * (j - 1) + 1]);
            double sb = ub - phase;
            if (on) { put(nx, ny, px, py, sb); close(); on = false; }
            else { open(); put(nx, ny, px, py, sb); on = true; }
          }
          if (done) break;
        }
      }
      if (on) put(vx[2 * j], vy[2 * j], vx[2 * j + 1], vy[2 * j + 1], vs[j]);
    }
    if (on) close();
  }
  *n_dashes = nd;
  return overflow ? -out : out;
}

// Topmost covering path per sample of a W x H canvas (sample of pixel (i, j)
// at (x0 + i + 1/2, y0 + j + 1/2)): top[j*W + i] = the largest path index
// whose quads cover the sample, -1 where none does (a renderer drawing opaque
// strokes in path order shows that path there).
void oracle_coverage(int n_paths, const int32_t* seg_begin, const int64_t* offsets,
                     const float* vx, const float* vy, double x0, double y0, int W, int H,
                     int mode, int32_t* top) {
  for (int64_t k = 0; k < (int64_t)W * H; ++k) top[k] = -1;
  for (int p = 0; p < n_paths; ++p) {
    for_each_quad(seg_begin, offsets, p, [&](int64_t r, int pp) {
      double x[4], y[4];
      quad_corners(vx, vy, r, x, y);
      double xl = std::min(std::min(x[0], x[1]), std::min(x[2], x[3]));
      double xh = std::max(std::max(x[0], x[1]), std::max(x[2], x[3]));
      double yl = std::min(std::min(y[0], y[1]), std::min(y[2], y[3]));
      double yh = std::max(std::max(y[0], y[1]), std::max(y[2], y[3]));
      int64_t i0, i1, j0, j1;
      sample_range(xl, xh, x0, W, &i0, &i1);
      sample_range(yl, yh, y0, H, &j0, &j1);
      for (int64_t j = j0; j <= j1; ++j)
        for (int64_t i = i0; i <= i1; ++i)
          if (quad_covers(x, y, mode, x0 + i + 0.5, y0 + j + 0.5))
            top[j * W + i] = std::max(top[j * W + i], (int32_t)pp);
    });
  }
}

// The same value for single samples (pixel (pi[k], pj[k]) of the same canvas),
// each from every quad of every path: for checking a large canvas at a few
// points.
void oracle_coverage_at(int n_paths, const int32_t* seg_begin, const int64_t* offsets,
                        const float* vx, const float* vy, double x0, double y0, int mode,
                        int n_pts, const int32_t* pi, const int32_t* pj, int32_t* out,
                        int nthreads) {
  parallel_paths(n_pts, nthreads, [&](int k) {
    double px = x0 + pi[k] + 0.5, py = y0 + pj[k] + 0.5;
    int32_t best = -1;
    for (int p = n_paths - 1; p >= 0 && best < 0; --p) {
      for_each_quad(seg_begin, offsets, p, [&](int64_t r, int pp) {
        if (best >= pp) return;
        double x[4], y[4];
        quad_corners(vx, vy, r, x, y);
        if (px < std::min(std::min(x[0], x[1]), std::min(x[2], x[3])) ||
            px > std::max(std::max(x[0], x[1]), std::max(x[2], x[3])) ||
            py < std::min(std::min(y[0], y[1]), std::min(y[2], y[3])) ||
            py > std::max(std::max(y[0], y[1]), std::max(y[2], y[3])))
          return;
        if (quad_covers(x, y, mode, px, py)) best = pp;
      });
    }
    out[k] = best;
  });
}

}  // extern "C"
