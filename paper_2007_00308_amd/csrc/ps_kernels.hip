// Polar-stroking kernels for gfx950 (MI355X) and the host side of the C ABI.
//
// Method: Kilgard, "Polar Stroking", ACM TOG 2020.
//   count  one thread per segment: FP64 interval setup, a-priori step counts,
//          the join or end cap after the segment; one thread per path: the
//          start cap
//   scan   3-phase exclusive scan of int32 counts into int64 offsets
//   emit   persistent wavefront tiles of 64*K - 1 ribs taken in ticket order;
//          per rib: link lookup, tangent angle, t solve (FP32, FP32 with an
//          FP64 fix-up, or FP64), FP64 point evaluation, coalesced stores;
//          the chord-sum arc length is scanned inside the tile and carried
//          between tiles by a decoupled look-back on fixed-point sums, so the
//          result does not depend on scheduling
//   dash   per-rib boundary counts, two scans, emission of the "on" pieces
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ps_device.h"

using namespace psd;

#define PS_VERSION "0.2.0"

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;                        // items per thread
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096 items per block
constexpr int kMinTileRibs = 64 * 1 - 1;              // smallest emit tile (K = 1)
constexpr double kFix = 4294967296.0;                 // arc length in fixed point: 2^-32 px
constexpr unsigned long long kValMask = (1ull << 62) - 1;
constexpr int kMaxDash = 64;
constexpr double kMaxDashPhase = 1099511627776.0;      // 2^40 periods

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ===========================================================================
// Workspace
// ===========================================================================
struct WsLayout {
  size_t status, rec_head, rec_tail, seg_ang, seg_ok, scan, tile_link, desc, dash_r, dash_d, dash_rpos, dash_dpos,
      dash_scan, total;
  int64_t max_tiles, n_links, max_ribs, nb_links, nb_ribs;
};

// Offsets of the workspace parts.  Status, records and the link-scan scratch
// come first and depend only on the batch, so ps_count and ps_scan (which are
// not told the vertex capacity) carve the same prefix as ps_emit.
WsLayout ws_layout(int64_t n_links, int64_t vertex_capacity, int n_dash) {
  WsLayout w;
  w.n_links = n_links;
  w.max_ribs = vertex_capacity / 2;
  w.max_tiles = w.max_ribs / kMinTileRibs + 2;
  w.nb_links = (n_links + kScanTile - 1) / kScanTile + 1;
  w.nb_ribs = (w.max_ribs + kScanTile - 1) / kScanTile + 1;
  size_t o = 0;
  w.status = o; o = align_up(o + 256, 256);
  w.rec_head = o; o = align_up(o + (size_t)n_links * kHeadPieces * 16, 256);
  w.rec_tail = o; o = align_up(o + (size_t)n_links * kTailPieces * 16, 256);
  w.seg_ang = o; o = align_up(o + (size_t)n_links * 16, 256);   // n_links >= n_segs
  w.seg_ok = o; o = align_up(o + (size_t)n_links, 256);
  w.scan = o; o = align_up(o + (size_t)(w.nb_links + 1) * 8, 256);
  w.tile_link = o; o = align_up(o + (size_t)(w.max_tiles + 1) * 4, 256);
  w.desc = o; o = align_up(o + (size_t)w.max_tiles * 8, 256);
  w.dash_r = w.dash_d = w.dash_rpos = w.dash_dpos = w.dash_scan = o;
  if (n_dash > 0) {
    w.dash_r = o; o = align_up(o + (size_t)(w.max_ribs + 1) * 4, 256);
    w.dash_d = o; o = align_up(o + (size_t)(w.max_ribs + 1) * 4, 256);
    w.dash_rpos = o; o = align_up(o + (size_t)(w.max_ribs + 1) * 8, 256);
    w.dash_dpos = o; o = align_up(o + (size_t)(w.max_ribs + 1) * 8, 256);
    w.dash_scan = o; o = align_up(o + (size_t)(w.nb_ribs + 1) * 8, 256);
  }
  w.total = o;
  return w;
}

// ===========================================================================
// Count (Eqs. p-value, Psi, continuous-delta, Delta_i; joins and caps)
// ===========================================================================
struct CountArgs {
  ps_batch B;
  double q;
  int32_t* link_ribs;
  v4u32* head;   // record heads, kHeadPieces per link slot
  v4u32* tail;   // record tails, kTailPieces per link slot
  double2* seg_ang;
  uint8_t* seg_ok;
  DevStatus* st;
  unsigned long long* scan_desc;   // look-back words of the one-pass link scan, cleared here
  int64_t scan_nb;
};

__device__ __forceinline__ void set_flag(DevStatus* st, unsigned f) { atomicOr(&st->flags, f); }

__device__ __forceinline__ void reset_status(DevStatus* st) {
  st->flags = 0; st->total_ribs = 0; st->fixups = 0; st->dash_ribs = 0; st->dash_count = 0;
  st->tile_counter = 0; st->dash_tile_counter = 0; st->scan_ticket = 0;
}

// largest p in [a, b] with seg_begin[p] <= i, given seg_begin[a] <= i
__device__ __forceinline__ int path_in(const int32_t* seg_begin, int a, int b, int i) {
  while (a < b) {
    const int m = (a + b + 1) >> 1;
    if (seg_begin[m] <= i) a = m; else b = m - 1;
  }
  return a;
}

__device__ __forceinline__ int path_of_seg(const int32_t* seg_begin, int n_paths, int i) {
  // largest p with seg_begin[p] <= i (the path that owns segment i)
  return path_in(seg_begin, 0, n_paths - 1, i);
}

// A segment contributes ribs if its values are finite and valid and it is
// not a single point (a zero-length segment strokes nothing).
// Segment states: usable, or the status bit its problem raises (the count
// kernel raises it, so the angles pass, which runs first, may reset the
// status word).
constexpr uint8_t kSegUsable = 1, kSegBadValue = 2, kSegNonFinite = 4;
__device__ inline uint8_t seg_state(const ps_batch& B, int i) {
  const int k = B.kind[i];
  if (k > PS_KIND_CUBIC) return kSegBadValue;
  const Seg s = load_seg(B, i);
  if (!seg_finite(s)) return kSegNonFinite;
  // w_B <= -1 puts a root of the conic's denominator in [0,1]: the curve runs
  // through a point at infinity and its stroke is unbounded
  if (k == PS_KIND_CONIC && !(s.w > -1.0)) return kSegBadValue;
  return seg_is_point(s) ? 0 : kSegUsable;
}

#pragma clang fp contract(off)

// Intervals split at their middle angle (at most two per segment): the
// interval index, the angle and the parameter range of the solve that gives
// the split's parameter.  The solve runs after the record is stored (nothing
// else depends on it), so its registers are never live beside the record's.
template <typename F>
struct SplitSolves {
  int n = 0, idx0 = 0, idx1 = 0;
  F psi0 = 0, psi1 = 0, lo0 = 0, lo1 = 0, hi0 = 0, hi1 = 0;
};

// Intervals of one usable segment, written into rec, from its start and end
// tangent angles.  Returns the step count N (the segment has N+1 ribs), or -1
// if it needs more than kMaxIv intervals.  The parameters of split intervals
// are left to finish_splits.  F is the arithmetic: double, or float for the
// single-precision study mode.
template <typename F>
__device__ int segment_setup(const ps_batch& B, int i, F q, F psi_start, F psi_end,
                             LinkRec& rec, SplitSolves<F>& sp, DevStatus* st) {
  const SegT<F> s = load_seg<F>(B, i);
  float X[4], Y[4];
  const int64_t S = B.n_segs;
  for (int k = 0; k < 4; ++k) {
    const int kk = k < s.npts ? k : s.npts - 1;
    X[k] = B.cx[kk * S + i];
    Y[k] = B.cy[kk * S + i];
  }
  F sx, sy;
  start_dir(s, sx, sy);
  const F psi0 = psi_start;   // unit_angle(sx, sy), computed by the angles kernel
  const F ax = s.x[1] - s.x[0], ay = s.y[1] - s.y[0];
  const F bx = s.x[2] - s.x[1], by = s.y[2] - s.y[1];
  const F cx = s.x[3] - s.x[2], cy = s.y[3] - s.y[2];
  bool collinear;
  F X3 = 0, Y3 = 0, Z3 = 0;
  if (s.kind == PS_KIND_LINE) {
    collinear = true;
  } else if (s.kind == PS_KIND_CUBIC) {
    X3 = crs(ax, ay, bx, by); Y3 = crs(ax, ay, cx, cy); Z3 = crs(bx, by, cx, cy);
    collinear = (X3 == 0 && Y3 == 0 && Z3 == 0);
  } else {
    // a conic of weight 0 is the chord P0 P2
    collinear = crs(ax, ay, bx, by) == 0 || (s.kind == PS_KIND_CONIC && s.w == 0);
  }

  // interval n gets dsum[n], its end parameter p[n] and end angle psi[n+1];
  // loops run to their constant maxima so every private array keeps constant
  // indices (and stays in registers)
  int n = 0, N = 0;
  F psi_run = psi0;
  rec.psi[0] = psi0;
  if (collinear) {
    // flat pieces of one step, split by +pi pivots at the simple roots of
    // g'(t).d where the segment reverses along its line (a cusp)
    const F inv = (F)1 / sqrt(sx * sx + sy * sy);
    const F dx = inv * sx, dy = inv * sy;
    F A = 0, B1 = 0, C = 0;
    if (s.kind == PS_KIND_CUBIC) {
      const F al = ax * dx + ay * dy, be = bx * dx + by * dy, ga = cx * dx + cy * dy;
      A = al - 2 * be + ga; B1 = 2 * (be - al); C = al;
    } else if (s.kind == PS_KIND_QUAD) {
      const F al = ax * dx + ay * dy, be = bx * dx + by * dy;
      B1 = be - al; C = al;
    } else if (s.kind == PS_KIND_CONIC) {
      const F al = ax * dx + ay * dy, be = bx * dx + by * dy, w = s.w;
      A = w * al - (al + be) + w * be; B1 = (al + be) - 2 * w * al; C = w * al;
    }
    F f[2] = {0, 0};
    const int nf = (s.kind == PS_KIND_LINE) ? 0 : simple_roots01(A, B1, C, f);
    const int flat = steps_of((F)0, q), fold = steps_of((F)kPi, q);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (k < nf) {
        N += flat; put_at(rec.dsum, n, N); put_at(rec.p, n, f[k]); put_at(rec.psi, n + 1, psi_run); ++n;
        N += fold; put_at(rec.dsum, n, N); put_at(rec.p, n, f[k]);
        psi_run = psi_run + (F)kPi; put_at(rec.psi, n + 1, psi_run); ++n;
      }
    }
    N += flat; put_at(rec.dsum, n, N); put_at(rec.psi, n + 1, psi_run); ++n;
    rec.n_iv = (uint8_t)n;
    return N;
  }

  // reversal parameters: simple roots of the cubic curvature sign;
  // pr[0..M] = 0, the roots, 1 (M <= 3)
  F pr[4] = {0, 1, 1, 1};
  int M = 1;
  if (s.kind == PS_KIND_CUBIC) {
    F r[2] = {0, 0};
    const int nr = simple_roots01(X3 - Y3 + Z3, Y3 - 2 * X3, X3, r);
    M = 1 + nr;
    pr[1] = nr >= 1 ? r[0] : (F)1;
    pr[2] = nr >= 2 ? r[1] : (F)1;
  }
  F Psi[4];
  Psi[0] = psi0;
#pragma unroll
  for (int k = 1; k < 3; ++k) {
    const F t = pr[k], u = 1 - t;
    const F gx = u * u * ax + 2 * u * t * bx + t * t * cx;
    const F gy = u * u * ay + 2 * u * t * by + t * t * cy;
    Psi[k] = (k < M) ? atan2(gy, gx) : (F)0;
  }
  put_at(Psi, M, psi_end);
  const F crsQ = crs(ax, ay, bx, by);
#pragma unroll
  for (int k = 1; k <= 3; ++k) {
    if (k > M) break;
    F d = adiff(Psi[k], Psi[k - 1]);   // the short way round
    F sigma = 0;                       // rotation sense of the interval
    if (s.kind == PS_KIND_CUBIC) {
      // the middle of the interval, then its quarter points (an exact cusp
      // makes the curvature vanish at a single point)
      const F w = pr[k] - pr[k - 1];
      sigma = sgn(cubic_curv(X3, Y3, Z3, pr[k - 1] + (F)0.5 * w));
      if (sigma == 0) sigma = sgn(cubic_curv(X3, Y3, Z3, pr[k - 1] + (F)0.25 * w));
      if (sigma == 0) sigma = sgn(cubic_curv(X3, Y3, Z3, pr[k - 1] + (F)0.75 * w));
    } else {
      // conics: g' x g'' = 4 w_B (a x b) / D^3 with D > 0, so a negative
      // weight (an external ellipse) turns the other way, the long way round
      sigma = sgn(crsQ) * (s.kind == PS_KIND_CONIC ? sgn(s.w) : (F)1);
    }
    if (sigma != 0 && d != 0 && sgn(d) != sigma && fabs(d) > (F)kUnwrapGuard) d += (F)kTwoPi * sigma;
    if (fabs(d) >= (F)kPi) {
      if (n + 2 > kMaxIv) { set_flag(st, PS_STATUS_INTERVALS); rec.n_iv = 0; return -1; }
      // split at the middle angle
      const F psi_s = psi_run + (F)0.5 * d;
      if (sp.n == 0) { sp.idx0 = n; sp.psi0 = psi_s; sp.lo0 = pr[k - 1]; sp.hi0 = pr[k]; }
      else { sp.idx1 = n; sp.psi1 = psi_s; sp.lo1 = pr[k - 1]; sp.hi1 = pr[k]; }
      ++sp.n;
      const int half = steps_of(fabs((F)0.5 * d), q);
      N += half; put_at(rec.dsum, n, N); put_at(rec.psi, n + 1, psi_s); ++n;
      N += half; put_at(rec.dsum, n, N); if (k < M) put_at(rec.p, n, pr[k]);
      psi_run = psi_s + (F)0.5 * d; put_at(rec.psi, n + 1, psi_run); ++n;
    } else {
      if (n + 1 > kMaxIv) { set_flag(st, PS_STATUS_INTERVALS); rec.n_iv = 0; return -1; }
      N += steps_of(fabs(d), q); put_at(rec.dsum, n, N); if (k < M) put_at(rec.p, n, pr[k]);
      psi_run = psi_run + d; put_at(rec.psi, n + 1, psi_run); ++n;
    }
  }
  rec.n_iv = (uint8_t)n;
  return N;
}

// The parameter of each split interval of segment i: the solve (in F) at its
// middle angle, stored into the interval boundaries p_1..p_4 (at pt) of the
// record already written.
template <typename F>
__device__ void finish_splits(const ps_batch& B, int i, const SplitSolves<F>& sp, double* pt) {
  const SegT<F> s = load_seg<F>(B, i);
  float X[4], Y[4];
  const int64_t S = B.n_segs;
  for (int k = 0; k < 4; ++k) {
    const int kk = k < s.npts ? k : s.npts - 1;
    X[k] = B.cx[kk * S + i];
    Y[k] = B.cy[kk * S + i];
  }
  const Hodo<F> h = hodo_of<F>(s.kind, X, Y, s.w);
  for (int m = 0; m < sp.n; ++m) {
    F sn, cs;
    if constexpr (sizeof(F) == 8) sincos(m ? sp.psi1 : sp.psi0, &sn, &cs);
    else sincosf(m ? sp.psi1 : sp.psi0, &sn, &cs);
    const SolveOut<F> so = solve_t<F>(h, -sn, cs, cs, sn, m ? sp.lo1 : sp.lo0, m ? sp.hi1 : sp.hi0);
    pt[m ? sp.idx1 : sp.idx0] = (double)so.t;
  }
}

template <typename F>
__device__ int join_steps(int style, F delta, F q) {
  if (delta == 0) return 0;
  if (style == PS_JOIN_BEVEL) return 1;
  if (style == PS_JOIN_TRIANGLE) return 2;
  if (style == PS_JOIN_MITER || style == PS_JOIN_MITER_CLIP) return 3;   // Sec. "Harder Joins"
  if (style == PS_JOIN_ROUND) {
    const F x = ceil(fabs(delta) / q - (F)kCountEps);
    return x < 0 ? 0 : (int)x;
  }
  return 0;
}

template <typename F>
__device__ int cap_steps(int style, F q) {
  if (style == PS_CAP_TRIANGLE) return 2;
  if (style == PS_CAP_SQUARE) return 4;
  if (style == PS_CAP_ROUND) return (int)ceil((F)kPi / q - (F)kCountEps);
  return 0;
}

// The state of segment k (decided on the exact inputs), and for a usable
// one its start and end tangent angles in F (Eq. Psi at t = 0 and 1, through
// the end gradients and their fallbacks).
template <typename F>
__device__ inline void seg_angles(const ps_batch& B, int k, uint8_t& state, double2& ang) {
  state = seg_state(B, k);
  ang = make_double2(0.0, 0.0);
  if (state & kSegUsable) {
    const SegT<F> s = load_seg<F>(B, k);
    F sx, sy, ex, ey;
    start_dir(s, sx, sy);
    end_dir(s, ex, ey);
    ang.x = (double)unit_angle(sx, sy);
    ang.y = (double)unit_angle(ex, ey);
  }
}

// First count pass, one thread per segment: its state and its start and
// end tangent angles.  The chain's first kernel, so its first thread resets
// the status word (problems found here are raised by the count kernel).
template <typename F>
__global__ void __launch_bounds__(256) count_angles_kernel(CountArgs A) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) reset_status(A.st);
  if (i >= A.B.n_segs) return;
  uint8_t state;
  double2 ang;
  seg_angles<F>(A.B, (int)i, state, ang);
  A.seg_ang[i] = ang;
  A.seg_ok[i] = state;
}

#pragma clang fp contract(on)

__device__ inline void clear_rec(LinkRec& r) {
  r.role = ROLE_EMPTY; r.n_iv = 0; r.kind = 0; r.flags = 0; r.r = 0; r.w = 1;
  for (int k = 0; k < kMaxIv; ++k) r.dsum[k] = INT_MAX;   // past the last interval
  for (int k = 0; k < 4; ++k) { r.x[k] = 0; r.y[k] = 0; }
  for (int k = 0; k < kMaxIv - 1; ++k) r.p[k] = 0;
  for (int k = 0; k <= kMaxIv; ++k) r.psi[k] = 0;
}

// A pivot link (join or cap) with J steps from psi0 through psi1 = psi0 + delta;
// `cap` is the cap style of a cap and the join style of a join.
__device__ inline LinkRec make_pivot(uint8_t role, double psi0, double psi1, int J, float px, float py,
                                     uint8_t cap, float half_w, bool first) {
  LinkRec r;
  clear_rec(r);
  r.role = J > 0 ? role : (uint8_t)ROLE_EMPTY;
  r.n_iv = 1;
  r.flags = (uint8_t)((cap << 4) | ((first && J > 0) ? kFirstInPath : 0));
  r.r = half_w;
  r.dsum[0] = J; r.psi[0] = psi0; r.psi[1] = psi1;
  r.x[0] = px; r.y[0] = py;
  if (J > 0 && role == ROLE_JOIN && (cap == PS_JOIN_MITER || cap == PS_JOIN_MITER_CLIP)) {
    // unit normals n = (-sin, cos) at both ends, for the miter vertices
    double s0, c0, s1, c1;
    sincos(psi0, &s0, &c0);
    sincos(psi1, &s1, &c1);
    r.p[0] = -s0; r.p[1] = c0; r.p[2] = -s1; r.p[3] = c1;
    r.flags |= kHasTail;
  }
  return r;
}

// The record heads of a count workgroup's link slots are gathered in LDS and
// written to memory with consecutive lanes on consecutive 16-byte pieces (the
// lanes of a wavefront hold segments of one form, scattered over the
// workgroup's links, so one store instruction from the threads that built
// the records would write 64 pieces far apart: a memory request each).  Stage
// position 0 is link slot sb = 2 i0 + p0 (i0: the workgroup's first segment,
// p0 its path); the workgroup's links come after it, with the start caps of
// any paths without segments in between, which the path threads write.  A
// slot past the stage is written directly.
constexpr int kCountThreads = 256;
constexpr int kStageSlots = 576;   // 2 x 256 segment and pivot links, and up to 64 start caps (36 KB)

struct HeadStage {
  v4u32* lds;        // kStageSlots x kHeadPieces
  int* ribs;         // kStageSlots rib counts
  unsigned* valid;   // a bit per stage slot: written by this workgroup
  int64_t sb;
};

// Record r of link slot `slot` with `ribs` ribs: its head and rib count into
// the stage (or to memory), its tail (if it has one) to memory.
__device__ __forceinline__ void put_rec(const CountArgs& A, const HeadStage& hs, int64_t slot,
                                        const LinkRec& r, int ribs) {
  v4u32 pc[kRecPieces];
  __builtin_memcpy(pc, &r, sizeof(LinkRec));
  const int64_t rel = slot - hs.sb;
  if (rel >= 0 && rel < kStageSlots) {
#pragma unroll
    for (int k = 0; k < kHeadPieces; ++k) hs.lds[rel * kHeadPieces + k] = pc[head_piece(k)];
    hs.ribs[rel] = ribs;
    atomicOr(&hs.valid[rel >> 5], 1u << (rel & 31));
  } else {
    v4u32* h = A.head + slot * kHeadPieces;
#pragma unroll
    for (int k = 0; k < kHeadPieces; ++k) h[k] = pc[head_piece(k)];
    A.link_ribs[slot] = ribs;
  }
  if (r.flags & kHasTail) {
    v4u32* t = A.tail + slot * kTailPieces;
    t[0] = pc[tail_piece(0)]; t[1] = pc[tail_piece(1)]; t[3] = pc[tail_piece(3)];
    if (tail_whole(r)) { t[2] = pc[tail_piece(2)]; t[4] = pc[tail_piece(4)]; }
  }
}

// p_1..p_4 of the tail of link slot `slot`
__device__ __forceinline__ double* tail_p(const CountArgs& A, int64_t slot) {
  return reinterpret_cast<double*>(A.tail + slot * kTailPieces + 3);
}

// The start cap of path p (segments b..e-1, b < e): from the reversed start
// tangent of its first usable segment, +pi round to it; none on a closed
// contour, a path of bad width or style, or one without usable segments.
template <typename F>
__device__ LinkRec start_cap(const CountArgs& A, int p, int b, int e, int& ribs) {
  const ps_batch& B = A.B;
  const float wd = B.width[p];
  const bool ok = isfinite(wd) && wd > 0 && B.cap[p] <= PS_CAP_TRIANGLE && B.join[p] <= PS_JOIN_MITER_CLIP;
  ribs = 0;
  if (ok && !(B.closed && B.closed[p])) {
    for (int k = b; k < e; ++k) {
      if (!(A.seg_ok[k] & kSegUsable)) continue;
      const F q = (F)A.q;
      const int J = cap_steps<F>(B.cap[p], q);
      const F c0 = (F)A.seg_ang[k].x - (F)kPi;
      ribs = J > 0 ? J + 1 : 0;
      return make_pivot(ROLE_SCAP, c0, c0 + (F)kPi, J, B.cx[k], B.cy[k], B.cap[p], 0.5f * wd, true);
    }
  }
  return make_pivot(ROLE_SCAP, 0, 0, 0, 0, 0, 0, 0.5f * wd, false);
}

// The links of segment i: its own record and step count (Eqs. p-value, Psi,
// continuous-delta, Delta_i), the join or end cap after it, and the start cap
// of its path when it is the path's first segment.  Link slots: path p's
// start cap at 2 b + p, segment i at 2 i + p + 1, the link after it at
// 2 i + p + 2 (b: the path's first segment).
template <typename F>
__device__ void count_segment(const CountArgs& A, const HeadStage& hs, int i, int p_lo, int p_hi) {
  const ps_batch& B = A.B;
  const int S = B.n_segs;
  const uint8_t state = A.seg_ok[i];
  if (state & kSegBadValue) set_flag(A.st, PS_STATUS_BAD_VALUE);
  if (state & kSegNonFinite) set_flag(A.st, PS_STATUS_NONFINITE);
  const bool ok_i = state & kSegUsable;
  const double2 ang = A.seg_ang[i];   // F values
  const int p = path_in(B.seg_begin, p_lo, p_hi, i);
  const int b = B.seg_begin[p], e = B.seg_begin[p + 1];
  const int64_t slot = 2 * (int64_t)i + p + 1;
  const float wd = B.width[p];
  const bool wok = isfinite(wd) && wd > 0;
  const bool sok = (B.join[p] <= PS_JOIN_MITER_CLIP) && (B.cap[p] <= PS_CAP_TRIANGLE);
  const bool closed = B.closed && B.closed[p];
  if (!isfinite(wd)) set_flag(A.st, PS_STATUS_NONFINITE);
  else if (!wok || !sok) set_flag(A.st, PS_STATUS_BAD_VALUE);
  const bool usable = wok && sok && ok_i;
  const float half_w = 0.5f * wd;
  const F q = (F)A.q;
  const F psi_e = (F)ang.y;
  {
    LinkRec r;
    clear_rec(r);
    r.kind = B.kind[i];
    r.r = half_w;
    int ribs = 0;
    SplitSolves<F> sp;
    if (usable) {
      const int N = segment_setup<F>(B, i, q, (F)ang.x, psi_e, r, sp, A.st);
      if (N > 0) {
        ribs = N + 1;
        r.role = ROLE_SEG;
        if (r.n_iv > 1) r.flags |= kHasTail;
        const int npts = npts_of(r.kind);
        for (int k = 0; k < 4; ++k) {
          const int kk = k < npts ? k : npts - 1;
          r.x[k] = B.cx[(int64_t)kk * S + i];
          r.y[k] = B.cy[(int64_t)kk * S + i];
        }
        r.w = (r.kind == PS_KIND_CONIC) ? B.conic_w[i] : 1.0f;
        // the first segment with ribs of the path (no usable segment before
        // it), and the first link with ribs (also no start cap ribs)
        bool first_seg = true;
        for (int k = i - 1; first_seg && k >= b; --k) first_seg = !(A.seg_ok[k] & kSegUsable);
        if (first_seg) r.flags |= kFirstSegInPath;
        if (first_seg && (closed || cap_steps<F>(B.cap[p], q) == 0)) r.flags |= kFirstInPath;
      }
    }
    put_rec(A, hs, slot, r, ribs);
    if (sp.n > 0 && ribs > 0) finish_splits<F>(B, i, sp, tail_p(A, slot));
  }
  if (i == b) {
    int ribs;
    const LinkRec c = start_cap<F>(A, p, b, e, ribs);
    put_rec(A, hs, slot - 1, c, ribs);
  }
  // the join after this segment, or the end cap
  const int64_t jslot = slot + 1;
  LinkRec pv;
  int J = 0;
  if (usable) {
    const int n = npts_of(B.kind[i]);
    const float ex = B.cx[(int64_t)(n - 1) * S + i], ey = B.cy[(int64_t)(n - 1) * S + i];
    // the next usable segment; after the last one a closed contour joins
    // back to its first
    int next = -1;
    for (int k = i + 1; k < e && next < 0; ++k)
      if (A.seg_ok[k] & kSegUsable) next = k;
    for (int k = b; k <= i && next < 0 && closed; ++k)
      if (A.seg_ok[k] & kSegUsable) next = k;
    if (next >= 0) {
      F d = adiff((F)A.seg_ang[next].x, psi_e);
      if (d == -(F)kPi) d = (F)kPi;   // antiparallel: turn +pi
      J = join_steps<F>(B.join[p], d, q);
      pv = make_pivot(ROLE_JOIN, psi_e, psi_e + d, J, ex, ey, B.join[p], half_w, false);
    } else {
      J = cap_steps<F>(B.cap[p], q);
      pv = make_pivot(ROLE_ECAP, psi_e, psi_e - (F)kPi, J, ex, ey, B.cap[p], half_w, false);
    }
  } else {
    pv = make_pivot(ROLE_JOIN, 0, 0, 0, 0, 0, 0, half_w, false);
  }
  put_rec(A, hs, jslot, pv, J > 0 ? J + 1 : 0);
}

// Second count pass.  Workgroups of 256 segments (each thread writes the
// links of one segment, count_segment), then workgroups of paths, whose
// threads write the start cap of each path without segments.
template <typename F>
__global__ void __launch_bounds__(kCountThreads) count_kernel(CountArgs A) {
  const ps_batch& B = A.B;
  const int64_t tid = (int64_t)blockIdx.x * kCountThreads + threadIdx.x;
  const int S = B.n_segs, P = B.n_paths;
  if (tid < A.scan_nb) A.scan_desc[tid] = 0ull;   // scan_nb <= S + P threads
  const int seg_blocks = (S + kCountThreads - 1) / kCountThreads;
  if ((int)blockIdx.x >= seg_blocks) {
    const int64_t pt = tid - (int64_t)seg_blocks * kCountThreads;
    if (pt < P) {
      const int p = (int)pt;
      const int b = B.seg_begin[p];
      if (b == B.seg_begin[p + 1]) {
        const LinkRec c = make_pivot(ROLE_SCAP, 0, 0, 0, 0, 0, 0, 0.5f * B.width[p], false);
        v4u32 pc[kRecPieces];
        __builtin_memcpy(pc, &c, sizeof(LinkRec));
        const int64_t slot = 2 * (int64_t)b + p;
        for (int k = 0; k < kHeadPieces; ++k) A.head[slot * kHeadPieces + k] = pc[head_piece(k)];
        A.link_ribs[slot] = 0;
      }
    }
    return;
  }
  __shared__ v4u32 stage[kStageSlots * kHeadPieces];
  __shared__ int stage_ribs[kStageSlots];
  __shared__ unsigned stage_valid[kStageSlots / 32];
  __shared__ int stage_p[2];   // the paths of the workgroup's first and last segments
  // The workgroup's segments are handed to its threads grouped by form
  // (unusable, line, quadratic, conic, cubic), so that a wavefront mostly
  // runs one form's setup instead of all of them one after another.  Which
  // thread takes a segment changes nothing in what is written.
  __shared__ int form_count[8];
  __shared__ int form_order[kCountThreads];
  const int i0 = (int)blockIdx.x * kCountThreads;
  const int nseg = S - i0 < kCountThreads ? S - i0 : kCountThreads;
  if (threadIdx.x < 8) form_count[threadIdx.x] = 0;
  if (threadIdx.x < kStageSlots / 32) stage_valid[threadIdx.x] = 0;
  if (threadIdx.x < 2) stage_p[threadIdx.x] = path_of_seg(B.seg_begin, P, threadIdx.x ? i0 + nseg - 1 : i0);
  __syncthreads();
  int form = -1, rank = 0;
  if ((int)threadIdx.x < nseg) {
    const int k = B.kind[i0 + threadIdx.x];
    form = !(A.seg_ok[i0 + threadIdx.x] & kSegUsable) ? 0
         : (k == PS_KIND_CUBIC ? 4 : (k == PS_KIND_CONIC ? 3 : (k == PS_KIND_QUAD ? 2 : 1)));
    rank = atomicAdd(&form_count[form], 1);
  }
  __syncthreads();
  if (form >= 0) {
    int at = rank;
    for (int f = 0; f < form; ++f) at += form_count[f];
    form_order[at] = (int)threadIdx.x;
  }
  __syncthreads();
  HeadStage hs;
  hs.lds = stage;
  hs.ribs = stage_ribs;
  hs.valid = stage_valid;
  hs.sb = 2 * (int64_t)i0 + stage_p[0];
  if ((int)threadIdx.x < nseg) count_segment<F>(A, hs, i0 + form_order[threadIdx.x], stage_p[0], stage_p[1]);
  __syncthreads();
  v4u32* const out = A.head + hs.sb * kHeadPieces;
  for (int c = threadIdx.x; c < kStageSlots * kHeadPieces; c += kCountThreads) {
    const int rel = c / kHeadPieces;
    if (stage_valid[rel >> 5] & (1u << (rel & 31))) out[c] = stage[c];
  }
  for (int rel = threadIdx.x; rel < kStageSlots; rel += kCountThreads)
    if (stage_valid[rel >> 5] & (1u << (rel & 31))) A.link_ribs[hs.sb + rel] = stage_ribs[rel];
}

// Scratch memory of ps_stroke_static: the workspace of one count -> scan ->
// emit chain, for callers that cannot allocate.  Every GPU the library runs
// on holds its own copy until the process ends.  Host code never uses this
// name for memory: it takes the array's device address from
// hipGetSymbolAddress, once per device.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

__global__ void copy_status_flags_kernel(const DevStatus* st, uint32_t* out) {
  if (threadIdx.x == 0) *out = st->flags;
}

__global__ void reset_status_kernel(DevStatus* st) {
  if (threadIdx.x == 0) reset_status(st);
}

// ===========================================================================
// Scan
// ===========================================================================
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// Exclusive scan of one value per thread across a block of kScanThreads.
__device__ __forceinline__ long long block_excl_scan(long long v, long long* total) {
  __shared__ long long wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long incl = wave_incl_scan(v);
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  long long base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kScanThreads / 64; ++k) {
    const long long s = wsum[k];
    if (k < wv) base += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

// The item count is n_max, or min(*n_dev, n_max) when n_dev is given (a
// length produced on the device, such as the rib total).
__device__ __forceinline__ int64_t scan_len(int64_t n_max, const int64_t* n_dev) {
  if (!n_dev) return n_max;
  const int64_t n = *n_dev;
  return n < n_max ? n : n_max;
}

template <typename TIn>
__global__ void __launch_bounds__(kScanThreads) scan_reduce_kernel(const TIn* in, int64_t n_max,
                                                                   const int64_t* n_dev,
                                                                   long long* block_sums) {
  const int64_t n = scan_len(n_max, n_dev);
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  long long s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < n) s += (long long)in[i];
  }
  long long tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) scan_blocks_kernel(long long* block_sums, int64_t nb) {
  __shared__ long long wsum[16];
  __shared__ long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
    const int64_t i = c0 + threadIdx.x;
    const long long v = i < nb ? block_sums[i] : 0;
    const long long incl = wave_incl_scan(v);
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    long long base = carry, tot = 0;
    for (int k = 0; k < 16; ++k) {
      if (k < wv) base += wsum[k];
      tot += wsum[k];
    }
    if (i < nb) block_sums[i] = base + incl - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) block_sums[nb] = carry;
}

template <typename TIn>
__global__ void __launch_bounds__(kScanThreads) scan_apply_kernel(const TIn* in, int64_t n_max,
                                                                  const int64_t* n_dev,
                                                                  const long long* block_sums,
                                                                  int64_t* out, int64_t nb,
                                                                  unsigned long long* total_out) {
  const int64_t n = scan_len(n_max, n_dev);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    out[n] = block_sums[nb];
    if (total_out) *total_out = (unsigned long long)block_sums[nb];
  }
  if ((int64_t)blockIdx.x * kScanTile >= n) return;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  long long v[kScanItems];
  long long s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    v[k] = i < n ? (long long)in[i] : 0;
    s += v[k];
  }
  long long tot;
  long long ex = block_excl_scan(s, &tot) + block_sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = ex;
    ex += v[k];
  }
}

// Look-back words are published with a device-scope atomic swap and read
// with device-scope relaxed atomic loads.  At device scope both reach the
// point where the XCDs' L2 caches are coherent, so a word published on one
// XCD is seen on every other one without whole-cache write-backs or
// invalidations (which release/acquire ordering would add per tile); the
// data the words describe needs no ordering with them.
__device__ __forceinline__ void desc_publish(unsigned long long* p, unsigned long long w) {
  (void)__hip_atomic_exchange(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long desc_read(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The sum of the values of look-back words before word `first` (exclusive of
// it) up to the nearest inclusive one, read by one wavefront.  Word: 2 state
// bits (0 not ready, 1 the unit's own sum, 2 the sum of everything up to and
// including the unit) and 62 value bits.  The first read takes the 16 words
// before `first` (one 128-byte line; the nearest inclusive word is usually
// among them), later ones 64 at a time: these reads are device-coherent, so
// they go past the XCD's L2, and reading 64 words per try made up about half
// of the emit's reads.  Without `block`, gives up (returns false) when a
// needed word is not ready.
__device__ __forceinline__ bool look_back(const unsigned long long* desc, int64_t first, bool block,
                                          unsigned long long& prefix) {
  const int lane = threadIdx.x & 63;
  int64_t bT = first - 1;
  int span = 16;
  prefix = 0;
  for (;;) {
    const int64_t Ti = bT - lane;
    // lanes past this read's span act as empty aggregates
    unsigned long long wd = 1ull << 62;
    if (lane < span) wd = Ti >= 0 ? desc_read(&desc[Ti]) : (2ull << 62);
    const unsigned stt = (unsigned)(wd >> 62);
    const unsigned long long incl = __ballot(stt == 2);
    const int stop = incl ? __builtin_ctzll(incl) : 64;   // nearest inclusive word
    const unsigned long long upto = stop >= 63 ? ~0ull : ((2ull << stop) - 1);
    if (__ballot(stt == 0) & upto) {
      if (!block) return false;
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    unsigned long long v = lane <= stop ? (wd & kValMask) : 0ull;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    prefix += v;
    if (stop < 64) return true;
    bT -= span;
    span = 64;
  }
}

// The link-rib scan in one pass: blocks of kLinkScanTile links take tickets in
// order, publish their sums and look back for their prefixes, so each link's
// offset is written once with no second pass.  With TS > 0 it also writes
// the tile table of an emit of TS-rib tiles (the tile_link entries and
// cleared look-back words that emit_prepare_kernel writes): each link writes
// the tiles whose first-read rib it holds, so the table needs no total.  The
// thread that owns position n_links writes offset[n_links] = R, the rib
// total, and the emit's overflow flag.  The look-back words (one per block)
// and the ticket are cleared by the count kernel and the status reset.
// 256 threads of 16 links per block (measured on the 4096-path batch, 166
// blocks: 11.3 us; 1024-thread blocks, whose look-backs all end within one
// 64-word read, 14.8 us: fewer blocks leave most CUs idle)
constexpr int kLinkScanThreads = 256;
constexpr int kLinkScanTile = kLinkScanThreads * kScanItems;
// the workspace holds ceil(L / kScanTile) + 1 look-back words for the link
// scan (WsLayout::nb_links), which covers its L / kLinkScanTile + 1 blocks
// only if its blocks are no smaller
static_assert(kLinkScanTile >= kScanTile, "link scan blocks must cover at least kScanTile links");

struct LinkScanArgs {
  const int32_t* link_ribs;
  int64_t n;
  int64_t* off;
  unsigned long long* desc;
  DevStatus* st;
  int TS;
  int32_t* tile_link;
  unsigned long long* tile_desc;
  int64_t capacity, max_tiles;
};

// floor(a / d) for 0 <= a < 2^52 and 0 < d < 2^20 from an FP64 estimate and
// one correction each way (a 64-bit integer division is a long sequence)
__device__ __forceinline__ int64_t div_small(int64_t a, int64_t d, double inv_d) {
  int64_t q = (int64_t)((double)a * inv_d);
  q -= (q * d > a) ? 1 : 0;
  q += ((q + 1) * d <= a) ? 1 : 0;
  return q;
}

__global__ void __launch_bounds__(kLinkScanThreads) link_scan_kernel(LinkScanArgs A) {
  __shared__ unsigned int blk_sh;
  __shared__ long long wsum[kLinkScanThreads / 64];
  __shared__ long long pre_sh;
  if (threadIdx.x == 0) blk_sh = (unsigned)atomicAdd(&A.st->scan_ticket, 1ull);
  __syncthreads();
  const int64_t blk = blk_sh;
  const int64_t n = A.n;
  const int64_t i0 = blk * kLinkScanTile + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  long long s = 0;
  if (i0 + kScanItems <= n && ((uintptr_t)A.link_ribs & 15) == 0) {
    const int4* src = reinterpret_cast<const int4*>(A.link_ribs + i0);
#pragma unroll
    for (int c = 0; c < kScanItems / 4; ++c) {
      const int4 q = src[c];
      v[4 * c] = q.x; v[4 * c + 1] = q.y; v[4 * c + 2] = q.z; v[4 * c + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) v[k] = i0 + k < n ? A.link_ribs[i0 + k] : 0;
  }
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) s += v[k];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long incl = wave_incl_scan(s);
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  long long before = 0, total = 0;
#pragma unroll
  for (int k = 0; k < kLinkScanThreads / 64; ++k) {
    before += k < wv ? wsum[k] : 0;
    total += wsum[k];
  }
  if (wv == 0) {
    unsigned long long prefix = 0;
    if (blk > 0) {
      if (lane == 0) desc_publish(&A.desc[blk], (1ull << 62) | ((unsigned long long)total & kValMask));
      look_back(A.desc, blk, true, prefix);
    }
    if (lane == 0) {
      desc_publish(&A.desc[blk], (2ull << 62) | ((prefix + (unsigned long long)total) & kValMask));
      pre_sh = (long long)prefix;
    }
  }
  __syncthreads();
  const long long ex0 = pre_sh + before + incl - s;
  // offsets: 16-byte stores when the thread's 16 items are whole and aligned
  if (i0 + kScanItems <= n && ((uintptr_t)(A.off + i0) & 15) == 0) {
    long long e = ex0;
    longlong2* dst = reinterpret_cast<longlong2*>(A.off + i0);
#pragma unroll
    for (int c = 0; c < kScanItems / 2; ++c) {
      longlong2 w;
      w.x = e; e += v[2 * c];
      w.y = e; e += v[2 * c + 1];
      dst[c] = w;
    }
  } else {
    long long e = ex0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      if (i0 + k < n) A.off[i0 + k] = e;
      e += v[k];
    }
  }
  if (i0 <= n && n < i0 + kScanItems) {
    // the thread that owns position n: the total, and the emit's flags
    long long e = ex0;
    for (int k = 0; k < kScanItems; ++k) e += (i0 + k < n) ? v[k] : 0;
    A.off[n] = e;
    A.st->total_ribs = (unsigned long long)e;
    if (A.TS > 0) {
      const int64_t n_tiles = (e + A.TS - 1) / A.TS;
      if (e == 0) A.tile_link[0] = 0;
      A.st->tile_counter = 0;
      atomicAnd(&A.st->flags, ~(unsigned)PS_STATUS_OVERFLOW);
      if (2 * e > A.capacity || n_tiles > A.max_tiles) atomicOr(&A.st->flags, (unsigned)PS_STATUS_OVERFLOW);
    }
  }
  if (A.TS > 0) {
    // the tile table: tile T (T >= 1) first reads rib T*TS - 1, held by the
    // link [a, b) with T*TS in [a + 1, b]; tile 0 by the first link with
    // ribs.  The thread walks its links with the next tile start past its
    // first offset (one division per thread).
    const int64_t TS = A.TS;
    int64_t T = div_small(ex0, TS, 1.0 / (double)TS) + 1;
    int64_t next = T * TS;
    long long a = ex0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t i = i0 + k;
      const long long b = a + v[k];
      if (i < n && v[k] > 0) {
        if (a == 0) {
          A.tile_link[0] = (int32_t)i;
          A.tile_desc[0] = 0ull;
        }
        while (next <= b && T <= A.max_tiles) {
          A.tile_link[T] = (int32_t)i;
          if (T < A.max_tiles) A.tile_desc[T] = 0ull;
          ++T;
          next += TS;
        }
      }
      a = b;
    }
  }
}

// ===========================================================================
// Emit (Eqs. func_t, func_N, RibVertices-N/P, arc-length-approximation)
// ===========================================================================
struct EmitArgs {
  const v4u32* head;   // record heads and tails (LinkRec)
  const v4u32* tail;
  const int64_t* off;
  int64_t n_links;
  float* vx;
  float* vy;
  float* vs;
  int64_t capacity;
  const int32_t* tile_link;
  unsigned long long* desc;
  DevStatus* st;
  int64_t max_tiles;
  float fix_tol;   // largest FP64 Newton step accepted on an FP32 root; beyond it the rib is re-solved in FP64
  double miter_limit;
};

// Tile T stores ribs [T*TS, (T+1)*TS) and also reads rib T*TS - 1.  Writes the
// link holding each tile's first-read rib, clears the look-back descriptors
// and the tile ticket.
__global__ void __launch_bounds__(256) emit_prepare_kernel(const int64_t* off, int64_t n_links,
                                                           int TS, int32_t* tile_link,
                                                           unsigned long long* desc,
                                                           DevStatus* st, int64_t capacity,
                                                           int64_t max_tiles) {
  const int64_t R = off[n_links];
  const int64_t n_tiles = (R + TS - 1) / TS;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // each emit reports its own overflow (cleared and set by the same thread)
  if (tid == 0) {
    st->tile_counter = 0;
    atomicAnd(&st->flags, ~(unsigned)PS_STATUS_OVERFLOW);
  }
  if (2 * R > capacity || n_tiles > max_tiles) {
    if (tid == 0) atomicOr(&st->flags, (unsigned)PS_STATUS_OVERFLOW);
    return;
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t T = tid; T < n_tiles; T += stride) desc[T] = 0ull;
  if (R == 0) {
    if (tid == 0) tile_link[0] = 0;
    return;
  }
  // tile T (0 <= T <= n_tiles, the last one a sentinel) first reads rib
  // f(T) = clamp(T*TS - 1, 0, R - 1); each link with ribs [a, b) writes the
  // tiles whose f(T) it holds: T*TS in [a+1, b], plus T = 0 for the link
  // holding rib 0 and the sentinel for the one holding rib R - 1
  for (int64_t l = tid; l < n_links; l += stride) {
    const int64_t a = off[l], b = off[l + 1];
    if (a >= b) continue;
    const int64_t t0 = (a == 0) ? 0 : (a + TS) / TS;
    const int64_t t1 = (b == R) ? n_tiles : b / TS;
    for (int64_t T = t0; T <= t1; ++T) tile_link[T] = (int32_t)l;
  }
}

// One rib: its centre G and parameter t (segments), its two vertices, and
// for the FP32 + FP64 fix-up mode whether it was re-solved in FP64.
struct RibOut {
  double gx, gy, t;
  float Nx, Ny, Px, Py;
  bool fixed;
};

// The interval k holding a segment rib j, Delta_Sigma(k-1) <= j <=
// Delta_Sigma(k): its boundary ribs d0 < d1, the tangent angles psa, psb and
// the parameters lo, hi at them.
struct RibIval {
  int d0, d1;
  double psa, psb, lo, hi;
};

// For a record held per lane (in LDS): k - 1 is the number of boundaries j
// has passed (dsum increases strictly and holds INT_MAX past the last
// interval), counted without a chain of dependent reads; the interval's data
// are then read by index.
__device__ __forceinline__ RibIval rib_ival(const LinkRec& rp, int j) {
  int k1 = 0;
#pragma unroll
  for (int m = 0; m < kMaxIv - 1; ++m) k1 += (j > rp.dsum[m]) ? 1 : 0;
  RibIval v;
  v.d0 = k1 ? rp.dsum[k1 - 1] : 0;
  v.d1 = rp.dsum[k1];
  v.psa = rp.psi[k1];
  v.psb = rp.psi[k1 + 1];
  v.lo = k1 ? rp.p[k1 - 1] : 0.0;
  v.hi = (k1 + 1 < (int)rp.n_iv) ? rp.p[k1 < kMaxIv - 2 ? k1 : kMaxIv - 2] : 1.0;
  return v;
}

// For a record every lane shares (in scalar registers): selections over the
// record's n_iv intervals, a wavefront-uniform count, so a one-interval
// segment selects nothing.
__device__ __forceinline__ RibIval rib_ival_uniform(const LinkRec& rp, int j) {
  const int n_iv = rp.n_iv;
  RibIval v;
  v.d0 = 0; v.d1 = rp.dsum[0];
  v.psa = rp.psi[0]; v.psb = rp.psi[1];
  v.lo = 0.0; v.hi = n_iv > 1 ? rp.p[0] : 1.0;
#pragma unroll
  for (int m = 1; m < kMaxIv; ++m) {
    if (m < n_iv) {
      const bool past = j > rp.dsum[m - 1];
      const double hi_m = (m + 1 < n_iv) ? rp.p[m < kMaxIv - 1 ? m : 0] : 1.0;
      v.d0 = past ? rp.dsum[m - 1] : v.d0;
      v.d1 = past ? rp.dsum[m] : v.d1;
      v.psa = past ? rp.psi[m] : v.psa;
      v.psb = past ? rp.psi[m + 1] : v.psb;
      v.lo = past ? rp.p[m - 1] : v.lo;
      v.hi = past ? hi_m : v.hi;
    }
  }
  return v;
}

// sin and cos in FP32 from an LDS table of kSinTab (sin, cos) pairs: x =
// k 2pi/kSinTab + y with |y| <= pi/kSinTab, sin y to y^3 and cos y - 1 to y^4
// (truncation below 4e-10 relative, under the FP32 rounding), then the
// angle-sum identities.  2pi/kSinTab is split in two floats, the first of 12
// significant bits, so that k times it is exact for |x| up to 200 (the
// unwrapped angles here stay within a few turns).
constexpr float kTab32Hi = 0.04907226562f;                    // 2pi/128 to 12 bits
constexpr float kTab32Lo = (float)(kTwoPi / kSinTab - 0.04907226562);
__device__ __forceinline__ void fill_sincos_tab32(float2* tab, const double2* tab64) {
  for (int k = threadIdx.x; k < kSinTab; k += blockDim.x) tab[k] = make_float2((float)tab64[k].x, (float)tab64[k].y);
}
__device__ __forceinline__ void sincos_tab32(const float2* tab, float x, float* s, float* c) {
  const float k = rintf(x * (float)(kSinTab / kTwoPi));
  const float y = fmaf(-k, kTab32Lo, fmaf(-k, kTab32Hi, x));
  const float z = y * y;
  const float sy = fmaf(y * z, -1.0f / 6, y);
  const float cm1 = z * fmaf(z, 1.0f / 24, -0.5f);
  const float2 t = tab[(int)k & (kSinTab - 1)];
  *s = fmaf(t.y, sy, fmaf(t.x, cm1, t.x));
  *c = fmaf(-t.x, sy, fmaf(t.y, cm1, t.y));
}

// The same from the FP64 table, its entries rounded to FP32 as they are read.
__device__ __forceinline__ void sincos_tab32d(const double2* tab, float x, float* s, float* c) {
  const float k = rintf(x * (float)(kSinTab / kTwoPi));
  const float y = fmaf(-k, kTab32Lo, fmaf(-k, kTab32Hi, x));
  const float z = y * y;
  const float sy = fmaf(y * z, -1.0f / 6, y);
  const float cm1 = z * fmaf(z, 1.0f / 24, -0.5f);
  const double2 t = tab[(int)k & (kSinTab - 1)];
  const float tx = (float)t.x, ty = (float)t.y;
  *s = fmaf(ty, sy, fmaf(tx, cm1, tx));
  *c = fmaf(-tx, sy, fmaf(ty, cm1, ty));
}

// g(t) in FP32 (the single-precision mode), relative to P0: the Bernstein
// weights of the other points times their offsets from P0, added to P0 once
// at the end, so only that last addition rounds at the size of the
// coordinates.
__device__ __forceinline__ void eval_point32(int kind, const float* X, const float* Y, float w, float t,
                                             float& gx, float& gy) {
  const float u = 1.0f - t;
  const float x1 = X[1] - X[0], y1 = Y[1] - Y[0];
  float ox, oy;
  if (kind == PS_KIND_CUBIC) {
    const float b1 = 3.0f * u * u * t, b2 = 3.0f * u * t * t, b3 = t * t * t;
    ox = b1 * x1 + b2 * (X[2] - X[0]) + b3 * (X[3] - X[0]);
    oy = b1 * y1 + b2 * (Y[2] - Y[0]) + b3 * (Y[3] - Y[0]);
  } else if (kind == PS_KIND_LINE) {
    ox = t * x1;
    oy = t * y1;
  } else {
    const float ww = (kind == PS_KIND_CONIC) ? w : 1.0f;
    const float b1 = 2.0f * u * t * ww, b2 = t * t;
    const float inv = __builtin_amdgcn_rcpf(u * u + b1 + b2);
    ox = (b1 * x1 + b2 * (X[2] - X[0])) * inv;
    oy = (b1 * y1 + b2 * (Y[2] - Y[0])) * inv;
  }
  gx = X[0] + ox;
  gy = Y[0] + oy;
}

// The parameter of an interior segment rib in FP64: the root of h(t).n = 0
// (Eq. angle2t; h is the hodograph in Bernstein form, a positive multiple of
// g') inside [lo, hi], by the rules of solve_t: with two roots inside, the
// one whose h points along T = (n.y, -n.x) (r0 on a tie); with none, the end
// with the smaller |h.n|.  Written for the emit's lanes: quadratics (A = 0,
// the equation linear) take the same instructions as cubics (qq = -B, and
// r1 = C/qq is the root), one reciprocal serves both roots (r0 = qq/A =
// qq^2/(A qq), r1 = C/qq = C A/(A qq)), and a zero or negative discriminant
// or a zero denominator gives roots that no interval holds.
__device__ __forceinline__ double emit_solve64(const Hodo<double>& h, double nx, double ny, double lo,
                                               double hi) {
  const double al = h.e0x * nx + h.e0y * ny;
  const double be = h.e1x * nx + h.e1y * ny;
  const double ga = h.e2x * nx + h.e2y * ny;
  const double A = al - 2.0 * be + ga, B = 2.0 * (be - al), C = al;
  const bool quad = A == 0.0;
  const double disc = fma(B, B, -4.0 * A * C);
  const double sq = quad ? fabs(B) : sqrt64(disc);   // sqrt64 gives 0 below 2^-960
  const double qq = -0.5 * (B + (B >= 0.0 ? sq : -sq));
  const double inv = rcp64(quad ? qq : A * qq);
  const bool real = disc >= 0.0;
  const double r1 = real ? (quad ? C : C * A) * inv : -1.0;
  const double r0 = real ? (quad ? r1 : qq * qq * inv) : -1.0;
  const bool in0 = r0 >= lo && r0 <= hi;
  const bool in1 = r1 >= lo && r1 <= hi && r1 != r0;
  double t = in0 ? r0 : (in1 ? r1 : hi);
  if (__ballot(in0 && in1)) {
    // scores h(t).T in power form: T-components of the Bernstein coefficients
    const double tx = ny, ty = -nx;
    const double a0 = h.e0x * tx + h.e0y * ty, b0 = h.e1x * tx + h.e1y * ty, c0 = h.e2x * tx + h.e2y * ty;
    const double aT = a0 - 2.0 * b0 + c0, bT = 2.0 * (b0 - a0);
    const double s0 = fma(fma(aT, r0, bT), r0, a0), s1 = fma(fma(aT, r1, bT), r1, a0);
    if (in0 && in1 && s1 > s0) t = r1;
  }
  if (__ballot(!(in0 || in1))) {
    const double hl = fma(fma(A, lo, B), lo, C), hh = fma(fma(A, hi, B), hi, C);
    if (!(in0 || in1)) t = (fabs(hl) < fabs(hh)) ? lo : hi;
  }
  return t;
}

// The same isolation in FP32 (the hardware square root and reciprocal) for
// the fix-up mode, whose FP64 Newton step then polishes the root: the root
// chosen by the rules of emit_solve64, and `found` false when no root lies
// in [lo, hi] (the rib then goes to the FP64 solve, which applies the end
// rule).
__device__ __forceinline__ float emit_solve32(const Hodo<float>& h, float nx, float ny, float lo, float hi,
                                              bool& found) {
  const float al = h.e0x * nx + h.e0y * ny;
  const float be = h.e1x * nx + h.e1y * ny;
  const float ga = h.e2x * nx + h.e2y * ny;
  const float A = al - 2.0f * be + ga, B = 2.0f * (be - al), C = al;
  const bool quad = A == 0.0f;
  const float disc = fmaf(B, B, -4.0f * A * C);
  const bool real = disc >= 0.0f;
  const float sq = quad ? fabsf(B) : __builtin_amdgcn_sqrtf(real ? disc : 0.0f);
  const float qq = -0.5f * (B + (B >= 0.0f ? sq : -sq));
  const float inv = __builtin_amdgcn_rcpf(quad ? qq : A * qq);
  const float r1 = real ? (quad ? C : C * A) * inv : -1.0f;
  const float r0 = real ? (quad ? r1 : qq * qq * inv) : -1.0f;
  const bool in0 = r0 >= lo && r0 <= hi;
  const bool in1 = r1 >= lo && r1 <= hi && r1 != r0;
  float t = in0 ? r0 : r1;
  if (__ballot(in0 && in1)) {
    const float tx = ny, ty = -nx;
    const float a0 = h.e0x * tx + h.e0y * ty, b0 = h.e1x * tx + h.e1y * ty, c0 = h.e2x * tx + h.e2y * ty;
    const float aT = a0 - 2.0f * b0 + c0, bT = 2.0f * (b0 - a0);
    const float s0 = fmaf(fmaf(aT, r0, bT), r0, a0), s1 = fmaf(fmaf(aT, r1, bT), r1, a0);
    if (in0 && in1 && s1 > s0) t = r1;
  }
  found = in0 || in1;
  return t;
}

// Segment rib j of interval v (Eqs. func_t, func_N): the tangent angle
// psi_j = psi_{k-1} + (j - Delta_Sigma(k-1)) delta_k / Delta_k (the boundary
// angles exactly at the interval ends), n(psi) = (-sin psi, cos psi), t from
// the tangent-angle solve (Eq. angle2t) on the interior ribs, G = g(t) and
// the vertices N = G - r n, P = G + r n (Eqs. RibVertices-N/P).  PREC picks
// the arithmetic (PS_PREC_*): FP64 throughout; FP32 throughout (the direction
// from an FP32 table, the solve and the point in FP32); or an FP32 solve that
// one FP64 Newton step polishes, with the rib re-solved in FP64 when that step
// is not small.
template <int PREC>
__device__ __forceinline__ void seg_rib(const LinkRec& rp, int j, const RibIval& v, float fix_tol,
                                        const double2* tab, const float2* tab32, RibOut& o) {
  const bool at0 = j == v.d0, at1 = j == v.d1;
  const bool solve = !at0 && !at1 && v.lo != v.hi;
  const int kind = rp.kind;
  o.fixed = false;
  float X[4], Y[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) { X[i] = rp.x[i]; Y[i] = rp.y[i]; }
  if constexpr (PREC == PS_PREC_FP32) {
    const float psa = (float)v.psa, psb = (float)v.psb;
    const float psi = at0 ? psa
                    : (at1 ? psb
                           : fmaf(psb - psa, (float)(j - v.d0) * __builtin_amdgcn_rcpf((float)(v.d1 - v.d0)), psa));
    float sn, cs;
    sincos_tab32(tab32, psi, &sn, &cs);
    const float nx = -sn, ny = cs;
    float t = at1 ? (float)v.hi : (float)v.lo;
    if (solve) {
      const Hodo<float> h = hodo_of<float>(kind, X, Y, rp.w);
      t = solve_t<float>(h, nx, ny, ny, -nx, (float)v.lo, (float)v.hi).t;
    }
    float gx, gy;
    eval_point32(kind, X, Y, rp.w, t, gx, gy);
    const float r = rp.r;
    o.gx = gx; o.gy = gy; o.t = t;
    o.Nx = fmaf(-r, nx, gx); o.Ny = fmaf(-r, ny, gy);
    o.Px = fmaf(r, nx, gx); o.Py = fmaf(r, ny, gy);
  } else {
    const double psi =
        at0 ? v.psa : (at1 ? v.psb : v.psa + (v.psb - v.psa) * ((double)(j - v.d0) * rcp64((double)(v.d1 - v.d0))));
    double sn, cs;
    sincos_tab(tab, psi, &sn, &cs);
    const double nx = -sn, ny = cs;
    double Xd[4], Yd[4];   // the FP32 inputs, converted once (exactly)
#pragma unroll
    for (int i = 0; i < 4; ++i) { Xd[i] = (double)X[i]; Yd[i] = (double)Y[i]; }
    double t = at1 ? v.hi : v.lo;
    if (solve) {
      const Hodo<double> hd = hodo_of<double>(kind, Xd, Yd, (double)rp.w);
      if constexpr (PREC == PS_PREC_FP32_FIXUP) {
        // the FP32 quadratic isolates and selects the root, one FP64 Newton
        // step on g'(t).n polishes it; no FP32 root, a step above fix_tol or
        // a step out of the interval (a root close to a cusp or to the other
        // root) sends the rib to the FP64 solve
        bool found;
        const float t0f = emit_solve32(hodo_of<float>(kind, X, Y, rp.w), (float)nx, (float)ny,
                                       (float)v.lo, (float)v.hi, found);
        const double al = hd.e0x * nx + hd.e0y * ny;
        const double be = hd.e1x * nx + hd.e1y * ny;
        const double ga = hd.e2x * nx + hd.e2y * ny;
        const double Aq = al - 2.0 * be + ga, Bq = 2.0 * (be - al);
        const double t0 = (double)t0f;
        const double hv = (Aq * t0 + Bq) * t0 + al;
        const float dv = (float)(2.0 * Aq * t0 + Bq);
        const double step = (double)__builtin_amdgcn_rcpf(dv) * hv;
        const double t1 = t0 - step;
        const bool need64 = !(found && dv != 0.0f && fabs(step) <= (double)fix_tol && t1 >= v.lo && t1 <= v.hi);
        t = t1;
        o.fixed = need64;
        if (__ballot(need64)) {
          if (need64) t = emit_solve64(hd, nx, ny, v.lo, v.hi);
        }
      } else {
        t = emit_solve64(hd, nx, ny, v.lo, v.hi);
      }
    }
    eval_point(kind, Xd, Yd, (double)rp.w, t, o.gx, o.gy);
    o.t = t;
    const double r = (double)rp.r;
    o.Nx = (float)(o.gx - r * nx); o.Ny = (float)(o.gy - r * ny);
    o.Px = (float)(o.gx + r * nx); o.Py = (float)(o.gy + r * ny);
  }
}

// The outer vertex of rib j (1 or 2) of a miter join (Sec. "Harder Joins:
// Miter Truncate and Revert", which leaves the construction to standard
// practice): with o0, o3 the outer unit normals at the join's two ends (the
// -n side of a left turn), the two outer offset lines meet at
// M = c + r (o0 + o3) / (1 + o0.o3); the miter ratio (miter length over
// stroke width) is 1/cos(|delta|/2) = 2/|o0 + o3|.  Within the limit both ribs
// take M; beyond it PS_JOIN_MITER reverts to the bevel's ends and
// PS_JOIN_MITER_CLIP cuts the miter square to its bisector b at limit * r
// from c, rib 1 on the incoming offset line, rib 2 on the outgoing one.  The
// join's record holds n0 and n3 in p[0..3].
__device__ __forceinline__ void miter_vertex(const LinkRec& rp, int j, int style, double limit,
                                             double& vx, double& vy) {
  const double cx = rp.x[0], cy = rp.y[0], r = rp.r;
  const double sg = (rp.psi[1] - rp.psi[0]) > 0 ? -1.0 : 1.0;
  const double n0x = rp.p[0], n0y = rp.p[1], n3x = rp.p[2], n3y = rp.p[3];
  const double o0x = sg * n0x, o0y = sg * n0y, o3x = sg * n3x, o3y = sg * n3y;
  const double sx = o0x + o3x, sy = o0y + o3y;
  const double half = 0.5 * sqrt(sx * sx + sy * sy);   // cos(|delta| / 2)
  if (half * limit >= 1.0) {
    const double f = r / (1.0 + o0x * o3x + o0y * o3y);
    vx = cx + f * sx; vy = cy + f * sy;
    return;
  }
  if (style == PS_JOIN_MITER) {
    vx = cx + r * (j == 1 ? o0x : o3x);
    vy = cy + r * (j == 1 ? o0y : o3y);
    return;
  }
  // tangents t = (cos, sin) = (n.y, -n.x); b = t0 for an exact reversal
  const double t0x = n0y, t0y = -n0x, t3x = n3y, t3y = -n3x;
  const double bx = half > 0 ? sx / (2 * half) : t0x, by = half > 0 ? sy / (2 * half) : t0y;
  const double u = (limit * r - r * (o0x * bx + o0y * by)) / (t0x * bx + t0y * by);
  if (j == 1) { vx = cx + r * o0x + u * t0x; vy = cy + r * o0y + u * t0y; }
  else { vx = cx + r * o3x - u * t3x; vy = cy + r * o3y - u * t3y; }
}

// Join or cap rib j: a pivot of J steps at a fixed point (Sec. "Tessellation
// Approach for Caps and Joins"), psi_j = psi_0 + j delta / J (exact at both
// ends); only the side away from the turn keeps its radius; the square cap's
// ribs 1 and 3 reach r sqrt 2; miter joins replace the outer vertex of ribs
// 1 and 2.  The direction is FP32 in every mode: the pivot point is exact and
// a rib's vertex is at most r sqrt 2 from it, so an angle error of 1e-6 rad
// (the FP32 rounding of psi within a few turns) moves it by under 1e-4 px at
// r = 64, below the FP32 rounding of the coordinates; nothing downstream
// depends on a pivot's direction (pivots add no arc length).  The miter
// vertices stay FP64.
template <int PREC>
__device__ __forceinline__ void piv_rib(const LinkRec& rp, int j, double miter_limit, const double2* tab,
                                        const float2* tab32, RibOut& o) {
  const int style = rp.flags >> 4;
  const int J = rp.dsum[0];
  const double psa = rp.psi[0], psb = rp.psi[1];
  const float psa32 = (float)psa;
  const float psi = j == 0 ? psa32
                  : (j == J ? (float)psb : fmaf((float)(psb - psa), (float)j * __builtin_amdgcn_rcpf((float)J), psa32));
  float sn, cs;
  if constexpr (PREC == PS_PREC_FP32) sincos_tab32(tab32, psi, &sn, &cs);
  else sincos_tab32d(tab, psi, &sn, &cs);
  const float nx = -sn, ny = cs;
  float rout = rp.r;
  if ((rp.role == ROLE_SCAP || rp.role == ROLE_ECAP) && style == PS_CAP_SQUARE && (j == 1 || j == 3))
    rout *= 1.41421356f;
  const bool left_turn = (psb - psa) > 0;
  const float rN = left_turn ? rout : 0.0f, rP = left_turn ? 0.0f : rout;
  const float cx = rp.x[0], cy = rp.y[0];
  o.gx = cx; o.gy = cy; o.t = 0.0; o.fixed = false;
  o.Nx = fmaf(-rN, nx, cx); o.Ny = fmaf(-rN, ny, cy);
  o.Px = fmaf(rP, nx, cx); o.Py = fmaf(rP, ny, cy);
  if (rp.role == ROLE_JOIN && (j == 1 || j == 2) && (style == PS_JOIN_MITER || style == PS_JOIN_MITER_CLIP)) {
    double vx, vy;
    miter_vertex(rp, j, style, miter_limit, vx, vy);
    if (left_turn) { o.Nx = (float)vx; o.Ny = (float)vy; }
    else { o.Px = (float)vx; o.Py = (float)vy; }
  }
}

// A chord |(dx, dy)| in FP32 (Eq. arc-length-approximation sums chords; they
// are taken in FP32 and their sums kept exact), as a whole number of 2^-32 px:
// dx and dy rounded to FP32, the hardware square root of dx^2 + dy^2 (each
// step within an ulp, so the chord within 2^-22 of its length), then scaled by
// 2^32.  A float of at least 2^-9 is already a whole number of units (its
// last bit is worth 2^-32 or more): its significand shifted into place.  A
// smaller one is rounded to the nearest unit in FP32, where the scaling is
// exact and the result is below 2^23.
__device__ __forceinline__ long long chord_fix(double dx, double dy) {
  const float fx = (float)dx, fy = (float)dy;
  const float c = __builtin_amdgcn_sqrtf(fmaf(fx, fx, fy * fy));
  const unsigned bits = __float_as_uint(c);
  const int sh = (int)(bits >> 23) - 118;   // the exponent less 127 + 23 - 32
  const unsigned long long m = (bits & 0x7fffffu) | 0x800000u;
  const unsigned small = (unsigned)rintf(c * 0x1p32f);
  return sh >= 0 ? (long long)(m << (sh & 63)) : (long long)small;
}

// Cross-lane moves on the VALU (DPP) rather than through the LDS crossbar.
// A lane whose source lies outside its row, or that row_mask leaves out,
// reads 0: the identity of the sums below.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ long long dpp_i64(long long v) {
  const unsigned lo = (unsigned)dpp_i32<CTRL, ROWS>((int)(unsigned)(unsigned long long)v);
  const unsigned hi = (unsigned)dpp_i32<CTRL, ROWS>((int)(unsigned)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
// the value of lane - 1 (wave_shr:1); lane 0, which has no source lane,
// keeps the DPP's old value: `first`
__device__ __forceinline__ double wave_shr1(double v, double first) {
  const unsigned long long a = (unsigned long long)__double_as_longlong(v);
  const unsigned long long f = (unsigned long long)__double_as_longlong(first);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)f, (int)(unsigned)a, 0x138, 0xf, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(f >> 32), (int)(unsigned)(a >> 32), 0x138,
                                                            0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ long long readlane_i64(long long v, int l) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(unsigned long long)v, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)v >> 32), l);
  return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double readlane_f64(double v, int l) {
  return __longlong_as_double(readlane_i64(__double_as_longlong(v), l));
}
// one step of a plain 32-bit inclusive scan (the add takes the DPP operand)
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned scan_step_u32(unsigned v) {
  return v + (unsigned)dpp_i32<CTRL, ROWS>((int)v);
}
// one step of the segmented scan: (c, f) <- (left) op (c, f), where op keeps
// the right sum when it holds a path start
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_scan_step(long long& c, int& f) {
  const long long cu = dpp_i64<CTRL, ROWS>(c);
  const int fu = dpp_i32<CTRL, ROWS>(f);
  c = f ? c : c + cu;
  f |= fu;
}

// Tile rounds.  With arc length, tiles wait on earlier tiles' look-back
// words, so tiles are claimed in increasing order by running wavefronts: one
// ticket (an atomic counter) per workgroup per round, the workgroup's waves
// taking tiles ticket * waves + w.  The ticket goes through one of two LDS
// slots by round parity, so one barrier per round suffices (a slot is written
// again two rounds later, after every wave has passed the barrier of the
// round between).  Without arc length no tile waits on another, and
// workgroup g simply takes rounds g, g + gridDim.x, ... with no atomic and no
// barrier.
template <bool ORDERED>
struct TileRounds {
  unsigned int ticket, round;
  __device__ __forceinline__ unsigned int first(unsigned long long* counter, unsigned int* slot) {
    round = 0;
    ticket = ORDERED ? claim(counter, slot) : blockIdx.x;
    return ticket;
  }
  __device__ __forceinline__ unsigned int next(unsigned long long* counter, unsigned int* slot) {
    ++round;
    ticket = ORDERED ? claim(counter, slot) : ticket + gridDim.x;
    return ticket;
  }
  __device__ __forceinline__ unsigned int claim(unsigned long long* counter, unsigned int* slot) {
    if (threadIdx.x == 0) slot[round & 1] = (unsigned int)atomicAdd(counter, 1ull);
    __syncthreads();
    return slot[round & 1];
  }
};

// Records of n (<= 12) consecutive link slots into LDS: the heads, then the
// tail pieces of the links that have a tail (the flags and interval counts
// are in the heads just written; a wavefront's LDS accesses complete in
// order), or INT_MAX for dsum[1..4] of the others.
__device__ __forceinline__ void stage_recs(const v4u32* head, const v4u32* tail, int n, LinkRec* rec,
                                           int lane) {
  v4u32* dst = reinterpret_cast<v4u32*>(rec);
  if (lane < n * kHeadPieces) dst[(lane >> 2) * kRecPieces + head_piece(lane & 3)] = head[lane];
  if (lane < n * kTailPieces) {
    const int i = lane / kTailPieces, k = lane - kTailPieces * i;
    if ((rec[i].flags & kHasTail) && (tail_whole(rec[i]) || k == 0 || k == 1 || k == 3))
      dst[i * kRecPieces + tail_piece(k)] = tail[lane];
    else if (k == 0) dst[i * kRecPieces + 1] = (v4u32){INT_MAX, INT_MAX, INT_MAX, INT_MAX};
  }
}

// Role-split emit.  Persistent workgroups of W wavefronts take one ticket per
// round and their wavefronts tiles ticket * W + w, so every tile a wavefront
// waits on belongs to a wavefront already running.  Tile T stores ribs
// [T*TS, (T+1)*TS), TS = 64*K.  A wavefront stages windows of kWin
// consecutive link slots (their offsets and records) in LDS
// and sweeps each window twice: once over its segment ribs, 64 at a time in
// rib order (solve, point, vertices, chords, arc-length scan), once over its
// join and cap ribs; a wavefront never mixes the two roles.  Chords join
// consecutive ribs of one segment, so the arc length is a scan over the
// segment ribs alone (a path restarts at its first segment rib); a pivot's s
// is the s of its segment's last rib, or 0 for a start cap.
//
// Arc length is accumulated in 64-bit fixed point (2^-32 px per unit): each
// chord is rounded once and every sum after that is an integer sum, so s does
// not depend on the tiling, the mapping or the order tiles finish in.
constexpr int kWin = 12;
struct SplitLDS {
  long long off[kWin + 1];
  LinkRec rec[kWin];
  long long ends[kWin + 1];   // ends[i + 1]: s at slot i's last rib (bit 63: add the tile prefix)
  int segpos[kWin + 1];       // exclusive positions of the slots' segment ribs
  int pivpos[kWin + 1];       // ... and of their pivot ribs
  int first[kWin];            // first rib of the slot in this tile, minus (r0 - 1)
  int jfirst[kWin];           // ... as a rib index within its link
  int endrel[kWin];           // the slot's last rib minus r0 (INT_MAX when past the tile)
};

// two buffers of per-rib partial sums: a tile whose predecessors have not all
// published yet is parked in one while the wavefront computes its next tile
__host__ __device__ constexpr size_t emit_split_lds_per_wave(int K, bool ws) {
  return sizeof(SplitLDS) + (ws ? 2 * (size_t)K * 64 * sizeof(long long) : 0);
}

// Stores of a tile's vertex pairs through a buffer resource that spans only
// the tile's own bytes: 32-bit offsets from the tile start instead of 64-bit
// addresses per lane, and a store outside the tile is dropped by the hardware.
// The stores are non-temporal (the output is not read again by the emit):
// measured 0.424 against 0.448 ms per emit on the 4096-path batch.
typedef unsigned int v2u32 __attribute__((ext_vector_type(2)));
constexpr int kStoreNT = 2;   // cache-policy operand: the nt (non-temporal) bit
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(float* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)bytes, 0x00020000);   // raw dwords (gfx9)
}
template <int POLICY = kStoreNT>
__device__ __forceinline__ void store_pair(__amdgpu_buffer_rsrc_t r, int rel, float a, float b) {
  const v2u32 d = {__float_as_uint(a), __float_as_uint(b)};
  __builtin_amdgcn_raw_buffer_store_b64(d, r, rel * 8, 0, POLICY);
}

// A computed tile whose arc length still needs its prefix.
struct TileState {
  int64_t tile, r0, r1;
  unsigned long long agg;
  bool seen_start, any_need;
  int buf;
};

// Finish a tile: collect its prefix from the look-back words of earlier tiles
// (waiting for any not yet published), publish its inclusive word, write vs.
template <int K>
__device__ __forceinline__ void finish_tile(const EmitArgs& A, const TileState& T, const long long* srel) {
  constexpr unsigned long long kNeed = 1ull << 63;
  const int lane = threadIdx.x & 63;
  unsigned long long prefix = 0;
  if (T.any_need) {
    look_back(A.desc, T.tile, true, prefix);
    if (lane == 0 && !T.seen_start)
      desc_publish(&A.desc[T.tile], (2ull << 62) | ((prefix + T.agg) & kValMask));
  }
  const long long pre = (long long)prefix;
  const long long* sr = srel + (size_t)T.buf * (64 * K);
  const int n = (int)(T.r1 - T.r0);
  const __amdgpu_buffer_rsrc_t rs = tile_rsrc(A.vs + 2 * T.r0, (uint32_t)n * 8u);
#pragma unroll 2
  for (int k = 0; k < K; ++k) {
    const int d = 64 * k + lane;
    if (d < n) {
      const unsigned long long sv = (unsigned long long)sr[d];
      const long long sf = (long long)(sv & ~kNeed) + ((sv & kNeed) ? pre : 0);
      const float sx = (float)((double)sf * (1.0 / kFix));
      store_pair(rs, d, sx, sx);
    }
  }
}

template <int K, int PREC, bool WXY, bool WS>
// 4 wavefronts per SIMD (at most 128 VGPRs); how many are resident is then up
// to the LDS per workgroup, which K sets.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
emit_split_kernel(EmitArgs A) {
  extern __shared__ unsigned char smem_raw[];
  unsigned char* wave_lds = smem_raw + (threadIdx.x >> 6) * emit_split_lds_per_wave(K, WS);
  SplitLDS& w = *reinterpret_cast<SplitLDS*>(wave_lds);
  long long* const srel_base = reinterpret_cast<long long*>(wave_lds + sizeof(SplitLDS));   // 2 x (rib - r0)
  __shared__ double2 sc_tab[kSinTab];
  __shared__ float2 sc_tab32[PREC == PS_PREC_FP32 ? kSinTab : 1];
  const int lane = threadIdx.x & 63;
  const int64_t L = A.n_links;
  const int64_t R = A.off[L];
  constexpr int TS = 64 * K;   // whole cache lines per tile (the first chord needs no lane of its own)
  constexpr unsigned long long kNeed = 1ull << 63;   // "add the tile's prefix"
  const int64_t n_tiles = (R + TS - 1) / TS;
  if (2 * R > A.capacity || n_tiles > A.max_tiles) return;
  unsigned long long fixups = 0;
  __shared__ unsigned int group_ticket[2];
  TileRounds<WS> rounds;
  const int n_waves = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  TileState parked;
  parked.tile = -1; parked.r0 = parked.r1 = 0; parked.agg = 0;
  parked.seen_start = parked.any_need = false; parked.buf = 0;
  // a workgroup without a tile leaves before filling the sincos table
  unsigned int ticket = rounds.first(&A.st->tile_counter, group_ticket);
  if ((int64_t)ticket * n_waves >= n_tiles) return;
  fill_sincos_tab(sc_tab);
  if (PREC == PS_PREC_FP32) {
    __syncthreads();
    fill_sincos_tab32(sc_tab32, sc_tab);
  }
  __syncthreads();
  for (;; ticket = rounds.next(&A.st->tile_counter, group_ticket)) {
    const int64_t first_tile = (int64_t)ticket * n_waves;
    if (first_tile >= n_tiles) break;
    const int64_t tile = first_tile + wave;
    if (tile < n_tiles) {
      const int buf = (WS && parked.tile >= 0) ? 1 - parked.buf : 0;
      long long* const srel = srel_base + (size_t)buf * (64 * K);
      const int64_t r0 = tile * TS;
      const int64_t r1 = (r0 + TS < R) ? r0 + TS : R;
      // ribs of the tile are addressed by 32-bit offsets from r0
      const uint32_t tile_bytes = (uint32_t)(r1 - r0) * 8u;
      const __amdgpu_buffer_rsrc_t vxt = tile_rsrc(A.vx + 2 * r0, tile_bytes);
      const __amdgpu_buffer_rsrc_t vyt = tile_rsrc(A.vy + 2 * r0, tile_bytes);
      int64_t base = A.tile_link[tile];
      long long run = 0;                 // segment chord sum since the tile start or its last path start
      bool seen_start = false;
      bool any_need = false;
      double cgx = 0, cgy = 0, ct = 0;   // the previous segment rib
      unsigned long long carry_end = kNeed;
      for (;;) {
        // ---- stage the window: offsets and records of kWin slots
        const int64_t idx = base + lane;
        const long long o_i = (lane <= kWin && idx <= L) ? A.off[idx] : LLONG_MAX;
        if (lane <= kWin) w.off[lane] = o_i;
        const long long o_n = __shfl(o_i, lane + 1 < 64 ? lane + 1 : 63, 64);
        {
          // only the slots that start before the tile's end (a prefix: the
          // offsets do not decrease) have ribs in it; the others keep stale
          // records, which nothing reads
          const int n_rec = __popcll(__ballot(lane < kWin && idx < L && o_i < r1));
          stage_recs(A.head + base * kHeadPieces, A.tail + base * kTailPieces, n_rec, w.rec, lane);
        }
        // ---- each slot's ribs inside the tile; the link holding r0 also
        // gives rib r0 - 1 when it is a segment begun earlier (first chord)
        int ns = 0, np = 0, fr = 0, jf = 0, er = INT_MAX;
        if (lane < kWin && idx < L) {
          const bool segl = w.rec[lane].role == ROLE_SEG;
          long long a = o_i > r0 ? o_i : r0;
          if (segl && r0 > 0 && o_i < r0 && r0 < o_n) a = r0 - 1;
          const long long b = o_n < r1 ? o_n : r1;
          const int n = b > a ? (int)(b - a) : 0;
          ns = segl ? n : 0;
          np = segl ? 0 : n;
          fr = (int)(a - (r0 - 1));
          jf = (int)(a - o_i);
          const long long e = o_n - 1 - r0;
          er = e < (long long)INT_MAX ? (int)e : INT_MAX;
        }
        const int ns_in = wave_incl_scan(ns), np_in = wave_incl_scan(np);
        const int segpos_l = ns_in - ns;   // lane m <= kWin: exclusive positions of slot m
        const int pivpos_l = np_in - np;
        const int NS = __builtin_amdgcn_readlane(ns_in, 63), NP = __builtin_amdgcn_readlane(np_in, 63);
        if (lane <= kWin) {
          w.segpos[lane] = ns_in - ns;
          w.pivpos[lane] = np_in - np;
          if (WS) w.ends[lane] = (lane == 0) ? (long long)carry_end : (long long)kNeed;
        }
        if (lane < kWin) { w.first[lane] = fr; w.jfirst[lane] = jf; w.endrel[lane] = er; }
        // ---- sweep A: segment ribs
        int i_lo = 0;   // the slot holding rib position q0 - 1 (or 0)
        for (int q0 = 0; q0 < NS; q0 += 64) {
          const int q = q0 + lane;
          RibOut o;
          o.gx = o.gy = o.t = 0; o.fixed = false;
          int rel = -1;   // rib - r0
          bool chord_ok = false, path_start = false;
          // largest i with segpos[i] <= q (the slot holding q: of equal
          // positions the last one has the ribs); the positions do not
          // decrease, so only the slots from i_lo up to the first one that
          // starts past this batch are compared, their positions read from
          // the slot lanes as wave-uniform values
          int i = i_lo;
          for (int m = i_lo + 1; m < kWin; m = __builtin_amdgcn_readfirstlane(m + 1)) {
            const int sp = __builtin_amdgcn_readlane(segpos_l, m);
            if (sp > q0 + 63) break;
            i = (q >= sp) ? m : i;
          }
          i_lo = __builtin_amdgcn_readlane(i, 63);
          if (q < NS) {
            const int d = q - w.segpos[i];
            const int j = w.jfirst[i] + d;
            rel = w.first[i] - 1 + d;
            const LinkRec& rp = w.rec[i];
            seg_rib<PREC>(rp, j, rib_ival(rp, j), A.fix_tol, sc_tab, sc_tab32, o);
            if (WXY && rel >= 0) {
              store_pair(vxt, rel, o.Nx, o.Px);
              store_pair(vyt, rel, o.Ny, o.Py);
            }
            fixups += o.fixed ? 1 : 0;
            chord_ok = j > 0;
            path_start = (rp.flags & kFirstSegInPath) && j == 0;
          }
          if (WS) {
            const bool mine = q < NS && rel >= 0;
            const double pgx = wave_shr1(o.gx, cgx), pgy = wave_shr1(o.gy, cgy), pt = wave_shr1(o.t, ct);
            long long c = 0;
            if (mine && chord_ok && o.t >= pt) {
              const double dx = o.gx - pgx, dy = o.gy - pgy;
              c = chord_fix(dx, dy);
            }
            int f = (mine && path_start) ? 1 : 0;
            if (__ballot(f != 0 || c >= (1ll << 50)) == 0ull) {
              unsigned lo = (unsigned)c & 0xffffffu, hi = (unsigned)(c >> 24);
              lo = scan_step_u32<0x111, 0xf>(lo); hi = scan_step_u32<0x111, 0xf>(hi);
              lo = scan_step_u32<0x112, 0xf>(lo); hi = scan_step_u32<0x112, 0xf>(hi);
              lo = scan_step_u32<0x114, 0xf>(lo); hi = scan_step_u32<0x114, 0xf>(hi);
              lo = scan_step_u32<0x118, 0xf>(lo); hi = scan_step_u32<0x118, 0xf>(hi);
              lo = scan_step_u32<0x142, 0xa>(lo); hi = scan_step_u32<0x142, 0xa>(hi);
              lo = scan_step_u32<0x143, 0xc>(lo); hi = scan_step_u32<0x143, 0xc>(hi);
              c = (long long)(((unsigned long long)hi << 24) + lo);
            } else {
              seg_scan_step<0x111, 0xf>(c, f);
              seg_scan_step<0x112, 0xf>(c, f);
              seg_scan_step<0x114, 0xf>(c, f);
              seg_scan_step<0x118, 0xf>(c, f);
              seg_scan_step<0x142, 0xa>(c, f);
              seg_scan_step<0x143, 0xc>(c, f);
            }
            const bool need = !(f || seen_start);
            const unsigned long long v =
                (unsigned long long)(f ? c : run + c) | (need ? kNeed : 0ull);
            if (mine) {
              srel[rel] = (long long)v;
              if (rel == w.endrel[i]) w.ends[i + 1] = (long long)v;   // the segment's last rib
            }
            any_need = any_need || (__ballot(mine && need) != 0ull);
            const long long c63 = readlane_i64(c, 63);
            const int f63 = __builtin_amdgcn_readlane(f, 63);
            run = f63 ? c63 : run + c63;
            seen_start = seen_start || (f63 != 0);
            // the last segment rib of this batch carries into the next one
            const int last = (NS - q0 < 64) ? NS - q0 - 1 : 63;
            cgx = readlane_f64(o.gx, last); cgy = readlane_f64(o.gy, last); ct = readlane_f64(o.t, last);
          }
        }
        // ---- sweep B: pivot ribs (the slot found as in sweep A)
        int ip_lo = 0;
        for (int p0 = 0; p0 < NP; p0 += 64) {
          const int pq = p0 + lane;
          int i = ip_lo;
          for (int m = ip_lo + 1; m < kWin; m = __builtin_amdgcn_readfirstlane(m + 1)) {
            const int sp = __builtin_amdgcn_readlane(pivpos_l, m);
            if (sp > p0 + 63) break;
            i = (pq >= sp) ? m : i;
          }
          ip_lo = __builtin_amdgcn_readlane(i, 63);
          if (pq < NP) {
            const int d = pq - w.pivpos[i];
            const int rel = w.first[i] - 1 + d;   // >= 0: pivots never reach back before r0
            RibOut o;
            piv_rib<PREC>(w.rec[i], w.jfirst[i] + d, A.miter_limit, sc_tab, sc_tab32, o);
            if (WXY) {
              store_pair(vxt, rel, o.Nx, o.Px);
              store_pair(vyt, rel, o.Ny, o.Py);
            }
            if (WS) {
              // a join or end cap takes its segment's end value (slot i - 1)
              const long long v = (w.rec[i].role == ROLE_SCAP) ? 0ll : w.ends[i];
              srel[rel] = v;
              any_need = any_need || ((unsigned long long)v & kNeed);
            }
          }
          if (WS) any_need = __ballot(any_need) != 0ull;
        }
        if (WS) carry_end = (unsigned long long)w.ends[kWin];
        const long long wend = w.off[kWin];   // first rib past the window
        if (wend >= r1) break;
        base += kWin;
      }
      if (WS) {
        const unsigned long long agg = (unsigned long long)run & kValMask;
        any_need = __ballot(any_need) != 0ull;
        if (lane == 0) desc_publish(&A.desc[tile], ((seen_start ? 2ull : 1ull) << 62) | agg);
        TileState cur;
        cur.tile = tile; cur.r0 = r0; cur.r1 = r1; cur.agg = agg;
        cur.seen_start = seen_start; cur.any_need = any_need; cur.buf = buf;
        // every tile is parked and finished after the wavefront's next one:
        // its predecessors have had a whole tile's time to publish (most
        // have not when the tile itself is done, so trying it at once first
        // cost a look-back read that mostly failed: 0.407 against 0.396 ms)
        if (parked.tile >= 0) finish_tile<K>(A, parked, srel_base);
        parked = cur;
      }
    }
  }
  if (WS && parked.tile >= 0) finish_tile<K>(A, parked, srel_base);
  if (PREC == PS_PREC_FP32_FIXUP) {
    unsigned long long v = fixups;
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0 && v) atomicAdd(&A.st->fixups, v);
  }
}

// PS_MAP_LINKS: the same tiles of 64*K ribs, tickets, parking and
// look-back, but a wavefront walks a tile link by link, all 64 lanes on ribs
// of one link at a time.  The link's header and body are then the same for
// every lane and come through scalar loads into scalar registers (the loads
// go through the constant address space), so there is no LDS window, no slot
// search and no per-lane record; the price is the lanes a link leaves idle
// in its last 64.  Chords and the arc-length scan are as in the tiles
// mapping, except that a path can only start at lane 0 (the first rib of its
// first segment), so the scan never needs the segmented form.
// A wavefront-uniform load of T at p into scalar registers: the words are
// read through the constant address space, which the compiler turns into
// scalar loads when the address is uniform.
template <typename T>
__device__ __forceinline__ T load_uniform(const T* p) {
  typedef __attribute__((address_space(4))) const unsigned int* CU32;
  const CU32 q = (CU32)p;
  unsigned int w[sizeof(T) / 4];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = q[i];
  T v;
  __builtin_memcpy(&v, w, sizeof(T));
  return v;
}

// Record of link l as scalar loads (l wave-uniform): the head, then the tail
// when the head's flags say it has one.
__device__ __forceinline__ LinkRec load_rec_uniform(const v4u32* head, const v4u32* tail, int64_t l) {
  typedef __attribute__((address_space(4))) const unsigned int* CU32;
  unsigned int w[kRecPieces * 4];
  const CU32 h = (CU32)(head + l * kHeadPieces);
#pragma unroll
  for (int k = 0; k < kHeadPieces; ++k)
    for (int d = 0; d < 4; ++d) w[head_piece(k) * 4 + d] = h[k * 4 + d];
  if ((w[0] >> 24) & kHasTail) {
    const CU32 t = (CU32)(tail + l * kTailPieces);
#pragma unroll
    for (int k = 0; k < kTailPieces; ++k)
      for (int d = 0; d < 4; ++d) w[tail_piece(k) * 4 + d] = t[k * 4 + d];
  } else {
#pragma unroll
    for (int k = 0; k < kTailPieces; ++k)
      for (int d = 0; d < 4; ++d) w[tail_piece(k) * 4 + d] = k == 0 ? (unsigned)INT_MAX : 0u;
  }
  LinkRec r;
  __builtin_memcpy(&r, w, sizeof(LinkRec));
  return r;
}

__host__ __device__ constexpr size_t emit_links_lds_per_wave(int K, bool ws) {
  return ws ? 2 * (size_t)K * 64 * sizeof(long long) : 16;
}

// inclusive 64-bit sum over the wavefront as two exact 32-bit scans (the
// low 24 and the high bits of chords below 2^50 units), or as a plain 64-bit
// scan when a chord is longer
__device__ __forceinline__ long long wave_sum_incl(long long c) {
  if (__ballot(c >= (1ll << 50)) == 0ull) {
    unsigned lo = (unsigned)c & 0xffffffu, hi = (unsigned)(c >> 24);
    lo = scan_step_u32<0x111, 0xf>(lo); hi = scan_step_u32<0x111, 0xf>(hi);
    lo = scan_step_u32<0x112, 0xf>(lo); hi = scan_step_u32<0x112, 0xf>(hi);
    lo = scan_step_u32<0x114, 0xf>(lo); hi = scan_step_u32<0x114, 0xf>(hi);
    lo = scan_step_u32<0x118, 0xf>(lo); hi = scan_step_u32<0x118, 0xf>(hi);
    lo = scan_step_u32<0x142, 0xa>(lo); hi = scan_step_u32<0x142, 0xa>(hi);
    lo = scan_step_u32<0x143, 0xc>(lo); hi = scan_step_u32<0x143, 0xc>(hi);
    return (long long)(((unsigned long long)hi << 24) + lo);
  }
  c += dpp_i64<0x111, 0xf>(c);
  c += dpp_i64<0x112, 0xf>(c);
  c += dpp_i64<0x114, 0xf>(c);
  c += dpp_i64<0x118, 0xf>(c);
  c += dpp_i64<0x142, 0xa>(c);
  c += dpp_i64<0x143, 0xc>(c);
  return c;
}

template <int K, int PREC, bool WXY, bool WS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
emit_links_kernel(EmitArgs A) {
  extern __shared__ unsigned char smem_raw[];
  long long* const srel_base =
      reinterpret_cast<long long*>(smem_raw + (threadIdx.x >> 6) * emit_links_lds_per_wave(K, WS));
  __shared__ double2 sc_tab[kSinTab];
  __shared__ float2 sc_tab32[PREC == PS_PREC_FP32 ? kSinTab : 1];
  const int lane = threadIdx.x & 63;
  const int64_t L = A.n_links;
  const int64_t R = A.off[L];
  constexpr int TS = 64 * K;
  constexpr unsigned long long kNeed = 1ull << 63;   // "add the tile's prefix"
  const int64_t n_tiles = (R + TS - 1) / TS;
  if (2 * R > A.capacity || n_tiles > A.max_tiles) return;
  unsigned long long fixups = 0;
  __shared__ unsigned int group_ticket[2];
  TileRounds<WS> rounds;
  const int n_waves = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  TileState parked;
  parked.tile = -1; parked.r0 = parked.r1 = 0; parked.agg = 0;
  parked.seen_start = parked.any_need = false; parked.buf = 0;
  unsigned int ticket = rounds.first(&A.st->tile_counter, group_ticket);
  if ((int64_t)ticket * n_waves >= n_tiles) return;
  fill_sincos_tab(sc_tab);
  if (PREC == PS_PREC_FP32) {
    __syncthreads();
    fill_sincos_tab32(sc_tab32, sc_tab);
  }
  __syncthreads();
  for (;; ticket = rounds.next(&A.st->tile_counter, group_ticket)) {
    const int64_t first_tile = (int64_t)ticket * n_waves;
    if (first_tile >= n_tiles) break;
    const int64_t tile = first_tile + wave;
    if (tile < n_tiles) {
      const int buf = (WS && parked.tile >= 0) ? 1 - parked.buf : 0;
      long long* const srel = srel_base + (size_t)buf * (64 * K);
      const int64_t r0 = tile * TS;
      const int64_t r1 = (r0 + TS < R) ? r0 + TS : R;
      const uint32_t tile_bytes = (uint32_t)(r1 - r0) * 8u;
      const __amdgpu_buffer_rsrc_t vxt = tile_rsrc(A.vx + 2 * r0, tile_bytes);
      const __amdgpu_buffer_rsrc_t vyt = tile_rsrc(A.vy + 2 * r0, tile_bytes);
      long long run = 0;          // segment chord sum since the tile start or its last path start
      bool seen_start = false;
      bool any_need = false;
      unsigned long long end_val = kNeed;   // s at the last segment rib so far (bit 63: add the prefix)
      for (int64_t l = __builtin_amdgcn_readfirstlane((int)A.tile_link[tile]); l < L; ++l) {
        const long long a = load_uniform(A.off + l), b = load_uniform(A.off + l + 1);
        if (a >= r1) break;
        if (b <= r0 || b == a) continue;   // no rib in the tile
        const LinkRec rp = load_rec_uniform(A.head, A.tail, l);
        if (rp.role == ROLE_SEG) {
          // a segment begun in an earlier tile also gives rib r0 - 1, the
          // first chord's other end
          const long long start = a < r0 ? r0 - 1 : a;
          const long long end = b < r1 ? b : r1;
          double cgx = 0, cgy = 0, ct = 0;
          for (long long q0 = start; q0 < end; q0 += 64) {
            const long long rib = q0 + lane;
            const bool act = rib < end;
            const int j = (int)(rib - a);
            const int rel = (int)(rib - r0);
            const bool mine = act && rib >= r0;
            RibOut o;
            o.gx = o.gy = o.t = 0; o.fixed = false;
            if (act) seg_rib<PREC>(rp, j, rib_ival_uniform(rp, j), A.fix_tol, sc_tab, sc_tab32, o);
            if (WXY && mine) {
              store_pair(vxt, rel, o.Nx, o.Px);
              store_pair(vyt, rel, o.Ny, o.Py);
            }
            fixups += (mine && o.fixed) ? 1 : 0;
            if (WS) {
              const double pgx = wave_shr1(o.gx, cgx), pgy = wave_shr1(o.gy, cgy), pt = wave_shr1(o.t, ct);
              long long c = 0;
              if (mine && j > 0 && o.t >= pt) {
                const double dx = o.gx - pgx, dy = o.gy - pgy;
                c = chord_fix(dx, dy);
              }
              // a path restarts at the first rib of its first segment
              if (q0 == a && (rp.flags & kFirstSegInPath)) { run = 0; seen_start = true; }
              c = wave_sum_incl(c);
              const unsigned long long v = (unsigned long long)(run + c) | (seen_start ? 0ull : kNeed);
              if (mine) srel[rel] = (long long)v;
              any_need = any_need || !seen_start;
              run += readlane_i64(c, 63);
              const int last = (end - q0 < 64) ? (int)(end - q0) - 1 : 63;
              if (end == b && q0 + 64 >= end) end_val = (unsigned long long)readlane_i64((long long)v, last);
              cgx = readlane_f64(o.gx, last); cgy = readlane_f64(o.gy, last); ct = readlane_f64(o.t, last);
            }
          }
        } else {
          const long long start = a < r0 ? r0 : a;
          const long long end = b < r1 ? b : r1;
          // a join or end cap takes its segment's end value, a start cap 0
          const unsigned long long pv = (rp.role == ROLE_SCAP) ? 0ull : end_val;
          if (WS && (pv & kNeed)) any_need = true;
          for (long long q0 = start; q0 < end; q0 += 64) {
            const long long rib = q0 + lane;
            if (rib < end) {
              const int rel = (int)(rib - r0);
              RibOut o;
              piv_rib<PREC>(rp, (int)(rib - a), A.miter_limit, sc_tab, sc_tab32, o);
              if (WXY) {
                store_pair(vxt, rel, o.Nx, o.Px);
                store_pair(vyt, rel, o.Ny, o.Py);
              }
              if (WS) srel[rel] = (long long)pv;
            }
          }
        }
      }
      if (WS) {
        const unsigned long long agg = (unsigned long long)run & kValMask;
        if (lane == 0) desc_publish(&A.desc[tile], ((seen_start ? 2ull : 1ull) << 62) | agg);
        TileState cur;
        cur.tile = tile; cur.r0 = r0; cur.r1 = r1; cur.agg = agg;
        cur.seen_start = seen_start; cur.any_need = any_need; cur.buf = buf;
        if (parked.tile >= 0) finish_tile<K>(A, parked, srel_base);
        parked = cur;
      }
    }
  }
  if (WS && parked.tile >= 0) finish_tile<K>(A, parked, srel_base);
  if (PREC == PS_PREC_FP32_FIXUP) {
    unsigned long long v = fixups;
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0 && v) atomicAdd(&A.st->fixups, v);
  }
}

// ===========================================================================
// Uniform parametric baseline and facet statistics (Sec. "Versus Uniform
// Parametric Tessellation")
// ===========================================================================
struct UniformArgs {
  const v4u32* head;
  const v4u32* tail;
  const int64_t* off;
  int64_t n_links;
  float* vx;
  float* vy;
  int64_t capacity;
  double miter_limit;
};

// largest l with off[l] <= r (the link holding rib r, r < off[n_links])
__device__ __forceinline__ int64_t rib_link(const int64_t* off, int64_t n_links, int64_t r) {
  int64_t a = 0, b = n_links - 1;
  while (a < b) {
    const int64_t m = (a + b + 1) >> 1;
    if (off[m] <= r) a = m; else b = m - 1;
  }
  return a;
}

// One thread per rib: segment ribs at t_j = j/N on Eq. NaiveStroking (N + 1
// ribs; the unit left normal of g'(t_j), taken 2^-20/N further into the
// segment where g' vanishes), joins and caps as the polar emit.
__global__ void __launch_bounds__(256) uniform_emit_kernel(UniformArgs A) {
  __shared__ double2 sc_tab[kSinTab];
  fill_sincos_tab(sc_tab);
  __syncthreads();
  const int64_t R = A.off[A.n_links];
  if (2 * R > A.capacity) return;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = rib_link(A.off, A.n_links, r);
    const int j = (int)(r - A.off[l]);
    LinkRec rp;
    {
      // the record of link l: its head, and its tail or INT_MAX for dsum[1..4]
      v4u32 pc[kRecPieces];
      const bool tl = (A.head[l * kHeadPieces][0] >> 24) & kHasTail;
#pragma unroll
      for (int k = 0; k < kHeadPieces; ++k) pc[head_piece(k)] = A.head[l * kHeadPieces + k];
#pragma unroll
      for (int k = 0; k < kTailPieces; ++k)
        pc[tail_piece(k)] = tl ? A.tail[l * kTailPieces + k]
                               : (k == 0 ? (v4u32){INT_MAX, INT_MAX, INT_MAX, INT_MAX} : (v4u32){0, 0, 0, 0});
      __builtin_memcpy(&rp, pc, sizeof(LinkRec));
    }
    float2 ox, oy;
    if (rp.role != ROLE_SEG) {
      RibOut o;
      piv_rib<PS_PREC_FP64>(rp, j, A.miter_limit, sc_tab, nullptr, o);
      ox = make_float2(o.Nx, o.Px); oy = make_float2(o.Ny, o.Py);
    } else {
      double X[4], Y[4];
      for (int i = 0; i < 4; ++i) { X[i] = rp.x[i]; Y[i] = rp.y[i]; }
      const double w = rp.w, rad = rp.r;
      const Hodo<double> h = hodo_of<double>(rp.kind, X, Y, w);
      const int N = (int)(A.off[l + 1] - A.off[l]) - 1;   // >= 1: a segment has two ribs or more
      const double t = (double)j / (double)N;
      double gx, gy, hx, hy;
      eval_point(rp.kind, X, Y, w, t, gx, gy);
      hodo_eval(h, t, hx, hy);   // a positive multiple of g'(t)
      if (hx == 0.0 && hy == 0.0) {
        const double d = ldexp(1.0, -20) / N;
        hodo_eval(h, t < 0.5 ? t + d : t - d, hx, hy);
      }
      const double inv = 1.0 / sqrt(hx * hx + hy * hy);
      const double nx = -hy * inv, ny = hx * inv;
      ox = make_float2((float)(gx - rad * nx), (float)(gx + rad * nx));
      oy = make_float2((float)(gy - rad * ny), (float)(gy + rad * ny));
    }
    *reinterpret_cast<float2*>(A.vx + 2 * r) = ox;
    *reinterpret_cast<float2*>(A.vy + 2 * r) = oy;
  }
}

__global__ void clear_stats_kernel(double* stats) {
  if (threadIdx.x < 4) stats[threadIdx.x] = 0.0;
}

// Boundary edge k -> k+1 on one side is regular when it is not empty and
// runs with the direction of travel (n rotated by -90 deg, n = P - N) at both
// of its ribs; the sign test is taken on the unnormalised product, without
// contraction, so that it is exact for coordinates of one magnitude.
__device__ bool facet_edge_ok(const float* vx, const float* vy, int64_t k, int side) {
#pragma clang fp contract(off)
  const double ex = (double)vx[2 * (k + 1) + side] - vx[2 * k + side];
  const double ey = (double)vy[2 * (k + 1) + side] - vy[2 * k + side];
  bool ok = !(ex == 0 && ey == 0);
  for (int64_t r = k; r <= k + 1; ++r) {
    const double nx = (double)vx[2 * r + 1] - vx[2 * r], ny = (double)vy[2 * r + 1] - vy[2 * r];
    ok = ok && !(nx == 0 && ny == 0) && !(ex * ny - ey * nx < 0);
  }
  return ok;
}

// One thread per segment: its ordinary facets on both sides (those with every
// edge within one rib regular; the reversed edges are the boundary inside an
// offset cusp), reduced per wavefront, then added into stats (max through the
// bit pattern, which orders non-negative doubles).
__global__ void __launch_bounds__(256) facet_stats_kernel(const int32_t* seg_begin, int n_paths,
                                                          int n_segs, const int64_t* off,
                                                          const float* vx, const float* vy,
                                                          double* stats) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double cnt = 0, mx = 0, sum = 0, sq = 0;
  if (i < n_segs) {
    const int p = path_of_seg(seg_begin, n_paths, (int)i);
    const int64_t slot = 2 * i + p + 1;
    const int64_t r0 = off[slot], r1 = off[slot + 1];
    for (int side = 0; side < 2; ++side) {
      // bit m of ok: edge r - 2 + m regular (edges outside the segment count as regular)
      unsigned ok = 0;
      for (int m = 0; m < 4; ++m) {
        const int64_t k = r0 - 1 + m;
        ok |= (unsigned)(k < r0 || k > r1 - 2 || facet_edge_ok(vx, vy, k, side)) << m;
      }
      for (int64_t r = r0 + 1; r + 1 < r1; ++r) {
        if (ok == 15u) {
          const double ax = vx[2 * (r - 1) + side], ay = vy[2 * (r - 1) + side];
          const double bx = vx[2 * r + side], by = vy[2 * r + side];
          const double cx = vx[2 * (r + 1) + side], cy = vy[2 * (r + 1) + side];
          const double e1x = bx - ax, e1y = by - ay, e2x = cx - bx, e2y = cy - by;
          const double ang = atan2(fabs(e1x * e2y - e1y * e2x), e1x * e2x + e1y * e2y);
          cnt += 1; sum += ang; sq += ang * ang; mx = fmax(mx, ang);
        }
        const int64_t k = r + 2;  // enters the window of rib r + 1
        ok = (ok >> 1) | ((unsigned)(k > r1 - 2 || facet_edge_ok(vx, vy, k, side)) << 3);
      }
    }
  }
  for (int d = 32; d >= 1; d >>= 1) {
    cnt += __shfl_xor(cnt, d, 64); sum += __shfl_xor(sum, d, 64); sq += __shfl_xor(sq, d, 64);
    mx = fmax(mx, __shfl_xor(mx, d, 64));
  }
  if ((threadIdx.x & 63) == 0 && cnt > 0) {
    atomicAdd(&stats[0], cnt);
    atomicMax(reinterpret_cast<unsigned long long*>(&stats[1]),
              (unsigned long long)__double_as_longlong(mx));
    atomicAdd(&stats[2], sum);
    atomicAdd(&stats[3], sq);
  }
}

// ===========================================================================
// Coverage of the quad strip (Sec. "Stroked Paths Tessellated to Quad Strips")
// ===========================================================================
struct CovArgs {
  const int64_t* off;        // link offsets [n_links+1]
  int64_t n_links;
  const int32_t* seg_begin;
  int n_paths;
  const float* vx;           // [2 * n_ribs], N then P per rib
  const float* vy;
  int64_t n_ribs;
  double x0, y0;             // corner of pixel (0,0); its sample at (x0+1/2, y0+1/2)
  int W, H;
  int32_t* top;              // [H*W] topmost covering path, -1 for none
};

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// The link holding rib r: the largest l with off[l] <= r (empty links share
// their offset with the next link, so this is the one that has ribs).
__device__ int64_t link_of_rib(const int64_t* off, int64_t n_links, int64_t r) {
  int64_t a = 0, b = n_links - 1;
  while (a < b) {
    const int64_t m = (a + b + 1) >> 1;
    if (off[m] <= r) a = m; else b = m - 1;
  }
  return a;
}

// The path owning link slot l: the largest p with 2*seg_begin[p] + p <= l.
__device__ int path_of_link(const int32_t* seg_begin, int n_paths, int64_t l) {
  int a = 0, b = n_paths - 1;
  while (a < b) {
    const int m = (a + b + 1) >> 1;
    if (2 * (int64_t)seg_begin[m] + m <= l) a = m; else b = m - 1;
  }
  return a;
}

// Sample index range [k0, k1] (sample k at o + k + 1/2, 0 <= k < n) of the
// samples in [lo - 1, hi + 1]; empty (k1 < k0) unless lo and hi are finite.
__device__ __forceinline__ void cov_range(double lo, double hi, double o, int n, int& k0, int& k1) {
  k0 = 0; k1 = -1;
  if (!(lo <= hi) || !isfinite(lo) || !isfinite(hi)) return;
  const double a = fmax(ceil(lo - o - 0.5) - 1.0, 0.0);
  const double b = fmin(floor(hi - o - 0.5) + 1.0, (double)n - 1.0);
  if (a <= b) { k0 = (int)a; k1 = (int)b; }
}

#pragma clang fp contract(off)
// One edge u -> v of a quad, seen from the sample row at height py.  It counts
// in the winding number when it crosses the row by the half-open rule (starts
// at or below py and ends above it, or the reverse); then its contribution at
// a sample px is dir (+1 going up, -1 going down) when
//   side = (vx - ux) * (py - uy) - (px - ux) * (vy - uy)
// is > 0 (up) or < 0 (down).  side is monotone in px with the sign of -dir,
// also in rounded FP64, so along the row the edge contributes for the samples
// below one flip index and not from it on.
struct CovEdge {
  double ux, dx, dy, t1;  // t1 = (vx - ux) * (py - uy)
  float xc;               // where it crosses the row (FP32 estimate)
  int dir;                // 0: does not cross the row
};

__device__ __forceinline__ CovEdge cov_edge(float ux, float uy, float vx, float vy, double py) {
  CovEdge e;
  e.ux = ux; e.dx = (double)vx - (double)ux; e.dy = (double)vy - (double)uy;
  e.t1 = e.dx * (py - (double)uy);
  e.dir = ((double)uy <= py) == ((double)vy <= py) ? 0 : ((double)uy <= py ? 1 : -1);
  e.xc = ux + ((float)py - uy) * ((vx - ux) / (vy - uy));
  return e;
}

__device__ __forceinline__ bool cov_contrib(const CovEdge& e, double px) {
  const double side = e.t1 - (px - e.ux) * e.dy;
  return e.dir > 0 ? side > 0 : side < 0;
}

// The flip index of a crossing edge on a row of W samples (sample k at
// x0 + k + 1/2): the smallest k in [0, W] from which the edge no longer
// contributes.  The crossing estimate is corrected by exact tests, with a
// bisection when it is further off than a few samples.
__device__ int cov_flip(const CovEdge& e, double x0, int W) {
  const double g = ceil((double)e.xc - x0 - 0.5);
  int k = isfinite(g) ? (int)fmin(fmax(g, 0.0), (double)W) : 0;
  int steps = 0;
  if (k > 0 && !cov_contrib(e, x0 + (k - 1) + 0.5)) {
    do { --k; ++steps; } while (k > 0 && steps < 8 && !cov_contrib(e, x0 + (k - 1) + 0.5));
    if (k > 0 && !cov_contrib(e, x0 + (k - 1) + 0.5)) steps = 99;
  } else if (k < W && cov_contrib(e, x0 + k + 0.5)) {
    do { ++k; ++steps; } while (k < W && steps < 8 && cov_contrib(e, x0 + k + 0.5));
    if (k < W && cov_contrib(e, x0 + k + 0.5)) steps = 99;
  }
  if (steps == 99 || !isfinite(g)) {
    int lo = 0, hi = W;
    while (lo < hi) {
      const int m = (lo + hi) >> 1;
      if (cov_contrib(e, x0 + m + 0.5)) lo = m + 1; else hi = m;
    }
    k = lo;
  }
  return k;
}
#pragma clang fp contract(on)

// Covered sample intervals of one row: the winding number at sample k is the
// sum of dir over the crossing edges whose flip index exceeds k, constant
// between sorted flip indices; a quad has 0, 2 or 4 crossing edges, so at most
// two maximal runs of nonzero winding.  Written as [a1, a1+n1) and [a2, a2+n2).
__device__ __forceinline__ void cov_add_run(int a, int b, int& a1, int& n1, int& a2, int& n2) {
  if (b <= a) return;
  if (n1 == 0) { a1 = a; n1 = b - a; return; }
  if (a <= a1 + n1 && b >= a1) {              // touches or overlaps the first run
    const int lo = min(a, a1), hi = max(b, a1 + n1);
    a1 = lo; n1 = hi - lo;
    if (n2 > 0 && a2 <= a1 + n1) {            // may now reach the second one
      const int h2 = max(a1 + n1, a2 + n2);
      n1 = h2 - a1; n2 = 0;
    }
    return;
  }
  if (n2 == 0) { a2 = a; n2 = b - a; }
  else { const int lo = min(a, a2), hi = max(b, a2 + n2); a2 = lo; n2 = hi - lo; }
  if (a2 < a1) { const int t = a1, u = n1; a1 = a2; n1 = n2; a2 = t; n2 = u; }
}

template <int N>
__device__ __forceinline__ void cov_runs(const CovEdge* e, double x0, int W, int& a1, int& n1, int& a2,
                                         int& n2) {
  int k[N], d[N], m = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    k[i] = 0; d[i] = 0;
    if (e[i].dir != 0) { k[i] = cov_flip(e[i], x0, W); d[i] = e[i].dir; ++m; }
  }
  // winding just below each flip index: runs between consecutive indices
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if (d[i] == 0) continue;
    int w = 0, nxt = W + 1;
#pragma unroll
    for (int t = 0; t < N; ++t)
      if (d[t] != 0) {
        if (k[t] > k[i] || (k[t] == k[i] && t > i)) { if (k[t] < nxt) nxt = k[t]; }
        if (k[t] > k[i]) w += d[t];
      }
    if (w != 0 && nxt <= W) cov_add_run(k[i], nxt, a1, n1, a2, n2);
  }
  (void)m;
}

// Smallest lane whose inclusive prefix exceeds k (every lane's prefix is in v).
__device__ __forceinline__ int cov_owner(int v, int k) {
  int a = 0, b = 63;
#pragma unroll
  for (int it = 0; it < 6; ++it) {
    const int m = (a + b) >> 1;
    if (__shfl(v, m, 64) > k) b = m; else a = m + 1;
  }
  return a;
}

// Inclusive sum and max over the wavefront on the DPP paths (rows of 16 lanes,
// then row broadcasts); lanes outside a step's source read 0, the identity of
// both (the values here are >= 0).
__device__ __forceinline__ int dpp_incl_sum(int v) {
  v += dpp_i32<0x111, 0xf>(v); v += dpp_i32<0x112, 0xf>(v);
  v += dpp_i32<0x114, 0xf>(v); v += dpp_i32<0x118, 0xf>(v);
  v += dpp_i32<0x142, 0xa>(v); v += dpp_i32<0x143, 0xc>(v);
  return v;
}
__device__ __forceinline__ int dpp_incl_max(int v) {
  v = max(v, dpp_i32<0x111, 0xf>(v)); v = max(v, dpp_i32<0x112, 0xf>(v));
  v = max(v, dpp_i32<0x114, 0xf>(v)); v = max(v, dpp_i32<0x118, 0xf>(v));
  v = max(v, dpp_i32<0x142, 0xa>(v)); v = max(v, dpp_i32<0x143, 0xc>(v));
  return v;
}

constexpr int kCovWaves = 4;   // wavefronts per workgroup
// A lane takes a group of kCovGroup consecutive samples of one row run, so
// that laying the samples out over the lanes is paid once per group; chunks
// of 64 groups per round whose canvas reads overlap
constexpr int kCovGroup = 4;
constexpr int kCovChunks = 1;

// One wavefront per 64 consecutive quads, taken from the end of the rib
// stream so that later paths land first and most samples need no atomic.
// The rows of the 64 quads are spread over the lanes by a prefix sum; each
// row lane finds the row's covered samples exactly (the flip index of every
// crossing edge, by the same FP64 side test a per-sample evaluation makes)
// as at most two runs.  The runs of 64 rows are then cut into groups of
// kCovGroup consecutive samples, laid end to end and taken 64 groups at a
// time: every row marks where its groups start in a per-wave LDS slot array,
// a max-scan over the marks gives each lane its row, and the lane reads,
// compares and raises the group's canvas words.
template <int MODE>
__global__ void __launch_bounds__(256) coverage_kernel(CovArgs A) {
  __shared__ int mark[kCovWaves][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t R = min(A.n_ribs, A.off[A.n_links]);
  const int64_t Q = R - 1;                      // quads r = 0 .. R-2
  const int64_t waves = (Q + 63) / 64;
  const int64_t wstride = (int64_t)gridDim.x * kCovWaves;
  for (int64_t w = (int64_t)blockIdx.x * kCovWaves + wv; w < waves; w += wstride) {
    const int64_t r = Q - 1 - (w * 64 + lane);
    float x[4] = {0, 0, 0, 0}, y[4] = {0, 0, 0, 0};
    int p = -1, j0 = 0, nrows = 0;
    if (r >= 0) {
      const int64_t l = link_of_rib(A.off, A.n_links, r), l2 = link_of_rib(A.off, A.n_links, r + 1);
      const int pa = path_of_link(A.seg_begin, A.n_paths, l), pb = path_of_link(A.seg_begin, A.n_paths, l2);
      const int64_t f = 2 * (int64_t)A.seg_begin[pa] + pa;
      const bool seg_a = ((l - f) & 1) == 1, seg_b = ((l2 - f) & 1) == 1;
      if (pa == pb && (l == l2 || !(seg_a && seg_b))) {
        const float2 ax = *reinterpret_cast<const float2*>(A.vx + 2 * r);
        const float2 ay = *reinterpret_cast<const float2*>(A.vy + 2 * r);
        const float2 bx = *reinterpret_cast<const float2*>(A.vx + 2 * r + 2);
        const float2 by = *reinterpret_cast<const float2*>(A.vy + 2 * r + 2);
        x[0] = ax.x; y[0] = ay.x; x[1] = ax.y; y[1] = ay.y;   // N_r, P_r
        x[2] = bx.y; y[2] = by.y; x[3] = bx.x; y[3] = by.x;   // P_{r+1}, N_{r+1}
        const double yl = fmin(fmin(y[0], y[1]), fmin(y[2], y[3]));
        const double yh = fmax(fmax(y[0], y[1]), fmax(y[2], y[3]));
        const double xl = fmin(fmin(x[0], x[1]), fmin(x[2], x[3]));
        const double xh = fmax(fmax(x[0], x[1]), fmax(x[2], x[3]));
        int i0, i1, j1;
        cov_range(xl, xh, A.x0, A.W, i0, i1);
        cov_range(yl, yh, A.y0, A.H, j0, j1);
        if (i1 >= i0 && j1 >= j0) { p = pa; nrows = j1 - j0 + 1; }
      }
    }
    const int incl = dpp_incl_sum(nrows);
    const int total = __shfl(incl, 63, 64);
    for (int base = 0; base < total; base += 64) {
      // this lane's row: row k of the wave's rows
      const int k = base + lane;
      const int o = cov_owner(incl, k);
      float qx[4], qy[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) { qx[c] = __shfl(x[c], o, 64); qy[c] = __shfl(y[c], o, 64); }
      const int qp = __shfl(p, o, 64);
      const int j = __shfl(j0, o, 64) + (k - (__shfl(incl, o, 64) - __shfl(nrows, o, 64)));
      int a1 = 0, n1 = 0, a2 = 0, n2 = 0;
      if (k < total) {
        const double py = A.y0 + j + 0.5;
        if (MODE == 0) {
          CovEdge e[4] = {cov_edge(qx[0], qy[0], qx[1], qy[1], py), cov_edge(qx[1], qy[1], qx[2], qy[2], py),
                          cov_edge(qx[2], qy[2], qx[3], qy[3], py), cov_edge(qx[3], qy[3], qx[0], qy[0], py)};
          cov_runs<4>(e, A.x0, A.W, a1, n1, a2, n2);
        } else {
          CovEdge t1[3] = {cov_edge(qx[0], qy[0], qx[1], qy[1], py), cov_edge(qx[1], qy[1], qx[2], qy[2], py),
                           cov_edge(qx[2], qy[2], qx[0], qy[0], py)};
          CovEdge t2[3] = {cov_edge(qx[0], qy[0], qx[2], qy[2], py), cov_edge(qx[2], qy[2], qx[3], qy[3], py),
                           cov_edge(qx[3], qy[3], qx[0], qy[0], py)};
          cov_runs<3>(t1, A.x0, A.W, a1, n1, a2, n2);
          cov_runs<3>(t2, A.x0, A.W, a1, n1, a2, n2);
        }
      }
      // this row's runs [a1, a1 + n1) and [a2, a2 + n2) make g1 + g2 groups,
      // positions [st, st + g1 + g2) of the wave's laid-out groups; group g
      // starts at canvas word c + G g (c = c1 before bnd, else c2) and ends
      // at its run's end e1 or e2
      constexpr int G = kCovGroup;
      const int g1 = (n1 + G - 1) / G, g2 = (n2 + G - 1) / G, ng = g1 + g2;
      const int incl2 = dpp_incl_sum(ng);
      const int total2 = __shfl(incl2, 63, 64);
      const int st = incl2 - ng, bnd = st + g1;
      const int rowbase = j * A.W;
      const int c1 = rowbase + a1 - G * st, c2 = rowbase + a2 - G * bnd;
      const int e1 = rowbase + a1 + n1, e2 = rowbase + a2 + n2;
      // kCovChunks chunks of 64 groups per round, so that their canvas reads
      // are all in flight before any result is needed
      int carry = 0;
      for (int base2 = 0; base2 < total2; base2 += 64 * kCovChunks) {
        int w0[kCovChunks], wl[kCovChunks], sp[kCovChunks];
        bool act[kCovChunks];
#pragma unroll
        for (int u = 0; u < kCovChunks; ++u) {
          const int b2 = base2 + 64 * u;
          mark[wv][lane] = 0;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          if (ng > 0 && st >= b2 && st < b2 + 64) mark[wv][st - b2] = lane + 1;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          const int m = dpp_incl_max(mark[wv][lane]);
          const int o2 = m > 0 ? m - 1 : carry;
          carry = __shfl(o2, 63, 64);
          const int g = b2 + lane;
          const int sb = __shfl(bnd, o2, 64);
          const int s1 = __shfl(c1, o2, 64), s2 = __shfl(c2, o2, 64);
          const int t1 = __shfl(e1, o2, 64), t2 = __shfl(e2, o2, 64);
          sp[u] = __shfl(qp, o2, 64);
          act[u] = g < total2;
          w0[u] = (g < sb ? s1 : s2) + G * g;   // first word of the group
          wl[u] = (g < sb ? t1 : t2) - 1;       // last word of its run
          __builtin_amdgcn_wave_barrier();
        }
        // unconditional reads (a lane past the end reads word 0; a short
        // group re-reads its run's last word), so that none waits inside a
        // branch of its own
        int cur[kCovChunks][G];
#pragma unroll
        for (int u = 0; u < kCovChunks; ++u)
#pragma unroll
          for (int k = 0; k < G; ++k) cur[u][k] = A.top[act[u] ? min(w0[u] + k, wl[u]) : 0];
        // values only grow, so a stale read costs at most a redundant atomic
#pragma unroll
        for (int u = 0; u < kCovChunks; ++u)
#pragma unroll
          for (int k = 0; k < G; ++k)
            if (act[u] && w0[u] + k <= wl[u] && cur[u][k] < sp[u]) atomicMax(A.top + w0[u] + k, sp[u]);
      }
    }
  }
}

// ===========================================================================
// Dash (Sec. "Dashing").  Boundary positions, pattern states and the
// interpolation are plain IEEE operations without FMA contraction, so a given
// rib stream is cut at the same places whoever computes it.
// ===========================================================================
#pragma clang fp contract(off)
struct DashArgs {
  const int64_t* off;        // link offsets [n_links+1]
  int64_t n_links;
  const int32_t* seg_begin;
  int n_paths;
  const float* vx;
  const float* vy;
  const float* vs;
  int32_t* cnt_r;            // per rib: ribs written
  int32_t* cnt_d;            // per rib: dashes started
  const int64_t* rib_pos;    // exclusive scans of the two
  const int64_t* dash_pos;
  float* dx;
  float* dy;
  float* ds;
  int64_t* range;
  int64_t rib_cap;
  int64_t dash_cap;
  int64_t max_ribs;          // ribs the input stream (and the per-rib scratch) can hold
  DevStatus* st;
  double phase;
  int n_pat;
  double cum[kMaxDash + 1];  // cumulative pattern, cum[n_pat] = period
};

__device__ __forceinline__ int64_t path_first_rib(const DashArgs& A, int p) {
  return A.off[2 * (int64_t)A.seg_begin[p] + p];
}

__device__ __forceinline__ int rib_path(const DashArgs& A, int64_t r) {
  // largest p whose first rib is <= r
  int a = 0, b = A.n_paths - 1;
  while (a < b) {
    const int m = (a + b + 1) >> 1;
    if (path_first_rib(A, m) <= r) a = m; else b = m - 1;
  }
  return a;
}

// pattern state at position u: "on" when u mod period lies in an even entry
__device__ __forceinline__ bool dash_on(const DashArgs& A, double u) {
  const double per = A.cum[A.n_pat];
  const double m = floor(u / per);
  const double x = u - m * per;
  int idx = 0;
  while (idx + 1 < A.n_pat && A.cum[idx + 1] <= x) ++idx;
  return (idx & 1) == 0;
}

// visit the boundaries u_b = m*period + cum[i] with u0 < u_b <= u1 in order.
// Steps longer than kMaxDashPeriods periods, steps ending kMaxDashU periods or
// more into the pattern, and non-finite ones are left undashed (and flagged):
// below kMaxDashU periods the period index m stays exact and u_b grows by at
// least 3/4 of a period per step of m, so the loop always ends.
constexpr double kMaxDashPeriods = 1048576.0;            // 2^20
constexpr double kMaxDashU = 1125899906842624.0;         // 2^50

template <class Fn>
__device__ __forceinline__ void dash_boundaries(const DashArgs& A, double u0, double u1, Fn fn) {
  if (!(u1 > u0)) return;
  const double per = A.cum[A.n_pat];
  if (!isfinite(u0) || !isfinite(u1) || (u1 - u0) > kMaxDashPeriods * per || !(u1 < kMaxDashU * per)) {
    atomicOr(&A.st->flags, (unsigned)PS_STATUS_DASH_OVERFLOW);
    return;
  }
  for (double m = floor(u0 / per);; m += 1.0) {
    for (int i = 0; i < A.n_pat; ++i) {
      const double ub = m * per + A.cum[i];
      if (ub <= u0) continue;
      if (ub > u1) return;
      fn(ub);
    }
  }
}

// Each ps_dash reports its own totals and overflow: clear them first (the
// other status bits belong to the count and emit of the same workspace).
__global__ void reset_dash_status_kernel(DevStatus* st) {
  if (threadIdx.x == 0) {
    atomicAnd(&st->flags, ~(unsigned)PS_STATUS_DASH_OVERFLOW);
    st->dash_ribs = 0;
    st->dash_count = 0;
  }
}

// The rib stream holds R = offsets[n_links] ribs; if that exceeds the vertex
// capacity the workspace was sized with (the emit overflowed), nothing is
// read or written and the dash reports an overflow.
__device__ __forceinline__ bool dash_input_fits(const DashArgs& A, int64_t R) {
  if (R <= A.max_ribs) return true;
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&A.st->flags, (unsigned)PS_STATUS_DASH_OVERFLOW);
  return false;
}

__global__ void __launch_bounds__(256) dash_count_kernel(DashArgs A) {
  const int64_t R = A.off[A.n_links];
  if (!dash_input_fits(A, R)) return;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int p = rib_path(A, r);
    const double u1 = (double)A.vs[2 * r] + A.phase;
    int ribs = 0, starts = 0;
    if (r == path_first_rib(A, p)) {
      if (dash_on(A, u1)) { ribs = 1; starts = 1; }
    } else {
      const double u0 = (double)A.vs[2 * (r - 1)] + A.phase;
      bool on = dash_on(A, u0);
      dash_boundaries(A, u0, u1, [&](double) {
        ++ribs;           // every boundary rib is written
        on = !on;
        if (on) ++starts; // a boundary that turns the pattern on starts a dash
      });
      if (on) ++ribs;
    }
    A.cnt_r[r] = ribs;
    A.cnt_d[r] = starts;
  }
}

__global__ void __launch_bounds__(256) dash_emit_kernel(DashArgs A) {
  const int64_t R = A.off[A.n_links];
  if (!dash_input_fits(A, R)) return;
  const int64_t tot_r = A.rib_pos[R], tot_d = A.dash_pos[R];
  const int64_t tid0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool over = tot_r > A.rib_cap || tot_d > A.dash_cap;
  if (tid0 == 0) {
    A.st->dash_ribs = (unsigned long long)tot_r;
    A.st->dash_count = (unsigned long long)tot_d;
    if (over) atomicOr(&A.st->flags, (unsigned)PS_STATUS_DASH_OVERFLOW);
  }
  if (over) return;
  for (int64_t r = tid0; r < R; r += (int64_t)gridDim.x * blockDim.x) {
    const int p = rib_path(A, r);
    int64_t o = A.rib_pos[r];
    int64_t dn = A.dash_pos[r];   // next dash index to open; dn-1 is the one running
    const float s1 = A.vs[2 * r];
    const double u1 = (double)s1 + A.phase;
    auto put = [&](float nx, float ny, float px, float py, float s) {
      A.dx[2 * o] = nx; A.dy[2 * o] = ny; A.dx[2 * o + 1] = px; A.dy[2 * o + 1] = py;
      A.ds[2 * o] = s; A.ds[2 * o + 1] = s;
      ++o;
    };
    bool on;
    if (r == path_first_rib(A, p)) {
      on = dash_on(A, u1);
      if (on) { A.range[2 * dn] = o; ++dn; put(A.vx[2 * r], A.vy[2 * r], A.vx[2 * r + 1], A.vy[2 * r + 1], s1); }
    } else {
      const double u0 = (double)A.vs[2 * (r - 1)] + A.phase;
      on = dash_on(A, u0);
      const double nx0 = A.vx[2 * (r - 1)], ny0 = A.vy[2 * (r - 1)];
      const double px0 = A.vx[2 * (r - 1) + 1], py0 = A.vy[2 * (r - 1) + 1];
      const double nx1 = A.vx[2 * r], ny1 = A.vy[2 * r], px1 = A.vx[2 * r + 1], py1 = A.vy[2 * r + 1];
      dash_boundaries(A, u0, u1, [&](double ub) {
        const double lam = (ub - u0) / (u1 - u0);
        const float bnx = (float)(nx0 + lam * (nx1 - nx0)), bny = (float)(ny0 + lam * (ny1 - ny0));
        const float bpx = (float)(px0 + lam * (px1 - px0)), bpy = (float)(py0 + lam * (py1 - py0));
        const float sb = (float)(ub - A.phase);
        if (on) {
          put(bnx, bny, bpx, bpy, sb);
          A.range[2 * (dn - 1) + 1] = o;   // the running dash ends here
          on = false;
        } else {
          A.range[2 * dn] = o;             // a new dash starts here
          ++dn;
          put(bnx, bny, bpx, bpy, sb);
          on = true;
        }
      });
      if (on) put(A.vx[2 * r], A.vy[2 * r], A.vx[2 * r + 1], A.vy[2 * r + 1], s1);
    }
    // a dash still on at the last rib of its path ends there
    const int64_t path_end = A.off[2 * (int64_t)A.seg_begin[p + 1] + p + 1];
    if (on && r + 1 == path_end) A.range[2 * (dn - 1) + 1] = o;
  }
}

#pragma clang fp contract(on)

}  // namespace

// ===========================================================================
// Host side
// ===========================================================================
namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define PS_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return fail(PS_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// An emit mapping: PS_MAP_TILES (K ribs per lane) or PS_MAP_LINKS, and the
// wavefronts per workgroup.
struct EmitConfig {
  int map = PS_MAP_TILES;
  int K = 7;
  int waves = 4;
};

int64_t n_links_of(const ps_batch* b) { return 2 * (int64_t)b->n_segs + b->n_paths; }

bool valid_k(int K) { return K == 4 || K == 6 || K == 7 || K == 8 || K == 16; }

// The mapping of an unplanned call (or of a plan told its mapping).
EmitConfig config_of(const ps_params* p) {
  EmitConfig c;
  if (p->emit_mapping == PS_MAP_LINKS) c.map = PS_MAP_LINKS;
  if (p->emit_ribs_per_lane) c.K = p->emit_ribs_per_lane;
  if (p->emit_waves) c.waves = p->emit_waves;
  return c;
}

int check_batch(const ps_batch* b) {
  if (!b) return fail(PS_E_ARG, "batch is NULL");
  if (b->n_paths < 0 || b->n_segs < 0) return fail(PS_E_ARG, "negative path or segment count");
  if (n_links_of(b) >= (int64_t)INT32_MAX)
    return fail(PS_E_ARG, "too many links (2*n_segs + n_paths must be < 2^31)");
  if (!b->seg_begin) return fail(PS_E_ARG, "seg_begin is NULL");
  if (b->n_segs > 0 && b->n_paths == 0) return fail(PS_E_ARG, "segments without paths");
  if (b->n_segs > 0 && (!b->kind || !b->cx || !b->cy || !b->conic_w))
    return fail(PS_E_ARG, "segment arrays must not be NULL");
  if (b->n_paths > 0 && (!b->width || !b->join || !b->cap))
    return fail(PS_E_ARG, "path arrays must not be NULL");
  return PS_OK;
}

int check_params(const ps_params* p) {
  if (!p) return fail(PS_E_ARG, "params is NULL");
  if (!(p->q >= 1e-4 && p->q <= M_PI)) return fail(PS_E_ARG, "q must be in [1e-4, pi] (got %g)", p->q);
  if (p->precision < PS_PREC_FP32 || p->precision > PS_PREC_FP64)
    return fail(PS_E_ARG, "unknown precision mode %d", p->precision);
  if (!(p->miter_limit >= 1.0) || !std::isfinite(p->miter_limit))
    return fail(PS_E_ARG, "miter_limit must be finite and >= 1 (got %g)", p->miter_limit);
  if (p->emit_mapping < PS_MAP_DEFAULT || p->emit_mapping > PS_MAP_LINKS)
    return fail(PS_E_ARG, "unknown emit mapping %d", p->emit_mapping);
  if (p->emit_ribs_per_lane != 0 && !valid_k(p->emit_ribs_per_lane))
    return fail(PS_E_ARG, "emit_ribs_per_lane must be 0, 4, 6, 7, 8 or 16");
  if (p->emit_waves < 0 || p->emit_waves > 4)
    return fail(PS_E_ARG, "emit_waves must be in [0, 4] (at most 256 threads per workgroup)");
  if (p->n_dash != 0) {
    if (p->n_dash < 2 || (p->n_dash & 1) || p->n_dash > kMaxDash)
      return fail(PS_E_ARG, "dash pattern needs an even count in [2, %d]", kMaxDash);
    if (!p->dash) return fail(PS_E_ARG, "dash pattern is NULL");
    double sum = 0;
    for (int i = 0; i < p->n_dash; ++i) {
      if (!(p->dash[i] >= 0) || !std::isfinite(p->dash[i]))
        return fail(PS_E_ARG, "dash entries must be finite and >= 0");
      sum += p->dash[i];
    }
    if (!(sum > 0)) return fail(PS_E_ARG, "dash pattern sums to zero");
    if (!(p->dash_phase >= 0) || !std::isfinite(p->dash_phase))
      return fail(PS_E_ARG, "dash phase must be finite and >= 0");
    if (!(p->dash_phase <= kMaxDashPhase * sum))
      return fail(PS_E_ARG, "dash phase must be at most 2^40 pattern periods");
  }
  return PS_OK;
}

int check_ws(const void* ws, size_t have, size_t need) {
  if (!ws) return fail(PS_E_ARG, "workspace is NULL");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(PS_E_ARG, "workspace must be 256-byte aligned");
  if (have < need) return fail(PS_E_WORKSPACE, "workspace has %zu bytes, needs %zu", have, need);
  return PS_OK;
}

struct WsView {
  DevStatus* st;
  v4u32* head;
  v4u32* tail;
  double2* seg_ang;   // per segment: start and end tangent angles (usable segments)
  uint8_t* seg_ok;    // per segment: state (usable, or the status bit its problem raises)
  long long* scan;
  int32_t* tile_link;
  unsigned long long* desc;
  int32_t* dash_r;
  int32_t* dash_d;
  int64_t* dash_rpos;
  int64_t* dash_dpos;
  long long* dash_scan;
};

WsView ws_view(void* ws, const WsLayout& w) {
  char* b = (char*)ws;
  WsView v;
  v.st = (DevStatus*)(b + w.status);
  v.head = (v4u32*)(b + w.rec_head);
  v.tail = (v4u32*)(b + w.rec_tail);
  v.seg_ang = (double2*)(b + w.seg_ang);
  v.seg_ok = (uint8_t*)(b + w.seg_ok);
  v.scan = (long long*)(b + w.scan);
  v.tile_link = (int32_t*)(b + w.tile_link);
  v.desc = (unsigned long long*)(b + w.desc);
  v.dash_r = (int32_t*)(b + w.dash_r);
  v.dash_d = (int32_t*)(b + w.dash_d);
  v.dash_rpos = (int64_t*)(b + w.dash_rpos);
  v.dash_dpos = (int64_t*)(b + w.dash_dpos);
  v.dash_scan = (long long*)(b + w.dash_scan);
  return v;
}

int grid_for(int64_t n, int threads) {
  const int64_t g = (n + threads - 1) / threads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 20));
}

int num_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
      cus = p.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

// blocks of the one-pass link scan: one per kLinkScanTile links, plus the one
// that owns position n_links
int64_t link_scan_blocks(int64_t n_links) { return n_links / kLinkScanTile + 1; }

// The one-pass link scan of a count -> scan -> emit chain (after the count
// kernel, which clears its look-back words), with the tile table of the
// emit of configuration c when c.K > 0.
int do_link_scan(const int32_t* link_ribs, int64_t L, int64_t* off, const WsView& v, const WsLayout& w,
                 int64_t cap, int K, hipStream_t s) {
  LinkScanArgs a;
  a.link_ribs = link_ribs; a.n = L; a.off = off; a.desc = (unsigned long long*)v.scan; a.st = v.st;
  a.TS = 64 * K; a.tile_link = v.tile_link; a.tile_desc = v.desc; a.capacity = cap;
  a.max_tiles = w.max_tiles;
  hipLaunchKernelGGL(link_scan_kernel, dim3((unsigned)link_scan_blocks(L)), dim3(kLinkScanThreads), 0, s, a);
  PS_HIP(hipGetLastError());
  return PS_OK;
}

int do_scan_i32(const int32_t* in, int64_t n_max, const int64_t* n_dev, int64_t* out,
                long long* scratch, unsigned long long* total, hipStream_t s) {
  const int64_t nb = std::max<int64_t>(1, (n_max + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(scan_reduce_kernel<int32_t>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in,
                     n_max, n_dev, scratch);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(1024), 0, s, scratch, nb);
  hipLaunchKernelGGL(scan_apply_kernel<int32_t>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in,
                     n_max, n_dev, (const long long*)scratch, out, nb, total);
  PS_HIP(hipGetLastError());
  return PS_OK;
}

// PS_MAP_TILES (the role-split walk of rib tiles) and PS_MAP_LINKS (one link
// per wavefront iteration), both over tiles of 64*K ribs.
template <int MAP, int K, int PREC, bool WXY, bool WS>
void emit_launcher(EmitArgs a, int grid, int block, hipStream_t s) {
  // above 64 KiB of dynamic LDS a kernel has to be allowed it once (every
  // configuration is first launched eagerly, before any graph capture)
  if constexpr (MAP == PS_MAP_TILES) {
    const size_t lds = (size_t)(block / 64) * emit_split_lds_per_wave(K, WS);
    static const hipError_t allowed = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&emit_split_kernel<K, PREC, WXY, WS>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)(4 * emit_split_lds_per_wave(K, WS)));
    (void)allowed;
    hipLaunchKernelGGL((emit_split_kernel<K, PREC, WXY, WS>), dim3(grid), dim3(block), lds, s, a);
  } else {
    const size_t lds = (size_t)(block / 64) * emit_links_lds_per_wave(K, WS);
    static const hipError_t allowed = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&emit_links_kernel<K, PREC, WXY, WS>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)(4 * emit_links_lds_per_wave(K, WS)));
    (void)allowed;
    hipLaunchKernelGGL((emit_links_kernel<K, PREC, WXY, WS>), dim3(grid), dim3(block), lds, s, a);
  }
}

using EmitLaunch = void (*)(EmitArgs, int, int, hipStream_t);

template <int MAP, int PREC, bool WXY, bool WS>
EmitLaunch pick_k(int K) {
  switch (K) {
    case 4: return emit_launcher<MAP, 4, PREC, WXY, WS>;
    case 6: return emit_launcher<MAP, 6, PREC, WXY, WS>;
    case 7: return emit_launcher<MAP, 7, PREC, WXY, WS>;
    case 8: return emit_launcher<MAP, 8, PREC, WXY, WS>;
    case 16: return emit_launcher<MAP, 16, PREC, WXY, WS>;
    default: return nullptr;
  }
}

template <int MAP, bool WXY, bool WS>
EmitLaunch pick_prec(int prec, int K) {
  switch (prec) {
    case PS_PREC_FP32: return pick_k<MAP, PS_PREC_FP32, WXY, WS>(K);
    case PS_PREC_FP32_FIXUP: return pick_k<MAP, PS_PREC_FP32_FIXUP, WXY, WS>(K);
    default: return pick_k<MAP, PS_PREC_FP64, WXY, WS>(K);
  }
}

template <int MAP>
EmitLaunch pick_mode(int prec, int K, bool wxy, bool ws) {
  if (wxy && ws) return pick_prec<MAP, true, true>(prec, K);
  if (wxy) return pick_prec<MAP, true, false>(prec, K);
  return pick_prec<MAP, false, true>(prec, K);
}

EmitLaunch pick_emit(int map, int prec, int K, bool wxy, bool ws) {
  if (map == PS_MAP_LINKS) return pick_mode<PS_MAP_LINKS>(prec, K, wxy, ws);
  return pick_mode<PS_MAP_TILES>(prec, K, wxy, ws);
}

// Largest Newton step (in t) accepted when polishing an FP32 root in FP64;
// a larger step means the FP32 root was ill-conditioned and the rib is
// re-solved in FP64.  PS_FIXUP_TOL overrides it, for precision studies.
float fixup_tolerance() {
  static float tol = [] {
    const char* e = getenv("PS_FIXUP_TOL");
    const float v = e ? (float)atof(e) : 0.0f;
    return v > 0 ? v : 1e-4f;
  }();
  return tol;
}

int launch_count(const ps_batch* b, const ps_params* p, int32_t* link_ribs, const WsView& v,
                 hipStream_t s) {
  // the angles pass resets the status word; without segments a kernel of its own does
  if (b->n_segs == 0) hipLaunchKernelGGL(reset_status_kernel, dim3(1), dim3(64), 0, s, v.st);
  const int64_t n = (int64_t)b->n_segs + b->n_paths;
  if (n > 0) {
    CountArgs a{*b, p->q, link_ribs, v.head, v.tail, v.seg_ang, v.seg_ok, v.st, (unsigned long long*)v.scan,
                link_scan_blocks(n_links_of(b))};
    // the setup in FP64, or in FP32 for the single-precision study mode
    const bool f32 = p->precision == PS_PREC_FP32;
    if (b->n_segs > 0)
      hipLaunchKernelGGL(f32 ? count_angles_kernel<float> : count_angles_kernel<double>,
                         dim3((unsigned)((b->n_segs + 255) / 256)), dim3(256), 0, s, a);
    // workgroups of segments, then of paths (launch bound kCountThreads)
    const int64_t blocks = ((int64_t)b->n_segs + kCountThreads - 1) / kCountThreads +
                           ((int64_t)b->n_paths + kCountThreads - 1) / kCountThreads;
    hipLaunchKernelGGL(f32 ? count_kernel<float> : count_kernel<double>, dim3((unsigned)blocks),
                       dim3(kCountThreads), 0, s, a);
  }
  PS_HIP(hipGetLastError());
  return PS_OK;
}

// `prepared`: the tile table of configuration c is already written (by the
// one-pass link scan of the same chain).
int launch_emit(const ps_batch* b, const ps_params* p, const int64_t* off, float* vx, float* vy,
                float* vs, int64_t cap, const WsView& v, const WsLayout& w, const EmitConfig& c,
                hipStream_t s, bool prepared = false) {
  const int64_t L = n_links_of(b);
  const int TS = 64 * c.K;
  EmitLaunch fn = pick_emit(c.map, p->precision, c.K, vx != nullptr, vs != nullptr);
  if (!fn) return fail(PS_E_ARG, "unsupported emit configuration K=%d", c.K);
  if (c.waves < 1 || c.waves > 4) return fail(PS_E_ARG, "waves_per_group must be in [1,4]");
  if (!prepared) {
    const unsigned prep_grid = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (L + 255) / 256), 8192);
    hipLaunchKernelGGL(emit_prepare_kernel, dim3(prep_grid), dim3(256), 0, s, off, L, TS, v.tile_link,
                       v.desc, v.st, cap, w.max_tiles);
  }
  EmitArgs a;
  a.head = v.head; a.tail = v.tail; a.off = off; a.n_links = L; a.vx = vx; a.vy = vy; a.vs = vs;
  a.capacity = cap; a.tile_link = v.tile_link; a.desc = v.desc; a.st = v.st;
  a.max_tiles = w.max_tiles;
  a.fix_tol = fixup_tolerance();
  a.miter_limit = p->miter_limit;
  const int block = 64 * c.waves;   // never above the kernel's launch bound of 256
  const int grid = num_cus() * (16 / c.waves);
  fn(a, grid, block, s);
  PS_HIP(hipGetLastError());
  return PS_OK;
}

int launch_dash(const ps_batch* b, const ps_params* p, const int64_t* off, const float* vx,
                const float* vy, const float* vs, float* dx, float* dy, float* ds, int64_t* range,
                int64_t rib_cap, int64_t dash_cap, const WsView& v, const WsLayout& w,
                hipStream_t s) {
  DashArgs a;
  a.off = off; a.n_links = n_links_of(b); a.seg_begin = b->seg_begin; a.n_paths = b->n_paths;
  a.vx = vx; a.vy = vy; a.vs = vs; a.cnt_r = v.dash_r; a.cnt_d = v.dash_d;
  a.rib_pos = v.dash_rpos; a.dash_pos = v.dash_dpos;
  a.dx = dx; a.dy = dy; a.ds = ds; a.range = range; a.rib_cap = rib_cap; a.dash_cap = dash_cap;
  a.max_ribs = w.max_ribs;
  a.st = v.st; a.phase = p->dash_phase; a.n_pat = p->n_dash;
  a.cum[0] = 0;
  for (int i = 0; i < p->n_dash; ++i) a.cum[i + 1] = a.cum[i] + p->dash[i];
  for (int i = p->n_dash + 1; i <= kMaxDash; ++i) a.cum[i] = 0;
  const int grid = num_cus() * 8;
  const int64_t* R_dev = off + a.n_links;
  hipLaunchKernelGGL(reset_dash_status_kernel, dim3(1), dim3(64), 0, s, v.st);
  hipLaunchKernelGGL(dash_count_kernel, dim3(grid), dim3(256), 0, s, a);
  int rc;
  if ((rc = do_scan_i32(v.dash_r, w.max_ribs, R_dev, v.dash_rpos, v.dash_scan, nullptr, s))) return rc;
  if ((rc = do_scan_i32(v.dash_d, w.max_ribs, R_dev, v.dash_dpos, v.dash_scan, nullptr, s))) return rc;
  hipLaunchKernelGGL(dash_emit_kernel, dim3(grid), dim3(256), 0, s, a);
  PS_HIP(hipGetLastError());
  return PS_OK;
}

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};

int static_scratch(void** out) {
  int dev = 0;
  PS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PS_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PS_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_static_ptr[dev] = p;
  }
  *out = g_static_ptr[dev];
  return PS_OK;
}


}  // namespace

// ===========================================================================
// Plan: autotuned emit mapping + one hipGraph for the whole chain
// ===========================================================================
struct ps_plan {
  ps_batch b;
  ps_params p;
  std::vector<double> dash;
  int32_t* link_ribs;
  int64_t* off;
  float *vx, *vy, *vs;
  int64_t cap;
  float *dx, *dy, *ds;
  int64_t* range;
  int64_t dash_rib_cap, dash_cap;
  void* ws;
  WsLayout w;
  EmitConfig cfg;
  // graph[0]: count -> scan -> emit (-> dash).  graph[1]: the same chain with
  // an event-record node between scan and emit and one after the emit; the
  // nodes record the plan's own events unless a timed launch points them at
  // the caller's.  Event nodes add launch latency, so plain launches replay
  // graph[0].
  hipGraph_t graph[2];
  hipGraphExec_t exec[2];
  hipGraphNode_t ev_node[2];
  hipEvent_t ev_own[2];
};

namespace {

int enqueue_count(ps_plan* P, hipStream_t s) {
  const WsView v = ws_view(P->ws, P->w);
  int rc;
  if ((rc = launch_count(&P->b, &P->p, P->link_ribs, v, s))) return rc;
  return do_link_scan(P->link_ribs, n_links_of(&P->b), P->off, v, P->w, P->cap, P->cfg.K, s);
}

int enqueue_emit(ps_plan* P, hipStream_t s) {
  const WsView v = ws_view(P->ws, P->w);
  int rc;
  if ((rc = launch_emit(&P->b, &P->p, P->off, P->vx, P->vy, P->vs, P->cap, v, P->w, P->cfg, s, true)))
    return rc;
  if (P->p.n_dash > 0) {
    if ((rc = launch_dash(&P->b, &P->p, P->off, P->vx, P->vy, P->vs, P->dx, P->dy, P->ds, P->range,
                          P->dash_rib_cap, P->dash_cap, v, P->w, s)))
      return rc;
  }
  return PS_OK;
}

// Appends an event-record node for `ev` to the graph being captured on cs,
// after everything captured so far; later captured work follows it.
int capture_event_node(hipStream_t cs, hipEvent_t ev, hipGraphNode_t* node) {
  hipStreamCaptureStatus st;
  unsigned long long id;
  hipGraph_t g;
  const hipGraphNode_t* deps;
  size_t n_deps;
  PS_HIP(hipStreamGetCaptureInfo_v2(cs, &st, &id, &g, &deps, &n_deps));
  PS_HIP(hipGraphAddEventRecordNode(node, g, deps, n_deps, ev));
  PS_HIP(hipStreamUpdateCaptureDependencies(cs, node, 1, hipStreamSetCaptureDependencies));
  return PS_OK;
}

// Captures the chain on a stream of its own into graph[timed] and
// instantiates it; the timed graph gets the two event-record nodes.
int capture_plan(ps_plan* P, int timed) {
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return fail(PS_E_HIP, "stream");
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return fail(PS_E_HIP, "begin capture failed");
  }
  int rc = enqueue_count(P, cs);
  if (!rc && timed) rc = capture_event_node(cs, P->ev_own[0], &P->ev_node[0]);
  if (!rc) rc = enqueue_emit(P, cs);
  if (!rc && timed) rc = capture_event_node(cs, P->ev_own[1], &P->ev_node[1]);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(cs, &g);
  (void)hipStreamDestroy(cs);
  if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
  if (e != hipSuccess || !g) return fail(PS_E_HIP, "end capture: %s", hipGetErrorString(e));
  P->graph[timed] = g;
  e = hipGraphInstantiate(&P->exec[timed], g, nullptr, nullptr, 0);
  if (e != hipSuccess) return fail(PS_E_HIP, "instantiate: %s", hipGetErrorString(e));
  return PS_OK;
}

int time_emit(ps_plan* P, const EmitConfig& c, hipStream_t s, float* ms) {
  const WsView v = ws_view(P->ws, P->w);
  hipEvent_t e0, e1;
  PS_HIP(hipEventCreate(&e0));
  PS_HIP(hipEventCreate(&e1));
  int rc = launch_emit(&P->b, &P->p, P->off, P->vx, P->vy, P->vs, P->cap, v, P->w, c, s);
  float best = 1e30f;
  for (int rep = 0; rep < 3 && rc == PS_OK; ++rep) {
    (void)hipEventRecord(e0, s);
    rc = launch_emit(&P->b, &P->p, P->off, P->vx, P->vy, P->vs, P->cap, v, P->w, c, s);
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float t = 0;
    (void)hipEventElapsedTime(&t, e0, e1);
    best = std::min(best, t);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = best;
  return rc;
}

}  // namespace

// ===========================================================================
// Public C ABI
// ===========================================================================
extern "C" {

const char* ps_version(void) { return PS_VERSION; }

const char* ps_last_error(void) { return g_err.c_str(); }

int64_t ps_num_links(const ps_batch* b) {
  if (check_batch(b) != PS_OK) return -1;
  return n_links_of(b);
}

size_t ps_workspace_bytes(const ps_batch* b, const ps_params* p, int64_t vertex_capacity) {
  if (check_batch(b) != PS_OK) return 0;
  const int nd = p ? p->n_dash : 0;
  return ws_layout(n_links_of(b), std::max<int64_t>(0, vertex_capacity), nd).total;
}

int ps_count(const ps_batch* b, const ps_params* p, int32_t* link_ribs, void* ws, size_t ws_bytes,
             void* stream) {
  int rc;
  if ((rc = check_batch(b)) || (rc = check_params(p))) return rc;
  if (!link_ribs && n_links_of(b) > 0) return fail(PS_E_ARG, "link_ribs is NULL");
  const WsLayout w = ws_layout(n_links_of(b), 0, 0);
  if ((rc = check_ws(ws, ws_bytes, w.total))) return rc;
  return launch_count(b, p, link_ribs, ws_view(ws, w), (hipStream_t)stream);
}

int ps_scan(const int32_t* link_ribs, int64_t n_links, int64_t* offsets, void* ws, size_t ws_bytes,
            void* stream) {
  if (n_links < 0 || n_links >= (int64_t)INT32_MAX) return fail(PS_E_ARG, "bad n_links");
  if (!offsets || (n_links > 0 && !link_ribs)) return fail(PS_E_ARG, "NULL array");
  const WsLayout w = ws_layout(n_links, 0, 0);
  int rc;
  if ((rc = check_ws(ws, ws_bytes, w.total))) return rc;
  const WsView v = ws_view(ws, w);
  return do_scan_i32(link_ribs, n_links, nullptr, offsets, v.scan, &v.st->total_ribs, (hipStream_t)stream);
}

int ps_emit(const ps_batch* b, const ps_params* p, const int64_t* offsets, float* vx, float* vy,
            float* vs, int64_t cap, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_batch(b)) || (rc = check_params(p))) return rc;
  if (!offsets || !vx || !vy) return fail(PS_E_ARG, "NULL array");
  if (cap < 0) return fail(PS_E_ARG, "negative capacity");
  const WsLayout w = ws_layout(n_links_of(b), cap, 0);
  if ((rc = check_ws(ws, ws_bytes, w.total))) return rc;
  return launch_emit(b, p, offsets, vx, vy, vs, cap, ws_view(ws, w), w, config_of(p), (hipStream_t)stream);
}

int ps_arclen(const ps_batch* b, const ps_params* p, const int64_t* offsets, float* vs, int64_t cap,
              void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_batch(b)) || (rc = check_params(p))) return rc;
  if (!offsets || !vs) return fail(PS_E_ARG, "NULL array");
  if (cap < 0) return fail(PS_E_ARG, "negative capacity");
  const WsLayout w = ws_layout(n_links_of(b), cap, 0);
  if ((rc = check_ws(ws, ws_bytes, w.total))) return rc;
  return launch_emit(b, p, offsets, nullptr, nullptr, vs, cap, ws_view(ws, w), w, config_of(p),
                     (hipStream_t)stream);
}

int ps_emit_uniform(const ps_batch* b, const ps_params* p, const int64_t* offsets, float* vx,
                    float* vy, int64_t cap, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_batch(b)) || (rc = check_params(p))) return rc;
  if (!offsets || !vx || !vy) return fail(PS_E_ARG, "NULL array");
  if (cap < 0) return fail(PS_E_ARG, "negative capacity");
  const WsLayout w = ws_layout(n_links_of(b), cap, 0);
  if ((rc = check_ws(ws, ws_bytes, w.total))) return rc;
  const WsView v = ws_view(ws, w);
  UniformArgs a;
  a.head = v.head; a.tail = v.tail; a.off = offsets; a.n_links = n_links_of(b); a.vx = vx; a.vy = vy;
  a.capacity = cap; a.miter_limit = p->miter_limit;
  if (a.n_links > 0)
    hipLaunchKernelGGL(uniform_emit_kernel, dim3(num_cus() * 8), dim3(256), 0,
                       (hipStream_t)stream, a);
  PS_HIP(hipGetLastError());
  return PS_OK;
}

int ps_facet_stats(const ps_batch* b, const int64_t* offsets, const float* vx, const float* vy,
                   double* stats, void* stream) {
  int rc;
  if ((rc = check_batch(b))) return rc;
  if (!offsets || !vx || !vy || !stats) return fail(PS_E_ARG, "NULL array");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(clear_stats_kernel, dim3(1), dim3(64), 0, s, stats);
  if (b->n_segs > 0)
    hipLaunchKernelGGL(facet_stats_kernel, dim3(grid_for(b->n_segs, 256)), dim3(256), 0, s,
                       b->seg_begin, b->n_paths, b->n_segs, offsets, vx, vy, stats);
  PS_HIP(hipGetLastError());
  return PS_OK;
}

int ps_coverage(const ps_batch* b, const int64_t* offsets, const float* vx, const float* vy,
                int64_t n_ribs, const ps_canvas* cv, int32_t* top, void* stream) {
  int rc;
  if ((rc = check_batch(b))) return rc;
  if (!cv) return fail(PS_E_ARG, "canvas is NULL");
  if (cv->width < 0 || cv->height < 0) return fail(PS_E_ARG, "negative canvas size");
  if (!std::isfinite(cv->x0) || !std::isfinite(cv->y0)) return fail(PS_E_ARG, "canvas origin not finite");
  if (cv->mode != PS_COVER_QUAD && cv->mode != PS_COVER_TRIANGLES)
    return fail(PS_E_ARG, "unknown coverage mode %d", cv->mode);
  if (n_ribs < 0) return fail(PS_E_ARG, "negative rib count");
  const int64_t npix = (int64_t)cv->width * cv->height;
  if (npix >= (int64_t)INT32_MAX) return fail(PS_E_ARG, "canvas must hold fewer than 2^31 pixels");
  if (npix == 0) return PS_OK;
  if (!offsets || !top || (n_ribs > 0 && (!vx || !vy))) return fail(PS_E_ARG, "NULL array");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(npix, 256)), dim3(256), 0, s, top, npix, -1);
  if (n_ribs > 1 && n_links_of(b) > 0) {
    CovArgs a{offsets, n_links_of(b), b->seg_begin, b->n_paths, vx, vy, n_ribs, cv->x0, cv->y0,
              cv->width, cv->height, top};
    const int blocks = grid_for((n_ribs - 1 + 63) / 64, kCovWaves);
    if (cv->mode == PS_COVER_QUAD)
      hipLaunchKernelGGL(coverage_kernel<0>, dim3(blocks), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL(coverage_kernel<1>, dim3(blocks), dim3(256), 0, s, a);
  }
  PS_HIP(hipGetLastError());
  return PS_OK;
}

int ps_dash(const ps_batch* b, const ps_params* p, const int64_t* offsets, const float* vx,
            const float* vy, const float* vs, int64_t vcap, float* dx, float* dy, float* ds,
            int64_t* range, int64_t rib_cap, int64_t dash_cap, void* ws, size_t ws_bytes,
            void* stream) {
  int rc;
  if ((rc = check_batch(b)) || (rc = check_params(p))) return rc;
  if (p->n_dash == 0) return fail(PS_E_ARG, "ps_dash needs a dash pattern");
  if (!offsets || !vx || !vy || !vs || !dx || !dy || !ds || !range) return fail(PS_E_ARG, "NULL array");
  if (vcap < 0 || rib_cap < 0 || dash_cap < 0) return fail(PS_E_ARG, "negative capacity");
  const WsLayout w = ws_layout(n_links_of(b), vcap, p->n_dash);
  if ((rc = check_ws(ws, ws_bytes, w.total))) return rc;
  return launch_dash(b, p, offsets, vx, vy, vs, dx, dy, ds, range, rib_cap, dash_cap, ws_view(ws, w), w,
                     (hipStream_t)stream);
}

int ps_stroke_static(const ps_batch* b, const ps_params* p, int32_t* link_ribs, int64_t* offsets,
                     float* vx, float* vy, float* vs, int64_t cap, uint32_t* status_flags,
                     void* stream) {
  int rc;
  if ((rc = check_batch(b)) || (rc = check_params(p))) return rc;
  if (p->n_dash != 0) return fail(PS_E_UNSUPPORTED, "ps_stroke_static does not dash");
  if (!offsets || !vx || !vy || (!link_ribs && n_links_of(b) > 0)) return fail(PS_E_ARG, "NULL array");
  if (cap < 0) return fail(PS_E_ARG, "negative capacity");
  const WsLayout w = ws_layout(n_links_of(b), cap, 0);
  if (w.total > kStaticScratchBytes)
    return fail(PS_E_WORKSPACE, "batch needs %zu bytes of scratch; the static scratch holds %zu",
                w.total, kStaticScratchBytes);
  void* base = nullptr;
  if ((rc = static_scratch(&base))) return rc;
  const hipStream_t s = (hipStream_t)stream;
  const WsView v = ws_view(base, w);
  const EmitConfig c = config_of(p);
  if ((rc = launch_count(b, p, link_ribs, v, s))) return rc;
  if ((rc = do_link_scan(link_ribs, n_links_of(b), offsets, v, w, cap, c.K, s))) return rc;
  if ((rc = launch_emit(b, p, offsets, vx, vy, vs, cap, v, w, c, s, true))) return rc;
  if (status_flags) hipLaunchKernelGGL(copy_status_flags_kernel, dim3(1), dim3(64), 0, s, v.st, status_flags);
  PS_HIP(hipGetLastError());
  return PS_OK;
}

int ps_read_status(const void* ws, ps_status* out, void* stream) {
  if (!ws || !out) return fail(PS_E_ARG, "NULL argument");
  DevStatus d;
  PS_HIP(hipMemcpyAsync(&d, ws, sizeof(d), hipMemcpyDeviceToHost, (hipStream_t)stream));
  PS_HIP(hipStreamSynchronize((hipStream_t)stream));
  out->flags = d.flags;
  out->reserved = 0;
  out->total_ribs = (int64_t)d.total_ribs;
  out->fixups = (int64_t)d.fixups;
  out->dash_ribs = (int64_t)d.dash_ribs;
  out->dash_count = (int64_t)d.dash_count;
  return PS_OK;
}

int ps_plan_create(const ps_batch* b, const ps_params* p, int32_t* link_ribs, int64_t* offsets,
                   float* vx, float* vy, float* vs, int64_t cap, float* dx, float* dy, float* ds,
                   int64_t* range, int64_t dash_rib_cap, int64_t dash_cap, void* ws,
                   size_t ws_bytes, void* stream, ps_plan** out) {
  int rc;
  if (!out) return fail(PS_E_ARG, "out is NULL");
  *out = nullptr;
  if ((rc = check_batch(b)) || (rc = check_params(p))) return rc;
  if (!link_ribs || !offsets || !vx || !vy || !vs) return fail(PS_E_ARG, "NULL array");
  if (p->n_dash > 0 && (!dx || !dy || !ds || !range)) return fail(PS_E_ARG, "NULL dash array");
  const WsLayout w = ws_layout(n_links_of(b), cap, p->n_dash);
  if ((rc = check_ws(ws, ws_bytes, w.total))) return rc;
  ps_plan* P = new (std::nothrow) ps_plan();
  if (!P) return fail(PS_E_NOMEM, "plan allocation failed");
  P->b = *b;
  P->p = *p;
  P->dash.assign(p->dash, p->dash + p->n_dash);
  P->p.dash = P->dash.empty() ? nullptr : P->dash.data();
  P->link_ribs = link_ribs; P->off = offsets; P->vx = vx; P->vy = vy; P->vs = vs; P->cap = cap;
  P->dx = dx; P->dy = dy; P->ds = ds; P->range = range;
  P->dash_rib_cap = dash_rib_cap; P->dash_cap = dash_cap;
  P->ws = ws; P->w = w;
  P->graph[0] = P->graph[1] = nullptr; P->exec[0] = P->exec[1] = nullptr;
  P->ev_node[0] = P->ev_node[1] = nullptr; P->ev_own[0] = P->ev_own[1] = nullptr;
  hipStream_t s = (hipStream_t)stream;
  // the emit mapping: the one given, or the fastest on this batch
  P->cfg = config_of(p);
  const WsView v = ws_view(ws, w);
  if ((rc = launch_count(b, &P->p, link_ribs, v, s)) ||
      (rc = do_link_scan(link_ribs, n_links_of(b), offsets, v, w, cap, 0, s))) {
    delete P;
    return rc;
  }
  if (p->emit_mapping == PS_MAP_DEFAULT) {
    float best = 1e30f;
    const int Ks[5] = {4, 6, 7, 8, 16};
    const int Ws[3] = {1, 2, 4};   // at most 256 threads: the emit kernel's launch bound
    for (int mi = 0; mi < 2; ++mi)
    for (int ki = 0; ki < 5; ++ki)
      for (int wi = 0; wi < 3; ++wi) {
        EmitConfig c;
        c.map = mi ? PS_MAP_LINKS : PS_MAP_TILES; c.K = Ks[ki]; c.waves = Ws[wi];
        float ms = 0;
        if ((rc = time_emit(P, c, s, &ms))) { delete P; return rc; }
        if (ms < best) { best = ms; P->cfg = c; }
      }
  }
  // capture the chain twice: plain, and with the emit's event-record nodes
  if (hipStreamSynchronize(s) != hipSuccess) { delete P; return fail(PS_E_HIP, "stream synchronize failed"); }
  for (int k = 0; k < 2; ++k)
    if (hipEventCreate(&P->ev_own[k]) != hipSuccess) { ps_plan_destroy(P); return fail(PS_E_HIP, "event create failed"); }
  for (int timed = 0; timed < 2; ++timed)
    if ((rc = capture_plan(P, timed))) { ps_plan_destroy(P); return rc; }
  *out = P;
  return PS_OK;
}

int ps_plan_launch(ps_plan* P, void* stream) {
  if (!P || !P->exec[0]) return fail(PS_E_ARG, "invalid plan");
  PS_HIP(hipGraphLaunch(P->exec[0], (hipStream_t)stream));
  return PS_OK;
}

int ps_plan_launch_timed(ps_plan* P, void* stream, void* emit_begin, void* emit_end) {
  if (!P || !P->exec[1]) return fail(PS_E_ARG, "invalid plan");
  if (!emit_begin || !emit_end) return fail(PS_E_ARG, "NULL event");
  // a launch takes the events its nodes hold when it is enqueued
  hipGraphExec_t x = P->exec[1];
  PS_HIP(hipGraphExecEventRecordNodeSetEvent(x, P->ev_node[0], (hipEvent_t)emit_begin));
  PS_HIP(hipGraphExecEventRecordNodeSetEvent(x, P->ev_node[1], (hipEvent_t)emit_end));
  const hipError_t e = hipGraphLaunch(x, (hipStream_t)stream);
  PS_HIP(hipGraphExecEventRecordNodeSetEvent(x, P->ev_node[0], P->ev_own[0]));
  PS_HIP(hipGraphExecEventRecordNodeSetEvent(x, P->ev_node[1], P->ev_own[1]));
  PS_HIP(e);
  return PS_OK;
}

int ps_plan_destroy(ps_plan* P) {
  if (!P) return PS_OK;
  for (int k = 0; k < 2; ++k) {
    if (P->exec[k]) (void)hipGraphExecDestroy(P->exec[k]);
    if (P->graph[k]) (void)hipGraphDestroy(P->graph[k]);
    if (P->ev_own[k]) (void)hipEventDestroy(P->ev_own[k]);
  }
  delete P;
  return PS_OK;
}

int ps_plan_config(const ps_plan* P, int32_t* mapping, int32_t* K, int32_t* waves) {
  if (!P) return fail(PS_E_ARG, "invalid plan");
  if (mapping) *mapping = P->cfg.map;
  if (K) *K = P->cfg.K;
  if (waves) *waves = P->cfg.waves;
  return PS_OK;
}

}  // extern "C"
