/*
 * ps.h -- C ABI of the MI355X polar-stroking tessellator.
 *
 * Method: M. J. Kilgard, "Polar Stroking: New Theory and Methods for Stroking
 * Paths", ACM TOG 39(4) art. 145, 2020.  A stroked path is tessellated into a
 * quad strip by stepping every segment, join and cap in uniform steps of
 * tangent angle q, with the number of steps known before any vertex is made.
 *
 * The pipeline is   ps_count -> ps_scan -> ps_emit (vertices + arc length)
 *                                         -> ps_dash (optional)
 * or the same chain captured once in a hipGraph by ps_plan_create.
 *
 * Conventions for every entry point:
 *  - All array pointers are DEVICE pointers unless marked "host", owned by the
 *    caller, and must stay valid until the stream work that uses them ends.
 *    The library allocates nothing per call and keeps no pointer after a call
 *    returns (a ps_plan keeps the pointers it was created with).
 *  - `stream` is a hipStream_t passed as void*; NULL is the null stream.  Every
 *    call is stream-ordered and asynchronous; no call synchronises the device
 *    except ps_read_status and ps_plan_create.
 *  - Return value: PS_OK (0) or a negative PS_E_* code.  Argument errors are
 *    found on the host before any work is queued; nothing is launched then.
 *    ps_last_error() gives a message for the last failing call of the thread.
 *  - Errors found on the device (capacity exceeded, non-finite input, an
 *    unsupported value) set bits of a status word kept in the workspace; read
 *    it with ps_read_status after the stream work.  On overflow no vertex is
 *    written past the capacity given.
 *  - The workspace `ws` (size from ps_workspace_bytes) carries per-link setup
 *    records from ps_count to ps_emit: pass the same ws, batch and params to
 *    both.  Calls that share a workspace must not overlap.
 */
#ifndef PS_POLAR_STROKE_H
#define PS_POLAR_STROKE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Segment forms (the table of segment generator functions): line, quadratic Bezier,
 * rational quadratic conic with middle weight w_B, cubic Bezier. */
enum { PS_KIND_LINE = 0, PS_KIND_QUAD = 1, PS_KIND_CONIC = 2, PS_KIND_CUBIC = 3 };
/* Join styles (Secs. "Easy Joins", "Harder Joins: Miter Truncate and Revert"):
 * J = 0, 1, ceil(|delta|/q), 2 steps, and J = 3 for the two miter styles, whose
 * outer vertices of ribs 1 and 2 are the miter vertices.  The miter ratio is
 * 1/cos(|delta|/2) (miter length over stroke width); beyond params->miter_limit
 * PS_JOIN_MITER reverts to a bevel and PS_JOIN_MITER_CLIP cuts the miter at
 * miter_limit * w/2 from the join point, square to its bisector. */
enum { PS_JOIN_NONE = 0, PS_JOIN_BEVEL = 1, PS_JOIN_ROUND = 2, PS_JOIN_TRIANGLE = 3,
       PS_JOIN_MITER = 4, PS_JOIN_MITER_CLIP = 5 };
/* Cap styles (Secs. "Easy Caps", "Harder Caps"): J = 0, ceil(pi/q), 4, 2. */
enum { PS_CAP_BUTT = 0, PS_CAP_ROUND = 1, PS_CAP_SQUARE = 2, PS_CAP_TRIANGLE = 3 };
/* Arithmetic of the segment ribs' direction and tangent-angle solve (Eq.
 * angle2t):
 *   FP32        single precision throughout: setup and counts (ps_count),
 *               direction, solve, point; a study mode, whose counts can
 *               differ from the FP64 ones and whose vertices can be far off
 *               on near-degenerate segments;
 *   FP32_FIXUP  FP64 setup, direction and point; FP32 root isolation
 *               polished by one FP64 Newton step, re-solved in FP64 where
 *               that is ill-conditioned;
 *   FP64        double precision for every segment rib (recommended: exact
 *               counts, vertices within the FP32 rounding of the FP64 result,
 *               and the fastest of the two modes that are).
 * Join and cap ribs take an FP32 direction in every mode (their vertices lie
 * within r sqrt 2 of an exact pivot point); the arc length is FP32 chords of
 * the FP64 rib points (each within 2^-22 of its length), summed exactly in
 * 64-bit fixed point. */
enum { PS_PREC_FP32 = 0, PS_PREC_FP32_FIXUP = 1, PS_PREC_FP64 = 2 };

enum {
  PS_OK = 0,
  PS_E_ARG = -1,          /* invalid argument (null pointer, size, q, ...)     */
  PS_E_WORKSPACE = -2,    /* workspace smaller than ps_workspace_bytes        */
  PS_E_HIP = -3,          /* a HIP runtime call failed                        */
  PS_E_NOMEM = -4,        /* host allocation for a plan failed                */
  PS_E_UNSUPPORTED = -5   /* option not implemented                           */
};

/* Device status bits (ps_status.flags). */
enum {
  PS_STATUS_OVERFLOW = 1u,       /* 2 * total ribs > vertex capacity: no emit  */
  PS_STATUS_NONFINITE = 2u,      /* a control point, weight or width not finite */
  PS_STATUS_BAD_VALUE = 4u,      /* unknown kind/style, w_B <= -1, width <= 0   */
  PS_STATUS_DASH_OVERFLOW = 8u,  /* dash output exceeded its capacity           */
  PS_STATUS_INTERVALS = 16u      /* a segment needed more than 5 intervals      */
};

/*
 * A batch of paths (Sec. "Path Preliminaries": a path is a sequence of
 * segments g_f(t), t in [0,1]; here successive segments of a path are taken
 * to share end points).  Structure-of-arrays, device memory:
 *   seg_begin [n_paths+1]  CSR: path p owns segments [seg_begin[p], seg_begin[p+1])
 *   kind      [n_segs]     PS_KIND_*
 *   cx, cy    [4*n_segs]   control point k of segment i at [k*n_segs + i];
 *                          a line uses k<2, a quadratic or conic k<3
 *   conic_w   [n_segs]     w_B of conics (> -1; a negative weight draws the
 *                          external arc, 0 the chord P0 P2); ignored for
 *                          other kinds
 *   width     [n_paths]    stroke width w (> 0)
 *   join, cap [n_paths]    PS_JOIN_*, PS_CAP_*
 *   closed    [n_paths]    1: a closed contour (a join from the last segment
 *                          with ribs back to the first, no caps); 0: open.
 *                          May be NULL (every path open).  Closing adds no
 *                          segment: a closed contour's last segment should end
 *                          where its first begins.
 */
typedef struct {
  int32_t n_paths;
  int32_t n_segs;
  const int32_t* seg_begin;
  const uint8_t* kind;
  const float* cx;
  const float* cy;
  const float* conic_w;
  const float* width;
  const uint8_t* join;
  const uint8_t* cap;
  const uint8_t* closed;
} ps_batch;

/* Emit mappings (how ribs are spread over wavefronts; the output bits do not
 * depend on it).  Both run persistent wavefronts over tiles of 64*K
 * consecutive ribs, K = emit_ribs_per_lane in {4, 6, 7, 8, 16}:
 *   PS_MAP_DEFAULT  unplanned calls: PS_MAP_TILES with K = 7, 4 wavefronts;
 *                   ps_plan_create: the fastest mapping on the batch, timed
 *   PS_MAP_TILES    each tile's links staged in LDS, its segment ribs and
 *                   join/cap ribs swept apart, 64 at a time
 *   PS_MAP_LINKS    each tile walked link by link: all 64 lanes take ribs of
 *                   the same link, whose record the wavefront holds once */
enum { PS_MAP_DEFAULT = 0, PS_MAP_TILES = 1, PS_MAP_LINKS = 2 };

/*
 * Parameters: q is the maximum tangent-angle step (Sec. "Uniform Tangent Angle
 * Step Tessellation"), in radians, 1e-4 <= q <= pi.  precision is PS_PREC_*.
 * Dashing (Sec. "Dashing"): n_dash on/off lengths (even count >= 2, all >= 0,
 * positive sum) in the HOST array dash, starting at pattern position
 * dash_phase >= 0 at arc length 0 of every path (at most 2^40 periods);
 * n_dash = 0 disables it.  miter_limit >= 1 bounds the miter ratio of the
 * miter joins (4 is the usual default of path-rendering standards).
 * emit_mapping is PS_MAP_*; emit_ribs_per_lane (K) and emit_waves
 * (wavefronts per workgroup, 1..4) choose its shape, 0 for the default.
 * These only affect speed.
 */
typedef struct {
  double q;
  int32_t precision;
  int32_t n_dash;
  const double* dash;
  double dash_phase;
  double miter_limit;
  int32_t emit_mapping;
  int32_t emit_ribs_per_lane;
  int32_t emit_waves;
  int32_t reserved;   /* 0 */
} ps_params;

/* Status read back from a workspace. */
typedef struct {
  uint32_t flags;       /* PS_STATUS_* bits                                */
  uint32_t reserved;
  int64_t total_ribs;   /* ribs of the last ps_scan (2 vertices per rib)   */
  int64_t fixups;       /* ribs re-solved in FP64 by the last ps_emit      */
  int64_t dash_ribs;    /* ribs written by the last ps_dash                */
  int64_t dash_count;   /* dashes written by the last ps_dash              */
} ps_status;

/*
 * Number of link slots, 2*n_segs + n_paths (Sec. "Complete Algorithm": a path
 * is divided into links, one per segment, cap and join).  Fixed slot layout:
 * path p with segments [b,e) owns slots 2b+p (start cap), 2i+p+1 (segment i)
 * and 2i+p+2 (the join after segment i, or the end cap after the last).  A
 * zero-length segment has no ribs and joins are made across it.
 */
int64_t ps_num_links(const ps_batch* batch);

/* Bytes of workspace needed for this batch and a vertex capacity (host only). */
size_t ps_workspace_bytes(const ps_batch* batch, const ps_params* params,
                          int64_t vertex_capacity);

/*
 * ps_count -- per-link setup and a-priori step counts (Eqs. p-value, Psi,
 * continuous-delta, Delta_i, DeltaSigmaK; Sec. "Tessellation Approach for Caps
 * and Joins").  Writes link_ribs[ps_num_links(batch)] (int32, device): the rib
 * count of every link slot, N+1 for a segment of N steps and J+1 for a join or
 * cap of J steps (0 when J = 0 or the segment has zero length).  The setup in
 * FP64 (end gradients, reversal parameters, tangent angles, interval splits)
 * is kept in ws for ps_emit.  Resets the status word.
 */
int ps_count(const ps_batch* batch, const ps_params* params, int32_t* link_ribs,
             void* ws, size_t ws_bytes, void* stream);

/*
 * ps_scan -- exclusive prefix sum of link_ribs[n_links] (int32, device) into
 * offsets[n_links+1] (int64, device); offsets[n_links] is the total rib count
 * R, also stored in the status word.  The counts are known a priori (Sec.
 * "The Polar Stroking Method"), so these are the output positions of every
 * link.  Integer arithmetic: the result is exact.
 */
int ps_scan(const int32_t* link_ribs, int64_t n_links, int64_t* offsets, void* ws,
            size_t ws_bytes, void* stream);

/*
 * ps_emit -- rib vertices (Eqs. func_t, func_N, RibVertices-N, RibVertices-P;
 * Sec. "Complete Algorithm") and, when vs is not NULL, cumulative arc length
 * (Eq. arc-length-approximation; Sec. "Cumulative Arc Length Texturing").
 * Rib r of link l is rib j = r - offsets[l] of that link; its vertices go to
 * vertex 2r (N = G - r_N n) and 2r+1 (P = G + r_P n), n = (-sin psi, cos psi):
 * vx, vy [vertex_capacity] float.  vs [vertex_capacity] float receives the arc
 * length at the rib for both of its vertices: a chord sum from 0 at the first
 * rib of each path, constant across joins and caps, with a step whose t
 * decreases adding nothing.  The sums are exact integers of 2^-32 px, so s
 * has the same bits whatever the mapping; they hold a path of up to 2^30 px
 * (about 1.07e9 px: longer paths wrap) with chords below 2^31 px.
 * Consecutive ribs of a path form its quads.
 * Requires ws from ps_count (same batch and params) and offsets from ps_scan.
 * If 2*R > vertex_capacity nothing is written and PS_STATUS_OVERFLOW is set;
 * each call clears that bit first, so a retry with enough capacity reports
 * no overflow.
 */
int ps_emit(const ps_batch* batch, const ps_params* params, const int64_t* offsets,
            float* vx, float* vy, float* vs, int64_t vertex_capacity, void* ws,
            size_t ws_bytes, void* stream);

/*
 * ps_arclen -- the arc-length output of ps_emit alone: fills vs as ps_emit
 * would, without writing vertices (same requirements as ps_emit).
 */
int ps_arclen(const ps_batch* batch, const ps_params* params, const int64_t* offsets,
              float* vs, int64_t vertex_capacity, void* ws, size_t ws_bytes, void* stream);

/*
 * ps_emit_uniform -- the uniform parametric baseline the paper compares
 * against (Sec. "Versus Uniform Parametric Tessellation"): the stroked region
 * of Eq. NaiveStroking sampled at t_j = j/N for every segment, with the rib
 * counts of ps_count (the same quad budget as polar stroking); n(t_j) is the
 * unit left normal of g'(t_j), taken 2^-20/N further into the segment where
 * g' vanishes.  Joins and caps are emitted as by ps_emit.  Writes vx, vy
 * [2R] like ps_emit (no arc length); same requirements as ps_emit.
 */
int ps_emit_uniform(const ps_batch* batch, const ps_params* params, const int64_t* offsets,
                    float* vx, float* vy, int64_t vertex_capacity, void* ws, size_t ws_bytes,
                    void* stream);

/*
 * ps_facet_stats -- ordinary facet angles of the segment ribs of a rib stream
 * (Sec. "Uniform Tangent Angle Step Tessellation": the angle at which one quad
 * meets the next; ordinary ones are below 2q for polar stroking).  On each side
 * of a segment's strip the facet at interior rib j is the angle between the
 * boundary edges E_{j-1} = V_{j-1}V_j and E_j = V_jV_{j+1}.  An edge is regular
 * when it is not empty and runs with the direction of travel at both of its
 * ribs (n rotated by -90 deg, n = P - N; a rib of zero width has none); the
 * boundary inside an offset cusp reverses.  A facet is ordinary when every edge
 * of the segment within one rib of it (E_{j-2} .. E_{j+1}) is regular, which
 * leaves out the facets beside offset cusps.  vx, vy [2R] and offsets as
 * written by ps_emit or ps_emit_uniform.  stats: DEVICE double[4] = count,
 * maximum, sum, sum of squares of the ordinary facet angles (radians),
 * overwritten.  Sums are accumulated with atomics, so their last bits may
 * depend on the order threads finish.
 */
int ps_facet_stats(const ps_batch* batch, const int64_t* offsets, const float* vx,
                   const float* vy, double* stats, void* stream);

/* Coverage modes of ps_coverage. */
enum {
  PS_COVER_QUAD = 0,       /* a quad covers where its winding number is nonzero     */
  PS_COVER_TRIANGLES = 1   /* the two triangles a triangle rasterizer would draw    */
};

typedef struct {
  double x0, y0;           /* world position of the corner of pixel (0, 0)          */
  int32_t width, height;   /* pixels; pixel (i, j) samples (x0+i+1/2, y0+j+1/2)      */
  int32_t mode;            /* PS_COVER_*                                             */
} ps_canvas;

/*
 * ps_coverage -- which path covers each pixel sample (Sec. "Stroked Paths
 * Tessellated to Quad Strips"; the support predicate, Eq.
 * polar-stroking-predicate, evaluated on the tessellation).  The quads of a
 * path are its consecutive ribs within a link, plus the quad from a link's
 * last rib to the next link's first rib unless both links are segments (then
 * no join ribs lie between them and the quad would draw a bevel).  Quad r has
 * corners N_r, P_r, P_{r+1}, N_{r+1}; in PS_COVER_QUAD it covers a sample
 * where its winding number is nonzero (edges counted by the half-open
 * crossing rule, in FP64 on the FP32 vertices), so a bow-tie quad covers its
 * two lobes; PS_COVER_TRIANGLES covers the union of triangles (N_r, P_r,
 * P_{r+1}) and (N_r, P_{r+1}, N_{r+1}) instead, which is what splitting the
 * quad for a triangle rasterizer draws.  top: DEVICE int32 [height * width],
 * row-major, overwritten with the largest covering path index, or -1 (a
 * renderer drawing opaque strokes in path order shows that path there).
 * vx, vy [2 * n_ribs] and offsets as written by ps_emit or ps_emit_uniform;
 * ribs beyond offsets[n_links] are ignored.  The canvas must hold fewer than
 * 2^31 pixels (PS_E_ARG otherwise).  Needs no workspace.
 */
int ps_coverage(const ps_batch* batch, const int64_t* offsets, const float* vx, const float* vy,
                int64_t n_ribs, const ps_canvas* canvas, int32_t* top, void* stream);

/*
 * ps_dash -- dashing by arc length (Sec. "Dashing").  Reads the rib stream of
 * ps_emit (vx, vy, vs of vertex_capacity entries, the capacity the workspace
 * was sized with; offsets from ps_scan) and writes the "on" pieces: dx, dy
 * [2*rib_capacity] and ds [2*rib_capacity] in the same vertex layout, and
 * dash_range [2*dash_capacity] int64 pairs [first rib, end rib) per dash.  A
 * pattern boundary s_b inside a step (s_{j-1}, s_j] inserts a rib interpolated
 * linearly in s; steps of zero length hold no boundary; the pattern restarts
 * at every path.  Each call first clears PS_STATUS_DASH_OVERFLOW and the dash
 * totals of the status word, then writes its own totals there; on overflow
 * nothing past the capacities is written and PS_STATUS_DASH_OVERFLOW is set,
 * and a second call with capacities of at least those totals fits.
 */
int ps_dash(const ps_batch* batch, const ps_params* params, const int64_t* offsets,
            const float* vx, const float* vy, const float* vs, int64_t vertex_capacity,
            float* dx, float* dy, float* ds, int64_t* dash_range, int64_t rib_capacity,
            int64_t dash_capacity, void* ws, size_t ws_bytes, void* stream);

/*
 * ps_stroke_static -- ps_count -> ps_scan -> ps_emit (vertices and, when vs is
 * not NULL, arc length) in one call that allocates nothing and takes no
 * workspace, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid it).  Its scratch
 * memory is a 64 MiB array in the library's device code, one per GPU the
 * library runs on, held until the process ends; batches whose workspace
 * (ps_workspace_bytes for this vertex_capacity, no dashing) exceeds it are
 * refused with PS_E_WORKSPACE before anything is queued (the 64-cubic path and
 * the 5,000-cubic walk fit; the 4,096-path batch does not).  Outputs as those
 * of ps_count, ps_scan and ps_emit: link_ribs [ps_num_links], offsets
 * [ps_num_links+1], vx, vy, vs [vertex_capacity], all DEVICE, caller-owned.
 * status_flags: DEVICE uint32, may be NULL; receives the PS_STATUS_* bits of
 * this call once the stream reaches its end.  params->n_dash must be 0
 * (PS_E_UNSUPPORTED otherwise).  The stream must belong to the current
 * device.  Every call on a GPU uses that GPU's one array: calls that overlap
 * on one GPU (other streams, other threads) race and must not be made.
 */
int ps_stroke_static(const ps_batch* batch, const ps_params* params, int32_t* link_ribs,
                     int64_t* offsets, float* vx, float* vy, float* vs, int64_t vertex_capacity,
                     uint32_t* status_flags, void* stream);

/* Copy the status word of ws to the host (synchronises `stream`). */
int ps_read_status(const void* ws, ps_status* out, void* stream);

/*
 * Batched form: ps_plan_create picks the emit mapping for this batch when
 * params->emit_mapping is PS_MAP_DEFAULT (it runs the pipeline several times
 * on `stream` and times every mapping; otherwise it takes the one given), then captures
 * count -> scan -> emit (-> dash when params->n_dash > 0) into a hipGraph
 * bound to these buffers, and a second copy with an event-record node
 * between scan and emit and one after the emit.  ps_plan_launch replays the
 * first on `stream`; ps_plan_launch_timed replays the second with its nodes
 * recording the caller's events emit_begin and emit_end (hipEvent_t, created
 * with timing), so their elapsed time is that launch's emit (the event nodes
 * add some launch latency, which is why plain launches skip them).
 * ps_plan_destroy frees the plan.  link_ribs [ps_num_links], offsets
 * [ps_num_links+1]; the dash buffers may be NULL when dashing is off.  The
 * plan keeps all pointers given here.
 */
typedef struct ps_plan ps_plan;
int ps_plan_create(const ps_batch* batch, const ps_params* params, int32_t* link_ribs,
                   int64_t* offsets, float* vx, float* vy, float* vs, int64_t vertex_capacity,
                   float* dx, float* dy, float* ds, int64_t* dash_range, int64_t dash_rib_capacity,
                   int64_t dash_capacity, void* ws, size_t ws_bytes, void* stream,
                   ps_plan** out);
int ps_plan_launch(ps_plan* plan, void* stream);
int ps_plan_launch_timed(ps_plan* plan, void* stream, void* emit_begin, void* emit_end);
int ps_plan_destroy(ps_plan* plan);
/* The emit mapping a plan runs: PS_MAP_TILES or PS_MAP_LINKS, K and
 * wavefronts per workgroup. */
int ps_plan_config(const ps_plan* plan, int32_t* mapping, int32_t* ribs_per_lane,
                   int32_t* waves_per_group);

/* Message for the last failing call on this thread ("" if none). */
const char* ps_last_error(void);

/* Library version string. */
const char* ps_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PS_POLAR_STROKE_H */
