"""GPU-vs-oracle parity through the C ABI (needs an MI355X).

Bar: link rib counts and offsets bit-exact; every vertex within 2e-3 px of the
FP64 oracle (FP32 with FP64 fix-up, and FP64); arc length within a tolerance
derived from FP32 output rounding of s (stated per case in the assertion).
"""
import math

import numpy as np
import pytest

import oracle
import paper_2007_00308_amd as ps
from paper_2007_00308_amd import workloads as W

pytestmark = pytest.mark.gpu

VERTEX_TOL = 2e-3


def _gpu(b, precision=ps.PS_PREC_FP64, **kw):
    db = ps.DeviceBatch(b)
    out = ps.stroke(db, b.q, precision=precision, **kw)
    import torch
    torch.cuda.synchronize()
    return db, out


def _np(t):
    return t.detach().cpu().numpy()


# Arc length per rib (Eq. arc-length-approximation): the GPU takes each chord
# of its FP64 rib points in FP32 (dx, dy rounded to FP32, the sum of squares
# and the hardware square root each within an ulp: the chord within 2^-22 of
# its length), as a whole number of 2^-32 px (at most 2^-33 off), sums them as
# exact integers and rounds the sum once to FP32.  The bound at a rib k chords
# into its path, whose oracle arc length is s, is one FP32 spacing of s (the
# final rounding, counted in full to cover the oracle's own FP64 sum), plus
# 2^-22 s (the FP32 chords), plus 2^-30 px per chord (the fixed-point rounding
# and the FP64 difference between the two sides' points).
ARC_PER_CHORD = 2.0 ** -30
ARC_REL = 2.0 ** -22


def _arc_tol(ref_s, k):
    ref_s = np.abs(np.asarray(ref_s, np.float64))
    return (np.spacing(ref_s.astype(np.float32)).astype(np.float64) + ARC_REL * ref_s
            + (k + 1) * ARC_PER_CHORD)


def _rib_index_in_path(b, off):
    """For every rib: how many ribs of its path come before it."""
    first = oracle.path_rib_begin(b, off)
    R = int(off[-1])
    owner = np.repeat(np.arange(b.n_paths), np.diff(first))
    return np.arange(R, dtype=np.int64) - first[owner]


def _check_arc(vs_gpu, ref_s, k, what=""):
    vs_gpu = np.asarray(vs_gpu, np.float64)
    err = np.abs(vs_gpu - ref_s)
    tol = _arc_tol(ref_s, k)
    bad = np.flatnonzero(err > tol)
    assert bad.size == 0, (f"{what} arc length off at {bad.size} ribs; first rib {bad[0]}: "
                           f"gpu {vs_gpu[bad[0]]!r} oracle {ref_s[bad[0]]!r} tol {tol[bad[0]]:.3e}")
    return float(err.max()) if err.size else 0.0


def _compare(b, precision=ps.PS_PREC_FP64, vertex_tol=VERTEX_TOL, check_s=True, emit=(ps.PS_MAP_DEFAULT, 0, 0)):
    ref = oracle.stroke(b)
    db, out = _gpu(b, precision, emit=emit)
    st = out["status"]
    assert st.flags == 0, st.flags
    np.testing.assert_array_equal(_np(out["link_ribs"]), ref["link_ribs"])
    np.testing.assert_array_equal(_np(out["offsets"]), ref["offsets"])
    R = int(ref["offsets"][-1])
    assert out["total_ribs"] == R
    vx, vy = _np(out["vx"]).astype(np.float64), _np(out["vy"]).astype(np.float64)
    err = np.hypot(vx - ref["vx"], vy - ref["vy"])
    worst = int(np.argmax(err)) if err.size else 0
    assert err.size == 0 or err.max() <= vertex_tol, (
        f"max vertex error {err.max():.3e} px at vertex {worst} (rib {worst // 2}, "
        f"t={ref['t'][worst // 2]}, psi={ref['psi'][worst // 2]})")
    s_err = 0.0
    if check_s and R:
        vs = _np(out["vs"]).astype(np.float64)
        assert np.array_equal(vs[0::2], vs[1::2])
        s_err = _check_arc(vs[0::2], ref["vs"], _rib_index_in_path(b, ref["offsets"]))
    return dict(R=R, vmax=float(err.max()) if err.size else 0.0, smax=s_err, fixups=st.fixups)


# --------------------------------------------------------------- configurations
def test_config1_full():
    r = _compare(W.config1())
    assert r["R"] > 1000


@pytest.mark.parametrize("prec", [ps.PS_PREC_FP32_FIXUP, ps.PS_PREC_FP64])
def test_config2_reduced(prec):
    _compare(W.config2(n_paths=96, max_segs=64), precision=prec)


@pytest.mark.parametrize("prec", [ps.PS_PREC_FP32_FIXUP, ps.PS_PREC_FP64])
def test_config2_reduced_link_mapping(prec):
    _compare(W.config2(n_paths=96, max_segs=64), precision=prec, emit=(ps.PS_MAP_LINKS, 7, 4))


def test_config2_full_in_the_bench_mapping():
    # the benchmark batch through an autotuned plan, as bench.py runs it:
    # every count bit-exact, every vertex and arc length against the oracle
    import torch
    b = W.config2_fast()
    db = ps.DeviceBatch(b)
    first = ps.stroke(db, b.q)
    R = first["total_ribs"]
    del first
    plan = ps.Plan(db, b.q, vertex_capacity=2 * R)
    plan.launch()
    torch.cuda.synchronize()
    assert plan.status().flags == 0
    ref = oracle.stroke(b)
    np.testing.assert_array_equal(_np(plan.link_ribs[:db.n_links]), ref["link_ribs"])
    np.testing.assert_array_equal(_np(plan.offsets), ref["offsets"])
    err = np.hypot(_np(plan.vx[:2 * R]).astype(np.float64) - ref["vx"],
                   _np(plan.vy[:2 * R]).astype(np.float64) - ref["vy"])
    assert err.max() <= VERTEX_TOL, err.max()
    vs = _np(plan.vs[:2 * R]).astype(np.float64)
    _check_arc(vs[0::2], ref["vs"], _rib_index_in_path(b, ref["offsets"]), "config 2")
    plan.close()


def test_config5_full_sampled():
    # 2^20 segments at q = pi/256 (4.9e8 vertices): every link count, and the
    # ribs of 200 sampled paths plus the longest one against the oracle
    import torch
    b = W.config5(q=math.pi / 256)
    db, out = _gpu(b)
    assert out["status"].flags == 0
    np.testing.assert_array_equal(_np(out["link_ribs"]), oracle.count(b))
    off = out["offsets"]
    sb = b.seg_begin.astype(np.int64)
    rng = np.random.default_rng(5)
    counts = np.diff(sb)
    idx = np.union1d(rng.choice(b.n_paths, 200, replace=False), [int(np.argmax(counts))])
    sub = b.subset(idx)
    ref = oracle.stroke(sub)
    rsb = sub.seg_begin.astype(np.int64)
    for k, p in enumerate(idx):
        a, e = int(off[2 * sb[p] + p]), int(off[2 * sb[p + 1] + p + 1])
        ra, re = int(ref["offsets"][2 * rsb[k] + k]), int(ref["offsets"][2 * rsb[k + 1] + k + 1])
        assert e - a == re - ra, p
        if e == a:
            continue
        vx = _np(out["vx"][2 * a:2 * e]).astype(np.float64)
        vy = _np(out["vy"][2 * a:2 * e]).astype(np.float64)
        err = np.hypot(vx - ref["vx"][2 * ra:2 * re], vy - ref["vy"][2 * ra:2 * re])
        assert err.max() <= VERTEX_TOL, (p, err.max())
        vs = _np(out["vs"][2 * a:2 * e:2]).astype(np.float64)
        _check_arc(vs, ref["vs"][ra:re], np.arange(re - ra), f"path {p}")
    # the same batch through an autotuned plan, as bench.py times it (its
    # one-pass link scan spans 529 blocks here, so look-backs read several
    # windows of 64 words): bits identical to the checked run
    R = out["total_ribs"]
    plan = ps.Plan(db, b.q, vertex_capacity=2 * R)
    plan.launch()
    torch.cuda.synchronize()
    st = plan.status()
    assert st.flags == 0 and st.total_ribs == R
    assert torch.equal(plan.offsets, out["offsets"])
    for k in ("vx", "vy", "vs"):
        assert torch.equal(getattr(plan, k)[:2 * R], out[k][:2 * R]), k
    plan.close()


def test_config3_full_path():
    r = _compare(W.config3())
    assert r["R"] > 100_000


def test_config4_reduced_precision_cases():
    _compare(W.config4(n_paths=160, max_segs=32), precision=ps.PS_PREC_FP32_FIXUP)
    _compare(W.config4(n_paths=160, max_segs=32), precision=ps.PS_PREC_FP64)


@pytest.mark.parametrize("q", [math.pi / 16, math.pi / 64, math.pi / 256])
def test_config5_reduced(q):
    _compare(W.config5(q=q, n_paths=512, total_segs=4096))


@pytest.mark.parametrize("join,cap", [(W.JOIN_ROUND, W.CAP_ROUND), (W.JOIN_BEVEL, W.CAP_SQUARE),
                                      (W.JOIN_TRIANGLE, W.CAP_TRIANGLE), (W.JOIN_NONE, W.CAP_BUTT),
                                      (W.JOIN_MITER, W.CAP_BUTT), (W.JOIN_MITER_CLIP, W.CAP_ROUND)])
def test_styles(join, cap):
    _compare(W.random_mixed(21, n_paths=60, max_segs=20, extent=2048.0, join=join, cap=cap))


@pytest.mark.parametrize("limit", [1.0, 1.5, 4.0, 50.0])
@pytest.mark.parametrize("join", [W.JOIN_MITER, W.JOIN_MITER_CLIP])
def test_miter_limits(join, limit):
    # polylines with turns of every size, both senses: miters within, beyond
    # and exactly at (limit 1) the limit, reverted or clipped
    b = W.random_mixed(33, n_paths=40, max_segs=12, extent=512.0, join=join, cap=W.CAP_SQUARE)
    b.kind[:] = W.KIND_L
    b.miter_limit = limit
    _compare(b)


def test_closed_contours():
    # every other path closed: the last segment ends at the first one's start
    # and a join replaces both caps
    b = W.random_mixed(45, n_paths=50, max_segs=9, extent=1024.0, join=W.JOIN_MITER, cap=W.CAP_ROUND)
    closed = np.zeros(b.n_paths, np.uint8)
    closed[::2] = 1
    for p in range(b.n_paths):
        s0, s1 = int(b.seg_begin[p]), int(b.seg_begin[p + 1]) - 1
        if closed[p]:
            n = W.NPTS[int(b.kind[s1])]
            b.cx[n - 1, s1], b.cy[n - 1, s1] = b.cx[0, s0], b.cy[0, s0]
    b.closed = closed
    r = _compare(b)
    ref = oracle.stroke(b)
    # closed contours have no cap ribs
    sb = b.seg_begin.astype(np.int64)
    start_caps = ref["link_ribs"][2 * sb[:-1] + np.arange(b.n_paths)]
    assert np.all(start_caps[closed == 1] == 0) and np.any(start_caps[closed == 0] > 0)


@pytest.mark.parametrize("prec", [ps.PS_PREC_FP32_FIXUP, ps.PS_PREC_FP64])
def test_external_conics(prec):
    # conic weights in [-0.8, 0): external ellipses, turning the long way
    # round (split in two halves); every tenth conic of weight 0 (its chord)
    b = W.random_mixed(52, n_paths=80, max_segs=16, extent=512.0)
    k = np.flatnonzero(b.kind == W.KIND_K)
    rng = np.random.default_rng(52)
    b.conic_w[k] = -rng.uniform(0.02, 0.8, k.size).astype(np.float32)
    b.conic_w[k[::10]] = 0.0
    assert k.size > 50
    _compare(b, precision=prec)


def _ellipse_arc(cx, cy, ax, by, a0, a1):
    # the conic control points of an arc of the ellipse (affine image of a
    # circular arc: tangent-intersection middle point, weight cos(half angle))
    m, h = 0.5 * (a0 + a1), 0.5 * (a1 - a0)
    unit = [(math.cos(a0), math.sin(a0)), (math.cos(m) / math.cos(h), math.sin(m) / math.cos(h)),
            (math.cos(a1), math.sin(a1))]
    return [(cx + ax * u, cy + by * v) for u, v in unit], math.cos(h)


def test_two_conic_ellipses():
    # ellipses of two conic segments, the second external (the same control
    # points backwards with the weight negated), closed, at several sizes
    segs, widths = [], []
    rng = np.random.default_rng(8)
    for _ in range(32):
        a0 = rng.uniform(-math.pi, math.pi); span = rng.uniform(0.3, 2.8)
        pts, w = _ellipse_arc(rng.uniform(200, 800), rng.uniform(200, 800), rng.uniform(20, 300),
                              rng.uniform(20, 300), a0, a0 + span)
        segs.append([(W.KIND_K, pts, w), (W.KIND_K, pts[::-1], -w)])
        widths.append(float(rng.uniform(1, 40)))
    b = W.paths(segs, widths=widths, q=math.pi / 64, closed=[1] * len(segs))
    r = _compare(b)
    ref = oracle.stroke(b)
    # five slots per ellipse: no caps (closed), and both joins are smooth
    assert np.all(ref["link_ribs"].reshape(-1, 5)[:, [0, 2, 4]] == 0)
    assert r["R"] > 32 * 128


def test_unbounded_conics_flagged():
    # w_B <= -1 runs through a point at infinity: flagged, no ribs
    b = W.random_mixed(4, n_paths=6, max_segs=6)
    k = np.flatnonzero(b.kind == W.KIND_K)
    assert k.size >= 2
    b.conic_w[k[0]] = -1.0
    b.conic_w[k[1]] = -7.5
    _, out = _gpu(b)
    assert out["status"].flags & ps.PS_STATUS_BAD_VALUE
    lr = _np(out["link_ribs"])
    for i in k[:2]:
        p = int(np.searchsorted(b.seg_begin, i, side="right")) - 1
        assert lr[2 * i + p + 1] == 0


def _matching_ribs(lr_a, off_a, lr_b, off_b):
    # rib indices (into a and into b) of the links whose counts agree
    same = lr_a == lr_b
    n = lr_a[same].astype(np.int64)
    rep = np.repeat(np.arange(n.size), n)
    within = np.arange(int(n.sum()), dtype=np.int64) - np.repeat(np.cumsum(n) - n, n)
    return off_a[:-1][same][rep] + within, off_b[:-1][same][rep] + within, same


def test_fp32_only_is_reported():
    # single precision throughout (setup, count and emit) is a study mode with
    # a looser bound: its counts may differ from the FP64 oracle's where a
    # turn over q lands within FP32 rounding of an integer (the FP64 count's
    # epsilon is below FP32 resolution); on these random curves at most 1 % of
    # the links differ, and the links that agree are close
    b = W.config2(n_paths=64, max_segs=32)
    ref = oracle.stroke(b)
    _, out = _gpu(b, ps.PS_PREC_FP32)
    lr = _np(out["link_ribs"])
    ia, ib, same = _matching_ribs(lr, _np(out["offsets"]), ref["link_ribs"], ref["offsets"])
    assert (~same).sum() <= same.size // 100, (~same).sum()
    vx, vy = _np(out["vx"]), _np(out["vy"])
    va = np.concatenate([2 * ia, 2 * ia + 1]); vb = np.concatenate([2 * ib, 2 * ib + 1])
    err = np.hypot(vx[va] - ref["vx"][vb], vy[va] - ref["vy"][vb])
    assert err.max() < 0.05, err.max()


# --------------------------------------------------------------------- edge cases
def test_edge_single_line_and_degenerate():
    segs = [(W.KIND_L, [(0, 0), (100, 0)], 1.0),
            (W.KIND_C, [(100, 0), (100, 0), (100, 0), (100, 0)], 1.0),     # zero length
            (W.KIND_C, [(100, 0), (150, 0), (120, 0), (200, 0)], 1.0),     # collinear with folds
            (W.KIND_Q, [(200, 0), (200, 0), (250, 50)], 1.0),              # coincident P1 = P0
            (W.KIND_K, [(250, 50), (300, 100), (350, 50)], 1e-5),          # near-degenerate weight
            (W.KIND_C, [(350, 50), (351, 51), (350, 51), (351, 50)], 1.0)]  # exact cusp
    b = W.path(segs, width=4.0, q=math.pi / 32, cap=W.CAP_ROUND)
    _compare(b)


def test_edge_empty_paths_and_batches():
    b = W.paths([[], [(W.KIND_L, [(0, 0), (5, 5)], 1.0)], [], []], widths=[1, 2, 3, 4],
                q=math.pi / 8, caps=[W.CAP_SQUARE] * 4)
    _compare(b)
    b0 = W.paths([[]], widths=[1.0], q=0.1)
    r = _compare(b0)
    assert r["R"] == 0


def _tiny_paths(seed, n_paths):
    """Thousands of paths of 0 to 3 segments: empty paths, zero-length and
    collinear (folding) segments, closed paths, miter and round joins, round
    and square caps."""
    rng = np.random.default_rng(seed)
    out, closed, joins, caps = [], [], [], []
    for _ in range(n_paths):
        n = int(rng.choice([0, 1, 1, 1, 2, 2, 3]))
        segs = []
        x, y = rng.uniform(0, 512, 2)
        for _ in range(n):
            r = rng.random()
            if r < 0.1:
                segs.append((W.KIND_C, [(x, y)] * 4, 1.0))   # a point: no ribs
                continue
            if r < 0.25:
                d = rng.uniform(20, 60)
                pts = [(x, y), (x + 1.5 * d, y), (x + 1.2 * d, y), (x + 2 * d, y)]   # folds twice
                segs.append((W.KIND_C, pts, 1.0))
            else:
                k = int(rng.choice([W.KIND_L, W.KIND_Q, W.KIND_K, W.KIND_C]))
                pts = [(x, y)] + [tuple(rng.uniform(0, 512, 2)) for _ in range(W.NPTS[k] - 1)]
                segs.append((k, pts, float(rng.uniform(0.3, 3.0)) if k == W.KIND_K else 1.0))
            x, y = segs[-1][1][-1]
        out.append(segs)
        closed.append(1 if (n and rng.random() < 0.2) else 0)
        joins.append(int(rng.choice([W.JOIN_MITER, W.JOIN_MITER_CLIP, W.JOIN_ROUND, W.JOIN_BEVEL])))
        caps.append(int(rng.choice([W.CAP_ROUND, W.CAP_SQUARE, W.CAP_BUTT])))
    widths = list(rng.uniform(1.0, 12.0, n_paths))
    return W.paths(out, widths=widths, q=math.pi / 16, joins=joins, caps=caps, closed=closed)


def test_count_workgroups_with_many_paths():
    # about 170 path starts per 256 segments: a count workgroup's link slots
    # overrun its LDS stage of 576, so the later ones are written directly;
    # record tails for miter joins and for segments of up to 5 intervals
    b = _tiny_paths(77, 3000)
    assert b.n_segs > 1024
    _compare(b)


def test_many_paths_every_record_reader():
    # the same records read by the links mapping (scalar loads of head and
    # tail) and by the uniform baseline (per-lane loads): bits equal to the
    # tiles mapping, and the baseline against the oracle
    import torch
    b = _tiny_paths(78, 1500)
    _, tiles = _gpu(b)
    db, links = _gpu(b, emit=(ps.PS_MAP_LINKS, 7, 4))
    for k in ("vx", "vy", "vs"):
        assert torch.equal(tiles[k], links[k]), k
    ref = oracle.stroke(b, uniform=True)
    vx, vy = torch.empty_like(links["vx"]), torch.empty_like(links["vy"])
    ps.ps_emit_uniform(db, links["params"], links["offsets"], vx, vy, links["capacity"], links["ws"])
    torch.cuda.synchronize()
    R = links["total_ribs"]
    assert R == int(ref["offsets"][-1])
    err = np.hypot(_np(vx)[:2 * R] - ref["vx"], _np(vy)[:2 * R] - ref["vy"])
    assert err.max() <= VERTEX_TOL, err.max()


@pytest.mark.parametrize("q", [math.pi, 1e-3])
def test_edge_extreme_q(q):
    b = W.random_mixed(5, n_paths=4, max_segs=3, extent=300.0, q=q)
    _compare(b)


def test_overflow_sets_status_and_writes_nothing():
    import torch
    b = W.config1()
    db = ps.DeviceBatch(b)
    ref = oracle.stroke(b)
    R = int(ref["offsets"][-1])
    params = ps.make_params(b.q)
    link_ribs = torch.empty(db.n_links, dtype=torch.int32, device="cuda")
    offsets = torch.empty(db.n_links + 1, dtype=torch.int64, device="cuda")
    ws = ps.alloc_workspace(ps.ps_workspace_bytes(db, params, 2 * R), link_ribs.device)
    ps.ps_count(db, params, link_ribs, ws)
    ps.ps_scan(link_ribs, db.n_links, offsets, ws)
    vx = torch.full((2 * R,), 12345.0, device="cuda")
    vy, vs = torch.full_like(vx, 12345.0), torch.full_like(vx, 12345.0)
    ps.ps_emit(db, params, offsets, vx, vy, vs, 2 * R - 2, ws)
    assert ps.ps_read_status(ws).flags & ps.PS_STATUS_OVERFLOW
    assert bool(torch.all(vx == 12345.0)) and bool(torch.all(vs == 12345.0))
    # a retry with enough capacity on the same workspace fits and reports no overflow
    ps.ps_emit(db, params, offsets, vx, vy, vs, 2 * R, ws)
    assert not (ps.ps_read_status(ws).flags & ps.PS_STATUS_OVERFLOW)
    err = np.hypot(_np(vx) - ref["vx"], _np(vy) - ref["vy"])
    assert err.max() <= VERTEX_TOL


def test_nonfinite_and_bad_values_flagged():
    b = W.random_mixed(3, n_paths=3, max_segs=4)
    b.cx[1, 2] = np.nan
    b.conic_w[:] = -1.0
    b.kind[b.kind == W.KIND_K] = W.KIND_K
    _, out = _gpu(b)
    assert out["status"].flags & ps.PS_STATUS_NONFINITE


# ------------------------------------------------------ mapping / determinism
MAPPINGS = [(m, K, w) for m in (ps.PS_MAP_TILES, ps.PS_MAP_LINKS) for K in (4, 6, 7, 8, 16) for w in (1, 2, 4)]


def test_mappings_agree_and_are_deterministic():
    # every emit mapping gives the same bits: vertices from per-rib arithmetic
    # that does not look at the neighbours, arc length from integer sums
    b = W.config2(n_paths=48, max_segs=96)
    outs = []
    for emit in MAPPINGS:
        _, o = _gpu(b, emit=emit)
        outs.append((emit, _np(o["vx"]), _np(o["vy"]), _np(o["vs"])))
    for cfg, vx, vy, vs in outs[1:]:
        assert np.array_equal(vx, outs[0][1]) and np.array_equal(vy, outs[0][2]), cfg
        assert np.array_equal(vs, outs[0][3]), cfg


def test_long_chords_take_the_64_bit_scan():
    # chords longer than 2^18 px (2^50 fixed-point units) are summed by the
    # 64-bit scan; FP32 outputs at these coordinates carry half an ulp of 2^-5 px
    segs = [(W.KIND_L, [(0, 0), (400000, 0)], 1.0),
            (W.KIND_L, [(400000, 0), (400000, 300000)], 1.0),
            (W.KIND_C, [(400000, 300000), (500000, 300000), (300000, 500000), (450000, 520000)], 1.0)]
    b = W.path(segs, width=8.0, q=math.pi / 8, join=W.JOIN_BEVEL, cap=W.CAP_BUTT)
    tol = 2.0 * float(np.spacing(np.float32(600000.0)))
    r = _compare(b, vertex_tol=tol)
    assert r["R"] > 4


def test_arclen_only_matches_emit():
    import torch
    b = W.config3(n_segs=800)
    db, out = _gpu(b)
    vs2 = torch.empty_like(out["vs"])
    ps.ps_arclen(db, out["params"], out["offsets"], vs2, out["capacity"], out["ws"])
    torch.cuda.synchronize()
    assert torch.equal(vs2, out["vs"])


# ------------------------------------------------------------------ dash
def test_dash_exact_on_axis_lines():
    # collinear axis lines with dyadic lengths: the rib stream is exact on both
    # sides, so dash counts, ranges and positions must agree exactly
    segs = [(W.KIND_L, [(x0, 0), (x1, 0)], 1.0) for x0, x1 in
            [(0, 7.5), (7.5, 31.25), (31.25, 32.0), (32.0, 80.0)]]
    b = W.path(segs, width=2.0, q=math.pi / 8, join=W.JOIN_ROUND, cap=W.CAP_BUTT)
    ref = oracle.stroke(b)
    pr = oracle.path_rib_begin(b, ref["offsets"])
    dref = oracle.dash(pr, ref["vx"], ref["vy"], ref["vs"], [10.0, 5.0], 3.0)
    _, out = _gpu(b, dash=(10.0, 5.0), dash_phase=3.0)
    rng = _np(out["dash_range"])
    np.testing.assert_array_equal(rng, dref["ranges"])
    np.testing.assert_array_equal(_np(out["dx"]), dref["dx"].astype(np.float32))
    np.testing.assert_array_equal(_np(out["ds"])[0::2], dref["ds"].astype(np.float32))


def _dash_same_stream(b, out, pattern, phase):
    """The oracle's dasher run on the GPU's own FP32 rib stream: ranges must be
    identical and every output vertex and arc length within the vertex bar
    (both sides cut the same stream with the same FP64 operations)."""
    pr = oracle.path_rib_begin(b, _np(out["offsets"]))
    dref = oracle.dash(pr, _np(out["vx"]), _np(out["vy"]), _np(out["vs"])[0::2], list(pattern), phase)
    rng = _np(out["dash_range"])
    np.testing.assert_array_equal(rng, dref["ranges"])
    dx, dy = _np(out["dx"]).astype(np.float64), _np(out["dy"]).astype(np.float64)
    ds = _np(out["ds"]).astype(np.float64)
    assert dx.shape == dref["dx"].shape and ds.shape[0] == 2 * dref["ds"].shape[0]
    assert np.array_equal(ds[0::2], ds[1::2])
    err = np.hypot(dx - dref["dx"], dy - dref["dy"])
    assert err.max() <= VERTEX_TOL, err.max()
    np.testing.assert_allclose(ds[0::2], dref["ds"], rtol=0, atol=VERTEX_TOL)
    return dref


def _dash_own_streams(b, out, pattern, phase):
    """Secondary check: the oracle dashing its own rib stream.  Each side cuts
    its own stream, so an FP32 arc length half an ulp apart can move a cut by a
    rib; the dash count and the cut positions must still agree."""
    ref = oracle.stroke(b)
    pr = oracle.path_rib_begin(b, ref["offsets"])
    dref = oracle.dash(pr, ref["vx"], ref["vy"], ref["vs"], list(pattern), phase)
    rng = _np(out["dash_range"])
    assert rng.shape == dref["ranges"].shape
    ds = _np(out["ds"])[0::2].astype(np.float64)
    np.testing.assert_allclose(ds[rng[:, 0]], dref["ds"][dref["ranges"][:, 0]], atol=0.05)
    np.testing.assert_allclose(ds[rng[:, 1] - 1], dref["ds"][dref["ranges"][:, 1] - 1], atol=0.05)
    return rng


def test_dash_config3_full_path():
    # the whole 5,000-cubic walk with its [10 on, 5 off] pattern
    b = W.config3()
    _, out = _gpu(b, dash=b.dash, dash_phase=b.dash_phase)
    dref = _dash_same_stream(b, out, b.dash, b.dash_phase)
    assert dref["ranges"].shape[0] > 10_000
    _dash_own_streams(b, out, b.dash, b.dash_phase)


def test_dash_overflow_then_retry_fits():
    # a dash call that overflows reports the totals; a second call on the same
    # workspace with those capacities must succeed (the overflow bit is the
    # call's own, not left over from the first)
    import torch
    b = W.config3(n_segs=200)
    db, out = _gpu(b, dash=(7.0, 3.0, 2.0, 3.0), dash_phase=0.0)   # workspace sized for dashing
    params = out["params"]
    dev = out["vx"].device
    small = 64
    bufs = [torch.empty(2 * small, dtype=torch.float32, device=dev) for _ in range(3)]
    rng = torch.empty(2 * small, dtype=torch.int64, device=dev)
    ps.ps_dash(db, params, out["offsets"], out["vx"], out["vy"], out["vs"], out["capacity"], *bufs, rng,
               small, small, out["ws"])
    st = ps.ps_read_status(out["ws"])
    assert st.flags & ps.PS_STATUS_DASH_OVERFLOW
    nr, nd = int(st.dash_ribs), int(st.dash_count)
    assert nr > small and nd > small
    bufs = [torch.empty(2 * nr, dtype=torch.float32, device=dev) for _ in range(3)]
    rng = torch.empty(2 * nd, dtype=torch.int64, device=dev)
    ps.ps_dash(db, params, out["offsets"], out["vx"], out["vy"], out["vs"], out["capacity"], *bufs, rng,
               nr, nd, out["ws"])
    st = ps.ps_read_status(out["ws"])
    assert not (st.flags & ps.PS_STATUS_DASH_OVERFLOW)
    assert (int(st.dash_ribs), int(st.dash_count)) == (nr, nd)


def test_dash_mixed_batch_with_closed_paths_and_external_conics():
    # dashing restarts at s = 0 on every path; closed contours run on through
    # the closing join; a four-entry pattern with a phase
    b = W.random_mixed(81, n_paths=30, max_segs=8, extent=600.0, join=W.JOIN_MITER, cap=W.CAP_ROUND)
    k = np.flatnonzero(b.kind == W.KIND_K)
    b.conic_w[k[::2]] = -np.float32(0.4)
    closed = np.zeros(b.n_paths, np.uint8)
    for p in range(0, b.n_paths, 3):
        s0, s1 = int(b.seg_begin[p]), int(b.seg_begin[p + 1]) - 1
        n = W.NPTS[int(b.kind[s1])]
        b.cx[n - 1, s1], b.cy[n - 1, s1] = b.cx[0, s0], b.cy[0, s0]
        closed[p] = 1
    b.closed = closed
    pattern, phase = (7.0, 3.0, 2.0, 3.0), 1.5
    _, out = _gpu(b, dash=pattern, dash_phase=phase)
    dref = _dash_same_stream(b, out, pattern, phase)
    assert dref["ranges"].shape[0] > 100
    _dash_own_streams(b, out, pattern, phase)


def test_dash_after_an_emit_overflow_touches_nothing():
    # an emit whose capacity is too small writes nothing; a dash over that
    # stream must then read and write nothing either (it reports an overflow)
    import torch
    b = W.config3(n_segs=100)
    db = ps.DeviceBatch(b)
    params = ps.make_params(b.q, dash=b.dash, dash_phase=b.dash_phase)
    link_ribs = torch.empty(db.n_links, dtype=torch.int32, device="cuda")
    offsets = torch.empty(db.n_links + 1, dtype=torch.int64, device="cuda")
    ref_R = int(oracle.offsets(oracle.count(b))[-1])
    cap = 2 * (ref_R // 2)                      # half the ribs fit
    need = ps.ps_workspace_bytes(db, params, cap)
    guard = 4096
    ws_all = ps.alloc_workspace(need + guard, "cuda")
    ws_all.fill_(0xA5)
    ws = ws_all[:need]
    ps.ps_count(db, params, link_ribs, ws)
    ps.ps_scan(link_ribs, db.n_links, offsets, ws)
    vx = torch.zeros(cap, device="cuda"); vy = torch.zeros_like(vx); vs = torch.zeros_like(vx)
    ps.ps_emit(db, params, offsets, vx, vy, vs, cap, ws)
    assert ps.ps_read_status(ws).flags & ps.PS_STATUS_OVERFLOW
    n = 64
    dx = torch.full((2 * n + 64,), 777.0, device="cuda"); dy = dx.clone(); ds = dx.clone()
    rng = torch.full((2 * n + 64,), -5, dtype=torch.int64, device="cuda")
    ps.ps_dash(db, params, offsets, vx, vy, vs, cap, dx, dy, ds, rng, n, n, ws)
    st = ps.ps_read_status(ws)
    assert st.flags & ps.PS_STATUS_DASH_OVERFLOW
    for t in (dx, dy, ds):
        assert bool(torch.all(t == 777.0))
    assert bool(torch.all(rng == -5))
    assert bool(torch.all(ws_all[need:] == 0xA5))


# ------------------------------------------------------------------ plan / graph
def test_small_links_overflow_the_lds_window():
    # single-segment paths with butt caps and many zero-length segments: a
    # 64-rib iteration then spans more than 64 link slots, so the emit falls
    # back from the LDS window to global reads for it
    segs = [[(W.KIND_L, [(0, 0), (0, 0)], 1.0)] * 40 + [(W.KIND_L, [(0, 0), (3, 1)], 1.0)]
            + [(W.KIND_L, [(3, 1), (3, 1)], 1.0)] * 40 for _ in range(30)]
    b = W.paths(segs, widths=[1.0] * 30, q=math.pi / 4, caps=[W.CAP_BUTT] * 30)
    _compare(b)


def test_plan_graph_replays_match_eager():
    import torch
    b = W.config2(n_paths=40, max_segs=64)
    db, eager = _gpu(b)
    plan = ps.Plan(db, b.q, vertex_capacity=eager["capacity"])
    R = eager["total_ribs"]
    for rep in range(3):
        plan.launch()
        torch.cuda.synchronize()
        assert torch.equal(plan.vx[:2 * R], eager["vx"]), rep
        assert torch.equal(plan.vs[:2 * R], eager["vs"]), rep
        # unrelated eager work between replays
        torch.ones(1 << 20, device="cuda").sum().item()
    assert plan.status().flags == 0
    # the timed launch: the same output, and events around the emit graph
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(); e1.record()
    plan.vx.zero_()
    plan.launch_timed(e0, e1)
    torch.cuda.synchronize()
    assert torch.equal(plan.vx[:2 * R], eager["vx"])
    assert e0.elapsed_time(e1) > 0
    plan.close()


# ------------------------------------------------ uniform baseline, facet angles
def _serpentines(seed, n, width=100.0, q=math.radians(4.0)):
    # cubic serpentines (one inflection) and loops drawn on the 2^-8 grid
    rng = np.random.default_rng(seed)
    segs = []
    for _ in range(n):
        P0 = rng.uniform(0, 512, 2); P3 = P0 + rng.uniform(-300, 300, 2)
        P1 = P0 + rng.uniform(-200, 200, 2); P2 = P3 + rng.uniform(-200, 200, 2)
        pts = [tuple(np.round(P * 256) / 256) for P in (P0, P1, P2, P3)]
        segs.append([(W.KIND_C, pts, 1.0)])
    return W.paths(segs, widths=[width] * n, q=q)


def test_uniform_baseline_matches_oracle():
    b = _serpentines(5, 64)
    ref = oracle.stroke(b, uniform=True)
    db, out = _gpu(b)
    import torch
    vx, vy = torch.empty_like(out["vx"]), torch.empty_like(out["vy"])
    ps.ps_emit_uniform(db, out["params"], out["offsets"], vx, vy, out["capacity"], out["ws"])
    torch.cuda.synchronize()
    R = out["total_ribs"]
    err = np.hypot(_np(vx)[:2 * R] - ref["vx"], _np(vy)[:2 * R] - ref["vy"])
    assert err.max() <= VERTEX_TOL, err.max()


def test_uniform_baseline_with_joins_closed_paths_and_external_conics():
    # pivots are emitted as in polar stroking; segments at t = j/N with the
    # normal of g' (a positive multiple of it for negative conic weights too)
    b = W.random_mixed(71, n_paths=40, max_segs=8, extent=400.0, join=W.JOIN_MITER, cap=W.CAP_SQUARE)
    k = np.flatnonzero(b.kind == W.KIND_K)
    b.conic_w[k[::2]] = -np.float32(0.5)
    b.conic_w[k[1::5]] = 0.0
    closed = np.zeros(b.n_paths, np.uint8)
    for p in range(0, b.n_paths, 3):
        s0, s1 = int(b.seg_begin[p]), int(b.seg_begin[p + 1]) - 1
        n = W.NPTS[int(b.kind[s1])]
        b.cx[n - 1, s1], b.cy[n - 1, s1] = b.cx[0, s0], b.cy[0, s0]
        closed[p] = 1
    b.closed = closed
    ref = oracle.stroke(b, uniform=True)
    db, out = _gpu(b)
    import torch
    vx, vy = torch.empty_like(out["vx"]), torch.empty_like(out["vy"])
    ps.ps_emit_uniform(db, out["params"], out["offsets"], vx, vy, out["capacity"], out["ws"])
    torch.cuda.synchronize()
    R = out["total_ribs"]
    assert R == int(ref["offsets"][-1])
    err = np.hypot(_np(vx)[:2 * R] - ref["vx"], _np(vy)[:2 * R] - ref["vy"])
    assert err.max() <= VERTEX_TOL, err.max()


def test_facet_stats_match_oracle():
    import torch
    b = _serpentines(6, 64)
    db, out = _gpu(b)
    R = out["total_ribs"]
    stats = torch.zeros(4, dtype=torch.float64, device="cuda")
    for uniform in (False, True):
        vx, vy = out["vx"], out["vy"]
        if uniform:
            vx, vy = torch.empty_like(vx), torch.empty_like(vy)
            ps.ps_emit_uniform(db, out["params"], out["offsets"], vx, vy, out["capacity"], out["ws"])
        ps.ps_facet_stats(db, out["offsets"], vx, vy, stats)
        torch.cuda.synchronize()
        got = oracle.stats_from_sums(_np(stats))
        # the same statistics of the same vertices, summed in another order
        ref = oracle.facet_stats(b, _np(out["offsets"]), _np(vx)[:2 * R], _np(vy)[:2 * R])
        assert got["count"] == ref["count"]
        for k in ("max_deg", "mean_deg", "sd_deg"):
            assert got[k] == pytest.approx(ref[k], rel=1e-9, abs=1e-12), (uniform, k)
    # polar stroking keeps ordinary facets below 2q
    ps.ps_facet_stats(db, out["offsets"], out["vx"], out["vy"], stats)
    torch.cuda.synchronize()
    assert oracle.stats_from_sums(_np(stats))["max_deg"] < 2 * 4.0 + 0.05


def test_facet_stats_on_exact_cusps_match_oracle():
    # exact cusps (P2 = P0 + P1 - P3): fans at the cusp, swallowtails of the
    # inner offset right after it; the same classification on both sides
    import torch
    rng = np.random.default_rng(12)
    segs = []
    for _ in range(96):
        P0 = rng.uniform(0, 512, 2); P3 = P0 + rng.uniform(-300, 300, 2)
        P1 = P0 + rng.uniform(-200, 200, 2); P2 = P0 + P1 - P3
        segs.append([(W.KIND_C, [tuple(np.round(P * 256) / 256) for P in (P0, P1, P2, P3)], 1.0)])
    b = W.paths(segs, widths=[60.0] * 96, q=math.radians(4.0))
    db, out = _gpu(b)
    R = out["total_ribs"]
    stats = torch.zeros(4, dtype=torch.float64, device="cuda")
    ps.ps_facet_stats(db, out["offsets"], out["vx"], out["vy"], stats)
    torch.cuda.synchronize()
    got = oracle.stats_from_sums(_np(stats))
    ref = oracle.facet_stats(b, _np(out["offsets"]), _np(out["vx"])[:2 * R], _np(out["vy"])[:2 * R])
    assert got["count"] == ref["count"] > 1000
    for k in ("max_deg", "mean_deg", "sd_deg"):
        assert got[k] == pytest.approx(ref[k], rel=1e-9, abs=1e-12), k


# ------------------------------------------------------------------ coverage
def _cover_gpu(b, o, x0, y0, Wd, Hd, mode):
    """ps_coverage on the oracle's own rib stream (uploaded as FP32)."""
    import torch
    db = ps.DeviceBatch(b)
    vx = torch.from_numpy(o["vx"].astype(np.float32)).cuda()
    vy = torch.from_numpy(o["vy"].astype(np.float32)).cuda()
    off = torch.from_numpy(np.ascontiguousarray(o["offsets"], np.int64)).cuda()
    top = torch.empty((Hd, Wd), dtype=torch.int32, device="cuda")
    ps.ps_coverage(db, off, vx, vy, vx.numel() // 2, top, x0, y0, mode)
    torch.cuda.synchronize()
    return _np(top)


def _tight_turns(seed, n=40, q=math.pi / 8, cap=W.CAP_BUTT):
    # small cubics stroked 30-60 wide, bending tighter than the half width:
    # bow-tie quads (butt caps leave the triangle split's excess visible)
    rng = np.random.default_rng(seed)
    segs = []
    for _ in range(n):
        c = rng.uniform(30, 220, 2)
        pts = [tuple(np.round((c + rng.uniform(-12, 12, 2)) * 64) / 64) for _ in range(4)]
        segs.append([(W.KIND_C, pts, 1.0)])
    return W.paths(segs, widths=list(rng.uniform(30, 60, n)), q=q, caps=[cap] * n, joins=[W.JOIN_ROUND] * n)


@pytest.mark.parametrize("mode", [ps.PS_COVER_QUAD, ps.PS_COVER_TRIANGLES])
@pytest.mark.parametrize("case", ["mixed", "styles", "config1", "tight", "closed"])
def test_coverage_matches_oracle(case, mode):
    if case == "mixed":
        b, frame = W.random_mixed(61, n_paths=40, max_segs=10, extent=300.0), (-20.0, -10.0, 333, 301)
    elif case == "styles":
        b = W.random_mixed(62, n_paths=30, max_segs=8, extent=256.0, join=W.JOIN_NONE, cap=W.CAP_SQUARE)
        frame = (0.0, 0.0, 256, 200)
    elif case == "config1":
        b, frame = W.config1(), (-16.5, -16.25, 97, 83)
    elif case == "tight":
        b, frame = _tight_turns(63), (0.0, 0.0, 257, 255)
    else:
        b = W.random_mixed(64, n_paths=30, max_segs=7, extent=200.0, join=W.JOIN_MITER, cap=W.CAP_ROUND)
        closed = np.ones(b.n_paths, np.uint8)
        for p in range(b.n_paths):
            s0, s1 = int(b.seg_begin[p]), int(b.seg_begin[p + 1]) - 1
            n = W.NPTS[int(b.kind[s1])]
            b.cx[n - 1, s1], b.cy[n - 1, s1] = b.cx[0, s0], b.cy[0, s0]
        b.closed = closed
        frame = (-5.0, -5.0, 215, 215)
    o = oracle.stroke(b)
    ref = oracle.coverage(b, o["offsets"], o["vx"], o["vy"], *frame, mode)
    got = _cover_gpu(b, o, *frame, mode)
    assert (ref >= 0).sum() > 500
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("shift", [1e5, 1e9])
def test_coverage_far_from_the_origin(shift):
    # at 1e5 the FP32 crossing estimate is a sample or so off and exact tests
    # correct it; at 1e9 (FP32 spacing 64 px) the kernel falls back to a
    # bisection with the exact test; both must still match sample for sample
    b = W.random_mixed(13, n_paths=10, max_segs=5, extent=96.0)
    b.cx[:] = (b.cx.astype(np.float64) + shift).astype(np.float32)
    b.cy[:] = (b.cy.astype(np.float64) + shift).astype(np.float32)
    o = oracle.stroke(b)
    for mode in (ps.PS_COVER_QUAD, ps.PS_COVER_TRIANGLES):
        frame = (shift - 8.0, shift - 4.0, 300, 200)
        ref = oracle.coverage(b, o["offsets"], o["vx"], o["vy"], *frame, mode)
        assert (ref >= 0).sum() > 1000
        np.testing.assert_array_equal(_cover_gpu(b, o, *frame, mode), ref)


def _degenerate_batch():
    # empty paths, zero-length and point segments, collinear folds, an exact
    # cusp, a conic of weight 0 and a closed contour of one line pair
    segs = [[],
            [(W.KIND_L, [(10, 10), (60, 10)], 1.0), (W.KIND_C, [(60, 10), (60, 10), (60, 10), (60, 10)], 1.0),
             (W.KIND_C, [(60, 10), (110, 10), (80, 10), (160, 10)], 1.0)],
            [],
            [(W.KIND_Q, [(20, 60), (20, 60), (70, 110)], 1.0), (W.KIND_K, [(70, 110), (40, 140), (120, 150)], 0.0),
             (W.KIND_C, [(120, 150), (121, 151), (120, 151), (121, 150)], 1.0)],
            [(W.KIND_L, [(30, 170), (90, 170)], 1.0), (W.KIND_L, [(90, 170), (30, 170)], 1.0)],
            [(W.KIND_L, [(140, 40), (140, 40)], 1.0)]]
    n = len(segs)
    return W.paths(segs, widths=[6.0, 8.0, 5.0, 12.0, 4.0, 3.0], q=math.pi / 16,
                   joins=[W.JOIN_ROUND, W.JOIN_MITER, W.JOIN_BEVEL, W.JOIN_NONE, W.JOIN_MITER_CLIP, W.JOIN_ROUND],
                   caps=[W.CAP_ROUND, W.CAP_SQUARE, W.CAP_BUTT, W.CAP_TRIANGLE, W.CAP_ROUND, W.CAP_ROUND],
                   closed=[0, 0, 0, 0, 1, 0][:n])


def test_next_rows_on_degenerate_batches():
    import torch
    b = _degenerate_batch()
    r = _compare(b)
    assert r["R"] > 50
    o = oracle.stroke(b)
    for mode in (ps.PS_COVER_QUAD, ps.PS_COVER_TRIANGLES):
        ref = oracle.coverage(b, o["offsets"], o["vx"], o["vy"], 0.0, 0.0, 200, 200, mode)
        np.testing.assert_array_equal(_cover_gpu(b, o, 0.0, 0.0, 200, 200, mode), ref)
    db, out = _gpu(b)
    R = out["total_ribs"]
    stats = torch.zeros(4, dtype=torch.float64, device="cuda")
    ps.ps_facet_stats(db, out["offsets"], out["vx"], out["vy"], stats)
    torch.cuda.synchronize()
    got = oracle.stats_from_sums(_np(stats))
    ref = oracle.facet_stats(b, _np(out["offsets"]), _np(out["vx"])[:2 * R], _np(out["vy"])[:2 * R])
    assert got["count"] == ref["count"]
    uref = oracle.stroke(b, uniform=True)
    vx, vy = torch.empty_like(out["vx"]), torch.empty_like(out["vy"])
    ps.ps_emit_uniform(db, out["params"], out["offsets"], vx, vy, out["capacity"], out["ws"])
    torch.cuda.synchronize()
    err = np.hypot(_np(vx)[:2 * R] - uref["vx"], _np(vy)[:2 * R] - uref["vy"])
    assert err.max() <= VERTEX_TOL, err.max()


def test_coverage_bow_ties_differ_from_triangles():
    b = _tight_turns(65)
    o = oracle.stroke(b)
    quad = _cover_gpu(b, o, 0.0, 0.0, 256, 256, ps.PS_COVER_QUAD)
    tri = _cover_gpu(b, o, 0.0, 0.0, 256, 256, ps.PS_COVER_TRIANGLES)
    assert np.array_equal(quad, oracle.coverage(b, o["offsets"], o["vx"], o["vy"], 0.0, 0.0, 256, 256))
    # the triangle split covers where the bow-ties leave gaps
    assert (tri >= 0).sum() > (quad >= 0).sum()


def test_coverage_edge_cases():
    b = W.random_mixed(66, n_paths=5, max_segs=4, extent=100.0)
    o = oracle.stroke(b)
    # a canvas away from every stroke, a one-pixel canvas, a one-row canvas
    for frame in ((5000.0, 5000.0, 40, 30), (50.25, 50.25, 1, 1), (0.0, 49.0, 150, 1)):
        got = _cover_gpu(b, o, *frame, ps.PS_COVER_QUAD)
        np.testing.assert_array_equal(got, oracle.coverage(b, o["offsets"], o["vx"], o["vy"], *frame))
    # a quad with a non-finite corner covers nothing
    q = W.path([(W.KIND_L, [(0, 0), (1, 0)], 1.0)], width=2.0, cap=W.CAP_BUTT)
    oq = dict(offsets=np.array([0, 0, 2, 2], np.int64),
              vx=np.array([0.25, 8.25, 0.25, 8.25], np.float32), vy=np.array([0.125, 0.125, 8.125, 8.125], np.float32))
    assert (_cover_gpu(q, oq, 0.0, 0.0, 12, 12, ps.PS_COVER_QUAD) == 0).sum() == 64
    oq["vx"][1] = np.nan
    assert np.all(_cover_gpu(q, oq, 0.0, 0.0, 12, 12, ps.PS_COVER_QUAD) == -1)
    # an empty batch: nothing covered
    e = W.paths([], widths=[])
    oe = dict(vx=np.zeros(0), vy=np.zeros(0), offsets=np.zeros(1, np.int64))
    assert np.all(_cover_gpu(e, oe, 0.0, 0.0, 16, 8, ps.PS_COVER_QUAD) == -1)


def test_coverage_full_batch_sampled():
    # the 4096-path batch on a 4096 x 4096 canvas, checked at sampled pixels
    b = W.config2()
    o = oracle.stroke(b)
    rng = np.random.default_rng(7)
    pi, pj = rng.integers(0, 4096, 384), rng.integers(0, 4096, 384)
    for mode in (ps.PS_COVER_QUAD, ps.PS_COVER_TRIANGLES):
        got = _cover_gpu(b, o, 0.0, 0.0, 4096, 4096, mode)
        ref = oracle.coverage_at(b, o["offsets"], o["vx"], o["vy"], 0.0, 0.0, pi, pj, mode)
        np.testing.assert_array_equal(got[pj, pi], ref)
        assert (ref >= 0).mean() > 0.5
