"""Pins for the FP64 oracle (CPU only).

Each test checks the oracle against something other than itself: hand-derived
cases (tests/golden), closed forms, brute-force sampling of the curve with an
independent de Casteljau evaluator (tests/geom_ref.py), and invariants the paper
states.  A plausible slip in the oracle -- a dropped term, a wrong sign, a
swapped index, a transposed operand -- fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2007_00308_amd import workloads as W
from tests import geom_ref as G

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_derived.json")))["cases"]


def gold(name):
    return next(c for c in GOLD if c["name"] == name)


def stroke1(kind, pts, q, w=1.0, width=2.0, join=W.JOIN_ROUND, cap=W.CAP_BUTT):
    b = W.single(kind, pts, w=w, width=width, q=q, join=join, cap=cap)
    return b, oracle.stroke(b)


def seg_ribs(o, b, seg=0, path=0):
    slot = 2 * seg + path + 1
    return slice(int(o["offsets"][slot]), int(o["offsets"][slot + 1]))


def angdiff(a, b):
    return (a - b + np.pi) % (2 * np.pi) - np.pi


# ---------------------------------------------------------------- golden cases
def test_golden_cusp():
    c = gold("exact cusp cubic")
    q = math.radians(c["q_deg"])
    iv = oracle.segment_intervals(c["kind"], c["points"], q)
    assert len(iv) == c["intervals"]
    assert [v[4] for v in iv] == c["steps"]
    b, o = stroke1(c["kind"], c["points"], q, width=c["width"])
    sl = seg_ribs(o, b)
    t = o["t"][sl]
    assert len(t) == c["ribs"]
    lo, hi = c["fan_ribs"]
    fan = np.abs(t - c["cusp_t"]) < 1e-12
    assert np.all(fan[lo:hi + 1]), np.nonzero(~fan[lo:hi + 1])
    assert not fan[lo - 1] and not fan[hi + 1]
    # the fan normals sweep pi in steps of at most q
    psi = o["psi"][sl][lo - 1:hi + 2]
    assert psi[-1] - psi[0] >= math.pi
    assert np.all(np.abs(np.diff(psi)) <= q * (1 + 1e-9))


def test_golden_line():
    c = gold("line segment")
    b, o = stroke1(c["kind"], c["points"], math.radians(c["q_deg"]), width=c["width"])
    assert o["link_ribs"].tolist() == [0, c["ribs"], 0]
    v = np.column_stack([o["vx"][0::2], o["vy"][0::2], o["vx"][1::2], o["vy"][1::2]])
    # vertex order per rib: N = G - (w/2) n, P = G + (w/2) n, n = (-sin psi, cos psi)
    np.testing.assert_allclose(v, np.array(c["vertices"])[:, [2, 3, 0, 1]], atol=1e-12)
    assert o["vs"][-1] == pytest.approx(c["length"], abs=1e-12)


def test_golden_quarter_circle():
    c = gold("quarter circle as a conic")
    q = math.radians(c["q_deg"])
    b, o = stroke1(c["kind"], c["points"], q, w=c["w"], width=c["width"])
    assert o["link_ribs"][1] == c["ribs"]
    Gx = 0.5 * (o["vx"][0::2] + o["vx"][1::2]); Gy = 0.5 * (o["vy"][0::2] + o["vy"][1::2])
    r = np.hypot(Gx, Gy)
    # FP32 rounding of the weight moves the conic off the circle by ~r*1e-8
    np.testing.assert_allclose(r, c["radius"], atol=1e-5)
    rN = np.hypot(o["vx"][0::2], o["vy"][0::2]); rP = np.hypot(o["vx"][1::2], o["vy"][1::2])
    np.testing.assert_allclose(np.sort(np.r_[rN, rP]),
                               np.sort(np.r_[np.full(len(r), c["radius"] - c["width"] / 2),
                                             np.full(len(r), c["radius"] + c["width"] / 2)]), atol=1e-5)
    # rib centres at uniform angles j*theta/N
    ang = np.arctan2(Gy, Gx)
    np.testing.assert_allclose(ang, np.linspace(0, math.pi / 2, c["ribs"]), atol=1e-7)
    assert o["vs"][-1] == pytest.approx(c["chord_sum"], abs=1e-5)


def test_golden_join():
    c = gold("right-angle round join")
    segs = [(k, pts, 1.0) for k, pts in c["segments"]]
    b = W.path(segs, width=c["width"], q=math.radians(c["q_deg"]), join=c["join"], cap=c["cap"])
    o = oracle.stroke(b)
    assert o["link_ribs"].tolist() == c["link_ribs"]
    j = slice(2, 35)
    # pivot at the shared point; outer vertex at w/2 on the outside (N side for a left turn)
    d_out = np.hypot(o["vx"][0::2][j] - 100, o["vy"][0::2][j] - 0)
    d_in = np.hypot(o["vx"][1::2][j] - 100, o["vy"][1::2][j] - 0)
    np.testing.assert_allclose(d_out, c["width"] / 2, atol=1e-12)
    np.testing.assert_allclose(d_in, 0, atol=1e-12)
    # the outer vertex lies outside the turn: below/right of the corner
    assert np.all(o["vx"][0::2][j] >= 100 - 1e-9) and np.all(o["vy"][0::2][j] <= 1e-9)


def _gold_path(c):
    segs = [(k, pts, (rest[0] if rest else 1.0)) for k, pts, *rest in c["segments"]]
    return W.path(segs, width=c["width"], q=math.radians(c["q_deg"]), join=c["join"], cap=c["cap"],
                  closed=bool(c["closed"]), miter_limit=c["miter_limit"])


def test_golden_closed_square_miter():
    c = gold("closed square with miter joins")
    b = _gold_path(c)
    o = oracle.stroke(b)
    assert o["link_ribs"].tolist() == c["link_ribs"]
    off = o["offsets"]
    for n, corner in enumerate(c["miter_corners"]):
        slot = 2 * n + 2                       # the join after segment n
        r1 = int(off[slot]) + 1                # ribs 1 and 2 of the join
        for r in (r1, r1 + 1):
            # left turns: the outer vertex is the N one (even index)
            assert (o["vx"][2 * r], o["vy"][2 * r]) == pytest.approx(tuple(corner), abs=1e-12)
    assert o["vs"][-1] == pytest.approx(c["total_length"], abs=1e-9)
    assert o["vs"][0] == 0.0
    # no caps: the first rib belongs to the first segment
    assert o["role"][0] == 0


def test_golden_miter_clip():
    c = gold("right-angle miter clipped")
    o = oracle.stroke(_gold_path(c))
    r1 = int(o["offsets"][2]) + 1
    assert (o["vx"][2 * r1], o["vy"][2 * r1]) == pytest.approx(tuple(c["rib1_outer"]), abs=1e-12)
    assert (o["vx"][2 * r1 + 2], o["vy"][2 * r1 + 2]) == pytest.approx(tuple(c["rib2_outer"]), abs=1e-12)


def test_golden_miter_revert():
    c = gold("sharp miter reverted to bevel")
    o = oracle.stroke(_gold_path(c))
    r0 = int(o["offsets"][2])
    assert o["link_ribs"][2] == 4
    V = lambda r: (o["vx"][2 * r], o["vy"][2 * r])
    assert V(r0 + 1) == pytest.approx(V(r0), abs=1e-12)
    assert V(r0 + 2) == pytest.approx(V(r0 + 3), abs=1e-12)
    # and those ends are at w/2 from the corner, on the offset lines
    assert math.dist(V(r0), (100, 0)) == pytest.approx(5.0, abs=1e-12)
    assert V(r0) == pytest.approx((100, -5), abs=1e-12)


def test_golden_closed_circle():
    c = gold("closed circle of conic quarters")
    o = oracle.stroke(_gold_path(c))
    assert o["link_ribs"].tolist() == c["link_ribs"]
    # w_B = cos 45 deg rounded to FP32 bends the arcs by ~1e-9 relative
    assert o["vs"][-1] == pytest.approx(c["chord_sum"], rel=1e-8)


def test_golden_two_conic_circle():
    c = gold("closed circle of two conics, one external")
    b = _gold_path(c)
    o = oracle.stroke(b)
    assert o["link_ribs"].tolist() == c["link_ribs"]
    seg2 = c["segments"][1]
    iv = oracle.segment_intervals(seg2[0], seg2[1], math.radians(c["q_deg"]), w=seg2[2])
    got = [(math.degrees(p0) % 360, math.degrees(d), n) for _, _, p0, d, n in iv]
    for g, e in zip(got, c["intervals_external"]):
        assert g == pytest.approx(tuple(e), abs=1e-9)
    assert len(got) == len(c["intervals_external"])
    # every segment rib on the circle, at the point whose tangent is psi
    R = c["radius"]
    Gx = 0.5 * (o["vx"][0::2] + o["vx"][1::2])
    Gy = 0.5 * (o["vy"][0::2] + o["vy"][1::2])
    psi = o["psi"]
    np.testing.assert_allclose(Gx, R * np.sin(psi), atol=2e-5)
    np.testing.assert_allclose(Gy, -R * np.cos(psi), atol=2e-5)
    # w_B = -cos 45 deg rounded to FP32 pulls the external arc up to 1e-5 px
    # inside the circle; the chord sum moves with the arc length, measured here
    # by dense sampling
    short = sum(c["radius"] * abs(v[3]) for sg in c["segments"]
                for v in oracle.segment_intervals(sg[0], sg[1], math.pi / 64, w=sg[2]))
    short -= sum(G.arc_length(sg[0], sg[1], w=sg[2]) for sg in c["segments"])
    assert 1e-5 < short < 3e-5
    assert o["vs"][-1] == pytest.approx(c["chord_sum"] - short, abs=2e-7)


def test_golden_zero_weight_conic_is_its_chord():
    c = gold("conic of weight zero is its chord")
    o = oracle.stroke(_gold_path(c))
    assert o["link_ribs"].tolist() == c["link_ribs"]
    line = dict(c, segments=[[W.KIND_L, c["line"]]])
    ol = oracle.stroke(_gold_path(line))
    for k in ("vx", "vy", "vs", "psi"):
        np.testing.assert_array_equal(o[k], ol[k])
    # the same conic with P0 == P2 is a point: no ribs
    pt = dict(c, segments=[[W.KIND_K, [[10, 20], [-37, 55], [10, 20]], 0.0]])
    assert oracle.stroke(_gold_path(pt))["link_ribs"].tolist() == [0, 0, 0]


@pytest.mark.parametrize("w", [-1.0, -1.5, -40.0])
def test_unbounded_conics_are_rejected(w):
    # w_B <= -1: the denominator (1-t)^2 + 2 w_B (1-t) t + t^2 has a root in
    # [0,1] (at t = 1/2 for w_B = -1), so the curve runs to infinity there
    pts = [(0, 0), (5, 5), (10, -1)]
    with pytest.raises(ValueError):
        oracle.segment_intervals(W.KIND_K, pts, math.pi / 64, w=w)
    b = W.single(W.KIND_K, pts, w=w, width=2.0, q=math.pi / 64)
    with pytest.raises(ValueError):
        oracle.count(b)
    t = 0.5 + 0.5 * math.sqrt((-1 - w) / (1 - w))
    assert (1 - t) ** 2 + 2 * w * (1 - t) * t + t * t == pytest.approx(0.0, abs=1e-12)


def test_external_conic_is_the_complementary_arc():
    # the same control points with weights w and -w trace complementary arcs
    # of one conic: together they turn a full 2 pi, and the external arc
    # leaves P0 backwards along -(P1 - P0)
    pts = [(0, 0), (30, 40), (90, 10)]
    for w in (0.2, 0.6, 0.95):
        q = math.pi / 256
        ti = sum(v[3] for v in oracle.segment_intervals(W.KIND_K, pts, q, w=w))
        te = sum(v[3] for v in oracle.segment_intervals(W.KIND_K, pts, q, w=-w))
        assert abs(ti) + abs(te) == pytest.approx(2 * math.pi, abs=1e-12)
        assert np.sign(ti) == -np.sign(te)
        iv = oracle.segment_intervals(W.KIND_K, pts, q, w=-w)
        assert iv[0][2] == pytest.approx(math.atan2(-40, -30), abs=1e-12)
        # points of the external arc satisfy the implicit equation of the
        # conic through the internal arc (fit on the internal arc)
        ti_ = np.linspace(0.05, 0.95, 7)
        P = G.point(W.KIND_K, pts, ti_, w)
        M = np.column_stack([P[:, 0] ** 2, P[:, 0] * P[:, 1], P[:, 1] ** 2, P[:, 0], P[:, 1], np.ones(7)])
        coef = np.linalg.svd(M)[2][-1]
        Q = G.point(W.KIND_K, pts, np.linspace(0.01, 0.99, 50), -w)
        res = (coef[0] * Q[:, 0] ** 2 + coef[1] * Q[:, 0] * Q[:, 1] + coef[2] * Q[:, 1] ** 2
               + coef[3] * Q[:, 0] + coef[4] * Q[:, 1] + coef[5])
        scale = np.abs(M @ coef).max() + np.abs(coef[:3]).max() * 1e4
        assert np.abs(res).max() < 1e-9 * scale


def test_collinear_external_conic_folds():
    # collinear control points with a negative weight: the curve leaves P0
    # backwards (along -(P1 - P0)), turns round (a +pi pivot at the fold),
    # overshoots P2 and turns round again to arrive along -(P2 - P1)
    pts = [(0, 0), (40, 0), (100, 0)]
    iv = oracle.segment_intervals(W.KIND_K, pts, math.pi / 64, w=-0.5)
    assert [v[3] for v in iv] == [0.0, math.pi, 0.0, math.pi, 0.0]
    assert [v[4] for v in iv] == [1, 64, 1, 64, 1]
    ts = np.linspace(0, 1, 200_001)
    x = G.point(W.KIND_K, pts, ts, -0.5)[:, 0]
    assert iv[1][0] == pytest.approx(ts[np.argmin(x)], abs=1e-5)
    assert iv[3][0] == pytest.approx(ts[np.argmax(x)], abs=1e-5)
    assert x.min() < 0 and x.max() > 100
    assert abs(angdiff(iv[0][2], math.pi)) < 1e-15


def test_miter_within_limit_is_on_both_offset_lines():
    # any turn: within the limit the miter vertex lies at w/2 from both
    # segments' lines (the meeting point of the two offset lines)
    rng = np.random.default_rng(17)
    for _ in range(40):
        a = rng.uniform(-3.0, 3.0)
        pts = [(0.0, 0.0), (64.0, 0.0), (64.0 + 64.0 * math.cos(a), 64.0 * math.sin(a))]
        b = W.path([(W.KIND_L, pts[:2], 1.0), (W.KIND_L, pts[1:], 1.0)], width=6.0, q=math.pi / 32,
                   join=W.JOIN_MITER, cap=W.CAP_BUTT, miter_limit=1e6)
        o = oracle.stroke(b)
        if o["link_ribs"][2] == 0:
            continue
        r1 = int(o["offsets"][2]) + 1
        k = 2 * r1 if a > 0 else 2 * r1 + 1
        M = np.array([o["vx"][k], o["vy"][k]])
        d1 = abs(M[1])                                                  # line y = 0
        end = np.array([b.cx[1, 1], b.cy[1, 1]], np.float64)            # the stored (FP32) end point
        u = (end - (64.0, 0.0)) / np.linalg.norm(end - (64.0, 0.0))
        d2 = abs((M[0] - 64.0) * u[1] - M[1] * u[0])                    # line through (64,0) along u
        assert d1 == pytest.approx(3.0, rel=1e-9) and d2 == pytest.approx(3.0, rel=1e-9)


@pytest.mark.parametrize("cap", [0, 1, 2, 3])
def test_golden_caps(cap):
    c = gold("caps")
    b, o = stroke1(c["kind"], c["points"], math.radians(c["q_deg"]), width=c["width"], cap=cap)
    J = c["cap_ribs"][str(cap)]
    assert o["link_ribs"].tolist() == [J, 2, J]
    if J == 0:
        return
    r = c["width"] / 2
    # start cap: outer vertices on the N side, behind the start point (x <= 0)
    sN = np.column_stack([o["vx"][0:2 * J:2], o["vy"][0:2 * J:2]])
    sP = np.column_stack([o["vx"][1:2 * J:2], o["vy"][1:2 * J:2]])
    np.testing.assert_allclose(sP, 0, atol=1e-12)
    assert np.all(sN[:, 0] <= 1e-9)
    d = np.hypot(sN[:, 0], sN[:, 1])
    if cap == W.CAP_SQUARE:
        np.testing.assert_allclose(d, [r, r * math.sqrt(2), r, r * math.sqrt(2), r], atol=1e-12)
        np.testing.assert_allclose(sN[2], [-r, 0], atol=1e-12)
    else:
        np.testing.assert_allclose(d, r, atol=1e-12)
    # the start cap ends on the N vertex of the segment's first rib (no twist)
    np.testing.assert_allclose(sN[-1], [o["vx"][2 * J], o["vy"][2 * J]], atol=1e-12)
    # end cap: outer vertices on the P side, ahead of the end point (x >= 50)
    e0 = J + 2
    eP = np.column_stack([o["vx"][2 * e0 + 1::2], o["vy"][2 * e0 + 1::2]])
    assert np.all(eP[:, 0] >= 50 - 1e-9)
    np.testing.assert_allclose(eP[0], [o["vx"][2 * e0 - 1], o["vy"][2 * e0 - 1]], atol=1e-12)


# ------------------------------------------------------ closed forms over ranges
@pytest.mark.parametrize("deg", [1.0, 30.0, 89.0, 90.0, 135.0, 170.0])
def test_circular_arc_counts_and_radii(deg):
    theta = math.radians(deg)
    q = math.pi / 64
    r, cx, cy, a0 = 200.0, 300.0, 250.0, 0.3
    P0 = (cx + r * math.cos(a0), cy + r * math.sin(a0))
    P2 = (cx + r * math.cos(a0 + theta), cy + r * math.sin(a0 + theta))
    m = r / math.cos(theta / 2)
    P1 = (cx + m * math.cos(a0 + theta / 2), cy + m * math.sin(a0 + theta / 2))
    b, o = stroke1(W.KIND_K, [P0, P1, P2], q, w=math.cos(theta / 2), width=6.0)
    N = o["link_ribs"][1] - 1
    # the FP32 inputs perturb the exact turning by ~1e-7 rad
    x = theta / q
    if abs(x - round(x)) > 1e-5:
        assert N == max(1, math.ceil(x))
    Gx = 0.5 * (o["vx"][0::2] + o["vx"][1::2]) - cx; Gy = 0.5 * (o["vy"][0::2] + o["vy"][1::2]) - cy
    np.testing.assert_allclose(np.hypot(Gx, Gy), r, rtol=2e-6)
    expect = 2 * r * N * math.sin(theta / (2 * N))
    # FP32 input rounding moves the end points by up to ~3e-5 px here
    assert o["vs"][-1] == pytest.approx(expect, rel=2e-6, abs=1e-4)
    assert o["vs"][-1] <= r * theta * (1 + 1e-6)


def test_parabola_t_matches_dense_tangents():
    pts = [(0, 0), (300, 400), (700, -50)]
    q = math.pi / 90
    b, o = stroke1(W.KIND_Q, pts, q)
    sl = seg_ribs(o, b)
    t, psi = o["t"][sl], o["psi"][sl]
    d, _ = G.tangent_dirs(W.KIND_Q, pts, t)
    err = np.abs(angdiff(np.arctan2(d[:, 1], d[:, 0]), psi))
    assert err.max() < 1e-6
    # total turning = angle between the two legs of the control polygon
    turn = abs(angdiff(math.atan2(-450, 400), math.atan2(400, 300)))
    assert len(t) - 1 == math.ceil(turn / q - 1e-9)


# ------------------------------------------------------------------ brute force
TINY = [
    (W.KIND_C, [(0, 0), (1, 2), (3, 2), (4, 0)], 1.0),          # arch
    (W.KIND_C, [(0, 0), (4, 3), (-1, 3), (3, 0)], 1.0),         # loop
    (W.KIND_C, [(0, 0), (2, 3), (2, -3), (4, 0)], 1.0),         # serpentine, 1 inflection
    (W.KIND_C, [(0, 0), (3, 2), (-1, 2), (2, 0)], 1.0),         # loop-ish
    (W.KIND_C, [(0, 0), (2, 2), (-2, -2), (5, 1)], 1.0),        # 2 inflections
    (W.KIND_C, [(0, 0), (1, 1), (0, 1), (1, 0)], 1.0),          # exact cusp
    (W.KIND_Q, [(0, 0), (5, 5), (10, -1)], 1.0),
    (W.KIND_K, [(0, 0), (5, 5), (10, -1)], 0.3),                # internal ellipse
    (W.KIND_K, [(0, 0), (5, 5), (10, -1)], 3.0),                # internal hyperbola
    (W.KIND_K, [(0, 0), (0, 7), (7, 7)], 1.0),                  # parabola as conic
    (W.KIND_K, [(0, 0), (5, 5), (10, -1)], -0.3),               # external ellipse
    (W.KIND_K, [(0, 0), (0, 7), (7, 7)], -0.85),                # external ellipse, long
]


@pytest.mark.parametrize("case", range(len(TINY)))
def test_brute_force_turning_and_reversals(case):
    kind, pts, w = TINY[case]
    q = math.pi / 128
    iv = oracle.segment_intervals(kind, pts, q, w=w)
    total = sum(abs(v[3]) for v in iv)
    dense, da = G.dense_turning(kind, pts, w=w)
    assert total == pytest.approx(dense, abs=2e-3)
    # reversals = sign changes of the sampled turning (ignoring cusp jumps),
    # sampled coarsely so finite-difference noise near an inflection cannot flip it
    _, da = G.dense_turning(kind, pts, w=w, n=20_001)
    small = da[np.abs(da) < 0.5]
    sg = np.sign(small[np.abs(small) > 1e-9])
    flips = int(np.sum(sg[1:] != sg[:-1]))
    # interior boundaries that are not half-angle splits
    bounds = [v[0] for v in iv[1:]]
    splits = sum(1 for k in range(1, len(iv)) if abs(iv[k][3] - iv[k - 1][3]) < 1e-15
                 and abs(iv[k][2] - (iv[k - 1][2] + iv[k - 1][3])) < 1e-12
                 and np.sign(iv[k][3]) == np.sign(iv[k - 1][3]))
    assert flips == len(bounds) - splits


@pytest.mark.parametrize("case", range(len(TINY)))
def test_brute_force_rib_directions(case):
    kind, pts, w = TINY[case]
    q = math.pi / 64
    b, o = stroke1(kind, pts, q, w=w)
    sl = seg_ribs(o, b)
    t, psi = o["t"][sl], o["psi"][sl]
    d, speed = G.tangent_dirs(kind, pts, t, w=w)
    ok = speed > 1e-3
    err = np.abs(angdiff(np.arctan2(d[ok, 1], d[ok, 0]), psi[ok]))
    assert err.max() < 1e-5
    # ribs with no usable tangent sit on a cusp found by sampling
    if np.any(~ok):
        ts = np.linspace(0, 1, 1_000_001)
        _, sp = G.tangent_dirs(kind, pts, ts, w=w, h=1e-7)
        tc = ts[np.argmin(sp)]
        assert np.all(np.abs(t[~ok] - tc) < 1e-6)
    # consecutive rib tangents differ by at most q
    assert np.all(np.abs(np.diff(psi)) <= q * (1 + 1e-9))


@pytest.mark.parametrize("case", range(len(TINY)))
def test_rib_points_on_curve_and_width(case):
    kind, pts, w = TINY[case]
    b, o = stroke1(kind, pts, math.pi / 64, w=w, width=0.5)
    sl = seg_ribs(o, b)
    t = o["t"][sl]
    Nx, Ny = o["vx"][0::2][sl], o["vy"][0::2][sl]
    Px, Py = o["vx"][1::2][sl], o["vy"][1::2][sl]
    ref = G.point(kind, pts, t, w)
    np.testing.assert_allclose(0.5 * (Nx + Px), ref[:, 0], atol=1e-12)
    np.testing.assert_allclose(0.5 * (Ny + Py), ref[:, 1], atol=1e-12)
    np.testing.assert_allclose(np.hypot(Px - Nx, Py - Ny), 0.5, atol=1e-12)
    # P lies to the left of the tangent psi
    psi = o["psi"][sl]
    side = (Px - Nx) * -np.sin(psi) + (Py - Ny) * np.cos(psi)
    assert np.all(side > 0)


@pytest.mark.parametrize("case", range(len(TINY)))
def test_arc_length_bounds(case):
    kind, pts, w = TINY[case]
    q = math.pi / 64
    b, o = stroke1(kind, pts, q, w=w)
    L = G.arc_length(kind, pts, w=w)
    S = o["vs"][-1]
    assert L * math.cos(q / 2) * (1 - 1e-9) <= S <= L * (1 + 1e-9)
    # converges as q shrinks
    _, o2 = stroke1(kind, pts, q / 8, w=w)
    assert abs(o2["vs"][-1] - L) < abs(S - L) + 1e-12


def test_conic_derivative_direction():
    # the closed-form t-solve of the conic must agree with dense sampling
    for w in (0.05, 0.5, 2.0, 20.0):
        pts = [(0, 0), (50, 80), (120, 10)]
        b, o = stroke1(W.KIND_K, pts, math.pi / 64, w=w)
        sl = seg_ribs(o, b)
        d, sp = G.tangent_dirs(W.KIND_K, pts, o["t"][sl], w=w, h=1e-8)
        ok = sp > 1e-6
        err = np.abs(angdiff(np.arctan2(d[ok, 1], d[ok, 0]), o["psi"][sl][ok]))
        assert err.max() < 1e-5, w


def test_collinear_fold_is_a_cusp():
    # a cubic running 0 -> 10, back to ~-3, then to 5 along the x axis
    pts = [(0, 0), (20, 0), (-15, 0), (5, 0)]
    q = math.pi / 16
    iv = oracle.segment_intervals(W.KIND_C, pts, q)
    # flat, pivot, flat, pivot, flat
    assert [v[4] for v in iv] == [1, 16, 1, 16, 1]
    assert [v[3] for v in iv] == [0.0, math.pi, 0.0, math.pi, 0.0]
    # the folds are where the sampled x velocity changes sign
    ts = np.linspace(0, 1, 1_000_001)
    x = G.point(W.KIND_C, pts, ts)[:, 0]
    turns = ts[1:-1][np.sign(np.diff(x))[1:] != np.sign(np.diff(x))[:-1]]
    np.testing.assert_allclose([iv[1][0], iv[3][0]], turns, atol=2e-6)


def test_collinear_quadratic_fold():
    # Q (0,0), (20,0), (10,0): g(t) = (40t - 30t^2, 0) runs out to x = 40/3 at
    # t = 2/3, where g' = 40 - 60t vanishes, and back to 10.  One fold: flat,
    # a +pi pivot of ceil(pi/q) steps at t = 2/3, flat (R10).
    pts = [(0, 0), (20, 0), (10, 0)]
    q = math.pi / 16
    iv = oracle.segment_intervals(W.KIND_Q, pts, q)
    assert [v[4] for v in iv] == [1, 16, 1]
    assert [v[3] for v in iv] == [0.0, math.pi, 0.0]
    assert iv[1][0] == iv[1][1]
    # the fold is where the densely sampled x velocity changes sign
    ts = np.linspace(0, 1, 1_000_001)
    x = G.point(W.KIND_Q, pts, ts)[:, 0]
    turns = ts[1:-1][np.sign(np.diff(x))[1:] != np.sign(np.diff(x))[:-1]]
    assert turns.size == 1
    np.testing.assert_allclose(iv[1][0], turns[0], atol=2e-6)
    # every pivot rib sits at the fold point, the far end of the segment's run
    b, o = stroke1(W.KIND_Q, pts, q, width=2.0)
    sl = seg_ribs(o, b)
    t = o["t"][sl]
    assert len(t) == 1 + 1 + 16 + 1
    np.testing.assert_allclose(t[1:18], turns[0], atol=2e-6)
    Gx = 0.5 * (o["vx"][0::2][sl] + o["vx"][1::2][sl])
    np.testing.assert_allclose(Gx[1:18], x.max(), atol=1e-9)
    np.testing.assert_allclose(x.max(), 40.0 / 3.0, atol=1e-9)


@pytest.mark.parametrize("pts", [
    [(0, 0), (0, 0), (40, 30), (80, 0)],        # P1 = P0
    [(0, 0), (40, 30), (80, 0), (80, 0)],       # P2 = P3
    [(0, 0), (0, 0), (80, 0), (80, 0)],         # P1 = P0 and P2 = P3 (a line)
    [(0, 0), (50, 50), (50, 50), (50, 50)],     # P1 = P2 = P3
    [(0, 0), (0, 0), (0, 0), (30, -40)],        # P0 = P1 = P2
])
def test_end_tangent_fallbacks_match_motion(pts):
    # first and last rib tangents, and the tangents the round caps pivot from,
    # equal the direction of motion just inside the ends
    b, o = stroke1(W.KIND_C, pts, math.pi / 32, cap=W.CAP_ROUND)
    sl = seg_ribs(o, b)
    psi = o["psi"][sl]
    cap0 = o["psi"][int(o["offsets"][1]) - 1]          # last rib of the start cap
    cap1 = o["psi"][int(o["offsets"][2])]              # first rib of the end cap
    assert abs(angdiff(cap0, psi[0])) < 1e-12 and abs(angdiff(cap1, psi[-1])) < 1e-12
    # chords over the first and last 1e-3 of t (the speed may vanish at an end)
    p = G.point(W.KIND_C, pts, np.array([0.0, 1e-3, 1 - 1e-3, 1.0]))
    d0 = p[1] - p[0]; d1 = p[3] - p[2]
    assert abs(angdiff(math.atan2(d0[1], d0[0]), psi[0])) < 2e-2
    assert abs(angdiff(math.atan2(d1[1], d1[0]), psi[-1])) < 2e-2


def test_zero_length_segments_are_transparent():
    segs = [(W.KIND_L, [(0, 0), (10, 0)], 1.0),
            (W.KIND_C, [(10, 0), (10, 0), (10, 0), (10, 0)], 1.0),
            (W.KIND_L, [(10, 0), (10, 10)], 1.0)]
    b = W.path(segs, width=2.0, q=math.pi / 8, cap=W.CAP_SQUARE)
    o = oracle.stroke(b)
    # slots: cap, L, join(L->L across the point), point, join(empty), L, cap
    assert o["link_ribs"].tolist() == [5, 2, 5, 0, 0, 2, 5]


# ------------------------------------------------------------- invariants
def _batch_invariants(b):
    o = oracle.stroke(b)
    q = b.q
    off = o["offsets"]
    assert off[0] == 0 and np.all(np.diff(off) == o["link_ribs"])
    role = o["role"]
    for p in range(b.n_paths):
        s0, s1 = b.seg_begin[p], b.seg_begin[p + 1]
        for slot in range(2 * s0 + p, 2 * s1 + p + 1):
            a, e = int(off[slot]), int(off[slot + 1])
            if e - a < 2:
                assert e == a
                continue
            psi = o["psi"][a:e]
            assert np.all(np.abs(np.diff(psi)) <= q * (1 + 1e-9) + 1e-12)
            if role[a] == oracle.ROLE_SEGMENT:
                N = np.column_stack([o["vx"][2 * a:2 * e:2], o["vy"][2 * a:2 * e:2]])
                P = np.column_stack([o["vx"][2 * a + 1:2 * e:2], o["vy"][2 * a + 1:2 * e:2]])
                np.testing.assert_allclose(np.hypot(*(P - N).T), b.width[p], rtol=1e-12)
    return o


def test_invariants_random_batch():
    b = W.random_mixed(7, n_paths=40, max_segs=12, extent=512.0)
    _batch_invariants(b)


def test_count_invariance_under_exact_transforms():
    b = W.random_mixed(11, n_paths=30, max_segs=10, extent=256.0)
    base = oracle.count(b)
    # rotation by 90 degrees, translation on the grid, scale by 2: all exact in FP32
    for f in (lambda x, y: (-y, x), lambda x, y: (x + 1024.0, y - 512.0), lambda x, y: (2 * x, 2 * y)):
        nx, ny = f(b.cx.astype(np.float64), b.cy.astype(np.float64))
        b2 = W.Batch(b.seg_begin, b.kind, nx.astype(np.float32), ny.astype(np.float32), b.conic_w,
                     b.width, b.join, b.cap, q=b.q)
        np.testing.assert_array_equal(oracle.count(b2), base)


def test_count_invariance_under_segment_reversal():
    b = W.random_mixed(13, n_paths=200, max_segs=1, extent=512.0, cusp_frac=0.1)
    base = oracle.count(b)
    cx, cy = b.cx.copy(), b.cy.copy()
    for i in range(b.n_segs):
        n = W.NPTS[int(b.kind[i])]
        cx[:n, i] = cx[:n, i][::-1]
        cy[:n, i] = cy[:n, i][::-1]
    b2 = W.Batch(b.seg_begin, b.kind, cx, cy, b.conic_w, b.width, b.join, b.cap, q=b.q)
    rev = oracle.count(b2)
    seg_slots = 2 * np.arange(b.n_segs) + np.arange(b.n_paths).repeat(1) + 1
    np.testing.assert_array_equal(rev[seg_slots], base[seg_slots])


# ------------------------------------------------------------------ dashing
def test_dash_straight_line():
    # one path, ribs along x with s = x: dash [10 on, 5 off]
    xs = np.array([0.0, 7.0, 12.0, 31.0, 33.0, 33.0, 40.0], np.float32)
    vx = np.repeat(xs, 2); vy = np.tile([-1.0, 1.0], len(xs)).astype(np.float32)
    d = oracle.dash(np.array([0, len(xs)]), vx, vy, xs, [10.0, 5.0])
    starts = d["ds"][d["ranges"][:, 0]]
    ends = d["ds"][d["ranges"][:, 1] - 1]
    np.testing.assert_allclose(starts, [0, 15, 30])
    np.testing.assert_allclose(ends, [10, 25, 40])
    # boundary ribs interpolate both vertices
    np.testing.assert_allclose(d["dx"][0::2], d["ds"])
    assert np.all(d["dy"][0::2] == -1) and np.all(d["dy"][1::2] == 1)


def test_dash_phase_and_restart():
    xs = np.linspace(0, 50, 11).astype(np.float32)
    vx = np.repeat(xs, 2); vy = np.zeros_like(vx)
    rb = np.array([0, 11, 22])
    d = oracle.dash(rb, np.r_[vx, vx], np.r_[vy, vy], np.r_[xs, xs], [4.0, 6.0], phase=7.0)
    # pattern position 7 at s=0 is in the gap (4..10): first dash starts at s=3
    starts = d["ds"][d["ranges"][:, 0]]
    np.testing.assert_allclose(starts, [3, 13, 23, 33, 43, 3, 13, 23, 33, 43])


# --------------------------------------------------- uniform baseline, facets
def test_facets_of_a_circle_equal_the_step():
    # polar stroking of a circular arc is a regular polygon on both sides:
    # every facet turns by the step 90/32 deg
    c = gold("quarter circle as a conic")
    b = W.single(c["kind"], c["points"], w=c["w"], width=c["width"], q=math.radians(c["q_deg"]))
    o = oracle.stroke(b)
    st = oracle.facet_stats(b, o["offsets"], o["vx"], o["vy"])
    assert st["count"] == 2 * (c["ribs"] - 2)
    assert st["max_deg"] == pytest.approx(90 / 32, abs=1e-3)
    assert st["mean_deg"] == pytest.approx(90 / 32, abs=1e-3)
    assert st["sd_deg"] < 1e-3


def test_facets_of_a_straight_segment_are_zero():
    b = W.single(W.KIND_C, [(0, 0), (10, 0), (30, 0), (60, 0)], width=4.0, q=math.pi / 16)
    for uniform in (False, True):
        o = oracle.stroke(b, uniform=uniform)
        st = oracle.facet_stats(b, o["offsets"], o["vx"], o["vy"])
        assert st["max_deg"] == 0.0


@pytest.mark.parametrize("case", range(len(TINY)))
def test_polar_facets_are_below_twice_q(case):
    # ordinary facet angles are bounded by 2q (Sec. "Uniform Tangent Angle
    # Step Tessellation")
    kind, pts, w = TINY[case]
    q = math.pi / 32
    b = W.single(kind, pts, w=w, width=3.0, q=q)
    o = oracle.stroke(b)
    st = oracle.facet_stats(b, o["offsets"], o["vx"], o["vy"])
    assert st["max_deg"] < 2 * math.degrees(q) + 1e-6


@pytest.mark.parametrize("case", range(len(TINY)))
def test_uniform_ribs_sit_at_uniform_parameters(case):
    # Eq. NaiveStroking sampled at t_j = j/N: rib centres on the curve at j/N,
    # rib direction along the normal of g'(j/N) (independent evaluator)
    kind, pts, w = TINY[case]
    b = W.single(kind, pts, w=w, width=3.0, q=math.pi / 32)
    o = oracle.stroke(b, uniform=True)
    sl = seg_ribs(o, b)
    N = sl.stop - sl.start - 1
    t = np.arange(N + 1) / N
    Gx = 0.5 * (o["vx"][0::2][sl] + o["vx"][1::2][sl]); Gy = 0.5 * (o["vy"][0::2][sl] + o["vy"][1::2][sl])
    ref = G.point(kind, pts, t, w)
    np.testing.assert_allclose(Gx, ref[:, 0], atol=1e-9 * (1 + np.abs(ref).max()))
    np.testing.assert_allclose(Gy, ref[:, 1], atol=1e-9 * (1 + np.abs(ref).max()))
    d, speed = G.tangent_dirs(kind, pts, t, w)
    nx = o["vx"][1::2][sl] - o["vx"][0::2][sl]; ny = o["vy"][1::2][sl] - o["vy"][0::2][sl]
    ok = speed > 1e-3 * speed.max()          # away from a cusp the normal is defined
    cross = (d[:, 0] * ny - d[:, 1] * nx) / 3.0          # |n| = width, so cross = +1
    np.testing.assert_allclose(cross[ok], 1.0, atol=1e-5)


def test_uniform_rib_on_an_exact_cusp_takes_the_nearby_tangent():
    # The exact cusp cubic of the golden cases has N = 68 steps, so its uniform
    # rib 34 sits at t = 1/2, where g' = 0.  Its normal then comes from the
    # tangent just before the cusp (2^-20/N back into the segment), which is
    # the direction of motion on the way in: the one-sided chord over
    # [1/2 - 2e-6, 1/2 - 1e-6] by the independent evaluator.  The way out has
    # the opposite direction, so taking the other side flips the cross product.
    c = gold("exact cusp cubic")
    pts = c["points"]
    b = W.single(c["kind"], pts, width=3.0, q=math.radians(c["q_deg"]))
    o = oracle.stroke(b, uniform=True)
    sl = seg_ribs(o, b)
    N = sl.stop - sl.start - 1
    assert N == 68
    j = N // 2
    p = G.point(c["kind"], pts, [0.5 - 2e-6, 0.5 - 1e-6, 0.5 + 1e-6, 0.5 + 2e-6])
    d_in, d_out = p[1] - p[0], p[3] - p[2]
    d_in /= np.hypot(*d_in); d_out /= np.hypot(*d_out)
    assert d_in @ d_out < -0.999                     # a cusp: the motion reverses
    r = sl.start + j
    n = np.array([o["vx"][2 * r + 1] - o["vx"][2 * r], o["vy"][2 * r + 1] - o["vy"][2 * r]]) / 3.0
    assert abs(np.hypot(*n) - 1.0) < 1e-12
    assert d_in[0] * n[1] - d_in[1] * n[0] > 1 - 1e-6


# ------------------------------------------------------------------ coverage
def _samples(W_, H_, x0=0.0, y0=0.0):
    i, j = np.meshgrid(np.arange(W_), np.arange(H_))
    return x0 + i + 0.5, y0 + j + 0.5


@pytest.mark.parametrize("join,extra", [(W.JOIN_NONE, 0), (W.JOIN_BEVEL, 6)])
def test_coverage_of_a_corner(join, extra):
    # two butt-capped lines meeting at a left turn, width 6, placed so that no
    # sample centre falls on an edge: the union of the two rectangles (16 x 6
    # and 6 x 16 samples, 3 x 3 shared = 183), plus for a bevel the 6 samples
    # of the triangle (20.25, 10.125), (20.25, 7.125), (23.25, 10.125); with no
    # join nothing bridges the two segments
    b = W.path([(W.KIND_L, [(4.25, 10.125), (20.25, 10.125)], 1.0),
                (W.KIND_L, [(20.25, 10.125), (20.25, 26.125)], 1.0)], width=6.0, join=join, cap=W.CAP_BUTT)
    o = oracle.stroke(b)
    top = oracle.coverage(b, o["offsets"], o["vx"], o["vy"], 0.0, 0.0, 32, 32)
    x, y = _samples(32, 32)
    r1 = (x > 4.25) & (x < 20.25) & (y > 7.125) & (y < 13.125)
    r2 = (x > 17.25) & (x < 23.25) & (y > 10.125) & (y < 26.125)
    bevel = (x > 20.25) & (y < 10.125) & (x - y < 13.125)
    want = r1 | r2 | (bevel if extra else False)
    assert int(want.sum()) == 183 + extra
    np.testing.assert_array_equal(top == 0, want)
    assert np.all(top[~want] == -1)


def _one_quad_path(N0, P0, P1, N1):
    # a butt-capped line whose two ribs are replaced by the given ones
    b = W.path([(W.KIND_L, [(0, 0), (1, 0)], 1.0)], width=2.0, cap=W.CAP_BUTT)
    off = np.array([0, 0, 2, 2], np.int64)
    vx = np.array([N0[0], P0[0], N1[0], P1[0]], np.float32)
    vy = np.array([N0[1], P0[1], N1[1], P1[1]], np.float32)
    return b, off, vx, vy


def test_coverage_of_a_bow_tie_quad():
    # ribs N0 P0 and N1 P1 that cross: the edges N0 P0 and P1 N1 meet at
    # X = (4.25, 4.125); the quad covers the two lobes (N1, N0, X) and
    # (P0, P1, X) -- 20 + 12 samples, counted by hand -- and the triangle
    # split (N0, P0, P1) + (N0, P1, N1) covers more
    a, bq, c, d = (0.25, 0.125), (8.25, 8.125), (8.25, 0.125), (0.25, 8.125)
    b, off, vx, vy = _one_quad_path(a, bq, c, d)
    x, y = _samples(12, 12)
    left = (x > 0.25) & (y > x - 0.125) & (y < 8.375 - x)
    right = (x < 8.25) & (y < x - 0.125) & (y > 8.375 - x)
    assert int(left.sum()) == 20 and int(right.sum()) == 12
    top = oracle.coverage(b, off, vx, vy, 0.0, 0.0, 12, 12, oracle.COVER_QUAD)
    np.testing.assert_array_equal(top == 0, left | right)
    t1 = (y > 0.125) & (y < x - 0.125) & (x < 8.25)
    t2 = (x > 0.25) & (y > 0.125) & (x + y < 8.375)
    top = oracle.coverage(b, off, vx, vy, 0.0, 0.0, 12, 12, oracle.COVER_TRIANGLES)
    np.testing.assert_array_equal(top == 0, t1 | t2)
    assert int((t1 | t2).sum()) > int((left | right).sum())


def test_coverage_of_a_ring_is_between_two_regular_polygons():
    # a closed circle of four conic quarters (radius 40 around (64, 64), width
    # 12, q = 5.625 deg: 16 steps a quarter) covers exactly the samples inside
    # the regular 64-gon of circumradius 46 and outside that of circumradius 34
    # (vertices at multiples of 5.625 deg)
    C, R, r = 64.0, 40.0, 6.0
    k = math.cos(math.pi / 4)
    quarter = [[(C + R, C), (C + R, C + R), (C, C + R)], [(C, C + R), (C - R, C + R), (C - R, C)],
               [(C - R, C), (C - R, C - R), (C, C - R)], [(C, C - R), (C + R, C - R), (C + R, C)]]
    b = W.path([(W.KIND_K, pts, k) for pts in quarter], width=2 * r, q=math.pi / 32,
               join=W.JOIN_ROUND, cap=W.CAP_ROUND, closed=True)
    o = oracle.stroke(b)
    top = oracle.coverage(b, o["offsets"], o["vx"], o["vy"], 0.0, 0.0, 128, 128)
    x, y = _samples(128, 128)
    d, phi = np.hypot(x - C, y - C), np.arctan2(y - C, x - C) % (2 * math.pi)
    step = math.pi / 32
    mid = (np.floor(phi / step) + 0.5) * step
    h = d * np.cos(phi - mid)                       # distance towards the sector's edge
    outer, inner = (R + r) * math.cos(step / 2), (R - r) * math.cos(step / 2)
    clear = (np.abs(h - outer) > 1e-4) & (np.abs(h - inner) > 1e-4)
    want = (h < outer) & (h > inner)
    assert clear.sum() > 128 * 128 - 50
    np.testing.assert_array_equal((top == 0)[clear], want[clear])


def test_coverage_converges_to_the_support_predicate():
    # round caps: the stroked region is every point within w/2 of the curve;
    # the samples on which the tessellated coverage disagrees with it shrink
    # as q does
    from scipy.spatial import cKDTree
    for kind, pts, w in TINY[:3] + TINY[7:8] + TINY[-2:-1]:
        P = np.asarray(pts, np.float64) * 12 + 20
        dense = G.point(kind, P, np.linspace(0, 1, 200_001), w)
        x, y = _samples(160, 160)
        # distances beyond 8 come back as inf (outside either way)
        dist = cKDTree(dense).query(np.column_stack([x.ravel(), y.ravel()]),
                                    distance_upper_bound=8.0)[0].reshape(x.shape)
        wrong = []
        for q in (math.pi / 8, math.pi / 32, math.pi / 128):
            b = W.single(kind, [tuple(p) for p in P], w=w, width=10.0, q=q, cap=W.CAP_ROUND)
            o = oracle.stroke(b)
            top = oracle.coverage(b, o["offsets"], o["vx"], o["vy"], 0.0, 0.0, 160, 160)
            sure = np.abs(dist - 5.0) > 2e-3
            wrong.append(int(((top == 0) != (dist < 5.0))[sure].sum()))
        inside = int((dist < 5.0).sum())
        assert wrong[2] <= wrong[1] <= wrong[0], (kind, wrong)
        assert wrong[2] <= 0.002 * inside + 2, (kind, wrong, inside)


def test_coverage_at_agrees_with_the_canvas():
    b = W.random_mixed(11, n_paths=12, max_segs=6, extent=96.0)
    o = oracle.stroke(b)
    vx, vy = o["vx"].astype(np.float32), o["vy"].astype(np.float32)
    for mode in (oracle.COVER_QUAD, oracle.COVER_TRIANGLES):
        top = oracle.coverage(b, o["offsets"], vx, vy, -8.0, -4.0, 120, 110, mode)
        rng = np.random.default_rng(3)
        pi, pj = rng.integers(0, 120, 400), rng.integers(0, 110, 400)
        got = oracle.coverage_at(b, o["offsets"], vx, vy, -8.0, -4.0, pi, pj, mode)
        np.testing.assert_array_equal(got, top[pj, pi])


def test_triangle_split_excess_shrinks_with_q():
    # a quad's winding number is the sum of its two triangles', so the split
    # covers every sample the quad does; what it adds at bow-ties shrinks as q
    # does (Sec. "Limitations"), on small cubics stroked wider than they bend
    rng = np.random.default_rng(65)
    segs, widths = [], []
    for _ in range(30):
        c = rng.uniform(30, 220, 2)
        segs.append([(W.KIND_C, [tuple(np.round((c + rng.uniform(-12, 12, 2)) * 64) / 64) for _ in range(4)], 1.0)])
        widths.append(float(rng.uniform(30, 60)))
    excess = []
    for q in (math.pi / 4, math.pi / 16, math.pi / 64):
        b = W.paths(segs, widths=widths, q=q, caps=[W.CAP_BUTT] * 30, joins=[W.JOIN_ROUND] * 30)
        o = oracle.stroke(b)
        quad = oracle.coverage(b, o["offsets"], o["vx"], o["vy"], 0.0, 0.0, 256, 256, oracle.COVER_QUAD)
        tri = oracle.coverage(b, o["offsets"], o["vx"], o["vy"], 0.0, 0.0, 256, 256, oracle.COVER_TRIANGLES)
        assert not np.any((quad >= 0) & (tri < 0))
        excess.append(int(((tri >= 0) & (quad < 0)).sum()))
    assert excess[0] > excess[1] > excess[2] and excess[0] > 100, excess


def test_coverage_skips_non_finite_quads():
    # a quad with a non-finite corner covers nothing (the others still do)
    b, off, vx, vy = _one_quad_path((0.25, 0.125), (8.25, 0.125), (8.25, 8.125), (0.25, 8.125))
    top = oracle.coverage(b, off, vx, vy, 0.0, 0.0, 12, 12)
    assert (top == 0).sum() == 64
    vx[1] = np.nan
    assert np.all(oracle.coverage(b, off, vx, vy, 0.0, 0.0, 12, 12) == -1)
    assert oracle.coverage_at(b, off, vx, vy, 0.0, 0.0, [3], [3])[0] == -1


@pytest.mark.parametrize("pattern", [[5.0], [5.0, 2.0, 1.0], [0.0, 0.0]])
def test_dash_rejects_bad_patterns(pattern):
    b = W.path([(W.KIND_L, [(0, 0), (40, 0)], 1.0)], width=2.0)
    o = oracle.stroke(b)
    with pytest.raises(ValueError):
        oracle.dash(oracle.path_rib_begin(b, o["offsets"]), o["vx"], o["vy"], o["vs"], pattern)


def test_dash_bounds_the_boundary_walk():
    # a phase beyond 2^40 periods, or a step ending 2^50 periods into the
    # pattern, is refused rather than walked (the FP64 period count would stop
    # advancing and the walk would not end)
    b = W.path([(W.KIND_L, [(0, 0), (40, 0)], 1.0)], width=2.0)
    o = oracle.stroke(b)
    pr = oracle.path_rib_begin(b, o["offsets"])
    with pytest.raises(ValueError):
        oracle.dash(pr, o["vx"], o["vy"], o["vs"], [5e-4, 5e-4], 1e15)
    # (an FP32 arc length that far out moves in steps of 2^27 periods or more,
    # so such a step also spans more than 2^20 periods)
    far = np.array([2.0 ** 51, 2.0 ** 51 + 2.0 ** 28], np.float32)
    with pytest.raises(ValueError):
        oracle.dash(pr, o["vx"], o["vy"], far, [0.5, 0.5], 0.0)
    # just inside both bounds it still dashes
    d = oracle.dash(pr, o["vx"], o["vy"], o["vs"], [10.0, 5.0], 15.0 * 2.0 ** 39)
    assert d["ranges"].shape[0] == 3
