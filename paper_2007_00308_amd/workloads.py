"""Seeded synthetic stroke workloads.

This module only draws random geometry: it holds none of the tessellation
arithmetic, so both the GPU path and the FP64 oracle can take their inputs from
it.  Every generator uses ``numpy.random.Generator(PCG64(seed))``.

Batch layout (the interface of the C ABI, see include/ps.h):
  seg_begin [P+1] int32   CSR: segments of path p are [seg_begin[p], seg_begin[p+1])
  kind      [S]   uint8   0 line, 1 quadratic, 2 conic, 3 cubic
  cx, cy    [4,S] float32 control point k of segment i at [k, i] (slots past the
                          segment's point count are ignored)
  conic_w   [S]   float32 middle weight w_B (conics only)
  width     [P]   float32 stroke width w
  join, cap [P]   uint8   join / cap style per path
  closed    [P]   uint8   1 for a closed contour (or None: every path open)
The paper gives no concrete path data (its figures and test paths are not
published with it), so every workload is synthetic with the shapes named in
the configuration descriptions below.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

KIND_L, KIND_Q, KIND_K, KIND_C = 0, 1, 2, 3
NPTS = {KIND_L: 2, KIND_Q: 3, KIND_K: 3, KIND_C: 4}
JOIN_NONE, JOIN_BEVEL, JOIN_ROUND, JOIN_TRIANGLE, JOIN_MITER, JOIN_MITER_CLIP = 0, 1, 2, 3, 4, 5
CAP_BUTT, CAP_ROUND, CAP_SQUARE, CAP_TRIANGLE = 0, 1, 2, 3

GRID = 2.0 ** -8   # coordinate grid that keeps cusp and mirror constructions exact in FP32


@dataclass
class Batch:
    seg_begin: np.ndarray
    kind: np.ndarray
    cx: np.ndarray
    cy: np.ndarray
    conic_w: np.ndarray
    width: np.ndarray
    join: np.ndarray
    cap: np.ndarray
    q: float = math.pi / 64
    dash: tuple = ()
    dash_phase: float = 0.0
    name: str = ""
    meta: dict = field(default_factory=dict)
    closed: np.ndarray | None = None
    miter_limit: float = 4.0

    @property
    def n_paths(self) -> int:
        return int(self.seg_begin.shape[0] - 1)

    @property
    def n_segs(self) -> int:
        return int(self.kind.shape[0])

    @property
    def n_links(self) -> int:
        return 2 * self.n_segs + self.n_paths

    def validate(self) -> None:
        P, S = self.n_paths, self.n_segs
        assert self.seg_begin.dtype == np.int32 and self.seg_begin[0] == 0 and self.seg_begin[-1] == S
        assert np.all(np.diff(self.seg_begin) >= 0)
        assert self.kind.dtype == np.uint8 and self.kind.shape == (S,)
        assert self.cx.dtype == np.float32 and self.cx.shape == (4, S)
        assert self.cy.dtype == np.float32 and self.cy.shape == (4, S)
        assert self.conic_w.dtype == np.float32 and self.conic_w.shape == (S,)
        assert self.width.dtype == np.float32 and self.width.shape == (P,)
        assert self.join.dtype == np.uint8 and self.join.shape == (P,)
        assert self.cap.dtype == np.uint8 and self.cap.shape == (P,)
        assert self.closed is None or (self.closed.dtype == np.uint8 and self.closed.shape == (P,))

    def subset(self, paths) -> "Batch":
        """Batch holding only the listed paths (in the given order)."""
        paths = np.asarray(paths, dtype=np.int64)
        segs = [np.arange(self.seg_begin[p], self.seg_begin[p + 1]) for p in paths]
        counts = np.array([len(s) for s in segs], dtype=np.int64)
        idx = np.concatenate(segs) if len(segs) else np.zeros(0, np.int64)
        sb = np.zeros(len(paths) + 1, np.int32)
        sb[1:] = np.cumsum(counts)
        return Batch(sb, self.kind[idx].copy(), np.ascontiguousarray(self.cx[:, idx]),
                     np.ascontiguousarray(self.cy[:, idx]), self.conic_w[idx].copy(),
                     self.width[paths].copy(), self.join[paths].copy(), self.cap[paths].copy(),
                     self.q, self.dash, self.dash_phase, self.name + "[subset]", dict(self.meta),
                     None if self.closed is None else self.closed[paths].copy(), self.miter_limit)


def _empty(S: int):
    return (np.zeros(S, np.uint8), np.zeros((4, S), np.float64), np.zeros((4, S), np.float64),
            np.ones(S, np.float32))


def _finish(seg_begin, kind, cx, cy, cw, width, join, cap, **kw) -> Batch:
    b = Batch(np.asarray(seg_begin, np.int32), np.asarray(kind, np.uint8),
              np.ascontiguousarray(cx, np.float32), np.ascontiguousarray(cy, np.float32),
              np.asarray(cw, np.float32), np.asarray(width, np.float32),
              np.asarray(join, np.uint8), np.asarray(cap, np.uint8), **kw)
    b.validate()
    return b


def _on_grid(v):
    return np.round(np.asarray(v, np.float64) / GRID) * GRID


def _mixed_paths(rng, counts, extent, *, cusp_frac=0.05, coincide_frac=0.05,
                 kind_p=(0.60, 0.25, 0.15), w_range=(0.25, 4.0)):
    """Connected paths of mixed cubic / quadratic / conic segments.

    Points are uniform in [0, extent)^2 on the 2^-8 grid.  A cusp cubic keeps
    P0 and P3 and sets P2 = P0 + P1 - P3, which places an exact cusp at t = 1/2.
    A coincident cubic gets one of P1=P0, P2=P3, P1=P2, (P1=P0 and P2=P3).
    """
    counts = np.asarray(counts, np.int64)
    S = int(counts.sum())
    P = len(counts)
    seg_begin = np.zeros(P + 1, np.int64)
    seg_begin[1:] = np.cumsum(counts)
    kind, cx, cy, cw = _empty(S)
    kinds = rng.choice([KIND_C, KIND_Q, KIND_K], size=S, p=list(kind_p)).astype(np.uint8)
    kind[:] = kinds
    # independent start point per path, then successive end points
    ends = _on_grid(rng.uniform(0, extent, size=(S + P, 2)))
    mids = _on_grid(rng.uniform(0, extent, size=(S, 2, 2)))
    special = rng.uniform(size=S)
    which = rng.integers(0, 4, size=S)
    cw[:] = rng.uniform(w_range[0], w_range[1], size=S).astype(np.float32)
    n_cusp = n_coinc = 0
    for p in range(P):
        for i in range(seg_begin[p], seg_begin[p + 1]):
            p0 = ends[i + p]
            p3 = ends[i + p + 1]
            k = kinds[i]
            if k == KIND_C:
                p1, p2 = mids[i, 0], mids[i, 1]
                if special[i] < cusp_frac:
                    p2 = p0 + p1 - p3
                    n_cusp += 1
                elif special[i] < cusp_frac + coincide_frac:
                    n_coinc += 1
                    w = which[i]
                    if w == 0:
                        p1 = p0
                    elif w == 1:
                        p2 = p3
                    elif w == 2:
                        p2 = p1
                    else:
                        p1, p2 = p0, p3
                pts = (p0, p1, p2, p3)
            else:
                pts = (p0, mids[i, 0], p3)
            for s, pt in enumerate(pts):
                cx[s, i], cy[s, i] = pt
    return seg_begin, kind, cx, cy, cw, dict(n_cusp=n_cusp, n_coincident=n_coinc)


def config1(seed: int = 1001) -> Batch:
    """One open path of 64 connected cubics, points uniform in [0,512)^2, w=8,
    q=pi/90, butt caps, round joins (the small 'plain method' case)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = _on_grid(rng.uniform(0, 512, size=(193, 2)))
    S = 64
    kind, cx, cy, cw = _empty(S)
    kind[:] = KIND_C
    for i in range(S):
        for s in range(4):
            cx[s, i], cy[s, i] = pts[3 * i + s]
    return _finish([0, S], kind, cx, cy, cw, [8.0], [JOIN_ROUND], [CAP_BUTT],
                   q=math.pi / 90, name="C1: 1 path x 64 cubics, q=pi/90")


def config2(seed: int = 1002, n_paths: int = 4096, max_segs: int = 512) -> Batch:
    """4,096 open paths, segments per path log-uniform in [1,512]; 60/25/15 %
    cubic/quadratic/conic (weight U[0.25,4]); 5% cusp cubics, 5% with
    coincident control points; coordinates in [0,4096)^2; width log-uniform in
    [0.5,64]; q=pi/64; round joins, butt caps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = np.clip(np.floor(np.exp(rng.uniform(0, math.log(max_segs + 1), size=n_paths))),
                     1, max_segs).astype(np.int64)
    sb, kind, cx, cy, cw, meta = _mixed_paths(rng, counts, 4096.0)
    width = np.exp(rng.uniform(math.log(0.5), math.log(64.0), size=n_paths))
    return _finish(sb, kind, cx, cy, cw, width, np.full(n_paths, JOIN_ROUND),
                   np.full(n_paths, CAP_BUTT), q=math.pi / 64,
                   name=f"C2: {n_paths} paths, log-uniform [1,{max_segs}] segments, q=pi/64",
                   meta=meta)


def config3(seed: int = 1003, n_segs: int = 5000) -> Batch:
    """One path of 5,000 C1-continuous cubics as a random walk (step ~N(40,10)
    px, heading jitter +-60 deg), width 2, q=pi/128, dash [10 on, 5 off].
    Interior handles mirror exactly about the joints, so every join is smooth."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = np.maximum(rng.normal(40.0, 10.0, size=n_segs), 1.0)
    dh = rng.uniform(-math.pi / 3, math.pi / 3, size=n_segs)
    h = np.cumsum(dh) + rng.uniform(-math.pi, math.pi)
    X = np.zeros((n_segs + 1, 2))
    X[0] = (8192.0, 8192.0)
    for i in range(n_segs):
        X[i + 1] = X[i] + L[i] * np.array([math.cos(h[i]), math.sin(h[i])])
    X = _on_grid(X)
    kind, cx, cy, cw = _empty(n_segs)
    kind[:] = KIND_C
    P2prev = None
    for i in range(n_segs):
        if i == 0:
            p1 = _on_grid(X[0] + (L[0] / 3) * np.array([math.cos(h[0]), math.sin(h[0])]))
        else:
            p1 = 2 * X[i] - P2prev
        hm = 0.5 * (h[i] + h[i + 1]) if i + 1 < n_segs else h[i]
        p2 = _on_grid(X[i + 1] - (L[i] / 3) * np.array([math.cos(hm), math.sin(hm)]))
        for s, pt in enumerate((X[i], p1, p2, X[i + 1])):
            cx[s, i], cy[s, i] = pt
        P2prev = p2
    assert np.abs(cx).max() < 65536 and np.abs(cy).max() < 65536
    return _finish([0, n_segs], kind, cx, cy, cw, [2.0], [JOIN_ROUND], [CAP_BUTT],
                   q=math.pi / 128, dash=(10.0, 5.0), dash_phase=0.0,
                   name=f"C3: 1 path x {n_segs} C1 cubics (random walk), q=pi/128, dash [10,5]")


def config4(seed: int = 1004, n_paths: int = 1024, max_segs: int = 64) -> Batch:
    """Precision study: config-2 style paths where a third of the segments are
    near-degenerate: control points within 1e-4 px of collinear (placed in
    [0,256)^2 so the FP32 grid is finer than the deviation), cubic cusps within
    1e-6 of t=0 or t=1, exact cusps perturbed by a few FP32 ulps into tiny loops
    or serpentines, and conic weights 10^U(-6,-2) or 10^U(2.5,3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = np.clip(np.floor(np.exp(rng.uniform(0, math.log(max_segs + 1), size=n_paths))),
                     1, max_segs).astype(np.int64)
    sb, kind, cx, cy, cw, meta = _mixed_paths(rng, counts, 256.0, cusp_frac=0.0, coincide_frac=0.0)
    S = int(counts.sum())
    roll = rng.uniform(size=S)
    n = dict(near_collinear=0, cusp_near_end=0, perturbed_cusp=0, extreme_weight=0)
    for i in range(S):
        if roll[i] > 1.0 / 3.0:
            continue
        c = rng.integers(0, 4)
        p0 = np.array([cx[0, i], cy[0, i]])
        pe = np.array([cx[NPTS[kind[i]] - 1, i], cy[NPTS[kind[i]] - 1, i]])
        if c == 0:
            # near-collinear: interior points on the chord (or beyond it), pushed off by eta
            d = pe - p0
            nrm = np.array([-d[1], d[0]]) / max(np.hypot(*d), 1e-30)
            for s in range(1, NPTS[kind[i]] - 1):
                lam = rng.uniform(-0.5, 1.5)
                pt = p0 + lam * d + rng.uniform(-1e-4, 1e-4) * nrm
                cx[s, i], cy[s, i] = pt
            n["near_collinear"] += 1
        elif c == 1 and kind[i] == KIND_C:
            # cusp at t_c within 1e-6 of an end: g'(t_c) = (1-t)^2 a + 2(1-t)t b + t^2 c = 0,
            # solved for the handle next to that end (the well-conditioned unknown)
            tc = rng.uniform(1e-8, 1e-6)
            p1 = np.array([cx[1, i], cy[1, i]])
            p2 = np.array([cx[2, i], cy[2, i]])
            if rng.uniform() < 0.5:
                u, t = 1.0 - tc, tc          # near t = 0: unknown a, keep P0, P2, P3
                cc = pe - p2
                a = -(2 * u * t * (p2 - p0) + t * t * cc) / (u * u - 2 * u * t)
                cx[1, i], cy[1, i] = p0 + a
            else:
                u, t = tc, 1.0 - tc          # near t = 1: unknown c, keep P0, P1, P3
                a = p1 - p0
                cc = -(u * u * a + 2 * u * t * (pe - p1)) / (t * t - 2 * u * t)
                cx[2, i], cy[2, i] = pe - cc
            n["cusp_near_end"] += 1
        elif c == 2 and kind[i] == KIND_C:
            # exact cusp (P2 = P0 + P1 - P3), then nudge P2 by a few ulps
            p1 = np.array([cx[1, i], cy[1, i]])
            p2 = p0 + p1 - pe
            ulp = float(np.spacing(np.float32(max(abs(p2).max(), 1.0))))
            p2 = p2 + rng.integers(-3, 4, size=2) * ulp
            cx[2, i], cy[2, i] = p2
            n["perturbed_cusp"] += 1
        elif kind[i] == KIND_K:
            cw[i] = 10.0 ** (rng.uniform(-6, -2) if rng.uniform() < 0.5 else rng.uniform(2.5, 3))
            n["extreme_weight"] += 1
    meta.update(n)
    assert np.abs(cx).max() < 1024 and np.abs(cy).max() < 1024
    width = np.exp(rng.uniform(math.log(0.5), math.log(16.0), size=n_paths))
    return _finish(sb, kind, cx, cy, cw, width, np.full(n_paths, JOIN_ROUND),
                   np.full(n_paths, CAP_BUTT), q=math.pi / 64,
                   name=f"C4: {n_paths} paths with near-degenerate segments, q=pi/64", meta=meta)


def zipf_counts(n_paths: int, total: int, s: float = 1.2) -> np.ndarray:
    i = np.arange(1, n_paths + 1, dtype=np.float64)
    H = np.sum(i ** -s)
    c = np.maximum(1, np.floor(total * i ** -s / H)).astype(np.int64)
    c[0] -= int(c.sum() - total)
    assert c.sum() == total and c.min() >= 1
    return c


def config5(seed: int = 1005, q: float = math.pi / 64, n_paths: int = 65536,
            total_segs: int = 1 << 20) -> Batch:
    """Throughput stress: 2^20 segments over 65,536 paths with rank-Zipf(1.2)
    segment counts (shuffled), segment mix as config 2, bevel joins, butt caps,
    coordinates in [0,4096)^2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = zipf_counts(n_paths, total_segs)
    rng.shuffle(counts)
    sb, kind, cx, cy, cw, meta = _mixed_paths_fast(rng, counts, 4096.0)
    width = np.exp(rng.uniform(math.log(0.5), math.log(64.0), size=n_paths))
    return _finish(sb, kind, cx, cy, cw, width, np.full(n_paths, JOIN_BEVEL),
                   np.full(n_paths, CAP_BUTT), q=q,
                   name=f"C5: {total_segs} segments over {n_paths} Zipf(1.2) paths, q={q:.5f}",
                   meta=meta)


def _mixed_paths_fast(rng, counts, extent, cusp_frac=0.05, coincide_frac=0.05,
                      kind_p=(0.60, 0.25, 0.15), w_range=(0.25, 4.0)):
    """Vectorised form of _mixed_paths for the large stress configuration."""
    counts = np.asarray(counts, np.int64)
    S = int(counts.sum())
    P = len(counts)
    seg_begin = np.zeros(P + 1, np.int64)
    seg_begin[1:] = np.cumsum(counts)
    kind = rng.choice([KIND_C, KIND_Q, KIND_K], size=S, p=list(kind_p)).astype(np.uint8)
    ends = _on_grid(rng.uniform(0, extent, size=(S + P, 2)))
    mids = _on_grid(rng.uniform(0, extent, size=(S, 2, 2)))
    path_of = np.repeat(np.arange(P), counts)
    i = np.arange(S)
    p0 = ends[i + path_of]
    p3 = ends[i + path_of + 1]
    p1 = mids[:, 0].copy()
    p2 = mids[:, 1].copy()
    special = rng.uniform(size=S)
    which = rng.integers(0, 4, size=S)
    isC = kind == KIND_C
    cusp = isC & (special < cusp_frac)
    p2[cusp] = p0[cusp] + p1[cusp] - p3[cusp]
    co = isC & (special >= cusp_frac) & (special < cusp_frac + coincide_frac)
    m = co & (which == 0); p1[m] = p0[m]
    m = co & (which == 1); p2[m] = p3[m]
    m = co & (which == 2); p2[m] = p1[m]
    m = co & (which == 3); p1[m] = p0[m]; p2[m] = p3[m]
    cx = np.zeros((4, S)); cy = np.zeros((4, S))
    cx[0], cy[0] = p0[:, 0], p0[:, 1]
    cx[1], cy[1] = p1[:, 0], p1[:, 1]
    # quadratic / conic: end point sits in slot 2
    last_x = np.where(isC, p2[:, 0], p3[:, 0]); last_y = np.where(isC, p2[:, 1], p3[:, 1])
    cx[2], cy[2] = last_x, last_y
    cx[3], cy[3] = np.where(isC, p3[:, 0], 0.0), np.where(isC, p3[:, 1], 0.0)
    cw = rng.uniform(w_range[0], w_range[1], size=S).astype(np.float32)
    return seg_begin, kind, cx, cy, cw, dict(n_cusp=int(cusp.sum()), n_coincident=int(co.sum()))


def config2_fast(seed: int = 1002, n_paths: int = 4096, max_segs: int = 512) -> Batch:
    """Same distribution as config2, drawn with the vectorised generator (used
    by the benchmark; config2 keeps the per-segment reference loop)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = np.clip(np.floor(np.exp(rng.uniform(0, math.log(max_segs + 1), size=n_paths))),
                     1, max_segs).astype(np.int64)
    sb, kind, cx, cy, cw, meta = _mixed_paths_fast(rng, counts, 4096.0)
    width = np.exp(rng.uniform(math.log(0.5), math.log(64.0), size=n_paths))
    return _finish(sb, kind, cx, cy, cw, width, np.full(n_paths, JOIN_ROUND),
                   np.full(n_paths, CAP_BUTT), q=math.pi / 64,
                   name=f"C2: {n_paths} paths, log-uniform [1,{max_segs}] segments, q=pi/64",
                   meta=meta)


def single(kind: int, pts, *, w: float = 1.0, width: float = 2.0, q: float = math.pi / 64,
           join: int = JOIN_ROUND, cap: int = CAP_BUTT) -> Batch:
    """A one-segment path from explicit control points (tests and examples)."""
    return path([(kind, pts, w)], width=width, q=q, join=join, cap=cap)


def path(segs, *, width: float = 2.0, q: float = math.pi / 64, join: int = JOIN_ROUND,
         cap: int = CAP_BUTT, closed: bool = False, miter_limit: float = 4.0) -> Batch:
    """One path from a list of (kind, points, conic_weight) tuples."""
    return paths([segs], widths=[width], q=q, joins=[join], caps=[cap],
                 closed=[closed] if closed else None, miter_limit=miter_limit)


def paths(list_of_segs, *, widths, q: float = math.pi / 64, joins=None, caps=None, closed=None,
          miter_limit: float = 4.0) -> Batch:
    P = len(list_of_segs)
    S = sum(len(s) for s in list_of_segs)
    kind, cx, cy, cw = _empty(S)
    sb = [0]
    i = 0
    for segs in list_of_segs:
        for (k, pts, w) in segs:
            kind[i] = k
            assert len(pts) == NPTS[k]
            for s, pt in enumerate(pts):
                cx[s, i], cy[s, i] = pt
            cw[i] = w
            i += 1
        sb.append(i)
    joins = [JOIN_ROUND] * P if joins is None else joins
    caps = [CAP_BUTT] * P if caps is None else caps
    cl = None if closed is None else np.asarray(closed, np.uint8)
    return _finish(sb, kind, cx, cy, cw, widths, joins, caps, q=q, name="explicit", closed=cl,
                   miter_limit=miter_limit)


def random_mixed(seed: int, n_paths: int, max_segs: int, extent: float = 1024.0,
                 q: float = math.pi / 64, join: int = JOIN_ROUND, cap: int = CAP_BUTT,
                 cusp_frac: float = 0.05, coincide_frac: float = 0.05) -> Batch:
    """Small mixed batches for parity tests (several tiles, ragged tails)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = rng.integers(1, max_segs + 1, size=n_paths)
    sb, kind, cx, cy, cw, meta = _mixed_paths_fast(rng, counts, extent, cusp_frac, coincide_frac)
    width = np.exp(rng.uniform(math.log(0.5), math.log(32.0), size=n_paths))
    return _finish(sb, kind, cx, cy, cw, width, np.full(n_paths, join), np.full(n_paths, cap),
                   q=q, name=f"mixed seed={seed}", meta=meta)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
