"""Independent numpy geometry used to pin the oracle.

de Casteljau evaluation of (rational) Bezier curves in homogeneous
coordinates, dense sampling and finite differences.  None of this shares code
or formulas with the oracle, which evaluates Bernstein polynomials directly and
solves the tangent-angle equation in closed form.
"""
import numpy as np

from paper_2007_00308_amd import workloads as W


def control(kind, pts, w=1.0):
    """Homogeneous control points (x*wt, y*wt, wt) for de Casteljau."""
    pts = np.asarray(pts, np.float32).astype(np.float64)   # batch coordinates are FP32
    wt = np.ones(len(pts))
    if kind == W.KIND_K:
        wt[1] = float(np.float32(w))   # the batch stores w_B in FP32
    return np.column_stack([pts[:, 0] * wt, pts[:, 1] * wt, wt])


def point(kind, pts, t, w=1.0):
    """Curve points at parameters t (array) by repeated linear interpolation."""
    t = np.atleast_1d(np.asarray(t, np.float64))[:, None, None]
    c = control(kind, pts, w)[None, :, :].repeat(t.shape[0], 0)
    while c.shape[1] > 1:
        c = (1 - t) * c[:, :-1] + t * c[:, 1:]
    h = c[:, 0]
    return h[:, :2] / h[:, 2:3]


def tangent_dirs(kind, pts, t, w=1.0, h=1e-7):
    """Unit tangent directions by central differences of point()."""
    t = np.asarray(t, np.float64)
    lo = np.clip(t - h, 0, 1)
    hi = np.clip(t + h, 0, 1)
    d = point(kind, pts, hi, w) - point(kind, pts, lo, w)
    n = np.hypot(d[:, 0], d[:, 1])
    return d / np.maximum(n, 1e-300)[:, None], n / np.maximum(hi - lo, 1e-300)


def dense_turning(kind, pts, w=1.0, n=1_000_001):
    """Total absolute turning of the tangent over [0,1] from n samples.  A jump
    of (nearly) pi between neighbouring samples is an exact cusp and counts pi."""
    t = np.linspace(0, 1, n)
    p = point(kind, pts, t, w)
    d = np.diff(p, axis=0)
    keep = np.hypot(d[:, 0], d[:, 1]) > 0
    ang = np.arctan2(d[keep, 1], d[keep, 0])
    da = np.diff(ang)
    da = (da + np.pi) % (2 * np.pi) - np.pi
    return float(np.sum(np.abs(da))), da


def arc_length(kind, pts, w=1.0, n=2_000_001):
    t = np.linspace(0, 1, n)
    p = point(kind, pts, t, w)
    return float(np.sum(np.hypot(*np.diff(p, axis=0).T)))
