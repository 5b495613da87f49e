"""FP64 CPU oracle for polar stroking -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct implementation of the paper's method
(Kilgard, "Polar Stroking", ACM TOG 2020), written in C++ (polar_oracle.cpp)
and bound here with ctypes.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
calls it and shares no code with it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "polar_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "libpolar_oracle.so")
_SAN_LIB_PATH = os.path.join(_HERE, "libpolar_oracle_san.so")
_lib = None

ROLE_SEGMENT, ROLE_JOIN, ROLE_START_CAP, ROLE_END_CAP = 0, 1, 2, 3


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with g++ (FP64, no FMA contraction, no fast-math).

    sanitize=True builds a separate copy instrumented with AddressSanitizer and
    UndefinedBehaviorSanitizer (CPU only, for the tests).  A process loads that
    copy instead of the plain one when PS_ORACLE_SANITIZE=1 is set, and needs
    the ASan runtime preloaded (LD_PRELOAD, see asan_runtime())."""
    out = _SAN_LIB_PATH if sanitize else _LIB_PATH
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp"
        flags = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                 "-pthread"]
        if sanitize:
            flags += ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                      "-fno-sanitize-recover=undefined"]
        subprocess.check_call(["g++", *flags, _SRC, "-o", tmp])
        os.replace(tmp, out)
    return out


def asan_runtime() -> str:
    """Path of g++'s ASan runtime, for LD_PRELOAD of a process that loads the
    sanitized oracle."""
    return subprocess.check_output(["g++", "-print-file-name=libasan.so"], text=True).strip()


def _load():
    global _lib
    if _lib is None:
        sanitize = os.environ.get("PS_ORACLE_SANITIZE") == "1"
        path = build(force=False, sanitize=sanitize)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.oracle_count.argtypes = [ctypes.c_int, ctypes.c_int] + [P] * 9 + [ctypes.c_double, P, ctypes.c_int]
        lib.oracle_count.restype = ctypes.c_int
        lib.oracle_emit.argtypes = ([ctypes.c_int, ctypes.c_int] + [P] * 9
                                    + [ctypes.c_double, ctypes.c_double, P] + [P] * 6
                                    + [ctypes.c_int, ctypes.c_int])
        lib.oracle_facet_stats.argtypes = [ctypes.c_int, P, P, P, P, P]
        lib.oracle_facet_stats.restype = None
        lib.oracle_emit.restype = ctypes.c_int
        lib.oracle_segment_intervals.argtypes = [ctypes.c_int, P, P, ctypes.c_double, ctypes.c_double,
                                                 P, P, P, P, P, ctypes.c_int]
        lib.oracle_segment_intervals.restype = ctypes.c_int
        lib.oracle_dash.argtypes = [ctypes.c_int, P, P, P, P, P, ctypes.c_int, ctypes.c_double,
                                    P, P, P, P, ctypes.c_int64, ctypes.c_int64, P]
        lib.oracle_dash.restype = ctypes.c_int64
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_coverage.argtypes = [ctypes.c_int, P, P, P, P, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
        lib.oracle_coverage.restype = None
        lib.oracle_coverage_at.argtypes = [ctypes.c_int, P, P, P, P, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int]
        lib.oracle_coverage_at.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _batch_args(b):
    closed = getattr(b, "closed", None)
    return [b.n_paths, b.n_segs, _p(b.seg_begin), _p(b.kind), _p(b.cx), _p(b.cy), _p(b.conic_w),
            _p(b.width), _p(b.join), _p(b.cap), None if closed is None else _p(closed)]


def num_threads() -> int:
    return _load().oracle_num_threads()


def count(b, q: float | None = None, nthreads: int = 0) -> np.ndarray:
    """Ribs per link slot, int32 [2*S + P]."""
    q = b.q if q is None else q
    out = np.zeros(b.n_links, np.int32)
    rc = _load().oracle_count(*_batch_args(b), ctypes.c_double(q), _p(out), nthreads)
    if rc != 0:
        raise ValueError(f"oracle_count failed ({rc})")
    return out


def offsets(link_ribs: np.ndarray) -> np.ndarray:
    """Exclusive prefix sum, int64 [L+1]."""
    off = np.zeros(link_ribs.shape[0] + 1, np.int64)
    np.cumsum(link_ribs, dtype=np.int64, out=off[1:])
    return off


def emit(b, off: np.ndarray, q: float | None = None, nthreads: int = 0, uniform: bool = False) -> dict:
    """Vertices (vx, vy: [2R], N then P per rib), arc length vs [R], and per-rib
    t, psi and role.  uniform: segment ribs at t = j/N instead (the baseline)."""
    q = b.q if q is None else q
    R = int(off[-1])
    vx = np.zeros(2 * R); vy = np.zeros(2 * R); vs = np.zeros(R)
    t = np.zeros(R); psi = np.zeros(R); role = np.zeros(R, np.uint8)
    off = np.ascontiguousarray(off, np.int64)
    limit = float(getattr(b, "miter_limit", 4.0))
    rc = _load().oracle_emit(*_batch_args(b), ctypes.c_double(limit), ctypes.c_double(q), _p(off),
                             _p(vx), _p(vy), _p(vs), _p(t), _p(psi), _p(role), int(uniform), nthreads)
    if rc != 0:
        raise ValueError(f"oracle_emit failed ({rc})")
    return dict(vx=vx, vy=vy, vs=vs, t=t, psi=psi, role=role)


def facet_stats(b, off: np.ndarray, vx: np.ndarray, vy: np.ndarray) -> dict:
    """Ordinary facet angles of the segment ribs of a rib stream (FP32 vertices,
    [2R] each): count, max, mean and standard deviation, in degrees."""
    vx = np.ascontiguousarray(vx, np.float32); vy = np.ascontiguousarray(vy, np.float32)
    off = np.ascontiguousarray(off, np.int64)
    st = np.zeros(4)
    _load().oracle_facet_stats(b.n_paths, _p(b.seg_begin), _p(off), _p(vx), _p(vy), _p(st))
    return stats_from_sums(st)


COVER_QUAD, COVER_TRIANGLES = 0, 1


def coverage(b, off: np.ndarray, vx: np.ndarray, vy: np.ndarray, x0: float, y0: float, W: int, H: int,
             mode: int = COVER_QUAD) -> np.ndarray:
    """Topmost covering path per sample of a W x H canvas ([H, W] int32, -1 where
    no quad covers), from an FP32 rib stream (vx, vy: [2R])."""
    vx = np.ascontiguousarray(vx, np.float32); vy = np.ascontiguousarray(vy, np.float32)
    off = np.ascontiguousarray(off, np.int64)
    top = np.empty((H, W), np.int32)
    _load().oracle_coverage(b.n_paths, _p(b.seg_begin), _p(off), _p(vx), _p(vy), ctypes.c_double(x0),
                            ctypes.c_double(y0), W, H, mode, _p(top))
    return top


def coverage_at(b, off: np.ndarray, vx: np.ndarray, vy: np.ndarray, x0: float, y0: float, pi, pj,
                mode: int = COVER_QUAD, nthreads: int = 0) -> np.ndarray:
    """The same value at single pixels (pi[k], pj[k]), each from every quad."""
    vx = np.ascontiguousarray(vx, np.float32); vy = np.ascontiguousarray(vy, np.float32)
    off = np.ascontiguousarray(off, np.int64)
    pi = np.ascontiguousarray(pi, np.int32); pj = np.ascontiguousarray(pj, np.int32)
    out = np.empty(pi.size, np.int32)
    _load().oracle_coverage_at(b.n_paths, _p(b.seg_begin), _p(off), _p(vx), _p(vy), ctypes.c_double(x0),
                               ctypes.c_double(y0), mode, pi.size, _p(pi), _p(pj), _p(out), nthreads)
    return out


def stats_from_sums(st) -> dict:
    n, mx, s1, s2 = (float(x) for x in st)
    mean = s1 / n if n else 0.0
    var = max(0.0, s2 / n - mean * mean) if n else 0.0
    d = 180.0 / np.pi
    return dict(count=int(n), max_deg=mx * d, mean_deg=mean * d, sd_deg=np.sqrt(var) * d)


def stroke(b, q: float | None = None, nthreads: int = 0, uniform: bool = False) -> dict:
    ribs = count(b, q, nthreads)
    off = offsets(ribs)
    out = emit(b, off, q, nthreads, uniform)
    out.update(link_ribs=ribs, offsets=off)
    return out


def path_rib_begin(b, off: np.ndarray) -> np.ndarray:
    """First rib of every path (and the total at the end), int64 [P+1]."""
    p = np.arange(b.n_paths + 1, dtype=np.int64)
    return np.ascontiguousarray(off[2 * b.seg_begin.astype(np.int64) + p])


def segment_intervals(kind: int, pts, q: float, w: float = 1.0):
    """Intervals of one segment: list of (t0, t1, psi0, delta, steps)."""
    px = np.zeros(4); py = np.zeros(4)
    for i, (x, y) in enumerate(pts):
        px[i], py[i] = np.float32(x), np.float32(y)
    cap = 8
    t0 = np.zeros(cap); t1 = np.zeros(cap); p0 = np.zeros(cap); d = np.zeros(cap)
    st = np.zeros(cap, np.int32)
    n = _load().oracle_segment_intervals(kind, _p(px), _p(py), ctypes.c_double(np.float32(w)),
                                         ctypes.c_double(q), _p(t0), _p(t1), _p(p0), _p(d), _p(st), cap)
    if n < 0:
        raise ValueError("unbounded conic (w_B <= -1)")
    return [(t0[k], t1[k], p0[k], d[k], int(st[k])) for k in range(n)]


def dash(rib_begin: np.ndarray, vx: np.ndarray, vy: np.ndarray, vs: np.ndarray, pattern,
         phase: float = 0.0) -> dict:
    """Dash an FP32 rib stream: returns dx, dy ([2R']), ds ([R']) and ranges [D,2]."""
    vx = np.ascontiguousarray(vx, np.float32); vy = np.ascontiguousarray(vy, np.float32)
    vs = np.ascontiguousarray(vs, np.float32)
    rib_begin = np.ascontiguousarray(rib_begin, np.int64)
    pat = np.ascontiguousarray(pattern, np.float64)
    if len(pat) < 2 or len(pat) % 2 or not (pat.sum() > 0):
        raise ValueError("bad dash pattern")
    if not (0 <= phase <= 2.0 ** 40 * pat.sum()):
        raise ValueError("dash phase must be in [0, 2^40 periods]")
    cap = 16
    while True:
        dx = np.zeros(2 * cap); dy = np.zeros(2 * cap); ds = np.zeros(cap)
        rng = np.zeros(2 * cap, np.int64)
        nd = np.zeros(1, np.int64)
        n = _load().oracle_dash(len(rib_begin) - 1, _p(rib_begin), _p(vx), _p(vy), _p(vs), _p(pat),
                                len(pat), ctypes.c_double(phase), _p(dx), _p(dy), _p(ds), _p(rng),
                                cap, cap, _p(nd))
        if n == np.iinfo(np.int64).min:
            raise ValueError("a step lies beyond 2^50 dash periods or spans more than 2^20")
        if n >= 0 and nd[0] <= cap:
            return dict(dx=dx[:2 * n], dy=dy[:2 * n], ds=ds[:n], ranges=rng[:2 * nd[0]].reshape(-1, 2))
        cap = max(2 * cap, int(abs(n)) + 1, int(nd[0]) + 1)
