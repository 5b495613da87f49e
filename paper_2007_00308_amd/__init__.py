"""MI355X polar-stroking tessellator: Python binding of the C ABI (include/ps.h).

Every function here only marshals arguments to libpolarstroke.so (hand-written
HIP kernels for gfx950); all tessellation work runs in those kernels.  PyTorch
provides device memory and the current HIP stream.  Loading fails loudly when
the native library has not been built -- there is no CPU fallback.

Method: M. J. Kilgard, "Polar Stroking: New Theory and Methods for Stroking
Paths", ACM TOG 39(4) art. 145, 2020.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libpolarstroke.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "ps.h")

PS_OK, PS_E_ARG, PS_E_WORKSPACE, PS_E_HIP, PS_E_NOMEM, PS_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
PS_MAP_DEFAULT, PS_MAP_TILES, PS_MAP_LINKS = 0, 1, 2
PS_PREC_FP32, PS_PREC_FP32_FIXUP, PS_PREC_FP64 = 0, 1, 2
PS_STATUS_OVERFLOW, PS_STATUS_NONFINITE, PS_STATUS_BAD_VALUE = 1, 2, 4
PS_STATUS_DASH_OVERFLOW, PS_STATUS_INTERVALS = 8, 16

_vp = ctypes.c_void_p


class ps_batch(ctypes.Structure):
    _fields_ = [("n_paths", ctypes.c_int32), ("n_segs", ctypes.c_int32), ("seg_begin", _vp),
                ("kind", _vp), ("cx", _vp), ("cy", _vp), ("conic_w", _vp), ("width", _vp),
                ("join", _vp), ("cap", _vp), ("closed", _vp)]


class ps_params(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("precision", ctypes.c_int32), ("n_dash", ctypes.c_int32),
                ("dash", _vp), ("dash_phase", ctypes.c_double), ("miter_limit", ctypes.c_double),
                ("emit_mapping", ctypes.c_int32), ("emit_ribs_per_lane", ctypes.c_int32),
                ("emit_waves", ctypes.c_int32), ("reserved", ctypes.c_int32)]


PS_COVER_QUAD, PS_COVER_TRIANGLES = 0, 1


class ps_canvas(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("mode", ctypes.c_int32)]


class ps_status(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("total_ribs", ctypes.c_int64), ("fixups", ctypes.c_int64),
                ("dash_ribs", ctypes.c_int64), ("dash_count", ctypes.c_int64)]


_lib = None


def declared_functions(header: str = HEADER) -> list:
    """Names of the functions include/ps.h declares."""
    text = re.sub(r"/\*.*?\*/", "", open(header).read(), flags=re.S)
    return re.findall(r"^[A-Za-z_][\w \*]*?\b(ps_\w+)\s*\(", text, flags=re.M)


def load(path: str = LIB_PATH):
    """Load libpolarstroke.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"native library missing: {path} (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    sig = {
        "ps_num_links": (ctypes.c_int64, [P(ps_batch)]),
        "ps_workspace_bytes": (ctypes.c_size_t, [P(ps_batch), P(ps_params), ctypes.c_int64]),
        "ps_count": (ctypes.c_int, [P(ps_batch), P(ps_params), _vp, _vp, ctypes.c_size_t, _vp]),
        "ps_scan": (ctypes.c_int, [_vp, ctypes.c_int64, _vp, _vp, ctypes.c_size_t, _vp]),
        "ps_emit": (ctypes.c_int, [P(ps_batch), P(ps_params), _vp, _vp, _vp, _vp, ctypes.c_int64,
                                   _vp, ctypes.c_size_t, _vp]),
        "ps_arclen": (ctypes.c_int, [P(ps_batch), P(ps_params), _vp, _vp, ctypes.c_int64, _vp,
                                     ctypes.c_size_t, _vp]),
        "ps_dash": (ctypes.c_int, [P(ps_batch), P(ps_params), _vp, _vp, _vp, _vp, ctypes.c_int64,
                                   _vp, _vp, _vp, _vp, ctypes.c_int64, ctypes.c_int64, _vp,
                                   ctypes.c_size_t, _vp]),
        "ps_read_status": (ctypes.c_int, [_vp, P(ps_status), _vp]),
        "ps_stroke_static": (ctypes.c_int, [P(ps_batch), P(ps_params), _vp, _vp, _vp, _vp, _vp,
                                            ctypes.c_int64, _vp, _vp]),
        "ps_plan_create": (ctypes.c_int, [P(ps_batch), P(ps_params), _vp, _vp, _vp, _vp, _vp,
                                          ctypes.c_int64, _vp, _vp, _vp, _vp, ctypes.c_int64,
                                          ctypes.c_int64, _vp, ctypes.c_size_t, _vp, P(_vp)]),
        "ps_plan_launch": (ctypes.c_int, [_vp, _vp]),
        "ps_plan_launch_timed": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
        "ps_plan_destroy": (ctypes.c_int, [_vp]),
        "ps_plan_config": (ctypes.c_int, [_vp, P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32)]),
        "ps_emit_uniform": (ctypes.c_int, [P(ps_batch), P(ps_params), _vp, _vp, _vp, ctypes.c_int64, _vp,
                                           ctypes.c_size_t, _vp]),
        "ps_facet_stats": (ctypes.c_int, [P(ps_batch), _vp, _vp, _vp, _vp, _vp]),
        "ps_coverage": (ctypes.c_int, [P(ps_batch), _vp, _vp, _vp, ctypes.c_int64, P(ps_canvas), _vp, _vp]),
        "ps_last_error": (ctypes.c_char_p, []),
        "ps_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class PsError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = load().ps_last_error().decode()
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


def _check(rc: int, where: str):
    if rc != PS_OK:
        raise PsError(rc, where)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


# ----------------------------------------------------------------------------
# Device-resident batches
# ----------------------------------------------------------------------------
class DeviceBatch:
    """A workloads.Batch copied to device tensors, with its ps_batch struct."""

    def __init__(self, b, device="cuda"):
        import torch
        b.validate()
        self.host = b
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        self.seg_begin = t(b.seg_begin)
        self.kind = t(b.kind)
        self.cx = t(b.cx.reshape(-1))
        self.cy = t(b.cy.reshape(-1))
        self.conic_w = t(b.conic_w)
        self.width = t(b.width)
        self.join = t(b.join)
        self.cap = t(b.cap)
        self.closed = None if b.closed is None else t(b.closed)
        self.miter_limit = float(b.miter_limit)
        self.n_paths, self.n_segs = b.n_paths, b.n_segs
        self.n_links = 2 * b.n_segs + b.n_paths
        self.struct = ps_batch(self.n_paths, self.n_segs, _ptr(self.seg_begin), _ptr(self.kind),
                               _ptr(self.cx), _ptr(self.cy), _ptr(self.conic_w), _ptr(self.width),
                               _ptr(self.join), _ptr(self.cap), _ptr(self.closed))


def make_params(q: float, precision: int = PS_PREC_FP64, dash=(), dash_phase: float = 0.0,
                miter_limit: float = 4.0, emit=(PS_MAP_DEFAULT, 0, 0)):
    """emit: (mapping PS_MAP_*, ribs per lane K, wavefronts per workgroup); 0 = default."""
    arr = (ctypes.c_double * max(1, len(dash)))(*dash) if len(dash) else None
    p = ps_params(float(q), int(precision), len(dash), ctypes.cast(arr, _vp) if arr else None,
                  float(dash_phase), float(miter_limit), int(emit[0]), int(emit[1]), int(emit[2]), 0)
    p._keep = arr   # keep the host pattern alive with the struct
    return p


# ----------------------------------------------------------------------------
# The ABI calls, one to one (argument marshalling only)
# ----------------------------------------------------------------------------
def ps_num_links(db: DeviceBatch) -> int:
    return int(load().ps_num_links(ctypes.byref(db.struct)))


def ps_workspace_bytes(db: DeviceBatch, params: ps_params, vertex_capacity: int) -> int:
    return int(load().ps_workspace_bytes(ctypes.byref(db.struct), ctypes.byref(params),
                                         int(vertex_capacity)))


def ps_count(db, params, link_ribs, ws, stream=None):
    _check(load().ps_count(ctypes.byref(db.struct), ctypes.byref(params), _ptr(link_ribs), _ptr(ws),
                           ws.numel() * ws.element_size(), _stream(stream)), "ps_count")


def ps_scan(link_ribs, n_links, offsets, ws, stream=None):
    _check(load().ps_scan(_ptr(link_ribs), int(n_links), _ptr(offsets), _ptr(ws),
                          ws.numel() * ws.element_size(), _stream(stream)), "ps_scan")


def ps_emit(db, params, offsets, vx, vy, vs, vertex_capacity, ws, stream=None):
    _check(load().ps_emit(ctypes.byref(db.struct), ctypes.byref(params), _ptr(offsets), _ptr(vx),
                          _ptr(vy), _ptr(vs), int(vertex_capacity), _ptr(ws),
                          ws.numel() * ws.element_size(), _stream(stream)), "ps_emit")


def ps_emit_uniform(db, params, offsets, vx, vy, vertex_capacity, ws, stream=None):
    _check(load().ps_emit_uniform(ctypes.byref(db.struct), ctypes.byref(params), _ptr(offsets), _ptr(vx),
                                  _ptr(vy), int(vertex_capacity), _ptr(ws), ws.numel() * ws.element_size(),
                                  _stream(stream)), "ps_emit_uniform")


def ps_facet_stats(db, offsets, vx, vy, stats, stream=None):
    _check(load().ps_facet_stats(ctypes.byref(db.struct), _ptr(offsets), _ptr(vx), _ptr(vy), _ptr(stats),
                                 _stream(stream)), "ps_facet_stats")


def ps_coverage(db, offsets, vx, vy, n_ribs, top, x0=0.0, y0=0.0, mode=PS_COVER_QUAD, stream=None):
    """top: int32 device tensor [height, width], overwritten with the topmost
    covering path index per pixel sample (-1 for none)."""
    H, W = top.shape
    cv = ps_canvas(float(x0), float(y0), int(W), int(H), int(mode))
    _check(load().ps_coverage(ctypes.byref(db.struct), _ptr(offsets), _ptr(vx), _ptr(vy), int(n_ribs),
                              ctypes.byref(cv), _ptr(top), _stream(stream)), "ps_coverage")


def ps_arclen(db, params, offsets, vs, vertex_capacity, ws, stream=None):
    _check(load().ps_arclen(ctypes.byref(db.struct), ctypes.byref(params), _ptr(offsets), _ptr(vs),
                            int(vertex_capacity), _ptr(ws), ws.numel() * ws.element_size(),
                            _stream(stream)), "ps_arclen")


def ps_dash(db, params, offsets, vx, vy, vs, vertex_capacity, dx, dy, ds, dash_range,
            rib_capacity, dash_capacity, ws, stream=None):
    _check(load().ps_dash(ctypes.byref(db.struct), ctypes.byref(params), _ptr(offsets), _ptr(vx),
                          _ptr(vy), _ptr(vs), int(vertex_capacity), _ptr(dx), _ptr(dy), _ptr(ds),
                          _ptr(dash_range), int(rib_capacity), int(dash_capacity), _ptr(ws),
                          ws.numel() * ws.element_size(), _stream(stream)), "ps_dash")


def ps_stroke_static(db, params, link_ribs, offsets, vx, vy, vs, vertex_capacity, status_flags=None,
                     stream=None):
    _check(load().ps_stroke_static(ctypes.byref(db.struct), ctypes.byref(params), _ptr(link_ribs),
                                   _ptr(offsets), _ptr(vx), _ptr(vy), _ptr(vs), int(vertex_capacity),
                                   _ptr(status_flags), _stream(stream)), "ps_stroke_static")


def ps_read_status(ws, stream=None) -> ps_status:
    st = ps_status()
    _check(load().ps_read_status(_ptr(ws), ctypes.byref(st), _stream(stream)), "ps_read_status")
    return st


def ps_version() -> str:
    return load().ps_version().decode()


def alloc_workspace(nbytes: int, device="cuda"):
    """A 256-byte aligned uint8 device buffer of at least nbytes."""
    import torch
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-int(buf.data_ptr())) % 256
    return buf[off:off + int(nbytes)]


# ----------------------------------------------------------------------------
# Convenience: the whole chain, with the rib total read back once
# ----------------------------------------------------------------------------
def stroke(db: DeviceBatch, q: float, precision: int = PS_PREC_FP64, vertex_capacity=None,
           with_arclen: bool = True, dash=(), dash_phase: float = 0.0, stream=None,
           emit=(PS_MAP_DEFAULT, 0, 0)) -> dict:
    """count -> scan -> (read total) -> emit [-> dash]; returns device tensors."""
    import torch
    dev = db.seg_begin.device
    params = make_params(q, precision, dash, dash_phase, db.miter_limit, emit)
    link_ribs = torch.empty(max(1, db.n_links), dtype=torch.int32, device=dev)
    offsets = torch.empty(db.n_links + 1, dtype=torch.int64, device=dev)
    ws0 = alloc_workspace(ps_workspace_bytes(db, params, 0), dev)
    ps_count(db, params, link_ribs, ws0, stream)
    ps_scan(link_ribs, db.n_links, offsets, ws0, stream)
    st = ps_read_status(ws0, stream)
    R = int(st.total_ribs)
    cap = 2 * R if vertex_capacity is None else int(vertex_capacity)
    ws = alloc_workspace(ps_workspace_bytes(db, params, cap), dev)
    ws[:ws0.numel()].copy_(ws0)   # the setup records live in the workspace prefix
    vx = torch.empty(max(2, cap), dtype=torch.float32, device=dev)
    vy = torch.empty_like(vx)
    vs = torch.empty_like(vx) if with_arclen else None
    ps_emit(db, params, offsets, vx, vy, vs, cap, ws, stream)
    out = dict(link_ribs=link_ribs[:db.n_links], offsets=offsets, vx=vx[:2 * R], vy=vy[:2 * R],
               vs=None if vs is None else vs[:2 * R], total_ribs=R, ws=ws, params=params,
               capacity=cap)
    if dash:
        # a first pass with a guessed capacity; on overflow the status word
        # holds the exact totals, and one more pass with those must fit
        rcap, dcap = max(16, 2 * R), max(16, R)
        for attempt in range(2):
            dx = torch.empty(2 * rcap, dtype=torch.float32, device=dev)
            dy = torch.empty_like(dx)
            ds = torch.empty_like(dx)
            rng = torch.empty(2 * dcap, dtype=torch.int64, device=dev)
            ps_dash(db, params, offsets, vx, vy, vs, cap, dx, dy, ds, rng, rcap, dcap, ws, stream)
            st = ps_read_status(ws, stream)
            if not (st.flags & PS_STATUS_DASH_OVERFLOW):
                break
            if attempt == 1:
                raise RuntimeError(f"ps_dash overflowed twice (needs {st.dash_ribs} ribs, "
                                   f"{st.dash_count} dashes)")
            rcap, dcap = max(16, int(st.dash_ribs)), max(16, int(st.dash_count))
        nr, nd = int(st.dash_ribs), int(st.dash_count)
        out.update(dx=dx[:2 * nr], dy=dy[:2 * nr], ds=ds[:2 * nr], dash_range=rng[:2 * nd].view(-1, 2))
    out["status"] = ps_read_status(ws, stream)
    return out


class Plan:
    """ps_plan_create / ps_plan_launch / ps_plan_destroy around owned buffers."""

    def __init__(self, db: DeviceBatch, q: float, vertex_capacity: int,
                 precision: int = PS_PREC_FP64, dash=(), dash_phase: float = 0.0,
                 dash_rib_capacity: int = 0, dash_capacity: int = 0, stream=None,
                 emit=(PS_MAP_DEFAULT, 0, 0)):
        """emit = (PS_MAP_DEFAULT, 0, 0) times every mapping on the batch; an
        explicit mapping is taken as is."""
        import torch
        dev = db.seg_begin.device
        self.db = db
        self.params = make_params(q, precision, dash, dash_phase, db.miter_limit, emit)
        self.capacity = int(vertex_capacity)
        self.link_ribs = torch.empty(max(1, db.n_links), dtype=torch.int32, device=dev)
        self.offsets = torch.empty(db.n_links + 1, dtype=torch.int64, device=dev)
        self.vx = torch.empty(max(2, self.capacity), dtype=torch.float32, device=dev)
        self.vy = torch.empty_like(self.vx)
        self.vs = torch.empty_like(self.vx)
        self.ws = alloc_workspace(ps_workspace_bytes(db, self.params, self.capacity), dev)
        nd = len(dash)
        self.dx = self.dy = self.ds = self.dash_range = None
        if nd:
            self.dx = torch.empty(2 * max(1, dash_rib_capacity), dtype=torch.float32, device=dev)
            self.dy = torch.empty_like(self.dx)
            self.ds = torch.empty_like(self.dx)
            self.dash_range = torch.empty(2 * max(1, dash_capacity), dtype=torch.int64, device=dev)
        h = _vp()
        _check(load().ps_plan_create(ctypes.byref(db.struct), ctypes.byref(self.params),
                                     _ptr(self.link_ribs), _ptr(self.offsets), _ptr(self.vx),
                                     _ptr(self.vy), _ptr(self.vs), self.capacity, _ptr(self.dx),
                                     _ptr(self.dy), _ptr(self.ds), _ptr(self.dash_range),
                                     int(dash_rib_capacity), int(dash_capacity), _ptr(self.ws),
                                     self.ws.numel(), _stream(stream), ctypes.byref(h)),
               "ps_plan_create")
        self.handle = h

    def launch(self, stream=None):
        _check(load().ps_plan_launch(self.handle, _stream(stream)), "ps_plan_launch")

    def launch_timed(self, emit_begin, emit_end, stream=None):
        """launch(), with the graph's event nodes recording the torch.cuda.Events
        emit_begin / emit_end on either side of the emit (the events must exist:
        record each once before)."""
        _check(load().ps_plan_launch_timed(self.handle, _stream(stream), _vp(emit_begin.cuda_event),
                                           _vp(emit_end.cuda_event)), "ps_plan_launch_timed")

    def config(self):
        """(mapping, K, wavefronts per workgroup) of the plan's emit."""
        m, k, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(load().ps_plan_config(self.handle, ctypes.byref(m), ctypes.byref(k), ctypes.byref(w)),
               "ps_plan_config")
        return int(m.value), int(k.value), int(w.value)

    def status(self, stream=None) -> ps_status:
        return ps_read_status(self.ws, stream)

    def close(self):
        if getattr(self, "handle", None):
            load().ps_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
