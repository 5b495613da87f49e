"""C ABI checks that need no GPU: the library loads, exports every function
include/ps.h declares, and host-side validation rejects bad arguments before
anything is queued (no compute call is made here)."""
import ctypes
import math

import pytest

import paper_2007_00308_amd as ps


def test_library_exports_every_declared_symbol():
    lib = ps.load()
    names = ps.declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert ps.ps_version()


def _batch(n_paths=1, n_segs=1):
    fake = 0x1000   # never dereferenced: validation fails first or no call is made
    return ps.ps_batch(n_paths, n_segs, fake, fake, fake, fake, fake, fake, fake, fake)


def test_num_links_and_workspace_are_host_only():
    lib = ps.load()
    b = _batch(3, 10)
    assert lib.ps_num_links(ctypes.byref(b)) == 23
    p = ps.make_params(math.pi / 64)
    w0 = lib.ps_workspace_bytes(ctypes.byref(b), ctypes.byref(p), 0)
    w1 = lib.ps_workspace_bytes(ctypes.byref(b), ctypes.byref(p), 1 << 20)
    assert 0 < w0 < w1
    pd = ps.make_params(math.pi / 64, dash=(10.0, 5.0))
    assert lib.ps_workspace_bytes(ctypes.byref(b), ctypes.byref(pd), 1 << 20) > w1


@pytest.mark.parametrize("q", [0.0, -1.0, 1e-6, 4.0, float("nan")])
def test_bad_q_rejected(q):
    lib = ps.load()
    b = _batch()
    p = ps.make_params(q)
    rc = lib.ps_count(ctypes.byref(b), ctypes.byref(p), 0x1000, 0x1000, 1 << 30, None)
    assert rc == ps.PS_E_ARG
    assert "q must be" in lib.ps_last_error().decode()


def test_null_and_negative_arguments_rejected():
    lib = ps.load()
    p = ps.make_params(0.1)
    assert lib.ps_count(None, ctypes.byref(p), 0x1000, 0x1000, 1 << 30, None) == ps.PS_E_ARG
    b = _batch(-1, 0)
    assert lib.ps_count(ctypes.byref(b), ctypes.byref(p), 0x1000, 0x1000, 1 << 30, None) == ps.PS_E_ARG
    b = ps.ps_batch(1, 1, 0, 0, 0, 0, 0, 0, 0, 0)
    assert lib.ps_count(ctypes.byref(b), ctypes.byref(p), 0x1000, 0x1000, 1 << 30, None) == ps.PS_E_ARG
    b = _batch(0, 3)   # segments without any path
    assert lib.ps_count(ctypes.byref(b), ctypes.byref(p), 0x1000, 0x1000, 1 << 30, None) == ps.PS_E_ARG
    assert lib.ps_scan(None, 5, 0x1000, 0x1000, 1 << 30, None) == ps.PS_E_ARG
    assert lib.ps_scan(0x1000, -1, 0x1000, 0x1000, 1 << 30, None) == ps.PS_E_ARG


def test_workspace_checks():
    lib = ps.load()
    b = _batch(2, 4)
    p = ps.make_params(0.1)
    need = lib.ps_workspace_bytes(ctypes.byref(b), ctypes.byref(p), 0)
    # too small
    assert lib.ps_count(ctypes.byref(b), ctypes.byref(p), 0x1000, 0x1000, need - 1, None) == ps.PS_E_WORKSPACE
    # misaligned
    assert lib.ps_count(ctypes.byref(b), ctypes.byref(p), 0x1000, 0x1008, need, None) == ps.PS_E_ARG
    assert "aligned" in lib.ps_last_error().decode()


@pytest.mark.parametrize("dash", [(1.0,), (1.0, 2.0, 3.0), (0.0, 0.0), (-1.0, 2.0), (float("inf"), 1.0)])
def test_bad_dash_rejected(dash):
    lib = ps.load()
    b = _batch()
    p = ps.make_params(0.1, dash=dash)
    rc = lib.ps_count(ctypes.byref(b), ctypes.byref(p), 0x1000, 0x1000, 1 << 30, None)
    assert rc == ps.PS_E_ARG


def test_dash_phase_beyond_2_40_periods_rejected():
    # the boundary walk counts periods in FP64; beyond 2^40 periods of phase
    # it could stall, so such a phase is refused before anything is queued
    lib = ps.load()
    b = _batch()
    ok = ps.make_params(0.1, dash=(5e-4, 5e-4), dash_phase=1e-3 * 2.0 ** 40)
    assert lib.ps_count(ctypes.byref(b), ctypes.byref(ok), 0x1000, 0x1000, 1 << 30, None) != ps.PS_E_ARG or \
        b"phase" not in lib.ps_last_error()
    bad = ps.make_params(0.1, dash=(5e-4, 5e-4), dash_phase=1e15)
    assert lib.ps_count(ctypes.byref(b), ctypes.byref(bad), 0x1000, 0x1000, 1 << 30, None) == ps.PS_E_ARG
    assert b"2^40" in lib.ps_last_error()


def test_bad_precision_and_emit_mapping_rejected():
    lib = ps.load()
    b = _batch()
    call = lambda p: lib.ps_count(ctypes.byref(b), ctypes.byref(p), 0x1000, 0x1000, 1 << 30, None)
    assert call(ps.make_params(0.1, precision=7)) == ps.PS_E_ARG
    for emit, ok in [((ps.PS_MAP_TILES, 3, 4), False), ((ps.PS_MAP_TILES, 8, 99), False),
                     ((ps.PS_MAP_TILES, 8, 5), False),      # above the 256-thread launch bound
                     ((3, 8, 4), False), ((-1, 0, 0), False),
                     ((ps.PS_MAP_TILES, 7, 4), True), ((ps.PS_MAP_DEFAULT, 0, 0), True),
                     ((ps.PS_MAP_LINKS, 0, 2), True)]:
        rc = call(ps.make_params(0.1, emit=emit))
        if ok:
            assert rc != ps.PS_E_ARG or b"emit" not in lib.ps_last_error(), emit
        else:
            assert rc == ps.PS_E_ARG and b"emit" in lib.ps_last_error(), emit


@pytest.mark.parametrize("limit", [0.0, 0.999, float("nan"), float("inf")])
def test_bad_miter_limit_rejected(limit):
    lib = ps.load()
    b = _batch()
    p = ps.make_params(0.1, miter_limit=limit)
    assert lib.ps_count(ctypes.byref(b), ctypes.byref(p), 0x1000, 0x1000, 1 << 30, None) == ps.PS_E_ARG
    assert b"miter_limit" in lib.ps_last_error()


def test_plan_rejects_null_buffers():
    lib = ps.load()
    b = _batch()
    p = ps.make_params(0.1)
    h = ctypes.c_void_p()
    rc = lib.ps_plan_create(ctypes.byref(b), ctypes.byref(p), None, None, None, None, None, 0,
                            None, None, None, None, 0, 0, 0x1000, 1 << 30, None, ctypes.byref(h))
    assert rc == ps.PS_E_ARG and not h.value
    assert lib.ps_plan_launch(None, None) == ps.PS_E_ARG
    assert lib.ps_plan_launch_timed(None, None, None, None) == ps.PS_E_ARG
    assert lib.ps_plan_config(None, None, None, None) == ps.PS_E_ARG
    assert lib.ps_plan_destroy(None) == ps.PS_OK


@pytest.mark.parametrize("canvas,what", [(None, b"canvas is NULL"),
                                         ((0.0, 0.0, -1, 4, 0), b"negative canvas"),
                                         ((float("nan"), 0.0, 4, 4, 0), b"origin"),
                                         ((0.0, 0.0, 4, 4, 2), b"mode")])
def test_coverage_rejects_bad_canvas(canvas, what):
    lib = ps.load()
    b = _batch()
    cv = None if canvas is None else ctypes.byref(ps.ps_canvas(*canvas))
    rc = lib.ps_coverage(ctypes.byref(b), 0x1000, 0x1000, 0x1000, 4, cv, 0x1000, None)
    assert rc == ps.PS_E_ARG
    assert what in lib.ps_last_error()


def test_coverage_of_an_empty_canvas_is_a_no_op():
    # nothing to write, so no device call is made
    lib = ps.load()
    b = _batch()
    for w, h in ((0, 5), (5, 0)):
        assert lib.ps_coverage(ctypes.byref(b), None, None, None, 0,
                               ctypes.byref(ps.ps_canvas(0.0, 0.0, w, h, 0)), None, None) == ps.PS_OK


def test_coverage_rejects_a_canvas_of_2_31_pixels():
    # pixel indices are 32-bit inside the kernel
    lib = ps.load()
    b = _batch()
    cv = ps.ps_canvas(0.0, 0.0, 65536, 32768, 0)
    assert lib.ps_coverage(ctypes.byref(b), 0x1000, 0x1000, 0x1000, 4, ctypes.byref(cv), 0x1000, None) == ps.PS_E_ARG
    assert b"2^31" in lib.ps_last_error()


def test_static_chain_refuses_large_batches_and_dashing_on_the_host():
    # both are decided before any device call
    lib = ps.load()
    b = _batch(1000, 1_000_000)
    p = ps.make_params(0.1)
    rc = lib.ps_stroke_static(ctypes.byref(b), ctypes.byref(p), 0x1000, 0x1000, 0x1000, 0x1000, 0x1000,
                              1 << 20, None, None)
    assert rc == ps.PS_E_WORKSPACE and b"static scratch" in lib.ps_last_error()
    pd = ps.make_params(0.1, dash=(10.0, 5.0))
    rc = lib.ps_stroke_static(ctypes.byref(_batch()), ctypes.byref(pd), 0x1000, 0x1000, 0x1000, 0x1000,
                              0x1000, 1 << 10, None, None)
    assert rc == ps.PS_E_UNSUPPORTED
