"""ps_stroke_static (the entry point that allocates nothing) against the
workspace entry points ps_count -> ps_scan -> ps_emit, through the C ABI.

The same kernels run on both sides, so counts, offsets, vertices and arc
lengths must agree bit for bit.  Two calls in a row, the second on a smaller
batch, check that the static scratch left by the first call (its status word,
link records, look-back words) does not leak into the second."""
import math

import numpy as np
import pytest

import paper_2007_00308_amd as ps
from paper_2007_00308_amd import workloads as W

pytestmark = pytest.mark.gpu


def _workspace_chain(db, q):
    import torch
    out = ps.stroke(db, q)
    torch.cuda.synchronize()
    return out


def _static_chain(db, q, cap):
    import torch
    params = ps.make_params(q, miter_limit=db.miter_limit)
    link_ribs = torch.full((max(1, db.n_links),), -7, dtype=torch.int32, device="cuda")
    offsets = torch.full((db.n_links + 1,), -7, dtype=torch.int64, device="cuda")
    vx = torch.full((max(2, cap),), 12345.0, device="cuda")
    vy, vs = torch.full_like(vx, 12345.0), torch.full_like(vx, 12345.0)
    flags = torch.full((1,), 0xFFFF, dtype=torch.int32, device="cuda")
    print(f"ps_stroke_static: {db.n_paths} paths, {db.n_segs} segments, capacity {cap}", flush=True)
    ps.ps_stroke_static(db, params, link_ribs, offsets, vx, vy, vs, cap, flags)
    torch.cuda.synchronize()
    return link_ribs[:db.n_links], offsets, vx, vy, vs, int(flags.item())


def _agree(db, q):
    ref = _workspace_chain(db, q)
    R = ref["total_ribs"]
    lr, off, vx, vy, vs, flags = _static_chain(db, q, 2 * R)
    assert flags == 0 and ref["status"].flags == 0
    assert int(off[-1].item()) == R
    assert np.array_equal(lr.cpu().numpy(), ref["link_ribs"].cpu().numpy())
    assert np.array_equal(off.cpu().numpy(), ref["offsets"].cpu().numpy())
    for a, b in ((vx, ref["vx"]), (vy, ref["vy"]), (vs, ref["vs"])):
        assert np.array_equal(a[:2 * R].cpu().numpy(), b.cpu().numpy())
    return R


def test_static_chain_matches_workspace_chain_twice_second_smaller():
    big = ps.DeviceBatch(W.config3(n_segs=2000))
    small = ps.DeviceBatch(W.config1())
    R1 = _agree(big, W.config3(n_segs=2000).q)
    R2 = _agree(small, W.config1().q)
    assert R2 < R1


def test_static_chain_reports_overflow_and_writes_nothing():
    import torch
    b = W.config1()
    db = ps.DeviceBatch(b)
    R = _workspace_chain(db, b.q)["total_ribs"]
    lr, off, vx, vy, vs, flags = _static_chain(db, b.q, 2 * R - 2)
    assert flags & ps.PS_STATUS_OVERFLOW
    assert bool(torch.all(vx == 12345.0)) and bool(torch.all(vs == 12345.0))
    # the next call on the same scratch with enough room reports nothing
    _agree(db, b.q)


def test_static_chain_refuses_a_batch_beyond_its_scratch():
    # the full 4096-path batch needs about 109 MB of workspace (its link
    # records alone are 98 MB), beyond the 64 MiB static scratch; the buffers
    # are sized for the batch all the same, so that nothing could be written
    # out of bounds even if the call were accepted
    import torch
    b = W.config2()
    db = ps.DeviceBatch(b)
    params = ps.make_params(b.q)
    cap = 2
    assert ps.ps_workspace_bytes(db, params, cap) > 64 << 20
    link_ribs = torch.empty(db.n_links, dtype=torch.int32, device="cuda")
    offsets = torch.empty(db.n_links + 1, dtype=torch.int64, device="cuda")
    vx = torch.empty(cap, device="cuda"); vy = torch.empty_like(vx); vs = torch.empty_like(vx)
    with pytest.raises(ps.PsError) as e:
        ps.ps_stroke_static(db, params, link_ribs, offsets, vx, vy, vs, cap)
    assert "static scratch" in str(e.value)
