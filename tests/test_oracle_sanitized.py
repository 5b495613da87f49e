"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

A child process loads the instrumented build of oracle/polar_oracle.cpp (ASan
runtime preloaded) and runs every oracle entry point on small seeded inputs:
counts and ribs of the 64-cubic path, a reduced 4096-path-style batch, a
near-degenerate batch, every join and cap style, external conics, the uniform
baseline, facet statistics, dashing and coverage.  Any out-of-bounds access,
use after free or undefined behaviour (signed overflow, NaN to integer casts,
misaligned loads, ...) aborts the child.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import math
import numpy as np
import oracle
from paper_2007_00308_amd import workloads as W

batches = [W.config1(), W.config2(n_paths=48, max_segs=48), W.config4(n_paths=48, max_segs=24),
           W.config3(n_segs=300), W.config5(q=math.pi / 64, n_paths=64, total_segs=512)]
for join, cap in [(W.JOIN_ROUND, W.CAP_ROUND), (W.JOIN_BEVEL, W.CAP_SQUARE),
                  (W.JOIN_TRIANGLE, W.CAP_TRIANGLE), (W.JOIN_NONE, W.CAP_BUTT),
                  (W.JOIN_MITER, W.CAP_BUTT), (W.JOIN_MITER_CLIP, W.CAP_ROUND)]:
    batches.append(W.random_mixed(21, n_paths=12, max_segs=10, extent=512.0, join=join, cap=cap))
ext = W.random_mixed(52, n_paths=16, max_segs=10, extent=512.0)
k = np.flatnonzero(ext.kind == W.KIND_K)
ext.conic_w[k] = -np.linspace(0.02, 0.8, k.size).astype(np.float32)
ext.conic_w[k[::5]] = 0.0
batches.append(ext)
for b in batches:
    o = oracle.stroke(b, nthreads=2)
    u = oracle.stroke(b, uniform=True, nthreads=2)
    oracle.facet_stats(b, o["offsets"], o["vx"], o["vy"])
    oracle.facet_stats(b, u["offsets"], u["vx"], u["vy"])
    pr = oracle.path_rib_begin(b, o["offsets"])
    oracle.dash(pr, o["vx"], o["vy"], o["vs"], [7.0, 3.0, 2.0, 3.0], 1.5)
    for mode in (oracle.COVER_QUAD, oracle.COVER_TRIANGLES):
        top = oracle.coverage(b, o["offsets"], o["vx"], o["vy"], 0.0, 0.0, 96, 64, mode)
        oracle.coverage_at(b, o["offsets"], o["vx"], o["vy"], 0.0, 0.0, [0, 5, 95], [0, 7, 63], mode, 2)
for kind, pts, w in [(W.KIND_C, [(0, 0), (20, 0), (-15, 0), (5, 0)], 1.0),
                     (W.KIND_Q, [(0, 0), (20, 0), (10, 0)], 1.0),
                     (W.KIND_K, [(0, 0), (50, 80), (120, 10)], -0.5),
                     (W.KIND_C, [(0, 0), (1, 1), (0, 1), (1, 0)], 1.0)]:
    oracle.segment_intervals(kind, pts, math.pi / 32, w)
loaded = [l.split()[-1] for l in open("/proc/self/maps") if "polar_oracle" in l]
assert loaded and all(p.endswith("libpolar_oracle_san.so") for p in loaded), loaded
print("sanitized oracle ok", flush=True)
"""


def test_oracle_clean_under_asan_and_ubsan():
    try:
        runtime = oracle.asan_runtime()
        oracle.build(force=True, sanitize=True)
    except (OSError, subprocess.CalledProcessError) as e:
        pytest.skip(f"no g++ sanitizer toolchain: {e}")
    if not os.path.exists(runtime):
        pytest.skip("g++ has no ASan runtime")
    env = dict(os.environ, PS_ORACLE_SANITIZE="1", LD_PRELOAD=runtime,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0 and "sanitized oracle ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
