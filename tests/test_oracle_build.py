"""The oracle itself as a program: its threaded vertex phase gives the
single-threaded results, and its C code runs clean under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only)."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2406_10357_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_threaded_vertex_phase_gives_identical_results():
    W = wl.config(2, scale=0.05)
    a = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="tree", threads=1)
    b = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="tree", threads=4)
    c = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="brute", threads=3)
    for r in (b, c):
        for k in ("L", "U", "subdivided", "bounded", "queries", "pushes", "stale", "discards", "argmax"):
            assert r[k] == a[k], k
    assert b["evals"] == a["evals"]


_SAN_CHILD = r"""
import sys
sys.path.insert(0, {root!r})
import numpy as np
import oracle
from oracle import hdo
hdo._LIB = {lib!r}
from paper_2406_10357_amd import workloads as wl
rng = np.random.default_rng(0)
# closest points, including degenerate triangles
for _ in range(200):
    p, a, b, c = rng.normal(size=(4, 3))
    oracle.closest_point(p, a, b, a if rng.random() < 0.2 else c)
W = wl.config(1)
t = oracle.Tree(W.VB, W.FB)
for x in rng.normal(size=(50, 3)):
    t.query(x)
del t
r1 = oracle.bound(W.VA, W.FA, W.VB, W.FB, 1e-3)
r2 = oracle.bound(W.VA, W.FA, W.VB, W.FB, 1e-3, backend="tree", threads=3, order=(2, 4, 1, 3))
assert r1["status"] == 0 and r2["status"] == 0 and abs(r1["L"] - r2["L"]) <= r1["eps_abs"]
# error paths: budget, invalid input
assert oracle.bound(W.VA, W.FA, W.VB, W.FB, 1e-9, m=1.5)["status"] == 2
bad = W.FA.copy(); bad[0, 0] = -1
assert oracle.bound(W.VA, bad, W.VB, W.FB, 1e-3)["status"] == 1
print("sanitized oracle ok")
"""


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan is not installed")
    # (leak detection is off: the interpreter itself keeps memory at exit;
    # out-of-bounds accesses, use after free and undefined behaviour abort)
    lib = str(tmp_path / "libhdo_san.so")
    oracle.build(force=True, sanitize=True, out=lib)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    code = _SAN_CHILD.format(root=ROOT, lib=lib)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "sanitized oracle ok" in r.stdout, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
