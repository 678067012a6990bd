"""Options of hd_bound, through the C ABI: absolute and relative tolerance,
the per-round log, the autotuner's cache file, and the test hook that makes
the bounds unsound (which the engine must detect).

Every test prints the case it is about to run before touching the GPU."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2406_10357_amd import workloads as wl

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hd():
    import torch
    import paper_2406_10357_amd as hd
    assert torch.cuda.is_available()
    hd.load_library()
    return hd, torch


def say(*a):
    print("[case]", *a, flush=True)


def _cu(x, torch):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("prec", [0, 2])
def test_absolute_and_relative_tolerance_agree(prec):
    """eps = epsilon * dA given as an absolute tolerance gives the run that
    the relative form gives (the same tolerance reaches the device)."""
    hd, torch = _hd()
    W = wl.config(2, scale=0.05)
    say("absolute vs relative eps, config2 scale 0.05, precision", prec)
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    args = (_cu(W.VA, torch), _cu(W.FA, torch), bvh)
    Lr, Ur, sr = hd.bound(*args, W.eps_rel, precision=prec, relative=True)
    La, Ua, sa = hd.bound(*args, sr["eps_abs"], precision=prec)
    assert sa["eps_abs"] == sr["eps_abs"] and sa["dA"] == sr["dA"]
    assert (La, Ua) == (Lr, Ur)
    for k in ("subdivided", "nodes_bounded", "rounds"):
        assert sa[k] == sr[k]
    assert Ua - La <= sa["eps_abs"]
    # an absolute tolerance is not scaled: ten times dA's share is ten times wider
    L2, U2, s2 = hd.bound(*args, 10 * sr["eps_abs"], precision=prec)
    assert s2["eps_abs"] == 10 * sr["eps_abs"] and U2 - L2 <= s2["eps_abs"]


def test_unsound_bounds_end_the_call_with_internal_error():
    """Test hook: every cascade bound lowered far below the vertex distances
    (no valid upper bound is) must be detected and reported as
    HD_E_INTERNAL, never returned as an interval; the next call is unaffected."""
    hd, torch = _hd()
    W = wl.config(1)
    say("test_bound_shift hook on config1")
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    args = (_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel)
    ref = hd.bound(*args, relative=True)
    for prec in (0, 1, 2):
        for sub in (0, 64):
            with pytest.raises(hd.HDError) as e:
                hd.bound(*args, relative=True, precision=prec, subbatch=sub, test_bound_shift=1.0)
            assert e.value.status == 5, (prec, sub)
    # the workspace is reusable after the error
    again = hd.bound(*args, relative=True)
    assert again[:2] == ref[:2]


@pytest.mark.parametrize("k,scale,prec", [(2, 0.05, 2), (3, 0.02, 1), (1, 1.0, 0)])
def test_round_log(k, scale, prec):
    """One record per round: cumulative counters and a lower bound that never
    decrease, an upper bound at or above the lower bound in every round (a
    child's bound may exceed its parent's: bounds are not inherited), and a
    final record consistent with the returned interval (the final FP64 step
    only lowers U) and the oracle's."""
    hd, torch = _hd()
    W = wl.config(k, scale=scale)
    say(f"round log config{k} scale {scale} precision {prec}")
    ref = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="tree")
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    L, U, st = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, relative=True, precision=prec,
                        round_log=256)
    log = st["round_log"]
    assert len(log) == st["round_records"] == st["rounds"] + 1
    assert [r["round"] for r in log] == list(range(len(log)))
    assert log[0]["split"] == 0 and sum(r["split"] for r in log) == st["subdivided"]
    for a, b in zip(log, log[1:]):
        assert b["bounded"] >= a["bounded"]
        assert all(y >= x for x, y in zip(a["discards"], b["discards"]))
        assert b["L"] >= a["L"]
        assert b["ms"] >= a["ms"]
    last = log[-1]
    assert last["active"] == 0 and last["parked"] == st["parked_final"]
    assert last["bounded"] == st["nodes_bounded"] and last["discards"] == st["discards"]
    assert last["L"] <= L
    assert last["U"] >= U - 1e-15 and last["U"] - last["L"] <= st["eps_abs"] * (1 + 1e-12)
    for r in log:
        assert r["U"] >= r["L"]
    assert L <= ref["U"] + 1e-12 * st["dA"] and ref["L"] <= U + 1e-12 * st["dA"]
    # the unlogged run is certified the same way
    L0, U0, s0 = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, relative=True, precision=prec)
    assert U0 - L0 <= s0["eps_abs"] * (1 + 1e-12) and abs(L0 - L) <= s0["eps_abs"]


_TUNE_CHILD = r"""
import json, sys
sys.path.insert(0, {root!r})
import torch
import paper_2406_10357_amd as hd
from paper_2406_10357_amd import workloads as wl
W = wl.config(2, scale=0.05)
cu = lambda x: torch.from_numpy(x).cuda()
bvh = hd.build_bvh(cu(W.VB), cu(W.FB))
L, U, st = hd.bound(cu(W.VA), cu(W.FA), bvh, W.eps_rel, relative=True, autotune=1, tuner_cache={path!r})
print(json.dumps({{"tuned": st["tuned"], "block": st["query_block"], "stack": st["query_stack"], "L": L, "U": U}}))
"""


def _child(path):
    code = _TUNE_CHILD.format(root=ROOT, path=str(path))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    return json.loads(out.stdout.strip().splitlines()[-1])


def test_tuner_cache_across_processes(tmp_path):
    """A first process tunes and writes its choice under (device,
    arithmetic, kernel-source hash); a second process takes that choice
    from the file without tuning; a corrupt file counts as empty."""
    _hd()
    path = tmp_path / "tuner.json"
    say("tuner cache, first process")
    a = _child(path)
    assert a["tuned"] == 1
    entries = json.loads(path.read_text())
    assert len(entries) == 1
    (key, val), = entries.items()
    assert "/fp32/" in key and val["block"] == a["block"] and val["stack"] == a["stack"]
    say("tuner cache, second process")
    b = _child(path)
    assert b["tuned"] == 2 and (b["block"], b["stack"]) == (a["block"], a["stack"])
    assert (b["L"], b["U"]) == (a["L"], a["U"])
    path.write_text("{ not json")
    say("tuner cache, corrupt file")
    c = _child(path)
    assert c["tuned"] == 1
    assert len(json.loads(path.read_text())) == 1


def test_query_options_out_of_range():
    """query_lanes other than 0, 1, 4 and query_shape outside 0..HD_QUERY_SHAPES
    are rejected as HD_E_INVALID; every shape in range gives a certified
    interval (FP64: the same one)."""
    hd, torch = _hd()
    W = wl.config(1)
    say("query option range on config1")
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    args = (_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel)
    for kw in (dict(query_lanes=2), dict(query_lanes=3), dict(query_shape=-1), dict(query_shape=10)):
        with pytest.raises(hd.HDError) as e:
            hd.bound(*args, relative=True, **kw)
        assert e.value.status == 1, kw
    ref = hd.bound(*args, relative=True, precision=0)
    for shape in range(1, 10):
        L, U, st = hd.bound(*args, relative=True, precision=0, query_shape=shape)
        assert (L, U) == ref[:2], shape
