"""The two-sided distance H(A,B) = max{h(A,B), h(B,A)} (hd_hausdorff: both
directions in one two-pair call sharing one lower bound) against the oracle,
which runs the two one-sided searches and takes the larger interval ends.

Every test prints the case it is about to run before touching the GPU."""
import numpy as np
import pytest

import oracle
from paper_2406_10357_amd import workloads as wl

pytestmark = pytest.mark.gpu


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


def _diag(V, F):
    P = V[np.unique(F)]
    return float(np.linalg.norm(P.max(0) - P.min(0)))


def _check(hd, torch, VA, FA, VB, FB, eps_abs, name, backend="brute", **opts):
    say(name, "nA", FA.shape[0], "nB", FB.shape[0], opts)
    L, U, (ab, ba), st = hd.hausdorff(_cu(VA, torch), _cu(FA, torch), _cu(VB, torch), _cu(FB, torch), eps_abs,
                                      **opts)
    ref = oracle.hausdorff(VA, FA, VB, FB, eps_abs, backend=backend)
    print(f"{name}: gpu H [{L:.12g}, {U:.12g}] oracle [{ref['L']:.12g}, {ref['U']:.12g}] "
          f"dirs gpu {ab} {ba} oracle ({ref['ab']['L']:.6g}, {ref['ab']['U']:.6g}) "
          f"({ref['ba']['L']:.6g}, {ref['ba']['U']:.6g}) nodes {st['nodes_bounded']}", flush=True)
    assert ref["status"] == 0 and st["status"] == 0
    assert U - L <= eps_abs * (1 + 1e-12)
    tol = 1e-12 * max(_diag(VA, FA), _diag(VB, FB))
    assert L <= ref["U"] + tol and ref["L"] <= U + tol
    assert abs(L - ref["L"]) <= eps_abs
    # each direction's interval holds its distance: it overlaps the oracle's
    for mine, theirs in ((ab, ref["ab"]), (ba, ref["ba"])):
        assert mine[0] <= mine[1]
        assert mine[0] <= theirs["U"] + tol and theirs["L"] <= mine[1] + tol
    assert L == max(ab[0], ba[0]) and U == max(ab[1], ba[1])
    return L, U, (ab, ba), st


@pytest.mark.parametrize("prec", [0, 2])
def test_two_sided_config1(prec):
    hd, torch = _hd()
    W = wl.config(1)
    _check(hd, torch, W.VA, W.FA, W.VB, W.FB, 1e-4 * _diag(W.VA, W.FA), f"H config1 precision {prec}",
           precision=prec)


@pytest.mark.parametrize("prec", [1, 2])
def test_two_sided_config2_small(prec):
    hd, torch = _hd()
    W = wl.config(2, scale=0.05)
    _check(hd, torch, W.VA, W.FA, W.VB, W.FB, 1e-4 * _diag(W.VA, W.FA), f"H config2@0.05 precision {prec}",
           backend="tree", precision=prec)


def test_two_sided_asymmetric_hemisphere():
    """A = the upper half of a sphere mesh, B = the whole noisy sphere: h(A,B)
    is small, h(B,A) large (the lower half is far from A), so H = h(B,A) and
    the A-to-B direction stops as soon as its bounds fall below the shared
    lower bound. Fewer triangles are bounded than by two one-sided calls."""
    hd, torch = _hd()
    W = wl.config(1)
    up = W.FA[(W.VA[W.FA][:, :, 2].mean(1) > 0)]
    used = np.unique(up)
    remap = -np.ones(W.VA.shape[0], np.int64)
    remap[used] = np.arange(used.size)
    VA, FA = W.VA[used], remap[up].astype(np.int32)
    eps = 1e-4 * _diag(W.VB, W.FB)
    L, U, (ab, ba), st = _check(hd, torch, VA, FA, W.VB, W.FB, eps, "H hemisphere vs sphere")
    # the B-to-A direction decides H; the A-to-B one stops once all its bounds
    # are below that (its interval then reaches up to H's lower bound)
    assert ba[0] == L and ab[0] < ba[0] and ab[1] <= ba[1]
    bvhB = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    bvhA = hd.build_bvh(_cu(VA, torch), _cu(FA, torch))
    s1 = hd.bound(_cu(VA, torch), _cu(FA, torch), bvhB, eps)[2]
    s2 = hd.bound(_cu(W.VB, torch), _cu(W.FB, torch), bvhA, eps)[2]
    print("nodes: two-sided", st["nodes_bounded"], "one-sided sum", s1["nodes_bounded"] + s2["nodes_bounded"])
    assert st["nodes_bounded"] <= s1["nodes_bounded"] + s2["nodes_bounded"]


def test_two_sided_relative_tolerance_and_batched_pairs():
    """Relative tolerance: eps times the larger diagonal; a few pairs of the
    many-pair generator."""
    import os
    hd, torch = _hd()
    pairs = wl.batched_pairs(6, nmax=4000, workers=min(8, os.cpu_count() or 1))
    for i, P in enumerate(pairs[:4]):
        eps_abs = 1e-4 * max(_diag(P.VA, P.FA), _diag(P.VB, P.FB))
        L, U, _, st = _check(hd, torch, P.VA, P.FA, P.VB, P.FB, eps_abs, f"H pair {i}", backend="tree")
        Lr, Ur, _, sr = hd.hausdorff(_cu(P.VA, torch), _cu(P.FA, torch), _cu(P.VB, torch), _cu(P.FB, torch), 1e-4,
                                     relative=True)
        assert sr["eps_abs"] == pytest.approx(eps_abs, rel=1e-12)
        assert Ur - Lr <= sr["eps_abs"] * (1 + 1e-12) and Lr <= U and L <= Ur
