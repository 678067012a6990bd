"""The fifth bound (order digit 5: the bound of Zheng et al. that the paper
quotes in its fourth-bound subsection) on the GPU against the oracle: the
bound in isolation, and the cascade with it (with the other bounds, alone,
and in any order).

Every test prints the case it is about to run before touching the GPU."""
import math

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


def _grid_soup(n, rng, amp=0.2):
    xs = np.linspace(-1, 1, n + 1)
    X, Y = np.meshgrid(xs, xs)
    V = np.stack([X.ravel(), Y.ravel(), amp * rng.normal(size=X.size)], 1)
    idx = np.arange((n + 1) ** 2).reshape(n + 1, n + 1)
    F = np.concatenate([np.stack([idx[:-1, :-1].ravel(), idx[:-1, 1:].ravel(), idx[1:, 1:].ravel()], 1),
                        np.stack([idx[:-1, :-1].ravel(), idx[1:, 1:].ravel(), idx[1:, :-1].ravel()], 1)])
    return V, F.astype(np.int32)


def _u5_definition(v, d, I, S_b, VB, FB):
    """min over S in {S1, S2, S3, S_b} of the largest vertex distance to S,
    from the oracle's closest points (vertex j's distance to its own S_j is d_j)."""
    return min(max(d[j] if S == I[j] else math.sqrt(oracle.closest_point(v[j], *VB[FB[S]])[0]) for j in range(3))
               for S in (*I, S_b))


def test_eval_fifth_bound_matches_oracle():
    """The bound in isolation on 500 triangles around and beyond a noisy grid:
    the barycenter's face is a closest one (ties between faces sharing an
    edge or a vertex are broken by each arithmetic in its own way), and the
    bound equals its definition at that face: the oracle's value where the
    oracle chose the same face, in FP64 to rounding, in FP32 within the
    stated margin."""
    hd, torch = _hd()
    rng = np.random.default_rng(77)
    VB, FB = _grid_soup(10, rng)
    tris, ds, Is = [], [], []
    for k in range(500):
        s = rng.choice([0.03, 0.2, 0.8])
        c0 = rng.uniform(-0.8, 0.8, size=3) * np.array([1, 1, 0.3])
        v = c0 + rng.normal(size=(3, 3)) * s
        res = [oracle.point_soup(x, VB, FB) for x in v]
        tris.append(v)
        ds.append([r[0] for r in res])
        Is.append([r[1] for r in res])
    tris, ds, Is = np.array(tris), np.array(ds), np.array(Is, np.int32)
    ref = [oracle.bound_u5(tris[i], ds[i], Is[i], VB, FB) for i in range(len(tris))]
    say("fifth bound in isolation,", len(tris), "triangles")
    bvh = hd.build_bvh(_cu(VB, torch), _cu(FB, torch))
    u = 2.0 ** -24
    edgeB = max(np.linalg.norm(VB[FB[:, i]] - VB[FB[:, (i + 1) % 3]], axis=1).max() for i in range(3))
    eT = np.max([np.linalg.norm(tris[:, i] - tris[:, (i + 1) % 3], axis=1) for i in range(3)], axis=0)
    ctr = 0.5 * (VB.min(0) + VB.max(0))
    coord = max(np.abs(VB - ctr).max(), np.abs(tris - ctr).max())
    for prec in (hd.PREC_FP64, hd.PREC_FP32):
        out, Sb = hd.eval_bound_u5(_cu(tris, torch), _cu(ds, torch), _cu(Is, torch), bvh, precision=prec)
        out, Sb = out.cpu().numpy(), Sb.cpu().numpy()
        same = 0
        for i in range(len(tris)):
            b = tris[i].mean(0)
            db = math.sqrt(oracle.closest_point(b, *VB[FB[Sb[i]]])[0])
            dmin = oracle.point_soup(b, VB, FB)[0]
            want = ref[i][0] if Sb[i] == ref[i][1] else _u5_definition(tris[i], ds[i], Is[i], Sb[i], VB, FB)
            same += Sb[i] == ref[i][1]
            if prec == hd.PREC_FP64:
                assert abs(db - dmin) <= 1e-12, i
                assert out[i] == pytest.approx(want, rel=1e-9, abs=1e-12), i
            else:
                mu_b = 16 * u * dmin + u * (48 * edgeB + 12 * coord)
                mu = 16 * u * max(ds[i].max(), want) + 48 * u * eT[i] + u * (48 * edgeB + 12 * coord)
                assert abs(db - dmin) <= 2 * mu_b, i
                assert abs(out[i] - want) <= mu, i
        print("precision", prec, "rows where the oracle chose the same face", same, "of", len(tris))


@pytest.mark.parametrize("k,scale,prec", [(1, 1.0, 0), (2, 0.05, 2), (3, 0.02, 1)])
def test_cascade_with_the_fifth_bound(k, scale, prec):
    """Orders with the fifth bound are certified against the oracle run with
    the same order; two orders of the same set give the same run (the
    decision is min over the set below L); the bound discards triangles."""
    hd, torch = _hd()
    W = wl.config(k, scale=scale)
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    args = (_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel)
    runs = {}
    for order in (12345, 54321, 5, 15):
        say(f"config{k}@{scale} precision {prec} order {order}")
        digits = tuple(int(c) for c in str(order))
        ref = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, order=digits, backend="tree")
        L, U, st = hd.bound(*args, precision=prec, order=order, relative=True)
        eps = st["eps_abs"]
        print(f"  gpu [{L:.12g}, {U:.12g}] oracle [{ref['L']:.12g}, {ref['U']:.12g}] "
              f"discards {st['discards']} + u5 {st['discards_u5']} (oracle {ref['discards']})", flush=True)
        assert st["status"] == 0 and U - L <= eps * (1 + 1e-12)
        assert L <= ref["U"] + 1e-12 * st["dA"] and ref["L"] <= U + 1e-12 * st["dA"]
        assert abs(L - ref["L"]) <= eps
        runs[order] = (L, U, st)
    a, b = runs[12345], runs[54321]
    assert a[:2] == b[:2]
    for key in ("subdivided", "nodes_bounded", "rounds"):
        assert a[2][key] == b[2][key], key
    assert runs[5][2]["discards_u5"] > 0
