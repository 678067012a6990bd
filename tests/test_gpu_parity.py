"""Parity of the HIP library against the FP64 CPU oracle, through the C ABI.

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


def _grid_soup(n, rng, amp=0.2, lo=-1, hi=1):
    xs = np.linspace(lo, hi, n + 1)
    X, Y = np.meshgrid(xs, xs)
    Z = amp * rng.normal(size=X.shape)
    V = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    idx = np.arange((n + 1) ** 2).reshape(n + 1, n + 1)
    F = np.concatenate([np.stack([idx[:-1, :-1].ravel(), idx[:-1, 1:].ravel(), idx[1:, 1:].ravel()], 1),
                        np.stack([idx[:-1, :-1].ravel(), idx[1:, 1:].ravel(), idx[1:, :-1].ravel()], 1)])
    return V, F.astype(np.int32)


def _margin(d, u, edge_max, coord_max):
    return 16 * u * d + u * (48 * edge_max + 12 * coord_max)


# ----------------------------------------------------------------------------
# point -> B queries (LBVH traversal + frame closest point)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["config2-small", "config3-small", "grid"])
def test_point_distances_match_oracle(which):
    hd, torch = _hd()
    rng = np.random.default_rng(5)
    if which == "grid":
        VB, FB = _grid_soup(12, rng)
        P = rng.uniform(-1.3, 1.3, size=(3000, 3))
    else:
        W = wl.config(2 if which == "config2-small" else 3, scale=0.05)
        VB, FB = W.VB, W.FB
        lo, hi = VB.min(0), VB.max(0)
        P = np.concatenate([rng.uniform(lo - 0.1, hi + 0.1, size=(1500, 3)), W.VA[:1500]])
    say("point_distances", which, "nB", FB.shape[0], "nP", P.shape[0])
    bvh = hd.build_bvh(_cu(VB, torch), _cu(FB, torch))
    d64, I64, Q64 = hd.point_distances(_cu(P, torch), bvh, precision=hd.PREC_FP64)
    d32, I32, Q32 = hd.point_distances(_cu(P, torch), bvh, precision=hd.PREC_FP32)
    d64, I64, Q64 = d64.cpu().numpy(), I64.cpu().numpy(), Q64.cpu().numpy()
    d32, I32 = d32.cpu().numpy(), I32.cpu().numpy()
    dref, Iref = oracle.points_soup(P, VB, FB)
    scale = np.abs(VB).max()
    # FP64: same distance; the face is the oracle's or one at the same distance
    assert np.abs(d64 - dref).max() <= 1e-12 * scale
    bad = np.nonzero(I64 != Iref)[0]
    for i in bad:
        a, b, c = VB[FB[I64[i]]]
        dd = math.sqrt(oracle.closest_point(P[i], a, b, c)[0])
        assert abs(dd - dref[i]) <= 1e-12 * scale
    # closest point lies on the reported face at the reported distance
    for i in range(0, P.shape[0], 97):
        a, b, c = VB[FB[I64[i]]]
        dq = math.sqrt(oracle.closest_point(Q64[i], a, b, c)[0])
        assert dq <= 1e-12 * scale
        assert abs(np.linalg.norm(Q64[i] - P[i]) - d64[i]) <= 1e-12 * scale
    # FP32: within the stated margin of the exact distance
    edge = max(np.linalg.norm(VB[FB[:, i]] - VB[FB[:, (i + 1) % 3]], axis=1).max() for i in range(3))
    ctr = 0.5 * (VB[np.unique(FB)].min(0) + VB[np.unique(FB)].max(0))
    coord = max(np.abs(VB - ctr).max(), np.abs(P - ctr).max())
    mu = _margin(dref, 2.0 ** -24, edge, coord)
    err = np.abs(d32 - dref)
    print("fp32 max |d32-d| / mu =", float((err / mu).max()), flush=True)
    assert (err <= mu).all()


# ----------------------------------------------------------------------------
# the bound formulas, in isolation
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_eval_bounds_match_oracle(seed):
    hd, torch = _hd()
    rng = np.random.default_rng(300 + seed)
    VB, FB = _grid_soup(8, rng)
    tris, ds, Is, qs = [], [], [], []
    for k in range(400):
        kind = ["generic", "thin"][k % 2]
        c0 = rng.uniform(-0.8, 0.8, size=3) * np.array([1, 1, 0.3]) + np.array([0, 0, rng.uniform(-0.5, 0.5)])
        s = rng.choice([0.03, 0.2, 0.8])
        a = rng.normal(size=3) * s
        if kind == "generic":
            v = np.array([a, a + rng.normal(size=3) * s, a + rng.normal(size=3) * s])
        else:
            e = rng.normal(size=3)
            v = np.array([a, a + e * s, a + e * s * 0.5 + rng.normal(size=3) * 1e-3 * s])
        v = v - v[0] + c0
        res = [oracle.point_soup(x, VB, FB) for x in v]
        tris.append(v)
        ds.append([r[0] for r in res])
        Is.append([r[1] for r in res])
        qs.append([r[2] for r in res])
    tris, ds, Is, qs = map(np.array, (tris, ds, Is, qs))
    ref = np.array([oracle.bounds(tris[i], ds[i], Is[i].astype(np.int32), qs[i], VB, FB)[0] for i in range(len(tris))])
    refcase = np.array([oracle.bounds(tris[i], ds[i], Is[i].astype(np.int32), qs[i], VB, FB)[1] for i in range(len(tris))])
    say("eval_bounds seed", seed, "n", len(tris))
    bvh = hd.build_bvh(_cu(VB, torch), _cu(FB, torch))
    out, case = hd.eval_bounds(_cu(tris, torch), _cu(ds, torch), _cu(Is.astype(np.int32), torch),
                               _cu(qs, torch), bvh, precision=hd.PREC_FP64)
    out, case = out.cpu().numpy(), case.cpu().numpy()
    assert (case == refcase).all()
    assert (np.isnan(out[:, 0]) == np.isnan(ref[:, 0])).all()
    m = ~np.isnan(ref)
    assert np.allclose(out[m], ref[m], rtol=1e-9, atol=1e-12)
    # FP32 evaluation stays within the triangle margin of FP64
    out32, _ = hd.eval_bounds(_cu(tris, torch), _cu(ds, torch), _cu(Is.astype(np.int32), torch),
                              _cu(qs, torch), bvh, precision=hd.PREC_FP32)
    out32 = out32.cpu().numpy()
    u = 2.0 ** -24
    edgeB = max(np.linalg.norm(VB[FB[:, i]] - VB[FB[:, (i + 1) % 3]], axis=1).max() for i in range(3))
    eT = np.max([np.linalg.norm(tris[:, i] - tris[:, (i + 1) % 3], axis=1) for i in range(3)], axis=0)
    ctr = 0.5 * (VB.min(0) + VB.max(0))
    coord = max(np.abs(VB - ctr).max(), np.abs(tris - ctr).max())
    mu = 16 * u * ds.max(1) + 48 * u * eT + u * (48 * edgeB + 12 * coord)
    err = np.abs(out32[:, 1:] - ref[:, 1:]).max(1)
    print("fp32 bound max err / mu =", float((err / mu).max()), flush=True)
    assert (err <= mu).all()


# ----------------------------------------------------------------------------
# the whole branch and bound
# ----------------------------------------------------------------------------

PRECS = {"fp64": 0, "fp32": 1, "fp32+recheck": 2}  # HD_PREC_* of include/hd.h


def _check_against_oracle(L, U, st, ref, name):
    eps = st["eps_abs"]
    print(f"{name}: gpu [{L:.12g}, {U:.12g}] oracle [{ref['L']:.12g}, {ref['U']:.12g}] eps {eps:.3g} "
          f"rounds {st['rounds']} subdiv {st['subdivided']} (oracle {ref['subdivided']}) "
          f"dL/dA {abs(L - ref['L']) / st['dA']:.3g} dU/dA {abs(U - ref['U']) / st['dA']:.3g}", flush=True)
    assert st["dA"] == pytest.approx(ref["dA"], rel=1e-14)
    assert U - L <= eps * (1 + 1e-12)
    assert L <= ref["U"] + 1e-12 * st["dA"] and ref["L"] <= U + 1e-12 * st["dA"]
    assert abs(L - ref["L"]) <= eps


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32+recheck"])
def test_config1_against_oracle(prec):
    hd, torch = _hd()
    W = wl.config(1)
    ref = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel)
    p = {"fp64": hd.PREC_FP64, "fp32": hd.PREC_FP32, "fp32+recheck": hd.PREC_FP32_RECHECK}[prec]
    say("config1", prec)
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    L, U, st = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, precision=p, relative=True)
    _check_against_oracle(L, U, st, ref, f"config1 {prec}")


@pytest.mark.parametrize("k,scale", [(2, 0.05), (3, 0.02), (5, 0.003)])
@pytest.mark.parametrize("prec", ["fp32", "fp32+recheck", "fp64"])
def test_small_configs_against_oracle(k, scale, prec):
    hd, torch = _hd()
    W = wl.config(k, scale=scale)
    ref = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="tree")
    assert ref["status"] == 0
    p = {"fp64": hd.PREC_FP64, "fp32": hd.PREC_FP32, "fp32+recheck": hd.PREC_FP32_RECHECK}[prec]
    say(f"config{k} scale {scale}", prec, "nA", W.FA.shape[0], "nB", W.FB.shape[0])
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    L, U, st = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, precision=p, relative=True)
    _check_against_oracle(L, U, st, ref, f"config{k}@{scale} {prec}")


def test_closed_forms_on_gpu():
    hd, torch = _hd()
    # offset triangle: h = d exactly
    rng = np.random.default_rng(11)
    v = rng.normal(size=(3, 3))
    n = np.cross(v[1] - v[0], v[2] - v[0])
    n /= np.linalg.norm(n)
    F = np.array([[0, 1, 2]], np.int32)
    say("closed form: offset triangle")
    bvh = hd.build_bvh(_cu(v, torch), _cu(F, torch))
    L, U, st = hd.bound(_cu(v + 0.37 * n, torch), _cu(F, torch), bvh, 1e-6, precision=hd.PREC_FP64, relative=True)
    assert L <= 0.37 + 1e-12 <= U + 2e-12 and U - L <= st["eps_abs"]
    # two-point closed form with an edge maximiser
    delta = 0.3
    VA = np.array([[-1, 0, 0], [1, 0, 0], [0.5, delta, 0]], float)
    VB = np.array([[-1, 0, 1], [1, 0, 1]], float)
    FB = np.array([[0, 0, 0], [1, 1, 1]], np.int32)
    h = math.sqrt(2 + 4 * delta ** 2 / 9)
    for prec in (hd.PREC_FP64, hd.PREC_FP32_RECHECK, hd.PREC_FP32):
        say("closed form: two points, precision", prec)
        bvh = hd.build_bvh(_cu(VB, torch), _cu(FB, torch))
        try:
            L, U, st = hd.bound(_cu(VA, torch), _cu(F, torch), bvh, 1e-6, precision=prec, relative=True)
        except hd.HDError as e:
            # plain FP32 cannot resolve a tolerance below its own margin at
            # the lower bound: it must say so (an input error, found after the
            # vertex round) rather than return a wrong interval
            assert prec == hd.PREC_FP32 and e.status == 1
            continue
        assert L <= h + 1e-12 <= U + 2e-12 and U - L <= st["eps_abs"] * (1 + 1e-12)
        assert L > math.sqrt(1.34) + 1e-3
    # self distance
    V, Fi = wl.icosphere(1)
    say("closed form: h(A,A)")
    bvh = hd.build_bvh(_cu(V, torch), _cu(Fi, torch))
    L, U, st = hd.bound(_cu(V, torch), _cu(Fi, torch), bvh, 1e-2, precision=hd.PREC_FP64, relative=True)
    assert L <= 1e-12 and U <= st["eps_abs"] * (1 + 1e-12)


def test_deterministic():
    hd, torch = _hd()
    W = wl.config(2, scale=0.05)
    say("determinism config2 scale 0.05")
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    r1 = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, relative=True)
    r2 = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, relative=True)
    assert r1[0] == r2[0] and r1[1] == r2[1]
    for k in ("subdivided", "nodes_bounded", "queries", "rounds"):
        assert r1[2][k] == r2[2][k]


@pytest.mark.parametrize("bad", ["eps", "index", "nan", "emptyA"])
def test_invalid_inputs(bad):
    hd, torch = _hd()
    V, F = wl.icosphere(0)
    VA, FA, eps = V.copy(), F.copy(), 1e-3
    if bad == "eps":
        eps = 0.0
    elif bad == "index":
        FA[3, 1] = V.shape[0]
    elif bad == "nan":
        VA[2, 0] = np.nan
    say("invalid input", bad)
    bvh = hd.build_bvh(_cu(V, torch), _cu(F, torch))
    ref = hd.bound(_cu(V, torch), _cu(F, torch), bvh, 1e-3, relative=True)
    if bad == "emptyA":
        FA = FA[:0]
    with pytest.raises(hd.HDError) as e:
        hd.bound(_cu(VA, torch), _cu(FA, torch), bvh, eps, relative=True)
    assert e.value.status == 1
    # an input error found on the device ends the call early: the next call
    # on the same workspace is unaffected
    again = hd.bound(_cu(V, torch), _cu(F, torch), bvh, 1e-3, relative=True)
    assert again[:2] == ref[:2] and again[2]["subdivided"] == ref[2]["subdivided"]
    FB = F.copy()
    FB[0, 0] = -1
    with pytest.raises(hd.HDError):
        hd.build_bvh(_cu(V, torch), _cu(FB, torch))


# ----------------------------------------------------------------------------
# batched pairs, selection by sub-batch, fallbacks and errors
# ----------------------------------------------------------------------------

def _small_pairs(k=5):
    out = []
    for i in range(k):
        rng = np.random.default_rng([9, i])
        V, F = wl.icosphere(1 + i % 2)
        VB = V + rng.normal(0, 0.01, size=V.shape) * (1 + i)
        VA = V * (1.0 + 0.02 * i) + 0.1 * i
        out.append((VA, F, VB + 0.1 * i, F.copy(), [1e-3, 3e-4, 1e-4][i % 3]))
    return out


@pytest.mark.parametrize("prec", ["fp32+recheck", "fp64"])
def test_batched_pairs_against_oracle_and_single(prec):
    hd, torch = _hd()
    pairs = _small_pairs()
    p = {"fp64": hd.PREC_FP64, "fp32+recheck": hd.PREC_FP32_RECHECK}[prec]
    say("batched", len(pairs), "pairs", prec)
    bvh = hd.build_bvh_batched([(_cu(VB, torch), _cu(FB, torch)) for _, _, VB, FB, _ in pairs])
    Ls, Us, st = hd.bound_batched([(_cu(VA, torch), _cu(FA, torch)) for VA, FA, _, _, _ in pairs], bvh,
                                  [e for *_, e in pairs], precision=p, relative=True)
    for i, (VA, FA, VB, FB, eps) in enumerate(pairs):
        ref = oracle.bound(VA, FA, VB, FB, eps)
        dA = ref["dA"]
        print(f"pair {i}: gpu [{Ls[i]:.10g}, {Us[i]:.10g}] oracle [{ref['L']:.10g}, {ref['U']:.10g}]", flush=True)
        assert Us[i] - Ls[i] <= eps * dA * (1 + 1e-12)
        assert Ls[i] <= ref["U"] + 1e-12 * dA and ref["L"] <= Us[i] + 1e-12 * dA
        assert abs(Ls[i] - ref["L"]) <= eps * dA
        say("single pair", i)
        b1 = hd.build_bvh(_cu(VB, torch), _cu(FB, torch))
        L1, U1, _ = hd.bound(_cu(VA, torch), _cu(FA, torch), b1, eps, precision=p, relative=True)
        assert L1 <= Us[i] + 1e-12 * dA and Ls[i] <= U1 + 1e-12 * dA


def _dA(VA, FA):
    V = VA[np.unique(FA)]
    return float(np.linalg.norm(V.max(0) - V.min(0)))


@pytest.mark.parametrize("npairs,nmax", [(24, 3000), (256, 100000)])
def test_batched_generator_pairs(npairs, nmax):
    """The many-pair workload in one call: every pair certified to its own
    tolerance; sampled pairs against the oracle (the small ones, which the
    oracle finishes in seconds)."""
    import os
    hd, torch = _hd()
    pairs = wl.batched_pairs(npairs, nmax=nmax, workers=min(16, os.cpu_count() or 1))
    nA = sum(P.FA.shape[0] for P in pairs)
    say("batched generator", npairs, "pairs, nmax", nmax, "faces", nA)
    bvh = hd.build_bvh_batched([(_cu(P.VB, torch), _cu(P.FB, torch)) for P in pairs])
    Ls, Us, st = hd.bound_batched([(_cu(P.VA, torch), _cu(P.FA, torch)) for P in pairs], bvh,
                                  [P.eps_rel for P in pairs], precision=hd.PREC_FP32_RECHECK, relative=True)
    assert st["status"] == 0
    for i, P in enumerate(pairs):
        dA = _dA(P.VA, P.FA)
        assert 0 <= Ls[i] <= Us[i], i
        assert Us[i] - Ls[i] <= P.eps_rel * dA * (1 + 1e-12), i
    # a stratified sample by size: the three smallest, the three largest and
    # evenly spaced ones between (at least 12 of the 256)
    order = np.argsort([P.FA.shape[0] for P in pairs])
    if npairs >= 24:
        mid = np.linspace(3, len(order) - 4, 8).round().astype(int)[1:-1]
        sample = list(order[:3]) + [int(order[j]) for j in mid] + list(order[-3:])
    else:
        sample = list(order[:3]) + [int(order[len(order) // 2])]
    for i in sample:
        P = pairs[i]
        ref = oracle.bound(P.VA, P.FA, P.VB, P.FB, P.eps_rel, backend="tree")
        dA = ref["dA"]
        print(f"pair {i} ({P.FA.shape[0]} F): gpu [{Ls[i]:.10g}, {Us[i]:.10g}] "
              f"oracle [{ref['L']:.10g}, {ref['U']:.10g}]", flush=True)
        assert Ls[i] <= ref["U"] + 1e-12 * dA and ref["L"] <= Us[i] + 1e-12 * dA
        assert abs(Ls[i] - ref["L"]) <= P.eps_rel * dA
        # on these pairs the oracle's maximum sits at a vertex that both
        # sides query, so L is not below the oracle's by more than rounding
        # once the pair's FP64 argmax step has run (24 pairs: in the scan's
        # last block; 256: in a launch of their own); the FP32 lower bound
        # alone is up to ~1e-8 dA lower. It may be higher: a two-level round
        # queries lattice points that the oracle's queue never reaches (every
        # queried point of A is a lower bound; the overlap above keeps it
        # below the oracle's U)
        assert ref["L"] - Ls[i] <= 1e-9 * dA, (i, Ls[i], ref["L"])


def test_subbatch_selection_is_certified():
    hd, torch = _hd()
    W = wl.config(2, scale=0.05)
    ref = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="tree")
    say("sub-batch 64 on config2 scale 0.05")
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    L, U, st = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, subbatch=64, relative=True)
    _check_against_oracle(L, U, st, ref, "config2 subbatch 64")
    assert st["rounds"] > 5


@pytest.mark.parametrize("k,scale,prec,K", [(2, 0.05, 2, 64), (2, 0.1, 2, 1000), (3, 0.05, 1, 500),
                                           (3, 0.05, 0, 500), (1, 1.0, 0, 16), (5, 0.01, 2, 3000)])
def test_device_subbatch_selection(k, scale, prec, K):
    """Sub-batches selected on the device (radix select on the upper bound):
    certified against the oracle, deterministic, every round splits about K
    (at least K while enough live records remain: the last key bin is taken
    whole), and against the host-driven loop's exact top-K sort (the round
    log selects it) the same interval up to eps."""
    hd, torch = _hd()
    W = wl.config(k, scale=scale)
    ref = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="tree")
    say(f"device sub-batch {K} on config{k} scale {scale} precision {prec}")
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    args = (_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel)
    L, U, st = hd.bound(*args, subbatch=K, precision=prec, relative=True)
    _check_against_oracle(L, U, st, ref, f"config{k}@{scale} device subbatch {K}")
    again = hd.bound(*args, subbatch=K, precision=prec, relative=True)
    assert again[:2] == (L, U)
    for key in ("subdivided", "nodes_bounded", "rounds", "stale"):
        assert again[2][key] == st[key], key
    # about K per round: never fewer rounds than the exact top-K would need
    assert st["rounds"] >= -(-st["subdivided"] // (4 * K)) and st["subdivided"] > 0
    Lh, Uh, sh = hd.bound(*args, subbatch=K, precision=prec, relative=True, round_log=1 << 14)
    _check_against_oracle(Lh, Uh, sh, ref, f"config{k}@{scale} host-sorted subbatch {K}")
    assert all(r["split"] <= K for r in sh["round_log"])


def test_small_capacity_still_certified():
    hd, torch = _hd()
    W = wl.config(2, scale=0.05)
    ref = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="tree")
    say("capacity = nA on config2 scale 0.05")
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    L, U, st = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, capacity=int(W.FA.shape[0] * 2), relative=True)
    _check_against_oracle(L, U, st, ref, "config2 small capacity")


def test_round_limit_with_list_growth():
    """A round limit on the thin-triangle workload at full size, whose first
    rounds outgrow the default frontier lists: the lists grow, the stalled
    round does not count, the partial intervals stay valid bounds, and a
    repeated call (now with grown lists) gives the same result."""
    hd, torch = _hd()
    W = wl.config(3)
    say("config3 full size with max_rounds 1, 2 and unlimited")
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    args = (_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel)
    Lf, Uf, sf = hd.bound(*args, precision=hd.PREC_FP32, relative=True)
    assert sf["status"] == 0 and sf["rounds"] > 2
    prev = 0
    for r in (1, 2):
        L, U, st = hd.bound(*args, precision=hd.PREC_FP32, max_rounds=r, relative=True)
        print(f"max_rounds {r}: rounds {st['rounds']} subdivided {st['subdivided']} [{L:.10g}, {U:.10g}]")
        assert st["status"] == 0 and st["rounds"] == r
        assert st["subdivided"] > prev
        prev = st["subdivided"]
        assert L <= Lf and L <= Uf and Lf <= U
    # the rounds split every active triangle whatever list sizes the earlier
    # calls left: the same result again
    L2, U2, s2 = hd.bound(*args, precision=hd.PREC_FP32, relative=True)
    assert (L2, U2, s2["subdivided"], s2["rounds"]) == (Lf, Uf, sf["subdivided"], sf["rounds"])


@pytest.mark.parametrize("lanes", [1, 4])
def test_tiny_stack_falls_back_and_agrees(lanes):
    """A one-entry stack (ring restarts, then the deep stack of the query
    launch's last block) gives the result of the default stack, with one
    lane or a quad per query."""
    hd, torch = _hd()
    W = wl.config(2, scale=0.05)
    say("tiny traversal stack on config2 scale 0.05, lanes", lanes)
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    a = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, query_lanes=lanes, relative=True)
    b = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, stack_depth=2, query_lanes=lanes, relative=True)
    assert b[2]["query_lanes"] == lanes and b[2]["query_stack"] == 1
    print("overflows", b[2]["stack_overflows"])
    assert b[2]["stack_overflows"] > 0
    assert a[0] == b[0] and a[1] == b[1]
    assert a[2]["subdivided"] == b[2]["subdivided"]


@pytest.mark.parametrize("lanes", [1, 4])
def test_tiny_stack_in_launches_of_many_blocks(lanes):
    """The overflowed traversals are redone by the last block of the query
    launch; launches of more than 256 blocks find that block in two levels
    (sixteen counting lines, then a top line). Full-size C2 with a one-entry
    stack: its first split round launches about 800 blocks with one lane per
    query and about 3,100 with a quad per query, and the interval must still
    be the default stack's."""
    hd, torch = _hd()
    W = wl.config(2)
    say("tiny traversal stack on config2 full size, lanes", lanes)
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    a = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, query_lanes=lanes, relative=True)
    b = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, stack_depth=2, query_lanes=lanes, relative=True)
    print("overflows", b[2]["stack_overflows"], "queries", b[2]["queries"])
    assert b[2]["query_lanes"] == lanes and b[2]["query_stack"] == 1
    assert b[2]["stack_overflows"] > 0
    assert a[0] == b[0] and a[1] == b[1]
    assert a[2]["subdivided"] == b[2]["subdivided"] and a[2]["queries"] == b[2]["queries"]


@pytest.mark.parametrize("which", ["config2-small", "config3-small", "grid"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_quad_query_kernel_agrees(which, prec):
    """Four lanes per point query against one lane per query. In FP64 the
    same closest face, distance and closest point, bit for bit (both find the
    minimum under the same tie rule). In FP32 the computed distances are not
    exactly monotone in the box tests, so near-ties may resolve to another
    face, visited in another order: there both distances lie within the FP32
    margin of the exact one."""
    hd, torch = _hd()
    rng = np.random.default_rng(9)
    if which == "grid":
        VB, FB = _grid_soup(12, rng)
        P = rng.uniform(-1.3, 1.3, size=(3001, 3))
    else:
        W = wl.config(2 if which == "config2-small" else 3, scale=0.05)
        VB, FB = W.VB, W.FB
        lo, hi = VB.min(0), VB.max(0)
        P = np.concatenate([rng.uniform(lo - 0.1, hi + 0.1, size=(1501, 3)), W.VA[:1500]])
    precision = hd.PREC_FP64 if prec == "fp64" else hd.PREC_FP32
    say("quad vs one-lane point queries", which, prec, "nP", P.shape[0])
    bvh = hd.build_bvh(_cu(VB, torch), _cu(FB, torch))
    d1, I1, Q1 = (x.cpu().numpy() for x in hd.point_distances(_cu(P, torch), bvh, precision=precision, lanes=1))
    d4, I4, Q4 = (x.cpu().numpy() for x in hd.point_distances(_cu(P, torch), bvh, precision=precision, lanes=4))
    dref, _ = oracle.points_soup(P, VB, FB)
    if prec == "fp64":
        assert np.array_equal(I1, I4)
        assert np.array_equal(d1, d4) and np.array_equal(Q1, Q4)
        assert np.abs(d4 - dref).max() <= 1e-12 * np.abs(VB).max()
        return
    edge = max(np.linalg.norm(VB[FB[:, i]] - VB[FB[:, (i + 1) % 3]], axis=1).max() for i in range(3))
    ctr = 0.5 * (VB[np.unique(FB)].min(0) + VB[np.unique(FB)].max(0))
    coord = max(np.abs(VB - ctr).max(), np.abs(P - ctr).max())
    mu = _margin(dref, 2.0 ** -24, edge, coord)
    same = I1 == I4
    print(f"faces differ at {int((~same).sum())} of {P.shape[0]} points", flush=True)
    assert np.array_equal(d1[same], d4[same]) and np.array_equal(Q1[same], Q4[same])
    assert (np.abs(d1 - dref) <= mu).all() and (np.abs(d4 - dref) <= mu).all()


@pytest.mark.parametrize("k,scale,prec", [(1, 1.0, "fp64"), (2, 0.05, "fp32+recheck"), (3, 0.02, "fp32")])
def test_quad_query_kernel_in_the_bound(k, scale, prec):
    """hd_bound with the four-lane query kernel, certified against the
    oracle. In FP64 also the same interval and counts as the one-lane kernel
    (identical query results); in FP32 a near-tie may pick another closest
    face, so only the certificates are compared."""
    hd, torch = _hd()
    W = wl.config(k, scale=scale)
    say("bound with quad queries, config", k, "scale", scale, prec)
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    args = (_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel)
    L1, U1, s1 = hd.bound(*args, precision=PRECS[prec], query_lanes=1, relative=True)
    L4, U4, s4 = hd.bound(*args, precision=PRECS[prec], query_lanes=4, relative=True)
    assert s1["query_lanes"] == 1 and s4["query_lanes"] == 4
    if prec == "fp64":
        assert (L1, U1) == (L4, U4)
        for key in ("rounds", "subdivided", "nodes_bounded", "queries", "discards", "rechecked64"):
            assert s1[key] == s4[key], key
    ref = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="tree")
    _check_against_oracle(L1, U1, s1, ref, f"config{k} one-lane queries")
    _check_against_oracle(L4, U4, s4, ref, f"config{k} quad queries")


def test_face_budget_exceeded():
    hd, torch = _hd()
    W = wl.config(1)
    say("budget m = 1.5 on config1")
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    args = (_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel)
    ref = hd.bound(*args, relative=True)
    for sub in (0, 64):
        with pytest.raises(hd.HDError) as e:
            hd.bound(*args, budget_m=1.5, relative=True, subbatch=sub)
        assert e.value.status == 2
        # the failed call gave its buffers back; the next call is unaffected
        again = hd.bound(*args, relative=True)
        assert again[:2] == ref[:2] and again[2]["subdivided"] == ref[2]["subdivided"]


def test_cascade_order_invariance_on_gpu():
    hd, torch = _hd()
    W = wl.config(1)
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    ref = None
    for order in (1234, 4321, 2314, 3142):
        say("order", order)
        L, U, st = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, order=order, relative=True)
        key = (L, U, st["subdivided"], st["nodes_bounded"])
        ref = ref or key
        assert key == ref


def test_autotuned_launch_shape_gives_the_same_result():
    """The autotuner only changes the query kernel's launch shape (block
    size, stack depth): the result and every count stay the same."""
    hd, torch = _hd()
    W = wl.config(2, scale=0.1)
    say("autotune on config2 scale 0.1")
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    args = (_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel)
    L0, U0, s0 = hd.bound(*args, relative=True)
    L1, U1, s1 = hd.bound(*args, autotune=2, relative=True)
    L2, U2, s2 = hd.bound(*args, relative=True)
    print("tuned shape: block", s1["query_block"], "stack", s1["query_stack"], "quad below", s1["query_quad_max"])
    assert (s1["query_block"], s1["query_stack"]) in [(128, 16), (64, 8), (64, 16), (128, 32), (256, 8), (256, 16),
                                                       (128, 12), (256, 12), (128, 24)]
    assert (s2["query_block"], s2["query_stack"]) == (s1["query_block"], s1["query_stack"])
    for k in ("subdivided", "nodes_bounded", "queries", "rounds", "pt_tri_evals"):
        assert s0[k] == s1[k] == s2[k], k
    assert (L0, U0) == (L1, U1) == (L2, U2)


def _random_soup(rng, n, spread=1.0):
    V = rng.normal(size=(3 * n, 3)) * spread
    F = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    return V, F


@pytest.mark.parametrize("seed,nA", [(0, 1), (1, 2), (2, 17), (3, 40), (4, 50)])
@pytest.mark.parametrize("prec", ["fp64", "fp32+recheck"])
def test_random_tiny_soups(seed, nA, prec):
    """Ragged tiny soups: random triangles A, and B small random triangles
    around each vertex of A, so that the maximum lies inside A's triangles
    and the rounds must subdivide (the dense-sampling pin of the oracle covers
    the same kind of input)."""
    hd, torch = _hd()
    rng = np.random.default_rng([77, seed])
    VA, FA = _random_soup(rng, nA)
    VB = np.concatenate([v + rng.normal(0, 0.08, size=(3, 3)) for v in VA])
    FB = np.arange(VB.shape[0], dtype=np.int32).reshape(-1, 3)
    eps = 1e-4
    ref = oracle.bound(VA, FA, VB, FB, eps)
    p = {"fp64": hd.PREC_FP64, "fp32+recheck": hd.PREC_FP32_RECHECK}[prec]
    say("random soups", seed, nA, FB.shape[0], prec)
    bvh = hd.build_bvh(_cu(VB, torch), _cu(FB, torch))
    L, U, st = hd.bound(_cu(VA, torch), _cu(FA, torch), bvh, eps, precision=p, relative=True)
    _check_against_oracle(L, U, st, ref, f"random {seed} {prec}")


@pytest.mark.parametrize("prec", ["fp64", "fp32+recheck"])
def test_degenerate_triangles(prec):
    """Zero-area triangles on both sides (repeated and collinear vertices),
    point and segment triangles in B, unreferenced vertices in both."""
    hd, torch = _hd()
    rng = np.random.default_rng(5)
    V, F = wl.icosphere(1)
    VA = np.concatenate([V, rng.normal(size=(5, 3)) * 3])  # 5 unreferenced vertices
    FA = np.concatenate([F, [[0, 0, 1], [2, 3, 3], [4, 4, 4]]]).astype(np.int32)
    # a collinear triangle: midpoint of an edge
    VA = np.concatenate([VA, [(V[5] + V[6]) / 2]])
    FA = np.concatenate([FA, [[5, 6, VA.shape[0] - 1]]]).astype(np.int32)
    VB = V * 1.05 + rng.normal(0, 0.01, size=V.shape)
    VB = np.concatenate([VB, rng.normal(size=(4, 3)) * 10])  # unreferenced
    FB = np.concatenate([F, [[0, 0, 0], [1, 1, 2], [3, 4, 3]]]).astype(np.int32)
    eps = 1e-3
    ref = oracle.bound(VA, FA, VB, FB, eps)
    p = {"fp64": hd.PREC_FP64, "fp32+recheck": hd.PREC_FP32_RECHECK}[prec]
    say("degenerate triangles", prec)
    bvh = hd.build_bvh(_cu(VB, torch), _cu(FB, torch))
    L, U, st = hd.bound(_cu(VA, torch), _cu(FA, torch), bvh, eps, precision=p, relative=True)
    _check_against_oracle(L, U, st, ref, f"degenerate {prec}")


def test_translation_closed_form():
    """A planar soup against its translate along the normal: h = |t|."""
    hd, torch = _hd()
    rng = np.random.default_rng(6)
    V, F = _grid_soup(10, rng, amp=0.0)
    t = 0.123
    say("translation closed form")
    bvh = hd.build_bvh(_cu(V + np.array([0, 0, t]), torch), _cu(F, torch))
    for prec in (hd.PREC_FP64, hd.PREC_FP32_RECHECK):
        L, U, st = hd.bound(_cu(V, torch), _cu(F, torch), bvh, 1e-6, precision=prec, relative=True)
        assert L <= t + 1e-12 <= U + 2e-12 and U - L <= st["eps_abs"] * (1 + 1e-12)


@pytest.mark.parametrize("n", [1, 2, 3, 255, 256, 257, 511, 513, 65535, 65536, 65537, 65536 + 257])
def test_build_sizes_at_tile_and_group_boundaries(n):
    """BVH builds whose triangle count falls on either side of a refit tile
    (256 leaves) and of a group of tiles (65536 leaves): every node box comes
    from the in-tile climb, the tile / group tables or the whole groups
    between, so FP64 point distances must equal the oracle's brute force.
    Half of the points are centroids of sampled triangles (distance 0 to
    their own triangle: a box that missed part of its subtree would show);
    the four-lane kernel (with the top-level table) must agree too."""
    hd, torch = _hd()
    rng = np.random.default_rng(1000 + n)
    C = rng.uniform(-1, 1, size=(n, 3))
    V = (C[:, None, :] + 0.05 * rng.normal(size=(n, 3, 3))).reshape(-1, 3)
    F = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    pick = rng.choice(n, size=min(n, 400), replace=False)
    P = np.concatenate([V[F[pick]].mean(1), rng.uniform(-1.2, 1.2, size=(300, 3))])
    say("build sizes: n", n, "points", P.shape[0])
    bvh = hd.build_bvh(_cu(V, torch), _cu(F, torch))
    dref, _ = oracle.points_soup(P, V, F)
    for lanes in (1, 4):
        d = hd.point_distances(_cu(P, torch), bvh, precision=hd.PREC_FP64, lanes=lanes)[0].cpu().numpy()
        assert np.abs(d - dref).max() <= 1e-12, (lanes, float(np.abs(d - dref).max()))


def test_build_graph_replays_match_eager():
    """BVH builds replayed from captured HIP graphs give what direct launches
    give: the same closest faces, distances and closest points, bit for bit,
    on every replay, with builds of other sizes (other graphs), direct builds
    and bound calls in between."""
    hd, torch = _hd()
    rng = np.random.default_rng(17)
    soups = [wl.config(2, scale=0.05), wl.config(1), wl.config(3, scale=0.02)]
    pts = []
    for W in soups:
        lo, hi = W.VB.min(0), W.VB.max(0)
        pts.append(_cu(np.concatenate([rng.uniform(lo - 0.05, hi + 0.05, size=(700, 3)), W.VA[:300]]), torch))
    dev = [(_cu(W.VB, torch), _cu(W.FB, torch)) for W in soups]

    def run(k, graphs):
        hd.build_graphs(graphs)
        bvh = hd.build_bvh(*dev[k])
        out = []
        for prec in (hd.PREC_FP64, hd.PREC_FP32):
            d, I, Q = hd.point_distances(pts[k], bvh, precision=prec)
            out += [d.cpu().numpy(), I.cpu().numpy(), Q.cpu().numpy()]
        W = soups[k]
        L, U, st = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, relative=True)
        torch.cuda.synchronize()
        return out, (L, U, st["subdivided"], st["nodes_bounded"])

    try:
        eager = [run(k, False) for k in range(len(soups))]
        for rep in range(4):
            for k in (0, 1, 2, 0):
                say("graph build, soup", k, "replay", rep)
                got = run(k, True)
                for a, b in zip(got[0], eager[k][0]):
                    assert np.array_equal(a, b)
                assert got[1] == eager[k][1]
            k = rep % len(soups)
            say("direct build between replays, soup", k)
            got = run(k, False)
            assert got[1] == eager[k][1]
    finally:
        hd.build_graphs(True)


@pytest.mark.parametrize("k", [3, 5])
def test_full_size_queries_on_sampled_points(k):
    """The point queries at a workload's full size (the BVH the bench builds),
    checked on sampled points against the oracle's brute force: A's vertices
    and points around B's surface. FP64: the exact distance, the closest face
    or one at the same distance; FP32 (one lane and a quad per query): within
    the stated margin."""
    hd, torch = _hd()
    W = wl.config(k)
    rng = np.random.default_rng(100 + k)
    VB, FB = W.VB, W.FB
    lo, hi = VB.min(0), VB.max(0)
    m = 96 if k == 3 else 48  # the oracle's brute force over 800 k faces takes ~0.1 s per point
    P = np.concatenate([W.VA[rng.choice(W.VA.shape[0], m, replace=False)],
                        VB[FB[rng.choice(FB.shape[0], 2 * m // 3), 0]] + rng.normal(0, 0.01, size=(2 * m // 3, 3)),
                        rng.uniform(lo, hi, size=(m // 3, 3))])
    say(f"config{k} full size, nB {FB.shape[0]}, {P.shape[0]} sampled points")
    bvh = hd.build_bvh(_cu(VB, torch), _cu(FB, torch))
    dref, Iref = oracle.points_soup(P, VB, FB)
    dref = np.asarray(dref)
    scale = np.abs(VB).max()
    d64, I64, _ = (x.cpu().numpy() for x in hd.point_distances(_cu(P, torch), bvh, precision=hd.PREC_FP64))
    assert np.abs(d64 - dref).max() <= 1e-12 * scale
    for i in np.nonzero(I64 != np.asarray(Iref))[0]:
        a, b, c = VB[FB[I64[i]]]
        assert abs(math.sqrt(oracle.closest_point(P[i], a, b, c)[0]) - dref[i]) <= 1e-12 * scale
    edge = max(np.linalg.norm(VB[FB[:, i]] - VB[FB[:, (i + 1) % 3]], axis=1).max() for i in range(3))
    ctr = 0.5 * (VB[np.unique(FB)].min(0) + VB[np.unique(FB)].max(0))
    coord = max(np.abs(VB - ctr).max(), np.abs(P - ctr).max())
    mu = _margin(dref, 2.0 ** -24, edge, coord)
    for lanes in (1, 4):
        d32 = hd.point_distances(_cu(P, torch), bvh, precision=hd.PREC_FP32, lanes=lanes)[0].cpu().numpy()
        print(f"lanes {lanes}: max |d32 - d| / margin = {np.max(np.abs(d32 - dref) / mu):.3g}")
        assert (np.abs(d32 - dref) <= mu).all()


def test_config5_full_size_against_oracle():
    """The large torus at full size (1 M vs 800 k faces), FP32 with the FP64
    recheck, in the launch configuration the bench times: certified and
    overlapping the oracle's interval."""
    hd, torch = _hd()
    W = wl.config(5)
    say("config5 full size against the oracle's AABB-tree run")
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    L, U, st = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, relative=True)
    ref = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="tree")
    assert ref["status"] == 0 and st["status"] == 0
    _check_against_oracle(L, U, st, ref, "config5 full size")


def test_config3_full_size_against_oracle():
    """The thin-triangle strip at full size (200 k faces of median aspect
    1000:1 against 180 k), plain FP32 as the workload specifies, in the
    launch configuration the bench times: certified and overlapping the
    oracle's interval (the oracle runs its own AABB tree, ~25 s)."""
    hd, torch = _hd()
    W = wl.config(3)
    say("config3 full size (FP32) against the oracle's AABB-tree run")
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    L, U, st = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, relative=True,
                        precision=hd.PREC_FP32)
    ref = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="tree")
    assert ref["status"] == 0 and st["status"] == 0
    _check_against_oracle(L, U, st, ref, "config3 full size")


@pytest.mark.parametrize("k,scale", [(2, 0.1), (5, 0.01), (1, 1.0)])
def test_deferred_recheck_band(k, scale):
    """Device-planned rounds leave the FP64 recheck band to accumulate and
    decide it once enough records wait or no active record is left; the
    host-driven loop (which the round log selects: every active triangle
    split each round, in the same order) decides it every round. Both are
    certified against the oracle and overlap."""
    hd, torch = _hd()
    W = wl.config(k, scale=scale)
    ref = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="tree")
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    args = (_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel)
    say(f"config{k} scale {scale}: planned rounds vs host loop, FP32 + recheck")
    L0, U0, s0 = hd.bound(*args, precision=hd.PREC_FP32_RECHECK, relative=True)
    L1, U1, s1 = hd.bound(*args, precision=hd.PREC_FP32_RECHECK, round_log=4096, relative=True)
    print("rechecked", s0["rechecked64"], s1["rechecked64"], "rounds", s0["rounds"], s1["rounds"])
    _check_against_oracle(L0, U0, s0, ref, "planned (deferred band)")
    _check_against_oracle(L1, U1, s1, ref, "host loop (band every round)")
    assert L0 <= U1 and L1 <= U0


@pytest.mark.parametrize("k,scale,prec,subbatch", [(1, 1.0, "fp64", 0), (2, 0.1, "fp32+recheck", 0),
                                                   (2, 0.1, "fp32+recheck", 1 << 30), (2, 0.1, "fp32+recheck", 300),
                                                   (3, 0.02, "fp32", 0), (3, 0.05, "fp32", 2000),
                                                   (5, 0.02, "fp32+recheck", 0), (5, 0.02, "fp32+recheck", 4096)])
def test_every_bounded_triangle_is_decided_once(k, scale, prec, subbatch):
    """Conservation over a converged run: every bounded triangle ends either
    discarded (by exactly one deciding bound), dropped by the sub-batch
    selection (its bound fell below L before it was split), parked at the end,
    or split, so nodes_bounded = sum(discards) + stale + parked_final +
    subdivided. A recheck record decided twice, or lost, breaks it; so does a
    record the selection loses or duplicates."""
    hd, torch = _hd()
    W = wl.config(k, scale=scale)
    say("conservation, config", k, "scale", scale, prec, "subbatch", subbatch)
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    L, U, st = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, precision=PRECS[prec],
                        subbatch=subbatch, relative=True)
    assert st["status"] == 0 and U - L <= st["eps_abs"] * (1 + 1e-12)
    decided = sum(st["discards"]) + st["stale"] + st["parked_final"] + st["subdivided"]
    print("bounded", st["nodes_bounded"], "decided", decided, "rechecked", st["rechecked64"], "stale", st["stale"],
          "rounds", st["rounds"])
    assert st["nodes_bounded"] == decided


@pytest.mark.parametrize("k,scale,prec", [(1, 1.0, "fp64"), (2, 0.1, "fp32+recheck"), (2, 1.0, "fp32+recheck"),
                                          (3, 0.02, "fp32"), (5, 0.02, "fp32+recheck"), (5, 0.02, "fp64")])
def test_two_level_rounds_against_one_level_and_oracle(k, scale, prec):
    """Small breadth-first rounds split each parent two levels deep (its 16
    grandchildren, from the 12 non-corner points of its resolution-4 lattice),
    the smallest ones four levels deep (256 descendants from its resolution-16
    lattice); split_levels = 1 keeps every round to one level, 2 to at most two.
    Every form certifies an interval that overlaps the oracle's within eps,
    keeps the conservation identity (a parent split several levels deep counts
    once as subdivided, its descendants as bounded), and the deeper forms need
    no more rounds than one level per round."""
    hd, torch = _hd()
    W = wl.config(k, scale=scale)
    ref = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="brute" if k == 1 else "tree")
    assert ref["status"] == 0
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    res = {}
    for lv in (1, 2, 0):
        say(f"config{k} scale {scale}", prec, "split_levels", lv)
        L, U, st = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, precision=PRECS[prec],
                            relative=True, split_levels=lv)
        _check_against_oracle(L, U, st, ref, f"config{k}@{scale} {prec} split_levels {lv}")
        decided = sum(st["discards"]) + st["stale"] + st["parked_final"] + st["subdivided"]
        assert st["nodes_bounded"] == decided
        res[lv] = st
    print("rounds one-level", res[1]["rounds"], "two-level", res[2]["rounds"], "default", res[0]["rounds"],
          "bounded", res[1]["nodes_bounded"], res[2]["nodes_bounded"], res[0]["nodes_bounded"])
    assert res[0]["rounds"] <= res[1]["rounds"] and res[2]["rounds"] <= res[1]["rounds"]
    if k in (1, 3):
        # these runs end in rounds of at most 64 parents: the four-level form
        # ran (it bounds other triangles than the two-level form)
        assert res[0]["nodes_bounded"] != res[2]["nodes_bounded"]
    # the vertex round and the first (large) rounds are the same in both forms
    assert res[0]["nodes_bounded"] >= W.FA.shape[0]


def test_split_levels_out_of_range():
    hd, torch = _hd()
    W = wl.config(1)
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    say("split_levels -1 is rejected")
    with pytest.raises(hd.HDError):
        hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, relative=True, split_levels=-1)


def test_round_limit_decides_the_waiting_band():
    """Rounds stopped by a round limit with recheck records still waiting:
    those are decided before the final U, which stays a valid upper bound."""
    hd, torch = _hd()
    W = wl.config(2)
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    args = (_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel)
    say("config2 full size, FP32 + recheck, max_rounds 1..3")
    Lf, Uf, sf = hd.bound(*args, relative=True)
    for r in (1, 2, 3):
        L, U, st = hd.bound(*args, max_rounds=r, relative=True)
        print(f"max_rounds {r}: [{L:.12g}, {U:.12g}] rechecked {st['rechecked64']}")
        assert st["status"] == 0 and st["rounds"] == r
        assert L <= Lf and Lf <= U and L <= Uf


@pytest.mark.parametrize("order", [5, 1245])
def test_batched_pairs_with_orders_without_the_third_bound(order):
    """The 256-pair workload with cascades whose FP64 re-bound is loose (no
    u3: the final U then rests on the stored FP32 bounds of millions of
    parked triangles): every pair certified to its tolerance, sampled pairs
    against the oracle with the same order."""
    import os
    hd, torch = _hd()
    pairs = wl.batched_pairs(256, workers=min(16, os.cpu_count() or 1))
    say("256 pairs, order", order)
    bvh = hd.build_bvh_batched([(_cu(P.VB, torch), _cu(P.FB, torch)) for P in pairs])
    Ls, Us, st = hd.bound_batched([(_cu(P.VA, torch), _cu(P.FA, torch)) for P in pairs], bvh,
                                  [P.eps_rel for P in pairs], order=order, relative=True)
    assert st["status"] == 0
    for i, P in enumerate(pairs):
        assert Us[i] - Ls[i] <= P.eps_rel * _dA(P.VA, P.FA) * (1 + 1e-12), i
    digits = tuple(int(c) for c in str(order))
    for i in (0, 1, 2, 100):
        P = pairs[i]
        ref = oracle.bound(P.VA, P.FA, P.VB, P.FB, P.eps_rel, order=digits, backend="tree")
        assert Ls[i] <= ref["U"] + 1e-12 * ref["dA"] and ref["L"] <= Us[i] + 1e-12 * ref["dA"]
        assert abs(Ls[i] - ref["L"]) <= ref["eps_abs"]
