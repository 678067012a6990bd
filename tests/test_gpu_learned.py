"""The learned proposal inside the engine: the frontier log against the
oracle, certification with the network in the loop, and the gain of a network
trained on the GPU over the plain sub-batched cascade."""
import numpy as np
import pytest

import oracle
from oracle import mlp
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


def test_first_logged_parent_matches_oracle():
    """One triangle over a bumpy soup: round 1 subdivides the triangle
    itself, so the first log row is its features and label, which the oracle
    computes from brute-force distances."""
    hd, torch = _hd()
    rng = np.random.default_rng(3)
    VB, FB = wl.icosphere(2)
    VB = VB * (1 + 0.05 * rng.normal(size=(VB.shape[0], 1)))
    VA = np.array([[0.9, 0.1, 0.2], [0.2, 0.95, 0.1], [0.3, 0.2, 0.9]])
    FA = np.array([[0, 1, 2]], dtype=np.int32)
    log = torch.empty((4096, 17), dtype=torch.float32, device="cuda")
    say("log of one triangle")
    bvh = hd.build_bvh(_cu(VB, torch), _cu(FB, torch))
    L, U, st = hd.bound(_cu(VA, torch), _cu(FA, torch), bvh, 1e-4, subbatch=1, log_out=log, relative=True)
    assert st["logged"] >= 1
    row = log[0].cpu().numpy().astype(np.float64)
    d, I = oracle.points_soup(VA, VB, FB)
    d, I = np.asarray(d), np.asarray(I)
    q = np.array([oracle.closest_point(x, *VB[FB[f]])[1] for x, f in zip(VA, I)])
    e1, e2 = VB[FB[:, 1]] - VB[FB[:, 0]], VB[FB[:, 2]] - VB[FB[:, 0]]
    nB = np.cross(e1, e2)
    nB /= np.linalg.norm(nB, axis=1)[:, None]
    u = sorted(set(I.tolist()))
    shared = float(len(u) == 2 and len(set(FB[u[0]]) & set(FB[u[1]])) >= 2)
    dA = float(np.linalg.norm(VA.max(0) - VA.min(0)))
    F = mlp.features(VA[None], d[None], q[None], nB[I][None], [len(u)], [shared], float(d.max()), dA)[0]
    P = mlp.lattice_points(VA[None])[0]
    dl, _ = oracle.points_soup(P, VB, FB)
    lab = mlp.label(np.array([np.max(dl)]), d[None], VA[None])[0]
    print("gpu", np.round(row, 5))
    print("cpu", np.round(np.append(F, lab), 5))
    # FP32 distances (margin ~1e-6 of the scale) and FP32 features
    assert abs(row[16] - lab) <= 1e-5
    assert np.allclose(row[:16], F, atol=2e-5, rtol=1e-4)


@pytest.mark.parametrize("mode", [1, 2])
def test_learned_modes_stay_certified(mode):
    """Any network (here an untrained one) only reorders the work: the interval
    is still certified and agrees with the oracle."""
    hd, torch = _hd()
    W = wl.config(2, scale=0.05)
    ref = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="tree")
    P = _cu(np.random.default_rng(0).normal(0, 0.2, hd.mlp_nparams()).astype(np.float32), torch)
    say("learned mode", mode, "untrained network, sub-batch 64")
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    L, U, st = hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, subbatch=64, learned=mode,
                        mlp_params=P, relative=True)
    dA = ref["dA"]
    print(f"gpu [{L:.10g}, {U:.10g}] oracle [{ref['L']:.10g}, {ref['U']:.10g}] rounds {st['rounds']} "
          f"skips {st['learned_skips']}")
    assert st["status"] == 0
    assert U - L <= W.eps_rel * dA * (1 + 1e-12)
    assert L <= ref["U"] + 1e-12 * dA and ref["L"] <= U + 1e-12 * dA
    assert abs(L - ref["L"]) <= W.eps_rel * dA


def test_learned_mode_needs_parameters():
    hd, torch = _hd()
    W = wl.config(1)
    bvh = hd.build_bvh(_cu(W.VB, torch), _cu(W.FB, torch))
    with pytest.raises(hd.HDError):
        hd.bound(_cu(W.VA, torch), _cu(W.FA, torch), bvh, W.eps_rel, learned=1, relative=True)


def test_trained_network_gains_over_plain_on_the_large_torus():
    """Train on frontier logs of the plain method on the torus, thin-strip
    and many-pair workloads; then, on the large torus (held out, here at a
    quarter of its size), time the certified bound (median of three calls
    after a warm-up): with the same sub-batch size the learned order must be
    faster than the plain upper-bound order (there the network finds no
    triangle that could still raise L, so every live triangle is split at
    once), and within 1.5x of the plain breadth-first rounds. All three
    intervals are certified and overlap."""
    import os
    import statistics
    hd, torch = _hd()
    from paper_2406_10357_amd import learned
    K = 4096
    W2, W3 = wl.config(2), wl.config(3, scale=0.25)
    pairs = wl.batched_pairs(32, nmax=20000, workers=min(16, os.cpu_count() or 1))
    say("logging the plain method on configs 2, 3 (quarter size) and 32 batched pairs")
    rows = learned.log_frontier([(W2.VA, W2.FA, W2.VB, W2.FB, W2.eps_rel), (W3.VA, W3.FA, W3.VB, W3.FB, W3.eps_rel),
                                 [(P.VA, P.FA, P.VB, P.FB, P.eps_rel) for P in pairs]], subbatch=K, cap=1 << 19)
    say("training on", rows.shape[0], "rows")
    P, losses, (before, after) = learned.train(rows, epochs=6)
    print(f"held-out loss {before:.4g} -> {after:.4g}; label variance {rows[:, 16].var():.4g}")
    assert after < rows[:, 16].var()
    W5 = wl.config(5, scale=0.25)
    VA, FA, VB, FB = (_cu(x, torch) for x in (W5.VA, W5.FA, W5.VB, W5.FB))
    bvh = hd.build_bvh(VB, FB)
    variants = {"plain sub-batched": dict(subbatch=K), "learned": dict(subbatch=K, learned=1, mlp_params=P),
                "plain breadth-first": dict()}
    res = {}
    for name, opts in variants.items():
        say("config 5 (quarter size),", name)
        hd.bound(VA, FA, bvh, W5.eps_rel, relative=True, **opts)
        runs = [hd.bound(VA, FA, bvh, W5.eps_rel, relative=True, **opts) for _ in range(3)]
        L, U, st = runs[-1]
        ms = statistics.median(r[2]["ms_total"] for r in runs)
        res[name] = (L, U, st, ms)
        print(f"  {name}: [{L:.10g}, {U:.10g}] nodes bounded {st['nodes_bounded']} subdivided {st['subdivided']} "
              f"rounds {st['rounds']} ms {ms:.3f}")
        assert st["status"] == 0
        assert U - L <= W5.eps_rel * st["dA"] * (1 + 1e-12)
    for a in res.values():
        for b in res.values():
            assert a[0] <= b[1] and b[0] <= a[1]
    ms_plain, ms_learned, ms_bf = (res[k][3] for k in ("plain sub-batched", "learned", "plain breadth-first"))
    print(f"learned {ms_learned:.3f} ms, plain sub-batched {ms_plain:.3f} ms, breadth-first {ms_bf:.3f} ms")
    assert ms_learned < ms_plain
    assert ms_learned <= 1.5 * ms_bf
