"""The learned proposal's network on the GPU against the FP64 oracle
(oracle/mlp.py with the same BF16 roundings), through the C ABI.

Tolerances come from the arithmetic: every product of two BF16-rounded
operands is exact in FP32, so the device and the emulating oracle differ only
by FP32 accumulation order and by an activation whose BF16 rounding lands on
the other side of a tie; both are bounded by 2^-7 times the sum of the absolute
values of the terms (computed by the oracle)."""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


def _hd():
    import torch
    import paper_2406_10357_amd as hd
    assert torch.cuda.is_available()
    hd.load_library()
    return hd, torch


def say(*a):
    print("[case]", *a, flush=True)


def _params(seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(seed)
    p[mlp.OFF_B1:mlp.OFF_W2] = rng.normal(0, 0.1, mlp.NH)
    p[mlp.OFF_B2:mlp.OFF_W3] = rng.normal(0, 0.1, mlp.NH)
    p[mlp.OFF_B3] = 0.2
    return p.astype(np.float32).astype(np.float64)  # what the device holds


def _abs_output(X, p):
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p)
    a1 = np.abs(mlp.bf16(X)) @ np.abs(mlp.bf16(W1)) + np.abs(b1)
    a2 = a1 @ np.abs(mlp.bf16(W2)) + np.abs(b2)
    return a2 @ np.abs(mlp.bf16(w3)) + abs(b3)


def test_nparams():
    hd, torch = _hd()
    assert hd.mlp_nparams() == mlp.NPARAM == 5313


@pytest.mark.parametrize("n", [1, 17, 1000, 40000])
def test_forward_matches_oracle(n):
    hd, torch = _hd()
    rng = np.random.default_rng(n)
    X = rng.normal(size=(n, 16)).astype(np.float32).astype(np.float64)
    p = _params(1)
    say("mlp forward", n, "rows")
    y = hd.mlp_forward(torch.from_numpy(X).float().cuda(), torch.from_numpy(p).float().cuda()).cpu().numpy()
    ref, _ = mlp.forward(X, p, emulate_bf16=True)
    tol = 2.0 ** -7 * _abs_output(X, p) + 1e-6
    err = np.abs(y - ref)
    print(f"max err {err.max():.3g}, max err/tol {np.max(err / tol):.3g}, median {np.median(err / tol):.3g}")
    assert np.all(err <= tol)
    assert np.median(err / tol) < 1e-2


@pytest.mark.parametrize("n", [16, 256, 333])
def test_gradient_matches_oracle(n):
    hd, torch = _hd()
    rng = np.random.default_rng(100 + n)
    X = rng.normal(size=(n, 16)).astype(np.float32).astype(np.float64)
    t = rng.normal(size=n).astype(np.float32).astype(np.float64)
    p = _params(2)
    say("mlp gradient", n, "rows")
    g, loss = hd.mlp_grad(torch.from_numpy(X).float().cuda(), torch.from_numpy(t).float().cuda(),
                          torch.from_numpy(p).float().cuda())
    g = g.cpu().numpy().astype(np.float64)
    gref = mlp.grad(X, t, p, emulate_bf16=True)
    gabs = mlp.grad_abs(X, t, p, emulate_bf16=True)
    tol = 2.0 ** -6 * gabs + 1e-7
    err = np.abs(g - gref)
    worst = int(np.argmax(err / tol))
    print(f"max err/tol {np.max(err / tol):.3g} at {worst}; median {np.median(err / tol):.3g}")
    assert np.all(err <= tol)
    assert float(loss.cpu()) == pytest.approx(mlp.loss(X, t, p, emulate_bf16=True), rel=1e-3)
    # and the exact FP64 gradient is close in direction
    gexact = mlp.grad(X, t, p)
    cos = g @ gexact / (np.linalg.norm(g) * np.linalg.norm(gexact))
    assert cos > 0.999


def test_first_adam_step_matches_oracle():
    hd, torch = _hd()
    rng = np.random.default_rng(7)
    n, batch = 512, 256
    X = rng.normal(size=(n, 16)).astype(np.float32).astype(np.float64)
    t = rng.normal(size=n).astype(np.float32).astype(np.float64)
    p = _params(3)
    rows = rng.permutation(n)[:batch].astype(np.int32)
    say("one Adam step")
    P = torch.from_numpy(p).float().cuda()
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    hd.mlp_train(torch.from_numpy(X).float().cuda(), torch.from_numpy(t).float().cuda(),
                 torch.from_numpy(rows).cuda(), batch, P, M, V, step0=0, lr=1e-3)
    g = mlp.grad(X[rows], t[rows], p, emulate_bf16=True)
    gabs = mlp.grad_abs(X[rows], t[rows], p, emulate_bf16=True)
    p1, _, _ = mlp.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr=1e-3)
    got = P.cpu().numpy().astype(np.float64)
    # where the gradient is clearly nonzero, the first step is lr * sign(g)
    clear = np.abs(g) > 2.0 ** -6 * gabs + 1e-6
    assert clear.sum() > 0.8 * mlp.NPARAM
    assert np.allclose(got[clear], p1[clear], atol=1e-6)
    assert np.all(np.abs(got - p) <= 1e-3 * (1 + 1e-3))


def test_training_fits_a_teacher():
    """Adam on the device fits a smooth target; the loss falls by an order of
    magnitude and the trained network generalises to held-out rows."""
    hd, torch = _hd()
    rng = np.random.default_rng(11)
    n = 20000
    X = rng.normal(size=(n, 16)).astype(np.float32)
    w = rng.normal(size=16) / 4
    t = (np.tanh(X @ w) + 0.3 * np.sin(X[:, 0] * X[:, 1])).astype(np.float32)
    p0 = mlp.init_params(5).astype(np.float32)
    P = torch.from_numpy(p0).cuda()
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    Xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    ntrain, batch, steps = 16000, 256, 1500
    rows = np.concatenate([rng.permutation(ntrain) for _ in range(steps * batch // ntrain + 1)])[:steps * batch]
    say("training", steps, "steps")
    loss0 = float(((hd.mlp_forward(Xd[ntrain:], P) - td[ntrain:]) ** 2).mean())
    losses = hd.mlp_train(Xd, td, torch.from_numpy(rows.astype(np.int32)).cuda(), batch, P, M, V, lr=3e-3)
    loss1 = float(((hd.mlp_forward(Xd[ntrain:], P) - td[ntrain:]) ** 2).mean())
    l = losses.cpu().numpy()
    print(f"held-out loss {loss0:.4g} -> {loss1:.4g}; minibatch loss {l[:10].mean():.4g} -> {l[-10:].mean():.4g}")
    assert np.all(np.isfinite(l))
    assert loss1 < 0.1 * loss0
    # the device's trained weights evaluated by the oracle give the same loss
    y_or, _ = mlp.forward(X[ntrain:].astype(np.float64), P.cpu().numpy().astype(np.float64), emulate_bf16=True)
    assert np.mean((y_or - t[ntrain:]) ** 2) == pytest.approx(loss1, rel=1e-2)


# ----------------------------------------------------------------------------
# features of frontier triangles
# ----------------------------------------------------------------------------

def _oracle_feature_inputs(VB, FB, tris):
    import oracle
    n = tris.shape[0]
    P = tris.reshape(-1, 3)
    d, I = oracle.points_soup(P, VB, FB)
    q = np.array([oracle.closest_point(x, *VB[FB[f]])[1] for x, f in zip(P, I)])
    d, I, q = np.asarray(d).reshape(n, 3), np.asarray(I).reshape(n, 3), q.reshape(n, 3, 3)
    e1 = VB[FB[:, 1]] - VB[FB[:, 0]]
    e2 = VB[FB[:, 2]] - VB[FB[:, 0]]
    nB = np.cross(e1, e2)
    nB /= np.linalg.norm(nB, axis=1)[:, None]
    nS = nB[I]
    from oracle import mlp
    distinct, shared = mlp.closest_pattern(I, FB)
    return d, I, q, nS, distinct, shared


def test_features_match_oracle():
    hd, torch = _hd()
    from paper_2406_10357_amd import workloads as wl
    W = wl.config(2, scale=0.05)
    rng = np.random.default_rng(21)
    # small triangles around points of A's surface, several sizes
    base = W.VA[rng.integers(0, W.VA.shape[0], 600)]
    size = np.exp(rng.uniform(np.log(1e-3), np.log(0.1), 600))[:, None, None]
    tris = base[:, None, :] + size * rng.normal(size=(600, 3, 3))
    d, I, q, nS, distinct, shared = _oracle_feature_inputs(W.VB, W.FB, tris)
    L = float(np.median(d)) * 0.8
    dA = 3.0
    say("features of", tris.shape[0], "triangles;", int(shared.sum()), "with a shared edge")
    bvh = hd.build_bvh(torch.from_numpy(W.VB).cuda(), torch.from_numpy(W.FB).cuda())
    X = hd.frontier_features(tris.reshape(-1, 9), d, I, q.reshape(-1, 9), bvh, L, dA).cpu().numpy()
    from oracle import mlp
    F = mlp.features(tris, d, q, nS, distinct, shared, L, dA)
    err = np.abs(X - F)
    # FP32 arithmetic on centred coordinates: differences of vertices of size
    # S carry errors of u*S, so a ratio or a direction over an edge l is off by
    # about u*S/l; 16 of those plus a few ulps of the feature itself
    S = np.abs(tris - 0.5 * (W.VB.min(0) + W.VB.max(0))).max()
    ell = np.max(np.linalg.norm(tris - np.roll(tris, 1, axis=1), axis=2), axis=1)
    u = 2.0 ** -24
    tol = (16 * u * S / ell)[:, None] * (1 + np.abs(F)) + 8 * u * (1 + np.abs(F))
    worst = np.unravel_index(np.argmax(err / tol), err.shape)
    print("max err/tol", float(np.max(err / tol)), "at", worst, X[worst], F[worst])
    assert np.array_equal(X[:, 9], F[:, 9]) and np.array_equal(X[:, 10], F[:, 10])
    assert np.all(err <= tol)
    assert shared.sum() > 0 and distinct.min() >= 1
