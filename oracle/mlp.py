"""FP64 CPU oracle of the learned proposal's network (test infrastructure only).

The paper has no learned component: the proposal is this project's addition
on top of the certified method. It predicts, for a frontier triangle, how far
above its largest vertex distance the maximum distance to B over the triangle
lies, and only orders work and picks which bounds to evaluate; every discard
and every certificate still comes from the rigorous bounds.

Network: 16 inputs -> 64 ReLU -> 64 ReLU -> 1, squared loss, Adam (Kingma and
Ba, 2015) on FP32 master weights. On the device the two hidden layers run as
BF16 matrix products with FP32 accumulation, the output layer as an FP32 dot
product with BF16 weights. `emulate_bf16=True` rounds the same operands to
BF16 here (round to nearest even), so that the device can be compared with
this oracle element by element; with `emulate_bf16=False` the network is the
exact FP64 function, whose gradient the finite-difference pin checks.

Parameter vector layout (5,313 values): W1 [16][64] (input-major), b1 [64],
W2 [64][64], b2 [64], w3 [64], b3.
"""
from __future__ import annotations

import numpy as np

NIN, NH = 16, 64
OFF_W1 = 0
OFF_B1 = OFF_W1 + NIN * NH
OFF_W2 = OFF_B1 + NH
OFF_B2 = OFF_W2 + NH * NH
OFF_W3 = OFF_B2 + NH
OFF_B3 = OFF_W3 + NH
NPARAM = OFF_B3 + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return (p[OFF_W1:OFF_B1].reshape(NIN, NH), p[OFF_B1:OFF_W2], p[OFF_W2:OFF_B2].reshape(NH, NH),
            p[OFF_B2:OFF_W3], p[OFF_W3:OFF_B3], p[OFF_B3])


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]]).astype(np.float64)


def init_params(seed=0):
    """He-normal hidden layers, small output layer, zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, np.sqrt(2.0 / NIN), (NIN, NH))
    W2 = rng.normal(0, np.sqrt(2.0 / NH), (NH, NH))
    w3 = rng.normal(0, np.sqrt(1.0 / NH), NH)
    return pack(W1, np.zeros(NH), W2, np.zeros(NH), w3, 0.0)


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _r(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


def forward(X, p, emulate_bf16=False):
    """Prediction y [n] and the activations the backward pass needs."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    e = emulate_bf16
    Xb = _r(X, e)
    Z1 = Xb @ _r(W1, e) + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = _r(H1, e) @ _r(W2, e) + b2
    H2 = np.maximum(Z2, 0.0)
    y = H2 @ _r(w3, e) + b3
    return y, (Xb, Z1, H1, Z2, H2)


def loss(X, t, p, emulate_bf16=False):
    y, _ = forward(X, p, emulate_bf16)
    return float(np.mean((y - t) ** 2))


def grad(X, t, p, emulate_bf16=False):
    """Gradient of the mean squared error with respect to the parameters
    (backpropagation; with emulation on, the rounded operands stand in for
    the exact ones, as the device does)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    e = emulate_bf16
    y, (Xb, Z1, H1, Z2, H2) = forward(X, p, e)
    n = X.shape[0]
    dy = 2.0 * (y - t) / n
    dw3 = H2.T @ dy
    db3 = dy.sum()
    dZ2 = np.outer(dy, _r(w3, e)) * (Z2 > 0)
    dZ2r = _r(dZ2, e)
    dW2 = _r(H1, e).T @ dZ2r
    db2 = dZ2.sum(0)
    dZ1 = (dZ2r @ _r(W2, e).T) * (Z1 > 0)
    dZ1r = _r(dZ1, e)
    dW1 = Xb.T @ dZ1r
    db1 = dZ1.sum(0)
    return pack(dW1, db1, dW2, db2, dw3, db3)


def grad_abs(X, t, p, emulate_bf16=False):
    """The same contractions over absolute values: a scale for the rounding
    error of each gradient entry (|sum of terms| <= sum of |terms|)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    e = emulate_bf16
    y, (Xb, Z1, H1, Z2, H2) = forward(X, p, e)
    n = X.shape[0]
    dy = np.abs(2.0 * (y - t) / n)
    dw3 = np.abs(H2).T @ dy
    db3 = dy.sum()
    dZ2 = np.outer(dy, np.abs(_r(w3, e))) * (Z2 > 0)
    dW2 = np.abs(_r(H1, e)).T @ dZ2
    db2 = dZ2.sum(0)
    dZ1 = (dZ2 @ np.abs(_r(W2, e)).T) * (Z1 > 0)
    dW1 = np.abs(Xb).T @ dZ1
    db1 = dZ1.sum(0)
    return pack(dW1, db1, dW2, db2, dw3, db3)


def adam_step(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# features of a frontier triangle (the network's 16 inputs)
# ---------------------------------------------------------------------------

def features(v, d, q, nS, distinct, shared_edge, L, dA):
    """16 features per triangle, in the order the device writes them.

    v [n,3,3] vertices, d [n,3] their distances to B, q [n,3,3] closest points,
    nS [n,3,3] unit normals of the closest B triangles, distinct [n] number of
    distinct closest triangles, shared_edge [n] 1 when exactly two distinct
    closest triangles share an edge, L the running lower bound, dA the
    tolerance scale. Ratios go through asinh so that deep levels (tiny
    triangles, large ratios) stay in range.
    """
    v = np.asarray(v, np.float64)
    d = np.asarray(d, np.float64)
    q = np.asarray(q, np.float64)
    nS = np.asarray(nS, np.float64)
    n = v.shape[0]
    e = np.stack([np.linalg.norm(v[:, 1] - v[:, 0], axis=1), np.linalg.norm(v[:, 2] - v[:, 1], axis=1),
                  np.linalg.norm(v[:, 0] - v[:, 2], axis=1)], 1)
    es = np.sort(e, 1)
    ell = es[:, 2]
    order = np.argsort(d, 1, kind="stable")
    ds = np.take_along_axis(d, order, 1)
    nT = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    area2 = np.linalg.norm(nT, axis=1)
    nTu = nT / np.where(area2 > 0, area2, 1.0)[:, None]
    cos = np.abs(np.einsum("nij,nj->ni", nS, nTu))
    cos = np.take_along_axis(cos, order, 1)
    u1 = np.min(np.stack([np.maximum(e[:, 0], e[:, 2]) + d[:, 0], np.maximum(e[:, 0], e[:, 1]) + d[:, 1],
                          np.maximum(e[:, 1], e[:, 2]) + d[:, 2]], 1), 1)
    acute = es[:, 2] ** 2 < es[:, 0] ** 2 + es[:, 1] ** 2
    R = np.where(area2 > 0, e[:, 0] * e[:, 1] * e[:, 2] / (2 * np.where(area2 > 0, area2, 1.0)), 0.0)
    g = np.where(acute & (area2 > 0), np.maximum(R, 0.5 * ell), 0.5 * ell)
    u2 = g + d.max(1)
    qd = np.max(np.stack([np.linalg.norm(q[:, 0] - q[:, 1], axis=1), np.linalg.norm(q[:, 1] - q[:, 2], axis=1),
                          np.linalg.norm(q[:, 2] - q[:, 0], axis=1)], 1), 1)
    F = np.zeros((n, 16))
    F[:, 0:3] = np.arcsinh(ds / ell[:, None])
    F[:, 3] = es[:, 0] / ell
    F[:, 4] = es[:, 1] / ell
    F[:, 5] = area2 / ell ** 2
    F[:, 6] = np.arcsinh((d.max(1) - L) / ell)
    F[:, 7] = np.arcsinh((u1 - L) / ell)
    F[:, 8] = np.arcsinh((u2 - L) / ell)
    F[:, 9] = (np.asarray(distinct, np.float64) - 1) / 2
    F[:, 10] = np.asarray(shared_edge, np.float64)
    F[:, 11:14] = cos
    F[:, 14] = np.arcsinh(qd / ell)
    F[:, 15] = np.log2(ell / dA) / 30.0
    return F


def closest_pattern(I, FB):
    """Columns 9 and 10 of the features, from the closest B triangles I [n,3]
    of a triangle's vertices and B's face array: the number of distinct
    closest triangles, and 1 when exactly two distinct ones share an edge
    (two common vertex indices: the reading of "share an edge" for soups;
    triangles that only repeat coordinates under other indices do not)."""
    I = np.asarray(I)
    FB = np.asarray(FB)
    distinct = np.zeros(I.shape[0])
    shared = np.zeros(I.shape[0])
    for i, r in enumerate(I):
        u = sorted(set(int(x) for x in r))
        distinct[i] = len(u)
        if len(u) == 2:
            shared[i] = 1.0 if len(set(FB[u[0]].tolist()) & set(FB[u[1]].tolist())) >= 2 else 0.0
    return distinct, shared


def label(hhat, d, v):
    """Training target: (sampled maximum distance - largest vertex distance)
    divided by the longest edge."""
    v = np.asarray(v, np.float64)
    e = np.stack([np.linalg.norm(v[:, 1] - v[:, 0], axis=1), np.linalg.norm(v[:, 2] - v[:, 1], axis=1),
                  np.linalg.norm(v[:, 0] - v[:, 2], axis=1)], 1)
    return (np.asarray(hhat, np.float64) - np.max(d, 1)) / e.max(1)


def lattice_points(v, k=4):
    """Barycentric lattice of resolution k on each triangle: the (k+1)(k+2)/2
    points sum_j (a_j / k) v_j with integer a_j >= 0, sum a_j = k."""
    v = np.asarray(v, np.float64)
    pts = []
    for i in range(k + 1):
        for j in range(k + 1 - i):
            w = np.array([k - i - j, i, j], np.float64) / k
            pts.append(np.einsum("j,njc->nc", w, v))
    return np.stack(pts, 1)
