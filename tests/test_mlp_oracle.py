"""Pins of the learned proposal's CPU oracle (oracle/mlp.py): finite
differences, a hand-computed network, one Adam step in closed form, BF16
rounding of known values, and the geometry of the features."""
import math

import numpy as np
import pytest

from oracle import mlp


def _rand_problem(n=7, seed=0):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(seed)
    p[mlp.OFF_B1:mlp.OFF_W2] = rng.normal(0, 0.1, mlp.NH)
    p[mlp.OFF_B2:mlp.OFF_W3] = rng.normal(0, 0.1, mlp.NH)
    p[mlp.OFF_B3] = 0.3
    X = rng.normal(size=(n, mlp.NIN))
    t = rng.normal(size=n)
    return X, t, p


def test_gradient_matches_central_differences():
    X, t, p = _rand_problem()
    g = mlp.grad(X, t, p)
    h = 1e-6
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(mlp.NPARAM, 200, replace=False),
                          [mlp.OFF_B1, mlp.OFF_W2 + 5, mlp.OFF_W3 + 63, mlp.OFF_B3]])
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fd = (mlp.loss(X, t, p + e) - mlp.loss(X, t, p - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * (1 + abs(g[i])), (i, fd, g[i])


def test_hand_computed_network():
    # hidden unit 0 of layer 1 sums the inputs, unit 0 of layer 2 doubles it,
    # the output takes 3x that plus 1: y = 6 relu(sum x) + 1
    W1 = np.zeros((16, 64)); W1[:, 0] = 1.0
    W2 = np.zeros((64, 64)); W2[0, 0] = 2.0
    w3 = np.zeros(64); w3[0] = 3.0
    p = mlp.pack(W1, np.zeros(64), W2, np.zeros(64), w3, 1.0)
    X = np.array([[0.5] * 16, [-1.0] * 16, [0.25] * 8 + [-0.125] * 8])
    y, _ = mlp.forward(X, p)
    assert np.allclose(y, [6 * 8.0 + 1, 1.0, 6 * 1.0 + 1], rtol=0, atol=1e-12)
    t = np.array([40.0, 2.0, 7.0])
    g = mlp.grad(X, t, p)
    # d loss / d b3 = mean 2 (y - t); d loss / d w3[0] = mean 2 (y - t) h2_0
    r = y - t
    assert g[mlp.OFF_B3] == pytest.approx(np.mean(2 * r), abs=1e-12)
    h2 = np.array([16.0, 0.0, 2.0])
    assert g[mlp.OFF_W3] == pytest.approx(np.mean(2 * r * h2), abs=1e-12)
    # d loss / d W1[k][0] = mean 2 r * 3 * 2 * [sum x > 0] * x_k
    active = (X.sum(1) > 0).astype(float)
    for k in (0, 9, 15):
        assert g[mlp.OFF_W1 + k * 64] == pytest.approx(np.mean(2 * r * 6 * active * X[:, k]), abs=1e-12)


def test_adam_first_step_is_a_signed_lr_step():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    assert np.allclose(p1, p - 0.01 * np.sign(g), atol=1e-9)


def test_bf16_rounding_of_known_values():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -3.0, 1 + 2 ** -8 + 2 ** -20, 65504.0])
    want = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -3.0, 1 + 2 ** -7, 65536.0])
    assert np.array_equal(mlp.bf16(vals), want)


def test_emulated_network_stays_within_bf16_of_exact():
    X, t, p = _rand_problem(n=64, seed=3)
    y0, _ = mlp.forward(X, p)
    y1, _ = mlp.forward(X, p, emulate_bf16=True)
    # each product of two rounded operands is within 2^-7 relative; the error
    # of the output is bounded by that times the sum of absolute terms
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p)
    a1 = np.abs(X) @ np.abs(W1) + np.abs(b1)
    a2 = a1 @ np.abs(W2) + np.abs(b2)
    bound = 3 * 2 ** -7 * (a2 @ np.abs(w3)) + 1e-12
    assert np.all(np.abs(y1 - y0) <= bound)


def _equilateral(n, rng):
    base = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.5, math.sqrt(3) / 2, 0.0]])
    out = []
    for _ in range(n):
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        s = rng.uniform(0.1, 3)
        out.append(s * base @ Q.T + rng.normal(size=3))
    return np.array(out)


def test_features_of_an_equilateral_triangle_and_rigid_invariance():
    rng = np.random.default_rng(4)
    v = _equilateral(5, rng)
    ell = np.linalg.norm(v[:, 1] - v[:, 0], axis=1)
    d = rng.uniform(0.01, 0.2, (5, 3)) * ell[:, None]
    nT = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    nT /= np.linalg.norm(nT, axis=1)[:, None]
    q = v - d[:, :, None] * nT[:, None, :]
    nS = np.repeat(nT[:, None, :], 3, 1)
    F = mlp.features(v, d, q, nS, np.ones(5), np.zeros(5), L=0.0, dA=10.0)
    assert np.allclose(F[:, 3], 1) and np.allclose(F[:, 4], 1)
    assert np.allclose(F[:, 5], math.sqrt(3) / 2)
    assert np.allclose(F[:, 11:14], 1)
    assert np.allclose(F[:, 0:3], np.arcsinh(np.sort(d, 1) / ell[:, None]))
    # rigid motion + common scale of the triangle, its closest points and L
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    s, tr = 2.5, rng.normal(size=3)
    F2 = mlp.features(s * v @ Q.T + tr, s * d, s * q @ Q.T + tr, nS @ Q.T, np.ones(5), np.zeros(5),
                      L=0.0, dA=10.0 * s)
    assert np.allclose(F, F2, atol=1e-12)


def test_lattice_points_and_label():
    v = np.array([[[0.0, 0, 0], [4.0, 0, 0], [0.0, 4, 0]]])
    P = mlp.lattice_points(v)
    assert P.shape == (1, 15, 3)
    got = {tuple(np.round(x, 9)) for x in P[0]}
    want = {(float(i), float(j), 0.0) for i in range(5) for j in range(5 - i)}
    assert got == want
    d = np.array([[0.1, 0.2, 0.3]])
    assert mlp.label(np.array([0.5]), d, v) == pytest.approx((0.5 - 0.3) / math.sqrt(32))


# ---------------------------------------------------------------------------
# hand-derived values of the remaining feature columns: the gaps above L of
# the largest vertex distance and of the two cheap bounds (6-8), the closest
# triangle pattern (9-10), the spread of the closest points (14) and the
# level (15)
# ---------------------------------------------------------------------------

def _one(v, d, q, L, dA, distinct=1, shared=0):
    nS = np.repeat(np.array([[[0.0, 0.0, 1.0]]]), 3, 1)
    return mlp.features(np.array([v], float), np.array([d], float), np.array([q], float), nS,
                        np.array([distinct]), np.array([shared]), L, dA)[0]


def test_feature_gaps_of_a_3_4_5_triangle():
    # right triangle: edges e12 = 3, e23 = 5, e31 = 4, longest edge l = 5
    v = [[0, 0, 0], [3, 0, 0], [0, 4, 0]]
    d = [0.1, 0.2, 0.3]
    q = [[0, 0, 0], [0, 0, 0], [0, 0.6, 0.8]]
    F = _one(v, d, q, L=0.05, dA=40.0)
    # max d - L = 0.25
    assert F[6] == pytest.approx(math.asinh(0.25 / 5), abs=1e-15)
    # u1 = min(max(3,4) + 0.1, max(3,5) + 0.2, max(5,4) + 0.3) = 4.1
    assert F[7] == pytest.approx(math.asinh((4.1 - 0.05) / 5), abs=1e-15)
    # not acute (25 = 9 + 16): g = l / 2 = 2.5, u2 = 2.5 + 0.3
    assert F[8] == pytest.approx(math.asinh((2.8 - 0.05) / 5), abs=1e-15)
    # closest points: largest pairwise distance |q3 - q1| = 1
    assert F[14] == pytest.approx(math.asinh(1.0 / 5), abs=1e-15)
    # log2(5 / 40) / 30 = -3 / 30
    assert F[15] == pytest.approx(-0.1, abs=1e-15)
    # one closest triangle: no pattern
    assert F[9] == 0 and F[10] == 0
    # L above every vertex distance gives a negative gap
    F = _one(v, d, q, L=0.5, dA=40.0)
    assert F[6] == pytest.approx(math.asinh(-0.2 / 5), abs=1e-15)


def test_feature_u2_gap_uses_the_circumradius_of_an_acute_triangle():
    # isosceles 6-5-5 (acute: 36 < 50), area 12: R = 6*5*5 / (4*12) = 3.125,
    # larger than l / 2 = 3 (circumcentre (0, 7/8): 4 - 7/8 = 3.125)
    v = [[-3, 0, 0], [3, 0, 0], [0, 4, 0]]
    d = [0.0, 0.5, 0.25]
    F = _one(v, d, v, L=0.125, dA=6.0)
    assert F[8] == pytest.approx(math.asinh((3.125 + 0.5 - 0.125) / 6), abs=1e-15)
    # u1 = min(max(6,5) + 0, max(6,5) + 0.5, max(5,5) + 0.25) = 5.25
    assert F[7] == pytest.approx(math.asinh((5.25 - 0.125) / 6), abs=1e-15)
    # closest points are the vertices: spread = l
    assert F[14] == pytest.approx(math.asinh(1.0), abs=1e-15)
    assert F[15] == pytest.approx(0.0, abs=1e-15)


def test_closest_triangle_pattern():
    FB = np.array([[0, 1, 2], [1, 2, 3], [2, 4, 5], [6, 7, 8], [9, 10, 11]])
    I = np.array([[4, 4, 4],   # one triangle
                  [0, 1, 1],   # two, sharing edge (1, 2)
                  [0, 2, 2],   # two, sharing vertex 2 only
                  [0, 1, 2],   # three (adjacent or not: no flag)
                  [3, 0, 3],   # two with no common index (a duplicate by coordinates would still not count)
                  [1, 0, 0]])  # order does not matter
    distinct, shared = mlp.closest_pattern(I, FB)
    assert distinct.tolist() == [1, 2, 2, 3, 2, 2]
    assert shared.tolist() == [0, 1, 0, 0, 0, 1]
    F = mlp.features(np.zeros((6, 3, 3)) + np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]]), np.full((6, 3), 0.1),
                     np.zeros((6, 3, 3)), np.zeros((6, 3, 3)), distinct, shared, 0.0, 1.0)
    assert F[:, 9].tolist() == [0.0, 0.5, 0.5, 1.0, 0.5, 0.5]
    assert F[:, 10].tolist() == [0, 1, 0, 0, 0, 1]
