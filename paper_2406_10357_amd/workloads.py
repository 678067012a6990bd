"""Seeded synthetic triangle-soup workloads.

This module only builds input meshes (vertex and face arrays) and states the
tolerance of each workload. It holds none of the method's arithmetic: no
distances, no bounds, no bounding-box diagonals. Both the HIP library and the
CPU oracle consume the arrays it returns.

Every generator is deterministic for a given seed. The meshes stand in for the
near-zero remeshed pairs, thin "bridge" triangles and many-pair benchmarks that
the paper measures on (Results section); none of those datasets' items are
reproduced here.

Conventions: V is (m, 3) float64, F is (n, 3) int32 with 0-based indices, and
every vertex is referenced by some face unless a generator says otherwise.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload", "icosphere", "perturb_along_normals", "torus_point", "torus_normal",
    "torus_grid", "torus_delaunay", "thin_strip_heightfield", "grid_heightfield",
    "geodesic_sphere", "sphere_hull", "config", "batched_pairs", "CONFIG_NAMES",
]


@dataclass
class Workload:
    name: str
    VA: np.ndarray
    FA: np.ndarray
    VB: np.ndarray
    FB: np.ndarray
    eps_rel: float                 # tolerance relative to the bbox diagonal of A
    precision: str = "fp32+recheck"  # arithmetic the workload names for the GPU path
    meta: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# Sphere meshes
# --------------------------------------------------------------------------

def _icosahedron():
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    V = np.array([
        [-1, phi, 0], [1, phi, 0], [-1, -phi, 0], [1, -phi, 0],
        [0, -1, phi], [0, 1, phi], [0, -1, -phi], [0, 1, -phi],
        [phi, 0, -1], [phi, 0, 1], [-phi, 0, -1], [-phi, 0, 1],
    ], dtype=np.float64)
    F = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int32)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    return V, F


def icosphere(level: int):
    """Unit icosphere: icosahedron refined `level` times by shared-midpoint 1->4
    subdivision, every new vertex projected to the unit sphere.
    Level 2 gives 162 vertices / 320 faces."""
    V, F = _icosahedron()
    V = [tuple(v) for v in V]
    for _ in range(level):
        cache = {}
        newF = []

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                p = (np.asarray(V[i]) + np.asarray(V[j])) * 0.5
                p = p / np.linalg.norm(p)
                cache[key] = len(V)
                V.append(tuple(p))
            return cache[key]

        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            newF += [[a, ab, ca], [ab, b, bc], [ca, bc, c], [ab, bc, ca]]
        F = np.array(newF, dtype=np.int32)
    return np.array(V, dtype=np.float64), np.asarray(F, dtype=np.int32)


def geodesic_sphere(freq: int):
    """Class-I geodesic sphere of frequency `freq`: each icosahedron face is
    split into freq^2 triangles on a barycentric lattice, vertices projected to
    the unit sphere and merged across faces. 20*freq^2 faces."""
    V0, F0 = _icosahedron()
    verts = {}
    Vout = []
    Fout = []

    def key_of(i, j, k, a, b, c):
        # canonical key of a lattice point shared between faces: sorted
        # (vertex id, weight) pairs with non-zero weight
        items = sorted([(a, i), (b, j), (c, k)])
        items = tuple((v, w) for v, w in items if w > 0)
        return items

    for a, b, c in F0:
        idx = {}
        for i in range(freq + 1):
            for j in range(freq + 1 - i):
                k = freq - i - j
                key = key_of(i, j, k, a, b, c)
                if key not in verts:
                    p = (i * V0[a] + j * V0[b] + k * V0[c]) / freq
                    p = p / np.linalg.norm(p)
                    verts[key] = len(Vout)
                    Vout.append(p)
                idx[(i, j)] = verts[key]
        for i in range(freq):
            for j in range(freq - i):
                Fout.append([idx[(i, j)], idx[(i + 1, j)], idx[(i, j + 1)]])
                if i + j < freq - 1:
                    Fout.append([idx[(i + 1, j)], idx[(i + 1, j + 1)], idx[(i, j + 1)]])
    return np.array(Vout, dtype=np.float64), np.array(Fout, dtype=np.int32)


def sphere_hull(npts: int, rng: np.random.Generator):
    """Triangulated sphere from the convex hull of `npts` uniform points on the
    unit sphere (2*npts - 4 faces)."""
    from scipy.spatial import ConvexHull
    P = rng.normal(size=(npts, 3))
    P /= np.linalg.norm(P, axis=1, keepdims=True)
    hull = ConvexHull(P)
    F = hull.simplices.astype(np.int32)
    used = np.unique(F)
    remap = -np.ones(npts, dtype=np.int64)
    remap[used] = np.arange(used.size)
    return P[used].copy(), remap[F].astype(np.int32)


def perturb_along_normals(V: np.ndarray, N: np.ndarray, sigma: float, rng: np.random.Generator):
    """V + xi * N with xi ~ N(0, sigma^2), one draw per vertex in vertex order."""
    xi = rng.normal(0.0, sigma, size=V.shape[0])
    return V + xi[:, None] * N


# --------------------------------------------------------------------------
# Displaced torus
# --------------------------------------------------------------------------

TORUS_R = 1.0
TORUS_r = 0.3


def _rho(u, v, amp=0.02, ku=7, kv=5):
    return TORUS_r + amp * np.sin(ku * u) * np.sin(kv * v)


def torus_point(u, v, amp=0.02, ku=7, kv=5):
    """Displaced torus P(u,v) = ((R + rho cos v) cos u, (R + rho cos v) sin u,
    rho sin v) with rho = r + amp sin(ku u) sin(kv v), R = 1, r = 0.3: the tube
    radius is displaced along the undisplaced surface normal."""
    rho = _rho(u, v, amp, ku, kv)
    w = TORUS_R + rho * np.cos(v)
    return np.stack([w * np.cos(u), w * np.sin(u), rho * np.sin(v)], axis=-1)


def torus_normal(u, v):
    """Unit normal of the undisplaced torus (the tube-radial direction)."""
    return np.stack([np.cos(v) * np.cos(u), np.cos(v) * np.sin(u), np.sin(v)], axis=-1)


def torus_grid(nu: int, nv: int, amp=0.02, ku=7, kv=5):
    """nu x nv periodic (u,v) grid on the displaced torus; each quad split on the
    (i,j)-(i+1,j+1) diagonal: nu*nv vertices, 2*nu*nv faces."""
    iu, iv = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    u = 2 * np.pi * iu / nu
    v = 2 * np.pi * iv / nv
    V = torus_point(u.ravel(), v.ravel(), amp, ku, kv)
    vid = lambda i, j: (i % nu) * nv + (j % nv)
    i = iu.ravel()
    j = iv.ravel()
    a = vid(i, j)
    b = vid(i + 1, j)
    c = vid(i + 1, j + 1)
    d = vid(i, j + 1)
    F = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], 0).astype(np.int32)
    return V, F


def periodic_delaunay(uv: np.ndarray, period: float):
    """Delaunay triangulation of points on the flat torus [0,period)^2.

    Points are replicated into a band around the square; a triangle of the
    tiled triangulation is kept when the vertex with the smallest original
    id among its three lies in the centre tile. Ids are then mapped back mod N.
    """
    from scipy.spatial import Delaunay
    n = uv.shape[0]
    band = 0.15 * period
    pts = [uv]
    ids = [np.arange(n)]
    tile = [np.zeros(n, dtype=bool)]
    for du in (-1, 0, 1):
        for dv in (-1, 0, 1):
            if du == 0 and dv == 0:
                continue
            shifted = uv + np.array([du * period, dv * period])
            keep = ((shifted[:, 0] > -band) & (shifted[:, 0] < period + band) &
                    (shifted[:, 1] > -band) & (shifted[:, 1] < period + band))
            pts.append(shifted[keep])
            ids.append(np.nonzero(keep)[0])
            tile.append(np.ones(int(keep.sum()), dtype=bool))
    P = np.concatenate(pts)
    orig = np.concatenate(ids)
    outside = np.concatenate(tile)
    tri = Delaunay(P).simplices
    o = orig[tri]                               # original ids
    which = np.argmin(o, axis=1)
    lowest_local = tri[np.arange(tri.shape[0]), which]
    keep = ~outside[lowest_local]
    F = o[keep].astype(np.int32)
    return F


def torus_delaunay(npts: int, seed, amp=0.02, ku=7, kv=5):
    """Displaced torus sampled at `npts` uniform (u,v) points and triangulated by
    a periodic Delaunay triangulation in (u,v): 2*npts faces, a closed torus."""
    rng = np.random.default_rng(seed)
    uv = rng.uniform(0.0, 2 * np.pi, size=(npts, 2))
    F = periodic_delaunay(uv, 2 * np.pi)
    V = torus_point(uv[:, 0], uv[:, 1], amp, ku, kv)
    return V, F, uv


# --------------------------------------------------------------------------
# Height fields on the unit square
# --------------------------------------------------------------------------

def _height(x, y):
    return 0.05 * np.sin(4 * np.pi * x) * np.cos(3 * np.pi * y)


def thin_strip_heightfield(ncols=2000, nrows=50, shear=196):
    """Unit square on an (ncols+1) x (nrows+1) vertex grid, displaced by
    z = 0.05 sin(4 pi x) cos(3 pi y), triangulated so that most triangles have
    an aspect ratio of about 1000:1.

    An axis-aligned split of a 2000 x 50 grid only reaches 40:1, so every row
    strip is sheared: bottom vertex i connects to top vertex i + shear. The
    parallelogram part gives 2*(ncols - shear) triangles and each end of the
    strip a fan of `shear` triangles, 2*ncols triangles per strip in all, each
    of area dx*dy/2."""
    nx = ncols + 1
    xs = np.arange(nx) / ncols
    ys = np.arange(nrows + 1) / nrows
    X, Y = np.meshgrid(xs, ys, indexing="xy")          # (nrows+1, nx)
    V = np.stack([X.ravel(), Y.ravel(), _height(X.ravel(), Y.ravel())], 1)
    faces = []
    s = shear
    for j in range(nrows):
        b = j * nx + np.arange(nx)            # bottom row ids
        t = (j + 1) * nx + np.arange(nx)      # top row ids
        i = np.arange(ncols - s)
        faces.append(np.stack([b[i], b[i + 1], t[i + s]], 1))
        faces.append(np.stack([b[i + 1], t[i + s + 1], t[i + s]], 1))
        k = np.arange(s)
        faces.append(np.stack([np.full(s, b[0]), t[k + 1], t[k]], 1))           # left fan
        k = np.arange(ncols - s, ncols)
        faces.append(np.stack([b[k], b[k + 1], np.full(s, t[ncols])], 1))       # right fan
    F = np.concatenate(faces).astype(np.int32)
    return V, F


def grid_heightfield(n=300, noise=1e-3, seed=0):
    """Isotropic (n+1) x (n+1) grid on the unit square with the same height
    field plus N(0, noise^2) z-noise: (n+1)^2 vertices, 2 n^2 faces."""
    rng = np.random.default_rng(seed)
    xs = np.arange(n + 1) / n
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    Z = _height(X, Y) + rng.normal(0.0, noise, size=X.shape)
    V = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    idx = np.arange((n + 1) * (n + 1)).reshape(n + 1, n + 1)
    a = idx[:-1, :-1].ravel()
    b = idx[:-1, 1:].ravel()
    c = idx[1:, 1:].ravel()
    d = idx[1:, :-1].ravel()
    F = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)]).astype(np.int32)
    return V, F


# --------------------------------------------------------------------------
# Named configurations
# --------------------------------------------------------------------------

CONFIG_NAMES = {
    1: "icosphere-L2-vs-normal-noise-1e-2 (320/320 F, eps 1e-4*dA, fp64)",
    2: "displaced-torus-160x160-vs-delaunay-20k (51200/40000 F, eps 1e-5*dA)",
    3: "thin-1000to1-heightfield-vs-300x300-grid (200000/180000 F, eps 1e-5*dA)",
    4: "batched-256-pairs (spheres/tori 1e3..1e5 F, eps 1e-4*dA)",
    5: "displaced-torus-1M-vs-delaunay-800k-sigma-5e-4 (1000000/800000 F, eps 1e-5*dA)",
}


def config(k: int, scale: float = 1.0) -> Workload:
    """Workload k (1, 2, 3 or 5). `scale` < 1 shrinks the meshes of configs 2, 3
    and 5 (same recipe, fewer triangles) for parity tests the oracle finishes
    quickly; scale = 1 gives the full sizes."""
    if k == 1:
        VA, FA = icosphere(2)
        rng = np.random.default_rng(0)
        VB = perturb_along_normals(VA, VA / np.linalg.norm(VA, axis=1, keepdims=True), 0.01, rng)
        return Workload("C1 " + CONFIG_NAMES[1], VA, FA, VB, FA.copy(), 1e-4, "fp64")
    if k == 2:
        n = max(8, int(round(160 * math.sqrt(scale))))
        VA, FA = torus_grid(n, n)
        VB, FB, _ = torus_delaunay(max(64, int(round(20000 * scale))), 0)
        return Workload("C2 " + CONFIG_NAMES[2], VA, FA, VB, FB, 1e-5, "fp32+recheck",
                        {"scale": scale})
    if k == 3:
        if scale >= 1.0:
            VA, FA = thin_strip_heightfield()
            VB, FB = grid_heightfield()
        else:
            ncols = max(40, int(round(2000 * math.sqrt(scale))))
            nrows = max(4, int(round(50 * math.sqrt(scale))))
            shear = max(1, int(round(196 * ncols / 2000)))
            VA, FA = thin_strip_heightfield(ncols, nrows, shear)
            VB, FB = grid_heightfield(max(10, int(round(300 * math.sqrt(scale)))))
        return Workload("C3 " + CONFIG_NAMES[3], VA, FA, VB, FB, 1e-5, "fp32",
                        {"scale": scale})
    if k == 5:
        nu = max(20, int(round(1000 * math.sqrt(scale))))
        nv = max(10, int(round(500 * math.sqrt(scale))))
        VA, FA = torus_grid(nu, nv)
        VB, FB, uv = torus_delaunay(max(64, int(round(400000 * scale))), 0)
        VB = perturb_along_normals(VB, torus_normal(uv[:, 0], uv[:, 1]), 5e-4,
                                   np.random.default_rng(1))
        return Workload("C5 " + CONFIG_NAMES[5], VA, FA, VB, FB, 1e-5, "fp32+recheck",
                        {"scale": scale})
    raise ValueError(f"no single-pair workload {k}")


def _smooth_displacement(P, N, rng, amp=0.01, nwaves=4):
    """Smooth random normal displacement: sum of `nwaves` low-frequency
    sinusoids of the position, scaled to amplitude `amp`."""
    disp = np.zeros(P.shape[0])
    for _ in range(nwaves):
        k = rng.normal(size=3)
        k *= rng.uniform(1.0, 4.0) / np.linalg.norm(k)
        ph = rng.uniform(0, 2 * np.pi)
        disp += np.sin(P @ k + ph)
    return P + (amp / nwaves) * disp[:, None] * N


def batched_pairs(npairs=256, nmin=1000, nmax=100000, seed=0, workers=1):
    """Many independent pairs of uneven size. Pair i draws from
    default_rng([seed, i]): a noisy geodesic sphere or displaced torus A with a
    log-uniform face count in [nmin, nmax], and B a re-triangulated copy of the
    same surface moved along its normal by N(0, sigma^2) with sigma
    log-uniform in [1e-4, 1e-2]. Tolerance 1e-4 relative per pair.
    workers > 1 generates the pairs in that many processes (same result)."""
    if workers > 1 and npairs > 1:
        import concurrent.futures as cf
        import multiprocessing as mp
        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            futs = [ex.submit(_one_pair, i, nmin, nmax, seed) for i in range(npairs)]
            return [f.result() for f in futs]
    return [_one_pair(i, nmin, nmax, seed) for i in range(npairs)]


def _one_pair(i, nmin, nmax, seed):
    rng = np.random.default_rng([seed, i])
    kind = "sphere" if rng.uniform() < 0.5 else "torus"
    nA = float(np.exp(rng.uniform(np.log(nmin), np.log(nmax))))
    sigma = float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-2))))
    wave_seed = int(rng.integers(1 << 31))
    if kind == "sphere":
        freq = max(2, int(round(math.sqrt(nA / 20.0))))
        VA, FA = geodesic_sphere(freq)
        wr = np.random.default_rng(wave_seed)
        VA = _smooth_displacement(VA, VA.copy(), wr)
        VB, FB = sphere_hull(max(8, int(round(nA / 2 + 2))), rng)
        NB = VB.copy()
        VB = _smooth_displacement(VB, NB, np.random.default_rng(wave_seed))
        VB = perturb_along_normals(VB, NB, sigma, rng)
    else:
        nv = max(4, int(round(math.sqrt(nA / 2 * TORUS_r / TORUS_R))))
        nu = max(4, int(round(nA / 2 / nv)))
        amp = 0.01
        VA, FA = torus_grid(nu, nv, amp=amp, ku=3, kv=2)
        VB, FB, uv = torus_delaunay(max(16, int(round(nA / 2))), rng.integers(1 << 31),
                                    amp=amp, ku=3, kv=2)
        VB = perturb_along_normals(VB, torus_normal(uv[:, 0], uv[:, 1]), sigma, rng)
    return Workload(f"pair{i}-{kind}", VA, FA, VB, FB, 1e-4, "fp32+recheck", {"sigma": sigma, "kind": kind})
