"""ctypes marshalling for the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HDO_OK, HDO_E_INVALID, HDO_E_CAPACITY, HDO_E_NOMEM, HDO_E_INTERNAL = 0, 1, 2, 3, 5

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hdo.c")
_LIB = os.path.join(_HERE, "libhdo.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True, sanitize: bool = False, out: str | None = None) -> str:
    """Compile hdo.c with gcc into a shared library and return its path."""
    out = out or _LIB
    flags = ["-O2", "-fno-fast-math", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra"]
    if sanitize:
        flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-std=c11", "-fPIC", "-shared", "-pthread",
                 "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", *flags, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


class _Result(C.Structure):
    _fields_ = [
        ("L", C.c_double), ("U", C.c_double), ("dA", C.c_double), ("eps_abs", C.c_double),
        ("subdivided", C.c_int64), ("bounded", C.c_int64), ("queries", C.c_int64),
        ("evals", C.c_int64), ("pushes", C.c_int64), ("stale", C.c_int64),
        ("discards", C.c_int64 * 6), ("max_queue", C.c_int64), ("status", C.c_int32),
        ("empty_queue", C.c_int32), ("argmax", C.c_double * 3),
    ]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = C.CDLL(_LIB)
            dp = C.POINTER(C.c_double)
            ip = C.POINTER(C.c_int32)
            lib.hdo_closest_point.restype = C.c_double
            lib.hdo_closest_point.argtypes = [dp, dp, dp, dp, dp]
            lib.hdo_point_soup.restype = C.c_double
            lib.hdo_point_soup.argtypes = [dp, dp, ip, C.c_int64, ip, dp]
            lib.hdo_points_soup.restype = None
            lib.hdo_points_soup.argtypes = [dp, C.c_int64, dp, ip, C.c_int64, dp, ip]
            lib.hdo_tree_build.restype = C.c_void_p
            lib.hdo_tree_build.argtypes = [dp, C.c_int64, ip, C.c_int64]
            lib.hdo_tree_query.restype = C.c_double
            lib.hdo_tree_query.argtypes = [C.c_void_p, dp, ip, dp, C.POINTER(C.c_int64)]
            lib.hdo_tree_free.restype = None
            lib.hdo_tree_free.argtypes = [C.c_void_p]
            lib.hdo_bound_u5.restype = C.c_double
            lib.hdo_bound_u5.argtypes = [dp, dp, ip, dp, ip, C.c_int64, ip]
            lib.hdo_bounds.restype = None
            lib.hdo_bounds.argtypes = [dp, dp, ip, dp, dp, ip, C.c_int64, dp, ip]
            lib.hdo_set_threads.restype = None
            lib.hdo_set_threads.argtypes = [C.c_int32]
            lib.hdo_bound.restype = C.c_int32
            lib.hdo_bound.argtypes = [dp, C.c_int64, ip, C.c_int64, dp, C.c_int64, ip,
                                      C.c_int64, C.c_double, C.c_double, ip, C.c_int32,
                                      C.c_int32, C.POINTER(_Result)]
            _lib = lib
    return _lib


def _d(x):
    a = np.ascontiguousarray(x, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _i(x):
    a = np.ascontiguousarray(x, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def closest_point(p, a, b, c):
    """Squared distance and closest point of triangle (a,b,c) to p."""
    lib = _load()
    arrs = [_d(x) for x in (p, a, b, c)]
    q, qp = _d(np.zeros(3))
    d2 = lib.hdo_closest_point(arrs[0][1], arrs[1][1], arrs[2][1], arrs[3][1], qp)
    return d2, q


def point_soup(p, VB, FB):
    """Brute-force (d, I, q) of p against the soup."""
    lib = _load()
    p_, pp = _d(p)
    V_, Vp = _d(VB)
    F_, Fp = _i(FB)
    I = C.c_int32(-1)
    q, qp = _d(np.zeros(3))
    d = lib.hdo_point_soup(pp, Vp, Fp, F_.shape[0], C.byref(I), qp)
    return d, I.value, q


def points_soup(P, VB, FB):
    """Brute-force distances (and closest triangles) of many points."""
    lib = _load()
    P_, Pp = _d(np.asarray(P).reshape(-1, 3))
    V_, Vp = _d(VB)
    F_, Fp = _i(FB)
    d, dp = _d(np.zeros(P_.shape[0]))
    I, Ip = _i(np.zeros(P_.shape[0], np.int32))
    lib.hdo_points_soup(Pp, P_.shape[0], Vp, Fp, F_.shape[0], dp, Ip)
    return d, I


class Tree:
    """The oracle's own median-split AABB tree over a soup."""

    def __init__(self, VB, FB):
        self._lib = _load()
        self.V, Vp = _d(VB)
        self.F, Fp = _i(FB)
        self.h = self._lib.hdo_tree_build(Vp, self.V.shape[0], Fp, self.F.shape[0])

    def query(self, p):
        p_, pp = _d(p)
        I = C.c_int32(-1)
        q, qp = _d(np.zeros(3))
        ev = C.c_int64(0)
        d = self._lib.hdo_tree_query(self.h, pp, C.byref(I), qp, C.byref(ev))
        return d, I.value, q, ev.value

    def __del__(self):
        if getattr(self, "h", None):
            self._lib.hdo_tree_free(self.h)
            self.h = None


def bounds(v, d, I, q, VB, FB):
    """All five bounds (uexact or NaN, u1..u4) of one triangle, and u3's case."""
    lib = _load()
    v_, vp = _d(np.asarray(v).reshape(9))
    d_, dp = _d(d)
    I_, Ip = _i(I)
    q_, qp = _d(np.asarray(q).reshape(9))
    V_, Vp = _d(VB)
    F_, Fp = _i(FB)
    out, op = _d(np.zeros(5))
    case = C.c_int32(0)
    lib.hdo_bounds(vp, dp, Ip, qp, Vp, Fp, F_.shape[0], op, C.byref(case))
    return out, case.value


def bound_u5(v, d, I, VB, FB):
    """The bound of Zheng et al. (quoted in the paper's fourth-bound
    subsection) of one triangle, and the closest B triangle of its barycenter."""
    lib = _load()
    v_, vp = _d(np.asarray(v).reshape(9))
    d_, dp = _d(d)
    I_, Ip = _i(I)
    V_, Vp = _d(VB)
    F_, Fp = _i(FB)
    Sb = C.c_int32(-1)
    u = lib.hdo_bound_u5(vp, dp, Ip, Vp, Fp, F_.shape[0], C.byref(Sb))
    return u, Sb.value


def bound(VA, FA, VB, FB, eps_rel, m=1e7, order=(1, 2, 3, 4), backend="brute", threads=1):
    """The branch and bound. Returns a dict with L, U, status and counters.
    threads > 1 splits only the vertex-query phase over that many threads
    (same results)."""
    lib = _load()
    lib.hdo_set_threads(int(threads))
    VA_, VAp = _d(VA)
    FA_, FAp = _i(FA)
    VB_, VBp = _d(VB)
    FB_, FBp = _i(FB)
    o_, op = _i(np.asarray(order, dtype=np.int32))
    r = _Result()
    st = lib.hdo_bound(VAp, VA_.shape[0], FAp, FA_.shape[0], VBp, VB_.shape[0], FBp,
                       FB_.shape[0], float(eps_rel), float(m), op, len(order),
                       1 if backend == "tree" else 0, C.byref(r))
    out = {k: getattr(r, k) for k, _ in _Result._fields_}
    out["discards"] = list(r.discards)
    out["argmax"] = list(r.argmax)
    out["status"] = st
    return out


def _diag(V, F):
    """Diagonal of the bounding box of the vertices the faces reference."""
    P = np.asarray(V, np.float64)[np.unique(np.asarray(F))]
    return float(np.linalg.norm(P.max(0) - P.min(0)))


def hausdorff(VA, FA, VB, FB, eps_abs, backend="brute", **kw):
    """The two-sided distance H(A,B) = max{h(A,B), h(B,A)} (Conclusion and
    future work): the branch and bound run in each direction to the same
    absolute tolerance; H lies in [max of the lower bounds, max of the upper
    bounds], an interval no wider than the tolerance. Returns a dict with L, U,
    status and the two one-sided results (ab, ba)."""
    ab = bound(VA, FA, VB, FB, eps_abs / _diag(VA, FA), backend=backend, **kw)
    ba = bound(VB, FB, VA, FA, eps_abs / _diag(VB, FB), backend=backend, **kw)
    status = ab["status"] or ba["status"]
    return {"L": max(ab["L"], ba["L"]), "U": max(ab["U"], ba["U"]), "status": status, "ab": ab, "ba": ba,
            "eps_abs": eps_abs}
