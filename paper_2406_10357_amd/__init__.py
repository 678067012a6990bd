"""Certified one-sided Pompeiu-Hausdorff bounds between triangle soups on
AMD Instinct MI355X.

Thin ctypes binding over the C ABI in include/hd.h (libhd.so, built by
build.py). Every step of the computation runs in the library's HIP kernels;
this module only marshals torch tensors (device memory) and the current
stream. There is no CPU fallback: without the built library on a GPU, every
call raises.
"""
from __future__ import annotations

import ctypes as C
import os

__all__ = ["HDError", "Bvh", "Options", "build_bvh", "bound", "build_bvh_batched", "bound_batched", "hausdorff",
           "point_distances", "eval_bounds",
           "load_library", "PREC_FP64", "PREC_FP32", "PREC_FP32_RECHECK"]

PREC_FP64, PREC_FP32, PREC_FP32_RECHECK = 0, 1, 2
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhd.so")
_lib = None

STATUS = {0: "HD_OK", 1: "HD_E_INVALID", 2: "HD_E_CAPACITY", 3: "HD_E_NOMEM", 4: "HD_E_DEVICE",
          5: "HD_E_INTERNAL"}


class HDError(RuntimeError):
    """A nonzero hd_status; `stats` holds the call's statistics when it has any
    (device_flag names what the device found wrong)."""

    def __init__(self, status: int, where: str, stats=None):
        self.status = status
        self.stats = stats
        flag = f" (device flag {stats['device_flag']})" if stats and stats.get("device_flag") else ""
        super().__init__(f"{where}: {STATUS.get(status, status)}{flag}")


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("order", C.c_int32), ("budget_m", C.c_double),
                ("capacity", C.c_int64), ("max_rounds", C.c_int32), ("stack_depth", C.c_int32),
                ("subbatch", C.c_int32), ("profile", C.c_int32), ("learned", C.c_int32),
                ("log_frontier", C.c_int32), ("mlp_params", C.c_void_p), ("log_out", C.c_void_p),
                ("log_cap", C.c_int64), ("autotune", C.c_int32), ("query_lanes", C.c_int32),
                ("eps_relative", C.c_int32), ("query_shape", C.c_int32), ("tuner_cache", C.c_char_p),
                ("round_log", C.c_void_p), ("round_log_cap", C.c_int64), ("test_bound_shift", C.c_double),
                ("split_levels", C.c_int32), ("pad_opt", C.c_int32)]


class RoundRecord(C.Structure):
    """One record of the per-round log (hd_round_record)."""
    _fields_ = [("round", C.c_int32), ("pad", C.c_int32), ("split", C.c_int64), ("active", C.c_int64),
                ("parked", C.c_int64), ("bounded", C.c_int64), ("discards", C.c_int64 * 5), ("L", C.c_double),
                ("U", C.c_double), ("ms", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}
        d["discards"] = list(self.discards)
        return d


class Stats(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("status", C.c_int32), ("nodes_bounded", C.c_int64),
                ("subdivided", C.c_int64), ("queries", C.c_int64), ("pt_tri_evals", C.c_int64),
                ("box_tests", C.c_int64), ("discards", C.c_int64 * 5), ("rechecked64", C.c_int64),
                ("parked_final", C.c_int64), ("max_frontier", C.c_int64),
                ("stack_overflows", C.c_int64), ("dA", C.c_double), ("eps_abs", C.c_double),
                ("L_rounds", C.c_double), ("U_rounds", C.c_double), ("mu_coef_d", C.c_double),
                ("mu_coef_0", C.c_double), ("ms_total", C.c_double),
                ("ms_query_kernels", C.c_double), ("ms_cascade_kernels", C.c_double),
                ("query_launches", C.c_int64), ("cascade_launches", C.c_int64),
                ("query_leaf_evals", C.c_int64), ("query_box_tests", C.c_int64),
                ("logged", C.c_int64), ("learned_skips", C.c_int64), ("query_block", C.c_int32),
                ("query_stack", C.c_int32), ("query_lanes", C.c_int32), ("query_quad_max", C.c_int32),
                ("round_records", C.c_int64), ("tuned", C.c_int32), ("pad1", C.c_int32), ("stale", C.c_int64),
                ("discards_u5", C.c_int64), ("device_flag", C.c_int32), ("pad2", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("pad1", "pad2")}
        d["discards"] = list(self.discards)
        return d


EXPORTS = ["hd_build_bvh", "hd_build_bvh_batched", "hd_free_bvh", "hd_bound", "hd_bound_batched",
           "hd_point_distances", "hd_eval_bounds", "hd_status_str", "hd_default_options",
           "hd_mlp_nparams", "hd_mlp_forward", "hd_mlp_grad", "hd_mlp_train", "hd_frontier_features",
           "hd_build_graphs", "hd_point_distances_noalloc", "hd_hausdorff",
           "hd_eval_bound_u5"]
NOALLOC_MAX_POINTS = 65536  # HD_NOALLOC_MAX_POINTS


def load_library(path: str | None = None):
    """Load libhd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or _LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2406_10357_amd/build.py "
                           "(or __graft_entry__.build())")
    lib = C.CDLL(path)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    lib.hd_build_bvh.restype = i32
    lib.hd_build_bvh.argtypes = [vp, i64, vp, i64, vp, C.POINTER(vp)]
    lib.hd_free_bvh.restype = None
    lib.hd_free_bvh.argtypes = [vp]
    lib.hd_build_graphs.restype = i32
    lib.hd_build_graphs.argtypes = [i32]
    lib.hd_bound.restype = i32
    lib.hd_bound.argtypes = [vp, i64, vp, i64, vp, dbl, C.POINTER(Options), vp, C.POINTER(C.c_double),
                             C.POINTER(Stats)]
    pp = C.POINTER(C.c_void_p)
    lib.hd_build_bvh_batched.restype = i32
    lib.hd_build_bvh_batched.argtypes = [i32, pp, C.POINTER(i64), pp, C.POINTER(i64), vp, C.POINTER(vp)]
    lib.hd_bound_batched.restype = i32
    lib.hd_bound_batched.argtypes = [i32, pp, C.POINTER(i64), pp, C.POINTER(i64), vp, C.POINTER(C.c_double),
                                     i32, C.POINTER(Options), vp, C.POINTER(C.c_double), C.POINTER(Stats)]
    lib.hd_point_distances.restype = i32
    lib.hd_point_distances.argtypes = [vp, i64, vp, i32, i32, vp, vp, vp, vp]
    lib.hd_eval_bound_u5.restype = i32
    lib.hd_eval_bound_u5.argtypes = [vp, vp, vp, i64, vp, i32, vp, vp, vp]
    lib.hd_hausdorff.restype = i32
    lib.hd_hausdorff.argtypes = [vp, i64, vp, i64, vp, i64, vp, i64, dbl, C.POINTER(Options), vp,
                                 C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(Stats)]
    lib.hd_point_distances_noalloc.restype = i32
    lib.hd_point_distances_noalloc.argtypes = [vp, i64, vp, i32, i32, vp, vp, vp, vp, vp]
    lib.hd_eval_bounds.restype = i32
    lib.hd_eval_bounds.argtypes = [vp, vp, vp, vp, i64, vp, i32, vp, vp, vp]
    lib.hd_status_str.restype = C.c_char_p
    lib.hd_status_str.argtypes = [i32]
    lib.hd_default_options.restype = None
    lib.hd_default_options.argtypes = [C.POINTER(Options)]
    lib.hd_frontier_features.restype = i32
    lib.hd_frontier_features.argtypes = [vp, vp, vp, vp, i64, vp, dbl, dbl, vp, vp]
    lib.hd_mlp_nparams.restype = i32
    lib.hd_mlp_nparams.argtypes = []
    lib.hd_mlp_forward.restype = i32
    lib.hd_mlp_forward.argtypes = [vp, i64, vp, vp, vp]
    lib.hd_mlp_grad.restype = i32
    lib.hd_mlp_grad.argtypes = [vp, vp, i64, vp, vp, vp, vp]
    lib.hd_mlp_train.restype = i32
    lib.hd_mlp_train.argtypes = [vp, vp, vp, i64, i32, vp, vp, vp, i64, C.c_float, vp, vp]
    _lib = lib
    return lib


def _torch():
    import torch
    return torch


def _dev(x, dtype):
    """A contiguous CUDA tensor of the given dtype (copied if needed)."""
    torch = _torch()
    if not isinstance(x, torch.Tensor):
        x = torch.as_tensor(x)
    if not x.is_cuda:
        x = x.to("cuda")
    return x.to(dtype).contiguous()


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(st, where, stats=None):
    if st != 0:
        raise HDError(st, where, stats.as_dict() if stats is not None else None)


class Bvh:
    """LBVH over soup B (device memory owned by the library)."""

    def __init__(self, handle, VB, FB):
        self.handle = handle
        self.VB, self.FB = VB, FB  # kept alive with the handle
        self.nB = FB.shape[0] if hasattr(FB, "shape") else sum(f.shape[0] for f in FB)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.hd_free_bvh(self.handle)
            self.handle = None


def build_bvh(VB, FB) -> Bvh:
    torch = _torch()
    lib = load_library()
    VB = _dev(VB, torch.float64)
    FB = _dev(FB, torch.int32)
    h = C.c_void_p()
    st = lib.hd_build_bvh(C.c_void_p(VB.data_ptr()), VB.shape[0], C.c_void_p(FB.data_ptr()), FB.shape[0],
                          _stream(), C.byref(h))
    _check(st, "hd_build_bvh")
    return Bvh(h, VB, FB)


def make_options(precision=PREC_FP32_RECHECK, order=1234, budget_m=1e7, capacity=0, max_rounds=0,
                 stack_depth=0, subbatch=0, profile=0, learned=0, mlp_params=None, log_out=None,
                 autotune=0, query_lanes=0, relative=False, tuner_cache=None, round_log=None,
                 test_bound_shift=0.0, query_shape=0, split_levels=0) -> Options:
    """mlp_params: device FP32 tensor of mlp_nparams() values (learned > 0);
    log_out: device FP32 tensor (rows, 17) that receives the frontier log;
    relative: eps is the paper's relative tolerance (times dA) instead of an
    absolute one; tuner_cache: path of the autotuner's JSON cache file;
    round_log: a ctypes array of RoundRecord that receives one record per round;
    split_levels: 1 keeps every round to one level of subdivision (0: small
    breadth-first rounds split two levels deep, the smallest four; 2: at most
    two; k >= 3: rounds of at most k triangles split two levels)."""
    o = Options()
    load_library().hd_default_options(C.byref(o))
    o.precision, o.order, o.budget_m = precision, order, budget_m
    o.capacity, o.max_rounds, o.stack_depth, o.subbatch = capacity, max_rounds, stack_depth, subbatch
    o.profile = profile
    o.learned = learned
    o.autotune = autotune
    o.query_lanes = query_lanes
    o.query_shape = query_shape
    o.eps_relative = 1 if relative else 0
    o.test_bound_shift = float(test_bound_shift)
    o.split_levels = split_levels
    if tuner_cache is not None:
        o._tuner_cache = os.fsencode(tuner_cache)  # kept alive with the options
        o.tuner_cache = o._tuner_cache
    if round_log is not None:
        o._round_log = round_log
        o.round_log = C.cast(round_log, C.c_void_p)
        o.round_log_cap = len(round_log)
    if mlp_params is not None:
        o.mlp_params = mlp_params.data_ptr()
    if log_out is not None:
        assert log_out.is_cuda and log_out.dtype == _torch().float32 and log_out.shape[-1] == 17
        o.log_frontier = 1
        o.log_out = log_out.data_ptr()
        o.log_cap = log_out.shape[0]
    return o


def _round_log(n):
    return (RoundRecord * n)() if n else None


def _with_log(d, log):
    if log is not None:
        d["round_log"] = [log[i].as_dict() for i in range(d["round_records"])]
    return d


def bound(VA, FA, bvh: Bvh, eps: float, round_log: int = 0, **opts):
    """Certified (L, U, stats) with L <= h(A,B) <= U and U - L <= eps (eps
    times dA with relative=True). round_log = n > 0 returns up to n per-round
    records in stats["round_log"]."""
    torch = _torch()
    lib = load_library()
    VA = _dev(VA, torch.float64)
    FA = _dev(FA, torch.int32)
    log = _round_log(round_log)
    o = make_options(round_log=log, **opts)
    LU = (C.c_double * 2)()
    stats = Stats()
    st = lib.hd_bound(C.c_void_p(VA.data_ptr()), VA.shape[0], C.c_void_p(FA.data_ptr()), FA.shape[0],
                      bvh.handle, float(eps), C.byref(o), _stream(), LU, C.byref(stats))
    _check(st, "hd_bound", stats)
    return LU[0], LU[1], _with_log(stats.as_dict(), log)


def hausdorff(VA, FA, VB, FB, eps: float, round_log: int = 0, **opts):
    """Certified (L, U, ((L_AB, U_AB), (L_BA, U_BA)), stats) for the two-sided
    distance H(A,B) = max{h(A,B), h(B,A)}: L <= H <= U, U - L <= eps (eps
    times the larger bounding-box diagonal with relative=True). The two
    one-sided intervals contain their distances but may be wider than eps."""
    torch = _torch()
    lib = load_library()
    VA, VB = _dev(VA, torch.float64), _dev(VB, torch.float64)
    FA, FB = _dev(FA, torch.int32), _dev(FB, torch.int32)
    log = _round_log(round_log)
    o = make_options(round_log=log, **opts)
    LU = (C.c_double * 2)()
    LUd = (C.c_double * 4)()
    stats = Stats()
    st = lib.hd_hausdorff(C.c_void_p(VA.data_ptr()), VA.shape[0], C.c_void_p(FA.data_ptr()), FA.shape[0],
                          C.c_void_p(VB.data_ptr()), VB.shape[0], C.c_void_p(FB.data_ptr()), FB.shape[0], float(eps),
                          C.byref(o), _stream(), LU, LUd, C.byref(stats))
    _check(st, "hd_hausdorff", stats)
    return LU[0], LU[1], ((LUd[0], LUd[1]), (LUd[2], LUd[3])), _with_log(stats.as_dict(), log)


def build_bvh_batched(soups) -> Bvh:
    """One BVH over many soups B_p; soups is a list of (VB, FB)."""
    torch = _torch()
    lib = load_library()
    Vs = [_dev(V, torch.float64) for V, _ in soups]
    Fs = [_dev(F, torch.int32) for _, F in soups]
    n = len(soups)
    vptr = (C.c_void_p * n)(*[V.data_ptr() for V in Vs])
    fptr = (C.c_void_p * n)(*[F.data_ptr() for F in Fs])
    ms = (C.c_int64 * n)(*[V.shape[0] for V in Vs])
    ns = (C.c_int64 * n)(*[F.shape[0] for F in Fs])
    h = C.c_void_p()
    st = lib.hd_build_bvh_batched(n, vptr, ms, fptr, ns, _stream(), C.byref(h))
    _check(st, "hd_build_bvh_batched")
    b = Bvh(h, Vs, Fs)
    b.npairs = n
    return b


def bound_batched(meshes, bvh: Bvh, eps, round_log: int = 0, **opts):
    """Certified [L_p, U_p] for many pairs at once; meshes is a list of
    (VA, FA) in the order of the soups given to build_bvh_batched; eps is one
    value or one per pair (absolute, or relative with relative=True).
    Returns (L list, U list, summed stats)."""
    torch = _torch()
    lib = load_library()
    Vs = [_dev(V, torch.float64) for V, _ in meshes]
    Fs = [_dev(F, torch.int32) for _, F in meshes]
    n = len(meshes)
    vptr = (C.c_void_p * n)(*[V.data_ptr() for V in Vs])
    fptr = (C.c_void_p * n)(*[F.data_ptr() for F in Fs])
    ms = (C.c_int64 * n)(*[V.shape[0] for V in Vs])
    ns = (C.c_int64 * n)(*[F.shape[0] for F in Fs])
    per = not isinstance(eps, (int, float))
    ev = (C.c_double * (n if per else 1))(*([float(e) for e in eps] if per else [float(eps)]))
    log = _round_log(round_log)
    o = make_options(round_log=log, **opts)
    LU = (C.c_double * (2 * n))()
    stats = Stats()
    st = lib.hd_bound_batched(n, vptr, ms, fptr, ns, bvh.handle, ev, 1 if per else 0, C.byref(o), _stream(),
                              LU, C.byref(stats))
    _check(st, "hd_bound_batched", stats)
    return [LU[2 * i] for i in range(n)], [LU[2 * i + 1] for i in range(n)], _with_log(stats.as_dict(), log)


def build_graphs(enable: bool) -> bool:
    """Whether BVH builds run as captured HIP graphs (process-wide); returns
    the previous setting."""
    return bool(load_library().hd_build_graphs(1 if enable else 0))


def point_distances(P, bvh: Bvh, precision=PREC_FP64, lanes=1):
    """(d, I, Q) of points P against B: distance, original face index, closest point
    (lanes: 1 or 4 lanes of a wave per point query)."""
    torch = _torch()
    lib = load_library()
    P = _dev(P, torch.float64)
    n = P.shape[0]
    d = torch.empty(n, dtype=torch.float64, device=P.device)
    I = torch.empty(n, dtype=torch.int32, device=P.device)
    Q = torch.empty((n, 3), dtype=torch.float64, device=P.device)
    st = lib.hd_point_distances(C.c_void_p(P.data_ptr()), n, bvh.handle, precision, lanes, C.c_void_p(d.data_ptr()),
                                C.c_void_p(I.data_ptr()), C.c_void_p(Q.data_ptr()), _stream())
    _check(st, "hd_point_distances")
    return d, I, Q


def point_distances_noalloc(P, bvh: Bvh, precision=PREC_FP64, lanes=1, out=None):
    """point_distances through the entry point that allocates nothing (its
    scratch is a static device array; at most NOALLOC_MAX_POINTS points).
    out: optional (d, I, Q, err) device tensors to write into. Returns
    (d, I, Q, err) with err a one-element device int32 tensor (the status the
    device wrote). Only enqueues work: read err after the stream."""
    torch = _torch()
    lib = load_library()
    P = _dev(P, torch.float64)
    n = P.shape[0]
    if out is None:
        out = (torch.empty(n, dtype=torch.float64, device=P.device), torch.empty(n, dtype=torch.int32, device=P.device),
               torch.empty((n, 3), dtype=torch.float64, device=P.device),
               torch.full((1,), -1, dtype=torch.int32, device=P.device))
    d, I, Q, err = out
    st = lib.hd_point_distances_noalloc(C.c_void_p(P.data_ptr()), n, bvh.handle, precision, lanes,
                                        C.c_void_p(d.data_ptr()), C.c_void_p(I.data_ptr()), C.c_void_p(Q.data_ptr()),
                                        C.c_void_p(err.data_ptr()), _stream())
    _check(st, "hd_point_distances_noalloc")
    return d, I, Q, err


def eval_bounds(v, d, I, q, bvh: Bvh, precision=PREC_FP64):
    """All five bounds (uexact or NaN, u1..u4) of n triangles, and u3's case."""
    torch = _torch()
    lib = load_library()
    v = _dev(v, torch.float64).reshape(-1, 9)
    n = v.shape[0]
    d = _dev(d, torch.float64).reshape(n, 3)
    I = _dev(I, torch.int32).reshape(n, 3)
    q = _dev(q, torch.float64).reshape(n, 9)
    out = torch.empty((n, 5), dtype=torch.float64, device=v.device)
    case = torch.empty(n, dtype=torch.int32, device=v.device)
    st = lib.hd_eval_bounds(C.c_void_p(v.data_ptr()), C.c_void_p(d.data_ptr()), C.c_void_p(I.data_ptr()),
                            C.c_void_p(q.data_ptr()), n, bvh.handle, precision, C.c_void_p(out.data_ptr()),
                            C.c_void_p(case.data_ptr()), _stream())
    _check(st, "hd_eval_bounds")
    return out, case


def eval_bound_u5(v, d, I, bvh: Bvh, precision=PREC_FP64):
    """The fifth bound (Zheng et al.) of n triangles and their barycenters'
    closest faces of B (original indices)."""
    torch = _torch()
    lib = load_library()
    v = _dev(v, torch.float64).reshape(-1, 9)
    n = v.shape[0]
    d = _dev(d, torch.float64).reshape(n, 3)
    I = _dev(I, torch.int32).reshape(n, 3)
    out = torch.empty(n, dtype=torch.float64, device=v.device)
    Sb = torch.empty(n, dtype=torch.int32, device=v.device)
    _check(lib.hd_eval_bound_u5(_ptr(v), _ptr(d), _ptr(I), n, bvh.handle, precision, _ptr(out), _ptr(Sb), _stream()),
           "hd_eval_bound_u5")
    return out, Sb


# ---------------------------------------------------------------------------
# learned proposal: the network
# ---------------------------------------------------------------------------

def mlp_nparams() -> int:
    return int(load_library().hd_mlp_nparams())


def _ptr(x):
    return C.c_void_p(x.data_ptr())


def mlp_forward(X, params):
    """Predictions of the network for the rows of X (n x 16)."""
    torch = _torch()
    lib = load_library()
    X = _dev(X, torch.float32).reshape(-1, 16)
    params = _dev(params, torch.float32)
    y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _check(lib.hd_mlp_forward(_ptr(X), X.shape[0], _ptr(params), _ptr(y), _stream()), "hd_mlp_forward")
    return y


def mlp_grad(X, t, params):
    """(gradient of the mean squared error, loss) for rows X, targets t."""
    torch = _torch()
    lib = load_library()
    X = _dev(X, torch.float32).reshape(-1, 16)
    t = _dev(t, torch.float32)
    params = _dev(params, torch.float32)
    g = torch.empty(mlp_nparams(), dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    _check(lib.hd_mlp_grad(_ptr(X), _ptr(t), X.shape[0], _ptr(params), _ptr(g), _ptr(loss), _stream()),
           "hd_mlp_grad")
    return g, loss


def mlp_train(X, t, rows, batch, params, adam_m, adam_v, step0=0, lr=1e-3):
    """Adam steps in place on params / adam_m / adam_v (device FP32 tensors);
    rows holds nsteps * batch row indices. Returns the minibatch losses."""
    torch = _torch()
    lib = load_library()
    X = _dev(X, torch.float32).reshape(-1, 16)
    t = _dev(t, torch.float32)
    rows = _dev(rows, torch.int32)
    nsteps = rows.numel() // batch
    for a in (params, adam_m, adam_v):
        assert a.is_cuda and a.dtype == torch.float32 and a.is_contiguous()
    loss = torch.empty(max(nsteps, 1), dtype=torch.float32, device=X.device)
    _check(lib.hd_mlp_train(_ptr(X), _ptr(t), _ptr(rows), nsteps, batch, _ptr(params), _ptr(adam_m),
                            _ptr(adam_v), step0, float(lr), _ptr(loss), _stream()), "hd_mlp_train")
    return loss[:nsteps]


def frontier_features(v, d, I, q, bvh: Bvh, L: float, dA: float):
    """The learned proposal's 16 features of n triangles (see hd_frontier_features)."""
    torch = _torch()
    lib = load_library()
    v = _dev(v, torch.float64).reshape(-1, 9)
    n = v.shape[0]
    d = _dev(d, torch.float64).reshape(n, 3)
    I = _dev(I, torch.int32).reshape(n, 3)
    q = _dev(q, torch.float64).reshape(n, 9)
    X = torch.empty((n, 16), dtype=torch.float32, device=v.device)
    _check(lib.hd_frontier_features(_ptr(v), _ptr(d), _ptr(I), _ptr(q), n, bvh.handle, float(L), float(dA),
                                    _ptr(X), _stream()), "hd_frontier_features")
    return X
