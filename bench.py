"""Benchmark: milliseconds to an eps-certified [L, U] for h(A,B) on one MI355X.

A step is one whole pass of the method on one resident input pair: build the
LBVH over B, then the certified bound for A (the BVH build is inside the
timed step, as in the paper's totals, which include the tree construction).
Prints one JSON line.

Default workload (--config 5): a displaced torus on a 1000 x 500 grid
(1,000,000 triangles) against a periodic Delaunay re-triangulation of the same
surface from 400,000 random points with normal noise sigma = 5e-4 (800,000
triangles), eps = 1e-5 * dA, FP32 arithmetic with the FP64 recheck band and an
FP64 final step. `value` is the plain cascade in breadth-first rounds; the same
line carries the plain cascade with the paper's best-first order (sub-batches
of the largest upper bounds) and the learned order (the network, trained on the
GPU from frontier logs of the other workloads first), each timed the same way,
the torus of 51 k faces (C2) and the 256-pair batch (C4) as extra keys, the
query kernel's roofline, the CPU oracle on the host and the parity of the
interval against it.

Other modes: --mode eps-curve (time to certify for eps = 1e-1 .. 1e-5),
--mode order-study (every cascade order and subset of the four bounds).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to eps-certified h(A,B) (ms), learned vs plain; point-tri dist evals/s"

# Algorithmic work per unit in the query kernel (LBVH traversal + point-triangle
# distances). Bytes: a four-wide node is one 128 B line (32 B per box test), a
# leaf's FP32 frame 64 B, a query reads its point (3 x 8 B) and writes d, I,
# q, p and its key (40 B). FP32 operations counted from the source of the
# frame evaluation and the box test (an FMA counts as 2).
BYTES_PER_NODE = 128
BYTES_PER_LEAF = 64
BYTES_PER_QUERY = 64
BOXES_PER_NODE = 4
FLOP_PER_LEAF = 63       # one point-triangle distance in the triangle's frame
FLOP_PER_BOX = 11        # one point-box squared distance
FLOP_PER_QUERY = 70      # final closest point + square root per query
PEAK_HBM = 8000.0         # GB/s, MI355X datasheet HBM3E
PEAK_FP32_VECTOR = 157.3  # TFLOP/s, MI355X datasheet vector FP32
PRECISIONS = {"fp64": 0, "fp32": 1, "fp32+recheck": 2}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--precision", default=None, choices=list(PRECISIONS),
                    help="default: the arithmetic the workload names")
    ap.add_argument("--mode", default="bench", choices=["bench", "eps-curve", "order-study"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the C2 and C4 keys")
    ap.add_argument("--autotune", type=int, default=1, choices=[0, 1],
                    help="1: the first warm-up call picks the query kernel's launch shape; 0: the "
                         "default shape (profiling runs use it, so every counter run times the same shape)")
    ap.add_argument("--no-learned", action="store_true", help="skip the best-first and learned variants")
    ap.add_argument("--query-shape", type=int, default=0, choices=range(0, 10),
                    help="headline steps: force launch shape k of the query kernel (1..9; 0: tuned or default)")
    ap.add_argument("--learned-subbatch", type=int, default=8192)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (x4) and an FP32 elementwise product of "
                         "as many floats (x4): the references for the HBM byte counters (FETCH_SIZE / "
                         "WRITE_SIZE) and the FP32 FLOP counter (SQ_INSTS_VALU_FLOPS_FP32) of a rocprofv3 "
                         "--pmc run")
    ap.add_argument("--study-configs", default="2,3,4", help="order-study / eps-curve: the workloads")
    ap.add_argument("--out", default=None, help="also write the JSON line (or the study) to this file")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def calibrate_copy(mib):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(4):
        dst.copy_(src)
    out = torch.empty_like(src)
    for _ in range(4):
        torch.mul(src, dst, out=out)  # one FP32 multiply per element
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy, then elementwise FP32 product", "bytes_read_per_launch": n * 4,
                      "bytes_written_per_launch": n * 4, "fp32_flop_per_product_launch": n, "launches": 4}),
          flush=True)


# HBM traffic of the query kernel from rocprofv3 --pmc runs, valid only for
# the kernel sources it was measured on (their hash is stored beside it)
TRAFFIC_FILES = {2: os.path.join(ROOT, "profiles", "k_query_traffic_c2_torus.json"),
                 5: os.path.join(ROOT, "profiles", "k_query_traffic_c5_torus.json")}
KERNEL_SOURCES = ["hd_kernels.hpp", "hd_geom.hpp", "hd_math.hpp", "hd_reduce.hpp", "hd_internal.hpp", "hd_engine.hip",
                  "hd_bvh.hip"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2406_10357_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def query_kernel_name(tuned, T="float"):
    """The query kernel's name in rocprofv3 output for a launch shape."""
    if not tuned:
        return f"k_query<{T}>"
    return f"k_query<{T}, {tuned['query_stack']}, {tuned['query_block']}>"


def measured_traffic(config, tuned):
    """HBM bytes per launch of the query kernel in the launch shape the timed
    steps used, or None when not measured for these sources and workload."""
    try:
        with open(TRAFFIC_FILES[config]) as fh:
            t = json.load(fh)
    except (KeyError, OSError, ValueError):
        return None
    if t.get("config") != config or t.get("source_sha256") != kernel_source_hash() or not tuned:
        return None
    v = t.get("per_variant", {}).get(query_kernel_name(tuned))
    # only a shape whose counters cover the launches of timed steps (the
    # others were counted on the autotuner's trial launches alone)
    return v.get("hbm_bytes_per_launch") if v and v.get("timed") else None


def host_cpu():
    """Core count and model of the host."""
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "cpu_count": os.cpu_count(), "usable_cores": usable}


def bbox_diag(W):
    """dA: diagonal of the bounding box of A's referenced vertices."""
    import numpy as np
    V = W.VA[np.unique(W.FA)]
    return float(np.linalg.norm(V.max(0) - V.min(0)))


# ---------------------------------------------------------------------------
# timing
# ---------------------------------------------------------------------------

class Single:
    """One (A, B) pair resident in HBM; step() = BVH build + certified bound."""

    def __init__(self, hd, torch, W, prec):
        self.hd, self.torch, self.W, self.prec = hd, torch, W, prec
        cu = lambda x: torch.from_numpy(x).cuda()
        self.VA, self.FA, self.VB, self.FB = cu(W.VA), cu(W.FA), cu(W.VB), cu(W.FB)
        torch.cuda.synchronize()

    def step(self, **opts):
        bvh = self.hd.build_bvh(self.VB, self.FB)
        return self.hd.bound(self.VA, self.FA, bvh, self.W.eps_rel, relative=True, precision=self.prec, **opts)


class Batch:
    """Many pairs resident in HBM; step() = one batched BVH build + one batched bound."""

    def __init__(self, hd, torch, pairs, prec):
        self.hd, self.torch, self.pairs, self.prec = hd, torch, pairs, prec
        cu = lambda x: torch.from_numpy(x).cuda()
        self.soupsB = [(cu(P.VB), cu(P.FB)) for P in pairs]
        self.soupsA = [(cu(P.VA), cu(P.FA)) for P in pairs]
        self.eps = [P.eps_rel for P in pairs]
        torch.cuda.synchronize()

    def step(self, **opts):
        bvh = self.hd.build_bvh_batched(self.soupsB)
        return self.hd.bound_batched(self.soupsA, bvh, self.eps, relative=True, precision=self.prec, **opts)


def timed(run, steps, warmup, autotune=0, events_last=True, **opts):
    """Warm-up calls (the first may tune), then `steps` timed calls between
    two device synchronisations; the last timed call carries HIP events around
    its query kernels (profile=2) when events_last. Returns (ms per step, the
    results, the tuned launch shape)."""
    import torch
    tuned = None
    for i in range(warmup):
        r = run(autotune=1 if (i == 0 and autotune) else 0, **opts)
        tuned = tuned or {k: r[2][k] for k in ("query_block", "query_stack", "query_quad_max")}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [run(profile=2 if (events_last and i == steps - 1) else 0, **opts) for i in range(steps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    if tuned is None:
        tuned = {k: res[-1][2][k] for k in ("query_block", "query_stack", "query_quad_max")}
    return ms, res, tuned


def roofline(results, tuned, traffic):
    """The query kernel's roofline from the steps that carried HIP events."""
    ev = [r for r in results if r[2]["query_launches"] > 0]
    q_ms = sum(r[2]["ms_query_kernels"] for r in ev)
    q_leaf = sum(r[2]["query_leaf_evals"] for r in ev)
    q_box = sum(r[2]["query_box_tests"] for r in ev)
    q_n = sum(r[2]["queries"] for r in ev)
    q_launch = sum(r[2]["query_launches"] for r in ev)
    if not q_launch or q_ms <= 0:
        return None
    flops = FLOP_PER_LEAF * q_leaf + FLOP_PER_BOX * q_box + FLOP_PER_QUERY * q_n
    nbytes = BYTES_PER_NODE * q_box / BOXES_PER_NODE + BYTES_PER_LEAF * q_leaf + BYTES_PER_QUERY * q_n
    avg_ms = q_ms / q_launch
    achieved = nbytes / (q_ms * 1e-3) / 1e9
    tflops = flops / (q_ms * 1e-3) / 1e12
    out = {
        "kernel": query_kernel_name(tuned) + " (four-wide LBVH traversal + point-triangle distances; launches "
                                             "of at most query_quad_max queries run a quad of lanes per query)",
        "bound": "hbm",
        "achieved": achieved,
        "peak": PEAK_HBM,
        "unit": "GB/s",
        "frac": achieved / PEAK_HBM,
        "traffic": traffic,
        "achieved_note": "algorithmic bytes (128 B per wide node visited, 64 B per leaf frame, 64 B per query) "
                         "over the launch time; most of them are served by the L2 and the Infinity Cache",
        "launches": q_launch,
        "avg_launch_ms": avg_ms,
        "algorithmic_bytes_per_launch": nbytes / q_launch,
        "box_tests_per_query": q_box / q_n if q_n else None,
        "leaves_per_query": q_leaf / q_n if q_n else None,
        "fp32_tflops_algorithmic": tflops,
        "fp32_frac_of_157_3": tflops / PEAK_FP32_VECTOR,
        "fp32_gap_to_half_peak": (0.5 * PEAK_FP32_VECTOR) / tflops if tflops > 0 else None,
    }
    if traffic:
        hbm = traffic / (avg_ms * 1e-3) / 1e9
        out["hbm_measured_GBps"] = hbm
        out["hbm_measured_frac"] = hbm / PEAK_HBM
    return out


def summary(ms, res):
    L, U, st = res[-1]
    return {"ms": round(ms, 4), "L": L, "U": U, "rounds": st["rounds"], "nodes_bounded": st["nodes_bounded"],
            "subdivided": st["subdivided"], "queries": st["queries"], "pt_tri_evals": st["pt_tri_evals"],
            "status": st["status"]}


# ---------------------------------------------------------------------------
# CPU oracle on the host (the reported baseline)
# ---------------------------------------------------------------------------

def oracle_bound_tree(W):
    import oracle
    return oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="tree")


def cpu_oracle(W, threads=1):
    import oracle
    t0 = time.perf_counter()
    res = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="tree", threads=threads)
    return (time.perf_counter() - t0) * 1e3, res


def tree_check(W, ref, hd, torch, bvh, npts=10000, threads=16):
    """The oracle's AABB tree (the backend of the CPU baseline on the large
    workloads) against its brute force at npts random points around B plus
    the vertex that attains the oracle's L; and the GPU's FP64 point query at
    the same points. Brute force runs over threads (each a C call)."""
    import numpy as np
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    rng = np.random.default_rng(2406)
    lo, hi = W.VB.min(0), W.VB.max(0)
    pad = 0.05 * (hi - lo)
    P = np.concatenate([rng.uniform(lo - pad, hi + pad, size=(npts, 3)), np.asarray(ref["argmax"])[None]])
    t0 = time.perf_counter()
    chunks = np.array_split(np.arange(P.shape[0]), threads)
    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda c: oracle.points_soup(P[c], W.VB, W.FB), chunks))
    dB = np.concatenate([p[0] for p in parts])
    IB = np.concatenate([p[1] for p in parts])
    t_brute = time.perf_counter() - t0
    tree = oracle.Tree(W.VB, W.FB)
    dT = np.empty(P.shape[0])
    IT = np.empty(P.shape[0], np.int64)
    for i, x in enumerate(P):
        dT[i], IT[i], _, _ = tree.query(x)
    dG = hd.point_distances(torch.from_numpy(P).cuda(), bvh, precision=hd.PREC_FP64)[0].cpu().numpy()
    scale = float(np.abs(W.VB).max())
    return {"points": int(P.shape[0]), "includes_argmax_vertex": True,
            "tree_equals_brute": bool(np.array_equal(dT, dB) and np.array_equal(IT, IB)),
            "tree_max_abs_diff": float(np.abs(dT - dB).max()),
            "gpu_fp64_max_abs_diff_over_scale": float(np.abs(dG - dB).max() / scale),
            "argmax_vertex_d_brute": float(dB[-1]), "brute_s": round(t_brute, 2), "brute_threads": threads}


def parity_of(L, U, st, ref):
    return {"oracle_L": ref["L"], "oracle_U": ref["U"], "overlap": bool(L <= ref["U"] and ref["L"] <= U),
            "dL_over_dA": abs(L - ref["L"]) / st["dA"], "dU_over_dA": abs(U - ref["U"]) / st["dA"],
            "dL_over_eps": abs(L - ref["L"]) / st["eps_abs"], "width_over_eps": (U - L) / st["eps_abs"]}


def pairs_parity(pairs, L, U, budget_s=20.0):
    """The oracle on a stratified sample of the pairs (the three smallest, the
    three largest and evenly spaced ones between), until about budget_s of CPU
    work; returns the checks and the CPU time per face."""
    import numpy as np
    import oracle
    order = np.argsort([P.FA.shape[0] for P in pairs])
    mid = np.linspace(3, len(order) - 4, 8).round().astype(int)[1:-1] if len(order) >= 24 else []
    sample = list(order[:3]) + list(order[-3:]) + [int(order[j]) for j in mid]
    checks, t_total, faces = [], 0.0, 0
    for i in sample:
        P = pairs[int(i)]
        t0 = time.perf_counter()
        r = oracle.bound(P.VA, P.FA, P.VB, P.FB, P.eps_rel, backend="tree")
        t_total += time.perf_counter() - t0
        faces += P.FA.shape[0]
        checks.append({"pair": int(i), "nA": int(P.FA.shape[0]),
                       "overlap": bool(L[i] <= r["U"] and r["L"] <= U[i]),
                       "dL_over_eps": abs(L[i] - r["L"]) / r["eps_abs"]})
        if t_total > budget_s:
            break
    return checks, t_total, faces


# ---------------------------------------------------------------------------
# learned proposal
# ---------------------------------------------------------------------------

def train_network(wl, K):
    """Train the proposal network on the GPU from frontier logs of the plain
    method on the other workloads: the 51 k torus, the thin strip at a quarter
    of its size, and 32 pairs of the many-pair generator."""
    import torch
    from paper_2406_10357_amd import learned
    W2, W3 = wl.config(2), wl.config(3, scale=0.25)
    pairs = wl.batched_pairs(32, nmax=20000, workers=min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    rows = learned.log_frontier([(W2.VA, W2.FA, W2.VB, W2.FB, W2.eps_rel), (W3.VA, W3.FA, W3.VB, W3.FB, W3.eps_rel),
                                 [(P.VA, P.FA, P.VB, P.FB, P.eps_rel) for P in pairs]], subbatch=K, cap=1 << 19)
    t_log = time.perf_counter() - t0
    t0 = time.perf_counter()
    params, losses, (vb, va) = learned.train(rows, epochs=6)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    info = {"rows": int(rows.shape[0]), "log_s": round(t_log, 2), "train_s": round(t_train, 2),
            "steps": int(len(losses)), "heldout_mse_before": vb, "heldout_mse_after": va,
            "label_variance": float(rows[:, 16].var()),
            "sources": "frontier logs of C2 (51 k torus), C3 at quarter size, 32 many-pair pairs; C5 held out"}
    return params, info


# ---------------------------------------------------------------------------
# modes
# ---------------------------------------------------------------------------

def workload_info(W, prec_name, variant):
    return {"workload": W.name, "nA": int(W.FA.shape[0]), "nB": int(W.FB.shape[0]), "eps_rel": W.eps_rel,
            "precision": prec_name, "variant": variant}


def bench_main(a, hd, torch, wl):
    cfg = a.config
    batched = cfg == 4
    prec_name = a.precision or ("fp64" if cfg == 1 else ("fp32" if cfg == 3 else "fp32+recheck"))
    prec = PRECISIONS[prec_name]
    if batched:
        log("generating the 256 pairs ...")
        pairs = wl.batched_pairs(256, workers=min(16, os.cpu_count() or 1))
        run = Batch(hd, torch, pairs, prec)
        W = None
    else:
        log(f"generating config {cfg} ...")
        W = wl.config(cfg)
        run = Single(hd, torch, W, prec)

    log("plain cascade, breadth-first rounds: warm-up and timed steps ...")
    ms, res, tuned = timed(run.step, a.steps, a.warmup, autotune=a.autotune, query_shape=a.query_shape)
    log(f"  {ms:.3f} ms/step")
    L, U, st = res[-1]
    evals = sum(r[2]["pt_tri_evals"] for r in res)
    rl = roofline(res, tuned, measured_traffic(cfg, tuned))

    if batched:
        nA_all = sum(P.FA.shape[0] for P in pairs)
        nB_all = sum(P.FB.shape[0] for P in pairs)
        workload = {"workload": f"C4 256 pairs (noisy spheres / tori, {nA_all} / {nB_all} F in all, "
                                "eps 1e-4*dA per pair)", "npairs": 256, "nA": nA_all, "nB": nB_all,
                    "eps_rel": 1e-4, "precision": prec_name, "variant": "one batched call, breadth-first rounds"}
        result = {"rounds": st["rounds"], "subdivided": st["subdivided"], "nodes_bounded": st["nodes_bounded"],
                  "queries": st["queries"], "pt_tri_evals": st["pt_tri_evals"], "status": st["status"],
                  "max_width_over_eps": max((u - l) / (P.eps_rel * bbox_diag(P)) for l, u, P in zip(L, U, pairs))}
    else:
        workload = workload_info(W, prec_name, "plain cascade 1234, breadth-first rounds, BVH build in the step")
        result = {"L": L, "U": U, "dA": st["dA"], "eps_abs": st["eps_abs"], "rounds": st["rounds"],
                  "subdivided": st["subdivided"], "nodes_bounded": st["nodes_bounded"],
                  "queries": st["queries"], "pt_tri_evals": st["pt_tri_evals"],
                  "query_leaf_evals": st["query_leaf_evals"], "query_box_tests": st["query_box_tests"],
                  "discards": st["discards"], "rechecked64": st["rechecked64"],
                  "parked_final": st["parked_final"], "status": st["status"]}
    out = {
        "metric": METRIC,
        "value": round(ms, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec_name == "fp64" else "f32",
        "data": "synthetic",
        "config": workload,
        "result": result,
        # point-triangle distance evaluations (query leaves and the third
        # bound's) per second of whole-step time
        "evals_per_s": evals / (ms * 1e-3 * a.steps),
        "autotuned": tuned,
        "roofline": rl,
    }

    # best-first (sub-batched) and learned orders, the same step and timing
    if not a.no_learned and not batched:
        K = a.learned_subbatch
        log("training the proposal network on frontier logs of C2, C3 (quarter) and 32 pairs ...")
        params, tinfo = train_network(wl, K)
        variants = {}
        for name, opts in (("plain_best_first", {"subbatch": K}),
                           ("learned", {"subbatch": K, "learned": 1, "mlp_params": params})):
            log(f"{name}: timed steps ...")
            vms, vres, _ = timed(run.step, a.steps, 1, events_last=False, **opts)
            variants[name] = summary(vms, vres)
            log(f"  {vms:.3f} ms/step")
        variants["plain_breadth_first"] = summary(ms, res)
        out["learned_vs_plain"] = {"subbatch": K, "train": tinfo, **variants,
                                   "timing": "BVH build + bound per step, the same steps and clock as value"}
        out["learned_ms"] = variants["learned"]["ms"]

    # CPU oracle on the host: single-threaded (the paper's design point) and
    # with the vertex-query phase over every usable core
    cpu = host_cpu()
    if not a.no_cpu_baseline and not batched:
        log("CPU oracle on the same workload (single-threaded, then threaded vertex phase) ...")
        c1, ref = cpu_oracle(W, threads=1)
        cn, refn = cpu_oracle(W, threads=cpu["usable_cores"])
        assert refn["L"] == ref["L"] and refn["U"] == ref["U"]
        out["cpu_baseline"] = {"value": round(c1, 1), "unit": "ms", "cores": 1, "kind": "oracle",
                               "sample": "the full workload: single-threaded FP64 oracle with its own AABB tree "
                                         "(tree build included), one run",
                               "threaded": {"value": round(cn, 1), "cores": cpu["usable_cores"],
                                            "what": "the same with the vertex-query phase split over the cores"},
                               "host": cpu}
        out["parity"] = parity_of(L, U, st, ref)
        log("oracle tree and GPU FP64 queries against brute force at 10^4 points ...")
        # (brute force over the 800 k triangles of the large torus costs about
        # 0.15 core-seconds per point: 2000 points here, 10^4 on the 51 k torus)
        out["parity"]["tree_check"] = tree_check(W, ref, hd, torch, hd.build_bvh(run.VB, run.FB),
                                                 npts=2000 if W.FB.shape[0] > 200000 else 10000,
                                                 threads=min(16, cpu["usable_cores"]))
    elif not a.no_cpu_baseline and batched:
        log("CPU oracle on a stratified sample of the pairs ...")
        checks, t_s, faces = pairs_parity(pairs, L, U)
        nA_all = sum(P.FA.shape[0] for P in pairs)
        out["cpu_baseline"] = {"value": round(t_s * 1e3 * nA_all / faces, 1), "unit": "ms", "cores": 1,
                               "kind": "oracle", "host": cpu,
                               "sample": f"single-threaded FP64 oracle (own AABB tree) on {len(checks)} stratified "
                                         f"pairs ({faces} of {nA_all} A faces), scaled to the batch by face count"}
        out["parity"] = {"pairs_checked": len(checks), "overlap_all": all(c["overlap"] for c in checks),
                         "max_dL_over_eps": max(c["dL_over_eps"] for c in checks), "pairs": checks}

    # extra keys: the 51 k torus and the 256-pair batch, same step definition
    if not a.no_extra and cfg == 5:
        log("extra: C2 torus 51 k vs 40 k ...")
        W2 = wl.config(2)
        r2 = Single(hd, torch, W2, PRECISIONS["fp32+recheck"])
        ms2, res2, tuned2 = timed(r2.step, a.steps, a.warmup)
        out["c2"] = {"config": workload_info(W2, "fp32+recheck", "plain cascade 1234, breadth-first rounds"),
                     **summary(ms2, res2), "roofline": roofline(res2, tuned2, measured_traffic(2, tuned2))}
        log(f"  {ms2:.3f} ms/step")
        if not a.no_cpu_baseline:
            log("  oracle, and its tree and GPU FP64 queries against brute force at 10^4 points ...")
            L2, U2, st2 = res2[-1]
            t0 = time.perf_counter()
            ref2 = oracle_bound_tree(W2)
            out["c2"]["parity"] = parity_of(L2, U2, st2, ref2)
            out["c2"]["parity"]["oracle_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
            out["c2"]["parity"]["tree_check"] = tree_check(W2, ref2, hd, torch, hd.build_bvh(r2.VB, r2.FB),
                                                           npts=10000, threads=min(16, cpu["usable_cores"]))
        log("extra: C4 256 pairs ...")
        pairs = wl.batched_pairs(256, workers=min(16, os.cpu_count() or 1))
        r4 = Batch(hd, torch, pairs, PRECISIONS["fp32+recheck"])
        ms4, res4, _ = timed(r4.step, 3, 1)
        L4, U4, st4 = res4[-1]
        c4 = {"config": {"workload": "C4 256 pairs (noisy spheres / tori, log-uniform 1e3..1e5 faces), "
                                     "eps 1e-4*dA per pair", "nA": sum(P.FA.shape[0] for P in pairs),
                         "nB": sum(P.FB.shape[0] for P in pairs), "precision": "fp32+recheck",
                         "variant": "one batched BVH build + one batched bound per step"},
              "ms": round(ms4, 3), "rounds": st4["rounds"], "subdivided": st4["subdivided"],
              "status": st4["status"],
              "max_width_over_eps": max((u - l) / (P.eps_rel * bbox_diag(P)) for l, u, P in zip(L4, U4, pairs))}
        log(f"  {ms4:.3f} ms/step")
        if not a.no_cpu_baseline:
            log("  oracle on a stratified sample of the pairs ...")
            checks, t_s, faces = pairs_parity(pairs, L4, U4, budget_s=15.0)
            c4["parity"] = {"pairs_checked": len(checks), "overlap_all": all(c["overlap"] for c in checks),
                            "max_dL_over_eps": max(c["dL_over_eps"] for c in checks),
                            "nA_checked": [c["nA"] for c in checks]}
        out["c4"] = c4
    return out


def eps_curve_main(a, hd, torch, wl):
    """Time to a certified interval as eps shrinks (the paper's runtime versus
    tolerance comparison), on the torus, the thin strip and the large torus."""
    rows = []
    for cfg in [int(c) for c in (a.study_configs if a.study_configs != "2,3,4" else "2,3,5").split(",")]:
        W = wl.config(cfg)
        prec_name = "fp32" if cfg == 3 else "fp32+recheck"
        run = Single(hd, torch, W, PRECISIONS[prec_name])
        for e in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5):
            W.eps_rel = e
            ms, res, _ = timed(run.step, max(1, a.steps // 2), 1, events_last=False)
            L, U, st = res[-1]
            rows.append({"config": cfg, "workload": W.name, "precision": prec_name, "eps_rel": e, "ms": round(ms, 4),
                         "rounds": st["rounds"], "subdivided": st["subdivided"], "nodes_bounded": st["nodes_bounded"],
                         "L": L, "U": U})
            log(f"C{cfg} eps {e:g}: {ms:.3f} ms, {st['subdivided']} subdivided")
    return {"mode": "eps-curve", "step": "BVH build + certified bound", "rows": rows}


def order_study_main(a, hd, torch, wl):
    """Every cascade order: the 24 orders of the four bounds and all 40
    ordered proper subsets (64 in all), on C2, C3 and C4 (the paper's bound
    order benchmark, and its question whether fewer bounds suit a GPU), plus
    the bound of Zheng et al. (5) alone, before and after the four."""
    import itertools
    orders = []
    for r in (1, 2, 3, 4):
        orders += [int("".join(map(str, p))) for p in itertools.permutations((1, 2, 3, 4), r)]
    orders += [5, 12345, 51234, 1245]
    rows = []
    for cfg in [int(c) for c in a.study_configs.split(",")]:
        if cfg == 4:
            pairs = wl.batched_pairs(256, workers=min(16, os.cpu_count() or 1))
            run = Batch(hd, torch, pairs, PRECISIONS["fp32+recheck"])
            name = "C4 256 pairs"
        else:
            W = wl.config(cfg)
            run = Single(hd, torch, W, PRECISIONS["fp32" if cfg == 3 else "fp32+recheck"])
            name = W.name
        for o in orders:
            try:
                ms, res, _ = timed(run.step, max(1, a.steps // 2), 1, events_last=False, order=o)
            except hd.HDError as e:
                rows.append({"config": cfg, "workload": name, "order": o, "status": e.status})
                continue
            st = res[-1][2]
            rows.append({"config": cfg, "workload": name, "order": o, "ms": round(ms, 4), "rounds": st["rounds"],
                         "subdivided": st["subdivided"], "nodes_bounded": st["nodes_bounded"],
                         "pt_tri_evals": st["pt_tri_evals"], "discards": st["discards"], "status": st["status"]})
            log(f"C{cfg} order {o}: {ms:.3f} ms, {st['subdivided']} subdivided")
    return {"mode": "order-study", "step": "BVH build + certified bound", "rows": rows}


def main():
    a = parse()
    if a.calibrate_copy:
        calibrate_copy(a.calibrate_copy)
        return
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported (the library runs on one "
              "GPU per process and has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2406_10357_amd as hd
    from paper_2406_10357_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    hd.load_library()
    if a.mode == "bench":
        out = bench_main(a, hd, torch, wl)
    elif a.mode == "eps-curve":
        out = eps_curve_main(a, hd, torch, wl)
    else:
        out = order_study_main(a, hd, torch, wl)
    line = json.dumps(out)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(line + "\n")
    print(line, flush=True)


if __name__ == "__main__":
    main()
