"""Benchmark: milliseconds to an eps-certified [L, U] for h(A,B) on one MI355X.

A step is one whole pass of the method on one resident input pair: build the
LBVH over B, then the certified bound for A (the BVH build is inside the
timed step, as in the paper's totals). Prints one JSON line.

Default workload: the near-zero case, a displaced torus on a 160 x 160 grid
(51,200 triangles) against a periodic Delaunay re-triangulation of the same
surface from 20,000 random points (40,000 triangles), eps = 1e-5 * dA, FP32
arithmetic with an FP64 recheck band and an FP64 final step.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to eps-certified h(A,B) (ms), learned vs plain; point-tri dist evals/s"

# Algorithmic work per unit in the query kernel (LBVH traversal + point-triangle
# distances). Bytes: a four-wide node is one 128 B line, a leaf's FP32 frame
# 64 B, a query reads its point (3 x 8 B) and writes d, I, q, p and its key
# (40 B). FP32 operations counted from the source of the frame evaluation and
# the box test (an FMA counts as 2).
BYTES_PER_NODE = 128
BYTES_PER_LEAF = 64
BYTES_PER_QUERY = 64
BOXES_PER_NODE = 4
FLOP_PER_LEAF = 63       # one point-triangle distance in the triangle's frame
FLOP_PER_BOX = 11        # one point-box squared distance
FLOP_PER_QUERY = 70      # final closest point + square root per query
PEAK_HBM = 8000.0         # GB/s, MI355X datasheet HBM3E
PEAK_FP32_VECTOR = 157.3  # TFLOP/s, MI355X datasheet vector FP32


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--precision", default="fp32+recheck", choices=["fp64", "fp32", "fp32+recheck"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", type=int, default=1, choices=[0, 1],
                    help="1: the first warm-up call picks the query kernel's launch shape; 0: the "
                         "default shape (profiling runs use it, so every counter run times the same shape)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-vs-plain comparison on the large torus")
    ap.add_argument("--learned-subbatch", type=int, default=8192)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (x4) and an FP32 elementwise product of "
                         "as many floats (x4): the references for the HBM byte counters (FETCH_SIZE / "
                         "WRITE_SIZE) and the FP32 FLOP counter (SQ_INSTS_VALU_FLOPS_FP32) of a rocprofv3 "
                         "--pmc run")
    return ap.parse_args()


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


# HBM traffic of the query kernel from a rocprofv3 --pmc run, valid only for
# the kernel sources it was measured on (their hash is stored beside it)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_query_traffic_c2_torus.json")
KERNEL_SOURCES = ["hd_kernels.hpp", "hd_geom.hpp", "hd_math.hpp", "hd_engine.hip", "hd_bvh.hip"]


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
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("config") != config or t.get("source_sha256") != kernel_source_hash() or not tuned:
        return None
    v = t.get("per_variant", {}).get(query_kernel_name(tuned))
    # only a shape whose counters cover the launches of timed steps (the
    # others were counted on the autotuner's trial launches alone)
    return v.get("hbm_bytes_per_launch") if v and v.get("timed") else None


def cpu_baseline(W, reps=3):
    import oracle
    times, res = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        res = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="tree")
        times.append((time.perf_counter() - t0) * 1e3)
    return statistics.median(times), res


def bbox_diag(W):
    """dA: diagonal of the bounding box of A's referenced vertices."""
    import numpy as np
    V = W.VA[np.unique(W.FA)]
    return float(np.linalg.norm(V.max(0) - V.min(0)))


def cpu_baseline_pairs(pairs, budget_s=15.0):
    """The oracle on the first pairs of the batch until about budget_s of CPU
    work, scaled to the whole batch by face count."""
    import oracle
    t_total, faces, res = 0.0, 0, []
    for W in pairs:
        t0 = time.perf_counter()
        r = oracle.bound(W.VA, W.FA, W.VB, W.FB, W.eps_rel, backend="tree")
        t_total += time.perf_counter() - t0
        faces += W.FA.shape[0]
        res.append(r)
        if t_total > budget_s:
            break
    all_faces = sum(W.FA.shape[0] for W in pairs)
    return t_total * 1e3 * all_faces / faces, res, faces


def learned_comparison(a, hd, torch, wl):
    """Train the proposal network on the GPU from frontier logs of the plain
    method (torus, thin strip at quarter size, 32 many-pair pairs), then time
    plain and learned on the large torus (1M vs 800k triangles) with the same
    sub-batched scheduler. Untimed by the step loop; reported beside it."""
    from paper_2406_10357_amd import learned
    K = a.learned_subbatch
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
    W5 = wl.config(5)
    VA, FA, VB, FB = (torch.from_numpy(x).cuda() for x in (W5.VA, W5.FA, W5.VB, W5.FB))
    bvh = hd.build_bvh(VB, FB)
    res = {0: [], 1: []}
    for rep in range(3):
        for mode in (0, 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L, U, st = hd.bound(VA, FA, bvh, W5.eps_rel, subbatch=K, learned=mode,
                                mlp_params=params if mode else None)
            res[mode].append(((time.perf_counter() - t0) * 1e3, L, U, st))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Lb, Ub, sb = hd.bound(VA, FA, bvh, W5.eps_rel)
    bf_ms = (time.perf_counter() - t0) * 1e3

    def summary(mode):
        ms = statistics.median(r[0] for r in res[mode])
        _, L, U, st = res[mode][-1]
        return {"ms": round(ms, 3), "L": L, "U": U, "nodes_bounded": st["nodes_bounded"],
                "subdivided": st["subdivided"], "rounds": st["rounds"], "queries": st["queries"]}

    return {"workload": f"C5 torus 1000x500 ({W5.FA.shape[0]} F) vs periodic Delaunay 400k ({W5.FB.shape[0]} F), "
                        "sigma 5e-4, eps 1e-5*dA, FP32+recheck", "subbatch": K,
            "train": {"rows": int(rows.shape[0]), "log_s": round(t_log, 2), "train_s": round(t_train, 2),
                      "steps": int(len(losses)), "heldout_mse_before": vb, "heldout_mse_after": va,
                      "label_variance": float(rows[:, 16].var())},
            "plain": summary(0), "learned": summary(1),
            "plain_breadth_first": {"ms": round(bf_ms, 3), "nodes_bounded": sb["nodes_bounded"], "rounds": sb["rounds"]},
            "timing": "hd_bound only (BVH prebuilt), median of 3"}


def main():
    a = parse()
    if a.calibrate_copy:
        calibrate_copy(a.calibrate_copy)
        return
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported (the library runs on one "
              "GPU per process and has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2406_10357_amd as hd
    from paper_2406_10357_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    prec = {"fp64": hd.PREC_FP64, "fp32": hd.PREC_FP32, "fp32+recheck": hd.PREC_FP32_RECHECK}[a.precision]
    batched = a.config == 4
    if batched:
        print("generating the 256 pairs ...", file=sys.stderr, flush=True)
        pairs = wl.batched_pairs(256, workers=min(16, os.cpu_count() or 1))
        cu = lambda x: torch.from_numpy(x).cuda()
        soupsB = [(cu(P.VB), cu(P.FB)) for P in pairs]
        soupsA = [(cu(P.VA), cu(P.FA)) for P in pairs]
        eps = [P.eps_rel for P in pairs]
        W = pairs[0]
    else:
        W = wl.config(a.config)
        VA = torch.from_numpy(W.VA).cuda()
        FA = torch.from_numpy(W.FA).cuda()
        VB = torch.from_numpy(W.VB).cuda()
        FB = torch.from_numpy(W.FB).cuda()
    torch.cuda.synchronize()

    def step(profile=0, autotune=0):
        if batched:
            bvh = hd.build_bvh_batched(soupsB)
            return hd.bound_batched(soupsA, bvh, eps, precision=prec, profile=profile, autotune=autotune)
        bvh = hd.build_bvh(VB, FB)
        return hd.bound(VA, FA, bvh, W.eps_rel, precision=prec, profile=profile, autotune=autotune)

    # the first warm-up call also picks the query kernel's launch shape
    tuned = None
    for i in range(a.warmup):
        r = step(autotune=1 if i == 0 and a.autotune else 0)
        tuned = tuned or {k: r[2][k] for k in ("query_block", "query_stack", "query_quad_max")}
        print(f"warmup {i + 1}/{a.warmup} done", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(a.steps):
        # the last timed step also takes HIP events around its query kernels
        # (every event record costs the stream a few µs, so one step carries them)
        results.append(step(profile=2 if i == a.steps - 1 else 0))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / a.steps
    print(f"timed {a.steps} steps: {ms:.3f} ms/step", file=sys.stderr, flush=True)

    L, U, st = results[-1]
    timed_q = [r for r in results if r[2]["query_launches"] > 0]  # the step with events
    q_ms = sum(r[2]["ms_query_kernels"] for r in timed_q)
    q_leaf = sum(r[2]["query_leaf_evals"] for r in timed_q)
    q_box = sum(r[2]["query_box_tests"] for r in timed_q)
    q_n = sum(r[2]["queries"] for r in timed_q)
    q_launch = sum(r[2]["query_launches"] for r in timed_q)
    evals = sum(r[2]["pt_tri_evals"] for r in results)
    flops = FLOP_PER_LEAF * q_leaf + FLOP_PER_BOX * q_box + FLOP_PER_QUERY * q_n
    nbytes = BYTES_PER_NODE * q_box / BOXES_PER_NODE + BYTES_PER_LEAF * q_leaf + BYTES_PER_QUERY * q_n
    achieved = nbytes / (q_ms * 1e-3) / 1e9 if q_ms > 0 else None
    tflops = flops / (q_ms * 1e-3) / 1e12 if q_ms > 0 else None

    if batched:
        nA_all = sum(P.FA.shape[0] for P in pairs)
        nB_all = sum(P.FB.shape[0] for P in pairs)
        workload = {"workload": f"C4 256 pairs (noisy spheres / tori, {nA_all} / {nB_all} F in all, "
                                "eps 1e-4*dA per pair)", "npairs": 256, "nA": nA_all, "nB": nB_all,
                    "eps_rel": 1e-4, "precision": a.precision, "variant": "one batched call, breadth-first rounds"}
        result = {"rounds": st["rounds"], "subdivided": st["subdivided"], "nodes_bounded": st["nodes_bounded"],
                  "queries": st["queries"], "pt_tri_evals": st["pt_tri_evals"],
                  "max_width_over_eps": max((u - l) / (P.eps_rel * bbox_diag(P)) for l, u, P in zip(L, U, pairs)),
                  "status": st["status"]}
    else:
        workload = {"workload": W.name, "nA": int(W.FA.shape[0]), "nB": int(W.FB.shape[0]),
                    "eps_rel": W.eps_rel, "precision": a.precision,
                    "variant": "plain cascade 1234, breadth-first rounds"}
        result = {"L": L, "U": U, "dA": st["dA"], "eps_abs": st["eps_abs"], "rounds": st["rounds"],
                  "subdivided": st["subdivided"], "nodes_bounded": st["nodes_bounded"],
                  "queries": st["queries"], "pt_tri_evals": st["pt_tri_evals"],
                  "query_leaf_evals": st["query_leaf_evals"], "query_box_tests": st["query_box_tests"],
                  "discards": st["discards"], "rechecked64": st["rechecked64"],
                  "parked_final": st["parked_final"]}
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
        "dtype": "f64" if a.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": workload,
        "result": result,
        # point-triangle distance evaluations (query leaves and the third
        # bound's) per second of whole-step time
        "evals_per_s": evals / (ms * 1e-3 * a.steps),
        "autotuned": tuned,
        "learned_ms": None,
        "roofline": {
            "kernel": query_kernel_name(tuned) + " (four-wide LBVH traversal + point-triangle distances; "
                      "launches of at most query_quad_max queries run a quad of lanes per query)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM,
            "unit": "GB/s",
            "frac": (achieved / PEAK_HBM) if achieved else None,
            "traffic": measured_traffic(a.config, tuned),
            "launches": q_launch,
            "avg_launch_ms": q_ms / q_launch if q_launch else None,
            "algorithmic_bytes_per_launch": nbytes / q_launch if q_launch else None,
            "fp32_tflops": tflops,
            "fp32_frac_of_157_3": (tflops / PEAK_FP32_VECTOR) if tflops else None,
        },
    }
    if not a.no_learned and not batched:
        print("learned vs plain on the large torus ...", file=sys.stderr, flush=True)
        lc = learned_comparison(a, hd, torch, wl)
        out["learned"] = lc
        out["learned_ms"] = lc["learned"]["ms"]
    if not a.no_cpu_baseline and batched:
        print("timing the CPU oracle on a sample of the pairs ...", file=sys.stderr, flush=True)
        cms, refs, faces = cpu_baseline_pairs(pairs)
        out["cpu_baseline"] = {"value": round(cms, 1), "unit": "ms", "cores": 1, "kind": "oracle",
                               "sample": f"single-threaded FP64 oracle (own AABB tree) on the first {len(refs)} "
                                         f"pairs ({faces} of {nA_all} A faces), scaled to the batch by face count"}
        ok = [bool(L[i] <= r["U"] and r["L"] <= U[i]) for i, r in enumerate(refs)]
        out["parity"] = {"pairs_checked": len(refs), "overlap_all": all(ok),
                         "max_dL_over_eps": max(abs(L[i] - r["L"]) / r["eps_abs"] for i, r in enumerate(refs))}
    elif not a.no_cpu_baseline:
        print("timing the CPU oracle on the same workload ...", file=sys.stderr, flush=True)
        cms, ref = cpu_baseline(W)
        out["cpu_baseline"] = {"value": round(cms, 3), "unit": "ms", "cores": 1, "kind": "oracle",
                               "sample": "the full workload, single-threaded FP64 oracle with its own AABB "
                                         "tree, median of 3 runs (tree build included)"}
        out["parity"] = {"oracle_L": ref["L"], "oracle_U": ref["U"],
                         "overlap": bool(L <= ref["U"] and ref["L"] <= U),
                         "dL_over_dA": abs(L - ref["L"]) / st["dA"], "dU_over_dA": abs(U - ref["U"]) / st["dA"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
