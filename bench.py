"""Throughput of one semi-Lagrangian step (foot -> walk -> interpolation) on
one MI355X, through the C-ABI.

Workload (default): the graded 1415 x 1415 grid refined towards the circle
r = 1/4 (2,002,225 nodes, 3,998,792 triangles), time-dependent swirl with
period 1, explicit-midpoint (RK2) feet, Courant number 5 on the
computational spacing, P1, FP64 coordinates and walk, 16 FP32 Gaussian-hill
fields sharing one location.  A step is one fused launch over all nodes.

Prints one JSON line: feet located+interpolated per second, the roofline
position of the step kernel (HBM-bound; algorithmic bytes per step over the
kernel's mean duration from HIP events on its stream), and the CPU oracle's
throughput on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "feet located+interpolated/sec; mean walk steps; learned vs plain walk"


def algorithmic_bytes(n_feet: int, n_tris: int, c_x: int, c_v: int, k: int, order: int = 1) -> int:
    """Each array the step must touch, counted once: per foot its coordinates,
    a start id, an element id, K values in and K values out; per triangle its
    three vertex ids (P2: 6 DOF ids, 8-byte start/elem pair per DOF)."""
    if order == 1:
        return n_feet * (c_x + 4 + 4 + 2 * k * c_v) + 12 * n_tris
    return n_feet * (c_x + 8 + 2 * k * c_v) + 24 * n_tris


def cpu_baseline(w, budget_s: float = 10.0):
    """The oracle (feet, brute-force bucket location with exact predicates,
    interpolation) on whole steps of the same workload until budget_s."""
    from oracle import oracle as O
    v = np.ascontiguousarray(w.v0, dtype=np.float64)
    t0 = time.perf_counter()
    steps = 0
    t_n = 0.0
    while True:
        v, _, _, _ = O.sl_step(w.xy, w.tri, v, w.field, t_n, w.dt, w.scheme)
        t_n += w.dt
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 50:
            break
    feet = steps * w.xy.shape[0]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": feet / el, "unit": "feet/s", "cores": min(threads, os.cpu_count() or 1), "kind": "oracle",
            "sample": f"{steps} whole oracle steps of the same workload ({feet} feet, {el:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--alpha", type=float, default=5.0)
    ap.add_argument("--n", type=int, default=1415)
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times (to scale HBM counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": 4 * n, "copy_bytes_written_per_launch": 4 * n, "launches": 5}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the multi-GPU sharding is a design "
                                   "(halo exchange of V^n rows), not an implementation", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2104_09189_amd import inputs as I
    from paper_2104_09189_amd import slwalk as S

    w = I.graded_swirl(alpha=args.alpha, n=args.n, k_fields=args.k)
    ctx = S.Context(0)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    mesh = S.Mesh(ctx, w.xy, w.tri, S.INTERNAL_ORDER)
    upload_s = time.perf_counter() - t0
    perm = mesh.dof_order()
    v_a = torch.from_numpy(np.ascontiguousarray(w.v0[perm])).to("cuda:0")
    v_b = torch.empty_like(v_a)
    n_feet = mesh.n_nodes

    # walk statistics of one step (separate call: counters are a different kernel variant)
    _, st = mesh.step(w.field, 0.0, w.dt, w.scheme, v_a, v_b, stats=True)

    def run(step0, count):
        nonlocal v_a, v_b
        for s in range(count):
            mesh.step(w.field, (step0 + s) * w.dt, w.dt, w.scheme, v_a, v_b)
            v_a, v_b = v_b, v_a

    run(0, args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    run(args.warmup, args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    value = n_feet * args.steps / (gpu_ms * 1e-3)

    # the step kernel alone, per launch (one launch per step in this mode)
    kernel_ms = []
    for s in range(min(args.steps, 20)):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        mesh.step(w.field, s * w.dt, w.dt, w.scheme, v_a, v_b)
        e1.record(stream)
        v_a, v_b = v_b, v_a
        kernel_ms.append((e0, e1))
    torch.cuda.synchronize()
    kms = float(np.mean([a.elapsed_time(b) for a, b in kernel_ms]))
    abytes = algorithmic_bytes(n_feet, mesh.n_tris, 16, 4, args.k)
    achieved = abytes / (kms * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "feet/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_nodes": int(n_feet), "n_tris": int(mesh.n_tris), "alpha": args.alpha,
                   "k_fields": args.k, "coords": "f64", "values": "f32", "order": 1, "scheme": "rk2",
                   "start": "steered incident triangle", "parallelism": "none (1 GPU)"},
        "field_values_per_s": value * args.k,
        "mean_walk_steps": st["walk_steps"] / max(st["feet"], 1),
        "walk": {k: st[k] for k in ("max_steps", "outside", "exact_tests", "fallback_walks", "edge_ties",
                                    "vertex_ties")},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_step<false, float>",
                     "kernel_ms": kms, "algorithmic_bytes": abytes},
        "upload_s": upload_s,
        "wall_s": wall,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
