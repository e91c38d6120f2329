"""Throughput of one semi-Lagrangian step (foot -> walk -> interpolation) on
one MI355X, through the C-ABI.

Workload (default): the graded 1415 x 1415 grid refined towards the circle
r = 1/4 (2,002,225 nodes, 3,998,792 triangles), time-dependent swirl with
period 1, explicit-midpoint (RK2) feet, Courant number 5 on the
computational spacing, P1, FP64 coordinates and feet, 16 FP32 Gaussian-hill
fields sharing one location.  A step is one fused kernel launch over all
nodes: foot, start element, barycentric walk, tie rule, weights, values.

The headline is strategy (a) of the paper (the walk starts from the node's
own incident triangle, here the one facing the foot).  Strategies (b) (start
from the element found at the previous step) and (c) (start from the element
found for a neighbouring node) are measured beside it, then K-field reuse,
the 64-mesh batch, and the learned start on the same mesh at Courant 50.

Prints one JSON line: feet located+interpolated per second, the roofline
position of the step kernel (HBM-bound; algorithmic bytes per launch over the
kernel's mean duration from HIP events around each launch of the timed
region), and the CPU oracle's throughput on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "feet located+interpolated/sec; mean walk steps; learned vs plain walk"
KERNEL_SRC = os.path.join(ROOT, "paper_2104_09189_amd", "csrc", "slw_kernels.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_step_graded1415_rk2_a5_K16_hbm_counters.md")


def algorithmic_bytes(n_feet: int, n_tris: int, c_x: int, c_v: int, k: int, order: int = 1) -> int:
    """Each array the step must touch, counted once: per foot its coordinates,
    a start id, an element id, K values in and K values out; per triangle its
    three vertex ids (P2: six DOF ids and an 8-byte start/element pair)."""
    if order == 1:
        return n_feet * (c_x + 4 + 4 + 2 * k * c_v) + 12 * n_tris
    return n_feet * (c_x + 8 + 2 * k * c_v) + 24 * n_tris


def kernel_source_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source (else None)."""
    try:
        txt = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    h = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not h or not b or h.group(1) != kernel_source_hash():
        return None
    return float(b.group(1))


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def hist_dict(step_hist) -> dict:
    """slw_stats.step_hist as {"[a,b)": count} (bin 0: no element change)."""
    out = {"[0,1)": int(step_hist[0])}
    for b in range(1, 16):
        lo, hi = 1 << (b - 1), (1 << b) if b < 15 else None
        out[f"[{lo},{hi if hi else 'inf'})"] = int(step_hist[b])
    return out


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
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "sample": f"{steps} whole oracle steps of the same workload ({feet} feet, {el:.1f} s)"}


def run_steps(mesh, w, v_a, v_b, step0, count, start_mode, per_launch_events=False):
    import torch
    evs = []
    stream = torch.cuda.current_stream()
    for s in range(count):
        if per_launch_events:
            e0 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        mesh.step(w.field, (step0 + s) * w.dt, w.dt, w.scheme, v_a, v_b, start_mode=start_mode)
        if per_launch_events:
            e1 = torch.cuda.Event(enable_timing=True)
            e1.record(stream)
            evs.append((e0, e1))
        v_a, v_b = v_b, v_a
    return v_a, v_b, evs


def measure(mesh, w, v0, steps, warmup, start_mode):
    """Warm up, then time exactly `steps` steps between two synchronisations;
    the kernel's own mean duration comes from events around each launch."""
    import torch
    from paper_2104_09189_amd import slwalk as S
    v_a = v0.clone()
    v_b = torch.empty_like(v_a)
    # walk statistics of one step (the counting variant of the kernel)
    t_stats = 0.0
    if start_mode in (S.START_PREV, S.START_HYBRID):
        # strategy (b) and the hybrid: the first step has no previous
        # elements; measure the one after it
        mesh.step(w.field, 0.0, w.dt, w.scheme, v_a, v_b, start_mode=start_mode)
        t_stats = w.dt
    _, st = mesh.step(w.field, t_stats, w.dt, w.scheme, v_a, v_b, start_mode=start_mode, stats=True)
    v_a, v_b, _ = run_steps(mesh, w, v_a, v_b, 0, warmup, start_mode)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    v_a, v_b, evs = run_steps(mesh, w, v_a, v_b, warmup, steps, start_mode, per_launch_events=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    return {"ms_per_step": gpu_ms / steps, "kernel_ms": kernel_ms, "wall_s": wall, "stats": st}


def measure_precision(alpha=5.0, steps=20, warmup=3):
    """FP32 coordinates, feet, weights and values (FP64 and exact fallback
    for the orientation signs) against the FP64 path on the 500 x 500
    jittered mesh in Morton input order, swirl, Euler, Courant alpha, P1, one
    field: time per step of each; the FP32 values' error per step from the
    same V^n (mid-run, relative to max |V^n|) and after the whole run to
    t = T (the FP64 path itself matches the oracle to 1e-12 per step in the
    tests); the share of feet located in the same element (the two paths
    round the coordinates differently, so feet near edges may legitimately
    land in a neighbour)."""
    import torch
    from paper_2104_09189_amd import inputs as I
    from paper_2104_09189_amd import slwalk as S
    w = I.swirl_500(alpha=alpha, order="morton")
    ctx = S.Context(0)
    res = {"workload": w.name, "n_nodes": int(w.xy.shape[0]), "n_tris": int(w.tri.shape[0]), "steps_to_T": w.steps}
    meshes, vals = {}, {}
    for name, flags, dtype in (("f64", 0, torch.float64), ("f32", S.COORDS_F32, torch.float32)):
        mesh = S.Mesh(ctx, w.xy, w.tri, S.INTERNAL_ORDER | flags)
        perm = mesh.dof_order()
        v0 = torch.from_numpy(np.ascontiguousarray(w.v0[perm])).to("cuda:0", dtype)
        r = measure(mesh, w, v0, steps, warmup, S.START_STEERED)
        res[name] = {"ms_per_step": r["ms_per_step"], "kernel_ms": r["kernel_ms"],
                     "feet_per_s": mesh.n_nodes / (r["ms_per_step"] * 1e-3)}
        meshes[name], vals[name] = (mesh, perm), v0
    # one step from the same V^n at mid-run (V^n from the FP64 run)
    m64, p64 = meshes["f64"]
    m32, p32 = meshes["f32"]
    mid = w.steps // 2
    va = vals["f64"].clone()
    vb = torch.empty_like(va)
    va, vb, _ = run_steps(m64, w, va, vb, 0, mid, S.START_STEERED)
    vn_user = np.empty_like(va.cpu().numpy())
    vn_user[p64] = va.cpu().numpy()
    t = mid * w.dt
    a64 = m64.step(w.field, t, w.dt, w.scheme, va)
    vn32 = torch.from_numpy(np.ascontiguousarray(vn_user[p32])).to("cuda:0", torch.float32)
    a32 = m32.step(w.field, t, w.dt, w.scheme, vn32)
    e64 = m64.locate_feet(w.field, t + w.dt, w.dt, w.scheme)["elem"]
    e32 = m32.locate_feet(w.field, t + w.dt, w.dt, w.scheme)["elem"]
    torch.cuda.synchronize()
    u64 = np.empty(a64.shape[0]); u64[p64] = a64.cpu().numpy()[:, 0]
    u32 = np.empty(a32.shape[0]); u32[p32] = a32.cpu().numpy()[:, 0].astype(np.float64)
    scale = float(np.abs(vn_user).max())
    g64 = np.empty(e64.shape[0], dtype=np.int64); g64[p64] = e64.cpu().numpy()
    g32 = np.empty(e32.shape[0], dtype=np.int64); g32[p32] = e32.cpu().numpy()
    res["step_error_f32_vs_f64"] = float(np.abs(u32 - u64).max() / scale)
    res["same_element_share"] = float((g64 == g32).mean())
    # the whole run to t = T in each precision
    ends = {}
    for name in ("f64", "f32"):
        mesh, perm = meshes[name]
        va = vals[name].clone()
        vb = torch.empty_like(va)
        va, vb, _ = run_steps(mesh, w, va, vb, 0, w.steps, S.START_STEERED)
        torch.cuda.synchronize()
        u = np.empty(va.shape[0]); u[perm] = va.cpu().numpy()[:, 0].astype(np.float64)
        ends[name] = u
    res["run_error_f32_vs_f64"] = float(np.abs(ends["f32"] - ends["f64"]).max() / np.abs(w.v0).max())
    res["speedup_f32"] = res["f64"]["ms_per_step"] / res["f32"]["ms_per_step"]
    return res


def measure_k_reuse(mesh, w, v0, reps=20):
    """One location reused by K fields (one K = 16 step) against K separate
    single-field steps (K locations) on the same mesh and feet."""
    import torch
    stream = torch.cuda.current_stream()
    k = v0.shape[1]
    v_out = torch.empty_like(v0)
    singles = [v0[:, i:i + 1].contiguous() for i in range(k)]
    outs = [torch.empty_like(x) for x in singles]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_k = timed(lambda: mesh.step(w.field, 0.0, w.dt, w.scheme, v0, v_out))
    t_1 = timed(lambda: [mesh.step(w.field, 0.0, w.dt, w.scheme, a, b) for a, b in zip(singles, outs)])
    return {"k_fields": k, "one_location_ms": t_k, "separate_locations_ms": t_1, "speedup": t_1 / t_k}


def measure_decomposition(mesh, w, v0, steps=20, warmup=3):
    """Where a step's time goes: strategy (a) and strategy (b) (almost no
    moves: the previous step's element), each with all K fields and with
    the first field alone, on the same mesh, feet and launch configuration.
    (a) minus (b) with one field is the cost of the walk's moves; (a) with K
    fields minus (a) with one is the cost of the other K - 1 fields; (b)
    with one field is the rest (coordinates, starts, feet, vertex ids, one
    field).  ms per step, HIP events around `steps` steps, after one
    untimed run of the first configuration."""
    from paper_2104_09189_amd import slwalk as S
    k = v0.shape[1]
    v1 = v0[:, :1].contiguous()
    out = {"k_fields": k}
    _time_steps(mesh, w.field, w.dt, w.scheme, v0, steps, warmup)  # clocks up before the first timed run
    for name, mode in (("a", S.START_STEERED), ("b", S.START_PREV)):
        for tag, v in ((f"k{k}", v0), ("k1", v1)):
            ms, st = _time_steps(mesh, w.field, w.dt, w.scheme, v, steps, warmup, start_mode=mode)
            out[f"{name}_{tag}_ms"] = ms
        out[f"{name}_mean_walk_steps"] = st["walk_steps"] / max(st["feet"], 1)
    out["walk_moves_ms"] = out["a_k1_ms"] - out["b_k1_ms"]
    out["other_fields_ms"] = out[f"a_k{k}_ms"] - out["a_k1_ms"]
    out["rest_ms"] = out["b_k1_ms"]
    return out


def measure_batch(steps=100):
    """64 jittered meshes, triangle counts log-uniform in [1e4, 5e5], own swirl
    period each, Courant 5, Euler, float coordinates (float filter, FP64 and
    exact fallback), one float field: one launch per step for all meshes,
    100 steps captured in one HIP graph, schedule chosen by the autotuner;
    against the plain path (one step launch per mesh)."""
    import torch
    from paper_2104_09189_amd import inputs as I
    from paper_2104_09189_amd import slwalk as S
    wl = I.batch_meshes()
    ctx = S.Context(0)
    # Hilbert order: measured faster than the Morton order for these short walks
    meshes = [S.Mesh(ctx, w.xy, w.tri, S.INTERNAL_ORDER | S.COORDS_F32 | S.HILBERT) for w in wl]
    va = [torch.from_numpy(np.ascontiguousarray(w.v0[m.dof_order()])).cuda() for w, m in zip(wl, meshes)]
    vb = [torch.empty_like(a) for a in va]
    b = S.Batch(ctx, meshes)
    b.set_fields([w.field for w in wl], [w.dt for w in wl])
    b.set_values(va, vb)
    schedule, block = b.autotune(S.SLW_EULER)
    b.set_step(0)
    g = b.capture(steps, S.SLW_EULER)
    stream = torch.cuda.current_stream()
    g.launch()                      # warm-up replay
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    g.launch()
    e1.record(stream)
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / steps
    st = b.step(S.SLW_EULER, stats=True)
    # plain path: one slw_step launch per mesh and step
    outs = [torch.empty_like(a) for a in va]

    def plain_step(n):
        for w, m, a, o in zip(wl, meshes, va, outs):
            m.step(w.field, n * w.dt, w.dt, w.scheme, a, o)
    plain_step(0)
    torch.cuda.synchronize()
    e0.record(stream)
    for n in range(10):
        plain_step(n)
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / 10
    n_nodes = sum(m.n_nodes for m in meshes)
    n_tris = sum(m.n_tris for m in meshes)
    abytes = n_nodes * (8 + 4 + 4 + 2 * 4) + 12 * n_tris
    g.free()
    # the same batch with strategy (b)'s start (each mesh's previous
    # elements), its own autotuned schedule, 100 steps in one graph
    b.set_start(S.START_PREV)
    b.set_step(0)
    b.step(S.SLW_EULER)                                    # previous elements for the autotuner
    schedule_b, block_b = b.autotune(S.SLW_EULER)
    b.set_step(0)
    gb = b.capture(steps, S.SLW_EULER)
    gb.launch()
    torch.cuda.synchronize()
    e0.record(stream)
    gb.launch()
    e1.record(stream)
    torch.cuda.synchronize()
    prev_ms = e0.elapsed_time(e1) / steps
    st_b = b.step(S.SLW_EULER, stats=True)
    gb.free()
    b.free()
    return {"workload": f"{len(meshes)} jittered meshes, swirl, Courant 5, float coordinates, 1 field, Hilbert order",
            "n_nodes": n_nodes, "n_tris": n_tris, "steps_in_graph": steps, "schedule": schedule, "block": block,
            "ms_per_step": graph_ms, "feet_per_s": n_nodes / (graph_ms * 1e-3),
            "roofline_frac": abytes / (graph_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "mean_walk_steps": st["walk_steps"] / max(st["feet"], 1),
            "plain_one_launch_per_mesh_ms_per_step": plain_ms, "speedup_vs_plain": plain_ms / graph_ms,
            "previous_element_start": {"schedule": schedule_b, "block": block_b, "ms_per_step": prev_ms,
                                       "feet_per_s": n_nodes / (prev_ms * 1e-3),
                                       "roofline_frac": abytes / (prev_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                       "mean_walk_steps": st_b["walk_steps"] / max(st_b["feet"], 1)}}


def _walk_histogram(steps: np.ndarray) -> dict:
    """Walk steps per foot: percentiles and counts in power-of-two bins."""
    edges = [0, 1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 1 << 30]
    counts, _ = np.histogram(steps, bins=edges)
    wave = steps[: steps.size // 64 * 64].reshape(-1, 64).max(axis=1)
    return {"mean": float(steps.mean()), "p50": float(np.percentile(steps, 50)),
            "p90": float(np.percentile(steps, 90)), "p99": float(np.percentile(steps, 99)),
            "max": int(steps.max()), "mean_wavefront_max": float(wave.mean()),
            "bins": {f"[{a},{b})": int(c) for a, b, c in zip(edges[:-1], edges[1:], counts)}}


def measure_learned(alpha=50.0, n=1415, k=16, steps=10, samples_per_step=200_000, train_steps=50, seed=5005,
                    w=None):
    """Learned start on the graded mesh at a large Courant number (or on the
    workload w): the network is trained on the GPU on feet that the plain
    walk locates over 50 steps (10M samples), then steps with the learned
    start (per-foot choice between the network's proposal and the steered
    start), with the learned index (the network's cell corrected by galloping
    searches in the chart tables) and with the exact chart-cell start (binary
    searches, no network) are timed beside the plain steered walk; all must
    give identical bits."""
    import torch
    from paper_2104_09189_amd import inputs as I
    from paper_2104_09189_amd import slwalk as S
    if w is None:
        w = I.graded_swirl(alpha=alpha, n=n, k_fields=k)
    k = w.v0.shape[1]
    ctx = S.Context(0)
    mesh = S.Mesh(ctx, w.xy, w.tri, S.INTERNAL_ORDER)
    # about one triangle per chart cell
    g = 1 << int(np.ceil(np.log2(np.sqrt(mesh.n_tris))))
    t0 = time.perf_counter()
    mesh.chart_build(g)
    chart_s = time.perf_counter() - t0
    nd = mesh.n_dofs
    rng = np.random.default_rng(seed)
    m = samples_per_step * train_steps
    X = torch.empty((m, 5), dtype=torch.float32, device="cuda:0")
    Y = torch.empty((m, 2), dtype=torch.float32, device="cuda:0")
    t0 = time.perf_counter()
    for s in range(train_steps):
        ids = torch.from_numpy(rng.integers(0, nd, samples_per_step).astype(np.int32)).to("cuda:0")
        sl = slice(s * samples_per_step, (s + 1) * samples_per_step)
        mesh.learned_gather(w.field, (s + 1) * w.dt, w.dt, w.scheme, ids, X[sl], Y[sl])
    torch.cuda.synchronize()
    gather_s = time.perf_counter() - t0
    net = S.Mlp(ctx, seed=0)
    net.fit_normalization(X)
    t0 = time.perf_counter()
    # minibatches of 65,536 samples (each fills the device: 1,024 workgroups)
    plan = [(3e-3, 65536, 24), (1e-3, 65536, 12)]
    for i, (lr, bs, ep) in enumerate(plan):
        loss = net.train(X, Y, epochs=ep, batch=bs, lr=lr, seed=seed + i)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    mesh.attach_mlp(net)
    del X, Y
    # the network's error on fresh feet (a step it was not trained on), in
    # chart cells: how far its proposal lands from the foot's element
    ids = torch.from_numpy(rng.integers(0, nd, 200_000).astype(np.int32)).to("cuda:0")
    Xe = torch.empty((ids.shape[0], 5), dtype=torch.float32, device="cuda:0")
    Ye = torch.empty((ids.shape[0], 2), dtype=torch.float32, device="cuda:0")
    mesh.learned_gather(w.field, (train_steps + 3.5) * w.dt, w.dt, w.scheme, ids, Xe, Ye)
    pe = net.forward(Xe).cpu().numpy()
    ye = Ye.cpu().numpy()
    ok = np.isfinite(ye[:, 0])
    err = np.abs(pe[ok] - ye[ok]) * g
    net_error = {"samples": int(ok.sum()), "unit": "chart cells (1/G)",
                 "du": {q: float(np.percentile(err[:, 0], p)) for q, p in (("p50", 50), ("p90", 90), ("p99", 99))},
                 "dv": {q: float(np.percentile(err[:, 1], p)) for q, p in (("p50", 50), ("p90", 90), ("p99", 99))},
                 "rms_chart_units": float(np.sqrt(np.mean((pe[ok] - ye[ok]) ** 2)))}
    del Xe, Ye
    v0 = torch.from_numpy(np.ascontiguousarray(w.v0[mesh.dof_order()])).to("cuda:0")
    stream = torch.cuda.current_stream()
    t_n = 7 * w.dt
    res = {}
    outs = {}
    for name, mode in (("plain_steered", S.START_STEERED), ("learned", S.START_LEARNED),
                       ("learned_index", S.START_LEARNED_INDEX), ("chart_exact", S.START_CHART)):
        vo = torch.empty_like(v0)
        mesh.step(w.field, t_n, w.dt, w.scheme, v0, vo, start_mode=mode)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            mesh.step(w.field, t_n, w.dt, w.scheme, v0, vo, start_mode=mode)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        outs[name] = vo.cpu().numpy()
        loc = mesh.locate_feet(w.field, t_n + w.dt, w.dt, w.scheme, start_mode=mode, want_steps=True,
                               want_bary=False)
        hist = _walk_histogram(loc["steps"].cpu().numpy().astype(np.int64))
        res[name] = {"ms_per_step": ms, "feet_per_s": mesh.n_nodes / (ms * 1e-3), "walk_steps": hist}
    identical = all(np.array_equal(outs["plain_steered"], outs[x]) for x in ("learned", "learned_index", "chart_exact"))
    base = res["plain_steered"]["ms_per_step"]
    return {"workload": w.name, "n_nodes": int(mesh.n_nodes), "n_tris": int(mesh.n_tris),
            "alpha": w.extra.get("alpha", alpha),
            "k_fields": k, "chart_g": g, "chart_build_s": chart_s, "training_samples": m,
            "gather_s": gather_s, "train_s": train_s, "train_plan": plan, "final_minibatch_loss": loss,
            "network_error": net_error,
            "starts": res, "identical_bits": identical,
            "speedup_learned_vs_plain": base / res["learned"]["ms_per_step"],
            "speedup_learned_index_vs_plain": base / res["learned_index"]["ms_per_step"],
            "speedup_chart_vs_plain": base / res["chart_exact"]["ms_per_step"]}


def torch_zeros_like_values(mesh, k=1):
    import torch
    return torch.zeros((mesh.n_nodes, k), dtype=torch.float32, device="cuda:0")


def wave_walks(mesh, w, t_n, mode) -> dict:
    """Walk lengths of one step's feet (element changes per foot) as the step
    kernel's wavefronts see them: 64 consecutive internal-order DOFs per
    wavefront, each waiting for its longest walk."""
    from paper_2104_09189_amd import slwalk as S
    if mode in (S.START_NEIGHBOR, S.START_HYBRID):
        # the step's own statistics (slw_locate_feet has neither the forest
        # nor the hybrid choice): the mean and maximum, no per-foot lengths
        _, st = mesh.step(w.field, t_n, w.dt, w.scheme, torch_zeros_like_values(mesh), start_mode=mode, stats=True)
        return {"mean": st["walk_steps"] / max(st["feet"], 1), "mean_wavefront_max": None, "p99": None,
                "max": st["max_steps"]}
    if mode == S.START_PREV:
        # the previous element of every DOF from the step before
        mesh.locate_feet(w.field, t_n, w.dt, w.scheme, start_mode=mode, want_bary=False, want_elem=False)
    loc = mesh.locate_feet(w.field, t_n + w.dt, w.dt, w.scheme, start_mode=mode, want_steps=True,
                           want_bary=False, want_elem=False)
    st = loc["steps"].cpu().numpy().astype(np.int64)
    return _walk_histogram(st)


def _library_defaults(mesh):
    """The step's settings as a fresh mesh has them (one foot per lane, the
    forest, the automatic hybrid threshold, chunks of 64 tiles per XCD turn,
    512 walk records in LDS)."""
    mesh.set_repack(0)
    mesh.set_chain(0)
    mesh.set_hybrid(0.0)
    mesh.set_xcd_chunk(64)
    mesh.set_lds_window(512)


def measure_courant_range(mesh, w, v0, steps=20, warmup=3, alphas=(1.0, 5.0, 20.0, 50.0, 100.0), chart_g=2048,
                          grid_g=16384):
    """The graded mesh across its Courant range: strategy (a) (steered
    incident start), strategy (b) (previous element), strategy (c) (the
    forest), the exact chart start, the jump-and-walk grid start and the
    hybrid (previous element, else the grid cell), each with ms per step,
    kernel time, HBM-roofline fraction and the walk lengths (mean, and the
    mean over wavefronts of each wavefront's longest walk, which sets its
    time)."""
    import dataclasses
    from paper_2104_09189_amd import inputs as I
    from paper_2104_09189_amd import slwalk as S
    if mesh.chart_g != chart_g:
        mesh.chart_build(chart_g)
    t0 = time.perf_counter()
    mesh.build_grid(grid_g)
    grid_build_s = time.perf_counter() - t0
    abytes = algorithmic_bytes(mesh.n_nodes, mesh.n_tris, 16, 4, v0.shape[1])
    out = {"grid": {"g": grid_g, "bytes": 4 * grid_g * grid_g, "build_s": grid_build_s}}
    for alpha in alphas:
        dt, _ = I.courant_dt(alpha, w.h)
        wa = dataclasses.replace(w, dt=dt)
        line = {"dt": dt}
        for name, mode in (("a_steered", S.START_STEERED), ("b_previous", S.START_PREV),
                           ("c_forest", S.START_NEIGHBOR), ("chart_exact", S.START_CHART),
                           ("grid", S.START_GRID), ("hybrid", S.START_HYBRID)):
            # the library's defaults: one foot per lane, the forest, hybrid
            # threshold automatic (0), chunks of 64 tiles per XCD turn, 512
            # walk records staged in LDS (the autotuner below leaves its
            # choices set on the mesh)
            _library_defaults(mesh)
            r = measure(mesh, wa, v0, steps, warmup, mode)
            # walk lengths of the step ending near t = 1/4 (the swirl's time
            # factor cos(pi t) is 0.7 there; it vanishes at t = 1/2)
            ww = wave_walks(mesh, wa, max(round(0.25 / dt) - 1, 0) * dt, mode)
            line[name] = {"ms_per_step": r["ms_per_step"], "kernel_ms": r["kernel_ms"],
                          "feet_per_s": mesh.n_nodes / (r["ms_per_step"] * 1e-3),
                          "roofline_frac": abytes / (r["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "mean_walk_steps": ww["mean"], "mean_wavefront_max": ww["mean_wavefront_max"],
                          "p99": ww["p99"], "max": ww["max"]}
            # the same after slw_step_autotune (the mode's knob, then the XCD
            # chunk), tuned on the step ending near t = 1/4 (previous
            # elements from the step before; near t = 1/2 the field vanishes
            # and no foot moves)
            t_tune = max(round(0.25 / dt) - 1, 1) * dt
            if mode in (S.START_PREV, S.START_HYBRID):
                mesh.step(wa.field, t_tune - dt, dt, wa.scheme, v0, start_mode=mode)
            with tempfile.TemporaryDirectory() as tmp:
                cache = os.path.join(tmp, "tune.json")
                knob, chunk, _ = mesh.autotune_step(wa.field, t_tune, dt, wa.scheme, v0, start_mode=mode,
                                                    cache_path=cache, with_chunk=True)
                m = re.search(r'"lds_window":\s*(\d+)', open(cache).read())
            rt = measure(mesh, wa, v0, steps, warmup, mode)
            line[name]["tuned"] = {"knob": knob, "xcd_chunk": chunk, "lds_window": int(m.group(1)) if m else None,
                                   "ms_per_step": rt["ms_per_step"], "kernel_ms": rt["kernel_ms"]}
        _library_defaults(mesh)
        best = min((v["kernel_ms"], k) for k, v in line.items() if k != "dt")
        line["fastest"] = best[1]
        out[f"alpha_{alpha:g}"] = line
    mesh.build_grid(0)
    return out


def measure_cpu_walk(w, gpu_walk_ms=None):
    """The paper's own walk on the host cores (Algorithm 1 in plain FP64,
    strategy (a)'s start: a random incident triangle as in the paper, and the
    incident triangle whose angle contains the foot direction), on one
    thread and on all cores, for the feet of the locators line (t = 8 dt).
    Walk only, as the GPU's walk-only locator beside it."""
    from oracle import oracle as O
    from oracle import walk as W
    q = O.feet(w.xy, w.field, 8 * w.dt, w.dt, w.scheme)
    M = W.Mesh(w.xy, w.tri)
    n = int(w.xy.shape[0])
    cores = W.max_threads()
    out = {"points": n, "cores": cores, "cpu_model": cpu_model(), "kind": "paper walk (Algorithm 1, FP64)"}
    for name, rule in (("sector_start", W.RULE_SECTOR), ("random_incident_start", W.RULE_RANDOM)):
        line = {}
        for threads in (1, cores):
            t0 = time.perf_counter()
            e, st = M.locate_nodes(q, rule, seed=11, threads=threads)
            el = time.perf_counter() - t0
            line[f"threads_{threads}_feet_per_s"] = n / el
            line[f"threads_{threads}_s"] = el
        line["mean_walk_steps"] = float(st[e >= 0].mean())
        line["outside"] = int((e == -1).sum())
        out[name] = line
    if gpu_walk_ms:
        out["gpu_walk_only_feet_per_s"] = n / (gpu_walk_ms * 1e-3)
        out["gpu_vs_all_cores"] = out["gpu_walk_only_feet_per_s"] / out["sector_start"][f"threads_{cores}_feet_per_s"]
    return out


def _time_steps(mesh, fld, dt, scheme, v, steps=20, warmup=3, **kw):
    """Kernel-inclusive ms per step (HIP events around `steps` steps on the
    current stream) and the statistics of one more step."""
    import torch
    out = torch.empty_like(v)
    for n in range(warmup):
        mesh.step(fld, n * dt, dt, scheme, v, out, **kw)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for n in range(steps):
        mesh.step(fld, n * dt, dt, scheme, v, out, **kw)
    e1.record(stream)
    torch.cuda.synchronize()
    _, st = mesh.step(fld, steps * dt, dt, scheme, v, out, stats=True, **kw)
    return e0.elapsed_time(e1) / steps, st


def measure_boundary(n=1001, alpha=5.0):
    """The variable step at the boundary and non-convex domains (n x n
    jittered grids, one FP64 field, Euler, Courant alpha, constant fields
    that carry feet out of the domain): ms per step with affine Dirichlet
    data (feet that leave take the datum at the first exit of their segment)
    and without (the outside value), on the square (convex: the walk's exit
    edge and the boundary loop decide), an L-shaped domain and a square with
    a hole (a walk blocked by the boundary ends in the exact quadtree search;
    exits are found by a scan of every boundary edge)."""
    import torch
    from paper_2104_09189_amd import inputs as I
    from paper_2104_09189_amd import slwalk as S
    ctx = S.Context(0)
    h = 1.0 / (n - 1)
    out = {"n": n, "alpha": alpha}
    cases = (("square", I.jittered_grid(n, 9101), I.constant(0.6, 0.3)),
             ("l_shaped", I.l_shaped(n, 9102), I.constant(-0.4, 0.4)),
             ("hole", I.square_with_hole(n, 9103), I.constant(-0.4, 0.0)))
    for name, (xy, tri), fld in cases:
        mesh = S.Mesh(ctx, xy, tri, S.INTERNAL_ORDER)
        v = torch.from_numpy(np.ascontiguousarray(I.gaussian_hill(xy)[mesh.dof_order()][:, None])).cuda()
        speed = max(abs(fld.p[0]), abs(fld.p[1]))
        dt = alpha * h / max(speed, 1e-9)
        line = {"n_nodes": int(mesh.n_nodes), "n_tris": int(mesh.n_tris), "nonconvex": bool(mesh.nonconvex),
                "boundary_loops": int(mesh.boundary_loops), "dt": dt}
        for bc in ("none", "affine"):
            if bc == "affine":
                mesh.set_boundary(S.BC_AFFINE, (0.7, -1.3, 2.1, 0.5))
            else:
                mesh.set_boundary(S.BC_NONE)
            ms, st = _time_steps(mesh, fld, dt, S.SLW_EULER, v)
            line[bc] = {"ms_per_step": ms, "feet_per_s": mesh.n_nodes / (ms * 1e-3),
                        "outside_share": st["outside"] / max(st["feet"], 1),
                        "mean_walk_steps": st["walk_steps"] / max(st["feet"], 1),
                        "exact_searches": st["boundary_searches"]}
        mesh.free()
        out[name] = line
    return out


def measure_p2(alpha=5.0):
    """P1 against P2 (eq. barycoords' quadratic Lagrange basis, vertex and
    edge-midpoint DOFs) on the 500 x 500 jittered mesh in Morton input order,
    swirl, Euler, Courant alpha, one FP64 field: ms per step, DOFs per second
    and the roofline fraction on each order's algorithmic bytes."""
    import torch
    from paper_2104_09189_amd import inputs as I
    from paper_2104_09189_amd import slwalk as S
    w = I.swirl_500(alpha=alpha, order="morton")
    ctx = S.Context(0)
    mesh = S.Mesh(ctx, w.xy, w.tri, S.INTERNAL_ORDER | S.P2)
    out = {"workload": w.name, "n_nodes": int(mesh.n_nodes), "n_dofs": int(mesh.n_dofs), "n_tris": int(mesh.n_tris)}
    for order, rows in ((1, mesh.n_nodes), (2, mesh.n_dofs)):
        v = torch.from_numpy(np.random.default_rng(7).normal(size=(rows, 1))).cuda()
        ms, st = _time_steps(mesh, w.field, w.dt, w.scheme, v, order=order)
        ab = algorithmic_bytes(rows, mesh.n_tris, 16, 8, 1, order)
        out[f"p{order}"] = {"ms_per_step": ms, "dofs_per_s": rows / (ms * 1e-3),
                            "roofline_frac": ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                            "mean_walk_steps": st["walk_steps"] / max(st["feet"], 1)}
    mesh.free()
    return out


def measure_locators(mesh, w, reps=10):
    """Point location alone on the feet of one step of the headline workload:
    the steered walk (strategy (a)), the walk from a bucket-grid start
    (slw_locate without starts), and the quadtree (no walk), all giving the
    same elements."""
    import torch
    from paper_2104_09189_amd import slwalk as S
    stream = torch.cuda.current_stream()
    feet = mesh.locate_feet(w.field, 8 * w.dt, w.dt, w.scheme, want_feet=True, want_bary=False)["feet"]
    info = None
    for cap in (16, 32, 64, 128):
        try:
            info = mesh.quadtree_build(cap, 24)
            info["leaf_cap"] = cap
            break
        except S.SlwError:
            continue
    out = {"points": int(feet.shape[0]), "quadtree": info}
    elems = {}

    def timed(name, fn):
        r = fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        out[name + "_ms"] = e0.elapsed_time(e1) / reps
        elems[name] = r.cpu().numpy()

    timed("walk_steered", lambda: mesh.locate_feet(feet=feet, feet_in=True, want_bary=False)["elem"])
    timed("walk_bucket_start", lambda: mesh.locate(feet, want_bary=False)[0])
    if info is not None:
        timed("quadtree", lambda: mesh.locate_quadtree(feet, want_bary=False)[0])
    # locate_feet reports user ids in DOF order; slw_locate in query order (the same here: internal order)
    out["identical"] = all(np.array_equal(elems["walk_steered"], v) for v in elems.values())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--alpha", type=float, default=5.0)
    ap.add_argument("--n", type=int, default=1415)
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--only-a", action="store_true", help="measure strategy (a) only")
    ap.add_argument("--only-b", action="store_true",
                    help="measure strategy (b) only (a short line, for hardware-counter runs)")
    ap.add_argument("--no-batch", action="store_true", help="skip the multi-mesh batch measurement")
    ap.add_argument("--only-batch", action="store_true",
                    help="measure the multi-mesh batch only (a short line, for hardware-counter runs)")
    ap.add_argument("--only-learned", action="store_true",
                    help="measure the learned start on the graded mesh only (training included; for traces)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-start measurement")
    ap.add_argument("--only-extra", action="store_true",
                    help="measure the boundary and P2 lines only")
    ap.add_argument("--only-decomp", action="store_true",
                    help="only the decomposition of the step's time (strategies (a) and (b), K fields and one)")
    ap.add_argument("--only-courant", action="store_true",
                    help="measure the Courant-range lines of the graded mesh only")
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
        print(json.dumps({"error": "this build runs on one GPU only; how the path would shard over several GPUs "
                                   "(replicated mesh, halo exchange of value rows) is a design, not an implementation",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2104_09189_amd import inputs as I
    from paper_2104_09189_amd import slwalk as S

    if args.only_batch:
        print(json.dumps({"batch": measure_batch()}), flush=True)
        return
    if args.only_learned:
        print(json.dumps({"learned": measure_learned()}), flush=True)
        return
    w = I.graded_swirl(alpha=args.alpha, n=args.n, k_fields=args.k)
    ctx = S.Context(0)
    t0 = time.perf_counter()
    mesh = S.Mesh(ctx, w.xy, w.tri, S.INTERNAL_ORDER)
    upload_s = time.perf_counter() - t0
    perm = mesh.dof_order()
    v0 = torch.from_numpy(np.ascontiguousarray(w.v0[perm])).to("cuda:0")
    n_feet = mesh.n_nodes

    if args.only_extra:
        print(json.dumps({"boundary": measure_boundary(), "p2": measure_p2()}), flush=True)
        return
    if args.only_courant:
        print(json.dumps({"courant_range": measure_courant_range(mesh, w, v0), "workload": w.name}), flush=True)
        return
    if args.only_decomp:
        print(json.dumps({"decomposition": measure_decomposition(mesh, w, v0), "workload": w.name}), flush=True)
        return
    if args.only_b:
        rb = measure(mesh, w, v0, args.steps, args.warmup, S.START_PREV)
        print(json.dumps({"strategy_b": {"ms_per_step": rb["ms_per_step"], "kernel_ms": rb["kernel_ms"],
                                         "mean_walk_steps": rb["stats"]["walk_steps"] / max(rb["stats"]["feet"], 1)},
                          "workload": w.name}), flush=True)
        return
    ra = measure(mesh, w, v0, args.steps, args.warmup, S.START_STEERED)
    value = n_feet / (ra["ms_per_step"] * 1e-3)
    abytes = algorithmic_bytes(n_feet, mesh.n_tris, 16, 4, args.k)
    achieved = abytes / (ra["kernel_ms"] * 1e-3) / 1e9
    traffic = measured_traffic() if (args.alpha == 5.0 and args.n == 1415 and args.k == 16) else None
    st = ra["stats"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "feet/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ra["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64/f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_nodes": int(n_feet), "n_tris": int(mesh.n_tris), "alpha": args.alpha,
                   "k_fields": args.k, "coords": "f64", "values": "f32", "order": 1, "scheme": "rk2",
                   "start": "strategy (a): incident triangle facing the foot", "parallelism": "none (1 GPU)"},
        "schedule": {"feet_per_lane": 1, "xcd_chunk": 64, "lds_window": 512,
                     "note": "library defaults: one foot per lane; chunks of 64 tiles of 256 nodes dealt to the "
                             "8 XCDs in turn; 512 walk records around each tile staged in LDS"},
        "field_values_per_s": value * args.k,
        "mean_walk_steps": st["walk_steps"] / max(st["feet"], 1),
        "walk": {**{k: st[k] for k in ("max_steps", "outside", "exact_tests", "fp64_tests", "fallback_walks",
                                       "edge_ties", "vertex_ties")},
                 "step_hist": hist_dict(st["step_hist"])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "k_step<false, float, 3, -7>",
                     "kernel_ms": ra["kernel_ms"], "algorithmic_bytes_per_launch": abytes},
        "upload_s": upload_s,
        "wall_s": ra["wall_s"],
    }
    if not args.only_a:
        rb = measure(mesh, w, v0, args.steps, args.warmup, S.START_PREV)
        stb = rb["stats"]
        out["strategy_b"] = {
            "start": "element found at the previous step", "value": n_feet / (rb["ms_per_step"] * 1e-3),
            "ms_per_step": rb["ms_per_step"], "kernel_ms": rb["kernel_ms"],
            "mean_walk_steps": stb["walk_steps"] / max(stb["feet"], 1),
            "roofline_frac": abytes / (rb["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
        for chain, key, desc in ((0, "strategy_c", "element found for the parent node, an adjacent root of a "
                                  "depth-one forest (when the parent is nearer than the node's own foot), else the "
                                  "steered start; roots first, two launches"),
                                 (2, "strategy_c_chain2", "element found for the preceding node of a 2-node Morton chain "
                                  "(nearer of it and the steered start)")):
            mesh.set_chain(chain)
            rc = measure(mesh, w, v0, args.steps, args.warmup, S.START_NEIGHBOR)
            stc = rc["stats"]
            out[key] = {
                "start": desc, "value": n_feet / (rc["ms_per_step"] * 1e-3), "ms_per_step": rc["ms_per_step"],
                "kernel_ms": rc["kernel_ms"], "mean_walk_steps": stc["walk_steps"] / max(stc["feet"], 1),
                "roofline_frac": abytes / (rc["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
        mesh.set_chain(0)
        out["courant_range"] = measure_courant_range(mesh, w, v0)
        out["k_field_reuse"] = measure_k_reuse(mesh, w, v0)
        out["decomposition"] = measure_decomposition(mesh, w, v0)
        out["locators"] = measure_locators(mesh, w)
        if not args.no_cpu:
            out["cpu_walk"] = measure_cpu_walk(w, out["locators"].get("walk_steered_ms"))
        out["precision"] = measure_precision()
        out["boundary"] = measure_boundary()
        out["p2"] = measure_p2()
    if not args.no_batch and not args.only_a:
        out["batch"] = measure_batch()
    if not args.no_learned and not args.only_a:
        out["learned"] = measure_learned()
        out["learned_uniform_mesh"] = measure_learned(w=I.swirl_500(alpha=20.0, order="morton"))
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
