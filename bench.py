#!/usr/bin/env python3
"""Benchmark of the Walk-on-Spheres hot path on one MI355X.

Workload (d = 7, batched vs plain): the differentiated 7-D configuration
(1024 queries on 32 segments towards the goal, 256 sphere obstacles, sigma = 2,
16384 walks per query) plus every 7-D environment of the 512-environment
ragged batch (log-uniform 16-2048 spheres, log-uniform 1-4096 queries,
sigma ~ U[0.5, 8], 2048 walks per query).  One step = one fused forward +
backward pass over all of it in ONE persistent launch (the value); the plain
form runs one forward and one backward launch per environment on the same
walks (reported beside it).  Inputs are seeded synthetic scenes, resident in
device memory before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-plain] [--no-cpu]
                    [--no-plan] [--only-batched]

Prints one JSON line (rank 0).  Runs on one GPU only.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import multiprocessing as mp
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "WoS walk-steps/s + ∇u queries/s at fixed std error (d=7), batched vs plain"
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak (datasheet)
PEAK_FP32_MFMA_TFLOPS = 157.3  # MI355X dense FP32 matrix-core peak (datasheet)
JOB_CPU_SHARE = 16
# one FP32 FMA per lane per cycle: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP x
# 2.4 GHz; the datasheet figure counts packed FP32, which these kernels do
# not use
PEAK_FP32_UNPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
KERNEL_SOURCES = ["paper_2406_01713_amd/csrc/wos_device.hpp", "paper_2406_01713_amd/csrc/wos_kernels.hip",
                  "paper_2406_01713_amd/csrc/wos_params.hpp"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def distance_flops_per_step(s):
    """FP32 operations of one distance evaluation that scans every obstacle:
    per sphere (and the goal ball) d subtractions, d multiply-adds (2 flops),
    one subtraction of the radius and one min: 3d + 2; per box 5d + 1; the
    outer box 4d."""
    d = s["d"]
    ms = len(s["sph_r"]) + (1 if s.get("goal_r") is not None else 0)
    mb = len(s["box_h"])
    return ms * (3 * d + 2) + mb * (5 * d + 1) + 4 * d


def n_clusters(m):
    """Clusters of 8 that a domain with m obstacles of one kind keeps (none
    below 64 obstacles)."""
    return -(-m // 8) if m >= 64 else 0


MFMA_FLOP_PER_PAIR = 24  # 12 features x (multiply + add) per (walker, cluster) pair


def executed_flops(s, st):
    """Distance arithmetic that one env's walks actually executed, from the
    work columns of the batched stats (per-walk means of sphere and box
    member distances), split by the unit that runs it:
      valu  member spheres 3d + 2, member boxes 5d + 1, cluster bounding
            boxes 6d + 2 (per axis two differences, a three-way max, a
            multiply-add; a square root and the margin), the goal 3d + 2 and
            the outer box 4d per walk-step: the vector ALUs;
      mfma  the cluster test, 16 clusters per matrix-core tile, 12-term dot
            product per (walker, cluster) pair, for every cluster tile at
            every walk-step: v_mfma_f32_16x16x4f32 (FP32 matrix cores).
    Returns (valu, mfma, walk_steps)."""
    d, n = s["d"], s["n_walks"]
    steps = st[:, 9]
    goal = 1.0 if s.get("goal_r") is not None else 0.0
    valu = (st[:, 12] * (3 * d + 2) + st[:, 13] * (5 * d + 1) + st[:, 15] * (6 * d + 2)
            + steps * (goal * (3 * d + 2) + 4 * d)) * n
    tiles = -(-n_clusters(len(s["sph_r"])) // 16) + -(-n_clusters(len(s["box_h"])) // 16)
    mfma = steps * n * tiles * 16 * MFMA_FLOP_PER_PAIR
    return float(valu.sum()), float(mfma.sum()), float((steps * n).sum())


def timed(fn, reps, torch, st):
    """Mean and minimum milliseconds of reps calls of fn (HIP events on the
    launch stream around each call), after one untimed call."""
    fn()
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        fn()
        b.record(st)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    return float(np.mean(ms)), float(np.min(ms))


def workload():
    from paper_2406_01713_amd import scenes as S
    envs = [S.scene_c3()]
    envs[0]["env_id"] = 0
    envs += S.scene_c4(dims={7})
    return envs


# ----------------------------------------------------------- CPU baseline ----

def _oracle_slice(args):
    scene, qidx, n_walks, seed, env = args
    from oracle import oracle as O
    s = dict(scene)
    t = time.perf_counter()
    steps = 0.0
    dom = O.Domain(s)
    for q in qidx:
        for w in range(n_walks):
            r = O.walk(s, s["queries"][q], w, int(q), env=env, dom=dom)
            steps += r["steps"]
    return steps, time.perf_counter() - t


def cpu_baseline(envs, budget_walks=400000):
    """The FP64 oracle, untuned, on a bounded sample of the same workload: the
    same share of walks from every environment (walks 0..k-1 of every m-th
    query), one process per host core."""
    total = sum(len(e["queries"]) * e["n_walks"] for e in envs)
    frac = budget_walks / total
    tasks = []
    for e, s in enumerate(envs):
        Q = len(s["queries"])
        nw = max(1, int(round(s["n_walks"] * math.sqrt(frac))))
        nq = max(1, int(round(Q * frac * s["n_walks"] / nw)))
        qidx = np.linspace(0, Q - 1, min(nq, Q)).astype(int)
        tasks.append((s, qidx, nw, s["seed"], s.get("env_id", e)))
    # one process per CPU this job may use: the affinity set, at most the 16
    # CPU threads the GPU host grants a one-GPU job (os.cpu_count() there
    # counts the whole machine)
    host_cpus = os.cpu_count() or 1
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = host_cpus
    cores = max(1, min(usable, JOB_CPU_SHARE))
    # split the largest tasks so all cores stay busy
    chunks = []
    for s, qidx, nw, seed, env in tasks:
        for part in np.array_split(qidx, max(1, min(len(qidx), cores))):
            if len(part):
                chunks.append((s, part, nw, seed, env))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_slice, chunks, chunksize=1)
    wall = time.perf_counter() - t0
    steps = sum(r[0] for r in res)
    walks = sum(len(c[1]) * c[2] for c in chunks)
    cpu_model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": steps / wall, "unit": "walk-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{walks} walks ({walks / total:.2e} of the workload: the same walk ids from every "
                      f"environment), FP64 single-threaded oracle x {cores} processes, {wall:.1f} s wall",
            "per_core": steps / wall / cores, "cpu": cpu_model, "host_cpus": host_cpus,
            "affinity_cpus": usable,
            "cores_note": f"one process per usable CPU thread, at most {JOB_CPU_SHARE} (the CPU share a "
                          "one-GPU job gets on the GPU host)"}


# ------------------------------------------------------------------ GPU ----

class Batch:
    def __init__(self, B, envs, torch, mode=0, full_scan=False):
        from paper_2406_01713_amd import scenes as S
        self.B = B
        self.opt = B.options(full_scan=full_scan)
        self.envs = envs
        if mode == 2:
            envs = [S.with_bdata(e, 2, ak=S.plane_wave_k(e["d"], e["sigma"], seed=i))
                    for i, e in enumerate(envs)]
        elif mode == 3:
            # the paper's formulation: a unit impulse at the goal point, zero data
            envs = [S.with_source(e, e["goal_c"]) for e in envs]
        self.doms = [B.Domain(e) for e in envs]
        Qs = [len(e["queries"]) for e in envs]
        self.off = np.concatenate([[0], np.cumsum(Qs)]).astype(np.int64)
        n = int(self.off[-1])
        qp = np.zeros((n, 8), dtype=np.float32)
        for e, s in enumerate(envs):
            qp[self.off[e]:self.off[e + 1], :s["d"]] = s["queries"]
        dev = "cuda"
        self.q = torch.as_tensor(qp, device=dev)
        self.nw = np.array([e["n_walks"] for e in envs], dtype=np.int64)
        self.sig = [e["sigma"] for e in envs]
        self.eps = [e["eps"] for e in envs]
        self.u = torch.empty(n, device=dev)
        self.g = torch.empty(n, 8, device=dev)
        self.st = torch.empty(n, B.BATCH_STATS, dtype=torch.float64, device=dev)
        self.ubar = torch.ones(n, device=dev)
        self.dx = torch.empty(n, 8, device=dev)
        self.ds = torch.empty(len(envs), dtype=torch.float64, device=dev)
        self.dg = torch.empty(len(envs), dtype=torch.float64, device=dev)
        self.seed = envs[0]["seed"]

    def run(self, stats=True, bwd=True):
        """One persistent launch: fused forward + backward (u-bar = 1), or the
        forward pass only."""
        if bwd:
            self.B.wos_estimate_batch(self.doms, self.q, self.off, self.sig, self.eps, self.nw, self.seed,
                                      self.u, self.g, self.st if stats else None, self.ubar, self.dx,
                                      self.ds, self.dg, opt=self.opt)
        else:
            self.B.wos_estimate_batch(self.doms, self.q, self.off, self.sig, self.eps, self.nw, self.seed,
                                      self.u, self.g, self.st if stats else None, opt=self.opt)


class Plain:
    """One forward launch and one backward launch per environment (plain
    kernels, one walk per lane), same walk identities as the batch.  Inputs
    and outputs are allocated before timing."""

    def __init__(self, B, envs, doms, torch, seed, full_scan=False):
        self.B, self.envs, self.doms, self.seed = B, envs, doms, seed
        self.full_scan = full_scan
        self.bufs = []
        for s in envs:
            q = torch.as_tensor(s["queries"], dtype=torch.float32, device="cuda")
            Q, d = q.shape
            self.bufs.append(dict(q=q, u=torch.empty(Q, device="cuda"), g=torch.empty(Q, d, device="cuda"),
                                  ub=torch.ones(Q, device="cuda"), dx=torch.empty(Q, d, device="cuda"),
                                  ds=torch.empty(1, dtype=torch.float64, device="cuda"),
                                  dg=torch.empty(1, dtype=torch.float64, device="cuda")))

    def run(self, only=None, fwd=True, bwd=True):
        """Per env: the forward launch (u, grad u) and / or the backward launch
        (dx, d sigma, d g_goal: its kernel makes the forward sums too)."""
        B = self.B
        for e, (s, dom, b) in enumerate(zip(self.envs, self.doms, self.bufs)):
            if only is not None and e not in only:
                continue
            opt = B.options(False, e, 0, full_scan=self.full_scan)
            if fwd:
                B.wos_estimate(dom, b["q"], s["n_walks"], s["sigma"], s["eps"], self.seed, b["u"], b["g"], None,
                               opt=opt)
            if bwd:
                B.wos_backward(dom, b["q"], s["n_walks"], s["sigma"], s["eps"], self.seed, b["ub"], b["dx"],
                               b["ds"], b["dg"], None, opt=opt)
        return [b["u"] for b in self.bufs]


def max_rel_diff(outs, ub, off):
    """Largest relative difference of the plain u against the batched u."""
    diff = 0.0
    for e, u in enumerate(outs):
        a = u.cpu().numpy()
        b = ub[off[e]:off[e + 1]]
        if len(a):
            diff = max(diff, float(np.max(np.abs(a - b) / np.maximum(np.abs(a), 1e-6))))
    return diff


def launch_work(envs, off, stats):
    """(walk-steps, VALU FLOP, MFMA FLOP) of a batched launch's stats."""
    ws = valu = mfma = 0.0
    for e, s in enumerate(envs):
        v, m, w = executed_flops(s, stats[off[e]:off[e + 1]])
        ws += w
        valu += v
        mfma += m
    return ws, valu, mfma


def ragged_c4(B, torch, st, reps=3, plain_reps=2, tune_cache=None):
    """The full ragged batch (512 envs, d uniform in 2..7, 16-2048 spheres,
    1-4096 queries, sigma U[0.5, 8], 2048 walks): one persistent launch,
    forward only and fused forward + backward (u-bar = 1), against the plain
    per-env launches (one walk per lane, no refill) on the same walks."""
    from paper_2406_01713_amd import scenes as S
    t = time.perf_counter()
    envs = S.scene_c4()
    draw_s = time.perf_counter() - t
    bat = Batch(B, envs, torch)
    t = time.perf_counter()
    tune = B.wos_autotune_batch(bat.doms, bat.q, bat.off, bat.sig, bat.eps, bat.nw, bat.seed, fused=True,
                                cache_path=tune_cache)
    tune["search_s"] = time.perf_counter() - t
    fwd_ms, fwd_min = timed(lambda: bat.run(bwd=False), reps, torch, st)
    ws_f, valu_f, mfma_f = launch_work(envs, bat.off, bat.st.cpu().numpy())
    fused_ms, fused_min = timed(lambda: bat.run(), reps, torch, st)
    stats = bat.st.cpu().numpy()
    ws, valu, mfma = launch_work(envs, bat.off, stats)
    by_d = {}
    for d in range(2, 8):
        es = [e for e, s in enumerate(envs) if s["d"] == d]
        by_d[str(d)] = {"envs": len(es), "queries": int(sum(len(envs[e]["queries"]) for e in es)),
                        "walk_steps": float(sum(executed_flops(envs[e], stats[bat.off[e]:bat.off[e + 1]])[2]
                                                for e in es))}
    pl = Plain(B, envs, bat.doms, torch, bat.seed)
    pf_ms, _ = timed(lambda: pl.run(bwd=False), plain_reps, torch, st)
    pb_ms, _ = timed(lambda: pl.run(fwd=False), plain_reps, torch, st)
    diff = max_rel_diff(pl.run(bwd=False), bat.u.cpu().numpy(), bat.off)
    torch.cuda.synchronize()
    res = {"workload": "512 envs, d U{2..7}, 16-2048 spheres r U[0.05, 0.4], 1-4096 queries, sigma U[0.5, 8], "
                       "eps 1e-4, 2048 walks; one persistent launch",
           "envs": len(envs), "queries": int(bat.off[-1]), "walks": int(bat.off[-1]) * 2048,
           "walk_steps_per_step": ws, "by_d": by_d, "draw_s": draw_s, "repeats": reps,
           "forward": {"ms": fwd_ms, "ms_min": fwd_min, "walk_steps_per_s": ws_f / (fwd_ms / 1e3),
                       "valu_tflops": valu_f / (fwd_ms / 1e3) / 1e12, "mfma_tflops": mfma_f / (fwd_ms / 1e3) / 1e12},
           "fused_fwd_bwd": {"ms": fused_ms, "ms_min": fused_min, "walk_steps_per_s": ws / (fused_ms / 1e3),
                             "valu_tflops": valu / (fused_ms / 1e3) / 1e12,
                             "mfma_tflops": mfma / (fused_ms / 1e3) / 1e12},
           "plain": {"forward_ms": pf_ms, "backward_ms": pb_ms, "launches_per_pass": len(envs),
                     "forward_walk_steps_per_s": ws_f / (pf_ms / 1e3),
                     "fwd_plus_bwd_walk_steps_per_s": ws / ((pf_ms + pb_ms) / 1e3),
                     "repeats": plain_reps, "max_rel_diff_u_vs_batched": diff},
           "batched_vs_plain_forward": pf_ms / fwd_ms,
           "batched_vs_plain_fwd_plus_bwd": (pf_ms + pb_ms) / fused_ms,
           "batched_vs_plain_like_for_like": pb_ms / fused_ms,
           "autotune": dict(tune, gain_vs_default=tune["ms_default"] / fused_ms)}
    del pl, bat
    return res


def c2_forward(B, torch, st, reps=3):
    """The 6-D forward configuration: 4096 uniform free queries x 4096 walks,
    256 spheres, sigma = 4, eps = 1e-4, FP32 u and grad u; the plain launch
    and the persistent launch of the one environment."""
    from paper_2406_01713_amd import scenes as S
    s = S.scene_c2()
    dom = B.Domain(s)
    q = torch.as_tensor(s["queries"], dtype=torch.float32, device="cuda")
    Q, d = q.shape
    u = torch.empty(Q, device="cuda")
    g = torch.empty(Q, d, device="cuda")
    sto = torch.empty(Q, d + 4, dtype=torch.float64, device="cuda")

    def plain():
        B.wos_estimate(dom, q, s["n_walks"], s["sigma"], s["eps"], s["seed"], u, g, sto)

    p_ms, p_min = timed(plain, reps, torch, st)
    ws_plain = float((sto.cpu().numpy()[:, d + 1] * s["n_walks"]).sum())
    bat = Batch(B, [s], torch)
    b_ms, b_min = timed(lambda: bat.run(bwd=False), reps, torch, st)
    ws, valu, mfma = launch_work([s], bat.off, bat.st.cpu().numpy())
    assert abs(ws - ws_plain) <= 1e-9 * ws, (ws, ws_plain)  # the same walks
    res = {"workload": "d6: 4096 uniform free queries x 4096 walks, 256 spheres r U[0.1, 0.4], sigma 4, eps 1e-4, "
                       "FP32 forward u and grad u", "walk_steps_per_step": ws, "repeats": reps,
           "plain": {"ms": p_ms, "ms_min": p_min, "walk_steps_per_s": ws / (p_ms / 1e3)},
           "batched": {"ms": b_ms, "ms_min": b_min, "walk_steps_per_s": ws / (b_ms / 1e3),
                       "valu_tflops": valu / (b_ms / 1e3) / 1e12, "mfma_tflops": mfma / (b_ms / 1e3) / 1e12},
           "grad_queries_per_s": Q / (b_ms / 1e3),
           "max_rel_diff_u_vs_batched": max_rel_diff([u], bat.u.cpu().numpy(), bat.off)}
    del bat
    return res


def counter_entry(khash):
    """The committed counter summary of the d = 7 launch (HBM bytes per launch,
    VALU busy fraction), if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_persistent_d7.json")
    if not os.path.exists(path):
        return {}
    try:
        t = json.load(open(path))
    except (OSError, ValueError):
        return {}
    if t.get("kernel_hash") != khash:
        return {}
    return t


def near_goal_starts(s, n, seed=5):
    """Clear starts 0.05-0.5 outside the goal sphere (random directions)."""
    from paper_2406_01713_amd import scenes as S
    return S.near_goal_points(s, n, gap_lo=0.05, gap_hi=0.5, seed=seed, delta=0.02)


TUNE_CACHE = None  # --tune-cache: where the searches also record their shapes


def tune_plan(B, torch, dom, s, starts, n_walks, sigma=None):
    """The launch-shape search on a plan's own batch (its starts as the
    queries of one environment) before the plan is built: the shape is
    recorded under the batch's mix key, which the plan's captured launch
    looks up."""
    q = torch.zeros(len(starts), 8, dtype=torch.float32, device="cuda")
    q[:, :s["d"]] = torch.as_tensor(np.asarray(starts), dtype=torch.float32)
    sig = s["sigma"] if sigma is None else sigma
    # the fused launch of a batch needs d u / d sigma, which a point source
    # has only for sigma > 0: there the forward launch stands in
    fused = not (s.get("source") is not None and sig == 0.0)
    t = time.perf_counter()
    r = B.wos_autotune_batch([dom], q, [0, len(starts)], [sig], [s["eps"]], n_walks, s["seed"], fused=fused,
                             cache_path=TUNE_CACHE)
    r["fused"] = fused
    r["search_s"] = time.perf_counter() - t
    return r


def planning(B, torch, n_steps, near_goal=False, source=False, tune=True):
    from paper_2406_01713_amd import scenes as S
    s0 = S.scene_c5()
    starts = near_goal_starts(s0, len(s0["queries"])) if near_goal else s0["queries"]
    s = S.with_source(s0, s0["goal_c"]) if source else s0
    dom = B.Domain(s)
    shape = tune_plan(B, torch, dom, s, starts, s["n_walks"]) if tune else None
    x = torch.as_tensor(starts, dtype=torch.float32, device="cuda")
    plan = B.Plan(dom, x, s["n_walks"], s["sigma"], s["eps"], s["s_ub"], s["seed"])
    plan.step(1)
    plan.read()
    t0 = time.perf_counter()
    plan.step(n_steps - 1)
    u, g, pl, stalls, status, step = plan.read()
    dt = time.perf_counter() - t0
    res = {"starts": len(x), "start_set": "0.05-0.5 outside the goal sphere" if near_goal else "uniform free",
           "goal": "unit impulse at the goal point, zero data" if source else "goal ball, g = 1",
           "steps": int(step[0]), "ms_per_step": 1000 * dt / max(1, n_steps - 1),
           "walks_per_gradient": s["n_walks"], "obstacles": "512 spheres + 512 boxes",
           "arrived": int((status == 1).sum()), "stopped_elsewhere": int((status == 2).sum()),
           "stalls_total": int(stalls.sum()), "mean_path_len": float(pl.mean())}
    if shape is not None:
        res["autotune"] = shape
    del plan
    return res


def eval_env_sweep(B, torch, dims=(2, 3, 4, 5), ns=(10 ** 3, 10 ** 4, 10 ** 5, 10 ** 6), reps=32):
    """The paper's dimensionality study (Sec. VI): in the evaluation
    environment (k_r = 0.3, c = 1, eps = 0.01, unit impulse at the goal
    point (8, 0), free extra coordinates 0), the angle between the gradient
    estimated with n walks and a reference gradient from many more walks, at
    x_start,1 = (-8, 0) (behind the obstacle: few walks reach the source) and
    at (5, 3.5) (in view of the goal); reps independent estimates per n
    (distinct query indices of one launch draw independent walks), the share
    of them with any signal, and the time of one single-query estimate."""
    from paper_2406_01713_amd import scenes as S
    points = {"x_start_1": ((-8.0, 0.0), 10 ** 9), "in_view": ((5.0, 3.5), 10 ** 8)}
    out = {"k_r": 0.3, "sigma": 1.0, "eps": 0.01, "goal": "unit impulse at (8, 0, 0, ...)", "reps": reps,
           "points": {k: {"x": list(v[0]), "reference_walks": v[1]} for k, v in points.items()}, "by_d": {}}
    st = torch.cuda.current_stream()
    for d in dims:
        s = S.scene_eval_env(d, k_r=0.3, sigma=1.0, eps=1e-2)
        dom = B.Domain(s)
        rd = {}
        for name, (p2, n_ref) in points.items():
            xp = np.zeros((1, d))
            xp[0, :2] = p2
            x = torch.as_tensor(xp, dtype=torch.float32, device="cuda")
            u1 = torch.empty(1, device="cuda")
            g1 = torch.empty(1, d, device="cuda")
            t = time.perf_counter()
            B.wos_estimate(dom, x, n_ref, s["sigma"], s["eps"], 987654321, u1, g1)
            torch.cuda.synchronize()
            t_ref = time.perf_counter() - t
            gt = g1.cpu().numpy()[0].astype(np.float64)
            xr = x.repeat(reps, 1).contiguous()
            ur = torch.empty(reps, device="cuda")
            gr = torch.empty(reps, d, device="cuda")
            err, sig, ms = {}, {}, {}
            for n in ns:
                B.wos_estimate(dom, xr, n, s["sigma"], s["eps"], 1, ur, gr)
                ge = gr.cpu().numpy().astype(np.float64)
                nz = np.linalg.norm(ge, axis=1) > 0
                cosv = (ge @ gt) / np.maximum(np.linalg.norm(ge, axis=1) * np.linalg.norm(gt), 1e-300)
                ang = np.degrees(np.arccos(np.clip(cosv, -1.0, 1.0)))
                ang[~nz] = 90.0  # no walk reached the source: no direction
                err[str(n)] = float(ang.mean())
                sig[str(n)] = float(nz.mean())
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                B.wos_estimate(dom, x, n, s["sigma"], s["eps"], 2, u1, g1)
                e0.record(st)
                for _ in range(5):
                    B.wos_estimate(dom, x, n, s["sigma"], s["eps"], 2, u1, g1)
                e1.record(st)
                torch.cuda.synchronize()
                ms[str(n)] = e0.elapsed_time(e1) / 5
            lx = np.log10(np.array(ns, dtype=np.float64))
            ly = np.log10(np.array([err[str(n)] for n in ns]))
            rd[name] = {"mean_angle_error_deg": err, "share_with_signal": sig, "ms_per_estimate": ms,
                        "log_log_slope": float(np.polyfit(lx, ly, 1)[0]),
                        "reference_grad_nonzero": bool(np.linalg.norm(gt) > 0), "reference_s": t_ref}
            log(f"eval env d={d} {name}: angle error (deg) "
                + ", ".join(f"n={n}: {err[str(n)]:.2f}" for n in ns)
                + f"; signal {sig[str(ns[0])]:.2f}..{sig[str(ns[-1])]:.2f}; reference {t_ref:.1f} s")
        out["by_d"][str(d)] = rd
    return out


def rr_validation(B, torch, n_walks=100000, max_steps=300, tune=True):
    """The RR task of Sec. VII (Table II): gradient ascent from q_start to a
    unit impulse at q_goal, 1e5 walks per gradient, s = min(0.1, d/2),
    eps = 0.02, c = 0 and 5, with the IK-point distance (N_col = 200) and the
    Lipschitz arm bound.  Link lengths and joint lower bounds are not in the
    paper (unit links, joints spanning 2 pi), so its path lengths are context,
    not a target."""
    from paper_2406_01713_amd import scenes as S
    out = {"n_walks": n_walks, "s_ub": 0.1, "eps": 0.02, "links": list(S.RR_LINKS),
           "q_start": list(S.RR_Q_START), "q_goal": list(S.RR_Q_GOAL),
           "paper_path_lengths": {"c=0": 4.5, "c=5": 3.8}, "runs": {}}
    st = torch.cuda.current_stream()
    for distance in ("ik", "lipschitz"):
        for sigma in (0.0, 5.0):
            s = S.scene_rr(distance, sigma=sigma, n_walks=n_walks)
            dom = B.Domain(s)
            shape = tune_plan(B, torch, dom, s, [S.RR_Q_START], n_walks) if tune else None
            x = torch.as_tensor(np.array([S.RR_Q_START]), dtype=torch.float32, device="cuda")
            plan = B.Plan(dom, x, n_walks, s["sigma"], s["eps"], s["s_ub"], s["seed"])
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            steps = 0
            status = 0
            while steps < max_steps:
                plan.step(10)
                steps += 10
                r = plan.read()
                status = int(r[4][0])
                if status != 0:
                    break
            e1.record(st)
            torch.cuda.synchronize()
            u, g, path, stalls, sts, step = plan.read()
            out["runs"][f"{distance}_c{sigma:g}"] = {
                "path_length": float(path[0]), "arrived": int(sts[0]) == 1, "plan_steps": int(step[0]),
                "stalls": int(stalls[0]), "ms_per_plan_step": e0.elapsed_time(e1) / max(int(step[0]), 1),
                "end": [float(v) for v in x.cpu().numpy()[0]]}
            if shape is not None:
                out["runs"][f"{distance}_c{sigma:g}"]["autotune"] = shape
            del plan
            log(f"RR {distance} c={sigma:g}: path {float(path[0]):.3f}, arrived {int(sts[0]) == 1}, "
                f"{int(step[0])} steps")
    return out


def eval_env_paths(B, torch, sigmas=(0.1, 1.0, 10.0), n_walks=100000, max_steps=600, tune=True):
    """Screening and path length in the evaluation environment (Sec. VI-A,
    d = 2, k_r = 0.3, eps = 0.01): gradient ascent from x_start,1 = (-8, 0)
    to the unit impulse at (8, 0) with 1e5 walks per gradient and
    s = min(0.1, d/2), for c = 0.1, 1 and 10.  At c = 10 every walk that
    reaches the source from 16 units away weighs below FP32's range (each step
    multiplies the weight by 1 / I_0(sqrt(c) R)); the FP32 walk keeps the
    weight's exponent apart and the planning graph steps along the direction
    formed from the FP64 sums, so this run moves as the others do."""
    from paper_2406_01713_amd import scenes as S
    out = {"start": [-8.0, 0.0], "goal": [8.0, 0.0], "n_walks": n_walks, "s_ub": 0.1, "runs": {}}
    for c in sigmas:
        s = S.scene_eval_env(2, k_r=0.3, sigma=c, eps=1e-2)
        dom = B.Domain(s)
        shape = tune_plan(B, torch, dom, s, s["queries"][:1], n_walks, sigma=c) if tune else None
        x = torch.as_tensor(s["queries"][:1], dtype=torch.float32, device="cuda")
        plan = B.Plan(dom, x, n_walks, c, s["eps"], 0.1, s["seed"])
        steps = 0
        while steps < max_steps:
            plan.step(20)
            steps += 20
            if int(plan.read()[4][0]) != 0:
                break
        u, g, path, stalls, sts, step = plan.read()
        out["runs"][f"c={c:g}"] = {"path_length": float(path[0]), "arrived": int(sts[0]) == 1,
                                   "plan_steps": int(step[0]), "stalls": int(stalls[0]),
                                   "end": [float(v) for v in x.cpu().numpy()[0]]}
        if shape is not None:
            out["runs"][f"c={c:g}"]["autotune"] = shape
        del plan
        log(f"eval env path c={c:g}: length {float(path[0]):.2f}, arrived {int(sts[0]) == 1}, "
            f"stalls {int(stalls[0])}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--plain-reps", type=int, default=3, help="timed repeats of the plain per-env path")
    ap.add_argument("--no-c4", action="store_true", help="skip the full ragged batch and the 6-D forward set")
    ap.add_argument("--no-tune", action="store_true", help="time the built-in launch shape (no autotune search)")
    ap.add_argument("--tune-cache", default=None, help="also write the searched launch shapes to this JSON file")
    ap.add_argument("--load-tune", default=None, help="use the launch shapes of this JSON file (no search)")
    ap.add_argument("--full-scan", action="store_true",
                    help="scan every obstacle each step (no cluster culling): same results, more work")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plan", action="store_true")
    ap.add_argument("--no-se", action="store_true")
    ap.add_argument("--no-source", action="store_true", help="skip the point-source workload")
    ap.add_argument("--no-eval-env", action="store_true",
                    help="skip the evaluation-environment dimension sweep")
    ap.add_argument("--only-batched", action="store_true", help="time the batched step only (profiling)")
    ap.add_argument("--plan-steps", type=int, default=200)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device 3 times (counter calibration)")
    args = ap.parse_args()
    global TUNE_CACHE
    TUNE_CACHE = args.tune_cache
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one MI355X: the walk kernels run on a single GPU "
              "(walk ranges and queries would shard across GPUs with one all-reduce of partial sums; not run here). "
              "Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.only_batched:
        args.no_plain = args.no_cpu = args.no_plan = args.no_se = args.no_source = args.no_eval_env = True
        args.no_c4 = True

    t = time.perf_counter()
    envs = workload()
    log(f"workload: {len(envs)} envs, {sum(len(e['queries']) for e in envs)} queries "
        f"({time.perf_counter() - t:.1f} s to draw)")
    cpu = None
    if not args.no_cpu:
        # before the GPU is initialised: the oracle pool forks this process
        t = time.perf_counter()
        cpu = cpu_baseline(envs)
        log(f"cpu baseline: {cpu['value']:.3g} walk-steps/s ({time.perf_counter() - t:.1f} s)")

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2406_01713_amd import binding as B

    bat = Batch(B, envs, torch, full_scan=args.full_scan)
    st = torch.cuda.current_stream()
    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mib} MiB x 3")

    tune = None
    if args.load_tune:
        # a shape chosen by an earlier search (e.g. for a profiled run)
        B.wos_set_autotune_cache(args.load_tune)
        log(f"launch shapes loaded from {args.load_tune}")
    elif not args.no_tune:
        # launch shape searched on this batch (fused fwd + bwd); the timed
        # launches below use it (the library keeps it for this batch mix)
        t = time.perf_counter()
        tune = B.wos_autotune_batch(bat.doms, bat.q, bat.off, bat.sig, bat.eps, bat.nw, bat.seed, fused=True,
                                    cache_path=args.tune_cache)
        tune["search_s"] = time.perf_counter() - t
        log(f"autotune: {tune}")
    for _ in range(args.warmup):
        bat.run()
    torch.cuda.synchronize()
    log("warm-up done")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(st)
    for i in range(args.steps):
        evs[i][0].record(st)
        bat.run()
        evs[i][1].record(st)
    t_end.record(st)
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps
    launch_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    log(f"batched fused fwd+bwd: {ms_step:.1f} ms/step")

    stats = bat.st.cpu().numpy()
    walk_steps, valu, mfma = launch_work(envs, bat.off, stats)
    flops_full = sum(float((stats[bat.off[e]:bat.off[e + 1], 9] * s["n_walks"]).sum()) * distance_flops_per_step(s)
                     for e, s in enumerate(envs))
    value = walk_steps / (ms_step / 1e3)
    valu_rate = valu / (launch_ms / 1e3) / 1e12
    mfma_rate = mfma / (launch_ms / 1e3) / 1e12
    khash = kernel_hash()
    counters = counter_entry(khash)
    ceilings = {}
    try:
        fma, _ = B.wos_microbench(0)
        sq, _ = B.wos_microbench(1)
        sph, _ = B.wos_microbench(2)
        ceilings = {"fma_tflops": fma / 1e12, "sqrt_per_s": sq, "sphere_evals_d7_per_s": sph,
                    "sphere_loop_d7_tflops": sph * 23 / 1e12,
                    "note": "wos_microbench: independent v_fma_f32 chains; v_sqrt_f32 chains; the "
                            "7-D sphere-distance loop (23 algorithmic FLOP per sphere)"}
    except B.WosError as exc:  # reported, not fatal
        log(f"microbench failed: {exc}")

    out = {"metric": METRIC, "value": value, "unit": "walk-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "d7 fused fwd+bwd, one persistent launch: 7-D segment queries "
                                  "(1024 q x 16384 walks, 256 spheres, sigma 2) + the 83 7-D envs of the "
                                  "512-env ragged batch (41660 q x 2048 walks, 16-2048 spheres)",
                      "envs": len(envs), "queries": int(bat.off[-1]),
                      "walks": int(sum(len(e["queries"]) * e["n_walks"] for e in envs)),
                      "walk_steps_per_step": walk_steps, "eps": 1e-4, "seed": int(bat.seed),
                      "obstacle_scan": "every obstacle" if args.full_scan else
                                       "cluster-culled (exact: same walks as a full scan)"},
           "roofline": {"bound": "alu", "achieved": valu_rate, "peak": PEAK_FP32_TFLOPS,
                        "unit": "TFLOP/s", "frac": valu_rate / PEAK_FP32_TFLOPS,
                        "traffic": counters.get("bytes_per_launch"),
                        "basis": "distance arithmetic executed on the vector ALUs: member sphere (3d + 2) and "
                                 "box (5d + 1) distances, cluster bounding-box tests (6d + 2) of the pairs the "
                                 "matrix-core test keeps, the goal (3d + 2) and the outer box (4d) per "
                                 "walk-step, counted by the kernel's work tallies; the cluster test runs on the "
                                 "matrix cores and is reported under 'mfma'",
                        "mfma": {"achieved": mfma_rate, "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                                 "frac": mfma_rate / PEAK_FP32_MFMA_TFLOPS, "flops_per_launch": mfma,
                                 "basis": "cluster tests (12-term dot product, 24 FLOP per walker and cluster) "
                                          "for every 16-cluster tile at every walk-step, "
                                          "v_mfma_f32_16x16x4f32; peak = MI355X dense FP32 matrix peak"},
                        "valu_busy": counters.get("valu_busy"),
                        "valu_busy_basis": "share of cycles the vector ALUs issue (SQ_ACTIVE_INST_VALU, "
                                           "rocprofv3 on these kernel sources)",
                        "frac_unpacked": valu_rate / PEAK_FP32_UNPACKED_TFLOPS,
                        "unpacked_peak": PEAK_FP32_UNPACKED_TFLOPS,
                        "unpacked_peak_basis": "256 CUs x 4 SIMDs x 16 lanes x 1 FP32 FMA (2 FLOP) per cycle "
                                               "x 2.4 GHz; the kernels are built without packed FP32",
                        "kernel": "persistent_kernel<fused fwd+bwd>",
                        "launch_ms": launch_ms,
                        "valu_flops_per_launch": valu,
                        "full_scan_flops_per_launch": flops_full,
                        "work_fraction": valu / flops_full,
                        "work_fraction_basis": "VALU distance FLOP executed / the FLOP of a scan of every "
                                               "obstacle at every walk-step (exact culling: same walks)",
                        "peak_basis": "MI355X FP32 vector peak, 157.3 TFLOP/s (datasheet); measured ceilings "
                                      "of this code's instruction types in 'measured'",
                        "measured": ceilings,
                        "kernel_hash": khash}}
    if tune is not None:
        out["autotune"] = dict(tune, basis="wos_autotune_batch on this batch before timing: coordinate descent "
                                            "over waves per block, units per wave, grid multiple, walks per lane, then lanes "
                                            "per walker G doubled (then halved) while faster; ms_default = one "
                                            "launch with the built-in shape (4, 4, 1, 2, G = 1)",
                               gain_vs_default=tune["ms_default"] / ms_step)

    if not args.no_plain:
        t = time.perf_counter()
        pl = Plain(B, envs, bat.doms, torch, bat.seed, full_scan=args.full_scan)
        plain_ms, plain_min = timed(lambda: pl.run(), args.plain_reps, torch, st)
        bwd_ms, bwd_min = timed(lambda: pl.run(fwd=False), args.plain_reps, torch, st)
        diff = max_rel_diff(pl.run(bwd=False), bat.u.cpu().numpy(), bat.off)
        out["plain"] = {"ms_per_step": plain_ms, "ms_min": plain_min, "repeats": args.plain_reps,
                        "walk_steps_per_s": walk_steps / (plain_ms / 1e3), "launches": 2 * len(envs),
                        "backward_only_ms": bwd_ms, "backward_only_ms_min": bwd_min,
                        "max_rel_diff_u_vs_batched": diff,
                        "note": "plain = a forward launch and a backward launch per env, one walk per lane; "
                                "the backward kernel alone makes the sums of the fused launch (u, grad u, "
                                "d sigma, d g_goal), so backward_only is the like-for-like comparison"}
        out["batched_vs_plain"] = plain_ms / ms_step
        out["batched_vs_plain_like_for_like"] = bwd_ms / ms_step
        log(f"plain fwd+bwd per env: {plain_ms:.1f} ms (backward alone {bwd_ms:.1f} ms), batched speed-up "
            f"{plain_ms / ms_step:.2f}x, like for like {bwd_ms / ms_step:.2f}x ({time.perf_counter() - t:.1f} s)")

    if not args.no_c4:
        t = time.perf_counter()
        out["ragged_c4"] = ragged_c4(B, torch, st, tune_cache=args.tune_cache)
        r = out["ragged_c4"]
        log(f"ragged C4: fused {r['fused_fwd_bwd']['ms']:.1f} ms ({r['fused_fwd_bwd']['walk_steps_per_s']:.3e} "
            f"walk-steps/s), forward {r['forward']['ms']:.1f} ms; plain fwd {r['plain']['forward_ms']:.1f} ms, "
            f"bwd {r['plain']['backward_ms']:.1f} ms ({time.perf_counter() - t:.1f} s)")
        t = time.perf_counter()
        out["c2_d6_forward"] = c2_forward(B, torch, st)
        r = out["c2_d6_forward"]
        log(f"C2 d6 forward: plain {r['plain']['ms']:.1f} ms, batched {r['batched']['ms']:.1f} ms "
            f"({time.perf_counter() - t:.1f} s)")

    if not args.no_se:
        # standard errors measured with plane-wave data (u = exp(k.x)) on the
        # same geometry and walks: n* = n (SE_grad / (0.01 |grad u|))^2
        pw = Batch(B, envs, torch, mode=2)
        pw.run()
        torch.cuda.synchronize()
        g = pw.g.cpu().numpy().astype(np.float64)
        sst = pw.st.cpu().numpy()
        need = 0.0
        have = 0.0
        zero_hit = 0
        for e, s in enumerate(envs):
            sl = slice(pw.off[e], pw.off[e + 1])
            gn = np.linalg.norm(g[sl, :s["d"]], axis=1)
            se = np.linalg.norm(sst[sl, 1:1 + s["d"]], axis=1)
            n = s["n_walks"]
            ok = gn > 0
            need += float(np.sum(n * (se[ok] / (0.01 * gn[ok])) ** 2))
            have += float(ok.sum() * n)
        u_goal = stats[:, 0]
        zero_hit = int(np.sum(bat.u.cpu().numpy() == 0))
        q_total = int(bat.off[-1])
        out["grad_queries_per_s_at_1pct_se"] = q_total / (ms_step / 1e3 * need / max(have, 1.0))
        out["se_note"] = ("SE from plane-wave boundary data on the same geometry and walks; "
                          f"with goal-indicator data {zero_hit}/{q_total} queries see no goal hit")

    if not args.no_source:
        # the same queries with the paper's point-source formulation (unit
        # impulse at each env's goal point, zero boundary data, goal ball
        # removed), fused forward + backward, one persistent launch
        t = time.perf_counter()
        ps = Batch(B, envs, torch, mode=3)
        ps.run()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(2):
            ps.run()
        e1.record(st)
        torch.cuda.synchronize()
        ps_ms = e0.elapsed_time(e1) / 2
        pst = ps.st.cpu().numpy()
        pu = ps.u.cpu().numpy()
        pg = ps.g.cpu().numpy().astype(np.float64)
        ws = sum(float((pst[ps.off[e]:ps.off[e + 1], 9] * s["n_walks"]).sum()) for e, s in enumerate(envs))
        need = have = 0.0
        for e, s in enumerate(envs):
            sl = slice(ps.off[e], ps.off[e + 1])
            gn = np.linalg.norm(pg[sl, :s["d"]], axis=1)
            se = np.linalg.norm(pst[sl, 1:1 + s["d"]], axis=1)
            ok = gn > 0
            need += float(np.sum(s["n_walks"] * (se[ok] / (0.01 * gn[ok])) ** 2))
            have += float(ok.sum() * s["n_walks"])
        q_total = int(ps.off[-1])
        out["point_source_d7"] = {
            "workload": "the same 84 envs and queries; unit impulse at each env's goal point, zero boundary "
                        "data, goal ball removed; fused fwd+bwd, one persistent launch",
            "ms_per_step": ps_ms, "walk_steps_per_s": ws / (ps_ms / 1e3), "walk_steps_per_step": ws,
            "queries_with_signal": int((pu > 0).sum()), "queries": q_total,
            "grad_queries_per_s_at_1pct_se": q_total / (ps_ms / 1e3 * need / max(have, 1.0)),
            "se_note": "d = 7: the point-source estimator has infinite variance (contributions grow like "
                       "r^(2-d) near the source), so sample SEs understate the error"}
        log(f"point source: {ps_ms:.1f} ms/step, {ws / (ps_ms / 1e3):.3e} walk-steps/s, "
            f"{int((pu > 0).sum())}/{q_total} queries with signal ({time.perf_counter() - t:.1f} s)")
        del ps

    if not args.no_plan:
        t = time.perf_counter()
        tune_p = not (args.no_tune or args.load_tune)
        out["planning_d7"] = planning(B, torch, args.plan_steps, tune=tune_p)
        out["planning_d7_near_goal"] = planning(B, torch, args.plan_steps, near_goal=True, tune=tune_p)
        log(f"planning: {out['planning_d7']['ms_per_step']:.1f} ms/step; near goal "
            f"{out['planning_d7_near_goal']['ms_per_step']:.1f} ms/step, "
            f"{out['planning_d7_near_goal']['arrived']} arrived ({time.perf_counter() - t:.1f} s)")
        if not args.no_source:
            t = time.perf_counter()
            out["planning_d7_point_source"] = planning(B, torch, args.plan_steps, source=True, tune=tune_p)
            out["planning_d7_point_source_near_goal"] = planning(B, torch, args.plan_steps, near_goal=True,
                                                                 source=True, tune=tune_p)
            log(f"planning to a point source: {out['planning_d7_point_source']['arrived']} / "
                f"{out['planning_d7_point_source_near_goal']['arrived']} arrived "
                f"({time.perf_counter() - t:.1f} s)")

    if not args.no_plan:
        t = time.perf_counter()
        out["rr_validation"] = rr_validation(B, torch, tune=not (args.no_tune or args.load_tune))
        out["eval_env_paths"] = eval_env_paths(B, torch, tune=not (args.no_tune or args.load_tune))
        log(f"RR validation and evaluation-environment paths ({time.perf_counter() - t:.1f} s)")

    if not args.no_eval_env:
        t = time.perf_counter()
        out["eval_env_dim_sweep"] = eval_env_sweep(B, torch)
        log(f"evaluation-environment sweep ({time.perf_counter() - t:.1f} s)")

    if cpu is not None:
        out["cpu_baseline"] = cpu

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
