"""Benchmark of the gfx950 2D Gaussian ray tracer.

Default workload (one step = the whole differentiable hot path once):
    1,000,000 surfels on a union of 8 spheres and 4 planes (F = 8 features),
    256 x 256 surface points x 64 cosine-weighted directions = 4,194,304 Monte
    Carlo rays; per step: LBVH refit of the current parameters, forward trace
    through the autograd wrapper, hand-written backward with N(0,1) upstream
    gradients on opacity, features and depth.
Prints ONE JSON line (value = whole-step Mrays/s, i.e. rays / (refit + fwd +
bwd)), with per-phase timings, the roofline of the dominant kernel measured
live with HIP events, and the FP64 oracle timed on the host for a bounded
sample of the same workload.

Other workloads (--workload): c2 (200K surfels, forward only), serve (three
resident scenes, Poisson request stream, packed launches vs one launch per
request), c5 (5M surfels, 33.5M rays, training-like step with perturbation
and refit).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def fwd_bytes(n_hits: np.ndarray, F: int) -> float:
    """Algorithmic bytes of a forward trace: per ray the ray (24 B), the
    outputs (4 (2 + F) B) and one surfel record (40 + 4F B) per composited
    hit."""
    R = n_hits.size
    return float(R * (24 + 4 * (2 + F)) + n_hits.astype(np.float64).sum() * (40 + 4 * F))


def bwd_bytes(n_hits: np.ndarray, F: int) -> float:
    """Algorithmic bytes of the backward: per ray the ray, the upstream
    gradients, the saved outputs, and per hit the surfel's parameters read and
    their gradient written."""
    R = n_hits.size
    return float(R * (24 + 4 * (2 + F) + 4 * (2 + F) + 4) + n_hits.astype(np.float64).sum() * 2 * (40 + 4 * F))


def cpu_baseline(sc, ro, rd, gO, gF, gD, budget_s: float = 12.0):
    """The FP64 oracle (brute-force forward + autograd gradient over its own
    hit lists) on a seeded sample of the rays, sized to about `budget_s`."""
    import oracle
    from oracle import grad as ograd
    threads = oracle.max_threads()
    g = np.random.default_rng(7)
    probe = np.sort(g.choice(ro.shape[0], 32, replace=False))
    t0 = time.perf_counter()
    oracle.trace(sc.astuple(), ro[probe], rd[probe], hit_cap=8)
    per_ray = (time.perf_counter() - t0) / probe.size
    n = int(max(64, min(65536, budget_s / max(per_ray, 1e-9))))
    idx = np.sort(g.choice(ro.shape[0], n, replace=False))
    t0 = time.perf_counter()
    r = oracle.trace(sc.astuple(), ro[idx], rd[idx], hit_cap=512)
    t1 = time.perf_counter()
    H = 512
    lists = np.where(np.arange(H)[None, :] < r["n_hits"][:, None], r["hits"], -1)
    lists = lists[:, :max(1, int(r["n_hits"].max()))]
    ograd.grad_given_hits(sc.astuple(), ro[idx], rd[idx], lists, gO[idx], gF[idx], gD[idx])
    t2 = time.perf_counter()
    return dict(value=round(n / (t2 - t0) / 1e6, 9), unit="Mrays/s", cores=int(threads), kind="oracle",
                sample=f"{n} of the {ro.shape[0]} rays (seeded), brute force over all {sc.n} surfels, FP64 "
                       f"forward {t1 - t0:.2f}s + autograd backward {t2 - t1:.2f}s",
                fwd_value=round(n / (t1 - t0) / 1e6, 9))


def gen_surface_workload(n_surfels, points, dirs, F=8):
    from paper_2412_15867_amd import synth
    lay = synth.layout()
    t0 = time.perf_counter()
    sc = synth.surface_scene(n_surfels, F=F, lay=lay)
    ro, rd = synth.mc_rays(points, dirs, lay=lay)
    log(f"generated {n_surfels} surfels, {ro.shape[0]} rays in {time.perf_counter() - t0:.1f}s")
    return sc, ro, rd


def run_c3(args):
    import torch
    from paper_2412_15867_amd import Scene, TraceConfig, TraceFn, synth, trace

    dev = torch.device("cuda:0")
    N = args.surfels
    sc, ro, rd = gen_surface_workload(N, args.points, args.dirs)
    R = ro.shape[0]
    F = sc.F
    gO, gF, gD, _ = synth.upstream(R, F)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    params = [t(a).requires_grad_(True) for a in sc.astuple()]
    ro_d, rd_d = t(ro), t(rd)
    gO_d, gF_d, gD_d = t(gO), t(gF), t(gD)
    torch.cuda.synchronize()
    b0 = time.perf_counter()
    scene = Scene(*[p.detach() for p in params])
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - b0) * 1e3
    scene.set_params(*params)
    info = scene.info()
    cfg = TraceConfig(k=args.k, recompute=args.recompute, hit_cap=args.hit_cap)
    log(f"built LBVH in {build_ms:.1f} ms, depth {info['max_depth']}; cfg {cfg}")

    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step(timed):
        for p in params:
            p.grad = None
        e = [ev() for _ in range(4)]
        e[0].record()
        scene.refit()
        e[1].record()
        O, Fo, D = TraceFn.apply(*params, ro_d, rd_d, scene, cfg)
        e[2].record()
        torch.autograd.backward([O, Fo, D], [gO_d, gF_d, gD_d])
        e[3].record()
        return e

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    events = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        events.append(step(True))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    refit_ms = np.array([e[0].elapsed_time(e[1]) for e in events])
    fwd_ms = np.array([e[1].elapsed_time(e[2]) for e in events])
    bwd_ms = np.array([e[2].elapsed_time(e[3]) for e in events])
    step_ms = wall * 1e3 / args.steps

    # hit statistics of this workload (the same forward, outputs kept)
    res = trace(scene, ro_d, rd_d, cfg, hit_cap=0)
    torch.cuda.synchronize()
    n_hits = res.n_hits.cpu().numpy()
    H = float(n_hits.mean())
    fb = fwd_bytes(n_hits, F)
    bb = bwd_bytes(n_hits, F)
    # pure forward kernel timing (no hit-list stores) for the forward-only rate
    fo = []
    for _ in range(3):
        a, b = ev(), ev()
        a.record()
        trace(scene, ro_d, rd_d, cfg, hit_cap=0, out=res)
        b.record()
        torch.cuda.synchronize()
        fo.append(a.elapsed_time(b))
    fwd_only_ms = float(np.median(fo))
    f_med, b_med = float(np.median(fwd_ms)), float(np.median(bwd_ms))
    dom_is_fwd = f_med >= b_med
    dom_ms = f_med if dom_is_fwd else b_med
    dom_bytes = fb if dom_is_fwd else bb
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    line = {
        "metric": "Mrays/s fwd+bwd @1M surfels (refit + forward + backward per step)",
        "value": round(R / (step_ms * 1e-3) / 1e6, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{N} surfels (8 spheres + 4 planes, F={F}), {args.points}x{args.dirs} "
                               f"cosine MC rays = {R}, refit+fwd+bwd, k={args.k}, T_min=1e-4, "
                               f"{'recompute' if args.recompute else 'store'} mode",
                   "surfels": N, "rays": R, "features": F, "k": args.k},
        "fwd_mrays_s": round(R / (fwd_only_ms * 1e-3) / 1e6, 3),
        "fwd_ms": round(fwd_only_ms, 3),
        "fwd_in_step_ms": round(f_med, 3),
        "bwd_ms": round(b_med, 3),
        "refit_ms": round(float(np.median(refit_ms)), 3),
        "build_ms": round(build_ms, 3),
        "hits_per_ray": round(H, 3),
        "bvh_depth": info["max_depth"],
        "roofline": {"bound": "hbm", "kernel": "k_trace (forward)" if dom_is_fwd else "k_backward",
                     "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                     "algorithmic_bytes_per_launch": dom_bytes, "launch_ms": round(dom_ms, 3)},
        "roofline_fwd": {"achieved": round(fb / (fwd_only_ms * 1e-3) / 1e9, 3), "bytes": fb},
    }
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a sample")
        line["cpu_baseline"] = cpu_baseline(sc, ro, rd, gO, gF, gD, budget_s=args.cpu_budget)
    scene.close()
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3", choices=["c3", "c2", "serve", "c5"])
    ap.add_argument("--surfels", type=int, default=1_000_000)
    ap.add_argument("--points", type=int, default=256 * 256)
    ap.add_argument("--dirs", type=int, default=64)
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--hit-cap", type=int, default=256)
    ap.add_argument("--recompute", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the trace shards rays across GPUs with no exchange in the "
              "forward and one gradient all-reduce in the backward, which this single-GPU build does not "
              "run; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c3":
        line = run_c3(args)
    else:
        from paper_2412_15867_amd import benchmarks
        line = benchmarks.run(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
