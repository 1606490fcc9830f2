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

Other workloads (--workload): pbr (the rendering-equation step: 1,024
pixels x 256 stratified directions on the 1M-surfel scene, SH colour, cubemap
sky, refit + trace + shading + backward), relight (the same pixels on
albedo / roughness surfels: trace with the blended normal, split-sum indirect
light, Eq. 15; the sky precompute timed apart), c1 (4,096-surfel cube, 64x64 camera rays) and
c2 (200K surfels, 4.2M MC rays), forward only against the brute-force GPU
tracer; serve (three
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
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "k_trace_traffic_1M_surfels_4M_rays.md")
CSRC = os.path.join(ROOT, "paper_2412_15867_amd", "csrc")
FWD_SOURCES = ("trace_fwd.hip", "trace_flat.hpp", "march.hpp", "irgs_device.hpp", "irgs_internal.hpp", "lbvh.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def forward_fingerprint() -> str:
    """Hash of the forward kernel's sources: measured traffic is reported
    only while the kernel is the one the counters were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in FWD_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_l2_hit_rate():
    """L2 hit rate (TCC_HIT / (TCC_HIT + TCC_MISS)) of the same in-step
    forward launch from the committed rocprofv3 summary, or None (missing,
    or taken on other kernel sources)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = next(json.loads(ln[len("traffic-data: "):]) for ln in fh if ln.startswith("traffic-data: "))
    except (OSError, StopIteration):
        return None
    if d.get("kernel_fingerprint") != forward_fingerprint() or "tcc_hit" not in d:
        return None
    return round(d["tcc_hit"] / max(d["tcc_hit"] + d["tcc_miss"], 1.0), 4)


def measured_traffic():
    """HBM-side bytes of one in-step forward launch from the committed
    rocprofv3 summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the
    same counter reads for a device copy of known size), or None when the
    summary is missing or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            for ln in fh:
                if ln.startswith("traffic-data: "):
                    d = json.loads(ln[len("traffic-data: "):])
                    break
            else:
                return None
    except OSError:
        return None
    if d.get("kernel_fingerprint") != forward_fingerprint():
        return None
    rd_scale = d["copy_bytes"] / (d["copy_fetch_kib"] * 1024.0)
    wr_scale = d["copy_bytes"] / (d["copy_write_kib"] * 1024.0)
    return round(d["fetch_kib"] * 1024.0 * rd_scale + d["write_kib"] * 1024.0 * wr_scale)


def calibration_copy(nbytes: int = 512 << 20, reps: int = 3):
    """A plain device-to-device copy of known size, for scaling the
    FETCH_SIZE / WRITE_SIZE counters of a profiled run."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"calibration copy: {reps} x {nbytes} bytes")


def fwd_bytes(n_hits: np.ndarray, F: int, FO: int | None = None) -> float:
    """Algorithmic bytes of a forward trace: per ray the ray (24 B), the
    outputs (4 (2 + FO) B, FO composited channels) and one surfel record
    (40 + 4F B) per composited hit."""
    FO = F if FO is None else FO
    R = n_hits.size
    return float(R * (24 + 4 * (2 + FO)) + n_hits.astype(np.float64).sum() * (40 + 4 * F))


def bwd_bytes(n_hits: np.ndarray, F: int, FO: int | None = None) -> float:
    """Algorithmic bytes of the backward: per ray the ray, the upstream
    gradients, the saved outputs, and per hit the surfel's parameters read and
    their gradient written."""
    FO = F if FO is None else FO
    R = n_hits.size
    return float(R * (24 + 4 * (2 + FO) + 4 * (2 + FO) + 4) + n_hits.astype(np.float64).sum() * 2 * (40 + 4 * F))


def cpu_baseline(sc, ro, rd, gO, gF, gD, budget_s: float = 12.0, sh_deg: int = -1):
    """The FP64 oracle (brute-force forward + autograd gradient over its own
    hit lists) on a seeded sample of the rays, sized to about `budget_s`."""
    import oracle
    from oracle import grad as ograd
    threads = oracle.max_threads()
    g = np.random.default_rng(7)
    # per-ray cost from two probe sizes (each call also pays a fixed per-surfel setup)
    tp = []
    for m in (64, 320):
        probe = np.sort(g.choice(ro.shape[0], m, replace=False))
        t0 = time.perf_counter()
        oracle.trace(sc.astuple(), ro[probe], rd[probe], hit_cap=8, sh_deg=sh_deg)
        tp.append(time.perf_counter() - t0)
    per_ray = max((tp[1] - tp[0]) / 256, 1e-9)
    n = int(max(256, min(65536, budget_s / per_ray)))
    idx = np.sort(g.choice(ro.shape[0], n, replace=False))
    t0 = time.perf_counter()
    r = oracle.trace(sc.astuple(), ro[idx], rd[idx], hit_cap=512, sh_deg=sh_deg)
    t1 = time.perf_counter()
    H = 512
    lists = np.where(np.arange(H)[None, :] < r["n_hits"][:, None], r["hits"], -1)
    lists = lists[:, :max(1, int(r["n_hits"].max()))]
    ograd.grad_given_hits(sc.astuple(), ro[idx], rd[idx], lists, gO[idx], gF[idx], gD[idx], sh_deg=sh_deg)
    t2 = time.perf_counter()
    return dict(value=round(n / (t2 - t0) / 1e6, 9), unit="Mrays/s", cores=int(threads), cpu_model=cpu_model(),
                kind="oracle",
                sample=f"{n} of the {ro.shape[0]} rays (seeded), brute force over all {sc.n} surfels, FP64 "
                       f"forward {t1 - t0:.2f}s + autograd backward {t2 - t1:.2f}s",
                fwd_value=round(n / (t1 - t0) / 1e6, 9))


def cpu_model() -> str:
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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
    sh = args.sh_deg >= 0
    if sh:  # view-dependent colour: RGB SH coefficients instead of the plain features
        sc = synth.Surfels(sc.mu, sc.quat, sc.scale, sc.opac, synth.sh_coefficients(N, args.sh_deg))
    R = ro.shape[0]
    F = sc.F
    FO = 3 if sh else F
    gO, gF, gD, _ = synth.upstream(R, FO)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    params = [t(a).requires_grad_(True) for a in sc.astuple()]
    ro_d, rd_d = t(ro), t(rd)
    gO_d, gF_d, gD_d = t(gO), t(gF), t(gD)
    torch.cuda.synchronize()
    b0 = time.perf_counter()
    scene = Scene(*[p.detach() for p in params], builder=args.builder, leaf_size=args.leaf_size)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - b0) * 1e3
    scene.set_params(*params)
    info = scene.info()
    cfg = TraceConfig(k=args.k, recompute=args.recompute, hit_cap=args.hit_cap, sh=sh, sort_rays=args.sort_rays)
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

    # The same step at the other k-buffer size (the paper's 16, or 32 when
    # the main run takes 16): k only changes the number of rounds, never the
    # result (same hits, same order), so this times the identical
    # computation at the other buffer size.
    alt = None
    alt_k = 16 if args.k != 16 else 32
    if not args.no_alt_k:
        cfg_main = cfg
        cfg = TraceConfig(k=alt_k, recompute=args.recompute, hit_cap=args.hit_cap, sh=sh, sort_rays=args.sort_rays)
        step(False)
        torch.cuda.synchronize()
        ev_alt = []
        t1 = time.perf_counter()
        for _ in range(args.steps):
            ev_alt.append(step(True))
        torch.cuda.synchronize()
        ms_alt = (time.perf_counter() - t1) * 1e3 / args.steps
        o_alt = trace(scene, ro_d, rd_d, cfg, hit_cap=0)
        o_main = trace(scene, ro_d, rd_d, cfg_main, hit_cap=0)
        same = all(torch.equal(getattr(o_main, k), getattr(o_alt, k))
                   for k in ("opacity", "feat", "depth", "T", "n_hits"))
        alt = {"k": alt_k, "value": round(R / (ms_alt * 1e-3) / 1e6, 3), "ms_per_step": round(ms_alt, 3),
               "fwd_in_step_ms": round(float(np.median([e[1].elapsed_time(e[2]) for e in ev_alt])), 3),
               "bwd_ms": round(float(np.median([e[2].elapsed_time(e[3]) for e in ev_alt])), 3),
               f"forward_output_bitwise_equal_to_k{args.k}": bool(same)}
        cfg = cfg_main

    # hit statistics of this workload (the same forward, outputs kept)
    res = trace(scene, ro_d, rd_d, cfg, hit_cap=0)
    torch.cuda.synchronize()
    n_hits = res.n_hits.cpu().numpy()
    H = float(n_hits.mean())
    fb = fwd_bytes(n_hits, F, FO)
    bb = bwd_bytes(n_hits, F, FO)
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
    # without stored lists the backward call traces the rays again first
    dom_bytes = fb if dom_is_fwd else (bb + fb if args.recompute else bb)
    bwd_name = "k_trace (retrace) + k_backward" if args.recompute else "k_backward"
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    line = {
        "metric": "Mrays/s fwd+bwd @1M surfels (refit + forward + backward per step)" +
                  (f", SH degree {args.sh_deg} colour" if sh else ""),
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
        "config": {"workload": f"{N} surfels (8 spheres + 4 planes, F={F}"
                               f"{f' = RGB SH degree {args.sh_deg}' if sh else ''}), {args.points}x{args.dirs} "
                               f"cosine MC rays = {R}, refit+fwd+bwd, k={args.k}, T_min=1e-4, "
                               f"{'recompute' if args.recompute else 'store'} mode, {args.builder} tree"
                               f"{', rays sorted by origin' if args.sort_rays else ''}",
                   "surfels": N, "rays": R, "features": F, "k": args.k, "tree": args.builder},
        "fwd_mrays_s": round(R / (fwd_only_ms * 1e-3) / 1e6, 3),
        **({f"k{alt_k}": alt} if alt else {}),
        "fwd_ms": round(fwd_only_ms, 3),
        "fwd_in_step_ms": round(f_med, 3),
        "bwd_ms": round(b_med, 3),
        "refit_ms": round(float(np.median(refit_ms)), 3),
        "build_ms": round(build_ms, 3),
        "hits_per_ray": round(H, 3),
        "bvh_depth": info["max_depth"],
        "roofline": {"bound": "hbm", "kernel": "k_trace (forward)" if dom_is_fwd else bwd_name,
                     "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": measured_traffic() if dom_is_fwd and not sh else None,
                     "l2_hit_rate": measured_l2_hit_rate() if dom_is_fwd and not sh else None,
                     "algorithmic_bytes_per_launch": dom_bytes, "launch_ms": round(dom_ms, 3)},
        "roofline_fwd": {"achieved": round(fb / (fwd_only_ms * 1e-3) / 1e9, 3), "bytes": fb},
        "max_memory_allocated_gib": round(torch.cuda.max_memory_allocated(dev) / 2**30, 3),
    }
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a sample")
        line["cpu_baseline"] = cpu_baseline(sc, ro, rd, gO, gF, gD, budget_s=args.cpu_budget,
                                            sh_deg=args.sh_deg)
    scene.close()
    return line


def _time_launches(fn, reps=3):
    import torch
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def run_forward_only(args, small: bool):
    """c1: 4,096-surfel cube, 64x64 pinhole rays; c2: 200K surfels, 4.2M MC
    rays.  Forward only, BVH tracer vs the brute-force GPU tracer (plain)."""
    import torch
    from paper_2412_15867_amd import Scene, TraceConfig, synth, trace
    dev = torch.device("cuda:0")
    if small:
        sc = synth.cube_scene()
        ro, rd = synth.pinhole_rays(64, 64)
        name = "4096 surfels (cube), 64x64 pinhole rays, forward, F=3"
        n_brute = ro.shape[0]
    else:
        sc, ro, rd = gen_surface_workload(200_000, 256 * 256, 64)
        name = "200000 surfels (8 spheres + 4 planes, F=8), 256x256x64 MC rays, forward"
        n_brute = 16384
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    scene = Scene(*(t(a) for a in sc.astuple()), builder=args.builder, leaf_size=args.leaf_size)
    ro_d, rd_d = t(ro), t(rd)
    R = ro.shape[0]
    cfg = TraceConfig(k=args.k)
    res = trace(scene, ro_d, rd_d, cfg)
    torch.cuda.synchronize()
    ms = _time_launches(lambda: trace(scene, ro_d, rd_d, cfg, out=res), reps=max(3, args.steps))
    n_hits = res.n_hits.cpu().numpy()
    sub = slice(0, n_brute)
    bres = trace(scene, ro_d[sub], rd_d[sub], TraceConfig(k=args.k, brute_force=True))
    torch.cuda.synchronize()
    bms = _time_launches(lambda: trace(scene, ro_d[sub], rd_d[sub], TraceConfig(k=args.k, brute_force=True),
                                       out=bres), reps=2)
    same = bool(torch.equal(bres.opacity, res.opacity[sub]) and torch.equal(bres.n_hits, res.n_hits[sub]))
    fb = fwd_bytes(n_hits, sc.F)
    ach = fb / (ms * 1e-3) / 1e9
    line = {"metric": "Mrays/s fwd", "value": round(R / (ms * 1e-3) / 1e6, 3), "unit": "Mrays/s", "n_gpus": 1,
            "steps": max(3, args.steps), "warmup": 1, "ms_per_step": round(ms, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": name + f", k={args.k}", "surfels": sc.n, "rays": R},
            "hits_per_ray": round(float(n_hits.mean()), 3),
            "plain_gpu_bruteforce": {"mrays_s": round(n_brute / (bms * 1e-3) / 1e6, 3), "rays": n_brute,
                                     "ms": round(bms, 3), "bitwise_equal_to_bvh": same},
            "roofline": {"bound": "hbm", "kernel": "k_trace (forward)", "achieved": round(ach, 3),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None}}
    if not args.no_cpu_baseline:
        import oracle
        g = np.random.default_rng(7)
        m = min(R, 4096 if small else 2048)
        idx = np.sort(g.choice(R, m, replace=False))
        t0 = time.perf_counter()
        oracle.trace(sc.astuple(), ro[idx], rd[idx])
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": round(m / dt / 1e6, 6), "unit": "Mrays/s", "cores": oracle.max_threads(),
                                "kind": "oracle", "sample": f"{m} seeded rays, brute force FP64 forward"}
    scene.close()
    return line


def run_serve(args):
    """Three resident scenes (300K, 1M, 3M surfels); Poisson arrivals of
    requests with log-uniform ray counts in [1K, 4M] over device ray pools;
    continuous batching into packed launches vs one launch per request."""
    import torch
    from paper_2412_15867_amd import Scene, TraceConfig, synth, trace, trace_packed, alloc_result
    from paper_2412_15867_amd.serve import Server, latency_stats, run_open_loop, run_per_request
    dev = torch.device("cuda:0")
    lay = synth.layout()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    sizes = (300_000, 1_000_000, 3_000_000)
    scenes = []
    for n in sizes:
        sc = synth.surface_scene(n, F=8, lay=lay)
        scenes.append(Scene(*(t(a) for a in sc.astuple()), builder=args.builder, leaf_size=args.leaf_size))
        del sc
    ro, rd = synth.mc_rays(256 * 256, 64, lay=lay)
    pool_o, pool_d = t(ro), t(rd)
    P = pool_o.shape[0]
    cfg = TraceConfig(k=args.k)
    n_req = args.requests
    scene_ids, counts, seeds = synth.serving_requests(n_req, len(scenes), 1000, P)
    offs = [int(s % (P - c + 1)) for s, c in zip(seeds, counts)]

    def make(i):
        o, c = offs[i], int(counts[i])
        return int(scene_ids[i]), pool_o[o:o + c], pool_d[o:o + c]

    # capacity: one packed launch of a large mixed batch
    items = []
    for j in range(6):
        o = (j * 700_000) % (P - 700_000)
        items.append((j % 3, pool_o[o:o + 700_000], pool_d[o:o + 700_000], alloc_result(700_000, 8, dev)))
    trace_packed(scenes, items, cfg)
    torch.cuda.synchronize()
    cap_ms = _time_launches(lambda: trace_packed(scenes, items, cfg), reps=2)
    cap = 6 * 700_000 / (cap_ms * 1e-3)
    mean_rays = float(np.mean(counts))
    rate = args.load * cap / mean_rays
    arrivals = synth.poisson_arrivals(n_req, rate)
    log(f"capacity {cap / 1e6:.1f} Mrays/s, {n_req} requests, mean {mean_rays:.0f} rays, rate {rate:.1f}/s")
    srv = Server(scenes, cfg, chunk_rays=args.chunk_rays, max_launch_rays=args.launch_rays)
    reqs = run_open_loop(srv, arrivals, make)
    torch.cuda.synchronize()
    packed = latency_stats(reqs)
    # same results alone (bitwise) for a few requests
    same = True
    for r in reqs[:: max(1, n_req // 8)]:
        a = trace(scenes[r.scene], r.ro, r.rd, cfg)
        same &= bool(torch.equal(a.opacity, r.result.opacity) and torch.equal(a.feat, r.result.feat))
    for r in reqs:
        r.result = None
    base_reqs = run_per_request(scenes, cfg, arrivals, make)
    torch.cuda.synchronize()
    base = latency_stats(base_reqs)
    line = {"metric": "serving Mrays/s with p50/p99 latency (packed continuous batching vs one launch per request)",
            "value": round(packed["mrays_s"], 3), "unit": "Mrays/s", "n_gpus": 1, "steps": n_req, "warmup": 1,
            "ms_per_step": round(packed["mean_ms"], 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"3 resident scenes {sizes} surfels, {n_req} Poisson requests, rays "
                                   f"log-uniform [1e3, {P}], offered load {args.load} of packed capacity, k={args.k}, "
                                   f"work items of {args.chunk_rays} rays, launches of up to {args.launch_rays}"},
            "packed": packed, "per_request": base, "launches": srv.launches,
            "launches_per_request": round(float(np.mean([r.launches for r in reqs])), 3),
            "capacity_mrays_s": round(cap / 1e6, 3), "mix_equals_alone": same}
    for s in scenes:
        s.close()
    return line


def run_c5(args):
    """5M surfels, 1024^2 surface points x 32 directions (33.5M rays):
    forward + backward, then centres += N(0, 1e-3), scales *= exp(N(0, 0.01))
    and a refit, per step."""
    import torch
    from paper_2412_15867_amd import Scene, TraceConfig, trace, trace_backward, synth
    dev = torch.device("cuda:0")
    sc, ro, rd = gen_surface_workload(5_000_000, 1024 * 1024, 32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    params = [t(a) for a in sc.astuple()]
    del sc
    ro_d, rd_d = t(ro), t(rd)
    R = ro.shape[0]
    del ro, rd
    gen = torch.Generator(device=dev)
    gen.manual_seed(synth.SEED_STEP)
    gO = torch.randn(R, device=dev, generator=gen)
    gF = torch.randn((R, 8), device=dev, generator=gen)
    gD = torch.randn(R, device=dev, generator=gen)
    b0 = time.perf_counter()
    scene = Scene(*params, builder=args.builder, leaf_size=args.leaf_size)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - b0) * 1e3
    cfg = TraceConfig(k=args.k, recompute=args.recompute, sort_rays=args.sort_rays)
    hit_cap = 0 if args.recompute else args.hit_cap
    ev = lambda: torch.cuda.Event(enable_timing=True)
    phases = []
    steps = args.steps
    t0 = None
    for i in range(args.warmup + steps):
        if i == args.warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        e = [ev() for _ in range(5)]
        e[0].record()
        res = trace(scene, ro_d, rd_d, cfg, hit_cap=hit_cap)
        e[1].record()
        grads = trace_backward(scene, ro_d, rd_d, res, gO, gF, gD, cfg=cfg)
        e[2].record()
        with torch.no_grad():
            params[0].add_(torch.randn(params[0].shape, device=dev, generator=gen), alpha=1e-3)
            params[2].mul_(torch.exp(0.01 * torch.randn(params[2].shape, device=dev, generator=gen)))
        e[3].record()
        scene.refit()
        e[4].record()
        del res, grads
        if i >= args.warmup:
            phases.append(e)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    f = [p[0].elapsed_time(p[1]) for p in phases]
    b = [p[1].elapsed_time(p[2]) for p in phases]
    u = [p[3].elapsed_time(p[4]) for p in phases]
    step_ms = wall * 1e3 / steps
    line = {"metric": "Mrays/s training-like step (fwd + bwd + perturb + refit)", "value":
            round(R / (step_ms * 1e-3) / 1e6, 3), "unit": "Mrays/s", "n_gpus": 1, "steps": steps,
            "warmup": args.warmup, "ms_per_step": round(step_ms, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"5000000 surfels, 1024x1024x32 = {R} MC rays, F=8, k={args.k}, "
                                   f"{'recompute' if args.recompute else 'store'} mode"
                                   f"{', rays sorted by origin' if args.sort_rays else ''}"},
            "fwd_ms": round(float(np.median(f)), 3), "bwd_ms": round(float(np.median(b)), 3),
            "refit_ms": round(float(np.median(u)), 3), "build_ms": round(build_ms, 3)}
    scene.close()
    return line


def run_pbr(args):
    """Rendering-equation step (Sec. 3.3 "Rendering", Eq. 13-15): P pixels of
    the 1M-surfel scene, N = 16 x 16 stratified directions each (the paper's
    N_r = 256), view-dependent SH colour of degree 3 in the trace, a 32 x 32
    cubemap sky; per step refit, rays, differentiable trace, shading, and the
    backward through shading and trace to surfels, materials and sky."""
    import torch
    from paper_2412_15867_amd import Scene, TraceConfig, render_pbr, synth, trace, mc_rays
    dev = torch.device("cuda:0")
    N_surf, P, St, Sp = args.surfels, args.pixels, 16, 16
    Nr = St * Sp
    lay = synth.layout()
    sc = synth.surface_scene(N_surf, F=8, lay=lay)
    surf = synth.Surfels(sc.mu, sc.quat, sc.scale, sc.opac, synth.sh_coefficients(N_surf, 3))
    px = synth.shading_pixels(P, Nr, lay=lay)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    params = [t(a).requires_grad_(True) for a in surf.astuple()]
    mats = [t(px[k]).requires_grad_(True) for k in ("albedo", "rough", "env")]
    x, n, wo, u = (t(px[k]) for k in ("x", "n", "wo", "u"))
    g_c = torch.from_numpy(np.random.default_rng(synth.SEED_PBR + 1).standard_normal((P, 3)).astype(np.float32)).to(dev)
    scene = Scene(*[p.detach() for p in params], builder=args.builder, leaf_size=args.leaf_size)
    scene.set_params(*params)
    cfg = TraceConfig(k=args.k, sh=True, hit_cap=args.hit_cap)
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step():
        for q in params + mats:
            q.grad = None
        e = [ev() for _ in range(4)]
        e[0].record()
        scene.refit()
        e[1].record()
        c = render_pbr(scene, params, x, n, wo, *mats, u, St, Sp, cfg)
        e[2].record()
        (c * g_c).sum().backward()
        e[3].record()
        return e

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    med = lambda i, j: float(np.median([e[i].elapsed_time(e[j]) for e in evs]))
    R = P * Nr
    ro, rd = mc_rays(x, n, u, St, Sp)
    res = trace(scene, ro, rd, cfg, hit_cap=0)
    torch.cuda.synchronize()
    nh = res.n_hits.cpu().numpy()
    fwd_ms = med(1, 2)
    fb = fwd_bytes(nh, surf.F, 3)
    line = {"metric": "Mrays/s rendering-equation step (refit + rays + trace + shading + backward)",
            "value": round(R / (step_ms * 1e-3) / 1e6, 3), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(step_ms, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{N_surf} surfels (8 spheres + 4 planes, SH degree 3 colour), {P} pixels x "
                                   f"{St}x{Sp} stratified directions = {R} rays, 32x32 cubemap, k={args.k}, "
                                   "T_min=1e-4, store mode", "pixels": P, "rays": R},
            "refit_ms": round(med(0, 1), 3), "render_fwd_ms": round(fwd_ms, 3), "bwd_ms": round(med(2, 3), 3),
            "hits_per_ray": round(float(nh.mean()), 3),
            "roofline": {"bound": "hbm", "kernel": "rays + k_trace + shading (forward)",
                         "achieved": round(fb / (fwd_ms * 1e-3) / 1e9, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(fb / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5), "traffic": None}}
    scene.close()
    return line


def run_relight(args):
    """Relighting step (the paper's relighting details): once per sky, the
    irradiance and GGX-prefiltered cubemaps (32 x 32, 8 roughness levels),
    the 32 x 32 split-sum table and the sky's sampling CDF; per frame, P
    pixels x 256 directions drawn by the sky's intensity (the paper's
    sampling for relighting; --relight-sampling stratified for 16 x 16
    strata) on the 1M-surfel scene whose 4 features are albedo and roughness,
    the trace blending them with the ray-facing normal, the split-sum
    indirect radiance per ray, and Eq. 15 (forward only)."""
    import torch
    from paper_2412_15867_amd import Scene, TraceConfig, synth, trace, mc_rays
    from paper_2412_15867_amd import brdf_table, env_cdf, env_prefilter, env_rays, relight
    dev = torch.device("cuda:0")
    N_surf, P, St, Sp, M, S = args.surfels, args.pixels, 16, 16, 8, 32
    Nr = St * Sp
    lay = synth.layout()
    sc = synth.surface_scene(N_surf, F=4, lay=lay)
    feat = sc.feat.copy()
    feat[:, 3] = 0.1 + 0.9 * feat[:, 3]
    px = synth.shading_pixels(P, Nr, lay=lay)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    scene = Scene(t(sc.mu), t(sc.quat), t(sc.scale), t(sc.opac), t(feat), builder=args.builder, leaf_size=args.leaf_size)
    x, n, wo, u, albedo, rough, env = (t(px[k]) for k in ("x", "n", "wo", "u", "albedo", "rough", "env"))
    strat = args.relight_sampling == "stratified"
    u3 = t(synth.sky_uniforms(P, Nr))
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def pre():
        e = [ev(), ev()]
        e[0].record()
        irr, pref = env_prefilter(env, M)
        tab = brdf_table(S, device=dev)
        cdf = env_cdf(env)
        e[1].record()
        return (irr, pref, tab, cdf), e

    def frame(tabs):
        irr, pref, tab, cdf = tabs
        if strat:
            return relight(scene, x, n, wo, albedo, rough, env, u, St, Sp, sampling="stratified", irr=irr, pref=pref,
                           table=tab, k=args.k)
        return relight(scene, x, n, wo, albedo, rough, env, u3, irr=irr, pref=pref, table=tab, cdf=cdf, k=args.k)

    for _ in range(args.warmup):
        tabs, _e = pre()
        frame(tabs)
    torch.cuda.synchronize()
    pre_evs = [pre()[1] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        frame(tabs)
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    pre_ms = float(np.median([e[0].elapsed_time(e[1]) for e in pre_evs]))
    R = P * Nr
    ro, rd = mc_rays(x, n, u, St, Sp) if strat else env_rays(x, n, u3, tabs[3], env.shape[1])[:2]
    cfg = TraceConfig(k=args.k, normals=True)
    es = [ev(), ev()]
    es[0].record()
    res = trace(scene, ro, rd, cfg)
    es[1].record()
    torch.cuda.synchronize()
    trace_ms = es[0].elapsed_time(es[1])
    res = trace(scene, ro, rd, cfg, hit_cap=0)
    torch.cuda.synchronize()
    nh = res.n_hits.cpu().numpy()
    fb = fwd_bytes(nh, 4, 7)
    samp = f"{St}x{Sp} stratified directions" if strat else f"{Nr} directions drawn by sky intensity"
    line = {"metric": "Mrays/s relighting frame (rays + trace with blended normal + split-sum + Eq. 15)",
            "value": round(R / (step_ms * 1e-3) / 1e6, 3), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(step_ms, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{N_surf} surfels (8 spheres + 4 planes; albedo + roughness features), {P} "
                                   f"pixels x {samp} = {R} rays, 32x32 cubemap, {M} "
                                   f"prefiltered levels, {S}x{S} BRDF table, k={args.k}, T_min=1e-4",
                       "pixels": P, "rays": R},
            "sky_precompute_ms": round(pre_ms, 3), "trace_ms": round(trace_ms, 3),
            "hits_per_ray": round(float(nh.mean()), 3),
            "roofline": {"bound": "hbm", "kernel": "k_trace (normal blending)",
                         "achieved": round(fb / (trace_ms * 1e-3) / 1e9, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(fb / (trace_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5), "traffic": None}}
    scene.close()
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3", choices=["c3", "c1", "c2", "serve", "c5", "pbr", "relight"])
    ap.add_argument("--pixels", type=int, default=1024, help="pbr / relight workloads: pixels (x 256 directions)")
    ap.add_argument("--relight-sampling", default="env", choices=["env", "stratified"],
                    help="relight workload: directions drawn by the sky's intensity or stratified")
    ap.add_argument("--requests", type=int, default=100)
    ap.add_argument("--load", type=float, default=0.8)
    ap.add_argument("--chunk-rays", type=int, default=65536, help="serve: rays per work item")
    ap.add_argument("--launch-rays", type=int, default=1 << 21, help="serve: rays per packed launch at most")
    ap.add_argument("--surfels", type=int, default=1_000_000)
    ap.add_argument("--points", type=int, default=256 * 256)
    ap.add_argument("--dirs", type=int, default=64)
    ap.add_argument("--k", type=int, default=None,
                    help="k-buffer size (default workload: 32; c5: 64; serve: 32; pbr / relight: 64 up to 2^19 rays, else 32; c1, c2: 16)")
    ap.add_argument("--no-alt-k", action="store_true",
                    help="default workload: skip the same step timed at the other k (16, or 32 when --k 16)")
    ap.add_argument("--leaf-size", type=int, default=0, help="surfels per leaf cluster (0: the library default)")
    ap.add_argument("--builder", default="ploc", choices=["ploc", "radix"],
                    help="binary tree under the 4-wide BVH: PLOC clustering or the Morton radix tree")
    ap.add_argument("--hit-cap", type=int, default=256)
    ap.add_argument("--recompute", action="store_true")
    ap.add_argument("--sort-rays", dest="sort_rays", action="store_true", default=None,
                    help="default and c5 workloads: trace rays in the Morton order of their origins "
                         "(default: on for c5, whose scene outgrows the caches)")
    ap.add_argument("--no-sort-rays", dest="sort_rays", action="store_false")
    ap.add_argument("--sh-deg", type=int, default=-1,
                    help="default workload with view-dependent colour: RGB SH coefficients of this degree (0..3)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with a 512 MiB device copy (for scaling profiled FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.k is None:  # k never changes the result: per workload the fastest measured
        if args.workload in ("pbr", "relight"):
            args.k = 64 if args.pixels * 256 <= (1 << 19) else 32  # tail-bound launches: fewer rounds
        elif args.workload == "c5":
            args.k = 64  # 5M surfels: past the Infinity Cache every round's re-traversal costs HBM latency
        elif args.workload == "serve":
            args.k = 32  # scenes up to 3M surfels (packed launches take 16 or 32)
        elif args.workload == "c3":
            args.k = 32  # half the rounds of the paper's 16 at 3 waves per SIMD; bit-identical results
        else:
            args.k = 16  # the paper's k
    if args.sort_rays is None:
        args.sort_rays = args.workload == "c5"
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the trace shards rays across GPUs with no exchange in the "
              "forward and one gradient all-reduce in the backward, which this single-GPU build does not "
              "run; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c3":
        line = run_c3(args)
    elif args.workload in ("c1", "c2"):
        line = run_forward_only(args, small=args.workload == "c1")
    elif args.workload == "serve":
        line = run_serve(args)
    elif args.workload == "pbr":
        line = run_pbr(args)
    elif args.workload == "relight":
        line = run_relight(args)
    else:
        line = run_c5(args)
    if args.calibrate_copy:
        calibration_copy()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
