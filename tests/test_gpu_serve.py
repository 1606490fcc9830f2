"""Serving loop on the GPU: each request's result is the same alone and in a
packed mix (bitwise), whatever its split into work items; a seeded sample of
every request's packed result passes the FP64 oracle's per-ray validation; a
small request submitted behind a large one completes first; a tiny budget
still completes every request without exceeding it; malformed requests are
rejected without stalling others."""
import numpy as np
import pytest
import torch

from paper_2412_15867_amd import synth
from gpu_util import dev, make_scene, note, to_np
from validate import validate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def world():
    lay = synth.layout()
    surf = [synth.surface_scene(n, F=8, lay=lay, seed=100 + n) for n in (20_000, 60_000)]
    surf.append(synth.cube_scene(4096, F=8))
    scenes = [make_scene(s) for s in surf]
    ro, rd = synth.mc_rays(4096, 16, lay=lay)
    yield scenes, dev(ro), dev(rd), surf, ro, rd
    for s in scenes:
        s.close()


def _scratch(max_launch_rays, inflight=2):
    from paper_2412_15867_amd import _lib
    return inflight * int(_lib.lib().irgs_trace_bytes(max_launch_rays, 8, 0))


def test_mix_equals_alone(world):
    from paper_2412_15867_amd import TraceConfig, trace
    from paper_2412_15867_amd.serve import Server
    scenes, ro, rd = world[:3]
    g = np.random.default_rng(40)
    spec = [(int(g.integers(0, 3)), int(g.integers(0, ro.shape[0] - 5000)), int(g.integers(1, 5000)))
            for _ in range(12)]
    note("serve mix (items of 1,000 rays, launches of 8,000)")
    srv = Server(scenes, TraceConfig(k=16), chunk_rays=1000, max_launch_rays=8000)
    reqs = [srv.submit(s, ro[o:o + n], rd[o:o + n]) for s, o, n in spec]
    srv.drain()
    torch.cuda.synchronize()
    assert all(r.status == "done" for r in reqs)
    assert srv.launches > 1 and max(r.launches for r in reqs) > 1
    for r, (s, o, n) in zip(reqs, spec):
        alone = trace(scenes[s], ro[o:o + n], rd[o:o + n], TraceConfig(k=16))
        for a, b in ((r.result.opacity, alone.opacity), (r.result.feat, alone.feat), (r.result.depth, alone.depth),
                     (r.result.T, alone.T), (r.result.n_hits, alone.n_hits)):
            assert torch.equal(a, b)


@pytest.mark.parametrize("k", [16, 32])
def test_packed_results_match_oracle(world, k):
    """Every request of a packed mix, split into items across launches,
    validated on a seeded sample of its rays against the brute-force FP64
    oracle (hit lists, order, termination, values within 1e-4)."""
    from paper_2412_15867_amd import TraceConfig
    from paper_2412_15867_amd.serve import Server
    scenes, ro, rd, surf, ro_np, rd_np = world
    g = np.random.default_rng(43 + k)
    spec = [(int(g.integers(0, 3)), int(g.integers(0, ro.shape[0] - 6000)), int(g.integers(50, 6000)))
            for _ in range(9)]
    note(f"serve oracle parity k={k}")
    srv = Server(scenes, TraceConfig(k=k), chunk_rays=1500, max_launch_rays=6000, hit_cap=256)
    reqs = [srv.submit(s, ro[o:o + n], rd[o:o + n]) for s, o, n in spec]
    srv.drain()
    torch.cuda.synchronize()
    exact = eligible = 0
    for i, (r, (s, o, n)) in enumerate(zip(reqs, spec)):
        assert r.status == "done"
        out = to_np(r.result)
        assert out["n_hits"].max() <= 256
        sample = np.sort(np.random.default_rng(1000 + i).choice(n, min(n, 24), replace=False))
        st = validate(surf[s].astuple(), ro_np[o:o + n], rd_np[o:o + n], out, rays=sample)
        exact += st["exact"]
        eligible += st["exact_eligible"]
    note(f"exact lists on {exact} of {eligible} unambiguous rays")


def test_small_request_completes_before_large(world):
    """Per-request completion: a 100-ray request submitted right after a
    65,536-ray one rides in the next launch and completes while the large
    request still has launches to go."""
    from paper_2412_15867_amd import TraceConfig
    from paper_2412_15867_amd.serve import Server
    scenes, ro, rd = world[:3]
    note("serve small behind large")
    srv = Server(scenes, TraceConfig(k=16), chunk_rays=4096, max_launch_rays=8192)
    big = srv.submit(1, ro, rd)
    srv.poll()  # the large request's first launch is on the device
    small = srv.submit(0, ro[:100], rd[:100])
    srv.drain()
    assert big.status == small.status == "done"
    assert big.launches >= 8 and small.launches == 1
    assert small.done_at < big.done_at


def test_small_budget_and_rejections(world):
    from paper_2412_15867_amd import TraceConfig
    from paper_2412_15867_amd.serve import Server, run_open_loop
    scenes, ro, rd = world[:3]
    note("serve small budget")
    bpr = 4 * (8 + 4)
    with pytest.raises(ValueError):  # the launch scratch alone does not fit
        Server(scenes, TraceConfig(k=16), max_launch_rays=4096, budget_bytes=_scratch(4096))
    srv = Server(scenes, TraceConfig(k=16), max_launch_rays=4096, chunk_rays=1024,
                 budget_bytes=_scratch(4096) + 3000 * bpr)
    bad = srv.submit(7, ro[:10], rd[:10])
    assert bad.status == "rejected"
    bad2 = srv.submit(0, ro[:10].cpu(), rd[:10].cpu())
    assert bad2.status == "rejected"
    too_big = srv.submit(0, ro[:5000], rd[:5000])
    assert too_big.status == "rejected"
    arrivals = np.cumsum(np.random.default_rng(41).exponential(2e-4, 40))
    g = np.random.default_rng(42)

    def make(i):
        n = int(g.integers(1, 3000))
        o = int(g.integers(0, ro.shape[0] - n))
        return int(g.integers(0, 3)), ro[o:o + n], rd[o:o + n]

    reqs = run_open_loop(srv, arrivals, make)
    assert all(r.status == "done" for r in reqs)
    assert srv.sched.peak_used <= 3000 * bpr
    assert srv.sched.used == 0
    assert all(r.latency is not None and r.latency > 0 for r in reqs)


def test_invalid_rays_are_misses_in_a_mix(world):
    from paper_2412_15867_amd import TraceConfig
    from paper_2412_15867_amd.serve import Server
    scenes, ro, rd = world[:3]
    note("serve nan rays")
    bad_o = ro[:64].clone()
    bad_o[::2, 0] = float("nan")
    srv = Server(scenes, TraceConfig(k=16), chunk_rays=16)
    a = srv.submit(1, bad_o, rd[:64].contiguous())
    b = srv.submit(0, ro[100:200], rd[100:200])
    e = srv.submit(2, ro[:0], rd[:0])
    srv.drain()
    assert a.status == b.status == e.status == "done"
    assert torch.all(a.result.n_hits[::2] == 0) and torch.all(a.result.T[::2] == 1)
