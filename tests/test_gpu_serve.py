"""Serving loop on the GPU: each request's result is the same alone and in a
packed mix (bitwise), a tiny budget still completes every request without
exceeding it, and malformed requests are rejected without stalling others."""
import numpy as np
import pytest
import torch

from paper_2412_15867_amd import synth
from gpu_util import dev, make_scene, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def world():
    lay = synth.layout()
    scenes = [make_scene(synth.surface_scene(n, F=8, lay=lay, seed=100 + n)) for n in (20_000, 60_000)]
    scenes.append(make_scene(synth.cube_scene(4096, F=8)))
    ro, rd = synth.mc_rays(4096, 16, lay=lay)
    yield scenes, dev(ro), dev(rd)
    for s in scenes:
        s.close()


def test_mix_equals_alone(world):
    from paper_2412_15867_amd import TraceConfig, trace
    from paper_2412_15867_amd.serve import Server
    scenes, ro, rd = world
    g = np.random.default_rng(40)
    spec = [(int(g.integers(0, 3)), int(g.integers(0, ro.shape[0] - 5000)), int(g.integers(1, 5000)))
            for _ in range(12)]
    note("serve mix")
    srv = Server(scenes, TraceConfig(k=16))
    reqs = [srv.submit(s, ro[o:o + n], rd[o:o + n]) for s, o, n in spec]
    srv.drain()
    torch.cuda.synchronize()
    assert all(r.status == "done" for r in reqs)
    assert srv.launches >= 1
    for r, (s, o, n) in zip(reqs, spec):
        alone = trace(scenes[s], ro[o:o + n], rd[o:o + n], TraceConfig(k=16))
        for a, b in ((r.result.opacity, alone.opacity), (r.result.feat, alone.feat), (r.result.depth, alone.depth),
                     (r.result.T, alone.T), (r.result.n_hits, alone.n_hits)):
            assert torch.equal(a, b)


def test_small_budget_and_rejections(world):
    from paper_2412_15867_amd import TraceConfig
    from paper_2412_15867_amd.serve import Server, run_open_loop
    scenes, ro, rd = world
    note("serve small budget")
    bpr = 4 * (8 + 4)
    srv = Server(scenes, TraceConfig(k=16), budget_bytes=3000 * bpr)
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
    scenes, ro, rd = world
    note("serve nan rays")
    bad_o = ro[:64].clone()
    bad_o[::2, 0] = float("nan")
    srv = Server(scenes, TraceConfig(k=16))
    a = srv.submit(1, bad_o, rd[:64].contiguous())
    b = srv.submit(0, ro[100:200], rd[100:200])
    srv.drain()
    assert a.status == b.status == "done"
    assert torch.all(a.result.n_hits[::2] == 0) and torch.all(a.result.T[::2] == 1)
