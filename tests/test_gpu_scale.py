"""Parity at the large workloads, on sampled rays the FP64 oracle can check
one by one: the 3M-surfel serving scene through the packed launch, and the
5M-surfel training-like scene after two perturb + refit updates (Sec. 4
implementation details: the BVH is updated every iteration) in one
33,554,432-ray launch.  The deferred-list overflow, the root restarts and the
deepest stacks run far more at these sizes than on the small scenes."""
import numpy as np
import pytest
import torch

from paper_2412_15867_amd import synth
from gpu_util import dev, make_scene, note, to_np
from validate import validate

pytestmark = pytest.mark.gpu

FIELDS = ("O", "F", "D", "T", "n_hits")


def test_serving_3m_scene_sampled():
    """Two requests packed together (the 3M-surfel and the 300K-surfel
    serving scenes), split into work items; on 128 sampled rays of each the
    packed outputs equal a trace of those rays alone bit for bit, and the
    lone trace's hit lists (up to 1,024, enough for the longest rays) pass
    the oracle's validation."""
    from paper_2412_15867_amd import TraceConfig, trace
    from paper_2412_15867_amd.serve import Server
    lay = synth.layout()
    surf = [synth.surface_scene(n, F=8, lay=lay) for n in (300_000, 3_000_000)]
    ro, rd = synth.mc_rays(64 * 64, 64, lay=lay, seed=synth.SEED_SERVING + 1)
    note("3M-surfel serving scene: build")
    scenes = [make_scene(s) for s in surf]
    ro_d, rd_d = dev(ro), dev(rd)
    srv = Server(scenes, TraceConfig(k=32))
    big = srv.submit(1, ro_d, rd_d)
    small = srv.submit(0, ro_d[:65536], rd_d[:65536])
    note("3M-surfel serving scene: packed launches")
    srv.drain()
    torch.cuda.synchronize()
    for r, s, n in ((big, surf[1], ro.shape[0]), (small, surf[0], 65536)):
        assert r.status == "done"
        packed = to_np(r.result)
        sample = np.sort(np.random.default_rng(60 + r.scene).choice(n, 128, replace=False))
        alone = to_np(trace(scenes[r.scene], dev(ro[sample]), dev(rd[sample]), TraceConfig(k=16), hit_cap=1024))
        for key in FIELDS:
            assert np.array_equal(packed[key][sample], alone[key]), key
        assert alone["n_hits"].max() <= 1024
        note(f"validating 128 rays on the {s.n}-surfel scene (longest list {alone['n_hits'].max()})")
        st = validate(s.astuple(), ro[sample], rd[sample], alone)
        note(f"  exact lists on {st['exact']} of {st['exact_eligible']} unambiguous rays")
    for s in scenes:
        s.close()


def test_5m_after_two_refits_one_33m_ray_launch():
    """The training-like workload: 5M surfels, 1024 x 1024 surface points x
    32 directions.  Two updates (centres += N(0, 1e-3), scales *=
    exp(N(0, 0.01)), drawn on the host and written into the scene's
    parameter tensors), each followed by a refit; then the whole ray set in
    one launch (k = 64, rays handed out in origin order, as the benchmark
    runs it).  256 sampled rays: their outputs equal a separate trace of
    those rays alone bit for bit (k = 16, caller order, with hit lists), and
    those lists pass the oracle's validation on the updated parameters."""
    from paper_2412_15867_amd import TraceConfig, trace
    lay = synth.layout()
    sc = synth.surface_scene(5_000_000, F=8, lay=lay)
    ro, rd = synth.mc_rays(1024 * 1024, 32, lay=lay)
    R = ro.shape[0]
    note("5M surfels: build")
    scene = make_scene(sc)
    params = [np.array(a, copy=True) for a in sc.astuple()]
    del sc
    g = np.random.default_rng(61)
    for step in range(2):
        params[0] = (params[0] + g.normal(0.0, 1e-3, params[0].shape)).astype(np.float32)
        params[2] = (params[2] * np.exp(g.normal(0.0, 0.01, params[2].shape))).astype(np.float32)
        with torch.no_grad():
            scene.mu.copy_(dev(params[0]))
            scene.scale.copy_(dev(params[2]))
        scene.refit()
        note(f"5M surfels: update {step + 1} and refit")
    ro_d, rd_d = dev(ro), dev(rd)
    note(f"5M surfels: one launch over {R} rays")
    full = trace(scene, ro_d, rd_d, TraceConfig(k=64, sort_rays=True))
    torch.cuda.synchronize()
    sample = np.sort(np.random.default_rng(62).choice(R, 256, replace=False))
    alone = to_np(trace(scene, dev(ro[sample]), dev(rd[sample]), TraceConfig(k=16), hit_cap=1024))
    torch.cuda.synchronize()
    full_np = {k: v.cpu().numpy() for k, v in (("O", full.opacity), ("F", full.feat), ("D", full.depth),
                                                  ("T", full.T), ("n_hits", full.n_hits))}
    del full, ro_d, rd_d
    for key in FIELDS:
        assert np.array_equal(full_np[key][sample], alone[key]), key
    assert alone["n_hits"].max() <= 1024
    note("validating 256 rays against the oracle over 5M surfels")
    # grazing rays along a surface cross the planes of many thousand discs
    st = validate(tuple(params), ro[sample], rd[sample], alone, cap=32768)
    note(f"  exact lists on {st['exact']} of {st['exact_eligible']} unambiguous rays; "
         f"mean hits {full_np['n_hits'].mean():.1f}")
    scene.close()
