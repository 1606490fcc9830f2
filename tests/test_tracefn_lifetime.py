"""Lifetime of the autograd wrapper's saved state, on the CPU.

The two library calls are replaced by CPU stand-ins (no arithmetic of the
method: they only allocate tensors of the right shapes), so this checks the
wrapper's reference structure alone: with the cyclic collector switched off,
every step's outputs and stored hit lists must be freed as soon as the step's
tensors go out of scope.  A Stage II loop (Sec. 3.3) differentiates through
the trace every iteration, so one leaked step per call exhausts memory."""
import gc
import weakref

import pytest
import torch

from paper_2412_15867_amd import tracer


class _FakeScene:
    def __init__(self, n, F):
        self.n, self.F = n, F
        self.mu = torch.zeros(n, 3)
        self.quat = torch.zeros(n, 4)
        self.scale = torch.ones(n, 2)
        self.opacity = torch.full((n,), 0.5)
        self.feat = torch.zeros(n, F)
        self.device = torch.device("cpu")


@pytest.fixture
def fake_calls(monkeypatch):
    made = []

    def fake_trace(scene, ro, rd, cfg, hit_cap=0, **kw):
        R = ro.shape[0]
        res = tracer.TraceResult(torch.zeros(R), torch.zeros(R, scene.F), torch.zeros(R), torch.ones(R),
                                 torch.zeros(R, dtype=torch.int32),
                                 torch.zeros(R, hit_cap, dtype=torch.int32) if hit_cap else None,
                                 torch.zeros(R, hit_cap) if hit_cap else None)
        made.append([weakref.ref(t) for t in (res.opacity, res.feat, res.depth, res.T, res.n_hits)
                     + ((res.hit_ids, res.hit_T) if hit_cap else ())])
        return res

    def fake_backward(scene, ro, rd, saved, gO, gF, gD, cfg=None, **kw):
        assert saved.n_hits is not None and saved.opacity.shape == (ro.shape[0],)
        return dict(mu=torch.zeros_like(scene.mu), quat=torch.zeros_like(scene.quat),
                    scale=torch.zeros_like(scene.scale), opacity=torch.zeros_like(scene.opacity),
                    feat=torch.zeros_like(scene.feat))

    monkeypatch.setattr(tracer, "trace", fake_trace)
    monkeypatch.setattr(tracer, "trace_backward", fake_backward)
    return made


@pytest.mark.parametrize("recompute", [False, True])
def test_outputs_and_hit_lists_freed_without_cyclic_gc(fake_calls, recompute):
    scene = _FakeScene(32, 8)
    params = [t.clone().requires_grad_(True) for t in (scene.mu, scene.quat, scene.scale, scene.opacity,
                                                       scene.feat)]
    scene.mu, scene.quat, scene.scale, scene.opacity, scene.feat = params
    ro, rd = torch.zeros(64, 3), torch.ones(64, 3)
    cfg = tracer.TraceConfig(recompute=recompute, hit_cap=16)
    was = gc.isenabled()
    gc.disable()
    try:
        for step in range(30):
            O, Fo, D = tracer.TraceFn.apply(*params, ro, rd, scene, cfg)
            torch.autograd.backward([O, Fo, D], [torch.ones_like(O), torch.ones_like(Fo), torch.ones_like(D)])
            # the stored lists and T go with the backward, while the outputs are still held
            assert all(r() is None for r in fake_calls[step][3:]), f"step {step}: saved state outlives backward"
            del O, Fo, D
            alive = [r for r in fake_calls[step] if r() is not None]
            assert not alive, f"step {step}: {len(alive)} forward tensors outlive the step"
    finally:
        if was:
            gc.enable()


def test_outputs_freed_when_backward_never_runs(fake_calls):
    scene = _FakeScene(8, 3)
    params = [t.clone().requires_grad_(True) for t in (scene.mu, scene.quat, scene.scale, scene.opacity,
                                                       scene.feat)]
    scene.mu, scene.quat, scene.scale, scene.opacity, scene.feat = params
    was = gc.isenabled()
    gc.disable()
    try:
        O, Fo, D = tracer.TraceFn.apply(*params, torch.zeros(4, 3), torch.ones(4, 3), scene,
                                        tracer.TraceConfig(hit_cap=4))
        del O, Fo, D
        assert all(r() is None for r in fake_calls[0])
    finally:
        if was:
            gc.enable()


def test_opacity_must_be_the_scene_tensor(fake_calls):
    scene = _FakeScene(8, 3)
    params = [t.clone().requires_grad_(True) for t in (scene.mu, scene.quat, scene.scale, scene.opacity,
                                                       scene.feat)]
    scene.mu, scene.quat, scene.scale, scene.opacity, scene.feat = params
    other = params[3].detach().clone().requires_grad_(True)
    with pytest.raises(ValueError):
        tracer.TraceFn.apply(params[0], params[1], params[2], other, params[4], torch.zeros(4, 3),
                             torch.ones(4, 3), scene, tracer.TraceConfig())


def test_opacity_gradient_takes_the_input_shape(fake_calls):
    scene = _FakeScene(8, 3)
    params = [t.clone().requires_grad_(True) for t in (scene.mu, scene.quat, scene.scale, scene.opacity,
                                                       scene.feat)]
    op2 = params[3].detach().clone().reshape(8, 1).requires_grad_(True)
    scene.mu, scene.quat, scene.scale, scene.feat = params[0], params[1], params[2], params[4]
    scene.opacity = op2.reshape(8)  # the scene keeps the flat view of the same storage
    O, Fo, D = tracer.TraceFn.apply(params[0], params[1], params[2], op2, params[4], torch.zeros(4, 3),
                                    torch.ones(4, 3), scene, tracer.TraceConfig())
    (O.sum() + Fo.sum() + D.sum()).backward()
    assert op2.grad is not None and op2.grad.shape == (8, 1)


def test_retained_graph_runs_backward_twice(fake_calls):
    scene = _FakeScene(8, 3)
    params = [t.clone().requires_grad_(True) for t in (scene.mu, scene.quat, scene.scale, scene.opacity,
                                                       scene.feat)]
    scene.mu, scene.quat, scene.scale, scene.opacity, scene.feat = params
    O, Fo, D = tracer.TraceFn.apply(*params, torch.zeros(4, 3), torch.ones(4, 3), scene,
                                    tracer.TraceConfig(hit_cap=4))
    O.sum().backward(retain_graph=True)
    Fo.sum().backward()
    with pytest.raises(RuntimeError):  # freed after the backward that did not retain it
        D.sum().backward()
