"""Backward parity of the HIP adjoint against the FP64 gradient oracle
(autograd over the same hit lists) and finite differences; store and
re-march modes; the torch.autograd.Function wrapper."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import grad as ograd
from paper_2412_15867_amd import synth
from gpu_util import dev, make_scene, note, to_np
from validate import validate

pytestmark = pytest.mark.gpu

NAMES = (("mu", "mu"), ("quat", "quat"), ("scale", "scale"), ("opacity", "opac"), ("feat", "feat"))


def grad_close(g_gpu, g_ref, rel=1e-3):
    """|d| <= rel (|g_ref| + mean |g_ref| of the group), per parameter group."""
    worst = {}
    for name, key in NAMES:
        a = g_gpu[name].reshape(g_ref[key].shape)
        b = g_ref[key]
        floor = np.abs(b).mean() + 1e-30
        err = np.abs(a - b) / (np.abs(b) + floor)
        worst[name] = float(err.max())
        assert err.max() <= rel, (name, err.max())
    return worst


def gpu_fwd_bwd(surf, ro, rd, gO, gF, gD, hit_cap=256, recompute=False, k=16, T_min=1e-4, sort_rays=False,
                t_min=0.0):
    from paper_2412_15867_amd import TraceConfig, trace, trace_backward
    scene = make_scene(surf)
    cfg = TraceConfig(k=k, T_min=T_min, recompute=recompute, sort_rays=sort_rays, t_min=t_min)
    res = trace(scene, dev(ro), dev(rd), cfg, hit_cap=hit_cap)
    grads = trace_backward(scene, dev(ro), dev(rd), res, dev(gO), dev(gF), dev(gD), cfg=cfg)
    torch.cuda.synchronize()
    out = {k2: v.cpu().numpy().astype(np.float64) for k2, v in grads.items()}
    fwd = to_np(res)
    scene.close()
    return fwd, out


def lists_of(fwd):
    H = fwd["hit_ids"].shape[1]
    return np.where(np.arange(H)[None, :] < fwd["n_hits"][:, None], fwd["hit_ids"], -1)


@pytest.fixture(scope="module")
def cube():
    sc = synth.cube_scene()
    ro, rd = synth.pinhole_rays(32, 32)
    gO, gF, gD, _ = synth.upstream(ro.shape[0], sc.F)
    return sc, ro, rd, gO, gF, gD


def test_cube_gradients_match_fp64_oracle(cube):
    sc, ro, rd, gO, gF, gD = cube
    note("cube backward store")
    fwd, g = gpu_fwd_bwd(sc.astuple(), ro, rd, gO, gF, gD)
    validate(sc.astuple(), ro, rd, fwd)
    ref = ograd.grad_given_hits(sc.astuple(), ro, rd, lists_of(fwd), gO, gF, gD)
    w = grad_close(g, ref)
    note(f"cube worst rel err {w}")


@pytest.mark.parametrize("recompute", [False, True])
@pytest.mark.parametrize("F", [12, 40])
def test_wide_features_match_fp64_oracle(F, recompute):
    """More features than the backward pre-reduces in LDS (F > 8): those
    launches take rays in the order of where they land; the sums are the
    same, with stored lists and with the rays traced again."""
    sc = synth.cube_scene(F=F)
    ro, rd = synth.pinhole_rays(32, 32)
    gO, gF, gD, _ = synth.upstream(ro.shape[0], F)
    note(f"cube backward F={F} recompute={recompute}")
    fwd, g = gpu_fwd_bwd(sc.astuple(), ro, rd, gO, gF, gD, recompute=recompute)
    ref = ograd.grad_given_hits(sc.astuple(), ro, rd, lists_of(fwd), gO, gF, gD)
    grad_close(g, ref)


@pytest.mark.parametrize("sort_rays", [False, True])
def test_recompute_equals_store(cube, sort_rays):
    """The backward without stored lists (rays traced again, optionally in
    the Morton order of their origins) gives the store mode's gradients."""
    sc, ro, rd, gO, gF, gD = cube
    note(f"cube backward recompute, sort_rays={sort_rays}")
    _, a = gpu_fwd_bwd(sc.astuple(), ro, rd, gO, gF, gD)
    _, b = gpu_fwd_bwd(sc.astuple(), ro, rd, gO, gF, gD, hit_cap=0, recompute=True, sort_rays=sort_rays)
    for name, _ in NAMES:
        np.testing.assert_allclose(a[name], b[name], rtol=1e-4, atol=1e-6 * np.abs(a[name]).max())


def test_small_hit_cap_falls_back_to_recompute(cube):
    """Rays with more hits than the stored capacity re-march."""
    sc, ro, rd, gO, gF, gD = cube
    note("cube backward hit_cap 4")
    fwd, a = gpu_fwd_bwd(sc.astuple(), ro, rd, gO, gF, gD, hit_cap=4)
    assert np.mean(fwd["n_hits"] > 4) > 0.2
    _, b = gpu_fwd_bwd(sc.astuple(), ro, rd, gO, gF, gD, hit_cap=256)
    for name, _ in NAMES:
        np.testing.assert_allclose(a[name], b[name], rtol=1e-4, atol=1e-6 * np.abs(b[name]).max())


@pytest.mark.parametrize("k", [4, 32])
def test_negative_t_min_store_and_remarch(cube, k):
    """Origins inside the cube and t_min = -10: hits behind and in front of
    the origin in one list.  Stored lists: the gradients match the FP64
    oracle on the validated lists; a stored capacity of 4 (the rest
    re-marched) and the recompute mode give the same gradients."""
    sc, ro, rd, gO, gF, gD = cube
    ro_in = (ro + 2.5 * rd).astype(np.float32)
    note(f"cube backward, negative t_min, k={k}")
    fwd, a = gpu_fwd_bwd(sc.astuple(), ro_in, rd, gO, gF, gD, k=k, t_min=-10.0)
    validate(sc.astuple(), ro_in, rd, fwd, t_min=-10.0)
    ref = ograd.grad_given_hits(sc.astuple(), ro_in, rd, lists_of(fwd), gO, gF, gD)
    grad_close(a, ref)
    fwd4, b = gpu_fwd_bwd(sc.astuple(), ro_in, rd, gO, gF, gD, k=k, t_min=-10.0, hit_cap=4)
    assert np.mean(fwd4["n_hits"] > 4) > 0.2
    _, c = gpu_fwd_bwd(sc.astuple(), ro_in, rd, gO, gF, gD, k=k, t_min=-10.0, hit_cap=0, recompute=True)
    for name, _ in NAMES:
        np.testing.assert_allclose(b[name], a[name], rtol=1e-4, atol=1e-6 * np.abs(a[name]).max())
        np.testing.assert_allclose(c[name], a[name], rtol=1e-4, atol=1e-6 * np.abs(a[name]).max())


def coaxial_splats(n, opacity, seed):
    """n splats stacked along -z in a random order, two rays down the axis."""
    g = np.random.default_rng(seed)
    perm = g.permutation(n)
    mu = np.stack([g.normal(0, 0.01, n), g.normal(0, 0.01, n), -0.05 * np.arange(n)], 1)[perm].astype(np.float32)
    q = np.tile(np.float32([1, 0, 0, 0]), (n, 1)) + g.normal(0, 0.05, (n, 4)).astype(np.float32)
    s = np.full((n, 2), 0.1, np.float32)
    o = np.full(n, opacity, np.float32)
    f = g.uniform(0, 1, (n, 3)).astype(np.float32)
    ro = np.float32([[0, 0, 1.0], [0.01, 0.02, 1.0]])
    rd = np.float32([[0, 0, -1.0], [0, 0, -1.0]])
    gO, gF, gD = np.float32([1, -0.5]), np.float32([[0.3, 0.2, 0.1], [1, 1, 1]]), np.float32([0.7, 0.1])
    return (mu, q, s, o, f), ro, rd, gO, gF, gD


def test_many_rounds_past_the_checkpoints():
    """k = 1 on 60 coaxial splats: 42 rounds, more than the 16 round
    checkpoints, re-marched (stored capacity 4: the re-march's private list
    holds them); the same rays traced again by the backward (no stored
    lists) and in store mode at k = 16."""
    surf, ro, rd, gO, gF, gD = coaxial_splats(60, 0.2, 30)
    note("deep rays k=1 re-march")
    _, a = gpu_fwd_bwd(surf, ro, rd, gO, gF, gD, hit_cap=4, recompute=False, k=1)
    note("deep rays k=1 retrace")
    fwd, r = gpu_fwd_bwd(surf, ro, rd, gO, gF, gD, hit_cap=64, recompute=True, k=1)
    assert np.all(fwd["n_hits"] > 30)
    ref = ograd.grad_given_hits(surf, ro, rd, lists_of(fwd), gO, gF, gD)
    grad_close(a, ref)
    grad_close(r, ref)
    _, b = gpu_fwd_bwd(surf, ro, rd, gO, gF, gD, hit_cap=64, recompute=False, k=16)
    for name, _ in NAMES:
        np.testing.assert_allclose(a[name], b[name], rtol=1e-4, atol=1e-6 * np.abs(b[name]).max())
        np.testing.assert_allclose(r[name], b[name], rtol=1e-4, atol=1e-6 * np.abs(b[name]).max())


def test_retrace_longer_than_its_list_capacity():
    """300 faint coaxial splats: every hit composites (T stays above T_min),
    more hits than the 256 the backward's retrace keeps per ray, so those
    rays re-march; oracle gradients and store mode agree."""
    surf, ro, rd, gO, gF, gD = coaxial_splats(300, 0.01, 33)
    note("300-hit rays retrace")
    fwd, r = gpu_fwd_bwd(surf, ro, rd, gO, gF, gD, hit_cap=512, recompute=True, k=16)
    assert np.all(fwd["n_hits"] > 256)
    ref = ograd.grad_given_hits(surf, ro, rd, lists_of(fwd), gO, gF, gD)
    grad_close(r, ref)
    _, b = gpu_fwd_bwd(surf, ro, rd, gO, gF, gD, hit_cap=512, recompute=False, k=16)
    for name, _ in NAMES:
        np.testing.assert_allclose(r[name], b[name], rtol=1e-4, atol=1e-6 * np.abs(b[name]).max())


@pytest.mark.parametrize("k", [1, 4, 16])
def test_remarch_longer_than_its_private_list(k):
    """700 faint coaxial splats, every one composited, with 4 stored hits
    per ray: the re-march holds only 512 hits in its private list, so these
    rays are walked back round by round from checkpoints -- at k = 1 the
    checkpoints are thinned five times (700 rounds, 16 checkpoints) -- and
    the gradients must still match the FP64 oracle."""
    surf, ro, rd, gO, gF, gD = coaxial_splats(700, 0.01, 34)
    note(f"700-hit rays re-march k={k}")
    fwd, a = gpu_fwd_bwd(surf, ro, rd, gO, gF, gD, hit_cap=4, recompute=False, k=k)
    full, _ = gpu_fwd_bwd(surf, ro, rd, gO, gF, gD, hit_cap=1024, recompute=False, k=16)
    assert np.all(full["n_hits"] > 512) and np.array_equal(full["n_hits"], fwd["n_hits"])
    ref = ograd.grad_given_hits(surf, ro, rd, lists_of(full), gO, gF, gD)
    grad_close(a, ref)


def test_finite_differences_on_surface_patch():
    """256 surfels nearest a surface point of the 1M-surfel scene, 1,024 rays
    aimed at the patch: GPU gradients vs FP64 central differences of the
    brute-force oracle (perturbations that change a hit list are skipped)."""
    lay = synth.layout()
    big, sid = synth.surface_scene(1_000_000, F=8, lay=lay, return_surface_id=True)
    g = np.random.default_rng(31)
    # a sphere patch: plane patches are coplanar up to FP32 rounding of the
    # inputs, where any perturbation reorders near-tied hits
    c = big.mu[g.choice(np.nonzero(sid < 8)[0])].astype(np.float64)
    d2 = np.sum((big.mu.astype(np.float64) - c) ** 2, 1)
    idx = np.argsort(d2)[:256]
    sub = big.subset(idx)
    rad = float(np.sqrt(d2[idx[-1]]))
    ro, rd = synth.random_rays_near(g, c, rad, 1024, dist=0.5)
    gO, gF, gD, _ = synth.upstream(1024, 8, seed=32)
    note("fd patch gpu")
    fwd, a = gpu_fwd_bwd(sub.astuple(), ro, rd, gO, gF, gD, hit_cap=256)
    validate(sub.astuple(), ro, rd, fwd)
    ref = ograd.grad_given_hits(sub.astuple(), ro, rd, lists_of(fwd), gO, gF, gD)
    grad_close(a, ref)
    # Finite differences see the oracle's own hit lists; keep the rays on
    # which the GPU list is the same, and differentiate those on both sides.
    orc = oracle.trace(sub.astuple(), ro, rd, hit_cap=256)
    same = np.array([fwd["n_hits"][r] == orc["n_hits"][r] and
                     np.array_equal(fwd["hit_ids"][r, :fwd["n_hits"][r]], orc["hits"][r, :orc["n_hits"][r]])
                     for r in range(ro.shape[0])])
    assert same.mean() > 0.5
    ro, rd, gO, gF, gD = ro[same], rd[same], gO[same], gF[same], gD[same]
    fwd, a = gpu_fwd_bwd(sub.astuple(), ro, rd, gO, gF, gD, hit_cap=256)
    # finite differences on the first 48 surfels (every parameter of each)
    keep = np.arange(48)
    surf = [np.array(x, dtype=np.float64) for x in sub.astuple()]
    note("fd patch finite differences")
    fd, skipped = ograd.fd_grad(surf, ro, rd, gO, gF, gD, hit_cap=512, surfel_idx=keep, rel_h=1e-8)
    total = 48 * 18
    assert skipped < 0.5 * total, skipped
    for name, key in NAMES:
        fv = fd[key].reshape(fd[key].shape[0], -1)[keep]
        av = a[name].reshape(a[name].shape[0], -1)[keep]
        m = ~np.isnan(fv)
        floor = np.abs(fv[m]).mean() + 1e-30
        err = np.abs(av[m] - fv[m]) / (np.abs(fv[m]) + floor)
        assert err.max() <= 2e-3, (name, err.max())
    note(f"fd skipped {skipped}")


def test_autograd_function_matches_direct_backward(cube):
    from paper_2412_15867_amd import TraceConfig, TraceFn, trace, trace_backward
    sc, ro, rd, gO, gF, gD = cube
    note("TraceFn")
    params = [dev(x).requires_grad_(True) for x in sc.astuple()]
    from paper_2412_15867_amd import Scene
    scene = Scene(*[p.detach() for p in params])
    # the scene must wrap the very tensors autograd differentiates
    scene.set_params(*params)
    cfg = TraceConfig(k=16)
    O, F, D = TraceFn.apply(*params, dev(ro), dev(rd), scene, cfg)
    loss = (O * dev(gO)).sum() + (F * dev(gF)).sum() + (D * dev(gD)).sum()
    loss.backward()
    res = trace(scene, dev(ro), dev(rd), cfg, hit_cap=64)
    direct = trace_backward(scene, dev(ro), dev(rd), res, dev(gO), dev(gF), dev(gD), cfg=cfg)
    for p, name in zip(params, ("mu", "quat", "scale", "opacity", "feat")):
        torch.testing.assert_close(p.grad, direct[name].reshape(p.shape), rtol=1e-4, atol=1e-5)
    scene.close()


@pytest.mark.parametrize("recompute", [False, True])
def test_autograd_function_matches_fp64_oracle(cube, recompute):
    """The autograd wrapper with plain features (RGB) against the FP64
    gradient oracle over the same, validated hit lists: dL/d(mu, q, s, o, f)
    for L = sum(gO O + gF . F + gD D)."""
    from paper_2412_15867_amd import Scene, TraceConfig, TraceFn, trace
    sc, ro, rd, gO, gF, gD = cube
    note(f"TraceFn vs oracle recompute={recompute}")
    params = [dev(x).requires_grad_(True) for x in sc.astuple()]
    scene = Scene(*[p.detach() for p in params])
    scene.set_params(*params)
    cfg = TraceConfig(k=16, recompute=recompute)
    O, F, D = TraceFn.apply(*params, dev(ro), dev(rd), scene, cfg)
    loss = (O * dev(gO)).sum() + (F * dev(gF)).sum() + (D * dev(gD)).sum()
    loss.backward()
    fwd = to_np(trace(scene, dev(ro), dev(rd), cfg, hit_cap=256))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(O.detach().cpu().numpy(), fwd["O"])
    validate(sc.astuple(), ro, rd, fwd)
    ref = ograd.grad_given_hits(sc.astuple(), ro, rd, lists_of(fwd), gO, gF, gD)
    got = {name: p.grad.detach().cpu().numpy().astype(np.float64)
           for p, name in zip(params, ("mu", "quat", "scale", "opacity", "feat"))}
    w = grad_close(got, ref)
    note(f"TraceFn worst rel err {w}")
    scene.close()


@pytest.mark.parametrize("k", [16, 32])
def test_full_size_headline_config_sampled(k):
    """The benchmarked configuration at full size -- 1M surfels, 256x256x64 =
    4,194,304 MC rays, k = 16 (the paper's) and 32 (the benchmark's), one
    launch each way -- with the forward
    validated on 4,096 sampled rays and the backward checked against the FP64
    oracle with upstream gradients non-zero only on 4,096 other sampled rays,
    whose hit lists are validated too (the gradient oracle differentiates
    along the GPU's lists, so those lists must be right); the backward also
    without stored lists (the rays traced again in three equal batches)."""
    from paper_2412_15867_amd import TraceConfig, trace, trace_backward
    lay = synth.layout()
    sc = synth.surface_scene(1_000_000, F=8, lay=lay)
    ro, rd = synth.mc_rays(256 * 256, 64, lay=lay)
    R = ro.shape[0]
    gO, gF, gD, idx = synth.upstream(R, 8, mask_rays=4096)
    note(f"full size forward + backward, k={k}")
    scene = make_scene(sc)
    cfg = TraceConfig(k=k)
    res = trace(scene, dev(ro), dev(rd), cfg, hit_cap=256)
    grads = trace_backward(scene, dev(ro), dev(rd), res, dev(gO), dev(gF), dev(gD), cfg=cfg)
    note("full size backward, rays traced again")
    grads_re = trace_backward(scene, dev(ro), dev(rd), res, dev(gO), dev(gF), dev(gD),
                              cfg=TraceConfig(k=k, recompute=True))
    torch.cuda.synchronize()
    fwd = to_np(res)
    g = {k: v.cpu().numpy().astype(np.float64) for k, v in grads.items()}
    g_re = {k: v.cpu().numpy().astype(np.float64) for k, v in grads_re.items()}
    scene.close()
    assert fwd["n_hits"].max() <= 256
    sample = np.sort(np.random.default_rng(50).choice(R, 4096, replace=False))
    note("validating 4,096 sampled rays")
    validate(sc.astuple(), ro, rd, fwd, rays=sample)
    note("validating the 4,096 masked rays")
    validate(sc.astuple(), ro, rd, fwd, rays=idx)
    # gradient: only the masked rays contribute; the oracle differentiates them
    note("oracle gradient on the masked rays")
    lists = lists_of({"hit_ids": fwd["hit_ids"][idx], "n_hits": fwd["n_hits"][idx]})
    lists = lists[:, :max(1, int(fwd["n_hits"][idx].max()))]
    ref = ograd.grad_given_hits(sc.astuple(), ro[idx], rd[idx], lists, gO[idx], gF[idx], gD[idx])
    touched = np.unique(lists[lists >= 0])
    for gg in (g, g_re):
        for name, key in NAMES:
            a = gg[name].reshape(gg[name].shape[0], -1)
            b = ref[key].reshape(ref[key].shape[0], -1)
            untouched = np.setdiff1d(np.arange(a.shape[0]), touched)
            assert np.all(a[untouched[:100000]] == 0), name
            a, b = a[touched], b[touched]
            floor = np.abs(b).mean() + 1e-30
            err = np.abs(a - b) / (np.abs(b) + floor)
            assert err.max() <= 1e-3, (name, err.max())


def test_autograd_loop_memory_flat():
    """A Stage II style loop (Sec. 3.3: the trace is differentiated every
    iteration): 30 TraceFn forward + backward steps over 1,048,576 rays with
    stored hit lists.  Without a cyclic garbage collection the device memory
    in use after each step must equal that after the first: no step's outputs
    or hit lists outlive it."""
    import gc
    from paper_2412_15867_amd import Scene, TraceConfig, TraceFn
    lay = synth.layout()
    sc = synth.surface_scene(200_000, F=8, lay=lay)
    ro, rd = synth.mc_rays(128 * 128, 64, lay=lay)
    R = ro.shape[0]
    gO, gF, gD, _ = synth.upstream(R, 8)
    params = [dev(x).requires_grad_(True) for x in sc.astuple()]
    scene = Scene(*[p.detach() for p in params])
    scene.set_params(*params)
    ro_d, rd_d, g = dev(ro), dev(rd), [dev(x) for x in (gO, gF, gD)]
    cfg = TraceConfig(k=16, hit_cap=128)
    note("TraceFn loop, 30 steps")
    was = gc.isenabled()
    gc.disable()
    try:
        base = None
        for step in range(30):
            for p in params:
                p.grad = None
            O, Fo, D = TraceFn.apply(*params, ro_d, rd_d, scene, cfg)
            torch.autograd.backward([O, Fo, D], g)
            del O, Fo, D
            torch.cuda.synchronize()
            used = torch.cuda.memory_allocated()
            if base is None:
                base = used
            assert used == base, f"step {step}: {used - base} bytes more in use than after step 0"
    finally:
        if was:
            gc.enable()
    scene.close()
