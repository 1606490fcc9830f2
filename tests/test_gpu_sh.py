"""View-dependent colour inside the trace (Sec. 3.1: colours modelled by
spherical harmonics; Sec. 3.3: the trace composites that colour and is
differentiable): HIP forward and backward with IRGS_FLAG_SH against the FP64
oracle run with the same SH reading."""

import numpy as np
import pytest
import torch

from oracle import grad as ograd
from paper_2412_15867_amd import synth
from gpu_util import dev, make_scene, note, to_np
from validate import validate

pytestmark = pytest.mark.gpu

NAMES = (("mu", "mu"), ("quat", "quat"), ("scale", "scale"), ("opacity", "opac"), ("feat", "feat"))


def sh_cube(deg):
    sc = synth.cube_scene()
    k = synth.sh_coefficients(sc.n, deg)
    return synth.Surfels(sc.mu, sc.quat, sc.scale, sc.opac, k)


@pytest.fixture(scope="module")
def rays():
    return synth.pinhole_rays(64, 64)


def run(surf, ro, rd, hit_cap=256, **kw):
    from paper_2412_15867_amd import TraceConfig, trace
    scene = make_scene(surf)
    res = trace(scene, dev(ro), dev(rd), TraceConfig(sh=True, **kw), hit_cap=hit_cap)
    torch.cuda.synchronize()
    out = to_np(res)
    scene.close()
    return out


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_sh_forward_matches_oracle(rays, deg):
    ro, rd = rays
    surf = sh_cube(deg)
    note(f"sh deg {deg} forward")
    g = run(surf, ro, rd, k=16)
    assert g["F"].shape == (ro.shape[0], 3)
    st = validate(surf.astuple(), ro, rd, g, sh_deg=deg)
    assert st["exact_eligible"] > 0.9 * st["rays"]


def test_sh_brute_force_bvh_and_k_bitwise(rays):
    ro, rd = rays
    surf = sh_cube(3)
    note("sh brute vs bvh vs k=32, 64")
    a = run(surf, ro, rd, k=16, brute_force=True)
    b = run(surf, ro, rd, k=16)
    c = run(surf, ro, rd, k=32)
    e = run(surf, ro, rd, k=64)
    for key in ("O", "F", "D", "T", "n_hits"):
        assert np.array_equal(a[key], b[key]), key
        assert np.array_equal(b[key], c[key]), key
        assert np.array_equal(b[key], e[key]), key


def test_sh_degree0_is_a_constant_colour(rays):
    """With only the constant term the colour is max(k0 / (2 sqrt(pi)) + 1/2, 0)
    for every direction: the same as plain features holding that colour."""
    from paper_2412_15867_amd import TraceConfig, trace
    ro, rd = rays
    surf = sh_cube(0)
    col = np.maximum(surf.feat.astype(np.float64) * (0.5 / np.sqrt(np.pi)) + 0.5, 0.0).astype(np.float32)
    plain = synth.Surfels(surf.mu, surf.quat, surf.scale, surf.opac, col)
    a = run(surf, ro, rd, k=16)
    scene = make_scene(plain)
    b = to_np(trace(scene, dev(ro), dev(rd), TraceConfig(k=16), hit_cap=256))
    scene.close()
    for key in ("O", "D", "T", "n_hits"):
        assert np.array_equal(a[key], b[key]), key
    np.testing.assert_allclose(a["F"], b["F"], atol=2e-6)


def grad_close(g_gpu, g_ref, rel=1e-3):
    for name, key in NAMES:
        a = g_gpu[name].reshape(g_ref[key].shape)
        b = g_ref[key]
        floor = np.abs(b).mean() + 1e-30
        err = np.abs(a - b) / (np.abs(b) + floor)
        assert err.max() <= rel, (name, err.max())


@pytest.mark.parametrize("deg", [0, 1, 3])
@pytest.mark.parametrize("recompute", [False, True])
def test_sh_backward_matches_fp64_oracle(rays, recompute, deg):
    """Degree 0 (F = 3) runs the SH kernel without the ray order, degrees 1
    and 3 (F = 12, 48) with it (stored lists)."""
    from paper_2412_15867_amd import TraceConfig, trace, trace_backward
    ro, rd = rays
    ro, rd = ro[::4], rd[::4]
    surf = sh_cube(deg)
    gO, gF, gD, _ = synth.upstream(ro.shape[0], 3)
    note(f"sh backward deg={deg} recompute={recompute}")
    scene = make_scene(surf)
    cfg = TraceConfig(k=16, sh=True, recompute=recompute)
    res = trace(scene, dev(ro), dev(rd), cfg, hit_cap=256)
    grads = trace_backward(scene, dev(ro), dev(rd), res, dev(gO), dev(gF), dev(gD), cfg=cfg)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy().astype(np.float64) for k, v in grads.items()}
    fwd = to_np(res)
    scene.close()
    H = fwd["hit_ids"].shape[1]
    lists = np.where(np.arange(H)[None, :] < fwd["n_hits"][:, None], fwd["hit_ids"], -1)
    ref = ograd.grad_given_hits(surf.astuple(), ro, rd, lists, gO, gF, gD, sh_deg=deg)
    grad_close(g, ref)
    assert np.abs(g["feat"]).max() > 0


def test_sh_autograd_function(rays):
    from paper_2412_15867_amd import Scene, TraceConfig, TraceFn, trace, trace_backward
    ro, rd = rays
    surf = sh_cube(2)
    params = [dev(x).requires_grad_(True) for x in surf.astuple()]
    scene = Scene(*[p.detach() for p in params])
    scene.set_params(*params)
    cfg = TraceConfig(k=16, sh=True)
    O, F, D = TraceFn.apply(*params, dev(ro), dev(rd), scene, cfg)
    assert F.shape == (ro.shape[0], 3)
    gO, gF, gD, _ = synth.upstream(ro.shape[0], 3, seed=50)
    (O * dev(gO)).sum().backward(retain_graph=True)
    g1 = params[4].grad.clone()
    for p in params:
        p.grad = None
    (F * dev(gF)).sum().backward()
    res = trace(scene, dev(ro), dev(rd), cfg, hit_cap=64)
    ref = trace_backward(scene, dev(ro), dev(rd), res, None, dev(gF), None, cfg=cfg)
    torch.cuda.synchronize()
    # the two launches add the same per-hit terms with FP32 atomics, in
    # different orders
    torch.testing.assert_close(params[4].grad, ref["feat"], rtol=1e-4, atol=1e-6)
    assert torch.count_nonzero(g1) == 0     # opacity upstream alone: no colour gradient
    scene.close()


def test_sh_argument_errors(rays):
    from paper_2412_15867_amd import TraceConfig, trace, trace_packed, alloc_result
    from paper_2412_15867_amd import _lib
    ro, rd = rays
    sc = synth.cube_scene(F=8)                 # 8 features are not an SH set
    scene = make_scene(sc)
    with pytest.raises(_lib.IrgsError):
        trace(scene, dev(ro), dev(rd), TraceConfig(k=16, sh=True))
    scene.close()
    scene = make_scene(sh_cube(1))
    with pytest.raises(_lib.IrgsError):
        trace(scene, dev(ro), dev(rd), TraceConfig(k=8, sh=True))   # SH: k = 16, 32 or 64
    with pytest.raises(ValueError):
        trace_packed([scene], [(0, dev(ro), dev(rd), alloc_result(ro.shape[0], 3, scene.device))],
                     TraceConfig(k=16, sh=True))
    scene.close()
