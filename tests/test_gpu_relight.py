"""Relighting variant (the paper's relighting details): the trace blending
albedo, roughness and the ray-facing normal, the pre-integrated sky and BRDF
table, and the split-sum indirect radiance, against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import relight as orl
from paper_2412_15867_amd import synth
from gpu_util import dev, make_scene, note, to_np
from validate import validate

pytestmark = pytest.mark.gpu

F32 = np.float32


def material_cube():
    """Cube scene whose 4 features are albedo (3) and roughness."""
    sc = synth.cube_scene(F=4)
    feat = sc.feat.copy()
    feat[:, 3] = 0.1 + 0.9 * feat[:, 3]
    return synth.Surfels(sc.mu, sc.quat, sc.scale, sc.opac, feat.astype(F32))


def test_prefilter_and_table_match_oracle():
    from paper_2412_15867_amd import brdf_table, env_prefilter
    E, M, S = 8, 4, 16
    env = np.random.default_rng(90).uniform(0, 3, (6, E, E, 3)).astype(F32)
    note("prefilter + table")
    irr, pref = env_prefilter(dev(env), M)
    tab = brdf_table(S)
    torch.cuda.synchronize()
    np.testing.assert_allclose(irr.cpu().numpy(), orl.irradiance(env), rtol=2e-5)
    # FP32 weighted means of 384 texels against FP64
    np.testing.assert_allclose(pref.cpu().numpy(), orl.prefilter(env, M), rtol=1e-4)
    np.testing.assert_allclose(tab.cpu().numpy(), orl.brdf_table(S), atol=2e-6)


def test_normal_channels_match_oracle_and_brute_force():
    from paper_2412_15867_amd import TraceConfig, trace
    surf = material_cube()
    ro, rd = synth.pinhole_rays(64, 64)
    note("trace with normals")
    scene = make_scene(surf)
    g = to_np(trace(scene, dev(ro), dev(rd), TraceConfig(k=16, normals=True), hit_cap=256))
    b = to_np(trace(scene, dev(ro), dev(rd), TraceConfig(k=16, normals=True, brute_force=True), hit_cap=256))
    scene.close()
    assert g["F"].shape == (ro.shape[0], 7)
    for key in ("O", "F", "D", "T", "n_hits"):
        assert np.array_equal(g[key], b[key]), key
    validate(surf.astuple(), ro, rd, g, with_normal=True)


def test_relight_lind_matches_oracle():
    from paper_2412_15867_amd import TraceConfig, brdf_table, env_prefilter, relight_lind, trace
    surf = material_cube()
    ro, rd = synth.pinhole_rays(64, 64)
    env = np.random.default_rng(91).uniform(0, 3, (6, 16, 16, 3)).astype(F32)
    note("relight lind")
    scene = make_scene(surf)
    res = trace(scene, dev(ro), dev(rd), TraceConfig(k=16, normals=True))
    irr, pref = env_prefilter(dev(env), 4)
    tab = brdf_table(16)
    lind = relight_lind(res.opacity, res.feat, dev(rd), irr, pref, tab).cpu().numpy()
    O, Fo = res.opacity.cpu().numpy(), res.feat.cpu().numpy()
    scene.close()
    want = orl.relight_lind(O, Fo, rd, irr.cpu().numpy().astype(np.float64), pref.cpu().numpy().astype(np.float64),
                            tab.cpu().numpy().astype(np.float64))
    assert np.all(np.isfinite(lind))
    np.testing.assert_array_equal(lind[O == 0], 0)
    # the nearest texel / level / cell is an integer decided by floating point
    # from the normalised blend: allow the rare ray whose FP32 decision lands
    # on the other side of a boundary
    ok = np.all(np.abs(lind - want) <= 1e-4 * (1 + np.abs(want)), axis=1)
    assert ok.mean() > 0.995, ok.mean()


def test_relight_chain_and_errors():
    from paper_2412_15867_amd import TraceConfig, _lib, relight, trace, trace_backward
    surf = material_cube()
    P, St, Sp = 32, 4, 8
    px = synth.shading_pixels(P, St * Sp)
    scene = make_scene(surf)
    c = relight(scene, *(dev(0.5 * px[k] if k == "x" else px[k]) for k in ("x", "n", "wo", "albedo", "rough", "env", "u")),
                St, Sp)
    torch.cuda.synchronize()
    assert c.shape == (P, 3) and torch.isfinite(c).all()
    ro, rd = synth.pinhole_rays(8, 8)
    res = trace(scene, dev(ro), dev(rd), TraceConfig(k=16, normals=True), hit_cap=16)
    with pytest.raises(_lib.IrgsError):       # forward only
        trace_backward(scene, dev(ro), dev(rd), res, dev(np.ones(64, F32)), None, None,
                       cfg=TraceConfig(k=16, normals=True))
    with pytest.raises(_lib.IrgsError):       # SH and normals are exclusive (and 4 features are no SH set)
        trace(scene, dev(ro), dev(rd), TraceConfig(k=16, normals=True, sh=True))
    scene.close()
