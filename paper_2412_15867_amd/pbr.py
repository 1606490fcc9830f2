"""Monte Carlo rendering-equation consumer of the trace (Sec. 3.3,
"Rendering"): stratified hemisphere rays per pixel, the differentiable
trace for visibility and indirect radiance (Eq. 13-14), and Eq. 15 with the
dielectric BRDF of Eq. 4.  Argument marshalling over include/irgs.h
(`irgs_mc_rays`, `irgs_mc_shade`, `irgs_mc_shade_backward`); every step runs
in libirgs.so.

    ro, rd = mc_rays(x, n, u, S_t, S_p)                   # (P N, 3) each
    O, F, _ = TraceFn.apply(*params, ro, rd, scene, cfg)  # visibility, L_ind
    c = ShadeFn.apply(albedo, rough, env, O.view(P, N), F.view(P, N, 3), n, wo, rd.view(P, N, 3))

or ``render_pbr(...)`` for the three together.  Relighting (forward only):
``env_prefilter`` / ``brdf_table`` pre-integrate the sky and the BRDF,
``relight_lind`` shades each ray's blended albedo / roughness / normal
(a trace with ``TraceConfig(normals=True)``) with the split-sum
approximation, ``env_cdf`` / ``env_rays`` draw incident directions by the
sky's intensity (weights 1 / (N pdf) for ``shade``), and ``relight(...)``
chains rays, trace, that and Eq. 15.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib
from ._lib import check
from .tracer import Scene, TraceConfig, TraceFn, _ptr, _req, _stream_handle


def mc_rays(x: torch.Tensor, n: torch.Tensor, u: torch.Tensor, S_t: int, S_p: int, offset: float = 1e-3):
    """Rays of N = S_t * S_p stratified hemisphere samples per pixel: origin
    x + offset n, direction from the uniforms u (P, N, 2) about the unit
    normals n (P, 3).  Returns (ro, rd), each (P N, 3), ray p N + i."""
    P = x.shape[0]
    N = int(S_t) * int(S_p)
    dev = x.device
    _req(x, "x", (P, 3), device=dev)
    _req(n, "n", (P, 3), device=dev)
    _req(u, "u", (P, N, 2), device=dev)
    ro = torch.empty((P * N, 3), dtype=torch.float32, device=dev)
    rd = torch.empty((P * N, 3), dtype=torch.float32, device=dev)
    with torch.cuda.device(dev):
        check(_lib.lib().irgs_mc_rays(P, int(S_t), int(S_p), _ptr(x), _ptr(n), _ptr(u), float(offset), _ptr(ro),
                                      _ptr(rd), _stream_handle(dev)), "irgs_mc_rays")
    return ro, rd


def _shade_in(n, wo, albedo, rough, wi, O, Lind, env, wgt=None):
    P, N = wi.shape[0], wi.shape[1]
    E = env.shape[1]
    dev = wi.device
    for t, name, shape in ((n, "n", (P, 3)), (wo, "wo", (P, 3)), (albedo, "albedo", (P, 3)), (rough, "rough", (P,)),
                           (wi, "wi", (P, N, 3)), (O, "O", (P, N)), (Lind, "Lind", (P, N, 3)),
                           (env, "env", (6, E, E, 3))):
        _req(t, name, shape, device=dev)
    if wgt is not None:
        _req(wgt, "wgt", (P, N), device=dev)
    return _lib.ShadeIn(P, N, E, *(t.data_ptr() for t in (n, wo, albedo, rough, wi, O, Lind, env)),
                        None if wgt is None else wgt.data_ptr())


def shade(n, wo, albedo, rough, wi, O, Lind, env, wgt=None) -> torch.Tensor:
    """Eq. 15 per pixel: (P, 3).  wi (P, N, 3) are the rays' directions, O
    (P, N) and Lind (P, N, 3) the trace's opacity and colour per ray, env the
    (6, E, E, 3) cubemap of the direct light; wgt (P, N) optional per-sample
    weights 1 / (N pdf) of another sampling density (default 2 pi / N)."""
    si = _shade_in(n, wo, albedo, rough, wi, O, Lind, env, wgt)
    c = torch.empty((wi.shape[0], 3), dtype=torch.float32, device=wi.device)
    with torch.cuda.device(wi.device):
        check(_lib.lib().irgs_mc_shade(ctypes.byref(si), _ptr(c), _stream_handle(wi.device)), "irgs_mc_shade")
    return c


def shade_backward(n, wo, albedo, rough, wi, O, Lind, env, g_c, wgt=None) -> dict:
    """Gradients of sum(g_c * c): albedo, rough, env (zero-initialised here),
    and the upstream gradients O, Lind of the trace outputs."""
    si = _shade_in(n, wo, albedo, rough, wi, O, Lind, env, wgt)
    _req(g_c, "g_c", (wi.shape[0], 3), device=wi.device)
    g = dict(albedo=torch.zeros_like(albedo), rough=torch.zeros_like(rough), env=torch.zeros_like(env),
             O=torch.empty_like(O), Lind=torch.empty_like(Lind))
    sg = _lib.ShadeGrads(*(g[k].data_ptr() for k in ("albedo", "rough", "env", "O", "Lind")))
    with torch.cuda.device(wi.device):
        check(_lib.lib().irgs_mc_shade_backward(ctypes.byref(si), _ptr(g_c), ctypes.byref(sg),
                                                _stream_handle(wi.device)), "irgs_mc_shade_backward")
    return g


class ShadeFn(torch.autograd.Function):
    """Differentiable Eq. 15: (albedo, rough, env, O, Lind, n, wo, wi[, wgt])
    -> c; gradients reach albedo, roughness, the cubemap and, through O and
    Lind, the trace (the sampling weights are constants)."""

    @staticmethod
    def forward(ctx, albedo, rough, env, O, Lind, n, wo, wi, wgt=None):
        args = [t.detach().contiguous() for t in (n, wo, albedo, rough, wi, O, Lind, env)]
        w = None if wgt is None else wgt.detach().contiguous()
        ctx.save_for_backward(*args, w)
        return shade(*args, wgt=w)

    @staticmethod
    def backward(ctx, g_c):
        n, wo, albedo, rough, wi, O, Lind, env, w = ctx.saved_tensors
        g = shade_backward(n, wo, albedo, rough, wi, O, Lind, env, g_c.contiguous(), wgt=w)
        return g["albedo"], g["rough"], g["env"], g["O"], g["Lind"], None, None, None, None


def render_pbr(scene: Scene, params, x, n, wo, albedo, rough, env, u, S_t: int, S_p: int,
               cfg: Optional[TraceConfig] = None, offset: float = 1e-3):
    """c_pbr (P, 3) of Eq. 15: stratified rays, the differentiable trace
    (colour channels = L_ind, opacity = 1 - V) and the shading.  `params` =
    the scene's own (mu, quat, scale, opacity, feat) tensors; the trace must
    composite 3 channels (RGB features, or SH colour with cfg.sh)."""
    cfg = cfg or TraceConfig()
    P = x.shape[0]
    N = int(S_t) * int(S_p)
    ro, rd = mc_rays(x, n, u, S_t, S_p, offset)
    O, F, _ = TraceFn.apply(*params, ro, rd, scene, cfg)
    if F.shape[1] != 3:
        raise ValueError("render_pbr needs a 3-channel trace colour")
    return ShadeFn.apply(albedo, rough, env, O.view(P, N), F.view(P, N, 3), n, wo, rd.view(P, N, 3))


# ---- relighting variant (forward only) -------------------------------------

def env_prefilter(env: torch.Tensor, M: int = 8):
    """Irradiance (6, E, E, 3) and GGX-prefiltered skies (M, 6, E, E, 3) of
    the cubemap env (6, E, E, 3), roughness levels (l + 1) / M."""
    E = env.shape[1]
    _req(env, "env", (6, E, E, 3), device=env.device)
    irr = torch.empty_like(env)
    pref = torch.empty((M, 6, E, E, 3), dtype=torch.float32, device=env.device)
    with torch.cuda.device(env.device):
        check(_lib.lib().irgs_env_prefilter(E, _ptr(env), int(M), _ptr(irr), _ptr(pref), _stream_handle(env.device)),
              "irgs_env_prefilter")
    return irr, pref


def brdf_table(S: int = 32, device=None) -> torch.Tensor:
    """Split-sum table (S, S, 2) at cell centres (n.v, roughness)."""
    device = device or torch.device("cuda:0")
    t = torch.empty((S, S, 2), dtype=torch.float32, device=device)
    with torch.cuda.device(device):
        check(_lib.lib().irgs_brdf_table(int(S), _ptr(t), _stream_handle(device)), "irgs_brdf_table")
    return t


def relight_lind(O, Fo, rd, irr, pref, table) -> torch.Tensor:
    """Split-sum indirect radiance (R, 3) of each ray from the trace outputs
    of IRGS_FLAG_NORMAL (O (R), Fo (R, 7) = albedo, roughness, normal)."""
    R = O.shape[0]
    dev = O.device
    E, M, S = irr.shape[1], pref.shape[0], table.shape[0]
    for t, name, shape in ((O, "O", (R,)), (Fo, "Fo", (R, 7)), (rd, "rd", (R, 3)), (irr, "irr", (6, E, E, 3)),
                           (pref, "pref", (M, 6, E, E, 3)), (table, "table", (S, S, 2))):
        _req(t, name, shape, device=dev)
    out = torch.empty((R, 3), dtype=torch.float32, device=dev)
    with torch.cuda.device(dev):
        check(_lib.lib().irgs_relight_lind(R, _ptr(O), _ptr(Fo), _ptr(rd), E, _ptr(irr), M, _ptr(pref), S,
                                           _ptr(table), _ptr(out), _stream_handle(dev)), "irgs_relight_lind")
    return out


def env_cdf(env: torch.Tensor) -> torch.Tensor:
    """(6 E^2,) FP32 CDF of the sky's texel weights (mean RGB x solid
    angle), in texel order, for env_rays."""
    E = env.shape[1]
    _req(env, "env", (6, E, E, 3), device=env.device)
    cdf = torch.empty(6 * E * E, dtype=torch.float32, device=env.device)
    with torch.cuda.device(env.device):
        check(_lib.lib().irgs_env_cdf(E, _ptr(env), _ptr(cdf), _stream_handle(env.device)), "irgs_env_cdf")
    return cdf


def env_rays(x: torch.Tensor, n: torch.Tensor, u: torch.Tensor, cdf: torch.Tensor, E: int, offset: float = 1e-3):
    """Rays drawn from the sky's intensity: uniforms u (P, N, 3) in [0, 1).
    Returns ro, rd (P N, 3) and the estimator weights (P, N) = 1 / (N pdf),
    0 below the horizon."""
    P, N = u.shape[0], u.shape[1]
    dev = x.device
    _req(x, "x", (P, 3), device=dev)
    _req(n, "n", (P, 3), device=dev)
    _req(u, "u", (P, N, 3), device=dev)
    _req(cdf, "cdf", (6 * E * E,), device=dev)
    ro = torch.empty((P * N, 3), dtype=torch.float32, device=dev)
    rd = torch.empty((P * N, 3), dtype=torch.float32, device=dev)
    w = torch.empty((P, N), dtype=torch.float32, device=dev)
    with torch.cuda.device(dev):
        check(_lib.lib().irgs_env_rays(P, N, _ptr(x), _ptr(n), _ptr(u), int(E), _ptr(cdf), float(offset), _ptr(ro),
                                       _ptr(rd), _ptr(w), _stream_handle(dev)), "irgs_env_rays")
    return ro, rd, w


def relight(scene: Scene, x, n, wo, albedo, rough, env, u, S_t: Optional[int] = None, S_p: Optional[int] = None,
            sampling: str = "env", irr=None, pref=None, table=None, cdf=None, k: int = 16, T_min: float = 1e-4,
            offset: float = 1e-3):
    """Relit colour (P, 3) under the sky env: incident rays, the trace
    blending each ray's albedo, roughness and normal (the scene's 4 features
    are albedo and roughness), split-sum indirect radiance, Eq. 15.
    sampling="env" (the paper's choice for relighting) draws the directions
    by the sky's intensity from uniforms u (P, N, 3); "stratified" takes the
    S_t x S_p stratified hemisphere of uniforms u (P, S_t S_p, 2)."""
    from .tracer import trace
    if irr is None or pref is None:
        irr, pref = env_prefilter(env)
    if table is None:
        table = brdf_table(device=env.device)
    P, N = u.shape[0], u.shape[1]
    if sampling == "env":
        ro, rd, wgt = env_rays(x, n, u, env_cdf(env) if cdf is None else cdf, env.shape[1], offset)
    elif sampling == "stratified":
        if S_t is None or S_p is None or int(S_t) * int(S_p) != N:
            raise ValueError("stratified sampling needs S_t * S_p = u.shape[1]")
        ro, rd = mc_rays(x, n, u, S_t, S_p, offset)
        wgt = None
    else:
        raise ValueError(f"unknown sampling {sampling!r}")
    res = trace(scene, ro, rd, TraceConfig(k=k, T_min=T_min, normals=True))
    lind = relight_lind(res.opacity, res.feat, rd, irr, pref, table)
    return shade(n, wo, albedo, rough, rd.view(P, N, 3), res.opacity.view(P, N), lind.view(P, N, 3), env, wgt)
