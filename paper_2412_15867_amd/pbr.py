"""Monte Carlo rendering-equation consumer of the trace (Sec. 3.3,
"Rendering"): stratified hemisphere rays per pixel, the differentiable
trace for visibility and indirect radiance (Eq. 13-14), and Eq. 15 with the
dielectric BRDF of Eq. 4.  Argument marshalling over include/irgs.h
(`irgs_mc_rays`, `irgs_mc_shade`, `irgs_mc_shade_backward`); every step runs
in libirgs.so.

    ro, rd = mc_rays(x, n, u, S_t, S_p)                   # (P N, 3) each
    O, F, _ = TraceFn.apply(*params, ro, rd, scene, cfg)  # visibility, L_ind
    c = ShadeFn.apply(albedo, rough, env, O.view(P, N), F.view(P, N, 3), n, wo, rd.view(P, N, 3))

or ``render_pbr(...)`` for the three together.
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


def _shade_in(n, wo, albedo, rough, wi, O, Lind, env):
    P, N = wi.shape[0], wi.shape[1]
    E = env.shape[1]
    dev = wi.device
    for t, name, shape in ((n, "n", (P, 3)), (wo, "wo", (P, 3)), (albedo, "albedo", (P, 3)), (rough, "rough", (P,)),
                           (wi, "wi", (P, N, 3)), (O, "O", (P, N)), (Lind, "Lind", (P, N, 3)),
                           (env, "env", (6, E, E, 3))):
        _req(t, name, shape, device=dev)
    return _lib.ShadeIn(P, N, E, *(t.data_ptr() for t in (n, wo, albedo, rough, wi, O, Lind, env)))


def shade(n, wo, albedo, rough, wi, O, Lind, env) -> torch.Tensor:
    """Eq. 15 per pixel: (P, 3).  wi (P, N, 3) are the rays' directions, O
    (P, N) and Lind (P, N, 3) the trace's opacity and colour per ray, env the
    (6, E, E, 3) cubemap of the direct light."""
    si = _shade_in(n, wo, albedo, rough, wi, O, Lind, env)
    c = torch.empty((wi.shape[0], 3), dtype=torch.float32, device=wi.device)
    with torch.cuda.device(wi.device):
        check(_lib.lib().irgs_mc_shade(ctypes.byref(si), _ptr(c), _stream_handle(wi.device)), "irgs_mc_shade")
    return c


def shade_backward(n, wo, albedo, rough, wi, O, Lind, env, g_c) -> dict:
    """Gradients of sum(g_c * c): albedo, rough, env (zero-initialised here),
    and the upstream gradients O, Lind of the trace outputs."""
    si = _shade_in(n, wo, albedo, rough, wi, O, Lind, env)
    _req(g_c, "g_c", (wi.shape[0], 3), device=wi.device)
    g = dict(albedo=torch.zeros_like(albedo), rough=torch.zeros_like(rough), env=torch.zeros_like(env),
             O=torch.empty_like(O), Lind=torch.empty_like(Lind))
    sg = _lib.ShadeGrads(*(g[k].data_ptr() for k in ("albedo", "rough", "env", "O", "Lind")))
    with torch.cuda.device(wi.device):
        check(_lib.lib().irgs_mc_shade_backward(ctypes.byref(si), _ptr(g_c), ctypes.byref(sg),
                                                _stream_handle(wi.device)), "irgs_mc_shade_backward")
    return g


class ShadeFn(torch.autograd.Function):
    """Differentiable Eq. 15: (albedo, rough, env, O, Lind, n, wo, wi) -> c;
    gradients reach albedo, roughness, the cubemap and, through O and Lind,
    the trace."""

    @staticmethod
    def forward(ctx, albedo, rough, env, O, Lind, n, wo, wi):
        args = [t.detach().contiguous() for t in (n, wo, albedo, rough, wi, O, Lind, env)]
        ctx.save_for_backward(*args)
        return shade(*args)

    @staticmethod
    def backward(ctx, g_c):
        n, wo, albedo, rough, wi, O, Lind, env = ctx.saved_tensors
        g = shade_backward(n, wo, albedo, rough, wi, O, Lind, env, g_c.contiguous())
        return g["albedo"], g["rough"], g["env"], g["O"], g["Lind"], None, None, None


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
