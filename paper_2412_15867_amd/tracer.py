"""PyTorch-facing API of the gfx950 2D Gaussian ray tracer.

PyTorch provides device memory and the stream; every step of the trace runs
in libirgs.so (``_lib``).  All calls are queued on
``torch.cuda.current_stream()``.

    scene = Scene(mu, quat, scale, opacity, feat)      # builds the LBVH
    res = trace(scene, ro, rd)                          # O, F, D, T, n_hits
    O, F, D = TraceFn.apply(mu, quat, scale, opacity, feat, ro, rd, scene, cfg)

The trace is Trace(r_o, r_d) -> (c_rt, o_rt) of Sec. 3.2 (Eq. 8); used on
surface points and incident directions it gives (L_ind, 1 - V) of Eq. 14.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import check

DEFAULT_ALPHA_MIN = 1.0 / 255.0
DEFAULT_T_MIN = 1e-4
DEFAULT_SIGMA = 3.0


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _req(t: torch.Tensor, name: str, shape, dtype=torch.float32, device=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU (got {t.device}); there is no CPU path")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


@dataclasses.dataclass
class TraceConfig:
    """Trace parameters (see irgs_params in include/irgs.h).  ``k`` (the
    k-buffer size of Sec. 3.2, the paper's 16) changes only the number of
    marching rounds, never the result; on gfx950 k = 32 runs as fast or
    faster on every workload measured, and k = 64 faster still for launches
    bound by their slowest rays and for scenes past the caches (fewer rounds
    outweigh the lower occupancy).  ``sort_rays`` hands rays to the traversal
    in the Morton order of their origins (results unchanged bit for bit)."""
    k: int = 16
    T_min: float = DEFAULT_T_MIN
    t_min: float = 0.0
    t_max: float = math.inf
    brute_force: bool = False
    recompute: bool = False      # backward: trace the rays again instead of storing hit lists
    # hits stored per ray for the backward (store mode, 8 bytes each); rays
    # with more re-march in the backward, about ten times a forward per ray,
    # so the capacity should cover nearly every ray (256 covers the 1M-surfel
    # Monte Carlo workload: at 64 its backward takes 696 ms instead of 24.5)
    hit_cap: int = 256
    sh: bool = False             # features are RGB SH coefficients (view-dependent colour, 3 channels)
    normals: bool = False        # 3 more channels, the ray-facing normal (relighting blend; differentiable)
    sort_rays: bool = False      # trace rays in the Morton order of their origins (same results)

    def flags(self) -> int:
        return ((_lib.FLAG_SH if self.sh else 0) | (_lib.FLAG_NORMAL if self.normals else 0) |
                (_lib.FLAG_SORT_RAYS if self.sort_rays else 0))

    def out_channels(self, F: int) -> int:
        """Composited feature channels for a scene with F features."""
        return 3 if self.sh else F + (3 if self.normals else 0)


class Scene:
    """A set of surfels plus its BVH.  The parameter tensors are borrowed:
    keep them alive, and call ``refit()`` after changing them in place.
    ``builder``: "ploc" (default; clustering by union surface area: fewer
    surfel tests per ray, slower build) or "radix" (Karras' radix tree over
    the Morton codes)."""

    def __init__(self, mu, quat, scale, opacity, feat, alpha_min: float = DEFAULT_ALPHA_MIN,
                 support_sigma: float = DEFAULT_SIGMA, build: bool = True, leaf_size: int = 0,
                 builder: str = "ploc"):
        n = mu.shape[0]
        F = feat.shape[1] if feat.dim() == 2 else 1
        self.device = mu.device
        self.n, self.F = int(n), int(F)
        self.alpha_min = float(alpha_min)
        self.support_sigma = float(support_sigma)
        self.leaf_size = int(leaf_size)
        if builder not in ("ploc", "radix"):
            raise ValueError(f"unknown builder {builder!r}")
        self.builder = builder
        self._set_tensors(mu, quat, scale, opacity, feat)
        h = ctypes.c_void_p()
        check(_lib.lib().irgs_scene_create(self.n, self.F, ctypes.byref(self._surfels()), ctypes.byref(h)),
              "irgs_scene_create")
        self._h = h
        self.built = False
        if build:
            self.build()

    def _set_tensors(self, mu, quat, scale, opacity, feat):
        n, dev = mu.shape[0], mu.device
        self.mu = _req(mu, "mu", (n, 3), device=dev)
        self.quat = _req(quat, "quat", (n, 4), device=dev)
        self.scale = _req(scale, "scale", (n, 2), device=dev)
        self.opacity = _req(opacity.reshape(n) if opacity.dim() == 2 else opacity, "opacity", (n,), device=dev)
        f = feat if feat.dim() == 2 else feat.reshape(n, 1)
        self.feat = _req(f, "feat", (n, self.F), device=dev)

    def _surfels(self):
        return _lib.Surfels(self.mu.data_ptr(), self.quat.data_ptr(), self.scale.data_ptr(),
                            self.opacity.data_ptr(), self.feat.data_ptr())

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("scene is closed")
        return self._h

    def params(self, cfg: TraceConfig, flags: int = 0) -> _lib.Params:
        return _lib.Params(int(cfg.k), self.F, self.alpha_min, float(cfg.T_min), float(cfg.t_min),
                           float(cfg.t_max), self.support_sigma, flags, self.leaf_size)

    def set_params(self, mu, quat, scale, opacity, feat):
        self._set_tensors(mu, quat, scale, opacity, feat)
        check(_lib.lib().irgs_scene_set_params(self.handle, ctypes.byref(self._surfels())), "irgs_scene_set_params")

    def build(self):
        with torch.cuda.device(self.device):
            p = self.params(TraceConfig(), _lib.FLAG_RADIX_TREE if self.builder == "radix" else 0)
            check(_lib.lib().irgs_scene_build(self.handle, ctypes.byref(p), _stream_handle(self.device)),
                  "irgs_scene_build")
        self.built = True

    def refit(self):
        with torch.cuda.device(self.device):
            check(_lib.lib().irgs_scene_refit(self.handle, _stream_handle(self.device)), "irgs_scene_refit")

    def info(self):
        n_int = ctypes.c_int64()
        depth = ctypes.c_int32()
        check(_lib.lib().irgs_scene_info(self.handle, ctypes.byref(n_int), ctypes.byref(depth)), "irgs_scene_info")
        return dict(n_internal=int(n_int.value), max_depth=int(depth.value))

    def export(self):
        """Tree arrays (order, nodes (N-1, 16) int32, leaf_parent) as device tensors."""
        n = self.n
        ni = max(n - 1, 1)
        order = torch.empty(n, dtype=torch.int32, device=self.device)
        nodes = torch.empty((ni, 16), dtype=torch.int32, device=self.device)
        parent = torch.empty(n, dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            check(_lib.lib().irgs_scene_export(self.handle, _ptr(order), _ptr(nodes), _ptr(parent),
                                               _stream_handle(self.device)), "irgs_scene_export")
        return order, nodes, parent

    def bytes(self) -> int:
        return int(_lib.lib().irgs_scene_bytes(self.n, self.F))

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.lib().irgs_scene_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class TraceResult:
    opacity: torch.Tensor
    feat: torch.Tensor
    depth: torch.Tensor
    T: Optional[torch.Tensor] = None
    n_hits: Optional[torch.Tensor] = None
    hit_ids: Optional[torch.Tensor] = None
    hit_T: Optional[torch.Tensor] = None
    counters: Optional[torch.Tensor] = None   # (R, 4): nodes, tests, inserts, rounds

    def out_struct(self) -> _lib.Out:
        H = 0 if self.hit_ids is None else int(self.hit_ids.shape[1])
        return _lib.Out(self.opacity.data_ptr(), self.feat.data_ptr(), self.depth.data_ptr(),
                        None if self.T is None else self.T.data_ptr(),
                        None if self.n_hits is None else self.n_hits.data_ptr(),
                        None if self.hit_ids is None else self.hit_ids.data_ptr(),
                        None if self.hit_T is None else self.hit_T.data_ptr(), H,
                        None if self.counters is None else self.counters.data_ptr())


def alloc_result(R: int, F: int, device, hit_cap: int = 0, with_T: bool = True, with_n: bool = True,
                 with_hit_T: bool = True, counters: bool = False) -> TraceResult:
    f32 = dict(dtype=torch.float32, device=device)
    res = TraceResult(
        torch.empty(R, **f32), torch.empty((R, F), **f32), torch.empty(R, **f32),
        torch.empty(R, **f32) if with_T else None,
        torch.empty(R, dtype=torch.int32, device=device) if with_n else None,
        torch.empty((R, hit_cap), dtype=torch.int32, device=device) if hit_cap > 0 else None,
        torch.empty((R, hit_cap), **f32) if (hit_cap > 0 and with_hit_T) else None)
    if counters:
        res.counters = torch.empty((R, 4), dtype=torch.int32, device=device)
    return res


def _rays(scene: Scene, ro: torch.Tensor, rd: torch.Tensor):
    R = ro.shape[0]
    _req(ro, "ro", (R, 3), device=scene.device)
    _req(rd, "rd", (R, 3), device=scene.device)
    return R


def trace(scene: Scene, ro: torch.Tensor, rd: torch.Tensor, cfg: Optional[TraceConfig] = None,
          hit_cap: int = 0, out: Optional[TraceResult] = None, counters: bool = False, **kw) -> TraceResult:
    """Forward trace of the rays (ro, rd), each (R, 3) float32 on the scene's
    device.  Returns opacity O (R), blended features (R, F), unnormalised
    depth (R), final transmittance T, n_hits and, with hit_cap > 0, the first
    hit_cap hit ids and the transmittance before each."""
    cfg = cfg or TraceConfig(**kw)
    R = _rays(scene, ro, rd)
    res = out or alloc_result(R, cfg.out_channels(scene.F), scene.device, hit_cap, counters=counters)
    flags = (_lib.FLAG_BRUTE_FORCE if cfg.brute_force else 0) | cfg.flags()
    p = scene.params(cfg, flags)
    o = res.out_struct()
    with torch.cuda.device(scene.device):
        check(_lib.lib().irgs_trace(scene.handle, ctypes.byref(p), R, _ptr(ro), _ptr(rd), ctypes.byref(o),
                                    _stream_handle(scene.device)), "irgs_trace")
    return res


def trace_noalloc(scene: Scene, ro: torch.Tensor, rd: torch.Tensor, out: TraceResult,
                  cfg: Optional[TraceConfig] = None, **kw) -> TraceResult:
    """`trace` into caller-allocated outputs through irgs_trace_noalloc: the
    library allocates nothing (its scratch is a fixed per-device array), so
    the call can sit inside HIP graph capture or an allocation-free loop.
    Calls that overlap on one GPU share that array and race."""
    cfg = cfg or TraceConfig(**kw)
    if cfg.sort_rays:
        raise ValueError("sort_rays needs a per-ray workspace: use trace()")
    R = _rays(scene, ro, rd)
    flags = (_lib.FLAG_BRUTE_FORCE if cfg.brute_force else 0) | cfg.flags()
    p = scene.params(cfg, flags)
    o = out.out_struct()
    with torch.cuda.device(scene.device):
        check(_lib.lib().irgs_trace_noalloc(scene.handle, ctypes.byref(p), R, _ptr(ro), _ptr(rd), ctypes.byref(o),
                                            _stream_handle(scene.device)), "irgs_trace_noalloc")
    return out


def trace_backward(scene: Scene, ro, rd, saved: TraceResult, g_opacity=None, g_feat=None, g_depth=None,
                   cfg: Optional[TraceConfig] = None, grads: Optional[dict] = None, **kw) -> dict:
    """Accumulate dL/d(mu, quat, scale, opacity, feat) for upstream gradients
    of (opacity, feat, depth).  Returns the gradient dict (allocated zeroed
    when not given).  Rays whose hits fit `saved`'s stored lists replay them;
    with ``cfg.recompute`` (or no stored lists) the rays are traced again in
    batches within a transient 4 GiB workspace and replayed; rays longer than
    the lists re-march, about ten times a forward per ray."""
    cfg = cfg or TraceConfig(**kw)
    R = _rays(scene, ro, rd)
    if saved.n_hits is None:
        raise ValueError("saved.n_hits is required")
    dev = scene.device
    if grads is None:
        grads = dict(mu=torch.zeros_like(scene.mu), quat=torch.zeros_like(scene.quat),
                     scale=torch.zeros_like(scene.scale), opacity=torch.zeros_like(scene.opacity),
                     feat=torch.zeros_like(scene.feat))
    gi = []
    for t, name, shape in ((g_opacity, "g_opacity", (R,)), (g_feat, "g_feat", (R, cfg.out_channels(scene.F))),
                           (g_depth, "g_depth", (R,))):
        gi.append(None if t is None else _req(t, name, shape, device=dev))
    flags = (_lib.FLAG_RECOMPUTE if cfg.recompute else 0) | cfg.flags()
    p = scene.params(cfg, flags)
    o = saved.out_struct()
    g_in = _lib.GradIn(*(None if t is None else t.data_ptr() for t in gi))
    g_out = _lib.Grads(*(None if grads.get(k) is None else grads[k].data_ptr()
                         for k in ("mu", "quat", "scale", "opacity", "feat")))
    with torch.cuda.device(dev):
        check(_lib.lib().irgs_trace_backward(scene.handle, ctypes.byref(p), R, _ptr(ro), _ptr(rd), ctypes.byref(o),
                                             ctypes.byref(g_in), ctypes.byref(g_out), _stream_handle(dev)),
              "irgs_trace_backward")
    return grads


class TraceFn(torch.autograd.Function):
    """Differentiable trace: (mu, quat, scale, opacity, feat, ro, rd) ->
    (opacity, feat, depth).  The scene must wrap the same parameter tensors
    and be built/refit for their current values.  Gradients flow to the five
    surfel tensors (not to the rays).  ``cfg.recompute`` traces the rays
    again in the backward instead of storing their hit lists from the forward
    (less memory held between the two)."""

    @staticmethod
    def forward(ctx, mu, quat, scale, opacity, feat, ro, rd, scene: Scene, cfg: Optional[TraceConfig] = None):
        cfg = cfg or TraceConfig()
        for a, b in ((mu, scene.mu), (quat, scene.quat), (scale, scene.scale), (opacity, scene.opacity),
                     (feat, scene.feat)):
            if a.data_ptr() != b.data_ptr():
                raise ValueError("TraceFn inputs must be the scene's own parameter tensors")
        hit_cap = 0 if cfg.recompute else int(cfg.hit_cap)
        res = trace(scene, ro, rd, cfg, hit_cap=hit_cap)
        ctx.scene, ctx.cfg = scene, cfg
        ctx.opacity_shape = opacity.shape
        # Everything the backward reads goes through save_for_backward, which
        # holds the returned tensors without a reference back to this node
        # and frees the lot after a backward that does not retain the graph.
        # Keeping them as ctx attributes would close a cycle (output ->
        # grad_fn -> ctx -> output) that keeps every step's hit lists alive
        # until a cyclic collection.
        ctx.save_for_backward(ro, rd, res.opacity, res.feat, res.depth, res.T, res.n_hits, res.hit_ids, res.hit_T)
        return res.opacity, res.feat, res.depth

    @staticmethod
    def backward(ctx, gO, gF, gD):
        ro, rd, O, Fo, D, T, n_hits, hit_ids, hit_T = ctx.saved_tensors
        saved = TraceResult(O, Fo, D, T, n_hits, hit_ids, hit_T)
        c = lambda t: None if t is None else t.contiguous()
        grads = trace_backward(ctx.scene, ro, rd, saved, c(gO), c(gF), c(gD), cfg=ctx.cfg)
        return (grads["mu"], grads["quat"], grads["scale"], grads["opacity"].reshape(ctx.opacity_shape),
                grads["feat"], None, None, None, None)


def trace_packed(scenes: Sequence[Scene], items: Sequence[tuple], cfg: Optional[TraceConfig] = None, **kw):
    """One persistent launch over several requests.  Each item is
    (scene_index, ro, rd, result) with ro/rd (R_i, 3) and result a
    TraceResult allocated for R_i rays and that scene's F; or
    (scene_index, ro, rd, result, begin, count): only rays
    [begin, begin + count) of the request, written at the same indices of
    its result."""
    cfg = cfg or TraceConfig(**kw)
    if not scenes:
        raise ValueError("no scenes")
    dev = scenes[0].device
    Fmax = max(s.F for s in scenes)
    if cfg.sh or cfg.normals:
        raise ValueError("SH colour and normal channels are not supported by the packed launch")
    p = _lib.Params(int(cfg.k), Fmax, scenes[0].alpha_min, float(cfg.T_min), float(cfg.t_min),
                    float(cfg.t_max), scenes[0].support_sigma, 0, 0)
    handles = (ctypes.c_void_p * len(scenes))(*[s.handle.value for s in scenes])
    works = (_lib.Work * max(len(items), 1))()
    for i, it in enumerate(items):
        si, ro, rd, res = it[:4]
        R = ro.shape[0]
        begin, count = (int(it[4]), int(it[5])) if len(it) > 4 else (0, R)
        _req(ro, "ro", (R, 3), device=dev)
        _req(rd, "rd", (R, 3), device=dev)
        if begin < 0 or count < 0 or begin + count > R:
            raise ValueError(f"item {i}: rays [{begin}, {begin + count}) outside [0, {R})")
        if res.opacity.shape[0] != R:
            raise ValueError(f"item {i}: result holds {res.opacity.shape[0]} rays, the request {R}")
        works[i].scene = int(si)
        works[i].ray_begin = begin
        works[i].ray_count = count
        works[i].ro = ro.data_ptr()
        works[i].rd = rd.data_ptr()
        works[i].out = res.out_struct()
    with torch.cuda.device(dev):
        check(_lib.lib().irgs_trace_packed(handles, len(scenes), ctypes.byref(p), works, len(items),
                                           _stream_handle(dev)), "irgs_trace_packed")
