"""MI355X-native (gfx950) differentiable 2D Gaussian ray tracing.

Hot path of arXiv 2412.15867 (Sec. 3.2-3.3): ray-splat intersection (Eq. 6),
2D Gaussian influence (Eq. 7), k-buffer hit marching and front-to-back
compositing (Eq. 2, 8) through a software LBVH, plus the hand-written
adjoint.  The compute runs in libirgs.so (include/irgs.h); this package is
argument marshalling (``trace``), the Monte Carlo rendering-equation
consumer of the trace (``pbr``), a serving loop (``serve``) and seeded input
generators (``synth``).

Submodules are imported lazily so that ``synth`` needs neither torch nor the
HIP library.
"""
import importlib

__all__ = ["Scene", "TraceConfig", "TraceResult", "TraceFn", "trace", "trace_noalloc", "trace_backward", "trace_packed",
           "alloc_result", "synth", "serve", "mc_rays", "shade", "shade_backward", "ShadeFn", "render_pbr",
           "env_prefilter", "brdf_table", "relight_lind", "relight"]

_TRACE_NAMES = {"Scene", "TraceConfig", "TraceResult", "TraceFn", "trace", "trace_noalloc", "trace_backward", "trace_packed",
                "alloc_result"}


_PBR_NAMES = {"mc_rays", "shade", "shade_backward", "ShadeFn", "render_pbr", "env_prefilter", "brdf_table",
              "relight_lind", "relight", "env_cdf", "env_rays"}


def __getattr__(name):
    if name in _TRACE_NAMES:
        return getattr(importlib.import_module(".tracer", __name__), name)
    if name in _PBR_NAMES:
        return getattr(importlib.import_module(".pbr", __name__), name)
    if name in ("synth", "serve", "build", "tracer", "pbr"):
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
