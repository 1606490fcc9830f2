"""FP64 oracle of 2D Gaussian ray tracing (2DGRT, Sec. 3.2 of the paper).

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library and never calls it.

* ``trace``       -- brute force: every ray against every surfel, hits sorted
                     by (depth, index), front-to-back compositing with the
                     transmittance cutoff (Eq. 2, 6, 7, 8).  C, FP64, OpenMP.
* ``candidates``  -- every surfel whose plane the ray crosses inside
                     (t_min, t_max), with its FP64 depth, u^2+v^2 and alpha.
* ``replay``      -- FP64 compositing of a given ordered hit list.
* ``frames``      -- tangent frame (t_u, t_v, n) of each quaternion.
* ``with_normal``  -- (trace / replay option) 3 more composited channels: each
                     hit's unit normal turned to face the ray (relighting).
* ``sh_basis``    -- real spherical-harmonic basis of directions (degree <= 3),
                     by the associated-Legendre recurrence; with ``sh_deg`` >= 0
                     ``trace`` / ``replay`` read the features as RGB SH
                     coefficients and composite the view-dependent colour
                     max(Y(d).k + 1/2, 0) (3 output channels).
* ``grad``        -- (submodule) FP64 autograd gradients over a given hit list
                     and central finite differences.
* ``shade``       -- (submodule) the Monte Carlo rendering-equation consumer
                     of the trace (Eq. 15 with Eq. 13-14 and Eq. 4): stratified
                     hemisphere directions, cubemap lookup, shading, gradients.

Inputs may be FP32 arrays; they are widened to FP64 exactly.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "trace_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

DEFAULTS = dict(alpha_min=1.0 / 255.0, T_min=1e-4, t_min=0.0, t_max=float("inf"), sigma=3.0, sh_deg=-1,
                with_normal=0)


class Params(ctypes.Structure):
    _fields_ = [("alpha_min", ctypes.c_double), ("T_min", ctypes.c_double),
                ("t_min", ctypes.c_double), ("t_max", ctypes.c_double), ("sigma", ctypes.c_double),
                ("sh_deg", ctypes.c_int32), ("with_normal", ctypes.c_int32)]


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        L.orc_trace.argtypes = [i64, i32, P, P, P, P, P, i64, P, P, ctypes.POINTER(Params),
                                P, P, P, P, P, i32, P, i32]
        L.orc_trace.restype = ctypes.c_int
        L.orc_candidates.argtypes = [i64, P, P, P, P, i64, P, P, ctypes.POINTER(Params), ctypes.c_double, i32,
                                     P, P, P, P, P, P, i32]
        L.orc_candidates.restype = ctypes.c_int
        L.orc_replay.argtypes = [i64, i32, P, P, P, P, P, i64, P, P, i32, P, P,
                                 P, P, P, P, P, P, P, i32, i32, i32]
        L.orc_replay.restype = ctypes.c_int
        L.orc_sh_basis.argtypes = [i64, P, i32, P]
        L.orc_sh_basis.restype = None
        L.orc_surfel_frames.argtypes = [i64, P, P, P, P]
        L.orc_surfel_frames.restype = None
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_params(**kw) -> Params:
    d = dict(DEFAULTS)
    d.update({k: v for k, v in kw.items() if k in d})
    return Params(d["alpha_min"], d["T_min"], d["t_min"], d["t_max"], d["sigma"], int(d["sh_deg"]),
                  int(bool(d["with_normal"])))


def out_channels(F: int, sh_deg: int) -> int:
    """Composited feature channels: 3 colours in SH mode, else F."""
    if sh_deg >= 0:
        if F != 3 * (sh_deg + 1) ** 2:
            raise ValueError(f"SH degree {sh_deg} needs {3 * (sh_deg + 1) ** 2} features, got {F}")
        return 3
    return F


def _surfels(s):
    mu, quat, scale, opac, feat = (_d(a) for a in s)
    if feat.ndim != 2:
        feat = feat.reshape(mu.shape[0], -1)
    return mu, quat, scale, opac.reshape(-1), feat


def max_threads() -> int:
    return int(lib().orc_max_threads())


def trace(surfels, ro, rd, hit_cap: int = 0, nthreads: int = 0, **kw):
    """Brute-force FP64 trace.  `surfels` = (mu, quat, scale, opac, feat)."""
    mu, quat, scale, opac, feat = _surfels(surfels)
    ro, rd = _d(ro).reshape(-1, 3), _d(rd).reshape(-1, 3)
    N, F, R = mu.shape[0], feat.shape[1], ro.shape[0]
    O, D, T = np.zeros(R), np.zeros(R), np.ones(R)
    prm = make_params(**kw)
    Fo = np.zeros((R, out_channels(F, prm.sh_deg) + (3 if prm.with_normal else 0)))
    nh = np.zeros(R, dtype=np.int32)
    hits = np.full((R, max(hit_cap, 1)), -1, dtype=np.int32)
    rc = lib().orc_trace(N, F, _p(mu), _p(quat), _p(scale), _p(opac), _p(feat), R, _p(ro), _p(rd),
                         ctypes.byref(prm), _p(O), _p(Fo), _p(D), _p(T), _p(nh), hit_cap,
                         _p(hits) if hit_cap > 0 else None, nthreads)
    if rc != 0:
        raise MemoryError("oracle trace failed")
    out = dict(O=O, F=Fo, D=D, T=T, n_hits=nh)
    if hit_cap > 0:
        out["hits"] = hits
    return out


def candidates(surfels, ro, rd, cap: int = 512, band: float = 1e-2, nthreads: int = 0, **kw):
    """Hits and near-hits (within relative `band` of the support or alpha_min
    threshold) of each ray, in surfel order."""
    mu, quat, scale, opac, _ = _surfels(surfels)
    ro, rd = _d(ro).reshape(-1, 3), _d(rd).reshape(-1, 3)
    N, R = mu.shape[0], ro.shape[0]
    ids = np.full((R, cap), -1, dtype=np.int32)
    tau = np.zeros((R, cap))
    rho2 = np.zeros((R, cap))
    alpha = np.zeros((R, cap))
    hit = np.zeros((R, cap), dtype=np.int8)
    cnt = np.zeros(R, dtype=np.int32)
    prm = make_params(**kw)
    lib().orc_candidates(N, _p(mu), _p(quat), _p(scale), _p(opac), R, _p(ro), _p(rd), ctypes.byref(prm),
                         band, cap, _p(ids), _p(tau), _p(rho2), _p(alpha), _p(hit), _p(cnt), nthreads)
    return dict(ids=ids, tau=tau, rho2=rho2, alpha=alpha, hit=hit.astype(bool), count=cnt)


def replay(surfels, ro, rd, lists, lengths, nthreads: int = 0, sh_deg: int = -1, with_normal: bool = False):
    """Composite the given ordered lists (R, H) int32 of length `lengths`."""
    mu, quat, scale, opac, feat = _surfels(surfels)
    ro, rd = _d(ro).reshape(-1, 3), _d(rd).reshape(-1, 3)
    lists = np.ascontiguousarray(lists, dtype=np.int32)
    lengths = np.ascontiguousarray(lengths, dtype=np.int32)
    N, F, R = mu.shape[0], feat.shape[1], ro.shape[0]
    H = lists.shape[1]
    O, D, T = np.zeros(R), np.zeros(R), np.ones(R)
    Fo = np.zeros((R, out_channels(F, sh_deg) + (3 if with_normal else 0)))
    Tpost = np.ones((R, H))
    tau = np.zeros((R, H))
    alpha = np.zeros((R, H))
    lib().orc_replay(N, F, _p(mu), _p(quat), _p(scale), _p(opac), _p(feat), R, _p(ro), _p(rd), H,
                     _p(lists), _p(lengths), _p(O), _p(Fo), _p(D), _p(T), _p(Tpost), _p(tau), _p(alpha),
                     int(sh_deg), int(bool(with_normal)), nthreads)
    return dict(O=O, F=Fo, D=D, T=T, Tpost=Tpost, tau=tau, alpha=alpha)


def frames(quat):
    quat = _d(quat).reshape(-1, 4)
    N = quat.shape[0]
    tu, tv, n = np.zeros((N, 3)), np.zeros((N, 3)), np.zeros((N, 3))
    lib().orc_surfel_frames(N, _p(quat), _p(tu), _p(tv), _p(n))
    return tu, tv, n


def sh_basis(dirs, deg: int) -> np.ndarray:
    """Real SH basis Y[l*l + l + m] (R, (deg+1)^2) of the normalised directions."""
    dirs = _d(dirs).reshape(-1, 3)
    Y = np.zeros((dirs.shape[0], (deg + 1) ** 2))
    lib().orc_sh_basis(dirs.shape[0], _p(dirs), int(deg), _p(Y))
    return Y
