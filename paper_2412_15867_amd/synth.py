"""Seeded synthetic inputs for the 2D Gaussian ray tracer.

This module only *draws inputs*: surfel parameters, rays and upstream
gradients.  It holds none of the tracer's arithmetic (no intersection, no
influence, no compositing), so that both the FP64 oracle and the GPU path can
be fed from it without sharing any of the method.

Every generator uses ``numpy.random.Generator(PCG64(seed))``, works in FP64
and casts once to FP32.  Arrays are C-contiguous, row-major:

    mu     (N, 3) float32   surfel centres
    quat   (N, 4) float32   rotation quaternion, (w, x, y, z)
    scale  (N, 2) float32   (s_u, s_v)
    opac   (N,)   float32   opacity o in [0, 1]
    feat   (N, F) float32   per-surfel features (RGB or RGB+albedo+rough+metal)
    ro, rd (R, 3) float32   ray origins and unit directions

The workloads stand in for the paper's datasets (Synthetic4Relight, TensoIR,
Stanford-ORB), which are not available: surfels tangent to surfaces as in a
converged 2DGS object (Sec. 3.2), cosine-weighted hemisphere rays leaving
surface points as in the Monte Carlo estimate of the rendering equation
(Eq. 15 and the composited-scene appendix), and a pinhole camera for the small
forward case.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Seeds of the standard workloads (fixed so that every run sees the same data).
SEED_CUBE = 24121          # 4,096-surfel cube scene and its 64x64 camera
SEED_LAYOUT = 24122        # placement of the spheres and planes
SEED_MC_RAYS = 24123       # Monte Carlo surface points and directions
SEED_UPSTREAM = 24124      # upstream gradients of the differentiable trace
SEED_SERVING = 24125       # request stream of the serving workload
SEED_STEP = 24126          # perturbations of the training-like step
SEED_SH = 24127            # spherical-harmonic colour coefficients
SEED_PBR = 24128           # pixels, materials, sky and sampling uniforms of the shading workload


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclasses.dataclass
class Surfels:
    mu: np.ndarray
    quat: np.ndarray
    scale: np.ndarray
    opac: np.ndarray
    feat: np.ndarray

    @property
    def n(self) -> int:
        return int(self.mu.shape[0])

    @property
    def F(self) -> int:
        return int(self.feat.shape[1])

    def permuted(self, perm: np.ndarray) -> "Surfels":
        return Surfels(*(np.ascontiguousarray(a[perm]) for a in
                         (self.mu, self.quat, self.scale, self.opac, self.feat)))

    def subset(self, idx: np.ndarray) -> "Surfels":
        return self.permuted(np.asarray(idx))

    def astuple(self):
        return (self.mu, self.quat, self.scale, self.opac, self.feat)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _unit(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def quat_from_frame(tu: np.ndarray, tv: np.ndarray, nrm: np.ndarray) -> np.ndarray:
    """Unit quaternion (w,x,y,z), w >= 0, of the rotation whose columns are
    (tu, tv, nrm).  Shepperd's branch on the largest of (w,x,y,z)^2."""
    m00, m10, m20 = tu[:, 0], tu[:, 1], tu[:, 2]
    m01, m11, m21 = tv[:, 0], tv[:, 1], tv[:, 2]
    m02, m12, m22 = nrm[:, 0], nrm[:, 1], nrm[:, 2]
    tr = m00 + m11 + m22
    cand = np.stack([tr, m00, m11, m22], axis=1)
    k = np.argmax(cand, axis=1)
    q = np.empty((tu.shape[0], 4))
    # case w largest
    s = np.sqrt(np.maximum(1.0 + tr, 1e-300)) * 2.0
    w0 = np.stack([0.25 * s, (m21 - m12) / s, (m02 - m20) / s, (m10 - m01) / s], 1)
    s = np.sqrt(np.maximum(1.0 + m00 - m11 - m22, 1e-300)) * 2.0
    w1 = np.stack([(m21 - m12) / s, 0.25 * s, (m01 + m10) / s, (m02 + m20) / s], 1)
    s = np.sqrt(np.maximum(1.0 + m11 - m00 - m22, 1e-300)) * 2.0
    w2 = np.stack([(m02 - m20) / s, (m01 + m10) / s, 0.25 * s, (m12 + m21) / s], 1)
    s = np.sqrt(np.maximum(1.0 + m22 - m00 - m11, 1e-300)) * 2.0
    w3 = np.stack([(m10 - m01) / s, (m02 + m20) / s, (m12 + m21) / s, 0.25 * s], 1)
    for i, c in enumerate((w0, w1, w2, w3)):
        sel = k == i
        q[sel] = c[sel]
    q *= np.where(q[:, :1] < 0, -1.0, 1.0)
    return _unit(q)


def onb(nrm: np.ndarray):
    """Right-handed orthonormal basis (b1, b2) with b1 x b2 = nrm
    (Duff et al. 2017, 'Building an orthonormal basis, revisited')."""
    x, y, z = nrm[:, 0], nrm[:, 1], nrm[:, 2]
    sign = np.where(z >= 0, 1.0, -1.0)
    a = -1.0 / (sign + z)
    b = x * y * a
    b1 = np.stack([1.0 + sign * x * x * a, sign * b, -sign * x], 1)
    b2 = np.stack([b, sign + y * y * a, -y], 1)
    return b1, b2


# ----------------------------------------------------------------------------
# 4,096-surfel cube scene + 64x64 pinhole camera (forward-only small case)
# ----------------------------------------------------------------------------

def cube_scene(n: int = 4096, F: int = 3, seed: int = SEED_CUBE) -> Surfels:
    """Centres uniform in [-1,1]^3, rotations from normalised N(0,1)
    quaternions, scales log-uniform in [0.01, 0.1] per tangent axis, opacity
    U[0.05, 0.99], features U[0, 1]."""
    g = _rng(seed)
    mu = g.uniform(-1.0, 1.0, size=(n, 3))
    q = _unit(g.standard_normal(size=(n, 4)))
    s = np.exp(g.uniform(math.log(0.01), math.log(0.1), size=(n, 2)))
    o = g.uniform(0.05, 0.99, size=n)
    f = g.uniform(0.0, 1.0, size=(n, F))
    return Surfels(_f32(mu), _f32(q), _f32(s), _f32(o), _f32(f))


def pinhole_rays(width: int = 64, height: int = 64, eye=(0.0, 0.0, 3.0),
                 half_fov_tan: float = 0.5):
    """Camera at `eye` looking down -z with +y up; square pixels; the vertical
    half-angle has tangent `half_fov_tan` (0.5 frames the cube's near face).
    Ray index = row * width + column; directions normalised in FP64."""
    i = np.arange(width, dtype=np.float64)
    j = np.arange(height, dtype=np.float64)
    I, J = np.meshgrid(i, j)                      # J rows, I columns
    x = ((I + 0.5) / (width / 2.0) - 1.0) * half_fov_tan * (width / height)
    y = -((J + 0.5) / (height / 2.0) - 1.0) * half_fov_tan
    d = np.stack([x, y, -np.ones_like(x)], -1).reshape(-1, 3)
    d = _unit(d)
    o = np.broadcast_to(np.asarray(eye, dtype=np.float64), d.shape)
    return _f32(o), _f32(d)


# ----------------------------------------------------------------------------
# Union of 8 spheres and 4 square planes (Monte Carlo workloads)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Layout:
    centers: np.ndarray   # (8, 3)
    radii: np.ndarray     # (8,)
    p_center: np.ndarray  # (4, 3)
    p_normal: np.ndarray  # (4, 3)
    p_e1: np.ndarray      # (4, 3)
    p_e2: np.ndarray      # (4, 3)
    half_side: float = 1.0

    def areas(self) -> np.ndarray:
        sph = 4.0 * math.pi * self.radii ** 2
        pl = np.full(len(self.p_center), (2.0 * self.half_side) ** 2)
        return np.concatenate([sph, pl])


def layout(seed: int = SEED_LAYOUT) -> Layout:
    """8 spheres: centre U[-0.6,0.6]^3, radius U[0.2,0.5]; 4 planes: square
    patches of side 2, centre U[-0.5,0.5]^3, normal = normalised N(0,1)^3."""
    g = _rng(seed)
    c = g.uniform(-0.6, 0.6, size=(8, 3))
    r = g.uniform(0.2, 0.5, size=8)
    pc = g.uniform(-0.5, 0.5, size=(4, 3))
    pn = _unit(g.standard_normal(size=(4, 3)))
    e1, e2 = onb(pn)
    return Layout(c, r, pc, pn, e1, e2)


def _sample_surface(g: np.random.Generator, lay: Layout, n: int):
    """Area-uniform points on the union; returns (x, outward normal, surface id)."""
    a = lay.areas()
    counts = g.multinomial(n, a / a.sum())
    xs, ns, sid = [], [], []
    for k, cnt in enumerate(counts):
        if cnt == 0:
            continue
        if k < 8:
            nn = _unit(g.standard_normal(size=(cnt, 3)))
            x = lay.centers[k] + lay.radii[k] * nn
        else:
            p = k - 8
            ab = g.uniform(-lay.half_side, lay.half_side, size=(cnt, 2))
            x = lay.p_center[p] + ab[:, :1] * lay.p_e1[p] + ab[:, 1:] * lay.p_e2[p]
            nn = np.broadcast_to(lay.p_normal[p], (cnt, 3)).copy()
        xs.append(x)
        ns.append(nn)
        sid.append(np.full(cnt, k, dtype=np.int32))
    x = np.concatenate(xs)
    nn = np.concatenate(ns)
    sid = np.concatenate(sid)
    perm = g.permutation(n)
    return x[perm], nn[perm], sid[perm]


def surface_scene(n: int, F: int = 8, seed: int | None = None,
                  lay: Layout | None = None, return_surface_id: bool = False):
    """Surfels tangent to the sphere/plane union: positions area-uniform,
    normal = outward sphere normal or plane normal, t_u a random in-plane unit
    vector, t_v = n x t_u; scales log-uniform [0.005, 0.02] per axis; opacity
    U[0.5, 1]; features U[0, 1]^F."""
    if lay is None:
        lay = layout()
    g = _rng(SEED_LAYOUT + n if seed is None else seed)
    x, nn, sid = _sample_surface(g, lay, n)
    r = g.standard_normal(size=(n, 3))
    tu = _unit(r - np.sum(r * nn, 1, keepdims=True) * nn)
    tv = np.cross(nn, tu)
    q = quat_from_frame(tu, tv, nn)
    s = np.exp(g.uniform(math.log(0.005), math.log(0.02), size=(n, 2)))
    o = g.uniform(0.5, 1.0, size=n)
    f = g.uniform(0.0, 1.0, size=(n, F))
    out = Surfels(_f32(x), _f32(q), _f32(s), _f32(o), _f32(f))
    return (out, sid) if return_surface_id else out


def cosine_dirs(g: np.random.Generator, nrm: np.ndarray, m: int) -> np.ndarray:
    """m cosine-weighted directions about each normal (Malley's method: uniform
    disk sample lifted to the hemisphere).  Shape (P, m, 3), FP64, unit."""
    P = nrm.shape[0]
    u1 = g.random(size=(P, m))
    u2 = g.random(size=(P, m))
    rr = np.sqrt(u1)
    ph = 2.0 * math.pi * u2
    lx, ly = rr * np.cos(ph), rr * np.sin(ph)
    lz = np.sqrt(np.maximum(0.0, 1.0 - u1))
    b1, b2 = onb(nrm)
    d = (lx[..., None] * b1[:, None, :] + ly[..., None] * b2[:, None, :]
         + lz[..., None] * nrm[:, None, :])
    return _unit(d)


def mc_rays(points: int, dirs: int, seed: int = SEED_MC_RAYS,
            lay: Layout | None = None, offset: float = 1e-3):
    """`points` area-uniform surface points on the union, `dirs` cosine-weighted
    directions each about the chosen side's normal (planes: random side;
    spheres: outward).  Origin = x + offset * n.  Ray index = point*dirs + j,
    so the rays of one point are consecutive."""
    if lay is None:
        lay = layout()
    g = _rng(seed)
    x, nn, sid = _sample_surface(g, lay, points)
    flip = np.where((sid >= 8) & (g.random(points) < 0.5), -1.0, 1.0)
    nn = nn * flip[:, None]
    d = cosine_dirs(g, nn, dirs).reshape(-1, 3)
    o = np.repeat(x + offset * nn, dirs, axis=0)
    return _f32(o), _f32(d)


def shading_pixels(P: int, N: int, E: int = 32, seed: int = SEED_PBR, lay: Layout | None = None):
    """Inputs of the rendering-equation workload: P area-uniform surface
    points x with normals n (planes: random side), view directions w_o
    uniform over the hemisphere of n, albedo U[0,1]^3, roughness U[0.1, 1],
    a (6, E, E, 3) cubemap sky U[0, 3] and the (P, N, 2) sampling uniforms.
    All float32."""
    if lay is None:
        lay = layout()
    g = _rng(seed)
    x, nn, sid = _sample_surface(g, lay, P)
    flip = np.where((sid >= 8) & (g.random(P) < 0.5), -1.0, 1.0)
    nn = nn * flip[:, None]
    wo = _unit(g.standard_normal((P, 3)))
    wo = np.where(((wo * nn).sum(1) < 0)[:, None], -wo, wo)
    return dict(x=_f32(x), n=_f32(nn), wo=_f32(wo), albedo=_f32(g.uniform(0, 1, (P, 3))),
                rough=_f32(g.uniform(0.1, 1.0, P)), env=_f32(g.uniform(0, 3, (6, E, E, 3))),
                u=_f32(g.uniform(0, 1, (P, N, 2))))


def sh_coefficients(n: int, deg: int, seed: int = SEED_SH) -> np.ndarray:
    """RGB coefficients of a view-dependent colour, (n, 3 (deg + 1)^2) float32,
    coefficient-major (3 j + c): the constant term U[-1.5, 1.5] per channel
    and degree-l terms N(0, 0.2 / l), the shape of trained splatting colours
    (a dominant base colour, weak view dependence)."""
    g = _rng(seed)
    nb = (deg + 1) ** 2
    k = np.zeros((n, nb, 3))
    k[:, 0, :] = g.uniform(-1.5, 1.5, (n, 3))
    for l in range(1, deg + 1):
        k[:, l * l:(l + 1) * (l + 1), :] = g.normal(0.0, 0.2 / l, (n, 2 * l + 1, 3))
    return _f32(k.reshape(n, 3 * nb))


def upstream(R: int, F: int, seed: int = SEED_UPSTREAM, mask_rays: int | None = None):
    """N(0,1) upstream gradients on opacity (R,), features (R,F), depth (R,).
    With `mask_rays`, only that many randomly chosen rays keep non-zero
    gradients (the rest are zero), so the oracle can check a subsample."""
    g = _rng(seed)
    gO = g.standard_normal(R)
    gF = g.standard_normal((R, F))
    gD = g.standard_normal(R)
    idx = None
    if mask_rays is not None and mask_rays < R:
        idx = np.sort(g.choice(R, size=mask_rays, replace=False))
        keep = np.zeros(R, dtype=bool)
        keep[idx] = True
        gO[~keep] = 0.0
        gF[~keep] = 0.0
        gD[~keep] = 0.0
    return _f32(gO), _f32(gF), _f32(gD), idx


def serving_requests(n_req: int, n_scenes: int = 3, rmin: int = 1000,
                     rmax: int = 4_194_304, seed: int = SEED_SERVING):
    """Request stream: scene uniform in {0..n_scenes-1}, ray count
    round(exp(U[ln rmin, ln rmax])), and a per-request ray seed."""
    g = _rng(seed)
    scene = g.integers(0, n_scenes, size=n_req)
    rays = np.round(np.exp(g.uniform(math.log(rmin), math.log(rmax), size=n_req))).astype(np.int64)
    seeds = g.integers(1, 2**31 - 1, size=n_req)
    return scene, rays, seeds


def poisson_arrivals(n_req: int, rate: float, seed: int = SEED_SERVING + 1) -> np.ndarray:
    """Arrival times (seconds) of an open-loop Poisson process."""
    g = _rng(seed)
    return np.cumsum(g.exponential(1.0 / rate, size=n_req))


def random_rays_near(g: np.random.Generator, centre: np.ndarray, radius: float, R: int,
                     dist: float = 1.0):
    """Rays whose origins lie on a sphere of radius `dist` around `centre` and
    that aim at points uniform in a ball of `radius` around it."""
    src = centre + dist * _unit(g.standard_normal((R, 3)))
    tgt = centre + radius * _unit(g.standard_normal((R, 3))) * g.random((R, 1)) ** (1 / 3)
    return _f32(src), _f32(_unit(tgt - src))


def sky_uniforms(P: int, N: int, seed: int = SEED_PBR + 2) -> np.ndarray:
    """(P, N, 3) float32 uniforms in [0, 1) for drawing incident directions
    from a sky's intensity (texel choice, then the point in the texel)."""
    return _rng(seed).random((P, N, 3)).astype(np.float32)



def grazing_rays(points: int, cos_lo: float = 1e-4, cos_hi: float = 2e-2, seed: int = SEED_MC_RAYS + 7,
                 lay: Layout | None = None):
    """Rays that skim their own surface: area-uniform surface points (planes:
    random side), directions at cos(theta) ~ U[cos_lo, cos_hi] to the normal
    with uniform azimuth, origin x + 1e-3 n.  The slowest rays of the
    Monte Carlo workloads look like these.  Returns float32 (ro, rd)."""
    if lay is None:
        lay = layout()
    g = _rng(seed)
    x, nn, sid = _sample_surface(g, lay, points)
    flip = np.where((sid >= 8) & (g.random(points) < 0.5), -1.0, 1.0)
    nn = nn * flip[:, None]
    b1, b2 = onb(nn)
    c = g.uniform(cos_lo, cos_hi, points)
    phi = g.uniform(0.0, 2.0 * np.pi, points)
    s = np.sqrt(1.0 - c * c)
    d = _unit((s * np.cos(phi))[:, None] * b1 + (s * np.sin(phi))[:, None] * b2 + c[:, None] * nn)
    return _f32(x + 1e-3 * nn), _f32(d)
