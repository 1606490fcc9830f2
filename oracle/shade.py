"""FP64 oracle of the Monte Carlo rendering-equation consumer of the trace
(Sec. 3.3, "Rendering": Eq. 15 evaluated with the light decomposition of
Eq. 13-14 and the BRDF of Sec. 3.1, Eq. 4).

TEST INFRASTRUCTURE (see the package docstring): never on the product path.

Per pixel (surface point x, unit normal n, unit view direction w_o towards
the camera, albedo a, roughness r) and its N_r = S_t * S_p incident
directions w_i:

    c_pbr = 2 pi / N_r * sum_i (f_d + f_s(w_i)) L_i(w_i) (w_i . n)      (Eq. 15)

(2 pi / N_r = 1 / (N_r pdf) of the uniform hemisphere; with another
sampling density each sample carries its own weight 1 / (N_r pdf(w_i)),
0 below the horizon, which the relighting variant uses)
    L_i   = V_i L_dir(w_i) + L_ind,i,  V_i = 1 - O_i                    (Eq. 13-14)
    f_d   = a / pi,  f_s = D F G / (4 (w_i . n)(w_o . n))               (Eq. 4)

with O_i and L_ind,i the opacity and composited colour the trace returns
for the ray (x, w_i).  Readings (the paper names the terms only):

* stratified uniform hemisphere sampling: sample i = (s, t) = (i // S_p,
  i % S_p) has cos(theta) = (s + u0) / S_t and phi = 2 pi (t + u1) / S_p for
  uniforms (u0, u1) supplied by the caller; the local direction
  (sin cos phi, sin sin phi, cos) is mapped to the world by the branchless
  orthonormal basis (t1, t2, n) of Duff et al. 2017;
* D = GGX / Trowbridge-Reitz with alpha = r^2:
  D = alpha^2 / (pi ((n.h)^2 (alpha^2 - 1) + 1)^2), h = normalise(w_i + w_o);
* F = Schlick with F0 = 0.04 (dielectric): F0 + (1 - F0)(1 - w_o.h)^5;
* G = Smith with the Schlick-GGX G1(x) = x / (x (1 - k) + k),
  k = (r + 1)^2 / 8;
* n.w_i and n.w_o enter G and the denominator of f_s clamped below at
  1e-4; the cosine factor of Eq. 15 is n.w_i itself;
* L_dir: an RGB cubemap of 6 faces of E x E texels, nearest texel, faces
  +x, -x, +y, -y, +z, -z with (s, t) = (-z, -y), (z, -y), (x, z), (x, -z),
  (x, -y), (-x, -y) divided by the major coordinate's magnitude, texel
  (floor((t + 1) E / 2), floor((s + 1) E / 2)) clamped to [0, E-1] (row, col).
"""
from __future__ import annotations

import numpy as np
import torch

F0 = 0.04
EPS_COS = 1e-4


def onb(n):
    """Branchless orthonormal basis (t1, t2) completing the unit normals n
    (Duff et al. 2017, 'Building an orthonormal basis, revisited')."""
    n = np.asarray(n, np.float64)
    sign = np.where(n[..., 2] >= 0.0, 1.0, -1.0)
    a = -1.0 / (sign + n[..., 2])
    b = n[..., 0] * n[..., 1] * a
    t1 = np.stack([1.0 + sign * n[..., 0] ** 2 * a, sign * b, -sign * n[..., 0]], -1)
    t2 = np.stack([b, sign + n[..., 1] ** 2 * a, -n[..., 1]], -1)
    return t1, t2


def stratified_dirs(n, u, S_t: int, S_p: int):
    """(P, S_t*S_p, 3) directions for unit normals n (P, 3) and uniforms
    u (P, S_t*S_p, 2)."""
    n = np.asarray(n, np.float64)
    u = np.asarray(u, np.float64)
    N = S_t * S_p
    i = np.arange(N)
    s, t = i // S_p, i % S_p
    ct = (s[None, :] + u[..., 0]) / S_t
    phi = 2.0 * np.pi * (t[None, :] + u[..., 1]) / S_p
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    t1, t2 = onb(n)
    loc = [st * np.cos(phi), st * np.sin(phi), ct]
    return loc[0][..., None] * t1[:, None, :] + loc[1][..., None] * t2[:, None, :] + loc[2][..., None] * n[:, None, :]


def cube_texel(d, E: int, dtype=np.float64):
    """(face, row, col) of the nearest texel of each direction d (..., 3).
    The texel is an integer decided by floating point: parity checks against
    an FP32 kernel take the decision in float32 (dtype) like the kernel."""
    d = np.asarray(d, dtype)
    ax = np.abs(d)
    major = np.argmax(ax, -1)  # ties go to the lower axis (x, then y)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    m = np.take_along_axis(ax, major[..., None], -1)[..., 0]
    pos = np.take_along_axis(d, major[..., None], -1)[..., 0] >= 0
    face = 2 * major + np.where(pos, 0, 1)
    s = np.select([face == 0, face == 1, face == 2, face == 3, face == 4, face == 5], [-z, z, x, x, x, -x])
    t = np.select([face == 0, face == 1, face == 2, face == 3, face == 4, face == 5], [-y, -y, z, -z, -y, -y])
    s, t = s / m, t / m
    one, half, e = dtype(1.0), dtype(0.5), dtype(E)
    col = np.clip(np.floor((s + one) * e * half), 0, E - 1).astype(np.int64)
    row = np.clip(np.floor((t + one) * e * half), 0, E - 1).astype(np.int64)
    return face, row, col


def ggx_D(ndh, r):
    """GGX / Trowbridge-Reitz normal distribution, alpha = r^2."""
    a2 = (r * r) ** 2
    return a2 / (np.pi * (ndh * ndh * (a2 - 1.0) + 1.0) ** 2)


def schlick_F(vdh):
    return F0 + (1.0 - F0) * (1.0 - vdh) ** 5


def smith_G(ndl_c, ndv_c, r):
    """Smith shadowing-masking with Schlick-GGX G1, k = (r + 1)^2 / 8."""
    k = (r + 1.0) ** 2 / 8.0
    return ndl_c / (ndl_c * (1.0 - k) + k) * ndv_c / (ndv_c * (1.0 - k) + k)


def _brdf_spec(n, wo, wi, r, lib):
    """Scalar specular lobe f_s and the raw cosine n.w_i (lib = np or torch)."""
    h = wi + wo[..., None, :]
    h = h / lib.sqrt((h * h).sum(-1, keepdims=True))
    ndl = (wi * n[..., None, :]).sum(-1)
    ndv = (wo * n).sum(-1)[..., None]
    ndh = (h * n[..., None, :]).sum(-1)
    vdh = (h * wo[..., None, :]).sum(-1)
    clamp = (lambda x: lib.clamp(x, min=EPS_COS)) if lib is torch else (lambda x: np.maximum(x, EPS_COS))
    ndl_c, ndv_c = clamp(ndl), clamp(ndv)
    r = r[..., None]
    fs = ggx_D(ndh, r) * schlick_F(vdh) * smith_G(ndl_c, ndv_c, r) / (4.0 * ndl_c * ndv_c)
    return fs, ndl


def shade(n, wo, albedo, rough, wi, O, Lind, env, texel_dtype=np.float64, wgt=None):
    """c_pbr (P, 3), FP64 numpy.  wi (P, N, 3), O (P, N), Lind (P, N, 3),
    env (6, E, E, 3); wgt (P, N) optional per-sample weights (see _weights)."""
    n, wo, albedo, rough, wi, O, Lind, env = (np.asarray(a, np.float64) for a in
                                                (n, wo, albedo, rough, wi, O, Lind, env))
    N, E = wi.shape[1], env.shape[1]
    # 1 / (N pdf): 2 pi / N for the uniform hemisphere, else the caller's
    # per-sample weights (0 for a sample below the horizon)
    w = 2.0 * np.pi / N if wgt is None else np.asarray(wgt, np.float64)[..., None]
    fs, ndl = _brdf_spec(n, wo, wi, rough, np)
    f, row, col = cube_texel(wi, E, texel_dtype)
    Ldir = env[f, row, col]                                      # (P, N, 3)
    Li = (1.0 - O)[..., None] * Ldir + Lind
    brdf = albedo[:, None, :] / np.pi + fs[..., None]
    return (w * brdf * Li * ndl[..., None]).sum(1)


def shade_grad(n, wo, albedo, rough, wi, O, Lind, env, g_c, texel_dtype=np.float64, wgt=None):
    """FP64 autograd gradients of sum(g_c * c_pbr) with respect to albedo,
    roughness, the cubemap, O and L_ind (optional per-sample weights wgt)."""
    t = lambda a: torch.tensor(np.asarray(a, np.float64))
    n_t, wo_t, wi_t = t(n), t(wo), t(wi)
    albedo_t, rough_t, O_t, Lind_t, env_t = (t(a).requires_grad_(True) for a in (albedo, rough, O, Lind, env))
    E = env_t.shape[1]
    N = wi_t.shape[1]
    fs, ndl = _brdf_spec(n_t, wo_t, wi_t, rough_t, torch)
    f, row, col = cube_texel(np.asarray(wi, np.float64), E, texel_dtype)
    Ldir = env_t[torch.tensor(f), torch.tensor(row), torch.tensor(col)]
    Li = (1.0 - O_t)[..., None] * Ldir + Lind_t
    brdf = albedo_t[:, None, :] / np.pi + fs[..., None]
    w = 2.0 * np.pi / N if wgt is None else t(wgt)[..., None]
    c = (w * brdf * Li * ndl[..., None]).sum(1)
    L = (t(g_c) * c).sum()
    g = torch.autograd.grad(L, [albedo_t, rough_t, env_t, O_t, Lind_t])
    return dict(zip(("albedo", "rough", "env", "O", "Lind"), (x.numpy() for x in g)))
