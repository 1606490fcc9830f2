"""FP64 oracle of the relighting variant of the trace's consumer (the
paper's relighting details: the trace alpha-blends albedo, roughness and
normal with normalised weights, and each incident ray's indirect radiance is
shaded with the split-sum approximation from a pre-integrated cubemap and a
pre-integrated BRDF table: L_ind = L_d + L_s).

TEST INFRASTRUCTURE (see the package docstring): never on the product path.

Readings (the paper cites the split-sum construction and gives no numbers):

* blend: {A, R, N} = sum_i w_i {a_i, r_i, n_i} / sum_i w_i with w_i = T_i
  alpha_i; n_i is the splat's unit normal turned to face the ray
  (n_i . d <= 0); N is renormalised; a ray with no hit (sum w = 0) carries
  no indirect radiance;
* the surface seen by the ray is viewed from v = -d; L_d = A / pi * E(N)
  with the irradiance E(N) = sum_texels L(w) max(w . N, 0) dOmega(w);
* L_s = P_R(refl) (F0 S_A(N.v, R) + S_B(N.v, R)), F0 = 0.04, refl = the
  mirror of d about N, P_R the GGX-prefiltered sky
  P_R(c) = sum L(w) D_R(c . h) max(w . c, 0) dOmega / sum D_R(c . h)
  max(w . c, 0) dOmega with h = normalise(w + c) (the normal = view =
  reflection assumption), at roughness levels r_l = (l + 1) / M (no level
  at r = 0, where GGX degenerates), the ray using the nearest level
  l = clamp(floor(R M + 1/2) - 1, 0, M - 1) and the nearest texel;
* the BRDF table (S_A, S_B) at cell centres (N.v, r) = ((i + 1/2)/S,
  (j + 1/2)/S) is the GGX-importance-sampled estimate over the 2D Hammersley
  set of 256 points (x_k, y_k) = ((k + 1/2)/256, radical inverse of k):
  h at cos^2(theta_h) = (1 - y) / (1 + (alpha^2 - 1) y), phi_h = 2 pi x,
  l = reflect(-v, h); if n.l > 0: g = G(n.l, n.v, r) (v.h) / ((n.h)(n.v)),
  F_c = (1 - v.h)^5, S_A += (1 - F_c) g, S_B += F_c g; then / 256 (the
  table lookup takes the nearest cell);
* texel solid angles are exact for the cube face parameterisation:
  dOmega = 4 / (E^2 (1 + s^2 + t^2)^{3/2}) at the texel centre (s, t);
* importance sampling of the sky (the paper samples the known environment
  by its intensity instead of the stratified hemisphere): intensity I = the
  mean of the texel's RGB (clamped at 0), texel weight I dOmega at its
  centre, the inclusive running sum of the weights in texel order
  (face, row, col) as the CDF; a sample (u0, u1, u2) picks the first texel
  whose CDF exceeds u0 * total (FP32, as the kernel decides it), then the
  point (s, t) = ((col + u1), (row + u2)) 2 / E - 1 of that texel, uniform
  in the face coordinates, so pdf(w) = p_j E^2 / 4 (1 + s^2 + t^2)^{3/2}
  with p_j = (CDF_j - CDF_{j-1}) / total; the estimator weight is
  1 / (N pdf) for n . w > 0 and 0 below the horizon; texels of zero
  intensity are never drawn (their directions then carry no light of any
  kind: an unbiased estimate needs a sky that is positive where light,
  direct or indirect, arrives).
"""
from __future__ import annotations

import numpy as np

from .shade import F0, cube_texel, ggx_D, smith_G

HAMMERSLEY_N = 256


def face_point(face, s, t):
    """Unnormalised direction of face coordinates (s, t) on a face (the
    inverse of the nearest-texel addressing)."""
    face, s, t = np.broadcast_arrays(np.asarray(face), np.asarray(s, np.float64), np.asarray(t, np.float64))
    one = np.ones_like(s)
    cand = np.stack([np.stack([one, -t, -s], -1), np.stack([-one, -t, s], -1), np.stack([s, one, t], -1),
                     np.stack([s, -one, -t], -1), np.stack([s, -t, one], -1), np.stack([-s, -t, -one], -1)])
    return np.take_along_axis(cand, face[None, ..., None].astype(np.int64), 0)[0]


def texel_dirs(E: int):
    """(6, E, E, 3) unit centre directions and (E, E) solid angles."""
    c = (np.arange(E) + 0.5) / E * 2.0 - 1.0
    t, s = np.meshgrid(c, c, indexing="ij")       # row index -> t, column -> s
    d = face_point(np.arange(6)[:, None, None], s[None], t[None])
    d = d / np.linalg.norm(d, axis=-1, keepdims=True)
    dw = 4.0 / (E * E * (1.0 + s * s + t * t) ** 1.5)
    return d, dw


def irradiance(env):
    """E(N) at every texel centre of the same cube resolution: (6, E, E, 3)."""
    env = np.asarray(env, np.float64)
    E = env.shape[1]
    d, dw = texel_dirs(E)
    w = d.reshape(-1, 3)
    L = (env * dw[None, :, :, None]).reshape(-1, 3)
    cos = np.maximum(w @ w.T, 0.0)                 # (out, in)
    return (cos @ L).reshape(6, E, E, 3)


def prefilter(env, M: int):
    """(M, 6, E, E, 3) GGX-prefiltered skies at r_l = (l + 1) / M."""
    env = np.asarray(env, np.float64)
    E = env.shape[1]
    d, dw = texel_dirs(E)
    w = d.reshape(-1, 3)
    L = env.reshape(-1, 3)
    dwf = np.broadcast_to(dw, (6, E, E)).reshape(-1)
    cos = w @ w.T                                   # out c . in w
    h = w[None, :, :] + w[:, None, :]               # (out, in, 3)
    hn = np.linalg.norm(h, axis=-1)
    ch = np.where(hn > 0, (h * w[:, None, :]).sum(-1) / np.where(hn > 0, hn, 1.0), 0.0)
    out = np.zeros((M, 6 * E * E, 3))
    for l in range(M):
        r = (l + 1) / M
        wt = ggx_D(ch, r) * np.maximum(cos, 0.0) * dwf[None, :]
        out[l] = (wt @ L) / wt.sum(1, keepdims=True)
    return out.reshape(M, 6, E, E, 3)


def _radical_inverse(k):
    k = np.asarray(k, np.uint64)
    r = np.zeros(k.shape, np.float64)
    f = 0.5
    for _ in range(32):
        r += f * (k & np.uint64(1))
        k = k >> np.uint64(1)
        f *= 0.5
    return r


def brdf_table(S: int):
    """(S, S, 2) split-sum table (S_A, S_B) at cell centres (n.v, r)."""
    k = np.arange(HAMMERSLEY_N)
    x = (k + 0.5) / HAMMERSLEY_N
    y = _radical_inverse(k)
    out = np.zeros((S, S, 2))
    for i in range(S):
        nv = (i + 0.5) / S
        v = np.array([np.sqrt(1.0 - nv * nv), 0.0, nv])
        for j in range(S):
            r = (j + 0.5) / S
            a2 = (r * r) ** 2
            c2 = (1.0 - y) / (1.0 + (a2 - 1.0) * y)
            ct, st = np.sqrt(c2), np.sqrt(1.0 - c2)
            phi = 2.0 * np.pi * x
            h = np.stack([st * np.cos(phi), st * np.sin(phi), ct], -1)
            vh = h @ v
            l = 2.0 * vh[:, None] * h - v[None, :]
            nl, nh = l[:, 2], h[:, 2]
            ok = nl > 0
            g = np.where(ok, smith_G(np.maximum(nl, 1e-300), nv, r) * vh / (nh * nv), 0.0)
            fc = (1.0 - vh) ** 5
            out[i, j, 0] = np.sum((1.0 - fc) * g) / HAMMERSLEY_N
            out[i, j, 1] = np.sum(fc * g) / HAMMERSLEY_N
    return out


def blend(O, Fo, F: int):
    """Normalised blend from the trace's outputs: features (..., F) then the
    normal (..., 3) composited with the same weights."""
    O = np.asarray(O, np.float64)
    Fo = np.asarray(Fo, np.float64)
    safe = np.where(O > 0, O, 1.0)[..., None]
    feat = Fo[..., :F] / safe
    nrm = Fo[..., F:F + 3]
    nn = np.linalg.norm(nrm, axis=-1, keepdims=True)
    nrm = nrm / np.where(nn > 0, nn, 1.0)
    return feat, nrm


def relight_lind(O, Fo, rd, irr, pref, table):
    """Indirect radiance (R, 3) of each ray from its trace outputs: O (R),
    Fo (R, 4 + 3) = blended (albedo, roughness) then normal, directions rd."""
    O = np.asarray(O, np.float64)
    rd = np.asarray(rd, np.float64)
    rd = rd / np.linalg.norm(rd, axis=-1, keepdims=True)
    (feat, N) = blend(O, Fo, 4)
    hit = O > 0
    N = np.where(hit[:, None], N, np.array([0.0, 0.0, 1.0]))   # rays without a hit: any direction, zeroed below
    A, Rg = feat[:, :3], feat[:, 3]
    E = irr.shape[1]
    M = pref.shape[0]
    S = table.shape[0]
    f, row, col = cube_texel(N, E, np.float32)
    Ld = A / np.pi * irr[f, row, col]
    v = -rd
    nv = np.clip((N * v).sum(-1), 0.0, 1.0)
    refl = rd - 2.0 * (rd * N).sum(-1, keepdims=True) * N
    lev = np.clip(np.floor(np.clip(Rg, 0.0, 1.0) * M + 0.5) - 1, 0, M - 1).astype(np.int64)
    f2, row2, col2 = cube_texel(refl, E, np.float32)
    Pr = pref[lev, f2, row2, col2]
    i = np.clip(np.floor(nv * S), 0, S - 1).astype(np.int64)
    j = np.clip(np.floor(np.clip(Rg, 0.0, 1.0) * S), 0, S - 1).astype(np.int64)
    Ls = Pr * (F0 * table[i, j, 0] + table[i, j, 1])[:, None]
    return np.where(hit[:, None], Ld + Ls, 0.0)


def env_cdf(env):
    """(6 E^2,) inclusive CDF of the texel weights max(mean RGB, 0) dOmega."""
    env = np.asarray(env, np.float64)
    E = env.shape[1]
    _, dw = texel_dirs(E)
    inten = np.fmax(env.mean(-1), 0.0)                       # NaN -> 0
    return np.cumsum((inten * dw[None]).reshape(-1))


def env_sample(x, n, u, cdf32, E: int, offset: float = 1e-3):
    """Rays drawn from the sky's intensity: x, n (P, 3), u (P, N, 3)
    uniforms in [0, 1), cdf32 the FP32 CDF both sides decide with.  Returns
    ro, rd (P, N, 3) and the estimator weights (P, N): 1 / (N pdf), 0 below
    the horizon or for a sky with no positive weight."""
    x, n, u = (np.asarray(a, np.float64) for a in (x, n, u))
    cdf32 = np.asarray(cdf32, np.float32)
    P, N = u.shape[0], u.shape[1]
    total32 = cdf32[-1]
    target = np.float32(u[..., 0].astype(np.float32) * total32)          # FP32 product, as the kernel
    target = np.where(target < total32, target, np.nextafter(total32, np.float32(0)))
    j = np.minimum(np.searchsorted(cdf32, target, side="right"), cdf32.size - 1)
    face, rc = j // (E * E), j % (E * E)
    row, col = rc // E, rc % E
    s = (col + u[..., 1]) * 2.0 / E - 1.0
    t = (row + u[..., 2]) * 2.0 / E - 1.0
    d = face_point(face, s, t)
    d = d / np.linalg.norm(d, axis=-1, keepdims=True)
    cdf = cdf32.astype(np.float64)
    total = float(total32)
    pj = (cdf[j] - np.where(j > 0, cdf[np.maximum(j - 1, 0)], 0.0)) / (total if total > 0 else 1.0)
    pdf = pj * E * E / 4.0 * (1.0 + s * s + t * t) ** 1.5
    up = (d * n[:, None, :]).sum(-1) > 0
    ok = up & (pdf > 0) & (total > 0)
    wgt = np.where(ok, 1.0 / (N * np.where(ok, pdf, 1.0)), 0.0)
    ro = np.broadcast_to(x[:, None, :] + offset * n[:, None, :], d.shape)
    return ro, d, wgt

