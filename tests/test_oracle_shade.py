"""Pins of the FP64 rendering-equation oracle (Sec. 3.3 "Rendering", Eq. 15
with the light decomposition of Eq. 13-14 and the BRDF of Eq. 4): sampling,
frame, cubemap addressing, BRDF terms against their defining integrals and
limits, the estimator against closed forms, gradients against finite
differences."""
import math

import numpy as np

from oracle import shade as osh


def _normals(seed, n):
    v = np.random.default_rng(seed).standard_normal((n, 3))
    v = v / np.linalg.norm(v, axis=1, keepdims=True)
    # include the axes and the branch point of the basis
    extra = np.array([[0, 0, 1.0], [0, 0, -1.0], [1.0, 0, 0], [0, 1.0, 0], [0, 1e-9, -1.0]])
    extra /= np.linalg.norm(extra, axis=1, keepdims=True)
    return np.concatenate([v, extra])


def test_onb_is_a_right_handed_orthonormal_frame():
    n = _normals(60, 200)
    t1, t2 = osh.onb(n)
    for a, b in ((t1, t2), (t1, n), (t2, n)):
        np.testing.assert_allclose((a * b).sum(1), 0, atol=1e-12)
    for a in (t1, t2):
        np.testing.assert_allclose(np.linalg.norm(a, axis=1), 1, atol=1e-12)
    np.testing.assert_allclose(np.cross(t1, t2), n, atol=1e-12)


def test_stratified_directions():
    """Unit directions in the upper hemisphere; sample (s, t) has its cosine
    in stratum s and its azimuth (in the local frame) in stratum t; with the
    stratum centres the cosines average exactly 1/2."""
    n = _normals(61, 20)
    St, Sp = 8, 16
    u = np.random.default_rng(62).uniform(0, 1, (n.shape[0], St * Sp, 2))
    w = osh.stratified_dirs(n, u, St, Sp)
    np.testing.assert_allclose(np.linalg.norm(w, axis=-1), 1, atol=1e-12)
    ct = (w * n[:, None, :]).sum(-1)
    s = np.arange(St * Sp) // Sp
    t = np.arange(St * Sp) % Sp
    assert np.all(ct >= s / St - 1e-12) and np.all(ct <= (s + 1) / St + 1e-12)
    t1, t2 = osh.onb(n)
    phi = np.mod(np.arctan2((w * t2[:, None, :]).sum(-1), (w * t1[:, None, :]).sum(-1)), 2 * np.pi)
    assert np.all(phi >= 2 * np.pi * t / Sp - 1e-9) and np.all(phi <= 2 * np.pi * (t + 1) / Sp + 1e-9)
    wc = osh.stratified_dirs(n, np.full_like(u, 0.5), St, Sp)
    np.testing.assert_allclose((wc * n[:, None, :]).sum(-1).mean(1), 0.5, atol=1e-14)


def _texel_dir(face, row, col, E):
    """Centre direction of a texel (the inverse of the addressing)."""
    s = 2 * (col + 0.5) / E - 1
    t = 2 * (row + 0.5) / E - 1
    return {0: (1, -t, -s), 1: (-1, -t, s), 2: (s, 1, t), 3: (s, -1, -t), 4: (s, -t, 1), 5: (-s, -t, -1)}[face]


def test_cubemap_addressing_round_trips():
    E = 8
    dirs, want = [], []
    for f in range(6):
        for r in range(E):
            for c in range(E):
                dirs.append(_texel_dir(f, r, c, E))
                want.append((f, r, c))
    got = np.stack(osh.cube_texel(np.array(dirs, float), E), -1)
    np.testing.assert_array_equal(got, np.array(want))
    # the six axes land on their own faces
    f, _, _ = osh.cube_texel(np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0], [0, -1.0, 0], [0, 0, 1.0],
                                       [0, 0, -1.0]]), 32)
    np.testing.assert_array_equal(f, np.arange(6))


def test_ggx_is_normalised_and_brdf_limits():
    """int D(h) (n.h) dw_h = 1 over the hemisphere; F(1) = F0, F(0) = 1;
    G = 1 at normal incidence and view; at the mirror direction
    f_s = D(1) F(n.w_o) G / (4 (n.w)^2) with D(1) = 1 / (pi alpha^2)."""
    x, w = np.polynomial.legendre.leggauss(400)
    c = 0.5 * (x + 1)                       # cos(theta_h) in (0, 1)
    for r in (0.3, 0.5, 0.8, 1.0):
        integral = 2 * np.pi * 0.5 * np.sum(w * osh.ggx_D(c, r) * c)
        assert abs(integral - 1) < 1e-6, (r, integral)
    assert abs(osh.schlick_F(1.0) - osh.F0) < 1e-15 and abs(osh.schlick_F(0.0) - 1) < 1e-15
    assert abs(osh.smith_G(1.0, 1.0, 0.7) - 1) < 1e-15
    n = np.array([[0, 0, 1.0]])
    th = 0.6
    wo = np.array([[math.sin(th), 0, math.cos(th)]])
    wi = np.array([[[-math.sin(th), 0, math.cos(th)]]])
    r = np.array([0.5])
    fs, ndl = osh._brdf_spec(n, wo, wi, r, np)
    a2 = 0.5 ** 4
    want = (1 / (np.pi * a2)) * osh.schlick_F(math.cos(th)) * osh.smith_G(math.cos(th), math.cos(th), 0.5) / (
        4 * math.cos(th) ** 2)
    assert abs(fs[0, 0] - want) < 1e-12 * want
    assert abs(ndl[0, 0] - math.cos(th)) < 1e-15


def _pixels(seed, P, St, Sp, E=8):
    g = np.random.default_rng(seed)
    n = _normals(seed, P)[:P]
    wo = g.standard_normal((P, 3))
    wo = wo / np.linalg.norm(wo, axis=1, keepdims=True)
    wo = np.where(((wo * n).sum(1) < 0)[:, None], -wo, wo)
    u = g.uniform(0, 1, (P, St * Sp, 2))
    wi = osh.stratified_dirs(n, u, St, Sp)
    return dict(n=n, wo=wo, albedo=g.uniform(0, 1, (P, 3)), rough=g.uniform(0.1, 1, P), wi=wi,
                O=g.uniform(0, 1, (P, St * Sp)), Lind=g.uniform(0, 2, (P, St * Sp, 3)),
                env=g.uniform(0, 3, (6, E, E, 3)))


def test_estimator_closed_forms():
    """Diffuse part: c(a) - c(0) = a L for a constant sky L, no occlusion and
    stratum-centre samples (2 pi / N sum cos / pi = 2 mean cos = 1); c is
    linear in L_ind and in the cubemap, and full occlusion (O = 1) removes
    the sky."""
    P, St, Sp = 6, 8, 8
    d = _pixels(63, P, St, Sp)
    wi = osh.stratified_dirs(d["n"], np.full((P, St * Sp, 2), 0.5), St, Sp)
    L = np.array([0.7, 1.3, 2.0])
    env = np.broadcast_to(L, (6, 8, 8, 3))
    zero = np.zeros((P, St * Sp))
    c1 = osh.shade(d["n"], d["wo"], d["albedo"], d["rough"], wi, zero, 0 * d["Lind"], env)
    c0 = osh.shade(d["n"], d["wo"], 0 * d["albedo"], d["rough"], wi, zero, 0 * d["Lind"], env)
    np.testing.assert_allclose(c1 - c0, d["albedo"] * L, rtol=1e-12)
    args = (d["n"], d["wo"], d["albedo"], d["rough"], d["wi"])
    a = osh.shade(*args, d["O"], d["Lind"], d["env"])
    b = osh.shade(*args, d["O"], 2 * d["Lind"], 2 * d["env"])
    np.testing.assert_allclose(b, 2 * a, rtol=1e-12)
    only_ind = osh.shade(*args, np.ones_like(d["O"]), d["Lind"], d["env"])
    np.testing.assert_allclose(only_ind, osh.shade(*args, d["O"], d["Lind"], 0 * d["env"]), rtol=1e-12)


def test_shade_gradients_match_finite_differences():
    P, St, Sp = 4, 4, 8
    d = _pixels(64, P, St, Sp, E=4)
    g_c = np.random.default_rng(65).standard_normal((P, 3))
    G = osh.shade_grad(d["n"], d["wo"], d["albedo"], d["rough"], d["wi"], d["O"], d["Lind"], d["env"], g_c)

    def L(**over):
        a = dict(d, **over)
        return float((g_c * osh.shade(a["n"], a["wo"], a["albedo"], a["rough"], a["wi"], a["O"], a["Lind"],
                                      a["env"])).sum())

    for name in ("albedo", "rough", "env", "O", "Lind"):
        x = np.array(d[name], np.float64)
        fd = np.zeros_like(x)
        it = np.nditer(x, flags=["multi_index"])
        for _ in it:
            i = it.multi_index
            h = 1e-6 * max(1.0, abs(x[i]))
            xp, xm = x.copy(), x.copy()
            xp[i] += h
            xm[i] -= h
            fd[i] = (L(**{name: xp}) - L(**{name: xm})) / (2 * h)
        np.testing.assert_allclose(G[name], fd, rtol=1e-6, atol=1e-8 * np.abs(fd).max(), err_msg=name)
