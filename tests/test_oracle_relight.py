"""Pins of the FP64 relighting oracle (the paper's relighting details: blended
albedo / roughness / normal, split-sum shading from a pre-integrated cubemap
and a pre-integrated BRDF table)."""
import math

import numpy as np

from oracle import relight as rl
from oracle import shade as osh


def test_texels_cover_the_sphere():
    for E in (4, 16, 32):
        d, dw = rl.texel_dirs(E)
        assert abs(6 * dw.sum() / (4 * math.pi) - 1) < 0.3 / E ** 2   # midpoint rule, O(1/E^2)
        f, r, c = osh.cube_texel(d.reshape(-1, 3), E)
        idx = np.arange(6 * E * E)
        np.testing.assert_array_equal((f * E + r) * E + c, idx)


def test_irradiance_closed_forms():
    """Constant sky L: E(N) = pi L; sky max(w_z, 0): E(+z) = 2 pi / 3."""
    E = 32
    L = np.array([0.5, 1.0, 2.0])
    irr = rl.irradiance(np.broadcast_to(L, (6, E, E, 3)))
    np.testing.assert_allclose(irr / (math.pi * L), 1, atol=5e-3)
    d, _ = rl.texel_dirs(E)
    sky = np.repeat(np.maximum(d[..., 2:3], 0.0), 3, -1)
    irr = rl.irradiance(sky)
    f, r, c = osh.cube_texel(np.array([[0, 0, 1.0]]), E)
    assert abs(irr[f[0], r[0], c[0], 0] / (2 * math.pi / 3) - 1) < 5e-3


def test_prefilter_preserves_constant_and_is_linear():
    E, M = 8, 4
    g = np.random.default_rng(80)
    a, b = g.uniform(0, 2, (6, E, E, 3)), g.uniform(0, 2, (6, E, E, 3))
    np.testing.assert_allclose(rl.prefilter(np.full((6, E, E, 3), 1.7), M), 1.7, rtol=1e-12)
    np.testing.assert_allclose(rl.prefilter(a + 2 * b, M), rl.prefilter(a, M) + 2 * rl.prefilter(b, M), rtol=1e-10)
    # rougher levels are smoother: the spread of a random sky shrinks with r
    p = rl.prefilter(a, M)
    spread = [p[l].std() for l in range(M)]
    assert all(spread[l + 1] < spread[l] for l in range(M - 1))


def test_brdf_table_against_dense_quadrature():
    """The importance-sampled table estimates S_A = int D G (1 - F_c) / (4 n.v)
    dw_l and S_B = int D G F_c / (4 n.v) dw_l over the hemisphere of l
    (h = normalise(l + v)); dense product quadrature in l agrees."""
    S = 8
    t = rl.brdf_table(S)
    assert np.all(t >= 0) and np.all(t.sum(-1) <= 1 + 1e-9)
    x, w = np.polynomial.legendre.leggauss(400)
    cl = 0.5 * (x + 1)
    phis = (np.arange(400) + 0.5) * 2 * np.pi / 400
    CL, PH = np.meshgrid(cl, phis, indexing="ij")
    W = (0.5 * w)[:, None] * (2 * np.pi / 400)
    sl = np.sqrt(1 - CL ** 2)
    l = np.stack([sl * np.cos(PH), sl * np.sin(PH), CL], -1)
    for i, j in ((3, 3), (5, 4), (6, 6), (7, 7), (2, 5)):
        nv, r = (i + 0.5) / S, (j + 0.5) / S
        v = np.array([math.sqrt(1 - nv * nv), 0.0, nv])
        h = l + v
        h /= np.linalg.norm(h, axis=-1, keepdims=True)
        D = osh.ggx_D(h[..., 2], r)
        G = osh.smith_G(CL, nv, r)
        fc = (1 - (h @ v)) ** 5
        A = np.sum(W * D * G * (1 - fc) / (4 * nv))
        B = np.sum(W * D * G * fc / (4 * nv))
        assert abs(t[i, j, 0] - A) < 0.03 and abs(t[i, j, 1] - B) < 0.01, (i, j, t[i, j], A, B)


def test_relight_lind_closed_form():
    """A ray hitting a blended surface head on (N = -d): under a constant sky
    L the diffuse part is A irr / pi (= A L to the cube's accuracy) and the
    specular part L (F0 S_A + S_B) at the table cell (S - 1, floor(R S)); a
    ray with no hit carries nothing."""
    E, M, S = 16, 4, 8
    L = np.array([1.0, 2.0, 0.5])
    sky = np.broadcast_to(L, (6, E, E, 3))
    irr, pref, tab = rl.irradiance(sky), rl.prefilter(sky, M), rl.brdf_table(S)
    A, Rg = np.array([0.2, 0.5, 0.9]), 0.6
    O = np.array([0.8, 0.0])
    N = np.array([0.0, 0.0, 1.0])
    Fo = np.zeros((2, 7))
    Fo[0, :3], Fo[0, 3], Fo[0, 4:] = 0.8 * A, 0.8 * Rg, 0.8 * N
    rd = np.array([[0.0, 0.0, -1.0], [0.0, 0.0, -1.0]])
    got = rl.relight_lind(O, Fo, rd, irr, pref, tab)
    want = A * L + L * (osh.F0 * tab[S - 1, int(Rg * S), 0] + tab[S - 1, int(Rg * S), 1])
    np.testing.assert_allclose(got[0], want, rtol=4e-3)
    np.testing.assert_array_equal(got[1], 0)


def test_trace_oracle_normal_channels():
    """A lone splat facing +z hit through its centre: the normal channels
    hold o n for a ray coming down and -o n for a ray coming up (the normal
    faces the ray), after the plain feature channels."""
    import oracle
    S = [np.zeros((1, 3)), np.array([[1.0, 0, 0, 0]]), np.array([[0.1, 0.1]]), np.array([0.6]),
         np.array([[0.2, 0.4, 0.6, 0.8]])]
    ro = np.array([[0, 0, 1.0], [0, 0, -1.0]])
    rd = np.array([[0, 0, -1.0], [0, 0, 1.0]])
    r = oracle.trace(S, ro, rd, with_normal=True)
    assert r["F"].shape == (2, 7)
    np.testing.assert_allclose(r["F"][:, :4], 0.6 * S[4].repeat(2, 0), rtol=1e-15)
    np.testing.assert_allclose(r["F"][0, 4:], [0, 0, 0.6], atol=1e-15)
    np.testing.assert_allclose(r["F"][1, 4:], [0, 0, -0.6], atol=1e-15)
    rep = oracle.replay(S, ro, rd, np.array([[0], [0]], np.int32), np.array([1, 1], np.int32), with_normal=True)
    np.testing.assert_allclose(rep["F"], r["F"], rtol=1e-15)
