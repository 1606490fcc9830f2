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


def _quad_cos_integral(env, nrm, m=24):
    """int L(w) max(w . nrm, 0) dw for the piecewise-constant cubemap, by an
    m x m midpoint rule inside every texel in the face coordinates
    (dw = ds dt / (1 + s^2 + t^2)^{3/2}); independent of the sampler."""
    E = env.shape[1]
    c = (np.arange(E * m) + 0.5) / (E * m) * 2.0 - 1.0
    t, s = np.meshgrid(c, c, indexing="ij")
    jac = (2.0 / (E * m)) ** 2 / (1.0 + s * s + t * t) ** 1.5
    tot = 0.0
    for f in range(6):
        d = rl.face_point(f, s, t)
        d = d / np.linalg.norm(d, axis=-1, keepdims=True)
        cos = np.maximum(d @ nrm, 0.0)
        L = env[f].mean(-1).repeat(m, 0).repeat(m, 1)
        tot += np.sum(L * cos * jac)
    return tot


def test_env_sampling_one_hot_sky():
    """A sky lit in one texel: every sample lands in that texel, with
    density E^2/4 (1 + s^2 + t^2)^{3/2} (probability 1 for the texel)."""
    E, P, N = 4, 2, 500
    env = np.zeros((6, E, E, 3))
    env[2, 1, 3] = [1.0, 2.0, 3.0]                              # face +y, row 1, col 3
    cdf = rl.env_cdf(env)
    assert np.all(np.diff(cdf) >= 0)
    g = np.random.default_rng(81)
    u = g.random((P, N, 3))
    n = np.array([[0, 1.0, 0], [0, -1.0, 0]])
    ro, rd, w = rl.env_sample(np.zeros((P, 3)), n, u, cdf.astype(np.float32), E)
    f, r, c = osh.cube_texel(rd.reshape(-1, 3), E)
    assert np.all(f == 2) and np.all(r == 1) and np.all(c == 3)
    s = (3 + u[..., 1]) * 2.0 / E - 1.0
    t = (1 + u[..., 2]) * 2.0 / E - 1.0
    pdf = E * E / 4.0 * (1 + s * s + t * t) ** 1.5
    np.testing.assert_allclose(w[0], 1.0 / (N * pdf[0]), rtol=1e-12)
    np.testing.assert_array_equal(w[1], 0.0)                    # the lit texel is below this horizon
    np.testing.assert_allclose(ro, np.broadcast_to((1e-3 * n)[:, None, :], ro.shape))


def test_env_sampling_frequencies_and_unbiased_estimate():
    """Texels are drawn with the CDF's probabilities, and the weighted sum
    sum_i w_i L(w_i) (w_i . n) estimates the integral of L cos over the
    hemisphere, computed independently by quadrature (within 5 sigma)."""
    E = 2
    g = np.random.default_rng(82)
    env = g.uniform(0.0, 1.0, (6, E, E, 3)) ** 3 * 10         # contrasty sky
    cdf = rl.env_cdf(env)
    _, dw = rl.texel_dirs(E)
    np.testing.assert_allclose(cdf[-1], np.sum(env.mean(-1) * dw[None]), rtol=1e-12)
    p = np.diff(np.concatenate([[0.0], cdf])) / cdf[-1]
    N = 400_000
    nrm = np.array([0.3, 0.5, 0.81])
    nrm /= np.linalg.norm(nrm)
    u = g.random((1, N, 3))
    _, rd, w = rl.env_sample(np.zeros((1, 3)), nrm[None], u, cdf.astype(np.float32), E)
    f, r, c = osh.cube_texel(rd[0], E)
    cnt = np.bincount((f * E + r) * E + c, minlength=6 * E * E) / N
    assert np.all(np.abs(cnt - p) <= 5 * np.sqrt(p * (1 - p) / N) + 1e-12)
    L = env[f, r, c].mean(-1)
    terms = N * w[0] * L * np.maximum(rd[0] @ nrm, 0.0)        # one-sample estimates
    est, sig = terms.mean(), terms.std() / np.sqrt(N)
    ref = _quad_cos_integral(env, nrm)
    assert abs(est - ref) < 5 * sig, (est, ref, sig)
    # a uniform sky: the estimate of the cosine integral is pi
    one = np.ones((6, 8, 8, 3))
    _, rd1, w1 = rl.env_sample(np.zeros((1, 3)), nrm[None], u[:, :100_000], rl.env_cdf(one).astype(np.float32), 8)
    t1 = 100_000 * w1[0] * np.maximum(rd1[0] @ nrm, 0.0)
    assert abs(t1.mean() - math.pi) < 5 * t1.std() / np.sqrt(t1.size)


def test_weighted_shading_reduces_to_stratified():
    """Eq. 15 with every weight 2 pi / N is the stratified estimator."""
    g = np.random.default_rng(83)
    P, N, E = 3, 8, 4
    n = np.tile([0, 0, 1.0], (P, 1))
    wo = osh.stratified_dirs(n, g.random((P, 1, 2)), 1, 1)[:, 0]
    a, r = g.random((P, 3)), g.uniform(0.1, 0.9, P)
    wi = osh.stratified_dirs(n, g.random((P, N, 2)), 2, 4)
    O, L, env = g.random((P, N)), g.random((P, N, 3)), g.random((6, E, E, 3))
    wgt = np.full((P, N), 2 * math.pi / N)
    np.testing.assert_allclose(osh.shade(n, wo, a, r, wi, O, L, env, wgt=wgt),
                               osh.shade(n, wo, a, r, wi, O, L, env), rtol=1e-13)
    g1 = osh.shade_grad(n, wo, a, r, wi, O, L, env, np.ones((P, 3)), wgt=wgt)
    g2 = osh.shade_grad(n, wo, a, r, wi, O, L, env, np.ones((P, 3)))
    for k in g1:
        np.testing.assert_allclose(g1[k], g2[k], rtol=1e-12, atol=1e-15)
