"""Pins of the FP64 gradient oracle (autograd over a given hit list):
closed-form derivatives of single-splat cases (Eq. 6-7) and central finite
differences of the brute-force C oracle (which re-selects and re-sorts the
hits) on small scenes."""
import math

import numpy as np

import oracle
from oracle import grad as ograd


def one(mu, q, s, o, f):
    return [np.asarray([mu], float), np.asarray([q], float), np.asarray([s], float),
            np.asarray([o], float), np.asarray([f], float)]


def test_lone_centre_ray_gradients(oracle_lib):
    """Ray through the centre: dO/do = 1, dO/dmu = 0, dO/dq = 0, dO/ds = 0,
    dD/dmu = o n / (n . r_d), dF/df = o."""
    g = np.random.default_rng(10)
    for _ in range(10):
        q = g.standard_normal(4)
        mu = g.uniform(-1, 1, 3)
        o = g.uniform(0.1, 1)
        S = one(mu, q, g.uniform(0.01, 0.1, 2), o, g.uniform(0, 1, 3))
        d = g.standard_normal(3)
        d /= np.linalg.norm(d)
        ro = mu - 1.5 * d
        lists = np.array([[0]])
        gO = ograd.grad_given_hits(S, ro[None], d[None], lists, [1.0], [[0, 0, 0]], [0.0])
        assert abs(gO["opac"][0] - 1) < 1e-12
        np.testing.assert_allclose(gO["mu"], 0, atol=1e-10)
        np.testing.assert_allclose(gO["quat"], 0, atol=1e-10)
        np.testing.assert_allclose(gO["scale"], 0, atol=1e-10)
        gD = ograd.grad_given_hits(S, ro[None], d[None], lists, [0.0], [[0, 0, 0]], [1.0])
        _, _, n = oracle.frames(q[None])
        np.testing.assert_allclose(gD["mu"][0], o * n[0] / np.dot(n[0], d), rtol=1e-9, atol=1e-12)
        assert abs(np.dot(gD["mu"][0], d) - o) < 1e-10
        gF = ograd.grad_given_hits(S, ro[None], d[None], lists, [0.0], [[1, 1, 1]], [0.0])
        np.testing.assert_allclose(gF["feat"][0], o, atol=1e-12)


def test_axis_aligned_oblique_gradients(oracle_lib):
    """q = identity, oblique ray: alpha = o exp(-(u^2+v^2)/2) with
    u = (p_x-mu_x)/s_u, v = (p_y-mu_y)/s_v, p on z = mu_z; so
    d alpha/d mu_x = alpha u / s_u, d alpha/d mu_z = -alpha (u d_x/(d_z s_u) + v d_y/(d_z s_v)),
    d alpha/d s_u = alpha u^2 / s_u, d alpha/d o = alpha / o."""
    g = np.random.default_rng(11)
    for _ in range(20):
        mu = g.uniform(-0.5, 0.5, 3)
        s = g.uniform(0.05, 0.3, 2)
        o = g.uniform(0.2, 1)
        ro = mu + np.array([g.uniform(-.1, .1), g.uniform(-.1, .1), 1.0])
        d = np.array([g.uniform(-.1, .1), g.uniform(-.1, .1), -1.0])
        d /= np.linalg.norm(d)
        tau = (mu[2] - ro[2]) / d[2]
        p = ro + tau * d
        u, v = (p[0] - mu[0]) / s[0], (p[1] - mu[1]) / s[1]
        a = o * math.exp(-(u * u + v * v) / 2)
        G = ograd.grad_given_hits(one(mu, [1, 0, 0, 0], s, o, [1]), ro[None], d[None], [[0]], [1.0], [[0]], [0.0])
        np.testing.assert_allclose(G["mu"][0, 0], a * u / s[0], rtol=1e-9)
        np.testing.assert_allclose(G["mu"][0, 1], a * v / s[1], rtol=1e-9)
        np.testing.assert_allclose(G["mu"][0, 2], -a * (u * d[0] / (d[2] * s[0]) + v * d[1] / (d[2] * s[1])),
                                   rtol=1e-8, atol=1e-12)
        np.testing.assert_allclose(G["scale"][0], [a * u * u / s[0], a * v * v / s[1]], rtol=1e-9)
        np.testing.assert_allclose(G["opac"][0], a / o, rtol=1e-12)


def test_two_layer_blend_gradient(oracle_lib):
    """Two coaxial splats (alpha = o1, o2): O = o1 + (1-o1) o2, so
    dO/do1 = 1 - o2 and dO/do2 = 1 - o1; F = o1 f1 + (1-o1) o2 f2."""
    S = [np.array([[0, 0, 0.0], [0, 0, -1.0]]), np.tile([1.0, 0, 0, 0], (2, 1)), np.full((2, 2), 0.1),
         np.array([0.3, 0.6]), np.array([[1.0], [5.0]])]
    ro, rd = np.array([[0, 0, 1.0]]), np.array([[0, 0, -1.0]])
    G = ograd.grad_given_hits(S, ro, rd, [[0, 1]], [1.0], [[0.0]], [0.0])
    np.testing.assert_allclose(G["opac"], [1 - 0.6, 1 - 0.3], rtol=1e-12)
    G = ograd.grad_given_hits(S, ro, rd, [[0, 1]], [0.0], [[1.0]], [0.0])
    np.testing.assert_allclose(G["opac"], [1.0 - 0.6 * 5.0, 0.7 * 5.0], rtol=1e-12)
    np.testing.assert_allclose(G["feat"][:, 0], [0.3, 0.7 * 0.6], rtol=1e-12)


def _small_scene(seed, n=48):
    g = np.random.default_rng(seed)
    mu = g.uniform(-0.15, 0.15, (n, 3))
    q = g.standard_normal((n, 4))
    s = np.exp(g.uniform(math.log(0.05), math.log(0.2), (n, 2)))
    o = g.uniform(0.1, 0.95, n)
    f = g.uniform(0, 1, (n, 3))
    R = 48
    src = g.standard_normal((R, 3))
    src = 2.0 * src / np.linalg.norm(src, axis=1, keepdims=True)
    tgt = g.uniform(-0.1, 0.1, (R, 3))
    d = tgt - src
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    gO, gF, gD = g.standard_normal(R), g.standard_normal((R, 3)), g.standard_normal(R)
    return [mu, q, s, o, f], src, d, gO, gF, gD


def test_autograd_matches_finite_differences(oracle_lib):
    """FP64 central differences of L through the brute-force oracle agree with
    autograd over the oracle's own hit lists (parameters whose perturbation
    changes a hit list are skipped and counted)."""
    S, ro, rd, gO, gF, gD = _small_scene(12)
    ref = oracle.trace(S, ro, rd, hit_cap=64)
    assert ref["n_hits"].max() < 64 and ref["n_hits"].sum() > 100
    A = ograd.grad_given_hits(S, ro, rd, ref["hits"], gO, gF, gD)
    Fd, skipped = ograd.fd_grad(S, ro, rd, gO, gF, gD, hit_cap=64)
    total = 0
    for name in ("mu", "quat", "scale", "opac", "feat"):
        m = ~np.isnan(Fd[name])
        total += m.sum()
        scale = np.abs(A[name]).mean() + 1e-12
        err = np.abs(A[name][m] - Fd[name][m])
        assert np.all(err <= 1e-5 * (np.abs(A[name][m]) + scale)), (name, err.max(), scale)
    assert skipped < 0.05 * total


def test_facing_normal_gradient_closed_form(oracle_lib):
    """Lone splat, ray through its centre, upstream gradient only on the 3
    normal channels: L = g_N . (o s n(q)) with s = -1 where n . d > 0
    (the normal turned to face the ray), alpha = o independent of q at the
    centre.  So dL/dq = o s J(q)^T g_N, J the Jacobian of the third column of
    scipy's rotation matrix of the raw quaternion (central differences of
    scipy, an implementation independent of the oracle's frame), dL/do =
    s g_N . n, dL/dmu = 0 and the feature gradient is 0."""
    from scipy.spatial.transform import Rotation
    g = np.random.default_rng(13)

    def ncol(q):  # scipy takes (x, y, z, w)
        return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()[:, 2]

    for trial in range(12):
        q = g.standard_normal(4)
        mu = g.uniform(-1, 1, 3)
        o = g.uniform(0.1, 1)
        S = one(mu, q, g.uniform(0.01, 0.1, 2), o, g.uniform(0, 1, 2))
        n = ncol(q)
        d = g.standard_normal(3)
        d /= np.linalg.norm(d)
        if abs(np.dot(n, d)) < 0.2:
            continue
        sgn = -1.0 if np.dot(n, d) > 0 else 1.0
        gN = g.standard_normal(3)
        ro = mu - 1.5 * d
        A = ograd.grad_given_hits(S, ro[None], d[None], np.array([[0]]), [0.0], [np.r_[0.0, 0.0, gN]], [0.0],
                                  with_normal=True)
        J = np.zeros((3, 4))
        for k in range(4):
            h = 1e-6
            e = np.zeros(4)
            e[k] = h
            J[:, k] = (ncol(q + e) - ncol(q - e)) / (2 * h)
        np.testing.assert_allclose(A["quat"][0], o * sgn * (J.T @ gN), rtol=1e-6, atol=1e-8)
        assert abs(A["opac"][0] - sgn * np.dot(gN, n)) < 1e-10
        np.testing.assert_allclose(A["mu"], 0, atol=1e-9)
        np.testing.assert_allclose(A["feat"], 0, atol=1e-12)


def test_facing_normal_autograd_matches_finite_differences(oracle_lib):
    """With the facing-normal channels (the relighting blend), FP64 central
    differences through the brute-force C oracle's own normal channels agree
    with autograd over the oracle's hit lists."""
    S, ro, rd, gO, gF, gD = _small_scene(14)
    gF6 = np.random.default_rng(15).standard_normal((ro.shape[0], S[4].shape[1] + 3))
    ref = oracle.trace(S, ro, rd, hit_cap=64, with_normal=True)
    assert ref["F"].shape[1] == S[4].shape[1] + 3
    A = ograd.grad_given_hits(S, ro, rd, ref["hits"], gO, gF6, gD, with_normal=True)
    Fd, skipped = ograd.fd_grad(S, ro, rd, gO, gF6, gD, hit_cap=64, with_normal=True)
    total = 0
    for name in ("mu", "quat", "scale", "opac", "feat"):
        m = ~np.isnan(Fd[name])
        total += m.sum()
        scale = np.abs(A[name]).mean() + 1e-12
        err = np.abs(A[name][m] - Fd[name][m])
        assert np.all(err <= 1e-5 * (np.abs(A[name][m]) + scale)), (name, err.max(), scale)
    assert skipped < 0.05 * total
