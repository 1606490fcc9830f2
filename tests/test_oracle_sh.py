"""Pins of the oracle's view-dependent colour (Sec. 3.1: colour modelled by
spherical harmonics; Sec. 3.3: the trace uses that colour): the real SH
basis against scipy and against its defining properties, the colour of a lone
splat in closed form, and gradients against finite differences."""
import math

import numpy as np
import pytest

import oracle
from oracle import grad as ograd


def _dirs(seed, n):
    d = np.random.default_rng(seed).standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_basis_matches_scipy(oracle_lib):
    """The C recurrence and scipy's harmonics (two independent routes) agree."""
    d = _dirs(40, 200)
    np.testing.assert_allclose(oracle.sh_basis(d, 3), ograd.sh_basis_scipy(d, 3), atol=1e-13)
    # unnormalised directions give the same basis
    np.testing.assert_allclose(oracle.sh_basis(3.7 * d, 3), oracle.sh_basis(d, 3), atol=1e-13)


def test_basis_orthonormal_on_the_sphere(oracle_lib):
    """Product quadrature (Gauss-Legendre in cos(polar) x uniform azimuth) is
    exact for products of degree <= 3 harmonics: the Gram matrix is I."""
    x, wx = np.polynomial.legendre.leggauss(8)
    az = (np.arange(16) + 0.5) * 2 * np.pi / 16
    ct, ph = np.meshgrid(x, az, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wx[:, None] * np.full(16, 2 * np.pi / 16)[None, :]).reshape(-1)
    Y = oracle.sh_basis(d, 3)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_basis_closed_forms(oracle_lib):
    """Y_00 = 1/(2 sqrt(pi)) everywhere; along +z only m = 0 survives with
    Y_l0 = sqrt((2l+1)/(4 pi)); the degree-1 signs fix the convention:
    Y_1,1(+x) = Y_1,-1(+y) = -sqrt(3/(4 pi)), Y_1,0(+z) = +sqrt(3/(4 pi))."""
    d = _dirs(41, 50)
    np.testing.assert_allclose(oracle.sh_basis(d, 0)[:, 0], 0.5 / math.sqrt(math.pi), rtol=1e-14)
    Yz = oracle.sh_basis(np.array([[0.0, 0.0, 1.0]]), 3)[0]
    for l in range(4):
        for m in range(-l, l + 1):
            want = math.sqrt((2 * l + 1) / (4 * math.pi)) if m == 0 else 0.0
            assert abs(Yz[l * l + l + m] - want) < 1e-14, (l, m)
    c1 = math.sqrt(3 / (4 * math.pi))
    assert abs(oracle.sh_basis(np.array([[1.0, 0, 0]]), 1)[0, 3] + c1) < 1e-14
    assert abs(oracle.sh_basis(np.array([[0, 1.0, 0]]), 1)[0, 1] + c1) < 1e-14
    # degree 2, m = -2 at (x, y, 0)/sqrt2: sqrt(15/(4 pi)) x y
    Y = oracle.sh_basis(np.array([[1.0, 1.0, 0.0]]), 2)[0]
    assert abs(Y[4] - math.sqrt(15 / (4 * math.pi)) * 0.5) < 1e-14


def _lone(k, o=0.8):
    """One splat at the origin facing +z, a ray down its centre."""
    mu = np.zeros((1, 3))
    q = np.array([[1.0, 0, 0, 0]])
    s = np.array([[0.1, 0.1]])
    return [mu, q, s, np.array([o]), np.asarray(k, float).reshape(1, -1)]


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_lone_splat_colour_closed_form(oracle_lib, deg):
    """Through the centre alpha = o, so F = o max(Y(d).k + 1/2, 0) with
    d = (0,0,-1): only the m = 0 terms act, Y_l0(-z) = (-1)^l sqrt((2l+1)/(4 pi))."""
    nb = (deg + 1) ** 2
    k = np.random.default_rng(42 + deg).uniform(-0.4, 0.4, (nb, 3))
    S = _lone(k)
    ro, rd = np.array([[0.0, 0.0, 1.0]]), np.array([[0.0, 0.0, -1.0]])
    r = oracle.trace(S, ro, rd, sh_deg=deg)
    col = np.full(3, 0.5)
    for l in range(deg + 1):
        col += (-1) ** l * math.sqrt((2 * l + 1) / (4 * math.pi)) * k[l * l + l]
    np.testing.assert_allclose(r["F"][0], 0.8 * np.maximum(col, 0), rtol=1e-13)
    assert r["F"].shape == (1, 3)
    assert abs(r["O"][0] - 0.8) < 1e-15


def test_colour_clamped_at_zero_and_replay_agrees(oracle_lib):
    k = np.zeros((4, 3))
    k[0] = [-5.0, 0.0, 1.0]          # very negative red, zero green (grey 1/2), bright blue
    S = _lone(k, o=0.5)
    ro, rd = np.array([[0.0, 0.0, 1.0]]), np.array([[0.0, 0.0, -1.0]])
    r = oracle.trace(S, ro, rd, sh_deg=1)
    c0 = 0.5 / math.sqrt(math.pi)
    np.testing.assert_allclose(r["F"][0], [0.0, 0.25, 0.5 * (0.5 + c0)], rtol=1e-14)
    rep = oracle.replay(S, ro, rd, np.array([[0]], np.int32), np.array([1], np.int32), sh_deg=1)
    np.testing.assert_allclose(rep["F"], r["F"], rtol=1e-14)
    with pytest.raises(ValueError):
        oracle.trace(S, ro, rd, sh_deg=2)   # 12 features need degree 1


def test_sh_gradients_match_finite_differences(oracle_lib):
    """Degree-3 colour on a small overlapping scene: FP64 autograd over the
    oracle's own hit lists against central differences of the brute-force
    oracle, every parameter group including the 48 coefficients."""
    g = np.random.default_rng(43)
    n, R = 32, 40
    mu = g.uniform(-0.15, 0.15, (n, 3))
    q = g.standard_normal((n, 4))
    s = np.exp(g.uniform(math.log(0.05), math.log(0.2), (n, 2)))
    o = g.uniform(0.1, 0.95, n)
    k = g.normal(0, 0.3, (n, 48))
    src = g.standard_normal((R, 3))
    src = 2.0 * src / np.linalg.norm(src, axis=1, keepdims=True)
    d = g.uniform(-0.1, 0.1, (R, 3)) - src
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    gO, gF, gD = g.standard_normal(R), g.standard_normal((R, 3)), g.standard_normal(R)
    S = [mu, q, s, o, k]
    ref = oracle.trace(S, src, d, hit_cap=64, sh_deg=3)
    assert ref["n_hits"].sum() > 80
    A = ograd.grad_given_hits(S, src, d, ref["hits"], gO, gF, gD, sh_deg=3)
    Fd, skipped = ograd.fd_grad(S, src, d, gO, gF, gD, hit_cap=64, sh_deg=3)
    total = 0
    for name in ("mu", "quat", "scale", "opac", "feat"):
        m = ~np.isnan(Fd[name])
        total += m.sum()
        scale = np.abs(A[name]).mean() + 1e-12
        err = np.abs(A[name][m] - Fd[name][m])
        assert np.all(err <= 1e-5 * (np.abs(A[name][m]) + scale)), (name, err.max(), scale)
    assert skipped < 0.05 * total
    assert np.abs(A["feat"]).max() > 0
