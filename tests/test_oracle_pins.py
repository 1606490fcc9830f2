"""Pins of the FP64 oracle against facts fixed by the paper's equations and by
mathematics -- closed forms, a library linear solve, invariants, special cases
and brute force -- so that a dropped term, a wrong sign, a transposed frame or
a wrong sort key in the oracle fails one of them.

Sec. 3.2: Eq. 6 (ray-plane depth), Eq. 7 (2D Gaussian at local u, v),
Eq. 2/8 (front-to-back blending), k-buffer marching gives the exact order.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from paper_2412_15867_amd import synth

AMIN = 1.0 / 255.0


def one_surfel(mu, q, s, o, f):
    return (np.asarray([mu], float), np.asarray([q], float), np.asarray([s], float),
            np.asarray([o], float), np.asarray([f], float))


def rand_quat(g):
    q = g.standard_normal(4)
    return q / np.linalg.norm(q)


def test_frame_matches_scipy_rotation(oracle_lib):
    """t_u, t_v are the first two columns of the rotation of q and n = t_u x t_v
    is its third column (library routine: scipy's quaternion -> matrix)."""
    g = np.random.default_rng(1)
    q = g.standard_normal((50, 4)) * g.uniform(0.1, 3.0, (50, 1))   # unnormalised on purpose
    tu, tv, n = oracle.frames(q)
    Rm = Rotation.from_quat(np.c_[q[:, 1:], q[:, :1]]).as_matrix()  # scipy is scalar-last
    np.testing.assert_allclose(tu, Rm[:, :, 0], atol=1e-13)
    np.testing.assert_allclose(tv, Rm[:, :, 1], atol=1e-13)
    np.testing.assert_allclose(n, Rm[:, :, 2], atol=1e-13)


def test_lone_splat_through_centre(oracle_lib):
    """A ray through a lone splat's centre: u = v = 0, G = 1, so O = o,
    F = o f, D = o tau0, T = 1 - o (Eq. 6-8)."""
    g = np.random.default_rng(2)
    for _ in range(20):
        mu = g.uniform(-1, 1, 3)
        q = rand_quat(g)
        s = np.exp(g.uniform(math.log(0.005), math.log(0.1), 2))
        o = g.uniform(0.05, 1.0)
        f = g.uniform(0, 1, 3)
        d = g.standard_normal(3)
        d /= np.linalg.norm(d)
        tau0 = g.uniform(0.5, 3.0)
        ro = mu - tau0 * d
        r = oracle.trace(one_surfel(mu, q, s, o, f), ro[None], d[None], hit_cap=4)
        assert r["n_hits"][0] == 1 and r["hits"][0, 0] == 0
        assert abs(r["O"][0] - o) <= 1e-12
        np.testing.assert_allclose(r["F"][0], o * f, atol=1e-12)
        assert abs(r["D"][0] - o * tau0) <= 1e-11
        assert abs(r["T"][0] - (1 - o)) <= 1e-12


def test_axis_aligned_oblique_closed_form(oracle_lib):
    """q = identity: t_u = x, t_v = y, n = z.  tau = (mu_z - o_z)/d_z,
    u = (p_x - mu_x)/s_u, v = (p_y - mu_y)/s_v (Eq. 6-7 specialised).
    q = 90 deg about z: t_u = y, t_v = -x."""
    g = np.random.default_rng(3)
    cases = 0
    for rot in ("id", "z90"):
        q = [1, 0, 0, 0] if rot == "id" else [math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)]
        for _ in range(200):
            mu = g.uniform(-0.5, 0.5, 3)
            s = g.uniform(0.05, 0.3, 2)
            o = g.uniform(0.2, 1.0)
            ro = mu + np.array([g.uniform(-0.3, 0.3), g.uniform(-0.3, 0.3), g.uniform(0.5, 2.0)])
            d = np.array([g.uniform(-0.3, 0.3), g.uniform(-0.3, 0.3), -1.0])
            d /= np.linalg.norm(d)
            tau = (mu[2] - ro[2]) / d[2]
            p = ro + tau * d
            if rot == "id":
                u, v = (p[0] - mu[0]) / s[0], (p[1] - mu[1]) / s[1]
            else:
                u, v = (p[1] - mu[1]) / s[0], -(p[0] - mu[0]) / s[1]
            a = o * math.exp(-(u * u + v * v) / 2)
            hit = (u * u + v * v <= 9) and a >= AMIN
            r = oracle.trace(one_surfel(mu, q, s, o, [1.0]), ro[None], d[None], hit_cap=2)
            if hit:
                cases += 1
                assert r["n_hits"][0] == 1
                assert abs(r["O"][0] - a) < 1e-12
                assert abs(r["D"][0] - a * tau) < 1e-11
            else:
                assert r["n_hits"][0] == 0 and r["O"][0] == 0.0
    assert cases > 50


def test_depth_and_uv_match_linear_solve(oracle_lib):
    """Library pin: the hit point solves r_o + tau r_d = mu + u s_u t_u + v s_v t_v
    (a 3x3 linear system, numpy.linalg.solve, frame from scipy)."""
    sc = synth.cube_scene(64, seed=11)
    g = np.random.default_rng(4)
    ro = g.uniform(-2, 2, (40, 3))
    tgt = sc.mu[g.integers(0, 64, 40)].astype(np.float64) + g.normal(0, 0.03, (40, 3))
    rd = tgt - ro
    rd /= np.linalg.norm(rd, axis=1, keepdims=True)
    c = oracle.candidates(sc.astuple(), ro, rd, cap=64, band=1e300, t_min=-np.inf)
    q = sc.quat.astype(np.float64)
    Rm = Rotation.from_quat(np.c_[q[:, 1:], q[:, :1]]).as_matrix()
    checked = 0
    for r in range(40):
        for k in range(c["count"][r]):
            i = c["ids"][r, k]
            s = sc.scale[i].astype(np.float64)
            A = np.stack([s[0] * Rm[i, :, 0], s[1] * Rm[i, :, 1], -rd[r]], 1)
            u, v, tau = np.linalg.solve(A, ro[r] - sc.mu[i].astype(np.float64))
            if abs(np.linalg.det(A)) < 1e-6:
                continue
            checked += 1
            assert abs(c["tau"][r, k] - tau) <= 1e-9 * max(1, abs(tau))
            assert abs(c["rho2"][r, k] - (u * u + v * v)) <= 1e-7 * max(1, u * u + v * v)
            a_ref = float(sc.opac[i]) * math.exp(-(u * u + v * v) / 2)
            assert abs(c["alpha"][r, k] - a_ref) <= 1e-7 * a_ref + 1e-15
    assert checked > 100


def test_parallel_stack_closed_form_and_cutoff(oracle_lib):
    """n coaxial splats crossed through their centres: alpha_i = o_i, hits in
    depth order; T after m hits = prod (1-o_j); with o = 0.2 the cutoff 1e-4 is
    crossed at hit ceil(ln 1e-4 / ln 0.8) = 42 (include-then-stop)."""
    g = np.random.default_rng(5)
    for n, expect in ((40, 40), (60, 42)):
        z = -0.05 * np.arange(n)
        perm = g.permutation(n)                    # storage order != depth order
        mu = np.stack([np.zeros(n), np.zeros(n), z], 1)[perm]
        q = np.tile([1.0, 0, 0, 0], (n, 1))
        s = np.full((n, 2), 0.1)
        o = np.full(n, 0.2)
        f = g.uniform(0, 1, (n, 3))[perm]
        r = oracle.trace((mu, q, s, o, f), np.array([[0, 0, 1.0]]), np.array([[0, 0, -1.0]]), hit_cap=64)
        assert r["n_hits"][0] == expect
        depth_order = np.argsort(-mu[:, 2], kind="stable")
        np.testing.assert_array_equal(r["hits"][0, :expect], depth_order[:expect])
        T = 0.8 ** np.arange(expect)
        tau = 1.0 + 0.05 * np.arange(expect)
        assert abs(r["O"][0] - (1 - 0.8 ** expect)) < 1e-13
        assert abs(r["T"][0] - 0.8 ** expect) < 1e-15
        assert abs(r["D"][0] - np.sum(T * 0.2 * tau)) < 1e-12
        np.testing.assert_allclose(r["F"][0], (T * 0.2) @ f[depth_order[:expect]], atol=1e-13)


def test_telescoping_and_replay(oracle_lib):
    """T_final = prod(1 - alpha_i) over the composited hits and O = 1 - T
    (Eq. 2 telescopes); replaying the oracle's own list reproduces it."""
    sc = synth.cube_scene(4096)
    ro, rd = synth.pinhole_rays(32, 32)
    r = oracle.trace(sc.astuple(), ro, rd, hit_cap=512)
    assert r["n_hits"].max() < 512
    np.testing.assert_allclose(r["O"] + r["T"], 1.0, atol=1e-12)
    rp = oracle.replay(sc.astuple(), ro, rd, r["hits"], r["n_hits"])
    mask = np.arange(512)[None, :] < r["n_hits"][:, None]
    prod = np.prod(np.where(mask, 1 - rp["alpha"], 1.0), axis=1)
    np.testing.assert_allclose(prod, r["T"], rtol=1e-12, atol=1e-300)
    for k in ("O", "D", "T"):
        np.testing.assert_allclose(rp[k], r[k], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(rp["F"], r["F"], rtol=1e-12, atol=1e-14)
    # T_min: only the last composited hit brings T below the cutoff
    nh = r["n_hits"]
    for i in np.nonzero(nh > 1)[0][:200]:
        Tp = rp["Tpost"][i, :nh[i]]
        assert np.all(Tp[:-1] >= 1e-4)


def test_support_and_alpha_thresholds(oracle_lib):
    """rho^2 <= 9 and alpha >= alpha_min are both inclusive; o < alpha_min never
    hits; a ray parallel to the plane (n . r_d = 0) never hits."""
    mu, q, s = [0, 0, 0], [1, 0, 0, 0], [0.1, 0.2]
    d = np.array([[0, 0, -1.0]])

    def hits_at(u, v, o):
        ro = np.array([[u * 0.1, v * 0.2, 1.0]])
        return oracle.trace(one_surfel(mu, q, s, o, [1]), ro, d)["n_hits"][0]

    assert hits_at(3 - 1e-9, 0, 1.0) == 1
    assert hits_at(3 + 1e-9, 0, 1.0) == 0
    assert hits_at(0, 3 - 1e-9, 1.0) == 1
    assert hits_at(0, 3 + 1e-9, 1.0) == 0
    # alpha = alpha_min * (1 +- 1e-9) at rho = 1 with o chosen accordingly
    o_edge = AMIN * math.exp(0.5)
    assert hits_at(1.0, 0, o_edge * (1 + 1e-9)) == 1
    assert hits_at(1.0, 0, o_edge * (1 - 1e-9)) == 0
    assert hits_at(0, 0, AMIN * 0.999) == 0
    assert hits_at(0, 0, AMIN) == 1
    ro = np.array([[-1.0, 0, 0]])
    assert oracle.trace(one_surfel(mu, q, s, 1.0, [1]), ro, np.array([[1.0, 0, 0]]))["n_hits"][0] == 0


def test_tmin_tmax_window(oracle_lib):
    """Only t_min < tau < t_max counts (both exclusive)."""
    mu = np.array([[0, 0, 0.0], [0, 0, -1.0]])
    q = np.tile([1.0, 0, 0, 0], (2, 1))
    s = np.full((2, 2), 0.1)
    o = np.array([0.5, 0.5])
    f = np.ones((2, 1))
    ro, rd = np.array([[0, 0, 1.0]]), np.array([[0, 0, -1.0]])
    S = (mu, q, s, o, f)
    assert oracle.trace(S, ro, rd)["n_hits"][0] == 2
    assert oracle.trace(S, ro, rd, t_min=1.0)["n_hits"][0] == 1
    assert oracle.trace(S, ro, rd, t_min=1.0 - 1e-12)["n_hits"][0] == 2
    assert oracle.trace(S, ro, rd, t_max=2.0)["n_hits"][0] == 1
    assert oracle.trace(S, ro, rd, t_max=2.0 + 1e-12)["n_hits"][0] == 2
    assert oracle.trace(S, np.array([[0, 0, -2.0]]), rd)["n_hits"][0] == 0   # both behind the origin


def test_permutation_invariance(oracle_lib):
    """Storage order does not change the result; hit ids map through the
    permutation."""
    sc = synth.cube_scene(4096)
    ro, rd = synth.pinhole_rays(32, 32)
    perm = np.random.default_rng(6).permutation(4096)
    a = oracle.trace(sc.astuple(), ro, rd, hit_cap=256)
    b = oracle.trace(sc.permuted(perm).astuple(), ro, rd, hit_cap=256)
    for k in ("O", "D", "T"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(a["F"], b["F"], rtol=1e-13, atol=1e-15)
    np.testing.assert_array_equal(a["n_hits"], b["n_hits"])
    mapped = np.where(b["hits"] >= 0, perm[np.maximum(b["hits"], 0)], -1)
    np.testing.assert_array_equal(a["hits"], mapped)


def test_empty_scene_and_misses(oracle_lib):
    e = (np.zeros((0, 3)), np.zeros((0, 4)), np.zeros((0, 2)), np.zeros(0), np.zeros((0, 3)))
    ro, rd = synth.pinhole_rays(8, 8)
    r = oracle.trace(e, ro, rd)
    assert np.all(r["O"] == 0) and np.all(r["T"] == 1) and np.all(r["D"] == 0) and np.all(r["F"] == 0)
    sc = synth.cube_scene(4096)
    r = oracle.trace(sc.astuple(), ro, -rd)        # pointing away from the cube
    assert np.all(r["n_hits"] == 0) and np.all(r["O"] == 0) and np.all(r["T"] == 1)
    bad_o = np.array([[np.nan, 0, 3.0], [0, 0, 3.0], [0, 0, 3.0]])
    bad_d = np.array([[0, 0, -1.0], [0, 0, 0.0], [np.inf, 0, -1]])
    r = oracle.trace(sc.astuple(), bad_o, bad_d)
    assert np.all(r["n_hits"] == 0) and np.all(r["T"] == 1)


def test_plane_of_surfels_upward_rays_visibility_one(oracle_lib):
    """Origin above an infinite plane of surfels, rays in the upper hemisphere:
    no hit, V = 1 - O = 1 exactly (Eq. 14)."""
    g = np.random.default_rng(7)
    n = 2000
    mu = np.c_[g.uniform(-1, 1, (n, 2)), np.zeros(n)]
    q = np.tile([1.0, 0, 0, 0], (n, 1))
    s = np.exp(g.uniform(math.log(0.005), math.log(0.02), (n, 2)))
    o = g.uniform(0.5, 1, n)
    f = g.uniform(0, 1, (n, 8))
    nrm = np.tile([0, 0, 1.0], (64, 1))
    d = synth.cosine_dirs(g, nrm, 16).reshape(-1, 3)
    ro = np.repeat(np.c_[g.uniform(-0.5, 0.5, (64, 2)), np.full(64, 1e-3)], 16, 0)
    r = oracle.trace((mu, q, s, o, f), ro, d)
    assert np.all(r["n_hits"] == 0) and np.all(1 - r["O"] == 1.0)
    r = oracle.trace((mu, q, s, o, f), ro, -d)     # downward: the plane occludes
    assert np.mean(r["n_hits"] > 0) > 0.5


def kbuffer_march(cand_tau, cand_id, cand_alpha, k, T_min):
    """The paper's k-buffer marching (after 3DGRT), in FP64 over a candidate
    list: each round keeps the k nearest hits strictly after the last one
    composited, composites them, and resumes.  Used to pin that the plain
    sort is what the marching reaches, for any k."""
    last = (-np.inf, -1)
    out, T = [], 1.0
    while True:
        buf = []
        for t, i, a in zip(cand_tau, cand_id, cand_alpha):
            if (t, i) > last:
                buf.append((t, i, a))
                buf.sort()
                buf = buf[:k]
        for t, i, a in buf:
            out.append(i)
            T *= 1 - a
            if T < T_min:
                return out
        if len(buf) < k:
            return out
        last = buf[-1][:2]


@pytest.mark.parametrize("k", [1, 2, 16, 64])
def test_kbuffer_marching_equals_sort(oracle_lib, k):
    sc = synth.cube_scene(4096)
    ro, rd = synth.pinhole_rays(16, 16)
    r = oracle.trace(sc.astuple(), ro, rd, hit_cap=256)
    c = oracle.candidates(sc.astuple(), ro, rd, cap=512)
    for i in range(ro.shape[0]):
        m = c["hit"][i, :c["count"][i]]
        ids = c["ids"][i, :c["count"][i]][m]
        lst = kbuffer_march(c["tau"][i, :c["count"][i]][m], ids, c["alpha"][i, :c["count"][i]][m], k, 1e-4)
        assert lst == list(r["hits"][i, :r["n_hits"][i]])


def test_surface_generator_frames(oracle_lib):
    """Generated quaternions put n = t_u x t_v on the surface normal (sphere:
    radial direction) and make (t_u, t_v, n) orthonormal."""
    lay = synth.layout()
    sc, sid = synth.surface_scene(20000, lay=lay, return_surface_id=True)
    tu, tv, n = oracle.frames(sc.quat)
    np.testing.assert_allclose(np.sum(tu * tv, 1), 0, atol=1e-6)
    np.testing.assert_allclose(np.linalg.norm(n, axis=1), 1, atol=1e-6)
    mu = sc.mu.astype(np.float64)
    on_sphere = sid < 8
    k = sid[on_sphere]
    radial = (mu[on_sphere] - lay.centers[k]) / lay.radii[k][:, None]
    np.testing.assert_allclose(np.linalg.norm(radial, axis=1), 1, atol=1e-5)
    np.testing.assert_allclose(np.sum(n[on_sphere] * radial, 1), 1, atol=1e-5)
    pn = lay.p_normal[sid[~on_sphere] - 8]
    np.testing.assert_allclose(np.sum(n[~on_sphere] * pn, 1), 1, atol=1e-5)
    assert on_sphere.mean() > 0.3


def test_cosine_hemisphere_moments():
    """Cosine-weighted directions: E[cos] = 2/3, all in the upper hemisphere."""
    g = np.random.default_rng(8)
    nrm = synth._unit(g.standard_normal((32, 3)))
    d = synth.cosine_dirs(g, nrm, 4096)
    c = np.sum(d * nrm[:, None, :], -1)
    assert c.min() >= 0
    assert abs(c.mean() - 2 / 3) < 3e-3
    np.testing.assert_allclose(np.linalg.norm(d, axis=-1), 1, atol=1e-12)
