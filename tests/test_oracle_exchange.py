"""Pins of the oracle's Adaptive Type Exchange (Sec. 3.2, Eq. 3; appendix
"Effective Rank and Type Switch"): closed forms of erank, the paper's
stated non-monotone root, covariance invariance of the P_x / P_y
reparameterisation checked with an independent covariance routine, proper
rotations, the switch rules, and unchanged renders of reparameterised 3D
Gaussians."""
import numpy as np
import pytest

import scenegen as sg


@pytest.fixture(scope="module")
def O():
    import oracle
    oracle.build(force=False)
    return oracle


def cov(s, q):
    """Sigma = R diag(s^2) R^T with R from the normalised quaternion (w, x, y, z)."""
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    return R @ np.diag(np.asarray(s, np.float64) ** 2) @ R.T, R


def test_erank_closed_forms(O):
    # isotropic 3, flat 2, line 1 (Eq. 3 with p uniform over 3, 2, 1 entries)
    for a in (1e-3, 0.5, 1.0, 7.0):
        assert O.erank(a, a, a) == pytest.approx(3.0, abs=1e-12)
        assert O.erank(a, a, 0.0) == pytest.approx(2.0, abs=1e-12)
        assert O.erank(0.0, a, a) == pytest.approx(2.0, abs=1e-12)
        assert O.erank(a, 0.0, 0.0) == pytest.approx(1.0, abs=1e-12)
    # two equal weights p, p and 1 - 2p: exp(-2 p log p - (1-2p) log(1-2p))
    s = np.array([1.0, 1.0, np.sqrt(2.0)])  # q = (1, 1, 2), p = (1/4, 1/4, 1/2)
    assert O.erank(*s) == pytest.approx(np.exp(1.5 * np.log(2.0)), rel=1e-12)
    # scale invariance
    assert O.erank(0.3, 0.7, 1.9) == pytest.approx(O.erank(3.0, 7.0, 19.0), rel=1e-12)
    assert O.erank(0.0, 0.0, 0.0) == 0.0


def test_erank_root_stated_in_the_paper(O):
    # erank(1, 1, s_z) rises to 3 at s_z = 1 and returns to 2 near s_z = 2.6
    f = lambda sz: O.erank(1.0, 1.0, sz) - 2.0
    lo, hi = 1.0, 4.0
    assert f(lo) > 0 > f(hi)
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) > 0 else (lo, mid)
    assert abs(lo - 2.609) < 1e-3
    assert O.erank(1.0, 1.0, 1.0) > O.erank(1.0, 1.0, 2.0) > O.erank(1.0, 1.0, 2.609)


def _random_gaussians(n, seed):
    rng = np.random.default_rng(seed)
    s = np.exp(rng.normal(-3.0, 1.0, (n, 3))).astype(np.float32)
    flat = rng.random(n) < 0.4
    s[flat, rng.integers(0, 3, flat.sum())] *= 1e-3  # one axis much smaller
    q = rng.normal(size=(n, 4)).astype(np.float32) * rng.uniform(0.5, 3.0, (n, 1)).astype(np.float32)
    t = (rng.random(n) < 0.5).astype(np.uint8)
    return s, q, t


def test_reparameterisation_keeps_covariance_and_handedness(O):
    s, q, t = _random_gaussians(400, 5)
    t[:] = 1
    r = O.type_exchange(s, q, t, theta=3.5)  # every 3D Gaussian converts
    assert (r["types"] == 0).all()
    moved = 0
    for i in range(len(s)):
        S0, _ = cov(s[i], q[i])
        S1, R1 = cov(r["scales"][i], r["quats"][i])
        assert np.abs(S1 - S0).max() <= 1e-12 * max(1.0, np.abs(S0).max())
        assert np.linalg.det(R1) > 0.0
        # the least significant scale is now the z one
        assert r["scales"][i][2] == s[i].min()
        assert sorted(r["scales"][i].tolist()) == sorted(s[i].tolist())
        moved += int(r["moved"][i] != 0)
    assert moved > 100


def test_permutation_matrices_as_written(O):
    # s_x least -> P_x: S* = diag(s_y, s_z, s_x); s_y least -> P_y: diag(s_z, s_x, s_y)
    q = np.array([[1.0, 0.0, 0.0, 0.0]] * 3, np.float32)
    s = np.array([[0.01, 0.5, 0.7], [0.5, 0.01, 0.7], [0.5, 0.7, 0.01]], np.float32)
    r = O.type_exchange(s, q, np.ones(3, np.uint8), theta=2.05)
    np.testing.assert_array_equal(r["moved"], [1, 2, 0])
    np.testing.assert_array_equal(r["scales"][0], s[0][[1, 2, 0]])
    np.testing.assert_array_equal(r["scales"][1], s[1][[2, 0, 1]])
    np.testing.assert_array_equal(r["scales"][2], s[2])
    # R* = P^T for R = I: P_x^T maps e_x -> e_y (the new x axis is the old y)
    _, R0 = cov(r["scales"][0], r["quats"][0])
    np.testing.assert_allclose(R0, np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]], float), atol=1e-12)


def test_switch_rules(O):
    q = np.tile(np.array([[0.9, 0.1, -0.3, 0.2]], np.float32), (6, 1))
    s = np.array([[0.2, 0.2, 0.2],      # 3D isotropic: stays 3D (erank 3)
                  [0.2, 0.3, 0.001],    # 3D flat: to 2D
                  [0.2, 0.2, 0.0],      # 2D flat: stays 2D (erank 2 < 2.05)
                  [0.2, 0.25, 0.18],    # 2D grown volumetric: to 3D
                  [0.0, 0.0, 0.0],      # degenerate: unchanged
                  [0.3, 0.001, 0.2]],   # 3D flat in y: to 2D through P_y
                 np.float32)
    t = np.array([1, 1, 0, 0, 1, 1], np.uint8)
    r = O.type_exchange(s, q, t, theta=2.05)
    np.testing.assert_array_equal(r["types"], [1, 0, 0, 1, 1, 0])
    np.testing.assert_array_equal(r["moved"], [0, 0, 0, 0, 0, 2])
    np.testing.assert_array_equal(r["scales"][3], s[3])  # 2D -> 3D keeps parameters


def test_reparameterised_3d_gaussians_render_the_same(O):
    """P7: a 3D Gaussian depends only on Sigma, so (S*, R*) renders like
    (S, R), normals included (the least-scale axis is the same axis)."""
    scene = sg.scene_random(60, seed=21, frac2d=0.0, log_mu=-2.5, log_sigma=0.5)
    cam = sg.look_at_camera((0.2, -0.1, -3.5), width=48, height=40, fx=45.0)
    r = O.type_exchange(scene["scales"], scene["rotations"], scene["types"], theta=3.5)
    assert (r["moved"] != 0).sum() > 20
    rep = dict(scene)
    rep["scales"] = r["scales"]
    rep["rotations"] = r["quats"].astype(np.float32)
    pix = O.full_pixels(cam)
    a = O.forward(scene, cam, pix, params64=None)
    # binary64 parameters of the reparameterised scene: exact permutation and
    # the binary64 quaternion
    p64 = {k: np.asarray(rep[k], np.float64) for k in ("means", "scales", "opacities", "sh")}
    p64["rotations"] = r["quats"]
    b = O.forward(rep, cam, pix, params64=p64)
    ok = (a["tie"] == 0) & (b["tie"] == 0)
    assert ok.mean() > 0.99
    assert np.abs(a["out"][ok] - b["out"][ok]).max() <= 1e-9
    np.testing.assert_array_equal(a["n_contrib"][ok], b["n_contrib"][ok])
