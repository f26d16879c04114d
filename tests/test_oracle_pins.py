"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test names the passage it follows.  None of them re-types the oracle's
general formulas: they use closed forms of special cases, the paper's own
alternative formulation (Eq. uv), invariances the paper proves, independent
library routines (scipy's spherical harmonics and rotations), brute force,
and finite differences.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenegen as sg
from tests.helpers import axis_camera, central_fd, make_scene, pack_G, grad_close

A_MIN = 1.0 / 255.0


def run(oracle_lib, scene, cam, opts=None, **kw):
    res = oracle_lib.forward(scene, cam, oracle_lib.full_pixels(cam), opts, **kw)
    return res, oracle_lib.images(res, cam)


def quat_wxyz_from_matrix(R):
    x, y, z, w = Rotation.from_matrix(R).as_quat()
    return np.array([w, x, y, z])


def matrix_from_quat_wxyz(q):
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


# ---------------------------------------------------------------------------
# P1: single primitive, closed form (Sec. 3.1 contribution alpha e^{-d/2},
# appendix: affine projection for 3D, ray-splat intersection for 2D).
# ---------------------------------------------------------------------------
def test_single_isotropic_3d_on_axis(oracle_lib):
    z, f, s, a, delta = 4.0, 64.0, 0.2, 0.7, 0.3
    cam = axis_camera(z=z, f=f)
    sc = make_scene([0, 0, 0], [s, s, s], [1, 0, 0, 0], a, np.zeros((1, 1, 3)), [1])
    res, im = run(oracle_lib, sc, cam, dict(dilation=delta))
    s32, d32 = float(np.float32(s)), float(np.float32(delta))  # the oracle's inputs are binary32
    sig2 = (f * s32 / z) ** 2 + d32
    ii = np.arange(64) + 0.5 - 32.0
    r2 = ii[:, None] ** 2 + ii[None, :] ** 2
    at = np.float32(a) * np.exp(-r2 / (2 * sig2))
    active = at >= A_MIN
    tie = im["tie"][0] != 0
    exp = np.where(active, at, 0.0)
    ok = ~tie
    assert tie.sum() < 10
    np.testing.assert_allclose(im["alpha"][0, 0][ok], exp[ok], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(im["rgb"][0][:, ok], 0.5 * np.stack([exp[ok]] * 3), atol=1e-14)
    np.testing.assert_allclose(im["depth"][0, 0][ok], z * exp[ok], atol=1e-13)
    np.testing.assert_allclose(im["normal"][0][2][ok], -exp[ok], atol=1e-14)
    np.testing.assert_allclose(im["normal"][0][:2][:, ok], 0.0, atol=1e-14)


def test_single_surfel_fronto_parallel(oracle_lib):
    z, f, a = 4.0, 64.0, 0.8
    sx, sy = 0.25, 0.12
    cam = axis_camera(z=z, f=f, W=80, H=48, cx=37.0, cy=21.0)
    sc = make_scene([0, 0, 0], [sx, sy, 0], [1, 0, 0, 0], a, np.zeros((1, 1, 3)), [0])
    res, im = run(oracle_lib, sc, cam)
    X = z * (np.arange(80) + 0.5 - 37.0) / f
    Y = z * (np.arange(48) + 0.5 - 21.0) / f
    d = (X[None, :] / np.float32(sx)) ** 2 + (Y[:, None] / np.float32(sy)) ** 2
    at = np.minimum(0.99, np.float32(a) * np.exp(-0.5 * d))
    exp = np.where(at >= A_MIN, at, 0.0)
    ok = im["tie"][0] == 0
    np.testing.assert_allclose(im["alpha"][0, 0][ok], exp[ok], rtol=1e-11, atol=1e-15)
    np.testing.assert_allclose(im["depth"][0, 0][ok], z * exp[ok], rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(im["normal"][0][2][ok], -exp[ok], atol=1e-14)


def test_ewa_offaxis_matches_numerical_jacobian(oracle_lib):
    """Off-axis 3D Gaussian: recover d from the image and compare with
    Sigma' = J W Sigma W^T J^T + delta I where J is the finite-difference
    Jacobian of the pinhole map at the centre (appendix, affine projection)."""
    f, a, delta = 300.0, 0.9, 0.3
    cam = axis_camera(z=3.0, f=f, W=128, H=128, cx=40.0, cy=70.0)
    mu = np.array([0.35, -0.2, 0.4])
    s = np.array([0.03, 0.012, 0.02])
    q = np.array([0.8, 0.3, -0.4, 0.2])
    sc = make_scene(mu, s, q, a, np.zeros((1, 1, 3)), [1])
    res, im = run(oracle_lib, sc, cam, dict(dilation=delta))
    mu32 = mu.astype(np.float32).astype(np.float64)
    s32 = s.astype(np.float32).astype(np.float64)
    q32 = q.astype(np.float32).astype(np.float64)
    R = matrix_from_quat_wxyz(q32 / np.linalg.norm(q32))
    Sig = R @ np.diag(s32 ** 2) @ R.T
    pc = mu32 + np.array([0, 0, 3.0])

    def proj(p):
        return np.array([f * p[0] / p[2] + 40.0, f * p[1] / p[2] + 70.0])
    h = 1e-6
    J = np.stack([(proj(pc + h * e) - proj(pc - h * e)) / (2 * h) for e in np.eye(3)], 1)
    Sp = J @ Sig @ J.T + float(np.float32(delta)) * np.eye(2)
    Si = np.linalg.inv(Sp)
    m2 = proj(pc)
    alpha = im["alpha"][0, 0]
    yy, xx = np.nonzero((alpha > 0.05) & (alpha < 0.85) & (im["tie"][0] == 0))
    assert len(yy) > 20
    dp = np.stack([xx + 0.5 - m2[0], yy + 0.5 - m2[1]], 1)
    d_exp = np.einsum("ni,ij,nj->n", dp, Si, dp)
    d_got = -2.0 * np.log(alpha[yy, xx] / np.float32(a))
    np.testing.assert_allclose(d_got, d_exp, rtol=2e-7, atol=1e-9)


# ---------------------------------------------------------------------------
# Eq. uv: the paper's homogeneous-plane form of the ray-splat intersection,
# u = (h_u^2 h_v^4 - h_u^4 h_v^2) / (h_u^1 h_v^2 - h_u^2 h_v^1), etc., with
# h_u = (WH)^T h_x, h_v = (WH)^T h_y, must agree with the oracle's plain
# ray-plane intersection.
# ---------------------------------------------------------------------------
def test_ray_splat_matches_paper_eq_uv(oracle_lib):
    rng = np.random.default_rng(7)
    fx, fy, cx, cy = 500.0, 450.0, 300.0, 200.0
    V = np.eye(4)
    V[:3, :3] = Rotation.from_euler("xyz", [0.1, -0.2, 0.05]).as_matrix()
    V[:3, 3] = [0.1, -0.3, 5.0]
    cam = dict(viewmat=V.astype(np.float32), fx=fx, fy=fy, cx=cx, cy=cy, width=600,
               height=400, znear=0.2)
    V64 = cam["viewmat"].astype(np.float64)
    for trial in range(5):
        mu = rng.uniform(-0.5, 0.5, 3)
        s = np.array([rng.uniform(0.05, 0.3), rng.uniform(0.05, 0.3), 0.0])
        q = rng.normal(size=4)
        prm = np.concatenate([mu, s, q])
        pxy = np.stack([rng.uniform(0, 600, 50), rng.uniform(0, 400, 50)], 1)
        got = oracle_lib.surfel_uv(prm, cam, pxy)
        R = matrix_from_quat_wxyz(q / np.linalg.norm(q))
        H = np.zeros((4, 4))
        H[:3, 0] = s[0] * R[:, 0]
        H[:3, 1] = s[1] * R[:, 1]
        H[:3, 3] = mu
        H[3, 3] = 1.0
        Kp = np.array([[fx, 0, cx, 0], [0, fy, cy, 0], [0, 0, 1, 0], [0, 0, 1, 0]])
        WH = Kp @ V64 @ H
        for i, (x, y) in enumerate(pxy):
            hu = WH.T @ np.array([-1.0, 0.0, 0.0, x])
            hv = WH.T @ np.array([0.0, -1.0, 0.0, y])
            den = hu[0] * hv[1] - hu[1] * hv[0]
            u = (hu[1] * hv[3] - hu[3] * hv[1]) / den
            v = (hu[3] * hv[0] - hu[0] * hv[3]) / den
            depth = (WH @ np.array([u, v, 0.0, 1.0]))[3]
            np.testing.assert_allclose(got[i], [u, v, depth], rtol=1e-9, atol=1e-9)


# ---------------------------------------------------------------------------
# P2: a fronto-parallel surfel is exactly a flat 3D Gaussian (s_z = 0,
# delta = 0): the affine map is exact on a plane parallel to the image, the
# premise of the "render 2D as flat 3D" ablation (Sec. 3.1 and Table 4).
# ---------------------------------------------------------------------------
def test_fronto_parallel_surfel_equals_flat_3d(oracle_lib):
    rng = np.random.default_rng(11)
    n = 40
    cam = axis_camera(z=4.0, f=100.0, W=96, H=80)
    mu = np.stack([rng.uniform(-1.2, 1.2, n), rng.uniform(-1.0, 1.0, n), rng.uniform(-1, 1, n)], 1)
    s = np.stack([rng.uniform(0.05, 0.2, n), rng.uniform(0.05, 0.2, n), np.zeros(n)], 1)
    th = rng.uniform(0, 2 * np.pi, n)
    q = np.stack([np.cos(th / 2), np.zeros(n), np.zeros(n), np.sin(th / 2)], 1)
    sh = rng.normal(0, 0.3, size=(n, 16, 3))
    op = rng.uniform(0.2, 0.95, n)
    s2 = make_scene(mu, s, q, op, sh, np.zeros(n))
    s3 = make_scene(mu, s, q, op, sh, np.ones(n))
    _, a = run(oracle_lib, s2, cam, dict(dilation=0.0))
    _, b = run(oracle_lib, s3, cam, dict(dilation=0.0))
    ok = (a["tie"][0] == 0) & (b["tie"][0] == 0)
    assert a["alpha"].max() > 0.5
    for k in ("rgb", "alpha", "depth", "normal"):
        np.testing.assert_allclose(a[k][0][:, ok], b[k][0][:, ok], rtol=1e-9, atol=1e-11)
    np.testing.assert_array_equal(a["n_contrib"][0][ok], b["n_contrib"][0][ok])


# ---------------------------------------------------------------------------
# P3: edge-on surfel.  With the camera centre in the surfel plane every ray
# misses the disc: the image is exactly zero with no NaN.  Near edge-on the
# integrated contribution shrinks like cos(theta) (foreshortening).
# ---------------------------------------------------------------------------
def test_edge_on_surfel_vanishes(oracle_lib):
    cam = axis_camera(z=4.0, f=64.0)
    c45 = math.cos(math.pi / 4)
    sc = make_scene([0, 0, 0], [0.3, 0.3, 0], [c45, 0, c45, 0], 0.9, np.zeros((1, 1, 3)), [0])
    res, im = run(oracle_lib, sc, cam)
    for k in ("rgb", "alpha", "depth", "normal"):
        assert np.all(np.isfinite(im[k]))
        assert np.all(im[k] == 0.0)
    assert np.all(im["T"] == 1.0)


def test_tilted_surfel_integral_follows_cosine(oracle_lib):
    f, z, a = 400.0, 10.0, 0.5
    cam = axis_camera(z=z, f=f, W=96, H=96)
    sums = []
    thetas = np.deg2rad([0.0, 60.0, 75.0])
    for th in thetas:
        q = [math.cos(th / 2), math.sin(th / 2), 0, 0]
        sc = make_scene([0, 0, 0], [0.08, 0.08, 0], q, a, np.zeros((1, 1, 3)), [0])
        _, im = run(oracle_lib, sc, cam)
        sums.append(im["alpha"].sum())
    sx = 0.08 * f / z
    # integral of a e^{-d/2} over d <= 2 ln(255 a): 2 pi sx sy a (1 - 1/(255 a))
    base = 2 * math.pi * sx * sx * np.float32(a) * (1 - 1 / (255 * np.float32(a)))
    for th, sm in zip(thetas, sums):
        np.testing.assert_allclose(sm, base * math.cos(th), rtol=0.02)


# ---------------------------------------------------------------------------
# P4: partition of unity (Eq. 2): with every colour 1 and a black background
# the colour equals alpha = 1 - T.
# ---------------------------------------------------------------------------
def test_white_scene_colour_equals_alpha(oracle_lib):
    sc = sg.scene_random(300, seed=5, sh_degree=0)
    Y00 = oracle_lib.sh_basis(0, np.array([[0.0, 0.0, 1.0]]))[0, 0]
    sc["sh"][:] = np.float32(0.5 / Y00)
    cam = sg.look_at_camera((0, 0, -4.0), width=96, height=72, fx=90.0)
    res, im = run(oracle_lib, sc, cam)
    assert im["alpha"].max() > 0.9
    Y32 = 0.5 + np.float64(np.float32(0.5 / Y00)) * Y00
    for ch in range(3):
        np.testing.assert_allclose(im["rgb"][0, ch], Y32 * im["alpha"][0, 0], atol=1e-13)
    np.testing.assert_allclose(im["alpha"][0, 0] + im["T"][0], 1.0, atol=1e-15)


# ---------------------------------------------------------------------------
# P13 and the stopping rule: a stack of identical fronto-parallel surfels
# centred on one pixel.  Each contributes exactly alpha; blending stops
# before the pair that would take T below 1e-4.
# ---------------------------------------------------------------------------
def test_stack_closed_form_counts(oracle_lib):
    f = 64.0
    cam = axis_camera(z=0.0, f=f, W=64, H=64)
    zs = 1.0 + 0.1 * np.arange(20)
    mu = np.stack([0.5 * zs / f, 0.5 * zs / f, zs], 1)  # projects to pixel centre (32.5, 32.5)
    n = len(zs)
    sc = make_scene(mu, np.tile([0.05, 0.05, 0.0], (n, 1)), np.tile([1, 0, 0, 0], (n, 1)),
                    np.full(n, 0.6), np.zeros((n, 1, 3)), np.zeros(n))
    pix = np.array([[0, 32, 32]], np.int32)
    res = oracle_lib.forward(sc, cam, pix)
    a = np.float64(np.float32(0.6))
    T = 1.0
    k = 0
    while T * (1 - a) >= 1e-4:
        T *= 1 - a
        k += 1
    assert k == 10
    assert res["n_contrib"][0] == 10
    assert res["last"][0] == 10
    np.testing.assert_allclose(res["T"][0], (1 - a) ** 10, rtol=1e-13)
    w = a * (1 - a) ** np.arange(10)
    np.testing.assert_allclose(res["out"][0, :3], 0.5 * w.sum(), rtol=1e-13)
    np.testing.assert_allclose(res["out"][0, 4], (w * sc["means"][:10, 2].astype(np.float64)).sum(), rtol=1e-12)
    np.testing.assert_allclose(res["out"][0, 7], -w.sum(), rtol=1e-13)


# ---------------------------------------------------------------------------
# Tie branches (Eq. 2 with either outcome of a decision taken within rounding
# of its threshold), closed forms on stacks of fronto-parallel surfels
# centred on one pixel, each contributing exactly its opacity there.
# ---------------------------------------------------------------------------
def _stack(alphas, f=64.0):
    n = len(alphas)
    zs = 1.0 + 0.1 * np.arange(n)
    mu = np.stack([0.5 * zs / f, 0.5 * zs / f, zs], 1)  # projects to pixel centre (32.5, 32.5)
    return make_scene(mu, np.tile([0.05, 0.05, 0.0], (n, 1)), np.tile([1, 0, 0, 0], (n, 1)),
                      alphas, np.zeros((n, 1, 3)), np.zeros(n))


def test_stop_tie_branches_closed_form(oracle_lib):
    # (1 - a)^10 = 1e-4 up to the rounding of a: the 10th pair's stop test is a tie
    a = np.float32(1.0 - 1e-4 ** 0.1)
    sc = _stack(np.full(14, a))
    cam = axis_camera(z=0.0, f=64.0, W=64, H=64)
    pix = np.array([[0, 32, 32]], np.int32)
    a64 = float(a)
    outs = {}
    for flip in (0, 1):
        r = oracle_lib.forward(sc, cam, pix, flip=flip)
        assert r["tie"][0] & 2 and r["nflags"][0] == 1
        k = int(r["n_contrib"][0])
        outs[k] = r
        w = a64 * (1 - a64) ** np.arange(k)
        np.testing.assert_allclose(r["T"][0], (1 - a64) ** k, rtol=1e-13)
        np.testing.assert_allclose(r["out"][0, :3], 0.5 * w.sum(), rtol=1e-13)
        assert r["last"][0] == k
    # the two branches stop before the 10th and before the 11th pair
    assert sorted(outs) == [9, 10]
    # the binary64 decision is the branch flip = 0 takes
    T10 = (1 - a64) ** 10
    assert oracle_lib.forward(sc, cam, pix)["n_contrib"][0] == (9 if T10 < 1e-4 else 10)


def test_activity_tie_branches_closed_form(oracle_lib):
    # a pair of contribution binary32(1/255) at the pixel sample, behind one
    # of 0.5: active in binary64 (1/255 rounds up), inactive on the flipped branch
    amin32 = np.float32(1.0 / 255.0)
    sc = _stack(np.array([0.5, amin32, 0.25], np.float32))
    cam = axis_camera(z=0.0, f=64.0, W=64, H=64)
    pix = np.array([[0, 32, 32]], np.int32)
    r0 = oracle_lib.forward(sc, cam, pix)
    r1 = oracle_lib.forward(sc, cam, pix, flip=1)
    assert r0["tie"][0] & 1 and r0["nflags"][0] == 1
    a = [0.5, float(amin32), 0.25]
    assert r0["n_contrib"][0] == 3 and r1["n_contrib"][0] == 2
    np.testing.assert_allclose(r0["T"][0], (1 - a[0]) * (1 - a[1]) * (1 - a[2]), rtol=1e-14)
    np.testing.assert_allclose(r1["T"][0], (1 - a[0]) * (1 - a[2]), rtol=1e-14)
    assert r0["last"][0] == 3 and r1["last"][0] == 3
    # gradients follow the branch: the skipped pair gets none on flip = 1
    G = np.zeros((1, 8))
    G[0, 3] = 1.0
    g0 = oracle_lib.backward(sc, cam, pix, G)
    g1 = oracle_lib.backward(sc, cam, pix, G, flip=1)
    assert g0["opacities"][1] != 0.0 and g1["opacities"][1] == 0.0
    # d alpha / d a_0 = prod of (1 - a_j) over the other blended pairs
    np.testing.assert_allclose(g1["opacities"][0], (1 - a[2]), rtol=1e-12)
    np.testing.assert_allclose(g0["opacities"][0], (1 - a[1]) * (1 - a[2]), rtol=1e-12)


def test_clamp_tie_spread_closed_form(oracle_lib):
    # one surfel of opacity binary32(0.99) centred on the pixel sample:
    # raw = 0.99000001 > 0.99 is clamped (zero derivative), within the clamp
    # margin; the unclamped branch has d alpha~ / d alpha = e^0 = 1
    sc = _stack(np.array([0.99], np.float32))
    cam = axis_camera(z=0.0, f=64.0, W=64, H=64)
    pix = np.array([[0, 32, 32]], np.int32)
    r = oracle_lib.forward(sc, cam, pix)
    assert r["tie"][0] & 4 and r["nflags"][0] == 0
    G = np.zeros((1, 8))
    G[0, 3] = 1.0  # L = alpha = alpha~, so dL/d alpha~ = 1
    g = oracle_lib.backward(sc, cam, pix, G)
    assert g["opacities"][0] == 0.0
    np.testing.assert_allclose(g["opacities_tie"][0], 1.0, rtol=1e-15)
    # away from the clamp there is no spread
    sc2 = _stack(np.array([0.9], np.float32))
    g2 = oracle_lib.backward(sc2, cam, pix, G)
    assert g2["opacities_tie"][0] == 0.0 and g2["opacities"][0] == pytest.approx(1.0)


# ---------------------------------------------------------------------------
# P5 / P6 / P12: order invariance, brute force vs binned, conservative rects,
# sorted keys vs numpy's stable sort.
# ---------------------------------------------------------------------------
def test_permutation_invariance(oracle_lib):
    sc = sg.scene_random(400, seed=9)
    cam = sg.look_at_camera((0.3, -0.2, -4.0), width=80, height=64, fx=70.0)
    res, a = run(oracle_lib, sc, cam)
    perm = np.random.default_rng(1).permutation(400)
    sp = sg.subset(sc, perm)
    res2, b = run(oracle_lib, sp, cam)
    for k in ("rgb", "alpha", "depth", "normal", "T", "n_contrib", "last"):
        np.testing.assert_array_equal(a[k], b[k])


def test_brute_force_equals_binned(oracle_lib):
    sc = sg.scene_random(64, seed=21, log_mu=-2.5)
    cam = sg.look_at_camera((0.0, 0.0, -3.5), width=64, height=64, fx=60.0)
    pix = oracle_lib.full_pixels(cam)
    a = oracle_lib.forward(sc, cam, pix, brute=False)
    b = oracle_lib.forward(sc, cam, pix, brute=True)
    assert a["out"][:, 3].max() > 0.5
    for k in ("out", "T", "n_contrib", "tie"):
        np.testing.assert_array_equal(a[k], b[k])


def test_rects_are_conservative(oracle_lib):
    sc = sg.scene_random(64, seed=23, log_mu=-2.3, log_sigma=0.8)
    cam = sg.look_at_camera((0.2, 0.1, -3.0), width=72, height=56, fx=60.0)
    st = oracle_lib.structural(sc, cam)
    pix = oracle_lib.full_pixels(cam)
    checked = 0
    for g in range(64):
        one = sg.subset(sc, [g])
        r = oracle_lib.forward(one, cam, pix, brute=True)
        act = r["out"][:, 3] > 0
        if not act.any():
            continue
        checked += 1
        assert st["valid"][g]
        x0, y0, x1, y1 = st["rect"][g]
        ys, xs = pix[act, 1], pix[act, 2]
        assert xs.min() >= x0 and xs.max() <= x1 and ys.min() >= y0 and ys.max() <= y1
    assert checked > 30


def test_sorted_pairs_match_numpy(oracle_lib):
    sc = sg.scene_random(500, seed=4)
    cams = [sg.look_at_camera((0, 0, -4.0), width=100, height=70, fx=80.0),
            sg.look_at_camera((1.0, 0.5, -3.5), width=100, height=70, fx=80.0)]
    st = oracle_lib.structural(sc, cams)
    keys, vals, ranges = oracle_lib.sorted_pairs(st, cams)
    # independent construction: emit pairs, numpy stable argsort
    tpv = [((c["width"] + 15) // 16, (c["height"] + 15) // 16) for c in cams]
    K, Vv = [], []
    base = 0
    n = 500
    for v, (tx, ty) in enumerate(tpv):
        for g in range(n):
            i = v * n + g
            if not st["valid"][i]:
                continue
            x0, y0, x1, y1 = st["rect"][i]
            for yy in range(y0 >> 4, (y1 >> 4) + 1):
                for xx in range(x0 >> 4, (x1 >> 4) + 1):
                    K.append(((base + yy * tx + xx) << 32) | int(st["zbits"][i]))
                    Vv.append(i)
        base += tx * ty
    K = np.array(K, np.uint64)
    Vv = np.array(Vv, np.uint32)
    o = np.argsort(K, kind="stable")
    np.testing.assert_array_equal(keys, K[o])
    np.testing.assert_array_equal(vals, Vv[o])
    tiles = (K[o] >> np.uint64(32)).astype(np.int64)
    for t in range(ranges.shape[0]):
        idx = np.nonzero(tiles == t)[0]
        if len(idx) == 0:
            assert ranges[t, 0] == ranges[t, 1] == 0
        else:
            assert ranges[t, 0] == idx[0] and ranges[t, 1] == idx[-1] + 1
    # depth keys are the bits of a positive float: monotone in depth
    z = st["zbits"][st["valid"] == 1].view(np.float32)
    assert np.all(z > 0.2)


# ---------------------------------------------------------------------------
# P7: reparameterisation (appendix "Effective Rank and Type Switch",
# S* = P S P^T, R* = R P^T keeps Sigma): the 3D image is unchanged.  Also
# q -> -q and q -> 2q, q/4.
# ---------------------------------------------------------------------------
PX = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], float)
PY = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]], float)


def test_3d_reparameterisation_invariance(oracle_lib):
    sc = sg.scene_random(120, seed=31, frac2d=0.0, log_mu=-2.6)
    cam = sg.look_at_camera((0.0, 0.3, -3.5), width=80, height=64, fx=70.0)
    _, base = run(oracle_lib, sc, cam)
    for P in (PX, PY):
        s2 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
        for g in range(120):
            q = sc["rotations"][g].astype(np.float64)
            R = matrix_from_quat_wxyz(q / np.linalg.norm(q))
            s = sc["scales"][g].astype(np.float64)
            s2["scales"][g] = np.diag(P @ np.diag(s) @ P.T)
            s2["rotations"][g] = quat_wxyz_from_matrix(R @ P.T)
        p64 = dict(means=sc["means"].astype(np.float64), scales=s2["scales"].astype(np.float64),
                   rotations=np.stack([quat_wxyz_from_matrix(
                       matrix_from_quat_wxyz(sc["rotations"][g] / np.linalg.norm(sc["rotations"][g]))
                       @ P.T) for g in range(120)]),
                   opacities=sc["opacities"].astype(np.float64), sh=sc["sh"].astype(np.float64))
        res, im = run(oracle_lib, s2, cam, params64=p64)
        # the structural module sees the float32-rounded quaternion; the
        # binary64 path sees the exact one
        ok = (base["tie"][0] == 0) & (im["tie"][0] == 0)
        for k in ("rgb", "alpha", "depth"):
            np.testing.assert_allclose(im[k][0][:, ok], base[k][0][:, ok], atol=2e-6)
        np.testing.assert_allclose(im["normal"][0][:, ok], base["normal"][0][:, ok], atol=2e-6)
    for fac in (-1.0, 2.0, 0.25):  # powers of two scale a binary32 quaternion exactly
        s3 = dict(sc)
        s3["rotations"] = (sc["rotations"] * np.float32(fac)).astype(np.float32)
        _, im = run(oracle_lib, s3, cam)
        for k in ("rgb", "alpha", "depth", "normal"):
            np.testing.assert_allclose(im[k], base[k], atol=1e-12)


# ---------------------------------------------------------------------------
# P8: a surfel ignores s_z while the modulation gate is inert (Sec. 3.2),
# and flipping (t_v, n) -> (-t_v, -n) describes the same disc.
# ---------------------------------------------------------------------------
def test_surfel_invariances(oracle_lib):
    sc = sg.scene_random(150, seed=41, frac2d=1.0, log_mu=-2.4)
    cam = sg.look_at_camera((0.2, 0.0, -3.5), width=80, height=64, fx=70.0)
    _, base = run(oracle_lib, sc, cam)
    s2 = dict(sc)
    s2["scales"] = sc["scales"].copy()
    s2["scales"][:, 2] = 0.3
    _, im = run(oracle_lib, s2, cam)
    for k in ("rgb", "alpha", "depth", "normal"):
        np.testing.assert_array_equal(im[k], base[k])
    s3 = dict(sc)
    q = sc["rotations"].astype(np.float64)
    qf = np.stack([-q[:, 1], q[:, 0], q[:, 3], -q[:, 2]], 1)  # q * (0,1,0,0): pi about local x
    s3["rotations"] = qf.astype(np.float32)
    _, im = run(oracle_lib, s3, cam)
    ok = (base["tie"][0] == 0) & (im["tie"][0] == 0)
    for k in ("rgb", "alpha", "depth", "normal"):
        np.testing.assert_allclose(im[k][0][:, ok], base[k][0][:, ok], atol=1e-9)


# ---------------------------------------------------------------------------
# P9: the SH basis (colour decoded from f, Sec. 3.1) against scipy's complex
# harmonics, orthonormality by quadrature, and the textbook degree-0/1 forms.
# ---------------------------------------------------------------------------
def _scipy_real_sh(degree, dirs):
    from scipy.special import sph_harm_y
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    th = np.arccos(np.clip(z, -1, 1))
    ph = np.arctan2(y, x)
    out = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), th, ph)
            if m < 0:
                out.append(math.sqrt(2) * Y.imag)
            elif m == 0:
                out.append(Y.real)
            else:
                out.append(math.sqrt(2) * Y.real)
    return np.stack(out, 1)


def test_sh_basis_matches_scipy(oracle_lib):
    d = np.random.default_rng(3).normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    np.testing.assert_allclose(oracle_lib.sh_basis(3, d), _scipy_real_sh(3, d), atol=1e-12)


def test_sh_basis_orthonormal_and_textbook(oracle_lib):
    zg, wz = np.polynomial.legendre.leggauss(12)
    ph = np.arange(24) * 2 * np.pi / 24
    Z, PH = np.meshgrid(zg, ph, indexing="ij")
    r = np.sqrt(1 - Z ** 2)
    d = np.stack([r * np.cos(PH), r * np.sin(PH), Z], -1).reshape(-1, 3)
    w = (np.repeat(wz, 24) * (2 * np.pi / 24))
    Y = oracle_lib.sh_basis(3, d)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)
    pts = np.array([[0.6, 0.0, 0.8], [0.0, 0.6, 0.8], [0.0, 0.0, 1.0]])
    Y = oracle_lib.sh_basis(1, pts)
    c0 = 0.5 / math.sqrt(math.pi)
    c1 = math.sqrt(3.0 / (4 * math.pi))
    np.testing.assert_allclose(Y[:, 0], c0, atol=1e-15)
    np.testing.assert_allclose(Y[:, 1], -c1 * pts[:, 1], atol=1e-15)  # Y_1^-1 = -c1 y
    np.testing.assert_allclose(Y[:, 2], c1 * pts[:, 2], atol=1e-15)   # Y_1^0 = c1 z
    np.testing.assert_allclose(Y[:, 3], -c1 * pts[:, 0], atol=1e-15)  # Y_1^1 = -c1 x


# ---------------------------------------------------------------------------
# P11: scale modulation (Eq. 6-7).  At the gate centre s_z = theta_z the gate
# is 1/2, so alpha* = alpha e^{-lambda theta_z / 2}, and
# d alpha*/d s_z = -lambda alpha* (theta_z / (4 T_z) + 1/2).
# ---------------------------------------------------------------------------
def test_modulation_gate_centre(oracle_lib):
    cam = axis_camera(z=4.0, f=64.0)
    sz = np.float32(1.05)
    th = float(sz)
    lam, Tz, a = 0.7, 0.001, 0.9
    opts = dict(lambda_z=lam, theta_z=th, temp_z=Tz)
    sc = make_scene([0.01, -0.02, 0], [0.2, 0.15, sz], [1, 0, 0, 0], a, np.zeros((1, 1, 3)), [0])
    res, im = run(oracle_lib, sc, cam, opts)
    a32 = float(np.float32(a))
    a_star = a32 * math.exp(-lam * th / 2)
    ref = dict(sc)
    ref["scales"] = sc["scales"].copy()
    ref["scales"][0, 2] = 0.0
    p64 = dict(means=ref["means"].astype(np.float64), scales=ref["scales"].astype(np.float64),
               rotations=ref["rotations"].astype(np.float64), opacities=np.array([a_star]),
               sh=ref["sh"].astype(np.float64))
    res2, im2 = run(oracle_lib, ref, cam, opts, params64=p64)
    ok = (im["tie"][0] == 0) & (im2["tie"][0] == 0)
    assert im["alpha"].max() > 0.3
    np.testing.assert_allclose(im["alpha"][0, 0][ok], im2["alpha"][0, 0][ok], rtol=1e-12, atol=1e-15)
    G = {k: np.zeros((1, c, 64, 64), np.float32) for k, c in
         (("rgb", 3), ("alpha", 1), ("depth", 1), ("normal", 3))}
    G["alpha"][:] = 1.0
    gr = oracle_lib.backward(sc, cam, oracle_lib.full_pixels(cam), pack_G(G), opts)
    ratio = gr["scales"][0, 2] / gr["opacities"][0]
    np.testing.assert_allclose(ratio, -lam * a32 * (th / (4 * Tz) + 0.5), rtol=1e-9)


# ---------------------------------------------------------------------------
# P10: the analytic (dual-number) gradient against binary64 central finite
# differences on the 64-Gaussian, 32x32 finite-difference workload, and on
# the modulation gate region.
# ---------------------------------------------------------------------------
def _loss(oracle_lib, sc, cam, pix, Gp, p64, opts=None):
    r = oracle_lib.forward(sc, cam, pix, opts, params64=p64, threads=1)
    return float((r["out"] * Gp).sum()), r


def _fd_check(oracle_lib, sc, cam, opts=None, seed=0, n_sh=60, rtol=1e-6):
    pix = oracle_lib.full_pixels(cam)
    G = sg.upstream_grads(1, cam["height"], cam["width"], seed)
    Gp = pack_G(G)
    an = oracle_lib.backward(sc, cam, pix, Gp, opts, threads=1)
    base = {k: sc[k].astype(np.float64) for k in ("means", "scales", "rotations", "opacities", "sh")}
    _, r0 = _loss(oracle_lib, sc, cam, pix, Gp, base, opts)
    checked = skipped = live = 0
    rng = np.random.default_rng(seed)
    coords = []
    n = sc["means"].shape[0]
    for g in range(n):
        for k, w in (("means", 3), ("scales", 3), ("rotations", 4), ("opacities", 1)):
            for j in range(w):
                if k == "scales" and j == 2 and sc["types"][g] == 0 and opts is None:
                    continue
                coords.append((k, g, j))
    shc = [("sh", int(g), int(j)) for g, j in zip(rng.integers(0, n, n_sh), rng.integers(0, sc["sh"].shape[1] * 3, n_sh))]
    same = lambda r: (np.array_equal(r["n_contrib"], r0["n_contrib"]) and
                      np.array_equal(r["tie"], r0["tie"]))
    loose = 0
    for (k, g, j) in coords + shc:
        fds = central_fd(lambda p: _loss(oracle_lib, sc, cam, pix, Gp, p, opts), base, k, g, j,
                         same)
        if fds is None:
            skipped += 1
            continue
        fd, fd2 = fds
        ga = an[k].reshape(n, -1)[g, j]
        gabs = an[k + "_abs"].reshape(n, -1)[g, j]
        # the two step sizes agree to the stencil's own error; that spread is
        # the only allowance beyond the relative bound
        spread = abs(fd - fd2)
        assert abs(fd - ga) <= rtol * (abs(ga) + gabs) + 2 * spread + 1e-9, \
            (k, g, j, fd, fd2, ga, gabs)
        loose += 2 * spread > rtol * (abs(ga) + gabs)
        checked += 1
        live += abs(fd) > 1e-3
    assert loose <= 0.1 * checked, (loose, checked)
    return checked, skipped, live


def test_gradients_vs_finite_differences(oracle_lib):
    sc, cam = sg.fd_subset()
    # the window sees the knot: most pixels covered, most primitives blended
    r = oracle_lib.forward(sc, cam, oracle_lib.full_pixels(cam))
    assert r["out"][:, 3].mean() > 0.3 and r["n_contrib"].sum() > 5000
    checked, skipped, live = _fd_check(oracle_lib, sc, cam, seed=3)
    assert checked > 600, (checked, skipped)
    assert skipped < 0.1 * (checked + skipped)
    assert live > 0.5 * checked, (live, checked)


def test_gradients_in_modulation_gate(oracle_lib):
    rng = np.random.default_rng(5)
    n = 6
    th, Tz = 1.05, 0.001
    mu = np.stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.3, 0.3, n), rng.uniform(-0.2, 0.2, n)], 1)
    sz = th + rng.uniform(-5 * Tz, 5 * Tz, n)
    s = np.stack([rng.uniform(0.05, 0.12, n), rng.uniform(0.05, 0.12, n), sz], 1)
    q = rng.normal(size=(n, 4))
    q[:, 0] += 3.0
    sc = make_scene(mu, s, q, rng.uniform(0.3, 0.9, n), rng.normal(0, 0.3, (n, 4, 3)), np.zeros(n))
    cam = axis_camera(z=3.0, f=60.0, W=48, H=40)
    checked, skipped, live = _fd_check(oracle_lib, sc, cam, opts=dict(theta_z=th, temp_z=Tz),
                                       seed=8, n_sh=10)
    assert checked > 40 and live > 20, (checked, live)
