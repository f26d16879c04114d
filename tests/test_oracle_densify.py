"""Pins of the oracle's screen-space translation gradient (the densification
statistic of 3DGS): translating every splat's footprint by delta is
evaluating at p - delta, so with every pixel sample shifted by h the
forward gives central differences.  Single splats (3D; a tilted 2D surfel,
whose depth moves with the pixel) are compared per splat; a scene of
overlapping splats is compared in sum (blending terms included).  Pixels
near the 1/255 threshold or the 0.99 clamp get a zero cotangent, since a
shifted sample may cross them."""
import numpy as np
import pytest

import scenegen as sg
from tests.helpers import axis_camera, make_scene


@pytest.fixture(scope="module")
def O():
    import oracle
    oracle.build(force=False)
    return oracle


def _loss(O, scene, cam, pix, Gp, off):
    res = O.forward(scene, cam, pix, {"pix_off": off})
    return float(np.sum(res["out"] * Gp)), res


def _masked_G(O, scene, cam, pix, seed):
    res = O.forward(scene, cam, pix)
    a = res["out"][:, 3]
    rng = np.random.default_rng(seed)
    G = rng.normal(size=(len(pix), 8))
    bad = (np.abs(a - 1 / 255) < 2 / 255) | (a > 0.95) | (res["tie"] != 0)
    G[bad] = 0.0
    return G


def _fd(O, scene, cam, pix, G, h=1e-4):
    lx = (_loss(O, scene, cam, pix, G, (h, 0.0))[0] - _loss(O, scene, cam, pix, G, (-h, 0.0))[0]) / (2 * h)
    ly = (_loss(O, scene, cam, pix, G, (0.0, h))[0] - _loss(O, scene, cam, pix, G, (0.0, -h))[0]) / (2 * h)
    return np.array([lx, ly])


@pytest.mark.parametrize("kind", ["3d", "2d_tilted"])
def test_single_splat_matches_shifted_samples(O, kind):
    cam = axis_camera(z=4.0, W=48, H=40, f=60.0)
    if kind == "3d":
        sc = make_scene([0.12, -0.05, 0.0], [0.25, 0.15, 0.2], [0.9, 0.2, -0.3, 0.1], 0.7,
                        np.full((1, 1, 3), 0.4), [1])
    else:
        sc = make_scene([0.1, 0.08, 0.3], [0.3, 0.2, 0.0], [0.8, 0.5, 0.2, -0.1], 0.8,
                        np.full((1, 1, 3), 0.4), [0])
    pix = O.full_pixels(cam)
    G = _masked_G(O, sc, cam, pix, seed=1)
    sgrad = O.screen_grad(sc, cam, pix, G)[0, 0]
    fd = -_fd(O, sc, cam, pix, G)  # shifting the samples by +h moves the splat by -h
    assert np.abs(sgrad).max() > 1e-3
    np.testing.assert_allclose(sgrad, fd, rtol=1e-5, atol=1e-8 * np.abs(fd).max())


def test_sum_over_splats_matches_global_shift(O):
    sc = sg.scene_random(40, seed=31, frac2d=0.5, log_mu=-2.3, log_sigma=0.3)
    cam = sg.look_at_camera((0.2, -0.1, -3.5), width=40, height=36, fx=45.0)
    pix = O.full_pixels(cam)
    G = _masked_G(O, sc, cam, pix, seed=2)
    sgrad = O.screen_grad(sc, cam, pix, G)[0]
    fd = -_fd(O, sc, cam, pix, G)
    tot = sgrad.sum(0)
    np.testing.assert_allclose(tot, fd, rtol=1e-5, atol=1e-8 * np.abs(sgrad).sum())
    assert (np.abs(sgrad).sum(1) > 0).sum() > 10


def test_densify_stats_units_and_counts(O):
    sc = sg.scene_random(60, seed=32, frac2d=0.5, log_mu=-2.5, log_sigma=0.3)
    cams = [sg.look_at_camera(e, width=40, height=30, fx=40.0)
            for e in [(0.0, 0.0, -3.5), (1.5, 0.3, -3.0)]]
    pix = np.concatenate([O.full_pixels(c, v) for v, c in enumerate(cams)])
    G = np.random.default_rng(3).normal(size=(len(pix), 8))
    norm, cnt = O.densify_stats(sc, cams, pix, G)
    sgrad = O.screen_grad(sc, cams, pix, G)
    st = O.structural(sc, cams, 0.3)
    valid = st["valid"].reshape(2, -1) == 1
    np.testing.assert_array_equal(cnt, valid.sum(0))
    expect = sum(np.where(valid[v], np.hypot(sgrad[v, :, 0] * 20.0, sgrad[v, :, 1] * 15.0), 0.0)
                 for v in range(2))
    np.testing.assert_allclose(norm, expect, rtol=1e-14)
    assert (cnt == 2).sum() > 10 and norm.max() > 0
