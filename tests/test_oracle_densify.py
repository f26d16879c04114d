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


def _ndc_to_pix(v, size):
    """Pixel coordinate of NDC coordinate v (3DGS's convention: NDC -1 and 1
    are the outer edges of pixels 0 and size - 1)."""
    return ((v + 1.0) * size - 1.0) * 0.5


def test_densify_stats_are_ndc_central_differences(O):
    """The statistic per splat is the sum over the views that do not cull it
    of the Euclidean norm of dL/d(translation of its footprint in NDC
    units).  Pinned by central differences of the oracle forward under a
    translation of h NDC units, converted to pixels through the NDC
    definition, per splat: the splats' footprints are disjoint and the
    cotangent of each pass is restricted to one splat's rectangle.  One
    view culls one of the splats (its footprint leaves the image)."""
    pos = [(-0.7, -0.35, 0.0), (0.0, -0.35, 0.1), (0.7, -0.35, -0.1), (-0.35, 0.35, 0.05),
           (0.4, 0.37, 0.0)]
    q = [(0.9, 0.2, -0.3, 0.1), (0.8, 0.5, 0.2, -0.1), (1.0, 0.0, 0.0, 0.0),
         (0.7, -0.3, 0.4, 0.2), (0.6, 0.1, 0.1, 0.7)]
    sc = make_scene(pos, [[0.09, 0.06, 0.05], [0.08, 0.07, 0.0], [0.07, 0.05, 0.06],
                          [0.08, 0.06, 0.0], [0.06, 0.09, 0.04]], q,
                    [0.8, 0.7, 0.9, 0.75, 0.85], np.full((5, 1, 3), 0.4), [1, 0, 1, 0, 1])
    cams = [sg.look_at_camera((0.05, 0.02, -3.0), width=64, height=48, fx=55.0),
            sg.look_at_camera((1.0, 0.1, -2.8), target=(1.0, 0.1, 0.0), width=56, height=44,
                              fx=60.0)]
    n = sc["means"].shape[0]
    pix = np.concatenate([O.full_pixels(c, v) for v, c in enumerate(cams)])
    G = np.random.default_rng(5).normal(size=(len(pix), 8))
    norm, cnt = O.densify_stats(sc, cams, pix, G)

    ref = np.zeros(n)
    ref_cnt = np.zeros(n, np.int64)
    for v, c in enumerate(cams):
        st = O.structural(sc, c, 0.3)
        r = st["rect"]
        pv = O.full_pixels(c)
        Gv = G[pix[:, 0] == v]
        res = O.forward(sc, c, pv)
        a = res["out"][:, 3]
        clean = ~((np.abs(a - 1 / 255) < 2 / 255) | (a > 0.95) | (res["tie"] != 0))
        inside = [(st["valid"][g] == 1) & (pv[:, 2] >= r[g, 0]) & (pv[:, 2] <= r[g, 2]) &
                  (pv[:, 1] >= r[g, 1]) & (pv[:, 1] <= r[g, 3]) for g in range(n)]
        # disjoint footprints: no pixel lies in two rectangles
        assert (np.sum(inside, 0) <= 1).all()
        W, H = c["width"], c["height"]
        h = 1e-6
        dx = _ndc_to_pix(h, W) - _ndc_to_pix(0.0, W)
        dy = _ndc_to_pix(h, H) - _ndc_to_pix(0.0, H)
        for g in range(n):
            if st["valid"][g] != 1:
                continue
            ref_cnt[g] += 1
            Gg = np.where((inside[g] & clean)[:, None], Gv, 0.0)

            def L(off):
                return float(np.sum(O.forward(sc, c, pv, {"pix_off": off})["out"] * Gg))
            # translating the footprint by +d is sampling it at p - d
            fx = (L((-dx, 0.0)) - L((dx, 0.0))) / (2 * h)
            fy = (L((0.0, -dy)) - L((0.0, dy))) / (2 * h)
            ref[g] += np.hypot(fx, fy)
        # the statistic of this view alone, with the same restriction
        Gc = np.where(np.any([ins & clean for ins in inside], 0)[:, None], Gv, 0.0)
        nv, cv = O.densify_stats(sc, c, pv, Gc)
        np.testing.assert_array_equal(cv, st["valid"])
    # one splat culled in the second view
    assert sorted(ref_cnt.tolist()) == [1, 2, 2, 2, 2]
    np.testing.assert_array_equal(cnt, ref_cnt)
    # the full statistic uses every pixel; restrict the cotangents for it too
    Gr = np.zeros_like(G)
    for v, c in enumerate(cams):
        st = O.structural(sc, c, 0.3)
        r = st["rect"]
        pv = O.full_pixels(c)
        res = O.forward(sc, c, pv)
        a = res["out"][:, 3]
        clean = ~((np.abs(a - 1 / 255) < 2 / 255) | (a > 0.95) | (res["tie"] != 0))
        keep = np.zeros(len(pv), bool)
        for g in range(n):
            if st["valid"][g] == 1:
                keep |= ((pv[:, 2] >= r[g, 0]) & (pv[:, 2] <= r[g, 2]) & (pv[:, 1] >= r[g, 1]) &
                         (pv[:, 1] <= r[g, 3]))
        sel = pix[:, 0] == v
        Gr[sel] = np.where((keep & clean)[:, None], G[sel], 0.0)
    norm, cnt = O.densify_stats(sc, cams, pix, Gr)
    assert norm.min() > 0
    np.testing.assert_allclose(norm, ref, rtol=1e-5)
