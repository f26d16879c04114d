"""GPU (HIP, gfx950) path vs the CPU oracle, through the C ABI.

Structural outputs (rects, tiles, depth keys, sorted (key, value) pairs,
tile ranges) must match bit for bit.  Every pixel is checked: where an
activity or stop decision sits within rounding of its threshold ("tie"
pixels) the oracle evaluates both outcomes and the GPU must match one of
them, with n_contrib and last bit-exact and images within 1e-4; gradients
are compared with the oracle's backward on the branch the GPU took, within
1e-3 of the oracle's per-element scale plus its binary32 rounding bound.
"""
import numpy as np
import pytest

import scenegen as sg
from tests.gpu_common import (IMG_KEYS, compare_grads, compare_images, compare_structural,
                              gpu_render, oracle_pixels, pack_G_all, say)

pytestmark = pytest.mark.gpu


def _cams_multi():
    eyes = [(0.0, 0.0, -3.0), (2.0, 0.5, -2.2), (-1.5, -1.0, -2.5)]
    return [sg.look_at_camera(e, width=96, height=80, fx=70.0) for e in eyes]


def _plane_scene():
    # every mean on the plane z = 0, seen along the z axis: all instances
    # share one depth key, so every radix pass of the depth sort has a
    # constant digit (the sort's copy-through path) and the blend order is
    # the index order
    sc = sg.scene_random(2000, seed=23, log_mu=-3.0)
    sc["means"] = sc["means"].copy()
    sc["means"][:, 2] = 0.0
    return sc


CASES = {
    # the 10k-Gaussian plain forward workload: 256x256, 16 full tiles per row
    "cube10k_256": lambda: (sg.scene_uniform_cube(), sg.camera_cube()),
    # ragged image (200x137: partial tiles on both edges), tilted surfels
    "random2k_200x137": lambda: (sg.scene_random(2000, seed=12, log_mu=-3.2),
                                 sg.look_at_camera((0.3, -0.2, -3.5), width=200, height=137,
                                                   fx=150.0)),
    # three views in one launch, sphere surface (70% surfels), SH degree 3
    "sphere20k_3views": lambda: (sg.scene_sphere(20_000, seed=14), _cams_multi()),
    # strongly anisotropic splats (scale log-sd 1.4: needles and slivers,
    # many at grazing angles) seen obliquely: exercises the quadrant culling
    # of 3D ellipses and the interval bound on surfels near their limits
    "aniso1500_173x131": lambda: (sg.scene_random(1500, seed=21, log_mu=-3.0, log_sigma=1.4),
                                  sg.look_at_camera((1.8, 1.2, -2.6), width=173, height=131,
                                                    fx=140.0)),
    # torus knot at reduced resolution (surface-like depth complexity)
    "knot60k_320x213": lambda: (sg.scene_torus_knot(60_000, seed=15),
                                sg.camera_torus_knot(width=320, height=213, f=240.0)),
    # a strip 258 tiles wide: the tile rectangles of splats past tile column
    # 255 do not fit the packed 8-bit form, so the duplicate reads theirs
    # unpacked (the per-instance fallback) beside packed ones
    "plane2k_160x120": lambda: (_plane_scene(),
                                sg.look_at_camera((0.0, 0.0, -3.0), width=160, height=120,
                                                  fx=120.0)),
    "strip3k_4128x40": lambda: (sg.scene_random(3000, seed=31, log_mu=-3.0),
                                sg.look_at_camera((0.0, 0.1, -3.5), width=4128, height=40,
                                                  fx=1500.0)),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    import oracle
    oracle.build(force=False)
    name = request.param
    scene, cams = CASES[name]()
    if isinstance(cams, dict):
        cams = [cams]
    V, H, W = len(cams), cams[0]["height"], cams[0]["width"]
    say(f"[case {name}] N={scene['means'].shape[0]} V={V} {W}x{H}")
    pix = oracle_pixels(cams)
    res = oracle.forward(scene, cams, pix)
    G = sg.upstream_grads(V, H, W, seed=101)
    say(f"[case {name}] gpu render + backward")
    imgs, state, grads = gpu_render(scene, cams, G=G)
    return dict(name=name, scene=scene, cams=cams, pix=pix, res=res, G=G, imgs=imgs,
                state=state, grads=grads)


def test_structural_bit_exact(case):
    _, D = compare_structural(case["state"], case["scene"], case["cams"])
    say(f"[{case['name']}] structural ok, D={D}")
    assert D > 0


def test_forward_matches_oracle(case):
    _, _, rep = compare_images(case["imgs"], case["state"], case["res"], case["pix"],
                               case["scene"], case["cams"])
    say(f"[{case['name']}] forward ok {rep}")
    assert case["imgs"]["alpha"].max() > 0.5


def test_backward_matches_oracle(case):
    import oracle
    _, flip, _ = compare_images(case["imgs"], case["state"], case["res"], case["pix"],
                                case["scene"], case["cams"])
    Gp = pack_G_all(case["G"], case["pix"])
    ref = oracle.backward(case["scene"], case["cams"], case["pix"], Gp, flip=flip)
    rep = compare_grads(case["grads"], ref)
    say(f"[{case['name']}] backward ok {rep}")


def test_forward_is_deterministic(case):
    imgs2, st2, _ = gpu_render(case["scene"], case["cams"])
    for k in IMG_KEYS:
        np.testing.assert_array_equal(imgs2[k], case["imgs"][k])
    np.testing.assert_array_equal(st2.debug("last"), case["state"].debug("last"))
    st2.free()


# ---------------------------------------------------------------------------
# Full-size training workload: 1M hybrid Gaussians (torus knot, 50/50), SH
# degree 3, at 1600x1064 as the workload states it and at 1920x1080 (the
# headline metric's size), in the launch configuration the benchmark times.
# Every structural output is compared in full; images and gradients on
# sampled pixels the oracle computes one by one (ties on the GPU's branch).
# ---------------------------------------------------------------------------
FULL_CAMS = {"1920x1080": lambda: sg.camera_torus_knot_1080p(),
             "1600x1064": lambda: sg.camera_torus_knot()}


@pytest.mark.parametrize("size", sorted(FULL_CAMS))
def test_full_size_1m_sampled(size):
    import oracle
    scene = sg.scene_torus_knot()
    cam = FULL_CAMS[size]()
    Hh, Ww = cam["height"], cam["width"]
    rng = np.random.default_rng(7)
    # sampled pixels: random over the image plus two full rows through the knot
    n = 3000
    pix = np.stack([np.zeros(n, np.int64), rng.integers(0, Hh, n), rng.integers(0, Ww, n)], 1)
    rows = np.array([[0, y, x] for y in (Hh // 2, (Hh * 2) // 3) for x in range(0, Ww, 3)])
    pix = np.ascontiguousarray(np.concatenate([pix, rows]), np.int32)
    say(f"[full {size}] oracle forward at sampled pixels")
    res = oracle.forward(scene, cam, pix)
    G = {k: np.zeros((1, c, Hh, Ww), np.float32)
         for k, c in (("rgb", 3), ("alpha", 1), ("depth", 1), ("normal", 3))}
    # cotangents on 1500 distinct sampled pixels (ties included), zero elsewhere
    _, first = np.unique(pix[:, 1].astype(np.int64) * Ww + pix[:, 2], return_index=True)
    gi = np.sort(first)[:1500]
    gsel = pix[gi]
    Gs = sg.upstream_grads(1, 1, len(gsel), seed=3)
    for k in IMG_KEYS:
        G[k][0][:, gsel[:, 1], gsel[:, 2]] = Gs[k][0][:, 0, :]
    say(f"[full {size}] gpu render + backward")
    imgs, state, grads = gpu_render(scene, cam, G=G)
    say(f"[full {size}] structural compare")
    _, D = compare_structural(state, scene, cam)
    say(f"[full {size}] D={D}; image compare")
    _, flip, rep = compare_images(imgs, state, res, pix, scene, cam)
    say(f"[full {size}] forward ok {rep}; oracle backward at {len(gsel)} pixels")
    ref = oracle.backward(scene, cam, gsel, pack_G_all(G, gsel), flip=flip[gi])
    rep = compare_grads(grads, ref)
    say(f"[full {size}] backward ok {rep}")
    state.free()


# ---------------------------------------------------------------------------
# Edge cases
# ---------------------------------------------------------------------------
def _empty_scene(n=0, K=16):
    return dict(means=np.zeros((n, 3), np.float32), scales=np.zeros((n, 3), np.float32),
                rotations=np.zeros((n, 4), np.float32), opacities=np.zeros(n, np.float32),
                sh=np.zeros((n, K, 3), np.float32), types=np.zeros(n, np.uint8), sh_degree=3)


def test_empty_scene_renders_background():
    cam = sg.look_at_camera((0, 0, -3.0), width=40, height=24, fx=40.0)
    imgs, st, grads = gpu_render(_empty_scene(), cam, opts=dict(bg=(0.25, 0.5, 0.75)),
                                 G=sg.upstream_grads(1, 24, 40, 1))
    assert st.sizes()["D"] == 0
    for c, b in enumerate((0.25, 0.5, 0.75)):
        np.testing.assert_array_equal(imgs["rgb"][0, c], np.float32(b))
    assert np.all(imgs["alpha"] == 0) and np.all(imgs["depth"] == 0)
    st.free()


def test_all_culled_and_tiny_images():
    sc = sg.scene_random(300, seed=3)
    behind = sg.look_at_camera((0, 0, 6.0), target=(0, 0, 12.0), width=33, height=17, fx=30.0)
    imgs, st, _ = gpu_render(sc, behind)
    assert st.sizes()["D"] == 0 and np.all(imgs["alpha"] == 0)
    st.free()
    import oracle
    for (w, h) in ((1, 1), (17, 1), (1, 31)):
        cam = sg.look_at_camera((0.1, 0.0, -3.0), width=w, height=h, fx=20.0)
        imgs, st, _ = gpu_render(sc, cam)
        pix = oracle_pixels(cam)
        res = oracle.forward(sc, cam, pix)
        compare_images(imgs, st, res, pix, sc, cam)
        compare_structural(st, sc, [cam])
        st.free()


def test_profile_flags_select_stage_events_and_work_accounting():
    """Stage events alone leave the plain forward in place (no pair counts);
    HGS_PROFILE_WORK records them and renders the same images; an unknown
    flag is EINVAL."""
    from paper_2512_02932_amd import _hgs
    from paper_2512_02932_amd.rasterizer import get_rasterizer, pair_counts
    rast = get_rasterizer(0)
    sc = sg.scene_random(300, seed=5)
    cam = sg.look_at_camera((0.1, 0.0, -3.0), width=40, height=24, fx=40.0)
    with pytest.raises(_hgs.HGSError):
        _hgs.hgs_profile_enable(rast.ctx, 4)
    try:
        _hgs.hgs_profile_read(rast.ctx, reset=True)
        _hgs.hgs_profile_enable(rast.ctx, _hgs.PROFILE_STAGES)
        imgs, st, _ = gpu_render(sc, cam)
        with pytest.raises(_hgs.HGSError):
            st.debug("wcount")
        st.free()
        prof = _hgs.hgs_profile_read(rast.ctx, reset=True)
        assert prof["raster_fwd"][1] == 1 and prof["raster_fwd"][0] > 0
        _hgs.hgs_profile_enable(rast.ctx, _hgs.PROFILE_WORK)
        imgs_w, st, _ = gpu_render(sc, cam)
        counts = pair_counts(st)
        assert counts["blend_3d"] + counts["blend_2d"] > 0
        st.free()
        assert _hgs.hgs_profile_read(rast.ctx, reset=True)["raster_fwd"][1] == 0
        for k in imgs:  # the same per-pixel arithmetic, plus counting
            np.testing.assert_allclose(imgs_w[k], imgs[k], rtol=0, atol=1e-6)
    finally:
        _hgs.hgs_profile_enable(rast.ctx, 0)


def test_nan_and_inf_parameters_are_dropped():
    sc = sg.scene_random(500, seed=8)
    cam = sg.look_at_camera((0, 0, -3.5), width=64, height=48, fx=50.0)
    bad = dict(sc)
    for k in ("means", "scales", "rotations", "opacities"):
        bad[k] = sc[k].copy()
    bad["means"][0] = np.nan
    bad["scales"][1] = np.inf
    bad["rotations"][2] = np.nan
    bad["opacities"][3] = np.nan
    bad["rotations"][4] = 0.0
    drop = np.ones(500, bool)
    drop[:5] = False
    ref_scene = sg.subset(sc, np.nonzero(drop)[0])
    a, sa, _ = gpu_render(bad, cam)
    b, sb, _ = gpu_render(ref_scene, cam)
    for k in IMG_KEYS:
        assert np.all(np.isfinite(a[k]))
        np.testing.assert_array_equal(a[k], b[k])
    assert np.all(sa.debug("tiles")[:5] == 0)
    sa.free()
    sb.free()


def test_autograd_function_matches_direct_backward():
    import torch
    from paper_2512_02932_amd.rasterizer import rasterize, to_device
    sc = sg.scene_random(800, seed=19)
    cam = sg.look_at_camera((0.2, 0.1, -3.2), width=72, height=56, fx=60.0)
    G = sg.upstream_grads(1, 56, 72, 4)
    t = to_device(sc, "cuda")
    leaves = {k: t[k].clone().requires_grad_(True) for k in ("means", "scales", "rotations",
                                                             "opacities", "sh")}
    out = rasterize(dict(leaves, types=t["types"]), cam)
    loss = sum((o * torch.from_numpy(G[k]).cuda()).sum() for o, k in zip(out, IMG_KEYS))
    loss.backward()
    _, st, direct = gpu_render(sc, cam, G=G)
    st.free()
    for k in direct:
        g = leaves[k].grad.cpu().numpy()
        np.testing.assert_allclose(g, direct[k], rtol=1e-4, atol=1e-6 * np.abs(direct[k]).max())
