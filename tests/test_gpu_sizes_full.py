"""Parity at the full sizes of the forward and large-batch workloads, in the
launch configuration the benchmark uses, on outputs the oracle computes one
by one: sampled pixels, sampled tiles and the structural arrays of sampled
views.

* 500k-Gaussian noisy sphere (70% surfels, SH3), one 1920x1080 camera,
  forward: structural bit-exact over the whole frame, images at sampled
  pixels.
* 6M-Gaussian multi-shell (60% surfels, SH3), 16 cameras at 3840x2160 in
  one launch, forward + backward: per-view structural arrays for three views,
  the sorted list of sampled tiles, images at sampled pixels and gradients of
  a loss on those pixels.  The oracle runs one view at a time; gradients of
  a sum over views are the sum of per-view gradients.
"""
import numpy as np
import pytest

import scenegen as sg
from gpu_common import (IMG_KEYS, PARAM_KEYS, check_pixels, compare_grads, compare_images,
                        compare_structural, gpu_at, gpu_render, say)

pytestmark = pytest.mark.gpu


def test_sphere_500k_1080p_forward_sampled():
    import oracle
    scene = sg.scene_sphere()
    cam = sg.camera_sphere()
    rng = np.random.default_rng(11)
    n = 3000
    pix = np.stack([np.zeros(n, np.int64), rng.integers(0, 1080, n), rng.integers(0, 1920, n)], 1)
    rows = np.array([[0, y, x] for y in (300, 540) for x in range(0, 1920, 3)])
    pix = np.ascontiguousarray(np.concatenate([pix, rows]), np.int32)
    say("[sphere500k] oracle forward at sampled pixels")
    res = oracle.forward(scene, cam, pix)
    say("[sphere500k] gpu render")
    imgs, state, _ = gpu_render(scene, cam)
    _, D = compare_structural(state, scene, cam)
    _, _, rep = compare_images(imgs, state, res, pix, scene, cam)
    say(f"[sphere500k] D={D} forward ok {rep}")
    state.free()


@pytest.mark.timeout(900)
def test_multishell_6m_16x4k_fwd_bwd_sampled():
    import torch
    import oracle
    from paper_2512_02932_amd.rasterizer import get_rasterizer, to_device

    say("[shell6m] generating scene and cameras")
    scene = sg.scene_multishell()
    cams = sg.fibonacci_cameras()
    V, H, W = len(cams), cams[0]["height"], cams[0]["width"]
    N = scene["means"].shape[0]
    views = (0, 7, 13)
    rng = np.random.default_rng(12)

    # sampled pixels per checked view, oracle forward one view at a time
    samples = {}
    for v in views:
        pix = np.stack([np.zeros(700, np.int64), rng.integers(0, H, 700),
                        rng.integers(0, W, 700)], 1)
        row = np.array([[0, H // 2, x] for x in range(0, W, 8)])
        pix = np.ascontiguousarray(np.concatenate([pix, row]), np.int32)
        say(f"[shell6m] oracle forward, view {v}")
        samples[v] = (pix, oracle.forward(scene, cams[v], pix))

    # cotangents: N(0,1) at 300 distinct sampled pixels (ties included), zero
    # elsewhere
    rast = get_rasterizer(0)
    sc = to_device(scene)
    G = {k: torch.zeros((V, c, H, W), device="cuda") for k, c in
         (("rgb", 3), ("alpha", 1), ("depth", 1), ("normal", 3))}
    gsel = {}
    for v in views:
        pix, res = samples[v]
        _, first = np.unique(pix[:, 1].astype(np.int64) * W + pix[:, 2], return_index=True)
        gsel[v] = np.sort(first)[:300]
        sel = pix[gsel[v]]
        Gs = sg.upstream_grads(1, 1, len(sel), seed=20 + v)
        ys = torch.from_numpy(sel[:, 1].astype(np.int64)).cuda()
        xs = torch.from_numpy(sel[:, 2].astype(np.int64)).cuda()
        for k in IMG_KEYS:
            G[k][v][:, ys, xs] = torch.from_numpy(Gs[k][0][:, 0, :]).cuda()
    say("[shell6m] gpu render 16 views + backward")
    imgs, state = rast.render(sc, cams, want_state=True)
    grads = {k: torch.zeros_like(sc[k]) for k in PARAM_KEYS}
    rast.backward(state, G, grads)
    torch.cuda.synchronize()
    sz = state.sizes()
    say(f"[shell6m] D={sz['D']}")

    # structural arrays of the checked views, and sampled tile lists
    tiles = state.debug("tiles")
    zb = state.debug("zbits")
    rect = state.debug("rect")
    ranges = state.debug("ranges")
    vals = state.debug("vals")
    tpv = ((W + 15) // 16) * ((H + 15) // 16)
    tiles_x = (W + 15) // 16
    for v in views:
        st = oracle.structural(scene, cams[v], 0.3)
        sl = slice(v * N, (v + 1) * N)
        np.testing.assert_array_equal(tiles[sl], st["tiles"])
        ok = st["valid"] == 1
        np.testing.assert_array_equal(zb[sl][ok], st["zbits"][ok])
        np.testing.assert_array_equal(rect[sl][ok], st["rect"][ok])
        r = st["rect"]
        for t in rng.integers(0, tpv, 12):
            ty, tx = divmod(int(t), tiles_x)
            cover = ok & (r[:, 0] >> 4 <= tx) & (r[:, 2] >> 4 >= tx) & \
                (r[:, 1] >> 4 <= ty) & (r[:, 3] >> 4 >= ty)
            g = np.nonzero(cover)[0]
            order = np.lexsort((g, st["zbits"][g]))
            a, b = ranges[v * tpv + int(t)]
            np.testing.assert_array_equal(vals[a:b], (v * N + g[order]).astype(np.uint32))
    say("[shell6m] structural ok")

    # images at sampled pixels, with per-pixel counts and transmittance
    per_px = {k: state.debug(k) for k in ("n_contrib", "last", "T_final")}
    flips = {}
    for v in views:
        pix, res = samples[v]
        one = {k: imgs[k][v:v + 1].cpu().numpy() for k in IMG_KEYS}
        flat = v * H * W + pix[:, 1].astype(np.int64) * W + pix[:, 2]
        gpu = dict(out=gpu_at(one, pix), n_contrib=per_px["n_contrib"][flat].astype(np.int64),
                   last=per_px["last"][flat].astype(np.int64),
                   T=per_px["T_final"][flat].astype(np.float64))
        _, flips[v], rep = check_pixels(scene, cams[v], pix, res, gpu)
        say(f"[shell6m] view {v} images ok {rep}")

    # gradients: sum of per-view oracle backward passes
    ref = None
    for v in views:
        sel = samples[v][0][gsel[v]]
        Gp = np.zeros((len(sel), 8))
        for k, cols in (("rgb", (0, 1, 2)), ("alpha", (3,)), ("depth", (4,)),
                        ("normal", (5, 6, 7))):
            g = G[k][v].cpu().numpy()
            for j, col in enumerate(cols):
                Gp[:, col] = g[j, sel[:, 1], sel[:, 2]]
        say(f"[shell6m] oracle backward, view {v}")
        r = oracle.backward(scene, cams[v], sel, Gp, flip=flips[v][gsel[v]])
        ref = r if ref is None else {k: ref[k] + r[k] for k in ref}
    rep = compare_grads({k: v.cpu().numpy() for k, v in grads.items()}, ref)
    say(f"[shell6m] backward ok {rep}")
    state.free()
