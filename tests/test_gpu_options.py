"""Render options through the C ABI: the compositing thresholds of Eq. 2
(alpha_min, alpha_max, t_min) at non-default values against the oracle
(structure bit-exact, every pixel, every gradient), the output-channel mask,
and the host-side rejection of invalid options."""
import numpy as np
import pytest

import scenegen as sg
from tests.gpu_common import (IMG_KEYS, compare_grads, compare_images, compare_structural,
                              gpu_render, oracle_pixels, pack_G_all, say)

pytestmark = pytest.mark.gpu

THRESHOLDS = {
    # stricter skip, lower clamp, early stop: shorter lists, more clamped pairs
    "strict": dict(alpha_min=0.02, alpha_max=0.9, t_min=0.01),
    # looser skip (wider support rectangles) and a late stop
    "loose": dict(alpha_min=1e-3, alpha_max=0.995, t_min=1e-6),
}


@pytest.mark.parametrize("name", sorted(THRESHOLDS))
def test_thresholds_match_oracle(name):
    import oracle
    o = THRESHOLDS[name]
    scene = sg.scene_random(2500, seed=51, log_mu=-3.0)
    cam = sg.look_at_camera((0.4, -0.3, -3.2), width=150, height=110, fx=130.0)
    pix = oracle_pixels(cam)
    res = oracle.forward(scene, cam, pix, o)
    G = sg.upstream_grads(1, 110, 150, seed=151)
    say(f"[thresholds {name}] gpu render + backward, opts {o}")
    imgs, state, grads = gpu_render(scene, cam, opts=o, G=G)
    _, D = compare_structural(state, scene, cam, o)
    _, flip, rep = compare_images(imgs, state, res, pix, scene, cam, o)
    say(f"[thresholds {name}] D={D} forward ok {rep}")
    ref = oracle.backward(scene, cam, pix, pack_G_all(G, pix), o, flip=flip)
    rep = compare_grads(grads, ref)
    say(f"[thresholds {name}] backward ok {rep}")
    # the options change the result: fewer pairs blended under the strict set
    base = oracle.forward(scene, cam, pix)
    nc = state.debug("n_contrib")
    if name == "strict":
        assert nc.sum() < base["n_contrib"].sum()
        assert float(imgs["alpha"].max()) <= 1.0 - 0.01 * (1 - 1e-6) + 1e-6
    else:
        assert nc.sum() > base["n_contrib"].sum()
    state.free()


def test_out_mask_selects_channels():
    import torch
    from paper_2512_02932_amd import _hgs
    from paper_2512_02932_amd.rasterizer import get_rasterizer, to_device
    scene = sg.scene_random(800, seed=52, log_mu=-2.8)
    cam = sg.look_at_camera((0.2, 0.1, -3.0), width=70, height=45, fx=60.0)
    rast = get_rasterizer(0)
    sc = to_device(scene, "cuda")
    full, _ = rast.render(sc, cam)
    mask = _hgs.OUT_RGB | _hgs.OUT_DEPTH
    imgs = rast.alloc_images(1, 45, 70)
    for k in IMG_KEYS:
        imgs[k].fill_(-7.0)
    rast.render(sc, cam, opts=dict(out_mask=mask), images=imgs)
    torch.cuda.synchronize()
    for k in ("rgb", "depth"):
        assert torch.equal(imgs[k], full[k]), k
    for k in ("alpha", "normal"):
        assert bool((imgs[k] == -7.0).all()), k
    # a selected channel must have its pointer
    part = {k: imgs[k] for k in ("rgb", "alpha")}
    with pytest.raises(_hgs.HGSError) as e:
        rast.render(sc, cam, opts=dict(out_mask=mask), images=part)
    assert e.value.status == _hgs.HGS_EINVAL
    # out_mask = 0: the channels given are written
    part = {k: torch.zeros_like(full[k]) for k in ("alpha", "normal")}
    rast.render(sc, cam, images=part)
    torch.cuda.synchronize()
    for k in part:
        assert torch.equal(part[k], full[k]), k


@pytest.mark.parametrize("bad", [dict(alpha_min=0.0), dict(alpha_min=0.5, alpha_max=0.4),
                                 dict(alpha_max=1.0), dict(t_min=0.0), dict(t_min=1.0),
                                 dict(alpha_min=float("nan")), dict(out_mask=16),
                                 dict(temp_z=0.0), dict(bg=(0.0, float("inf"), 0.0))])
def test_invalid_options_are_rejected(bad):
    from paper_2512_02932_amd import _hgs
    from paper_2512_02932_amd.rasterizer import get_rasterizer, to_device
    scene = sg.scene_random(10, seed=53)
    cam = sg.look_at_camera((0.0, 0.0, -3.0), width=16, height=16, fx=16.0)
    rast = get_rasterizer(0)
    with pytest.raises(_hgs.HGSError) as e:
        rast.render(to_device(scene, "cuda"), cam, opts=bad)
    assert e.value.status == _hgs.HGS_EINVAL
