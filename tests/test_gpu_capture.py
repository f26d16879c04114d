"""The render only enqueues: the pair capacity (fixed or learned), the
overflow flag when the pairs exceed it, and a render + backward captured
into a HIP graph whose replays equal the eager call."""
import numpy as np
import pytest

import scenegen as sg
from tests.gpu_common import IMG_KEYS, PARAM_KEYS, say

pytestmark = pytest.mark.gpu


def _setup(seed=61, n=3000, width=120, height=90, eye=(0.3, -0.2, -3.3), fx=110.0, log_mu=-3.0):
    import torch
    from paper_2512_02932_amd.rasterizer import get_rasterizer, to_device
    scene = sg.scene_random(n, seed=seed, log_mu=log_mu)
    cam = sg.look_at_camera(eye, width=width, height=height, fx=fx)
    G = sg.upstream_grads(1, height, width, seed=seed + 100)
    Gt = {k: torch.from_numpy(v).cuda() for k, v in G.items()}
    return get_rasterizer(0), to_device(scene, "cuda"), cam, Gt


def _eager(rast, sc, cam, Gt):
    import torch
    images, st = rast.render(sc, cam, want_state=True)
    st.check()
    grads = {k: torch.zeros_like(sc[k]) for k in PARAM_KEYS}
    rast.backward(st, Gt, grads)
    torch.cuda.synchronize()
    D = st.sizes()["D"]
    st.free()
    return {k: v.clone() for k, v in images.items()}, grads, D


def test_fixed_capacity_overflow_is_flagged_then_recovers():
    import torch
    from paper_2512_02932_amd import _hgs
    rast, sc, cam, Gt = _setup()
    ref, _, D = _eager(rast, sc, cam, Gt)
    assert D > 1000
    try:
        rast.set_pair_capacity(D // 2)
        imgs, st = rast.render(sc, cam, want_state=True)
        with pytest.raises(_hgs.HGSError) as e:
            st.check()
        assert e.value.status == _hgs.HGS_ECAPACITY
        assert st.sizes()["D"] == D // 2  # the sorted list holds the pairs that fit
        st.free()
        # exactly enough room: complete and identical
        rast.set_pair_capacity(D)
        imgs, st = rast.render(sc, cam, want_state=True)
        st.check()
        torch.cuda.synchronize()
        for k in IMG_KEYS:
            assert torch.equal(imgs[k], ref[k]), k
        st.free()
    finally:
        rast.set_pair_capacity(0)


def test_learned_capacity_grows_after_an_overflow():
    """Same shape, a closer camera: many more pairs than the learned
    capacity.  The render flags the overflow; hgs_state_check enlarges the
    capacity, and the next render is complete."""
    import torch
    from paper_2512_02932_amd import _hgs
    # 60k splats: about 149k pairs seen from 8 units, 554k from 1.6
    rast, sc, cam_far, Gt = _setup(seed=62, n=60_000, eye=(0.0, 0.0, -8.0), log_mu=-2.3)
    cam_near = sg.look_at_camera((0.0, 0.0, -1.6), width=cam_far["width"],
                                 height=cam_far["height"], fx=110.0)
    ref_far, _, D_far = _eager(rast, sc, cam_far, Gt)
    # a fresh context learns the far view's capacity, then meets the near one
    from paper_2512_02932_amd.rasterizer import Rasterizer
    r2 = Rasterizer(0)
    try:
        imgs, st = r2.render(sc, cam_far, want_state=True)
        st.check()
        st.free()
        imgs, st = r2.render(sc, cam_near, want_state=True)
        with pytest.raises(_hgs.HGSError) as e:
            st.check()
        assert e.value.status == _hgs.HGS_ECAPACITY
        st.free()
        imgs, st = r2.render(sc, cam_near, want_state=True)
        st.check()
        D_near = st.sizes()["D"]
        st.free()
        # reference: a render with a fixed capacity that holds every pair
        rast.set_pair_capacity(4 * D_near)
        try:
            ref_near_imgs, _, D_ref = _eager(rast, sc, cam_near, Gt)
        finally:
            rast.set_pair_capacity(0)
        assert D_near == D_ref and D_near > 1.5 * D_far + 65536
        torch.cuda.synchronize()
        for k in IMG_KEYS:
            assert torch.equal(imgs[k], ref_near_imgs[k]), k
        say(f"[capacity] far D={D_far}, near D={D_near}: overflow flagged, then complete")
    finally:
        r2.close()


def test_captured_render_backward_replays_equal_eager():
    import torch
    rast, sc, cam, Gt = _setup(seed=63)
    ref_img, ref_g, D = _eager(rast, sc, cam, Gt)
    # a second scene for eager work between the replays
    _, sc2, cam2, Gt2 = _setup(seed=64, n=1500, width=70, height=50)

    s = torch.cuda.Stream()
    images = rast.alloc_images(1, cam["height"], cam["width"])
    grads = {k: torch.zeros_like(sc[k]) for k in PARAM_KEYS}
    with torch.cuda.stream(s):
        # warm-up on the capture stream: sizes the workspace and its capacity
        _, st = rast.render(sc, cam, images=images, want_state=True)
        rast.backward(st, Gt, grads)
        st.free()
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        _, st_c = rast.render(sc, cam, images=images, want_state=True)
        rast.backward(st_c, Gt, grads)
    try:
        for rep in range(3):
            for k in IMG_KEYS:
                images[k].fill_(float("nan"))
            for k in PARAM_KEYS:
                grads[k].fill_(float("nan"))
            # eager work of another shape in between
            other, _, _ = _eager(rast, sc2, cam2, Gt2)
            assert float(other["alpha"].max()) > 0.0
            g.replay()
            torch.cuda.synchronize()
            for k in IMG_KEYS:
                assert torch.equal(images[k], ref_img[k]), (rep, k)
            for k in PARAM_KEYS:
                a = grads[k].double().cpu().numpy()
                r = ref_g[k].double().cpu().numpy()
                # the backward adds per-pair terms with atomics in any order
                assert np.all(np.abs(a - r) <= 1e-4 * np.abs(r) + 1e-5 * np.abs(r).max()), (rep, k)
        say(f"[capture] D={D}: 3 replays equal the eager render and backward")
    finally:
        del g
        st_c.free()


def test_captured_training_step_replays_equal_eager():
    """Render, colour loss (the entry point that allocates nothing), Haar
    cotangents, the three-set FDO backward, densification statistics and
    Adam, captured as one graph: each replay from the same starting
    parameters equals the eager step."""
    import torch
    from paper_2512_02932_amd.rasterizer import (adam_step, color_loss, fdo_cotangents,
                                                 get_rasterizer, to_device)
    rast = get_rasterizer(0)
    scene = sg.scene_random(2500, seed=65, log_mu=-3.0)
    cam = sg.look_at_camera((0.2, -0.3, -3.2), width=112, height=84, fx=100.0)
    H, W = cam["height"], cam["width"]
    N, deg = scene["means"].shape[0], scene["sh_degree"]
    sc = to_device(scene, "cuda")
    with np.errstate(divide="ignore"):
        raw0 = {"means": sc["means"].clone(), "scales": torch.log(sc["scales"]),
                "rotations": sc["rotations"].clone(),
                "opacities": torch.logit(sc["opacities"].double()).float(),
                "sh": sc["sh"].clone()}
    act0 = {k: sc[k].clone() for k in raw0}
    raw = {k: v.clone() for k, v in raw0.items()}
    m = {k: torch.zeros_like(v) for k, v in raw0.items()}
    v = {k: torch.zeros_like(x) for k, x in raw0.items()}
    upd = {k: torch.zeros_like(x) for k, x in raw0.items()}
    images = rast.alloc_images(1, H, W)
    rng = np.random.default_rng(66)
    target = torch.from_numpy(rng.uniform(0.0, 1.0, (1, 3, H, W)).astype(np.float32)).cuda()
    losses = torch.zeros(4, dtype=torch.float64, device="cuda")
    gnorm = torch.zeros(N, device="cuda")
    gcnt = torch.zeros(N, device="cuda")
    gcol = torch.empty_like(images["rgb"])
    gl = torch.empty_like(images["rgb"])
    gh = torch.empty_like(images["rgb"])

    def reset():
        for k in raw0:
            raw[k].copy_(raw0[k])
            sc[k].copy_(act0[k])
            m[k].zero_()
            v[k].zero_()
        for t in (losses, gnorm, gcnt):
            t.zero_()

    def body():
        _, state = rast.render(sc, cam, images=images, want_state=True)
        color_loss(images["rgb"], target, 0.2, losses=losses[0:2], grad=gcol, noalloc=True)
        fdo_cotangents(images["rgb"], target, 0.2, 0.4, losses=losses[2:4], grad_low=gl,
                       grad_high=gh)
        rast.backward_fdo(state, {"rgb": gcol}, gl, gh, upd)
        rast.densify_stats(state, gnorm, gcnt)
        adam_step(N, deg, raw, upd, m, v, 1, activated={k: sc[k] for k in raw})
        return state

    def snap():
        torch.cuda.synchronize()
        return dict(img={k: x.clone() for k, x in images.items()}, loss=losses.clone(),
                    upd={k: x.clone() for k, x in upd.items()},
                    raw={k: x.clone() for k, x in raw.items()}, gnorm=gnorm.clone(),
                    gcnt=gcnt.clone())

    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        reset()
        body().free()
    ref = snap()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        reset()
    s.synchronize()
    with torch.cuda.graph(g, stream=s):
        st_c = body()
    try:
        for rep in range(3):
            reset()
            other = rast.render(sc, sg.look_at_camera((0.0, 0.0, -3.0), width=40, height=30,
                                                      fx=30.0))[0]
            assert float(other["alpha"].max()) > 0.0
            reset()
            g.replay()
            got = snap()
            for k in IMG_KEYS:
                assert torch.equal(got["img"][k], ref["img"][k]), (rep, k)
            np.testing.assert_allclose(got["loss"].cpu().numpy(), ref["loss"].cpu().numpy(),
                                       rtol=1e-9)
            np.testing.assert_array_equal(got["gcnt"].cpu().numpy(), ref["gcnt"].cpu().numpy())
            for a, b in [(got["upd"][k], ref["upd"][k]) for k in PARAM_KEYS] + \
                    [(got["gnorm"], ref["gnorm"])]:
                a = a.double().cpu().numpy()
                b = b.double().cpu().numpy()
                assert np.all(np.abs(a - b) <= 1e-4 * np.abs(b) + 1e-5 * np.abs(b).max()), rep
            # Adam's first step moves a raw parameter by about -lr sign(g):
            # equal wherever the update is clear of zero
            for k in PARAM_KEYS:
                u = ref["upd"][k].double().cpu().numpy()
                clear = np.abs(u) > 1e-3 * np.abs(u).max()
                a = got["raw"][k].double().cpu().numpy()
                b = ref["raw"][k].double().cpu().numpy()
                fin = np.isfinite(b)
                np.testing.assert_array_equal(np.isfinite(a), fin)
                sel = clear & fin
                d = np.abs(a[sel] - b[sel])
                assert d.size == 0 or d.max() <= 1e-5, (rep, k, float(d.max()))
        say("[capture] training step: 3 replays equal the eager step")
    finally:
        del g
        st_c.free()
