"""Training-step kernels on the GPU (hgs_color_loss, hgs_adam_step) against
the oracle.

Colour loss: the binary32 moments form b2 = s_x^2 + s_y^2 + C2 as
S - mu^2, whose absolute error is about 1e-7 (S_xx + S_yy) <= 5e-8 against
b2 >= C2 = 9e-4, so SSIM and its derivative maps carry relative errors up
to ~5e-5 in flat regions: gradients are compared element-wise within 2e-4
of the largest magnitude, L1 within 1e-6 and D-SSIM within 5e-5 relative.

Adam: every quantity within a few binary32 roundings (2e-6) of the
magnitudes of its own terms, since its sums cancel: m = b1 m0 + (1-b1) g
against b1|m0| + (1-b1)|g|, v likewise, the parameter against |p| plus the
update's sensitivity to m^ and v^ (and the update's own rounding), the
activated value against the parameter's bound through the activation's
slope.  The chained gradient of a log-scale or logit goes through exp, add
and divide roundings, inside the same 2e-6.  Three steps with fresh
gradients, each step starting from the GPU's binary32 state."""
import numpy as np
import pytest

from gpu_common import PARAM_KEYS, say

pytestmark = pytest.mark.gpu


def _pair(V, H, W, seed):
    rng = np.random.default_rng(seed)
    y = rng.uniform(0.0, 1.0, (V, 3, H, W))
    # smooth target plus a rendered image with a bit of everything
    x = np.clip(y + rng.normal(0.0, 0.08, y.shape), 0.0, 1.0)
    x[..., : H // 3, :] = y[..., : H // 3, :]  # identical band: sign(0) and SSIM = 1 there
    return x.astype(np.float32), y.astype(np.float32)


@pytest.mark.parametrize("V,H,W", [(1, 32, 48), (2, 37, 53), (1, 5, 7), (1, 1, 1), (1, 64, 33),
                                   (1, 540, 960)])
def test_color_loss_matches_oracle(V, H, W):
    import torch
    from oracle import train
    from paper_2512_02932_amd.rasterizer import color_loss
    x, y = _pair(V, H, W, seed=V * 7 + H * 3 + W)
    grad, losses = color_loss(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), 0.2)
    torch.cuda.synchronize()
    grad, losses = grad.cpu().numpy(), losses.cpu().numpy()
    ref = train.color_loss(x.astype(np.float64), y.astype(np.float64), 0.2)
    assert losses[0] == pytest.approx(ref["l1"], rel=1e-6, abs=1e-12)
    assert losses[1] == pytest.approx(ref["dssim"], rel=5e-5, abs=1e-9)
    err = float(np.abs(grad - ref["grad"]).max())
    scale = float(np.abs(ref["grad"]).max())
    assert err <= 2e-4 * scale + 1e-30, (err, scale)
    say(f"[train] colour loss {V}x{H}x{W}: L1 {losses[0]:.6f} D-SSIM {losses[1]:.6f}, "
        f"grad err {err / max(scale, 1e-30):.2e} of max")


def test_color_loss_of_identical_images_is_zero():
    import torch
    from paper_2512_02932_amd.rasterizer import color_loss
    rng = np.random.default_rng(5)
    x = torch.from_numpy(rng.uniform(0, 1, (1, 3, 40, 40)).astype(np.float32)).cuda()
    grad, losses = color_loss(x, x.clone(), 0.2)
    torch.cuda.synchronize()
    assert abs(float(losses[0])) == 0.0
    assert abs(float(losses[1])) <= 1e-6
    assert float(grad.abs().max()) <= 1e-6 / (3 * 40 * 40)


def _adam_state(n, deg, seed):
    rng = np.random.default_rng(seed)
    K = (deg + 1) ** 2
    raw = {"means": rng.normal(size=(n, 3)), "scales": rng.normal(-4, 1, (n, 3)),
           "rotations": rng.normal(size=(n, 4)), "opacities": rng.normal(size=(n,)),
           "sh": rng.normal(0, 0.3, (n, K, 3))}
    raw = {k: v.astype(np.float32) for k, v in raw.items()}
    return raw, rng


LR = dict(lr_means=1.6e-4, lr_scales=5e-3, lr_rotations=1e-3, lr_opacities=2.5e-2,
          lr_sh_dc=2.5e-3, lr_sh_rest=2.5e-3 / 20)


def _oracle_lr(K):
    return {"means": LR["lr_means"], "scales": LR["lr_scales"], "rotations": LR["lr_rotations"],
            "opacities": LR["lr_opacities"],
            "sh": np.array([LR["lr_sh_dc"]] + [LR["lr_sh_rest"]] * (K - 1))[:, None]}


@pytest.mark.parametrize("n,deg", [(1001, 3), (5, 0), (1, 1)])
def test_adam_matches_oracle(n, deg):
    import torch
    from oracle import train
    from paper_2512_02932_amd.rasterizer import adam_step
    K = (deg + 1) ** 2
    raw, rng = _adam_state(n, deg, seed=n + deg)
    dev = {k: torch.from_numpy(v.copy()).cuda() for k, v in raw.items()}
    m = {k: torch.zeros_like(v) for k, v in dev.items()}
    v = {k: torch.zeros_like(x) for k, x in dev.items()}
    act = {k: torch.zeros_like(x) for k, x in dev.items()}
    ref_raw = {k: x.astype(np.float64) for k, x in raw.items()}
    ref_m = {k: np.zeros_like(x) for k, x in ref_raw.items()}
    ref_v = {k: np.zeros_like(x) for k, x in ref_raw.items()}
    for step in range(1, 4):
        g = {k: rng.normal(size=x.shape).astype(np.float32) for k, x in raw.items()}
        # the oracle starts from the GPU's binary32 state of the previous
        # step, so each step is compared on its own
        cur = {k: t.cpu().numpy().astype(np.float64) for k, t in dev.items()}
        cm = {k: t.cpu().numpy().astype(np.float64) for k, t in m.items()}
        cv = {k: t.cpu().numpy().astype(np.float64) for k, t in v.items()}
        adam_step(n, deg, dev, {k: torch.from_numpy(x).cuda() for k, x in g.items()}, m, v, step,
                  activated=act, **LR)
        torch.cuda.synchronize()
        r_raw, r_m, r_v, r_act = train.adam_step(cur, g, cm, cv, step, _oracle_lr(K))
        b1, b2, eps = 0.9, 0.999, 1e-15
        bc1, bc2 = 1.0 / (1.0 - b1 ** step), 1.0 / (1.0 - b2 ** step)
        u = 2e-6  # a few binary32 roundings per term
        for k in PARAM_KEYS:
            lr = np.broadcast_to(np.asarray(_oracle_lr(K)[k], np.float64), r_raw[k].shape)
            gr = g[k].astype(np.float64)  # the chained raw gradient, for the bounds only
            if k == "scales":
                gr = gr * np.exp(cur[k])
            elif k == "opacities":
                sg = 1.0 / (1.0 + np.exp(-cur[k]))
                gr = gr * sg * (1.0 - sg)
            tol_m = u * (b1 * np.abs(cm[k]) + (1 - b1) * np.abs(gr))
            tol_v = u * (b2 * cv[k] + (1 - b2) * gr * gr)
            mh, vh = r_m[k] * bc1, r_v[k] * bc2
            sq = np.sqrt(vh)
            # the update lr m^/(sqrt v^ + eps) moves with m^ and v^; p rounds once
            tol_p = u * np.abs(cur[k]) + lr * ((tol_m * bc1 + u * np.abs(mh)) / (sq + eps) +
                                               np.abs(mh) * tol_v * bc2 /
                                               np.maximum(2 * sq * (sq + eps) ** 2, 1e-300))
            # the activated value carries the parameter's error through the
            # activation's slope (1, exp itself, sigmoid <= 1/4)
            slope = np.abs(r_act[k]) if k == "scales" else 1.0
            for got, want, tol in ((dev[k], r_raw[k], tol_p), (m[k], r_m[k], tol_m),
                                   (v[k], r_v[k], tol_v),
                                   (act[k], r_act[k], tol_p * slope + u * np.abs(r_act[k]))):
                gg = got.cpu().numpy().astype(np.float64)
                bad = np.abs(gg - want) > tol + 1e-30
                assert not bad.any(), (k, step, np.argwhere(bad)[:3].tolist(), gg[bad][:3],
                                       want[bad][:3])
        ref_raw = r_raw
    say(f"[train] adam n={n} deg={deg}: 3 steps ok")


def test_adam_skips_null_arrays_and_activated():
    import torch
    from paper_2512_02932_amd.rasterizer import adam_step
    n, deg = 100, 3
    raw, rng = _adam_state(n, deg, seed=3)
    dev = {k: torch.from_numpy(v.copy()).cuda() for k, v in raw.items()}
    g = {k: torch.from_numpy(rng.normal(size=x.shape).astype(np.float32)).cuda()
         for k, x in raw.items()}
    m = {k: torch.zeros_like(x) for k, x in dev.items()}
    v = {k: torch.zeros_like(x) for k, x in dev.items()}
    part = {k: t for k, t in dev.items() if k != "rotations"}
    adam_step(n, deg, part, g, m, v, 1, **LR)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dev["rotations"].cpu().numpy(), raw["rotations"])
    assert float(m["rotations"].abs().max()) == 0.0
    assert not np.array_equal(dev["means"].cpu().numpy(), raw["means"])


def test_bad_arguments():
    import torch
    from paper_2512_02932_amd import _hgs as H
    from paper_2512_02932_amd.rasterizer import get_rasterizer
    rast = get_rasterizer(0)
    p = torch.zeros(64, device="cuda").data_ptr()
    with pytest.raises(H.HGSError) as e:
        H.hgs_color_loss(rast.ctx, 1, 4, 4, p, p, 1.5, 0, 0, 0)
    assert e.value.status == H.HGS_EINVAL
    with pytest.raises(H.HGSError) as e:
        H.hgs_color_loss(rast.ctx, 1, 4, 4, 0, p, 0.2, 0, 0, 0)
    assert e.value.status == H.HGS_EINVAL
    H.hgs_color_loss(rast.ctx, 0, 4, 4, 0, 0, 0.2, 0, 0, 0)  # empty: no-op
    g = H.hgs_grads()
    g.means = p
    z = H.hgs_grads()
    o = H.hgs_adam_opts(beta1=0.9, beta2=0.999, eps=1e-15, step=1)
    with pytest.raises(H.HGSError) as e:
        H.hgs_adam_step(rast.ctx, 4, 3, g, z, z, z, None, o, 0)  # means without grad/moments
    assert e.value.status == H.HGS_EINVAL
    o.step = 0
    with pytest.raises(H.HGSError) as e:
        H.hgs_adam_step(rast.ctx, 4, 3, z, z, z, z, None, o, 0)
    assert e.value.status == H.HGS_EINVAL


DENSIFY_CASES = {
    "random2k_200x137": lambda: (__import__("scenegen").scene_random(2000, seed=12, log_mu=-3.2),
                                 [__import__("scenegen").look_at_camera(
                                     (0.3, -0.2, -3.5), width=200, height=137, fx=150.0)]),
    "sphere20k_3views": lambda: (__import__("scenegen").scene_sphere(20_000, seed=14),
                                 [__import__("scenegen").look_at_camera(e, width=96, height=80,
                                                                        fx=70.0)
                                  for e in [(0.0, 0.0, -3.0), (2.0, 0.5, -2.2),
                                            (-1.5, -1.0, -2.5)]]),
}


@pytest.mark.parametrize("name", sorted(DENSIFY_CASES))
@pytest.mark.parametrize("fdo", [False, True])
def test_densify_stats_match_oracle(name, fdo):
    """|dL/d screen centre| in NDC units summed over the views where the
    splat is not culled, and those views' count; with FDO the statistic of
    the three losses' sum.  Per splat within 2e-3 of its value plus 2e-5 of
    the largest (the accumulator slots' binary32 sums, as the gradients)."""
    import torch
    import oracle
    import scenegen as sg
    from gpu_common import compare_images, oracle_pixels, pack_G_all
    from paper_2512_02932_amd.rasterizer import get_rasterizer, to_device
    scene, cams = DENSIFY_CASES[name]()
    V, H, W = len(cams), cams[0]["height"], cams[0]["width"]
    N = scene["means"].shape[0]
    pix = oracle_pixels(cams)
    res = oracle.forward(scene, cams, pix)
    G = sg.upstream_grads(V, H, W, seed=301)
    Gl = sg.upstream_grads(V, H, W, seed=302)["rgb"]
    Gh = sg.upstream_grads(V, H, W, seed=303)["rgb"]
    rast = get_rasterizer(0)
    sc = to_device(scene)
    imgs, state = rast.render(sc, cams, want_state=True)
    torch.cuda.synchronize()
    _, flip, _ = compare_images({k: v.cpu().numpy() for k, v in imgs.items()}, state, res, pix,
                                scene, cams)
    gdev = {k: torch.from_numpy(v).cuda() for k, v in G.items()}
    grads = {k: torch.zeros_like(sc[k]) for k in PARAM_KEYS}
    if fdo:
        rast.backward_fdo(state, gdev, torch.from_numpy(Gl).cuda(), torch.from_numpy(Gh).cuda(),
                          grads)
        Gtot = dict(G, rgb=G["rgb"] + Gl + Gh)
    else:
        rast.backward(state, gdev, grads)
        Gtot = G
    norm = torch.zeros(N, device="cuda")
    cnt = torch.zeros(N, device="cuda")
    rast.densify_stats(state, norm, cnt)
    rast.densify_stats(state, norm, cnt)  # adds: twice the statistic
    torch.cuda.synchronize()
    state.free()
    ref_norm, ref_cnt = oracle.densify_stats(scene, cams, pix, pack_G_all(Gtot, pix), flip=flip)
    np.testing.assert_array_equal(cnt.cpu().numpy(), 2 * ref_cnt)
    got = norm.cpu().numpy() / 2
    bad = np.abs(got - ref_norm) > 2e-3 * ref_norm + 2e-5 * ref_norm.max()
    assert not bad.any(), (int(bad.sum()), got[bad][:5], ref_norm[bad][:5])
    say(f"[train] densify {name} fdo={fdo}: {int((ref_cnt > 0).sum())} visible, "
        f"max rel err {float(np.max(np.abs(got - ref_norm) / np.maximum(ref_norm, 1e-30))):.2e}")


def test_densify_stats_needs_a_backward():
    import torch
    import scenegen as sg
    from paper_2512_02932_amd import _hgs as H
    from paper_2512_02932_amd.rasterizer import get_rasterizer, to_device
    rast = get_rasterizer(0)
    sc = to_device(sg.scene_random(100, seed=1))
    _, state = rast.render(sc, sg.look_at_camera((0, 0, -3), width=32, height=32, fx=30.0),
                           want_state=True)
    with pytest.raises(H.HGSError) as e:
        rast.densify_stats(state, torch.zeros(100, device="cuda"))
    assert e.value.status == H.HGS_ESTATE
    state.free()


# ---------------------------------------------------------------------------
# Full size: the launch configuration the benchmark times (1M hybrid
# Gaussians, SH3, 1920x1080).
# ---------------------------------------------------------------------------
def test_full_size_color_loss_1080p():
    test_color_loss_matches_oracle(1, 1080, 1920)


def test_full_size_adam_1m():
    import torch
    from oracle import train
    from paper_2512_02932_amd.rasterizer import adam_step
    n, deg = 1_000_000, 3
    K = (deg + 1) ** 2
    raw, rng = _adam_state(n, deg, seed=77)
    dev = {k: torch.from_numpy(v.copy()).cuda() for k, v in raw.items()}
    m = {k: torch.zeros_like(v) for k, v in dev.items()}
    v = {k: torch.zeros_like(x) for k, x in dev.items()}
    act = {k: torch.zeros_like(x) for k, x in dev.items()}
    g = {k: rng.normal(size=x.shape).astype(np.float32) for k, x in raw.items()}
    adam_step(n, deg, dev, {k: torch.from_numpy(x).cuda() for k, x in g.items()}, m, v, 1,
              activated=act, **LR)
    torch.cuda.synchronize()
    z = {k: np.zeros(x.shape) for k, x in raw.items()}
    r_raw, r_m, r_v, r_act = train.adam_step({k: x.astype(np.float64) for k, x in raw.items()},
                                             g, z, z, 1, _oracle_lr(K))
    for k in PARAM_KEYS:
        lr = np.broadcast_to(np.asarray(_oracle_lr(K)[k], np.float64), r_raw[k].shape)
        # first step from zero moments: m = (1-b1) g, v = (1-b2) g^2, p - lr g/|g|
        for got, want, tol in ((dev[k], r_raw[k], 2e-6 * np.abs(raw[k]) + 2e-6 * lr),
                               (m[k], r_m[k], 2e-6 * np.abs(r_m[k])),
                               (v[k], r_v[k], 2e-6 * np.abs(r_v[k]))):
            gg = got.cpu().numpy().astype(np.float64)
            assert (np.abs(gg - want) <= tol + 1e-30).all(), k
    say("[train] adam at 1M SH3: ok")


def test_full_size_densify_1m_1080p_sampled():
    """Cotangents on 1500 distinct sampled pixels of the 1080p image (tie
    pixels included, on the branch the GPU took); the oracle evaluates those
    pixels only."""
    import torch
    import oracle
    import scenegen as sg
    from gpu_common import IMG_KEYS, compare_images, pack_G_all
    from paper_2512_02932_amd.rasterizer import get_rasterizer, to_device
    scene = sg.scene_torus_knot()
    cam = sg.camera_torus_knot_1080p()
    N = scene["means"].shape[0]
    rng = np.random.default_rng(9)
    pix = np.stack([np.zeros(4000, np.int64), rng.integers(0, 1080, 4000),
                    rng.integers(0, 1920, 4000)], 1).astype(np.int32)
    _, first = np.unique(pix[:, 1].astype(np.int64) * 1920 + pix[:, 2], return_index=True)
    pix = np.ascontiguousarray(pix[np.sort(first)[:1500]])
    res = oracle.forward(scene, cam, pix)
    sel = pix
    G = {k: np.zeros((1, c, 1080, 1920), np.float32)
         for k, c in (("rgb", 3), ("alpha", 1), ("depth", 1), ("normal", 3))}
    Gs = sg.upstream_grads(1, 1, len(sel), seed=11)
    for k in IMG_KEYS:
        G[k][0][:, sel[:, 1], sel[:, 2]] = Gs[k][0][:, 0, :]
    rast = get_rasterizer(0)
    sc = to_device(scene)
    imgs, state = rast.render(sc, cam, want_state=True)
    torch.cuda.synchronize()
    _, flip, _ = compare_images({k: v.cpu().numpy() for k, v in imgs.items()}, state, res, pix,
                                scene, cam)
    grads = {k: torch.zeros_like(sc[k]) for k in PARAM_KEYS}
    rast.backward(state, {k: torch.from_numpy(v).cuda() for k, v in G.items()}, grads)
    norm = torch.zeros(N, device="cuda")
    cnt = torch.zeros(N, device="cuda")
    rast.densify_stats(state, norm, cnt)
    torch.cuda.synchronize()
    state.free()
    ref_norm, ref_cnt = oracle.densify_stats(scene, cam, sel, pack_G_all(G, sel), flip=flip)
    np.testing.assert_array_equal(cnt.cpu().numpy(), ref_cnt)
    got = norm.cpu().numpy()
    bad = np.abs(got - ref_norm) > 2e-3 * ref_norm + 2e-5 * ref_norm.max()
    assert not bad.any(), (int(bad.sum()), got[bad][:5], ref_norm[bad][:5])
    say(f"[train] densify at 1M / 1080p: {int((ref_norm > 0).sum())} splats touched by the "
        f"sampled cotangents, {int(ref_cnt.sum())} visible")
