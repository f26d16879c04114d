"""Batched serving (hgs_server_*): every served image equals the plain
per-request render of the same scene and camera, alone and in a mix of
scenes and resolutions, over repeated graph replays, after a pair-capacity
overflow, and against the oracle on sampled pixels."""
import numpy as np
import pytest

import scenegen as sg
from gpu_common import IMG_KEYS, check_pixels, say

pytestmark = pytest.mark.gpu

SCENES = None


def _scenes():
    global SCENES
    if SCENES is None:
        SCENES = [sg.scene_random(20_000, seed=61, frac2d=0.5),
                  sg.scene_sphere(n=30_000, frac2d=0.7, seed=62),
                  sg.scene_torus_knot(n=40_000, frac2d=0.5, seed=63)]
    return SCENES


def _requests():
    sizes = [(96, 64), (200, 137), (256, 256), (320, 180)]
    reqs = []
    for i in range(10):
        w, h = sizes[i % len(sizes)]
        cam = sg.orbit_camera(3.0 + 0.2 * i, 0.6 * i, 0.05 * (i % 5) - 0.1, w, h)
        reqs.append((i % 3, cam))
    # the 40k knot in 64 x 64 pixels: thousands of pairs per tile, so the
    # served forward runs split (half-quadrant) work units
    reqs.append((2, sg.orbit_camera(3.0, 0.4, 0.1, 64, 64)))
    return reqs


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2512_02932_amd.rasterizer import get_rasterizer, to_device
    rast = get_rasterizer(0)
    sids = [rast.scene_init(to_device(s), copy_resident=True) for s in _scenes()]
    plain = []
    for sid, cam in _requests():
        imgs, _ = rast.render_scene(sid, cam)
        torch.cuda.synchronize()
        plain.append({k: v.cpu().numpy() for k, v in imgs.items()})
    yield rast, sids, plain
    for sid in sids:
        rast.scene_release(sid)


def _serve(rast, sids, reqs, **cfg):
    import torch
    from paper_2512_02932_amd.serving import Server
    srv = Server(rast, **cfg)
    try:
        imgs = []
        for tag, (si, cam) in enumerate(reqs):
            im = srv.alloc_images(cam["height"], cam["width"])
            for t in im.values():
                t.fill_(float("nan"))
            srv.submit(sids[si], cam, im, tag)
            imgs.append(im)
        done = srv.drain(timeout_s=60.0)
        torch.cuda.synchronize()
        assert sorted(done) == list(range(len(reqs))), done
        st = srv.stats()
        return [{k: v.cpu().numpy() for k, v in im.items()} for im in imgs], st
    finally:
        srv.close()


def _same(a, b, tol=1e-4):
    for k in IMG_KEYS:
        assert np.isfinite(a[k]).all(), k
        err = float(np.abs(a[k] - b[k]).max())
        assert err <= tol, (k, err)


@pytest.mark.parametrize("use_graph", [True, False])
def test_served_images_equal_plain_render(env, use_graph):
    rast, sids, plain = env
    reqs = _requests()
    say(f"[serving] {len(reqs)} requests, graph={use_graph}")
    out, st = _serve(rast, sids, reqs, max_requests=4, max_batches=2, max_instances=200_000,
                     max_pairs=4_000_000, max_tiles=4096, use_graph=use_graph)
    say(f"[serving] stats {st}")
    assert st["batches"] >= 3 and st["rerendered"] == 0
    for i, o in enumerate(out):
        _same(o, plain[i])


def test_result_alone_equals_result_in_mix(env):
    rast, sids, plain = env
    reqs = _requests()
    alone, _ = _serve(rast, sids, [reqs[5]], max_requests=8, max_batches=1,
                      max_instances=200_000, max_pairs=4_000_000, max_tiles=4096, use_graph=True)
    mixed, st = _serve(rast, sids, reqs, max_requests=8, max_batches=1, max_instances=200_000,
                       max_pairs=4_000_000, max_tiles=4096, use_graph=True)
    assert st["batches"] <= 2
    _same(alone[0], mixed[5], tol=0.0)
    _same(mixed[5], plain[5])


def test_graph_replays_with_eager_work_between(env):
    import torch
    from paper_2512_02932_amd.serving import Server
    rast, sids, plain = env
    reqs = _requests()
    srv = Server(rast, max_requests=3, max_batches=2, max_instances=200_000,
                 max_pairs=4_000_000, max_tiles=4096, use_graph=True)
    try:
        for rep in range(3):
            imgs = []
            for tag, (si, cam) in enumerate(reqs):
                im = srv.alloc_images(cam["height"], cam["width"])
                srv.submit(sids[si], cam, im, 100 * rep + tag)
                imgs.append(im)
            srv.drain(timeout_s=60.0)
            # eager work of the program between replays
            x = torch.randn(1 << 20, device="cuda")
            _ = float((x * x).sum())
            torch.cuda.synchronize()
            for i, im in enumerate(imgs):
                _same({k: v.cpu().numpy() for k, v in im.items()}, plain[i])
            say(f"[serving] replay {rep} ok, stats {srv.stats()}")
    finally:
        srv.close()


def test_pair_overflow_rerenders(env):
    rast, sids, plain = env
    reqs = _requests()[:4]
    out, st = _serve(rast, sids, reqs, max_requests=4, max_batches=1, max_instances=200_000,
                     max_pairs=1000, max_tiles=4096, use_graph=True)
    say(f"[serving] overflow stats {st}")
    assert st["rerendered"] == len(reqs) and st["max_pairs"] > 1000
    for i, o in enumerate(out):
        _same(o, plain[i])


def test_served_images_match_oracle_on_samples(env):
    import oracle
    rast, sids, _ = env
    reqs = _requests()
    out, _ = _serve(rast, sids, reqs, max_requests=4, max_batches=2, max_instances=200_000,
                    max_pairs=4_000_000, max_tiles=4096, use_graph=True)
    rng = np.random.default_rng(7)
    for i in (0, 3, 6, 10):
        si, cam = reqs[i]
        H, W = cam["height"], cam["width"]
        pix = np.stack([np.zeros(400, np.int32), rng.integers(0, H, 400),
                        rng.integers(0, W, 400)], 1).astype(np.int32)
        res = oracle.forward(_scenes()[si], cam, pix)
        o = out[i]
        g = np.stack([o["rgb"][0, 0], o["rgb"][0, 1], o["rgb"][0, 2], o["alpha"][0, 0],
                      o["depth"][0, 0], o["normal"][0, 0], o["normal"][0, 1],
                      o["normal"][0, 2]], -1)[pix[:, 1], pix[:, 2]]
        # every sampled pixel; a tie pixel must match one of its branches
        _, _, rep = check_pixels(_scenes()[si], cam, pix, res, dict(out=g.astype(np.float64)))
        say(f"[serving] request {i}: oracle {rep}")


def test_submit_rejects_oversized_and_bad_requests(env):
    from paper_2512_02932_amd import _hgs as H
    from paper_2512_02932_amd.serving import Server
    rast, sids, _ = env
    srv = Server(rast, max_requests=2, max_batches=1, max_instances=25_000, max_pairs=100_000,
                 max_tiles=64, use_graph=False)
    try:
        cam = sg.orbit_camera(4.0, 0.0, 0.0, 64, 64)
        im = srv.alloc_images(64, 64)
        with pytest.raises(H.HGSError) as e:
            srv.submit(sids[1], cam, im, 1)  # 30k instances > 25k
        assert e.value.status == H.HGS_ECAPACITY
        big = sg.orbit_camera(4.0, 0.0, 0.0, 256, 256)  # 256 tiles > 64
        with pytest.raises(H.HGSError) as e:
            srv.submit(sids[0], big, srv.alloc_images(256, 256), 2)
        assert e.value.status == H.HGS_ECAPACITY
        with pytest.raises(H.HGSError) as e:
            srv.submit(999, cam, im, 3)
        assert e.value.status == H.HGS_EINVAL
        srv.submit(sids[0], cam, im, 4)
        assert srv.drain(timeout_s=30.0) == [4]
    finally:
        srv.close()
