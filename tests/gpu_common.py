"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the oracle on the same seeded inputs, and compare."""
import sys

import numpy as np

IMG_KEYS = ("rgb", "alpha", "depth", "normal")
PARAM_KEYS = ("means", "scales", "rotations", "opacities", "sh")
IMG_TOL = 1e-4      # max-abs on images, non-tie pixels
GRAD_RTOL = 1e-3    # per element, relative to |ref| + sum|terms|
GRAD_COND = 1e-5    # per element, times the binary32 condition scale (~170 ulp)
GRAD_L2 = 1e-3      # per tensor relative L2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_render(scene_np, cams, opts=None, G=None, want_state=True):
    """Returns (images dict of numpy [V,C,H,W], state, grads dict or None)."""
    import torch
    from paper_2512_02932_amd.rasterizer import get_rasterizer, to_device
    rast = get_rasterizer(0)
    sc = to_device(scene_np, "cuda")
    images, state = rast.render(sc, cams, opts, want_state=want_state)
    grads = None
    if G is not None:
        gi = {k: torch.from_numpy(np.ascontiguousarray(G[k], np.float32)).cuda() for k in IMG_KEYS}
        grads = {k: torch.zeros_like(sc[k]) for k in PARAM_KEYS}
        rast.backward(state, gi, grads)
        torch.cuda.synchronize()
        grads = {k: v.cpu().numpy() for k, v in grads.items()}
    torch.cuda.synchronize()
    imgs = {k: v.cpu().numpy() for k, v in images.items()}
    return imgs, state, grads


def oracle_pixels(cams):
    import oracle
    if isinstance(cams, dict):
        cams = [cams]
    return np.concatenate([oracle.full_pixels(c, v) for v, c in enumerate(cams)])


def pack_G_all(G, pix):
    """[V,C,H,W] dict -> [P,8] rows for the listed (view, y, x) pixels."""
    v, y, x = pix[:, 0], pix[:, 1], pix[:, 2]
    cols = [G["rgb"][v, 0, y, x], G["rgb"][v, 1, y, x], G["rgb"][v, 2, y, x],
            G["alpha"][v, 0, y, x], G["depth"][v, 0, y, x],
            G["normal"][v, 0, y, x], G["normal"][v, 1, y, x], G["normal"][v, 2, y, x]]
    return np.ascontiguousarray(np.stack(cols, 1), np.float64)


def gpu_at(imgs, pix):
    v, y, x = pix[:, 0], pix[:, 1], pix[:, 2]
    return np.stack([imgs["rgb"][v, 0, y, x], imgs["rgb"][v, 1, y, x], imgs["rgb"][v, 2, y, x],
                     imgs["alpha"][v, 0, y, x], imgs["depth"][v, 0, y, x],
                     imgs["normal"][v, 0, y, x], imgs["normal"][v, 1, y, x],
                     imgs["normal"][v, 2, y, x]], 1).astype(np.float64)


def compare_structural(state, scene_np, cams, opts=None):
    """Bit-exact: culls, rects, tiles, depth keys, sorted pairs, ranges."""
    import oracle
    dil = (opts or {}).get("dilation", 0.3)
    st = oracle.structural(scene_np, cams, dil)
    tiles = state.debug("tiles")
    np.testing.assert_array_equal(tiles, st["tiles"])
    valid = st["valid"] == 1
    np.testing.assert_array_equal(state.debug("zbits")[valid], st["zbits"][valid])
    np.testing.assert_array_equal(state.debug("rect")[valid], st["rect"][valid])
    keys, vals, ranges = oracle.sorted_pairs(st, cams)
    np.testing.assert_array_equal(state.debug("keys"), keys)
    np.testing.assert_array_equal(state.debug("vals"), vals)
    np.testing.assert_array_equal(state.debug("ranges"), ranges)
    return st, len(keys)


def compare_images(imgs, state, res, pix, max_tie_frac=0.01):
    """GPU vs oracle at pixels `pix`: images within IMG_TOL, n_contrib and
    last bit-exact, on pixels without a near-threshold decision."""
    tie = res["tie"] != 0
    ok = ~tie
    assert tie.mean() <= max_tie_frac, f"tie fraction {tie.mean():.4f}"
    g = gpu_at(imgs, pix)
    err = np.abs(g - res["out"])
    worst = err[ok].max() if ok.any() else 0.0
    assert worst <= IMG_TOL, f"max image error {worst:.3e}"
    V = int(pix[:, 0].max()) + 1
    HW = state.sizes()["HW"]
    Hh = imgs["alpha"].shape[2]
    Ww = imgs["alpha"].shape[3]
    flat = pix[:, 0].astype(np.int64) * HW + pix[:, 1].astype(np.int64) * Ww + pix[:, 2]
    nc = state.debug("n_contrib")[flat]
    last = state.debug("last")[flat]
    T = state.debug("T_final")[flat]
    np.testing.assert_array_equal(nc[ok], res["n_contrib"][ok])
    np.testing.assert_array_equal(last[ok], res["last"][ok])
    assert np.abs(T[ok] - res["T"][ok]).max() <= IMG_TOL
    return dict(max_err=float(worst), ties=int(tie.sum()), pixels=int(len(pix)), V=V, H=Hh)


def compare_grads(gg, ref):
    """Per element |g - ref| <= 1e-3 (|ref| + sum|terms|) + 1e-5 cond, where
    cond bounds the rounding of a binary32 evaluation (the dL/dalpha~ factor
    T (f - S) counted as T (|f| + |S|)); and per tensor relative L2 <= 1e-3."""
    report = {}
    for k in PARAM_KEYS:
        g = np.asarray(gg[k], np.float64).reshape(ref[k].shape)
        r = ref[k]
        scale = np.abs(r) + ref[k + "_abs"]
        bad = np.abs(g - r) > GRAD_RTOL * scale + GRAD_COND * ref[k + "_cond"] + 1e-9
        den = np.linalg.norm(r)
        rel = float(np.linalg.norm(g - r) / den) if den > 0 else float(np.linalg.norm(g))
        report[k] = (int(bad.sum()), rel)
        assert bad.sum() == 0, (k, int(bad.sum()), np.argwhere(bad)[:5].tolist(),
                                g[bad][:5].tolist(), r[bad][:5].tolist())
        assert rel <= GRAD_L2, (k, rel)
    return report
