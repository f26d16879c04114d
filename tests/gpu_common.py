"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the oracle on the same seeded inputs, and compare."""
import os
import sys

import numpy as np

IMG_KEYS = ("rgb", "alpha", "depth", "normal")
PARAM_KEYS = ("means", "scales", "rotations", "opacities", "sh")
IMG_TOL = 1e-4      # max-abs on images
GRAD_RTOL = 1e-3    # per element, relative to |ref| + sum|terms|
# Per element, times the oracle's rounding bound of the dL/dalpha~ path
# (counted in binary32 unit roundoffs, u = 2^-24): eight units per step.
GRAD_COND = 8.0 * 2.0 ** -24
GRAD_L2 = 1e-3      # per tensor relative L2
MAX_TIE_BITS = 4    # branches tried per tie pixel: 2^4 outcome combinations


def say(*a):
    """Prints a progress or report line; with HGS_PARITY_LOG set, also
    appends it to that file (the parity summary of a run)."""
    print(*a, flush=True)
    sys.stdout.flush()
    path = os.environ.get("HGS_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(" ".join(str(x) for x in a) + "\n")


def gpu_render(scene_np, cams, opts=None, G=None, want_state=True):
    """Returns (images dict of numpy [V,C,H,W], state, grads dict or None)."""
    import torch
    from paper_2512_02932_amd.rasterizer import get_rasterizer, to_device
    rast = get_rasterizer(0)
    sc = to_device(scene_np, "cuda")
    images, state = rast.render(sc, cams, opts, want_state=want_state)
    if state is not None:
        state.check()  # the pairs fit the capacity: the images are complete
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
    o = dict(oracle.DEFAULT_OPTS)
    o.update(opts or {})
    st = oracle.structural(scene_np, cams, o["dilation"], o["alpha_min"])
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


def gpu_counts(state, imgs, pix):
    """GPU n_contrib, last and T_final at pixels `pix` ([P,3] view, y, x)."""
    HW = state.sizes()["HW"]
    Ww = imgs["alpha"].shape[3]
    flat = pix[:, 0].astype(np.int64) * HW + pix[:, 1].astype(np.int64) * Ww + pix[:, 2]
    return (state.debug("n_contrib")[flat].astype(np.int64),
            state.debug("last")[flat].astype(np.int64),
            state.debug("T_final")[flat].astype(np.float64))


def gpu_pixels(state, imgs, pix):
    """The GPU's outputs at `pix`: dict(out [P,8], n_contrib, last, T)."""
    nc, last, T = gpu_counts(state, imgs, pix)
    return dict(out=gpu_at(imgs, pix), n_contrib=nc, last=last, T=T)


def resolve_ties(scene, cams, pix, res, gpu, opts=None):
    """Tie pixels: a pixel where an activity (alpha_min) or stop (t_min)
    decision lies within rounding of its threshold has two correct outcomes
    of that decision (Eq. 2 with either choice).  For each tie pixel the
    oracle evaluates the branches (every combination of its first
    MAX_TIE_BITS ties) and the one the GPU took is identified by its
    n_contrib, last, T_final and images; the oracle's outputs of that branch
    replace the binary64 decision's.  `gpu` is gpu_pixels(...) at `pix`.
    Returns (res with the branches substituted, flip [P] of the branches,
    report).  A tie pixel whose GPU result matches no branch is left as it
    is, and the comparison that follows fails there."""
    import oracle
    res = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in res.items()}
    flip = np.zeros(len(pix), np.uint32)
    idx = np.flatnonzero((res["tie"] & 3) != 0)
    rep = dict(tie_pixels=int(len(idx)), other_branch=0, unmatched=0)
    if len(idx) == 0:
        return res, flip, rep
    sub = np.ascontiguousarray(pix[idx])
    g_out = gpu["out"][idx]
    chosen = np.full(len(idx), -1, np.int64)
    for mask in range(2 ** MAX_TIE_BITS):
        r = oracle.forward(scene, cams, sub, opts, flip=mask)
        used = mask < (1 << np.minimum(r["nflags"], 31).astype(np.int64))
        ok = used & (chosen < 0) & (np.abs(r["out"] - g_out).max(1) <= IMG_TOL)
        if gpu.get("n_contrib") is not None:  # images only (no state) otherwise
            ok &= ((r["n_contrib"] == gpu["n_contrib"][idx]) & (r["last"] == gpu["last"][idx]) &
                   (np.abs(r["T"] - gpu["T"][idx]) <= IMG_TOL))
        chosen[ok] = mask
        for k in ("out", "T", "n_contrib", "last"):
            res[k][idx[ok]] = r[k][ok]
        if (chosen >= 0).all():
            break
    flip[idx[chosen > 0]] = chosen[chosen > 0]
    rep["other_branch"] = int((chosen > 0).sum())
    rep["unmatched"] = int((chosen < 0).sum())
    return res, flip, rep


def check_pixels(scene, cams, pix, res, gpu, opts=None):
    """resolve_ties, then every pixel of `pix`: images within IMG_TOL,
    n_contrib and last bit-exact, T_final within IMG_TOL.  Returns
    (res on the GPU's branches, flip, report)."""
    res, flip, trep = resolve_ties(scene, cams, pix, res, gpu, opts)
    err = np.abs(gpu["out"] - res["out"])
    worst = float(err.max()) if len(pix) else 0.0
    assert worst <= IMG_TOL, (f"max image error {worst:.3e}", trep,
                              pix[np.argmax(err.max(1))].tolist())
    if gpu.get("n_contrib") is not None:
        np.testing.assert_array_equal(gpu["n_contrib"], res["n_contrib"])
        np.testing.assert_array_equal(gpu["last"], res["last"])
        assert np.abs(gpu["T"] - res["T"]).max(initial=0.0) <= IMG_TOL
    rep = dict(max_err=worst, pixels=int(len(pix)),
               clamp_ties=int(((res["tie"] & 4) != 0).sum()), **trep)
    return res, flip, rep


def compare_images(imgs, state, res, pix, scene, cams, opts=None):
    """GPU vs oracle at every pixel of `pix`, tie pixels on the branch the
    GPU took (check_pixels).  Returns (res on the GPU's branches, flip,
    report)."""
    return check_pixels(scene, cams, pix, res, gpu_pixels(state, imgs, pix), opts)


def compare_grads(gg, ref, keys=PARAM_KEYS):
    """Per element
        |g - ref| <= 1e-3 (|ref| + sum|terms|) + GRAD_COND cond + tie,
    where cond is the oracle's rounding bound of a binary32 evaluation of the
    dL/dalpha~ path and tie the spread between the two branches of clamp
    ties; per tensor relative L2 <= 1e-3; and every element of at least 1%
    of the tensor's largest magnitude within a plain 1e-3 |ref|.  The report
    counts, per tensor, the elements that pass only through the cond or tie
    allowance, and those large elements that miss the plain bound (0).
    "Large" leaves out elements that are sums of much larger terms of both
    signs (sum|terms| > 10 |ref|): the binary32 accumulation of a splat's
    per-pixel terms, in whatever order the atomics land, can miss 1e-3 |ref|
    there by cancellation alone; the per-term bound still holds for them."""
    report = {}
    for k in keys:
        g = np.asarray(gg[k], np.float64).reshape(ref[k].shape)
        r = ref[k]
        err = np.abs(g - r)
        base = GRAD_RTOL * (np.abs(r) + ref[k + "_abs"]) + 1e-9
        allow = GRAD_COND * ref[k + "_cond"] + ref[k + "_tie"]
        bad = err > base + allow
        den = np.linalg.norm(r)
        rel = float(np.linalg.norm(g - r) / den) if den > 0 else float(np.linalg.norm(g))
        big = np.abs(r) >= 1e-2 * np.abs(r).max(initial=0.0)
        cancel = ref[k + "_abs"] > 10.0 * np.abs(r)
        report[k] = dict(bad=int(bad.sum()), rel_l2=rel, via_allowance=int((err > base).sum()),
                         big_over_plain=int((big & ~cancel & (err > GRAD_RTOL * np.abs(r))).sum()),
                         big_cancelling=int((big & cancel).sum()), n=int(r.size))
        assert bad.sum() == 0, (k, int(bad.sum()), np.argwhere(bad)[:5].tolist(),
                                g[bad][:5].tolist(), r[bad][:5].tolist())
        assert rel <= GRAD_L2, (k, rel)
        # elements of at least 1% of the tensor's largest magnitude pass the
        # plain relative bound, without the per-term and rounding allowances
        assert report[k]["big_over_plain"] == 0, (k, report[k])
    return report
