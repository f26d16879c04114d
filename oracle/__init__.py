"""CPU reference renderer for the hybrid 2D/3D rasterizer: TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so``, built from
``hgs_oracle.cpp`` by :func:`build`.  It shares no code with the GPU library.

Functions
---------
structural(scene, cams, dilation)      binary32 culls, rects, tiles, keys, signs
sorted_pairs(st, cams)                 (key, value) list, stably sorted, + ranges
forward(scene, cams, pix, ...)         binary64 per-pixel composite (Eq. 1-2)
backward(scene, cams, pix, G, ...)     binary64 gradients (dual numbers)
sh_basis(degree, dirs)                 real SH basis used for colour
erank(sx, sy, sz) / type_exchange(...)  Adaptive Type Exchange (Eq. 3, P_x/P_y)
fdo.dwt / fdo.fdo_losses / fdo.fdo_project   Frequency-Decoupled Optimization (Alg. 1)
train.color_loss / train.adam_step       L1 + D-SSIM colour loss, Adam on raw parameters
surfel_uv(params, cam, pxy)            ray-plane (u, v, depth) of one surfel
full_pixels(cams) / all outputs reshaped to images: render_images(...)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hgs_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

DEFAULT_OPTS = dict(bg=(0.0, 0.0, 0.0), dilation=0.3, lambda_z=1.0, theta_z=1.05,
                    temp_z=0.001, pix_off=(0.0, 0.0), alpha_min=1.0 / 255.0, alpha_max=0.99,
                    t_min=1e-4)
# Tie margins (relative): activity |raw - alpha_min|, stop |T' - t_min|, clamp
# |raw - alpha_max|.  A decision this close to its threshold may go either way
# in a binary32 evaluation.
DEFAULT_MARGINS = (1e-4, 1e-3, 1e-3)


def build(force: bool = True) -> str:
    """Compile the oracle (g++, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC",
                               "-shared", "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = C.CDLL(_LIB)
        P = C.c_void_p
        _lib.oracle_structural.argtypes = ([P] * 5 + [C.c_int64, P, C.c_int, C.c_float,
                                                      C.c_double] + [P] * 5)
        _lib.oracle_sorted_pairs.argtypes = [P, P, P, C.c_int64, P, C.c_int, P, P, C.c_int64, P,
                                             C.c_int64]
        _lib.oracle_sorted_pairs.restype = C.c_int64
        _lib.oracle_forward.argtypes = ([P] * 6 + [C.c_int64, C.c_int] + [P] * 5 +
                                        [P, C.c_int, P, P, P, C.c_int64, P, C.c_int, C.c_int] +
                                        [P] * 6)
        _lib.oracle_backward.argtypes = ([P] * 6 + [C.c_int64, C.c_int] + [P] * 5 +
                                         [P, C.c_int, P, P, P, C.c_int64, P, P, C.c_int] +
                                         [P] * 6)
        _lib.oracle_screen_grad.argtypes = ([P] * 6 + [C.c_int64, C.c_int] + [P] * 5 +
                                            [P, C.c_int, P, P, P, C.c_int64, P, P, C.c_int, P])
        _lib.oracle_sh_basis.argtypes = [C.c_int, P, C.c_int64, P]
        _lib.oracle_surfel_uv.argtypes = [P, P, P, C.c_int64, P]
        _lib.oracle_erank.argtypes = [C.c_double, C.c_double, C.c_double]
        _lib.oracle_erank.restype = C.c_double
        _lib.oracle_type_exchange.argtypes = [P, P, P, C.c_int64, C.c_double, P, P, P, P, P]
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def pack_cams(cams) -> np.ndarray:
    if isinstance(cams, dict):
        cams = [cams]
    out = np.zeros((len(cams), 23), np.float32)
    for i, c in enumerate(cams):
        out[i, :16] = np.asarray(c["viewmat"], np.float32).reshape(16)
        out[i, 16:20] = [c["fx"], c["fy"], c["cx"], c["cy"]]
        out[i, 20] = c["width"]
        out[i, 21] = c["height"]
        out[i, 22] = c["znear"]
    return out


def _opts_vec(opts):
    o = dict(DEFAULT_OPTS)
    o.update(opts or {})
    return np.array(list(o["bg"]) + [o["dilation"], o["lambda_z"], o["theta_z"], o["temp_z"]] +
                    list(o["pix_off"]) + [o["alpha_min"], o["alpha_max"], o["t_min"]], np.float64)


def _f32(scene):
    return [np.ascontiguousarray(scene[k], np.float32) for k in
            ("means", "scales", "rotations", "opacities", "sh")] + \
        [np.ascontiguousarray(scene["types"], np.uint8)]


def _f64(scene, params64=None):
    src = params64 if params64 is not None else scene
    return [np.ascontiguousarray(src[k], np.float64) for k in
            ("means", "scales", "rotations", "opacities", "sh")]


def structural(scene, cams, dilation=0.3, alpha_min=1.0 / 255.0):
    lib = _load()
    m, s, r, o, _, t = _f32(scene)
    n = m.shape[0]
    cp = pack_cams(cams)
    V = cp.shape[0]
    valid = np.zeros(V * n, np.uint8)
    rect = np.zeros((V * n, 4), np.int32)
    tiles = np.zeros(V * n, np.uint32)
    zb = np.zeros(V * n, np.uint32)
    flip = np.zeros(V * n, np.uint8)
    lib.oracle_structural(_p(m), _p(s), _p(r), _p(o), _p(t), n, _p(cp), V, float(dilation),
                          float(alpha_min), _p(valid), _p(rect), _p(tiles), _p(zb), _p(flip))
    return dict(valid=valid, rect=rect, tiles=tiles, zbits=zb, flip=flip, n=n)


def tile_counts(cams):
    cp = pack_cams(cams)
    return [((int(c[20]) + 15) // 16) * ((int(c[21]) + 15) // 16) for c in cp]


def sorted_pairs(st, cams):
    lib = _load()
    cp = pack_cams(cams)
    V = cp.shape[0]
    wh = np.ascontiguousarray(cp[:, 20:22].astype(np.int32))
    n_tiles = int(sum(tile_counts(cams)))
    D = int(st["tiles"].astype(np.int64).sum())
    keys = np.zeros(max(D, 1), np.uint64)
    vals = np.zeros(max(D, 1), np.uint32)
    ranges = np.zeros((n_tiles, 2), np.uint32)
    got = lib.oracle_sorted_pairs(_p(st["valid"]), _p(st["rect"]), _p(st["zbits"]), st["n"],
                                  _p(wh), V, _p(keys), _p(vals), D, _p(ranges), n_tiles)
    assert got == D, (got, D)
    return keys[:D], vals[:D], ranges


def full_pixels(cam, view=0):
    H, W = cam["height"], cam["width"]
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    return np.ascontiguousarray(np.stack([np.full(H * W, view), yy.ravel(), xx.ravel()], 1),
                                np.int32)


def _flip_arr(flip, P):
    if flip is None:
        return None
    f = np.ascontiguousarray(np.broadcast_to(np.asarray(flip, np.uint32), (P,)), np.uint32)
    return f


def forward(scene, cams, pix, opts=None, *, params64=None, brute=False, threads=None,
            margins=DEFAULT_MARGINS, flip=None):
    """Binary64 forward at pixels ``pix`` ([P,3] = view, y, x).

    Returns dict(out=[P,8] (r,g,b,alpha,depth,nx,ny,nz), T=[P], n_contrib=[P],
    last=[P], tie=[P] bit flags (1 activity threshold, 2 stop, 4 clamp),
    nflags=[P] (activity and stop ties met), wcount=[2] (active pairs up to
    and including the stop, per type 2D/3D)).  ``flip`` ([P] or a scalar):
    bit k takes the other outcome of the k-th activity or stop tie of the
    pixel, a branch that a binary32 evaluation may legitimately follow.
    """
    lib = _load()
    m, s, r, o, sh, t = _f32(scene)
    m6, s6, r6, o6, sh6 = _f64(scene, params64)
    cp = pack_cams(cams)
    pix = np.ascontiguousarray(pix, np.int32).reshape(-1, 3)
    P = pix.shape[0]
    out = np.zeros((P, 8), np.float64)
    T = np.zeros(P, np.float64)
    cnt = np.zeros((P, 2), np.int32)
    tie = np.zeros(P, np.uint8)
    nfl = np.zeros(P, np.int32)
    wc = np.zeros(2, np.int64)
    ov = _opts_vec(opts)
    mg = np.asarray(margins, np.float64)
    fl = _flip_arr(flip, P)
    lib.oracle_forward(_p(m), _p(s), _p(r), _p(o), _p(sh), _p(t), m.shape[0],
                       int(scene["sh_degree"]), _p(m6), _p(s6), _p(r6), _p(o6), _p(sh6), _p(cp),
                       cp.shape[0], _p(ov), _p(mg), _p(pix), P,
                       None if fl is None else _p(fl), int(brute),
                       int(threads or os.cpu_count() or 1), _p(out), _p(T), _p(cnt), _p(tie),
                       _p(nfl), _p(wc))
    return dict(out=out, T=T, n_contrib=cnt[:, 0], last=cnt[:, 1], tie=tie, nflags=nfl,
                wcount=wc)


def backward(scene, cams, pix, G, opts=None, *, params64=None, threads=None,
             margins=DEFAULT_MARGINS, flip=None):
    """Binary64 gradients of L = sum_p <G_p, out_p> over pixels ``pix``, on
    the branches ``flip`` (see :func:`forward`).

    Returns dict of gradients (means [N,3], scales [N,3], rotations [N,4],
    opacities [N], sh [N,K,3]) and, as tolerance scales, the same keys with
    suffixes ``_abs`` (sums of the absolute per-pair terms), ``_cond`` (the
    rounding bound of a binary32 evaluation of the dL/dalpha~ path, in units
    of the binary32 unit roundoff; SH terms are products, so ``sh_cond`` is
    zero) and ``_tie`` (the difference between the clamped and unclamped
    branches at clamp ties; zero for SH).
    """
    lib = _load()
    m, s, r, o, sh, t = _f32(scene)
    m6, s6, r6, o6, sh6 = _f64(scene, params64)
    cp = pack_cams(cams)
    pix = np.ascontiguousarray(pix, np.int32).reshape(-1, 3)
    G = np.ascontiguousarray(G, np.float64)
    n = m.shape[0]
    K = sh.shape[1]
    gp = np.zeros((n, 11), np.float64)
    ap = np.zeros((n, 11), np.float64)
    gs = np.zeros((n, K, 3), np.float64)
    as_ = np.zeros((n, K, 3), np.float64)
    cp_ = np.zeros((n, 11), np.float64)
    xp = np.zeros((n, 11), np.float64)
    mg = np.asarray(margins, np.float64)
    fl = _flip_arr(flip, pix.shape[0])
    lib.oracle_backward(_p(m), _p(s), _p(r), _p(o), _p(sh), _p(t), n, int(scene["sh_degree"]),
                        _p(m6), _p(s6), _p(r6), _p(o6), _p(sh6), _p(cp), cp.shape[0],
                        _p(_opts_vec(opts)), _p(mg), _p(pix), pix.shape[0],
                        None if fl is None else _p(fl), _p(G),
                        int(threads or os.cpu_count() or 1), _p(gp), _p(gs), _p(ap), _p(as_),
                        _p(cp_), _p(xp))
    z = np.zeros_like(gs)
    out = dict(sh=gs, sh_abs=as_, sh_cond=z, sh_tie=z)
    for key, sl in (("means", slice(0, 3)), ("scales", slice(3, 6)), ("rotations", slice(6, 10)),
                    ("opacities", 10)):
        out[key] = gp[:, sl]
        out[key + "_abs"] = ap[:, sl]
        out[key + "_cond"] = cp_[:, sl]
        out[key + "_tie"] = xp[:, sl]
    return out


def screen_grad(scene, cams, pix, G, opts=None, *, params64=None, threads=None,
                margins=DEFAULT_MARGINS, flip=None):
    """dL/d delta [V, N, 2] (binary64): the gradient of L = sum_p <G_p, out_p>
    with respect to a translation of each splat's screen footprint (pixel
    units) in each view, on the tie branches ``flip`` (see :func:`forward`)."""
    lib = _load()
    m, s, r, o, sh, t = _f32(scene)
    m6, s6, r6, o6, sh6 = _f64(scene, params64)
    cp = pack_cams(cams)
    pix = np.ascontiguousarray(pix, np.int32)
    G = np.ascontiguousarray(G, np.float64)
    n = m.shape[0]
    V = cp.shape[0]
    out = np.zeros((V, n, 2), np.float64)
    mg = np.asarray(margins, np.float64)
    fl = _flip_arr(flip, pix.shape[0])
    lib.oracle_screen_grad(_p(m), _p(s), _p(r), _p(o), _p(sh), _p(t), n,
                           int(scene["sh_degree"]), _p(m6), _p(s6), _p(r6), _p(o6), _p(sh6),
                           _p(cp), V, _p(_opts_vec(opts)), _p(mg), _p(pix), pix.shape[0],
                           None if fl is None else _p(fl), _p(G),
                           int(threads or os.cpu_count() or 1), _p(out))
    return out


def densify_stats(scene, cams, pix, G, opts=None, *, flip=None):
    """3DGS's densification statistics for one backward: per splat, the sum
    over the views in which it is not culled of |dL/d(screen centre)| in
    NDC units (the pixel-unit gradient times (W/2, H/2)), and the number of
    those views.  Returns (grad_norm [N], count [N])."""
    if isinstance(cams, dict):
        cams = [cams]
    sg = screen_grad(scene, cams, pix, G, opts, flip=flip)
    o = dict(DEFAULT_OPTS)
    o.update(opts or {})
    st = structural(scene, cams, o["dilation"], o["alpha_min"])
    n = sg.shape[1]
    valid = st["valid"].reshape(len(cams), n) == 1
    norm = np.zeros(n)
    for v, c in enumerate(cams):
        nd = np.hypot(sg[v, :, 0] * c["width"] / 2.0, sg[v, :, 1] * c["height"] / 2.0)
        norm += np.where(valid[v], nd, 0.0)
    return norm, valid.sum(0).astype(np.int64)


def sh_basis(degree, dirs):
    lib = _load()
    d = np.ascontiguousarray(dirs, np.float64)
    K = (degree + 1) ** 2
    Y = np.zeros((d.shape[0], K), np.float64)
    lib.oracle_sh_basis(int(degree), _p(d), d.shape[0], _p(Y))
    return Y


def surfel_uv(params10, cam, pxy):
    lib = _load()
    prm = np.ascontiguousarray(params10, np.float64)
    pxy = np.ascontiguousarray(pxy, np.float64)
    out = np.zeros((pxy.shape[0], 3), np.float64)
    lib.oracle_surfel_uv(_p(prm), _p(pack_cams(cam)), _p(pxy), pxy.shape[0], _p(out))
    return out


def erank(sx, sy, sz):
    """Effective rank (Eq. 3) of scales (sx, sy, sz), binary64."""
    return _load().oracle_erank(float(sx), float(sy), float(sz))


def type_exchange(scales, rotations, types, theta=2.05):
    """Adaptive Type Exchange of n primitives (binary64 decisions).

    Returns dict(types u8[n], scales f32[n,3], quats f64[n,4] (unit, w >= 0
    where the rotation was rebuilt), erank f64[n], moved i32[n] (0 none,
    1 P_x, 2 P_y))."""
    lib = _load()
    s = np.ascontiguousarray(scales, np.float32)
    r = np.ascontiguousarray(rotations, np.float32)
    t = np.ascontiguousarray(types, np.uint8)
    n = s.shape[0]
    to = np.zeros(n, np.uint8)
    so = np.zeros((n, 3), np.float32)
    qo = np.zeros((n, 4), np.float64)
    er = np.zeros(n, np.float64)
    mv = np.zeros(n, np.int32)
    lib.oracle_type_exchange(_p(s), _p(r), _p(t), n, float(theta), _p(to), _p(so), _p(qo),
                             _p(er), _p(mv))
    return dict(types=to, scales=so, quats=qo, erank=er, moved=mv)


def images(res, cam, n_views=1):
    """Reshape a full-image ``forward`` result into [V,C,H,W] arrays."""
    H, W = cam["height"], cam["width"]
    o = res["out"].reshape(n_views, H, W, 8)
    return dict(rgb=o[..., 0:3].transpose(0, 3, 1, 2), alpha=o[..., 3:4].transpose(0, 3, 1, 2),
                depth=o[..., 4:5].transpose(0, 3, 1, 2), normal=o[..., 5:8].transpose(0, 3, 1, 2),
                T=res["T"].reshape(n_views, H, W), n_contrib=res["n_contrib"].reshape(n_views, H, W),
                last=res["last"].reshape(n_views, H, W), tie=res["tie"].reshape(n_views, H, W))


from . import fdo  # noqa: E402  (Frequency-Decoupled Optimization, binary64)
from . import train  # noqa: E402  (colour loss and Adam, binary64)
