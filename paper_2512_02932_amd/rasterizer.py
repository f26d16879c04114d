"""PyTorch-facing API of the gfx950 hybrid rasterizer.

PyTorch supplies device memory and the current stream; every computation runs
in ``libhgs.so`` through the C ABI (include/hgs.h).

* ``Rasterizer``: one context per device; resident or borrowed scenes.
* ``render(...)``: forward only (serving / evaluation).
* ``HybridRasterize``: a ``torch.autograd.Function``.  Its forward keeps an
  opaque library state, and its backward calls ``hgs_render_backward``, which
  recomputes transmittance in reverse.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _hgs as H

SCENE_KEYS = ("means", "scales", "rotations", "opacities", "sh", "types")
DEFAULT_OPTS = dict(bg=(0.0, 0.0, 0.0), dilation=0.3, lambda_z=1.0, theta_z=1.05, temp_z=0.001,
                    alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4, out_mask=0)

DEBUG = dict(keys=(0, np.uint64, 1), vals=(1, np.uint32, 1), ranges=(2, np.uint32, 2),
             rect=(3, np.int32, 4), tiles=(4, np.uint32, 1), zbits=(5, np.uint32, 1),
             T_final=(6, np.float32, 1), last=(7, np.uint32, 1), n_contrib=(8, np.uint32, 1),
             wcount=(9, np.uint32, 1))


def _ptr(t):
    return None if t is None else t.data_ptr()


def make_camera(cam: dict) -> H.hgs_camera:
    c = H.hgs_camera()
    vm = np.asarray(cam["viewmat"], np.float32).reshape(16)
    for i in range(16):
        c.viewmat[i] = float(vm[i])
    c.fx, c.fy, c.cx, c.cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.znear = float(cam.get("znear", 0.2))
    return c


def make_cameras(cams) -> C.Array:
    if isinstance(cams, dict):
        cams = [cams]
    arr = (H.hgs_camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = make_camera(c)
    return arr


def make_opts(opts: dict | None) -> H.hgs_opts:
    o = dict(DEFAULT_OPTS)
    o.update(opts or {})
    r = H.hgs_opts()
    for i in range(3):
        r.bg[i] = float(o["bg"][i])
    for k in ("dilation", "lambda_z", "theta_z", "temp_z", "alpha_min", "alpha_max", "t_min"):
        setattr(r, k, float(o[k]))
    r.out_mask = int(o["out_mask"])
    return r


def _check_scene(t: dict):
    for k in SCENE_KEYS:
        x = t[k]
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.is_contiguous()):
            raise ValueError(f"scene[{k!r}] must be a contiguous CUDA tensor")
    for k in SCENE_KEYS[:-1]:
        if t[k].dtype != torch.float32:
            raise ValueError(f"scene[{k!r}] must be float32")
    if t["types"].dtype != torch.uint8:
        raise ValueError("scene['types'] must be uint8")


def scene_desc(t: dict) -> H.hgs_scene_desc:
    _check_scene(t)
    n = t["means"].shape[0]
    K = t["sh"].shape[1]
    deg = int(round(K ** 0.5)) - 1
    d = H.hgs_scene_desc()
    d.n = n
    d.sh_degree = deg
    d.means, d.scales, d.rotations, d.opacities, d.sh, d.types = (
        t[k].data_ptr() for k in SCENE_KEYS)
    return d


class State:
    """Owns one ``hgs_state``; freed on ``free()`` or garbage collection."""

    def __init__(self, rast: "Rasterizer", handle, keep=()):
        self.rast = rast
        self.handle = handle
        self.keep = keep  # tensors the state borrows

    def sizes(self):
        VN, D, T, HW, V = H.hgs_state_sizes(self.rast.ctx, self.handle)
        return dict(VN=VN, D=D, n_tiles=T, HW=HW, V=V)

    def debug(self, name: str) -> np.ndarray:
        what, dt, width = DEBUG[name]
        sz = self.sizes()
        count = {"keys": sz["D"], "vals": sz["D"], "ranges": sz["n_tiles"], "rect": sz["VN"],
                 "tiles": sz["VN"], "zbits": sz["VN"], "T_final": sz["V"] * sz["HW"],
                 "last": sz["V"] * sz["HW"], "n_contrib": sz["V"] * sz["HW"],
                 "wcount": sz["V"] * sz["HW"]}[name]
        out = np.zeros((max(count, 1), width), dt)
        H.hgs_state_debug(self.rast.ctx, self.handle, what, out.ctypes.data, out.nbytes)
        out = out[:count]
        return out[:, 0] if width == 1 else out

    def check(self):
        """Synchronises and raises HGSError (ECAPACITY) if the render
        produced more pairs than its capacity (``hgs_state_check``)."""
        H.hgs_state_check(self.rast.ctx, self.handle)

    def free(self):
        if self.handle is not None:
            H.hgs_state_free(self.rast.ctx, self.handle)
            self.handle = None
            self.keep = ()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Rasterizer:
    """A library context bound to one CUDA (HIP) device."""

    def __init__(self, device: int | torch.device = 0):
        if isinstance(device, torch.device):
            device = device.index or 0
        self.device = int(device)
        self.ctx = H.hgs_create(self.device)

    def close(self):
        if self.ctx is not None:
            H.hgs_destroy(self.ctx)
            self.ctx = None

    def set_pair_capacity(self, max_pairs: int):
        """Fixed pair capacity of later renders (0: learned, the default)."""
        H.hgs_set_pair_capacity(self.ctx, max_pairs)

    # ----- scenes -----
    def scene_init(self, scene: dict, copy_resident: bool) -> int:
        return H.hgs_scene_init(self.ctx, scene_desc(scene), 1 if copy_resident else 0)

    def scene_release(self, sid: int):
        H.hgs_scene_release(self.ctx, sid)

    # ----- forward -----
    def alloc_images(self, n_views, height, width, channels=("rgb", "alpha", "depth", "normal")):
        dev = torch.device("cuda", self.device)
        nc = dict(rgb=3, alpha=1, depth=1, normal=3)
        return {k: torch.empty((n_views, nc[k], height, width), device=dev, dtype=torch.float32)
                for k in channels}

    def render_scene(self, sid: int, cams, opts=None, images=None, want_state=False, stream=None):
        cam_arr = make_cameras(cams)
        V = len(cam_arr)
        Hh, Ww = cam_arr[0].height, cam_arr[0].width
        if images is None:
            images = self.alloc_images(V, Hh, Ww)
        im = H.hgs_images()
        for k in ("rgb", "alpha", "depth", "normal"):
            t = images.get(k)
            if t is not None:
                nc = dict(rgb=3, alpha=1, depth=1, normal=3)[k]
                if tuple(t.shape) != (V, nc, Hh, Ww) or t.dtype != torch.float32 or not t.is_contiguous():
                    raise ValueError(f"image {k!r} must be float32 [{V},{nc},{Hh},{Ww}] contiguous")
            setattr(im, k, _ptr(t))
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        st = H.hgs_render(self.ctx, sid, cam_arr, make_opts(opts), im, want_state, s)
        return images, (State(self, st) if want_state else None)

    def render(self, scene: dict, cams, opts=None, images=None, want_state=False):
        """Forward render of a borrowed scene (tensors on this device)."""
        sid = self.scene_init(scene, copy_resident=False)
        try:
            images, state = self.render_scene(sid, cams, opts, images, want_state)
        finally:
            self.scene_release(sid)
        if state is not None:
            state.keep = tuple(scene[k] for k in SCENE_KEYS)
        return images, state

    # ----- backward -----
    def backward(self, state: State, grad_images: dict, grads: dict, accumulate=False, stream=None):
        gi = H.hgs_grad_images()
        for k in ("rgb", "alpha", "depth", "normal"):
            t = grad_images.get(k)
            if t is not None and not t.is_contiguous():
                raise ValueError(f"grad image {k!r} must be contiguous")
            setattr(gi, k, _ptr(t))
        g = H.hgs_grads()
        for k in ("means", "scales", "rotations", "opacities", "sh"):
            setattr(g, k, _ptr(grads.get(k)))
        g.accumulate = 1 if accumulate else 0
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        H.hgs_render_backward(self.ctx, state.handle, gi, g, s)

    def densify_stats(self, state: State, grad_norm=None, count=None, stream=None):
        """3DGS densification statistics of the last backward on `state`
        (``hgs_densify_stats``): adds into float32 [N] tensors."""
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        H.hgs_densify_stats(self.ctx, state.handle, _ptr(grad_norm), _ptr(count), s)

    def backward_fdo(self, state: State, grad_color: dict, grad_low_rgb, grad_high_rgb,
                     update: dict, sets=None, accumulate=False, n_conflict=None, stream=None):
        """Alg. 1's backward (``hgs_render_backward_fdo``): three cotangent
        sets in one traversal, projected per primitive into `update`.
        `sets`: None or a list of three gradient dicts that receive g_color,
        g_low and g_high before the projection."""
        gi = H.hgs_grad_images()
        for k in ("rgb", "alpha", "depth", "normal"):
            t = grad_color.get(k)
            if t is not None and not t.is_contiguous():
                raise ValueError(f"grad image {k!r} must be contiguous")
            setattr(gi, k, _ptr(t))
        for t in (grad_low_rgb, grad_high_rgb):
            if t is not None and not t.is_contiguous():
                raise ValueError("frequency cotangents must be contiguous")
        u = _grads(update, accumulate)
        arr = None
        if sets is not None:
            arr = (H.hgs_grads * 3)(*[_grads(d, False) for d in sets])
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        H.hgs_render_backward_fdo(self.ctx, state.handle, gi, _ptr(grad_low_rgb),
                                  _ptr(grad_high_rgb), u, arr, _ptr(n_conflict), s)


def _grads(d: dict, accumulate: bool) -> H.hgs_grads:
    g = H.hgs_grads()
    for k in ("means", "scales", "rotations", "opacities", "sh"):
        t = d.get(k)
        if t is not None and (not t.is_contiguous() or t.dtype != torch.float32):
            raise ValueError(f"gradient {k!r} must be contiguous float32")
        setattr(g, k, _ptr(t))
    g.accumulate = 1 if accumulate else 0
    return g


_RASTERIZERS: dict[int, Rasterizer] = {}


def get_rasterizer(device=0) -> Rasterizer:
    if isinstance(device, torch.device):
        device = device.index or 0
    r = _RASTERIZERS.get(int(device))
    if r is None:
        r = Rasterizer(int(device))
        _RASTERIZERS[int(device)] = r
    return r


class HybridRasterize(torch.autograd.Function):
    """Differentiable hybrid rendering: (means, scales, rotations, opacities,
    sh) -> (rgb, alpha, depth, normal), each [V,C,H,W].  ``types`` (uint8)
    and the cameras are not differentiated."""

    @staticmethod
    def forward(ctx, means, scales, rotations, opacities, sh, types, cams, opts):
        rast = get_rasterizer(means.device)
        scene = dict(means=means.contiguous(), scales=scales.contiguous(),
                     rotations=rotations.contiguous(), opacities=opacities.contiguous(),
                     sh=sh.contiguous(), types=types.contiguous())
        images, state = rast.render(scene, cams, opts, want_state=True)
        ctx.state = state
        ctx.shapes = [(t.shape, t.device) for t in (means, scales, rotations, opacities, sh)]
        return images["rgb"], images["alpha"], images["depth"], images["normal"]

    @staticmethod
    def backward(ctx, g_rgb, g_alpha, g_depth, g_normal):
        state = ctx.state
        rast = state.rast
        grads = {k: torch.empty(shp, device=dev, dtype=torch.float32)
                 for k, (shp, dev) in zip(("means", "scales", "rotations", "opacities", "sh"),
                                          ctx.shapes)}
        gi = {k: (None if t is None else t.contiguous())
              for k, t in (("rgb", g_rgb), ("alpha", g_alpha), ("depth", g_depth),
                           ("normal", g_normal))}
        rast.backward(state, gi, grads)
        state.free()
        return (grads["means"], grads["scales"], grads["rotations"], grads["opacities"],
                grads["sh"], None, None, None)


def rasterize(scene: dict, cams, opts=None):
    """Differentiable render; returns (rgb, alpha, depth, normal)."""
    return HybridRasterize.apply(scene["means"], scene["scales"], scene["rotations"],
                                 scene["opacities"], scene["sh"], scene["types"], cams, opts)


def to_device(scene_np: dict, device="cuda") -> dict:
    """numpy scene (scenegen layout) -> torch tensors on ``device``."""
    out = {}
    for k in SCENE_KEYS:
        out[k] = torch.from_numpy(np.ascontiguousarray(scene_np[k])).to(device)
    return out


def pair_counts(state: State) -> dict:
    """Algorithmic pair counts of a forward render, by type: blended pairs
    (backward work) and active pairs up to and including each pixel's stop
    (forward work)."""
    w = state.debug("wcount").astype(np.int64)
    b3 = int((w & 0x7FFF).sum())
    b2 = int(((w >> 15) & 0x7FFF).sum())
    stopped = (w >> 31) & 1
    s2 = int((stopped & ((w >> 30) & 1)).sum())
    s3 = int(stopped.sum()) - s2
    return dict(blend_3d=b3, blend_2d=b2, fwd_3d=b3 + s3, fwd_2d=b2 + s2)


def type_exchange(scales: torch.Tensor, rotations: torch.Tensor, types: torch.Tensor,
                  theta_e: float = 2.05, counts: torch.Tensor | None = None):
    """Adaptive Type Exchange in place (``hgs_type_exchange``): scales
    float32 [N,3], rotations float32 [N,4] (wxyz), types uint8 [N], all on
    one device.  ``counts`` (int32 [2] on that device) accumulates the number
    of 3D->2D and 2D->3D switches; returns it."""
    n = scales.shape[0]
    for t, shp, dt in ((scales, (n, 3), torch.float32), (rotations, (n, 4), torch.float32),
                       (types, (n,), torch.uint8)):
        if tuple(t.shape) != shp or t.dtype != dt or not t.is_contiguous():
            raise ValueError(f"expected {dt} {list(shp)} contiguous, got {t.dtype} {list(t.shape)}")
    if counts is None:
        counts = torch.zeros(2, dtype=torch.int32, device=scales.device)
    rast = get_rasterizer(scales.device)
    s = torch.cuda.current_stream(rast.device).cuda_stream
    H.hgs_type_exchange(rast.ctx, n, _ptr(scales), _ptr(rotations), _ptr(types), theta_e,
                        _ptr(counts), s)
    return counts


def fdo_cotangents(render_rgb: torch.Tensor, target_rgb: torch.Tensor, lambda_low: float = 0.2,
                   lambda_high: float = 0.4, losses: torch.Tensor | None = None,
                   grad_low: torch.Tensor | None = None, grad_high: torch.Tensor | None = None):
    """Frequency losses and weighted cotangents (``hgs_fdo_cotangents``).
    render_rgb, target_rgb: float32 [V, 3, H, W] on one device.  Returns
    (grad_low, grad_high, losses) with losses a float64 [2] device tensor
    (L_low, L_high) that the call adds into; grad_low / grad_high may be
    given (shaped like the images) to receive the cotangents."""
    if render_rgb.shape != target_rgb.shape or render_rgb.dim() != 4 or render_rgb.shape[1] != 3:
        raise ValueError("render_rgb and target_rgb must both be [V, 3, H, W]")
    for t in (render_rgb, target_rgb):
        if t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("images must be contiguous float32")
    V, _, Hh, Ww = render_rgb.shape
    g_low = torch.empty_like(render_rgb) if grad_low is None else grad_low
    g_high = torch.empty_like(render_rgb) if grad_high is None else grad_high
    for t in (g_low, g_high):
        if t.shape != render_rgb.shape or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("grad_low / grad_high must be contiguous float32 like the images")
    if losses is None:
        losses = torch.zeros(2, dtype=torch.float64, device=render_rgb.device)
    rast = get_rasterizer(render_rgb.device)
    s = torch.cuda.current_stream(rast.device).cuda_stream
    H.hgs_fdo_cotangents(rast.ctx, V, Hh, Ww, _ptr(render_rgb), _ptr(target_rgb), lambda_low,
                         lambda_high, _ptr(g_low), _ptr(g_high), _ptr(losses), s)
    return g_low, g_high, losses


def fdo_project(types: torch.Tensor, sh_degree: int, g_color: dict, g_low: dict, g_high: dict,
                update: dict | None = None, accumulate=False, n_conflict=None):
    """Alg. 1 on three parameter-gradient dicts (``hgs_fdo_project``); returns
    the update dict (allocated like g_color when not given)."""
    n = types.shape[0]
    if update is None:
        update = {k: torch.empty_like(v) for k, v in g_color.items()}
    rast = get_rasterizer(types.device)
    s = torch.cuda.current_stream(rast.device).cuda_stream
    H.hgs_fdo_project(rast.ctx, n, sh_degree, _ptr(types), _grads(g_color, False),
                      _grads(g_low, False), _grads(g_high, False), _grads(update, accumulate),
                      _ptr(n_conflict), s)
    return update


def color_loss(render_rgb: torch.Tensor, target_rgb: torch.Tensor, lambda_dssim: float = 0.2,
               losses: torch.Tensor | None = None, want_grad: bool = True,
               grad: torch.Tensor | None = None, noalloc: bool = False):
    """L_color = (1 - lambda) L1 + lambda D-SSIM (``hgs_color_loss``, or
    ``hgs_color_loss_noalloc`` with noalloc=True: no device allocation in
    the library).  Returns (grad or None, losses) with losses a float64 [2]
    device tensor (L1, D-SSIM) that the call adds into; `grad` may be given
    (same shape as the images) to receive the cotangent."""
    if render_rgb.shape != target_rgb.shape or render_rgb.dim() != 4 or render_rgb.shape[1] != 3:
        raise ValueError("render_rgb and target_rgb must both be [V, 3, H, W]")
    for t in (render_rgb, target_rgb):
        if t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("images must be contiguous float32")
    V, _, Hh, Ww = render_rgb.shape
    if grad is None and want_grad:
        grad = torch.empty_like(render_rgb)
    if grad is not None and (grad.shape != render_rgb.shape or grad.dtype != torch.float32 or
                             not grad.is_contiguous()):
        raise ValueError("grad must be a contiguous float32 tensor shaped like the images")
    if losses is None:
        losses = torch.zeros(2, dtype=torch.float64, device=render_rgb.device)
    rast = get_rasterizer(render_rgb.device)
    s = torch.cuda.current_stream(rast.device).cuda_stream
    fn = H.hgs_color_loss_noalloc if noalloc else H.hgs_color_loss
    fn(rast.ctx, V, Hh, Ww, _ptr(render_rgb), _ptr(target_rgb), lambda_dssim, _ptr(grad),
       _ptr(losses), s)
    return grad, losses


# 3DGS's default learning rates (the spatial scale of the means' rate and
# its decay are the caller's).
ADAM_DEFAULTS = dict(lr_means=1.6e-4, lr_scales=5e-3, lr_rotations=1e-3, lr_opacities=2.5e-2,
                     lr_sh_dc=2.5e-3, lr_sh_rest=2.5e-3 / 20, beta1=0.9, beta2=0.999, eps=1e-15)


def adam_step(n: int, sh_degree: int, raw: dict, grads: dict, exp_avg: dict, exp_avg_sq: dict,
              step: int, activated: dict | None = None, **lr):
    """One fused Adam step (``hgs_adam_step``) on raw parameter dicts."""
    o = H.hgs_adam_opts()
    for k, v in {**ADAM_DEFAULTS, **lr}.items():
        setattr(o, k, float(v))
    o.step = int(step)
    dev = raw["means"].device
    rast = get_rasterizer(dev)
    s = torch.cuda.current_stream(rast.device).cuda_stream
    H.hgs_adam_step(rast.ctx, n, sh_degree, _grads(raw, False), _grads(grads, False),
                    _grads(exp_avg, False), _grads(exp_avg_sq, False),
                    None if activated is None else _grads(activated, False), o, s)
