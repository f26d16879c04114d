"""ctypes binding of ``libhgs.so`` (include/hgs.h).  Argument marshalling only.

The functions carry the C names (``hgs_create``, ``hgs_render`` ...).  Every
step of the render runs in the HIP library.  If the library is missing, the
load raises immediately; nothing falls back to another implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhgs.so")

HGS_OK, HGS_EINVAL, HGS_ENOMEM, HGS_EHIP, HGS_ECAPACITY, HGS_ESTATE = 0, -1, -2, -3, -4, -5

EXPORTS = ("hgs_create", "hgs_destroy", "hgs_scene_init", "hgs_scene_release", "hgs_render",
           "hgs_render_backward", "hgs_state_free", "hgs_state_sizes", "hgs_state_debug",
           "hgs_state_check", "hgs_last_error", "hgs_profile_enable", "hgs_profile_read",
           "hgs_server_create", "hgs_server_destroy", "hgs_server_submit", "hgs_server_poll",
           "hgs_server_stats", "hgs_type_exchange", "hgs_fdo_cotangents", "hgs_fdo_project",
           "hgs_render_backward_fdo", "hgs_color_loss", "hgs_adam_step", "hgs_densify_stats",
           "hgs_color_loss_noalloc", "hgs_set_pair_capacity")

STAGES = ("preprocess", "scan", "duplicate", "sort", "ranges", "raster_fwd", "raster_bwd",
          "preprocess_bwd", "fill", "depth_sort", "fdo_cotangents", "fdo_project", "color_loss",
          "adam", "densify", "fdo_preprocess_bwd")


class hgs_scene_desc(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32),
                ("means", C.c_void_p), ("scales", C.c_void_p), ("rotations", C.c_void_p),
                ("opacities", C.c_void_p), ("sh", C.c_void_p), ("types", C.c_void_p)]


class hgs_camera(C.Structure):
    _fields_ = [("viewmat", C.c_float * 16), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32),
                ("height", C.c_int32), ("znear", C.c_float)]


class hgs_opts(C.Structure):
    _fields_ = [("bg", C.c_float * 3), ("dilation", C.c_float), ("lambda_z", C.c_float),
                ("theta_z", C.c_float), ("temp_z", C.c_float), ("alpha_min", C.c_float),
                ("alpha_max", C.c_float), ("t_min", C.c_float), ("out_mask", C.c_uint32)]


OUT_RGB, OUT_ALPHA, OUT_DEPTH, OUT_NORMAL = 1, 2, 4, 8


class hgs_images(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("alpha", C.c_void_p), ("depth", C.c_void_p),
                ("normal", C.c_void_p)]


class hgs_grad_images(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("alpha", C.c_void_p), ("depth", C.c_void_p),
                ("normal", C.c_void_p)]


class hgs_adam_opts(C.Structure):
    _fields_ = [("lr_means", C.c_float), ("lr_scales", C.c_float), ("lr_rotations", C.c_float),
                ("lr_opacities", C.c_float), ("lr_sh_dc", C.c_float), ("lr_sh_rest", C.c_float),
                ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("step", C.c_int32)]


class hgs_grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("rotations", C.c_void_p),
                ("opacities", C.c_void_p), ("sh", C.c_void_p), ("accumulate", C.c_int32)]


class hgs_server_config(C.Structure):
    _fields_ = [("max_requests", C.c_int32), ("max_batches", C.c_int32),
                ("max_instances", C.c_int64), ("max_pairs", C.c_int64),
                ("max_tiles", C.c_int64), ("use_graph", C.c_int32)]


class hgs_request(C.Structure):
    _fields_ = [("scene_id", C.c_int32), ("camera", hgs_camera), ("out", hgs_images),
                ("tag", C.c_uint64)]


class HGSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hgs status {status}: {msg}")
        self.status = status


_lib = None


def load(path: str | None = None):
    """Load the HIP library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP runtime.  Load it first so that libhgs.so binds
    # to the runtime already in the process instead of bringing up a second
    # one (two HSA runtimes in one process cannot share the device).
    import torch  # noqa: F401
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built; run paper_2512_02932_amd.build.build() "
                           "(or __graft_entry__.build()) first")
    lib = C.CDLL(p)
    P = C.c_void_p
    lib.hgs_create.argtypes = [C.c_int32, C.POINTER(P)]
    lib.hgs_destroy.argtypes = [P]
    lib.hgs_destroy.restype = None
    lib.hgs_scene_init.argtypes = [P, C.POINTER(hgs_scene_desc), C.c_int32, C.POINTER(C.c_int32)]
    lib.hgs_scene_release.argtypes = [P, C.c_int32]
    lib.hgs_render.argtypes = [P, C.c_int32, C.POINTER(hgs_camera), C.c_int32,
                               C.POINTER(hgs_opts), C.POINTER(hgs_images), C.POINTER(P), P]
    lib.hgs_render_backward.argtypes = [P, P, C.POINTER(hgs_grad_images), C.POINTER(hgs_grads), P]
    lib.hgs_state_free.argtypes = [P, P]
    lib.hgs_state_free.restype = None
    lib.hgs_state_sizes.argtypes = [P, P, C.POINTER(C.c_int64)]
    lib.hgs_state_debug.argtypes = [P, P, C.c_int32, P, C.c_int64]
    lib.hgs_state_check.argtypes = [P, P]
    lib.hgs_profile_enable.argtypes = [P, C.c_int32]
    lib.hgs_profile_read.argtypes = [P, P, P, C.c_int32]
    lib.hgs_last_error.argtypes = []
    lib.hgs_last_error.restype = C.c_char_p
    lib.hgs_server_create.argtypes = [P, C.POINTER(hgs_server_config), C.POINTER(hgs_opts),
                                      C.POINTER(P)]
    lib.hgs_server_destroy.argtypes = [P]
    lib.hgs_server_destroy.restype = None
    lib.hgs_server_submit.argtypes = [P, C.POINTER(hgs_request)]
    lib.hgs_server_poll.argtypes = [P, C.POINTER(C.c_uint64), C.c_int32, C.POINTER(C.c_int32)]
    lib.hgs_server_stats.argtypes = [P, C.POINTER(C.c_int64)]
    lib.hgs_type_exchange.argtypes = [P, C.c_int64, P, P, P, C.c_double, P, P]
    lib.hgs_fdo_cotangents.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, P, C.c_double,
                                       C.c_double, P, P, P, P]
    lib.hgs_fdo_project.argtypes = [P, C.c_int64, C.c_int32, P, C.POINTER(hgs_grads),
                                    C.POINTER(hgs_grads), C.POINTER(hgs_grads),
                                    C.POINTER(hgs_grads), P, P]
    lib.hgs_render_backward_fdo.argtypes = [P, P, C.POINTER(hgs_grad_images), P, P,
                                            C.POINTER(hgs_grads), P, P, P]
    lib.hgs_densify_stats.argtypes = [P, P, P, P, P]
    lib.hgs_color_loss.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, P, C.c_double, P, P, P]
    lib.hgs_color_loss_noalloc.argtypes = lib.hgs_color_loss.argtypes
    lib.hgs_set_pair_capacity.argtypes = [P, C.c_int64]
    lib.hgs_adam_step.argtypes = [P, C.c_int64, C.c_int32] + [C.POINTER(hgs_grads)] * 4 + \
        [P, C.POINTER(hgs_adam_opts), P]
    for name in ("hgs_create", "hgs_scene_init", "hgs_scene_release", "hgs_render",
                 "hgs_render_backward", "hgs_state_sizes", "hgs_state_debug", "hgs_state_check",
                 "hgs_profile_enable", "hgs_profile_read", "hgs_server_create",
                 "hgs_server_submit", "hgs_server_poll", "hgs_server_stats",
                 "hgs_type_exchange", "hgs_fdo_cotangents", "hgs_fdo_project",
                 "hgs_render_backward_fdo", "hgs_color_loss", "hgs_adam_step", "hgs_densify_stats",
                 "hgs_color_loss_noalloc", "hgs_set_pair_capacity"):
        getattr(lib, name).restype = C.c_int32
    _lib = lib
    return lib


def check(status: int):
    if status != HGS_OK:
        msg = _lib.hgs_last_error().decode() if _lib is not None else ""
        raise HGSError(status, msg)


# --- thin wrappers with the C names -----------------------------------------
def hgs_create(device: int = 0):
    lib = load()
    h = C.c_void_p()
    check(lib.hgs_create(int(device), C.byref(h)))
    return h


def hgs_destroy(ctx):
    load().hgs_destroy(ctx)


def hgs_scene_init(ctx, desc: hgs_scene_desc, copy_resident: int) -> int:
    sid = C.c_int32()
    check(load().hgs_scene_init(ctx, C.byref(desc), int(copy_resident), C.byref(sid)))
    return sid.value


def hgs_scene_release(ctx, scene_id: int):
    check(load().hgs_scene_release(ctx, int(scene_id)))


def hgs_render(ctx, scene_id, cams, opts, images, want_state: bool, stream: int):
    """cams: ctypes array of hgs_camera; returns a state handle or None."""
    st = C.c_void_p()
    check(load().hgs_render(ctx, int(scene_id), cams, len(cams),
                            C.byref(opts) if opts is not None else None, C.byref(images),
                            C.byref(st) if want_state else None, C.c_void_p(stream)))
    return st if want_state else None


def hgs_render_backward(ctx, state, grad_images, grads, stream: int):
    check(load().hgs_render_backward(ctx, state, C.byref(grad_images), C.byref(grads),
                                     C.c_void_p(stream)))


def hgs_state_free(ctx, state):
    load().hgs_state_free(ctx, state)


def hgs_state_sizes(ctx, state):
    arr = (C.c_int64 * 5)()
    check(load().hgs_state_sizes(ctx, state, arr))
    return list(arr)


def hgs_state_debug(ctx, state, what: int, dst_ptr: int, capacity: int):
    check(load().hgs_state_debug(ctx, state, int(what), C.c_void_p(dst_ptr), int(capacity)))


def hgs_state_check(ctx, state):
    check(load().hgs_state_check(ctx, state))


def hgs_set_pair_capacity(ctx, max_pairs: int):
    check(load().hgs_set_pair_capacity(ctx, int(max_pairs)))


PROFILE_STAGES, PROFILE_WORK = 1, 2  # HGS_PROFILE_STAGES, HGS_PROFILE_WORK


def hgs_profile_enable(ctx, on):
    """on: False / 0 (off), True (stage events), or a set of PROFILE_* flags."""
    check(load().hgs_profile_enable(ctx, int(on)))


def hgs_profile_read(ctx, reset: bool = False):
    """Returns {stage: (total_ms, launches)}."""
    ms = (C.c_double * len(STAGES))()
    calls = (C.c_int64 * len(STAGES))()
    check(load().hgs_profile_read(ctx, ms, calls, 1 if reset else 0))
    return {name: (ms[i], calls[i]) for i, name in enumerate(STAGES)}


def hgs_server_create(ctx, cfg: hgs_server_config, opts=None):
    srv = C.c_void_p()
    check(load().hgs_server_create(ctx, C.byref(cfg), C.byref(opts) if opts is not None else None,
                                   C.byref(srv)))
    return srv


def hgs_server_destroy(srv):
    load().hgs_server_destroy(srv)


def hgs_server_submit(srv, req: hgs_request):
    check(load().hgs_server_submit(srv, C.byref(req)))


def hgs_server_poll(srv, capacity: int = 256):
    """Returns the list of completed tags."""
    tags = (C.c_uint64 * max(capacity, 1))()
    n = C.c_int32()
    check(load().hgs_server_poll(srv, tags, int(capacity), C.byref(n)))
    return [int(tags[i]) for i in range(n.value)]


def hgs_server_stats(srv):
    """(batches, completed, rerendered, pending, lanes_busy, max_pairs)."""
    st = (C.c_int64 * 6)()
    check(load().hgs_server_stats(srv, st))
    return tuple(int(x) for x in st)


def hgs_type_exchange(ctx, n: int, scales_ptr: int, rots_ptr: int, types_ptr: int, theta: float,
                      counts_ptr: int, stream: int):
    check(load().hgs_type_exchange(ctx, int(n), C.c_void_p(scales_ptr), C.c_void_p(rots_ptr),
                                   C.c_void_p(types_ptr), float(theta), C.c_void_p(counts_ptr),
                                   C.c_void_p(stream)))


def hgs_fdo_cotangents(ctx, V: int, H: int, W: int, ren_ptr: int, tgt_ptr: int, lambda_low: float,
                       lambda_high: float, glow_ptr: int, ghigh_ptr: int, losses_ptr: int,
                       stream: int):
    check(load().hgs_fdo_cotangents(ctx, int(V), int(H), int(W), C.c_void_p(ren_ptr),
                                    C.c_void_p(tgt_ptr), float(lambda_low), float(lambda_high),
                                    C.c_void_p(glow_ptr), C.c_void_p(ghigh_ptr),
                                    C.c_void_p(losses_ptr), C.c_void_p(stream)))


def hgs_fdo_project(ctx, n: int, sh_degree: int, types_ptr: int, gc, gl, gh, update,
                    conflict_ptr: int, stream: int):
    check(load().hgs_fdo_project(ctx, int(n), int(sh_degree), C.c_void_p(types_ptr), C.byref(gc),
                                 C.byref(gl), C.byref(gh), C.byref(update),
                                 C.c_void_p(conflict_ptr), C.c_void_p(stream)))


def hgs_render_backward_fdo(ctx, state, grad_images, glow_ptr: int, ghigh_ptr: int, update, sets,
                            conflict_ptr: int, stream: int):
    """`sets` is None or a ctypes array of three hgs_grads."""
    check(load().hgs_render_backward_fdo(ctx, state, C.byref(grad_images), C.c_void_p(glow_ptr),
                                         C.c_void_p(ghigh_ptr), C.byref(update),
                                         None if sets is None else C.cast(sets, C.c_void_p),
                                         C.c_void_p(conflict_ptr), C.c_void_p(stream)))


def hgs_color_loss(ctx, V: int, H: int, W: int, ren_ptr: int, tgt_ptr: int, lam: float,
                   grad_ptr: int, losses_ptr: int, stream: int):
    check(load().hgs_color_loss(ctx, int(V), int(H), int(W), C.c_void_p(ren_ptr),
                                C.c_void_p(tgt_ptr), float(lam), C.c_void_p(grad_ptr),
                                C.c_void_p(losses_ptr), C.c_void_p(stream)))


def hgs_color_loss_noalloc(ctx, V: int, H: int, W: int, ren_ptr: int, tgt_ptr: int, lam: float,
                           grad_ptr: int, losses_ptr: int, stream: int):
    check(load().hgs_color_loss_noalloc(ctx, int(V), int(H), int(W), C.c_void_p(ren_ptr),
                                        C.c_void_p(tgt_ptr), float(lam), C.c_void_p(grad_ptr),
                                        C.c_void_p(losses_ptr), C.c_void_p(stream)))


NOALLOC_MAX_ELEMS = 8388608  # HGS_NOALLOC_MAX_ELEMS


def hgs_adam_step(ctx, n: int, sh_degree: int, raw, grads, m, v, act, opts, stream: int):
    """`act` may be None."""
    check(load().hgs_adam_step(ctx, int(n), int(sh_degree), C.byref(raw), C.byref(grads),
                               C.byref(m), C.byref(v),
                               None if act is None else C.cast(C.pointer(act), C.c_void_p),
                               C.byref(opts), C.c_void_p(stream)))


def hgs_densify_stats(ctx, state, norm_ptr: int, count_ptr: int, stream: int):
    check(load().hgs_densify_stats(ctx, state, C.c_void_p(norm_ptr), C.c_void_p(count_ptr),
                                   C.c_void_p(stream)))
