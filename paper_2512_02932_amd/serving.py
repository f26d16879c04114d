"""Batched serving over resident scenes (``hgs_server_*`` in include/hgs.h).

A :class:`Server` admits forward render requests into batches in flight
("lanes").  Each lane renders its requests in one pipeline pass, captured
once as a hipGraph, on its own stream.  This module only marshals arguments.
"""
from __future__ import annotations

import torch

from . import _hgs as H
from .rasterizer import Rasterizer, _ptr, make_camera, make_opts

CHANNELS = dict(rgb=3, alpha=1, depth=1, normal=3)


class Server:
    def __init__(self, rast: Rasterizer, *, max_requests=8, max_batches=2,
                 max_instances=8_000_000, max_pairs=64_000_000, max_tiles=65_536,
                 use_graph=True, opts=None):
        cfg = H.hgs_server_config(int(max_requests), int(max_batches), int(max_instances),
                                  int(max_pairs), int(max_tiles), 1 if use_graph else 0)
        self.rast = rast
        self.handle = H.hgs_server_create(rast.ctx, cfg, make_opts(opts))
        self._keep = {}  # tag -> images, alive until completion

    def close(self):
        if self.handle is not None:
            H.hgs_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc_images(self, height, width, channels=tuple(CHANNELS)):
        dev = torch.device("cuda", self.rast.device)
        return {k: torch.empty((1, CHANNELS[k], height, width), device=dev, dtype=torch.float32)
                for k in channels}

    def submit(self, scene_id: int, cam: dict, images: dict, tag: int):
        req = H.hgs_request()
        req.scene_id = int(scene_id)
        req.camera = make_camera(cam)
        for k in CHANNELS:
            t = images.get(k)
            if t is not None:
                shp = (1, CHANNELS[k], cam["height"], cam["width"])
                if tuple(t.shape) != shp or t.dtype != torch.float32 or not t.is_contiguous():
                    raise ValueError(f"image {k!r} must be float32 {list(shp)} contiguous")
            setattr(req.out, k, _ptr(t))
        req.tag = int(tag)
        H.hgs_server_submit(self.handle, req)
        self._keep[int(tag)] = images

    def poll(self, capacity=256):
        tags = H.hgs_server_poll(self.handle, capacity)
        for t in tags:
            self._keep.pop(t, None)
        return tags

    def stats(self):
        b, c, r, p, busy, mp = H.hgs_server_stats(self.handle)
        return dict(batches=b, completed=c, rerendered=r, pending=p, lanes_busy=busy,
                    max_pairs=mp)

    def drain(self, timeout_s=60.0):
        """Polls until nothing is pending or in flight; returns the tags."""
        import time
        done, t0 = [], time.perf_counter()
        while True:
            done += self.poll()
            st = self.stats()
            if st["pending"] == 0 and st["lanes_busy"] == 0:
                return done + self.poll()
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"server did not drain: {st}")
