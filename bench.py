#!/usr/bin/env python
"""Benchmark of the hybrid 2D/3D rasterizer on one MI355X.

Headline metric: training-step throughput, forward + backward, in
Mpixels/s, on 1M hybrid Gaussians (50/50 surfels / 3D Gaussians on a noisy
(2,3) torus knot, SH degree 3) rendered at 1920x1080, with N(0,1)
cotangents on every output channel.  A step is one pass of the whole
rendering hot path:
  preprocess, scan, duplicate, radix sort, ranges, raster forward,
  raster backward, preprocess backward.
Inputs are resident in HBM before timing starts.

Prints ONE JSON line (rank 0).  It carries a `roofline` object for the
dominant kernel and a `cpu_baseline` object for the CPU oracle, timed on a
bounded band of image rows.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Per-pair VALU lane-operations of the minimal formulas (a transcendental
# counts as 4 issue slots), used for the raster kernels' ALU roofline.  The
# pinned counts are those of the binary32 formulas the kernels evaluate
# (record-local frame); the survey counts are the plan's estimates (forward
# 27 / 45, backward about three times the forward), reported beside them.
OPS_FWD = {"3d": 27, "2d": 34}
OPS_BWD = {"3d": 71, "2d": 82}
OPS_FWD_SURVEY = {"3d": 27, "2d": 45}
OPS_BWD_SURVEY = {"3d": 81, "2d": 135}
# Each RGB-only cotangent set of the three-set backward adds per blended pair
# its colour dot product, suffix and dL/d alpha~ (6), colour and alpha_eff
# slots (6), the record-geometry chain (12 for 3D, 15 for 2D) and its
# accumulating adds (9 for 3D, 13 for 2D).
OPS_BWD_RGB = {"3d": 33, "2d": 40}
# VALU issue peak with packed FP32 disabled: 256 CU x 64 lanes x 2.4 GHz.
VALU_PEAK = 256 * 64 * 2.4e9
HBM_PEAK = 8.0e12

# name: (scene builder, camera builder, backward?, description)
WORKLOADS = {
    "knot1m_1080p": ("scene_torus_knot", "camera_torus_knot_1080p", True,
                     "torus-knot 1M hybrid Gaussians (50% surfels), SH3, 1920x1080, fwd+bwd"),
    "knot1m_1600x1064": ("scene_torus_knot", "camera_torus_knot", True,
                         "torus-knot 1M hybrid Gaussians (50% surfels), SH3, 1600x1064, fwd+bwd"),
    "cube10k_256": ("scene_uniform_cube", "camera_cube", False,
                    "uniform cube 10k Gaussians (5k surfels), SH0, 256x256, forward"),
    "sphere500k_1080p": ("scene_sphere", "camera_sphere", False,
                         "noisy sphere 500k Gaussians (70% surfels), SH3, 1920x1080, forward"),
    "multishell6m_16x4k": ("scene_multishell", "fibonacci_cameras", True,
                           "multi-shell 6M Gaussians (60% surfels), SH3, 16 views of 3840x2160 "
                           "in one launch, fwd+bwd"),
}
# the per-config legs of the default run (the headline is knot1m_1080p)
CONFIG_LEGS = ("cube10k_256", "sphere500k_1080p", "knot1m_1600x1064", "multishell6m_16x4k")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _cpu_info():
    """CPU model, logical CPUs of the host and CPUs this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def cpu_baseline(scene_np, cam, G_np, rows_all: int = 160, rows_one: int = 12, repeats: int = 3):
    """The CPU oracle (binary64, as it stands) on bands of image rows through
    the centre of the image, forward + backward: median of `repeats` runs
    with every core this job may use (at most 16, the host share of one GPU)
    on `rows_all` rows, and median of `repeats` runs on one thread on
    `rows_one` rows."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    H, W = cam["height"], cam["width"]
    model, n_host, usable = _cpu_info()
    cores = max(1, min(usable, 16))

    def band(rows):
        y0 = H // 2 - rows // 2
        ys = np.arange(y0, y0 + rows)
        pix = np.stack(np.meshgrid([0], ys, np.arange(W), indexing="ij"), -1).reshape(-1, 3)
        pix = np.ascontiguousarray(pix, np.int32)
        v, y, x = pix[:, 0], pix[:, 1], pix[:, 2]
        Gp = np.stack([G_np["rgb"][v, 0, y, x], G_np["rgb"][v, 1, y, x], G_np["rgb"][v, 2, y, x],
                       G_np["alpha"][v, 0, y, x], G_np["depth"][v, 0, y, x],
                       G_np["normal"][v, 0, y, x], G_np["normal"][v, 1, y, x],
                       G_np["normal"][v, 2, y, x]], 1).astype(np.float64)
        return pix, Gp, y0

    def run(rows, threads):
        pix, Gp, y0 = band(rows)
        times = []
        for _ in range(repeats):
            t0 = time.perf_counter()
            oracle.forward(scene_np, cam, pix, threads=threads)
            oracle.backward(scene_np, cam, pix, Gp, threads=threads)
            times.append(time.perf_counter() - t0)
        dt = float(np.median(times))
        return dict(value=round(len(pix) / dt / 1e6, 6), unit="Mpixels/s", threads=threads,
                    sample=f"rows {y0}..{y0 + rows - 1} of {W}x{H} ({len(pix)} px)",
                    seconds=[round(t, 2) for t in times])

    all_c = run(rows_all, cores)
    one = run(rows_one, 1)
    return {"value": all_c["value"], "unit": "Mpixels/s", "cores": cores, "kind": "oracle",
            "sample": f"{all_c['sample']}, forward+backward, binary64, {cores} threads, median of "
                      f"{repeats} ({all_c['seconds']} s)",
            "single_thread": one, "cpu_model": model, "host_logical_cpus": n_host,
            "cpus_usable": usable}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/traffic_<workload>.md), or None if there is none or the
    kernel's source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    if "```json" not in txt:
        return None
    blob = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
    ent = blob.get(kernel)
    if ent is None:
        return None
    src = os.path.join(ROOT, ent["source"])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    return int(ent["bytes"]) if sha == ent["sha256_16"] else None


def _pool_get(pool, srv_or_rast, H, W):
    free = pool.setdefault((H, W), [])
    if free:
        return free.pop()
    return srv_or_rast.alloc_images(1, H, W) if hasattr(srv_or_rast, "ctx") else \
        srv_or_rast.alloc_images(H, W)


def serving(rast, n_warm=200, n_meas=2000, rates=(200.0, 800.0), check=20):
    """Served-view latency on four resident scenes with Poisson arrivals, at
    a light and a heavy load.  At each rate the same request trace is
    replayed (a) through the batched server (one graph-captured pass per
    batch, batches in flight on several streams) and (b) as one plain render
    launch per request.  Latency = completion - arrival, over the measured
    requests."""
    import numpy as np
    import torch
    import scenegen as sg
    from paper_2512_02932_amd.rasterizer import to_device
    from paper_2512_02932_amd.serving import Server

    log("[serving] generating 4 resident scenes")
    scenes = sg.serving_scenes()
    sids = [rast.scene_init(to_device(sc), copy_resident=True) for sc in scenes]
    n_gauss = [int(sc["means"].shape[0]) for sc in scenes]
    del scenes
    results = {}
    for rate in rates:
        results[rate] = _serve_rate(rast, sids, n_warm, n_meas, rate, check)
    for sid in sids:
        rast.scene_release(sid)
    base = results[rates[0]]
    out = {"workload": f"4 resident scenes ({'/'.join(str(n) for n in n_gauss)} Gaussians, SH3), "
                       f"Poisson arrivals, {n_warm} warm-up + {n_meas} measured requests per rate, "
                       "resolutions 256^2/512^2/1280x720/1920x1080, orbit r in [3,5]",
           "rate_req_per_s": rates[0], **base}
    for rate in rates[1:]:
        out[f"at_{int(rate)}_req_per_s"] = results[rate]
    return out


def _serve_rate(rast, sids, n_warm, n_meas, rate, check):
    import numpy as np
    import torch
    import scenegen as sg
    from paper_2512_02932_amd.serving import Server
    reqs = sg.serving_requests(n_warm + n_meas, rate=rate, seed=45)
    px = np.array([r["camera"]["width"] * r["camera"]["height"] for r in reqs], np.float64)
    torch.cuda.synchronize()
    check_ids = set(range(n_warm, n_warm + n_meas, max(1, n_meas // check)))

    def run(batched):
        pool, kept = {}, {}
        lat = np.zeros(len(reqs))
        out_imgs = {}
        srv = None
        if batched:
            srv = Server(rast, max_requests=8, max_batches=3, max_instances=12_000_000,
                         max_pairs=96_000_000, max_tiles=8 * 8160, use_graph=True)
        stream = torch.cuda.current_stream()
        t0 = time.perf_counter()
        i = done = 0
        while done < len(reqs):
            now = time.perf_counter() - t0
            while i < len(reqs) and reqs[i]["t"] <= now:
                cam = reqs[i]["camera"]
                im = _pool_get(pool, srv if batched else rast, cam["height"], cam["width"])
                if batched:
                    srv.submit(sids[reqs[i]["scene"]], cam, im, i)
                    kept[i] = im
                else:
                    rast.render_scene(sids[reqs[i]["scene"]], cam, images=im)
                    stream.synchronize()
                    lat[i] = time.perf_counter() - t0 - reqs[i]["t"]
                    if i in check_ids:
                        out_imgs[i] = im["rgb"].clone()
                    pool[(cam["height"], cam["width"])].append(im)
                    done += 1
                i += 1
            if batched:
                for tag in srv.poll():
                    lat[tag] = time.perf_counter() - t0 - reqs[tag]["t"]
                    im = kept.pop(tag)
                    if tag in check_ids:
                        out_imgs[tag] = im["rgb"].clone()
                    cam = reqs[tag]["camera"]
                    pool[(cam["height"], cam["width"])].append(im)
                    done += 1
        t_end = time.perf_counter() - t0
        st = srv.stats() if batched else None
        if srv is not None:
            srv.close()
        m = lat[n_warm:]
        span = t_end - reqs[n_warm]["t"]
        res = {"p50_ms": round(float(np.percentile(m, 50)) * 1e3, 3),
               "p99_ms": round(float(np.percentile(m, 99)) * 1e3, 3),
               "mean_ms": round(float(m.mean()) * 1e3, 3),
               "req_per_s": round(n_meas / span, 1),
               "mpix_per_s": round(float(px[n_warm:].sum()) / span / 1e6, 1)}
        if st is not None:
            res["batches"] = st["batches"]
            res["rerendered"] = st["rerendered"]
        return res, out_imgs

    log(f"[serving] {rate:g} req/s: batched graph server")
    b, b_imgs = run(True)
    log(f"[serving] batched {b}")
    log(f"[serving] {rate:g} req/s: one launch per request")
    p, p_imgs = run(False)
    log(f"[serving] per-request {p}")
    diff = max(float((b_imgs[k] - p_imgs[k]).abs().max()) for k in b_imgs)
    return {"batched_graph": b, "one_launch_per_request": p, "max_abs_diff_batched_vs_plain": diff}

def time_steps(rast, step, steps, prof_steps=5):
    """Whole-step time of `steps` steps with stage profiling off, then the
    per-launch stage times (HIP events on the launch stream) from
    `prof_steps` further steps with it on, so the events are not part of
    the timed work.  Returns (ms per step, {stage: ms per launch})."""
    import torch
    from paper_2512_02932_amd import _hgs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _hgs.hgs_profile_enable(rast.ctx, True)
    _hgs.hgs_profile_read(rast.ctx, reset=True)
    for _ in range(prof_steps):
        step()
    torch.cuda.synchronize()
    prof = _hgs.hgs_profile_read(rast.ctx, reset=True)
    _hgs.hgs_profile_enable(rast.ctx, False)
    stage = {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1] > 0}
    return (t1 - t0) * 1e3 / steps, stage


def stage_roofline(N, K, V, D, P, T_tot, counts, stage_ms, ms_step, backward):
    """Per-stage algorithmic bytes and VALU lane-ops of one step (the
    accounting of the method's work, not of this implementation's), the
    least time each needs at the chip's peaks, and the fractions
        f_s = max(B_s / BW, Ops_s / VALU) / T_s,
        f   = sum_s max(B_s / BW, Ops_s / VALU) / T_step.
    The sort is charged its single-pass lower bound, 24 bytes per pair."""
    fwd = counts["fwd_3d"] * OPS_FWD["3d"] + counts["fwd_2d"] * OPS_FWD["2d"]
    bwd = counts["blend_3d"] * OPS_BWD["3d"] + counts["blend_2d"] * OPS_BWD["2d"]
    model = {
        "preprocess": (("preprocess",), N * (45 + 12 * K) + V * N * (72 + 4 + 4 + 8),
                       V * N * (250 + 6 * K)),
        "scan": (("scan",), 8 * V * N, 0),
        "duplicate": (("duplicate",), 16 * V * N + 12 * D, 0),
        "sort": (("depth_sort", "sort"), 24 * D, 0),
        "ranges": (("ranges",), 8 * D + 8 * T_tot, 0),
        "raster_fwd": (("raster_fwd",), 72 * D + 44 * P, fwd),
    }
    if backward:
        model["raster_bwd"] = (("fill", "raster_bwd"), 72 * D + 44 * P + 64 * D, bwd)
        model["preprocess_bwd"] = (("preprocess_bwd",), V * N * (72 + 64) + 2 * N * (45 + 12 * K),
                                   V * N * (600 + 6 * K))
    out, least = {}, 0.0
    for name, (keys, byt, ops) in model.items():
        t = sum(stage_ms.get(k, 0.0) for k in keys)
        tb, to = byt / HBM_PEAK * 1e3, ops / VALU_PEAK * 1e3
        tmin = max(tb, to)
        least += tmin
        out[name] = {"ms": round(t, 4), "bytes": int(byt), "ops": int(ops),
                     "bound": "hbm" if tb >= to else "alu",
                     "frac": round(tmin / t, 4) if t > 0 else None}
    return {"stages": out, "combined_frac": round(least / ms_step, 4),
            "least_ms": round(least, 4), "peaks": {"hbm_GBps": HBM_PEAK / 1e9,
                                                   "valu_Tops": round(VALU_PEAK / 1e12, 4)},
            "note": "f = sum over stages of max(bytes / HBM peak, VALU lane-ops / VALU peak), "
                    "divided by the measured step time"}


def dominant_roofline(stage_ms, counts, N, K, V, workload):
    """The roofline object of the longest kernel among raster forward,
    raster backward, preprocess and preprocess backward."""
    cands = [k for k in ("raster_fwd", "raster_bwd", "preprocess", "preprocess_bwd")
             if k in stage_ms]
    dom = max(cands, key=lambda k: stage_ms[k])
    if dom in ("raster_fwd", "raster_bwd"):
        kname = "raster_fwd_kernel<false>" if dom == "raster_fwd" else "raster_bwd_kernel<1>"
        ops, ops_s = (OPS_FWD, OPS_FWD_SURVEY) if dom == "raster_fwd" else (OPS_BWD, OPS_BWD_SURVEY)
        key = "fwd" if dom == "raster_fwd" else "blend"
        work = counts[f"{key}_3d"] * ops["3d"] + counts[f"{key}_2d"] * ops["2d"]
        work_s = counts[f"{key}_3d"] * ops_s["3d"] + counts[f"{key}_2d"] * ops_s["2d"]
        achieved = work / (stage_ms[dom] * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(achieved, 4), "peak": round(VALU_PEAK / 1e12, 4),
                "unit": "Tops/s", "frac": round(achieved / (VALU_PEAK / 1e12), 4),
                "traffic": measured_traffic(kname, workload), "kernel": kname,
                "ops_per_pair": ops, "pairs": {k: counts[f"{key}_{k}"] for k in ("3d", "2d")},
                "frac_survey_ops": round(work_s / (stage_ms[dom] * 1e-3) / VALU_PEAK, 4),
                "launch_ms": round(stage_ms[dom], 4)}
    byt = (N * (45 + 12 * K) + V * N * 88) if dom == "preprocess" else \
        (V * N * 136 + 2 * N * (45 + 12 * K))
    achieved = byt / (stage_ms[dom] * 1e-3) / 1e9
    kname = f"{dom}_kernel<{DEG_OF_K[K]}>"
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK / 1e9,
            "unit": "GB/s", "frac": round(achieved / (HBM_PEAK / 1e9), 4),
            "traffic": measured_traffic(kname, workload), "kernel": kname,
            "launch_ms": round(stage_ms[dom], 4)}


def render_leg(rast, name, steps, warmup):
    """One workload: `steps` timed steps (render, and for the backward
    workloads render_backward with N(0,1) cotangents on every channel), with
    the inputs resident in HBM.  Returns the leg's record and the objects
    the headline's further legs reuse."""
    import torch
    import scenegen as sg
    from paper_2512_02932_amd.rasterizer import pair_counts, to_device
    scene_fn, cam_fn, backward, desc = WORKLOADS[name]
    log(f"[{name}] generating")
    scene_np = getattr(sg, scene_fn)()
    cams = getattr(sg, cam_fn)()
    cam_list = cams if isinstance(cams, list) else [cams]
    V = len(cam_list)
    H, W = cam_list[0]["height"], cam_list[0]["width"]
    sc = to_device(scene_np, "cuda")
    N = int(scene_np["means"].shape[0])
    K = int(scene_np["sh"].shape[1])
    G_np = G = grads = None
    if backward:
        G_np = sg.upstream_grads(V, H, W, seed=3)
        G = {k: torch.from_numpy(v).cuda() for k, v in G_np.items()}
        grads = {k: torch.empty_like(sc[k]) for k in ("means", "scales", "rotations", "opacities", "sh")}
    images = rast.alloc_images(V, H, W)
    torch.cuda.synchronize()

    def step():
        _, state = rast.render(sc, cams, images=images, want_state=backward)
        if backward:
            rast.backward(state, G, grads)
            state.free()

    log(f"[{name}] warmup {warmup}")
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # work accounting of this workload (identical every step), and a check
    # that the pairs fit the render's capacity
    from paper_2512_02932_amd import _hgs
    # the forward records its pair counts (work accounting)
    _hgs.hgs_profile_enable(rast.ctx, _hgs.PROFILE_STAGES | _hgs.PROFILE_WORK)
    _, st = rast.render(sc, cams, images=images, want_state=True)
    _hgs.hgs_profile_enable(rast.ctx, False)
    _hgs.hgs_profile_read(rast.ctx, reset=True)
    st.check()
    counts = pair_counts(st)
    sizes = st.sizes()
    st.free()
    torch.cuda.synchronize()
    log(f"[{name}] timing {steps} steps")
    ms, stage_ms = time_steps(rast, step, steps)
    P = V * H * W
    T_tot = int(sizes["n_tiles"])
    D = int(sizes["D"])
    rec = {"workload": desc, "gaussians": N, "views": V, "width": W, "height": H,
           "sh_degree": int(round(K ** 0.5)) - 1, "backward": backward, "steps": steps,
           "ms_per_step": round(ms, 4), "mpix_per_s": round(P / (ms * 1e-3) / 1e6, 3),
           "pairs_D": D, "tiles": T_tot, "pair_counts": counts,
           "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
           "stage_roofline": stage_roofline(N, K, V, D, P, T_tot, counts, stage_ms, ms, backward),
           "roofline": dominant_roofline(stage_ms, counts, N, K, V, name)}
    log(f"[{name}] {rec['mpix_per_s']} Mpix/s, {rec['ms_per_step']} ms/step, "
        f"combined f {rec['stage_roofline']['combined_frac']}")
    keep = dict(scene_np=scene_np, cam=cams, sc=sc, G=G, G_np=G_np, images=images, grads=grads,
                counts=counts)
    return rec, keep


def exchange_leg(scene_np, workload, copies=8, replays=5):
    """Adaptive Type Exchange, timed alone on the knot scene's own
    parameters and on a 16M-primitive set of the same scale distribution.
    `copies` launches, each on its own copy of the parameters, are captured
    in one graph (no host launch cost between them).  Two passes: "fresh"
    restores the untouched parameters before each replay (9% switch, 6% are
    reparameterised), "steady" replays on already exchanged parameters
    (nothing switches: the state between exchanges in training).  A 1 GiB
    read-write before each timed replay evicts the restore's dirty lines.
    Algorithmic bytes: 13 read per primitive (scales, type), plus 1 written
    per switch, plus 44 more (rotation read and written, scales written) per
    reparameterised one."""
    import numpy as np
    import torch
    from paper_2512_02932_amd import _hgs
    from paper_2512_02932_amd.rasterizer import get_rasterizer
    rast = get_rasterizer(0)
    res = {}
    sets = {"knot1m": (scene_np["scales"], scene_np["rotations"], scene_np["types"])}
    sets["16m"] = tuple(np.concatenate([a] * 16) for a in sets["knot1m"])
    flush = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
    for name, (s, q, t) in sets.items():
        S0, Q0, T0 = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (s, q, t))
        n = S0.shape[0]
        bufs = [(S0.clone(), Q0.clone(), T0.clone()) for _ in range(copies)]
        counts = torch.zeros((copies, 2), dtype=torch.int32, device="cuda")

        def launch_all():
            st = torch.cuda.current_stream().cuda_stream
            for j, (S, Q, T) in enumerate(bufs):
                _hgs.hgs_type_exchange(rast.ctx, n, S.data_ptr(), Q.data_ptr(), T.data_ptr(), 2.05,
                                       counts[j].data_ptr(), st)

        def restore():
            for S, Q, T in bufs:
                S.copy_(S0); Q.copy_(Q0); T.copy_(T0)
            counts.zero_()

        restore()
        launch_all()  # eager
        torch.cuda.synchronize()
        eager = bufs[0][0].clone()
        sw = int(counts[0].sum())
        moved = int(((bufs[0][0] != S0).any(1) | (bufs[0][1] != Q0).any(1)).sum())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            launch_all()

        def timed(fresh):
            tot = 0.0
            for _ in range(replays):
                if fresh:
                    restore()
                else:
                    counts.zero_()
                flush.add_(1.0)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                g.replay()
                e1.record()
                e1.synchronize()
                tot += e0.elapsed_time(e1)
                assert torch.equal(bufs[0][0], eager)
                assert int(counts[copies - 1].sum()) == (sw if fresh else 0)
            return tot / (replays * copies)

        res[name] = {"n": n, "switched": sw, "reparameterised": moved}
        for kind, byt in (("fresh", 13 * n + sw + 44 * moved), ("steady", 13 * n)):
            ms = timed(kind == "fresh")
            gbs = byt / (ms * 1e-3) / 1e9
            res[name][kind] = {"ms": round(ms, 5),
                               "roofline": {"bound": "hbm", "achieved": round(gbs, 1),
                                            "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                                            "frac": round(gbs / (HBM_PEAK / 1e9), 4),
                                            "traffic": measured_traffic(
                                                f"type_exchange_kernel<true>/{name}/{kind}", workload),
                                            "kernel": "type_exchange_kernel<true>"}}
        log(f"[exchange] {name}: {res[name]}")
        del g, bufs, S0, Q0, T0, eager
    del flush
    torch.cuda.empty_cache()
    return res

DEG_OF_K = {1: 0, 4: 1, 9: 2, 16: 3}


def fdo_leg(rast, sc, cam, images, G, counts, N, K, steps, warmup, workload):
    """Frequency-Decoupled Optimization step on the headline workload:
    render (with state), Haar cotangents of the rendered RGB against a
    fixed synthetic target (the render of the step plus N(0, 0.05) noise,
    clipped), the three-set backward (colour cotangents = the headline's
    N(0,1) cotangents) and Alg. 1's projection into one update (one view
    and no stored sets: per Gaussian, the Alg. 1 weights and one backward
    of the slots combined with them)."""
    import numpy as np
    import torch
    from paper_2512_02932_amd import _hgs
    from paper_2512_02932_amd.rasterizer import fdo_cotangents
    H, W = cam["height"], cam["width"]
    _, st = rast.render(sc, cam, images=images, want_state=True)
    st.free()
    torch.cuda.synchronize()
    rng = np.random.default_rng(17)
    target = torch.from_numpy(np.clip(images["rgb"].cpu().numpy() +
                                      rng.normal(0.0, 0.05, (1, 3, H, W)), 0.0, 1.0)
                              .astype(np.float32)).cuda()
    upd = {k: torch.empty_like(sc[k]) for k in ("means", "scales", "rotations", "opacities", "sh")}
    losses = torch.zeros(2, dtype=torch.float64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")

    def step():
        _, state = rast.render(sc, cam, images=images, want_state=True)
        gl, gh, _ = fdo_cotangents(images["rgb"], target, 0.2, 0.4, losses=losses)
        rast.backward_fdo(state, G, gl, gh, upd, n_conflict=cnt)
        state.free()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    cnt.zero_()
    ms, stage = time_steps(rast, step, steps)
    n_conf = int(cnt.item()) // (steps + 5)
    P = 11 + 3 * K
    cot_bytes = 3 * H * W * 16
    # one-view FDO preprocess backward per Gaussian: the three slot records
    # (3 x 64 B), means, scales, rotation, opacity, type, flag, rect (62 B)
    # and SH (4 * 3K) read; the update (4 * (11 + 3K)) written
    w_bytes = N * (3 * 64 + 62 + 4 * 3 * K + 4 * (11 + 3 * K))
    ops = (counts["blend_3d"] * (OPS_BWD["3d"] + 2 * OPS_BWD_RGB["3d"]) +
           counts["blend_2d"] * (OPS_BWD["2d"] + 2 * OPS_BWD_RGB["2d"]))

    def hbm(kernel, byt, ms_k, key):
        gbs = byt / (ms_k * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": round(gbs / (HBM_PEAK / 1e9), 4),
                "traffic": measured_traffic(key, workload), "kernel": kernel}

    tops = ops / (stage["raster_bwd"] * 1e-3) / 1e12
    out = {"ms_per_step": round(ms, 4), "mpix_per_s": round(H * W / (ms * 1e-3) / 1e6, 3),
           "conflicts_per_step": n_conf, "gaussians": N,
           "losses_last": [float(x) / (steps + warmup) for x in losses.cpu().tolist()],
           "stage_ms": {k: round(v, 4) for k, v in stage.items()},
           "preprocess_bwd_launches_per_step": 1,  # fdo_fused_bwd_kernel
           "roofline": {
               "raster_bwd_3set": {"bound": "alu", "achieved": round(tops, 4),
                                   "peak": round(VALU_PEAK / 1e12, 4), "unit": "Tops/s",
                                   "frac": round(tops / (VALU_PEAK / 1e12), 4),
                                   "traffic": measured_traffic("raster_bwd_kernel<3>", workload),
                                   "kernel": "raster_bwd_kernel<3>"},
               "fdo_cotangents": hbm("fdo_cotangents_kernel", cot_bytes, stage["fdo_cotangents"],
                                     "fdo_cotangents_kernel"),
               "fdo_preprocess_bwd": hbm(f"fdo_fused_bwd_kernel<{DEG_OF_K[K]}>", w_bytes,
                                         stage["fdo_preprocess_bwd"],
                                         f"fdo_fused_bwd_kernel<{DEG_OF_K[K]}>")}}
    log(f"[fdo] {out}")
    return out


def train_leg(rast, scene_np, cam, steps, warmup, workload):
    """One training iteration on the headline workload, as the paper trains
    (Sec. 3.3 losses, Alg. 1, 3DGS densification statistics and Adam with
    its default learning rates): render; L_color = 0.8 L1 + 0.2 D-SSIM and
    the Haar frequency cotangents against a fixed synthetic target (the
    initial render plus N(0, 0.05), clipped); the three-set backward and
    projection; the densification statistics; one fused Adam step on the raw
    parameters, writing the activated scene the next render reads.  The
    type exchange (every 500 iterations) is timed apart.
    Timed twice: eager (one launch sequence per iteration), and the same
    iteration captured once into a HIP graph and replayed (the colour loss
    then uses its entry point that allocates nothing; Adam's bias-correction
    step count is the captured one)."""
    import numpy as np
    import torch
    from paper_2512_02932_amd.rasterizer import adam_step, color_loss, fdo_cotangents, to_device
    H, W = cam["height"], cam["width"]
    N = int(scene_np["means"].shape[0])
    deg = int(scene_np["sh_degree"])
    sc = to_device(scene_np, "cuda")
    raw = {"means": sc["means"].clone(), "scales": torch.log(sc["scales"]),
           "rotations": sc["rotations"].clone(),
           "opacities": torch.logit(sc["opacities"].double()).float(), "sh": sc["sh"].clone()}
    m = {k: torch.zeros_like(v) for k, v in raw.items()}
    v = {k: torch.zeros_like(x) for k, x in raw.items()}
    act = {k: sc[k] for k in raw}
    upd = {k: torch.zeros_like(x) for k, x in raw.items()}
    images = rast.alloc_images(1, H, W)
    rast.render(sc, cam, images=images)
    torch.cuda.synchronize()
    rng = np.random.default_rng(23)
    target = torch.from_numpy(np.clip(images["rgb"].cpu().numpy() +
                                      rng.normal(0.0, 0.05, (1, 3, H, W)), 0.0, 1.0)
                              .astype(np.float32)).cuda()
    losses = torch.zeros(4, dtype=torch.float64, device="cuda")
    gnorm = torch.zeros(N, device="cuda")
    gcnt = torch.zeros(N, device="cuda")
    gcol = torch.empty_like(images["rgb"])
    it = [0]

    def body(noalloc):
        _, state = rast.render(sc, cam, images=images, want_state=True)
        color_loss(images["rgb"], target, 0.2, losses=losses[0:2], grad=gcol, noalloc=noalloc)
        gl, gh, _ = fdo_cotangents(images["rgb"], target, 0.2, 0.4, losses=losses[2:4])
        rast.backward_fdo(state, {"rgb": gcol}, gl, gh, upd)
        rast.densify_stats(state, gnorm, gcnt)
        adam_step(N, deg, raw, upd, m, v, it[0], activated=act)
        return state

    def step():
        it[0] += 1
        body(False).free()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    l0 = losses.cpu().numpy() / max(warmup, 1)
    losses.zero_()
    ms, stage = time_steps(rast, step, steps)
    stage = {k: round(v, 4) for k, v in stage.items()}
    l1 = losses.cpu().numpy() / (steps + 5)

    # the same iteration as one graph, replayed
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        it[0] += 1
        body(True).free()  # sizes the workspaces on the capture stream
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    it[0] += 1
    with torch.cuda.graph(g, stream=s):
        st_c = body(True)
    for _ in range(2):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) * 1e3 / steps
    del g
    st_c.free()

    K = (deg + 1) ** 2
    adam_bytes = N * (11 + 3 * K) * 4 * 8  # raw, grad, m, v read; raw, m, v, activated written
    ssim_bytes = 3 * H * W * (8 + 12 + 12 + 8 + 4)  # images, A/B/C out and in, images, grad
    out = {"ms_per_iteration": round(ms, 4), "iterations_per_s": round(1e3 / ms, 2),
           "graph_ms_per_iteration": round(ms_graph, 4),
           "graph_iterations_per_s": round(1e3 / ms_graph, 2),
           "gaussians": N, "width": W, "height": H,
           "losses_warmup_mean": {"l1": float(l0[0]), "dssim": float(l0[1]),
                                  "low": float(l0[2]), "high": float(l0[3])},
           "losses_timed_mean": {"l1": float(l1[0]), "dssim": float(l1[1]),
                                 "low": float(l1[2]), "high": float(l1[3])},
           "stage_ms": stage,
           "roofline": {
               "adam": {"bound": "hbm", "achieved": round(adam_bytes / (stage["adam"] * 1e-3) / 1e9, 1),
                        "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                        "frac": round(adam_bytes / (stage["adam"] * 1e-3) / HBM_PEAK, 4),
                        "traffic": measured_traffic("adam_kernel", workload),
                        "kernel": "adam_kernel"},
               "color_loss": {"bound": "hbm",
                              "achieved": round(ssim_bytes / (stage["color_loss"] * 1e-3) / 1e9, 1),
                              "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                              "frac": round(ssim_bytes / (stage["color_loss"] * 1e-3) / HBM_PEAK, 4),
                              "kernel": "ssim_fwd_kernel + ssim_bwd_kernel"}}}
    log(f"[train] {out}")
    del sc, raw, m, v, upd, images
    torch.cuda.empty_cache()
    return out


def _reap_children():
    """Ends any child process still alive (none is expected), so the run
    leaves nothing behind; returns what was found."""
    try:
        import psutil
    except ImportError:
        return []
    found = []
    for ch in psutil.Process().children(recursive=True):
        try:
            found.append(f"{ch.pid}:{' '.join(ch.cmdline())[:80]}")
            ch.terminate()
        except psutil.Error:
            pass
    if found:
        psutil.wait_procs(psutil.Process().children(recursive=True), timeout=5)
    return found


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="knot1m_1080p", choices=sorted(WORKLOADS))
    ap.add_argument("--legs", default=",".join(CONFIG_LEGS),
                    help="comma-separated per-config legs to time after the headline "
                         "('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-train", action="store_true",
                    help="skip the training-iteration timing")
    ap.add_argument("--no-fdo", action="store_true",
                    help="skip the Frequency-Decoupled Optimization step timing")
    ap.add_argument("--no-exchange", action="store_true",
                    help="skip the Adaptive Type Exchange kernel timing")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the served-view latency measurement")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after timing, run one device-to-device copy of this many MiB "
                         "(reference dispatch for scaling HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_02932_amd.rasterizer import get_rasterizer

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    rast = get_rasterizer(0)
    head, keep = render_leg(rast, args.workload, args.steps, args.warmup)
    scene_np, cam, sc = keep["scene_np"], keep["cam"], keep["sc"]

    if args.calib_copy_mb > 0:
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calib_copy_mb} MiB done")
        del src, dst

    out = {
        "metric": "fwd+bwd Mpixels/s @1M hybrid Gaussians 1080p; served-view p50/p99 ms",
        "value": head["mpix_per_s"], "unit": "Mpixels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": head["workload"], "gaussians": head["gaussians"],
                   "width": head["width"], "height": head["height"], "sh_degree": head["sh_degree"],
                   "pairs_D": head["pairs_D"], "stage_ms": head["stage_ms"]},
        "roofline": head["roofline"],
        "stage_roofline": head["stage_roofline"],
    }
    if not args.no_fdo and head["backward"] and head["views"] == 1:
        out["fdo"] = fdo_leg(rast, sc, cam, keep["images"], keep["G"], keep["counts"],
                             head["gaussians"], int(scene_np["sh"].shape[1]), args.steps,
                             args.warmup, args.workload)
    if not args.no_train and head["views"] == 1:
        out["train_step"] = train_leg(rast, scene_np, cam, args.steps, args.warmup, args.workload)
    if not args.no_exchange:
        out["type_exchange"] = exchange_leg(scene_np, args.workload)
    G_np = keep["G_np"]
    del keep, sc
    torch.cuda.empty_cache()
    legs = [x for x in args.legs.split(",") if x and x != args.workload]
    if legs:
        out["configs"] = {}
        for name in legs:
            rec, k2 = render_leg(rast, name, min(args.steps, 10 if name.startswith("multishell")
                                                  else args.steps), min(args.warmup, 2))
            del k2
            torch.cuda.empty_cache()
            out["configs"][name] = rec
    if not args.no_serving:
        out["serving"] = serving(rast)
    if not args.no_cpu_baseline and G_np is not None:
        log("[bench] cpu baseline")
        out["cpu_baseline"] = cpu_baseline(scene_np, cam, G_np)
    torch.cuda.synchronize()
    left = _reap_children()
    if left:
        log(f"[bench] ended child processes: {left}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
