"""Seeded synthetic scenes, cameras and upstream gradients.

This module is shared by the GPU path's tests, the benchmark and the CPU
oracle's tests.  It only draws random inputs and builds cameras; it holds none
of the rendering arithmetic (no projection, no SH decoding, no compositing).

The representation follows the paper's statement of a hybrid primitive
(Sec. 3.1, "Hybrid Gaussian Rasterization"): centre mu, scale s, rotation
quaternion r, opacity alpha, SH coefficients f, and a type flag t (0 = 2D
surfel, 1 = 3D Gaussian).  2D primitives are created with s_z = 0, as the
paper initialises them.  Types are drawn at random (appendix "Implementation
Details": types are initialised at random).

Conventions of the arrays (all little-endian, C-contiguous):
  means      f32[N,3]   world position
  scales     f32[N,3]   activated (positive) scales; scales[:,2] = 0 for 2D
  rotations  f32[N,4]   quaternion (w, x, y, z), not necessarily unit length
  opacities  f32[N]     activated opacity in (0, 1)
  sh         f32[N,K,3] SH coefficients, K = (degree+1)^2, channel-last
  types      u8[N]      0 = 2D surfel, 1 = 3D Gaussian

A camera is a dict with a row-major world->camera matrix ``viewmat``
(f32[4,4], OpenCV axes: x right, y down, z forward), intrinsics fx, fy, cx,
cy, the image size and z_near.
"""
from __future__ import annotations

import math

import numpy as np

SCENE_KEYS = ("means", "scales", "rotations", "opacities", "sh", "types")

# Range of a degree-0 coefficient whose decoded colour lies in (0, 1): the
# constant real spherical harmonic is 1/(2 sqrt(pi)), so colour 0.5 +/- 0.5
# corresponds to a coefficient of +/- sqrt(pi).
_SH0_HALF_RANGE = math.sqrt(math.pi)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _quat_mul(a, b):
    aw, ax, ay, az = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    bw, bx, by, bz = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([
        aw * bw - ax * bx - ay * by - az * bz,
        aw * bx + ax * bw + ay * bz - az * by,
        aw * by - ax * bz + ay * bw + az * bx,
        aw * bz + ax * by - ay * bx + az * bw,
    ], axis=-1)


def quats_aligning_z(normals: np.ndarray, spin: np.ndarray) -> np.ndarray:
    """Quaternions (w,x,y,z) whose rotation maps e_z to ``normals`` after an
    in-plane spin by ``spin`` radians about e_z.  Used to orient surfels so
    that their third axis follows a surface normal."""
    n = normals / np.linalg.norm(normals, axis=1, keepdims=True)
    ez = np.array([0.0, 0.0, 1.0])
    axis = np.cross(np.broadcast_to(ez, n.shape), n)
    s = np.linalg.norm(axis, axis=1)
    c = n[:, 2]
    ang = np.arctan2(s, c)
    safe = s > 1e-12
    axis_u = np.where(safe[:, None], axis / np.where(safe, s, 1.0)[:, None],
                      np.array([1.0, 0.0, 0.0]))
    q_align = np.concatenate([np.cos(ang / 2)[:, None],
                              np.sin(ang / 2)[:, None] * axis_u], axis=1)
    q_spin = np.stack([np.cos(spin / 2), np.zeros_like(spin),
                       np.zeros_like(spin), np.sin(spin / 2)], axis=1)
    return _quat_mul(q_align, q_spin)


def look_at_camera(eye, target=(0.0, 0.0, 0.0), *, width: int, height: int,
                   fx: float, fy: float | None = None, cx: float | None = None,
                   cy: float | None = None, znear: float = 0.2,
                   up=(0.0, -1.0, 0.0)) -> dict:
    """Pinhole camera at ``eye`` looking at ``target``; world ``up`` maps to
    camera -y (OpenCV axes)."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    right = np.cross(f, np.asarray(up, np.float64))
    if np.linalg.norm(right) < 1e-9:
        right = np.cross(f, np.array([0.0, 0.0, 1.0]))
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    R = np.stack([right, down, f])
    t = -R @ eye
    V = np.eye(4)
    V[:3, :3] = R
    V[:3, 3] = t
    return dict(viewmat=V.astype(np.float32), fx=float(fx),
                fy=float(fy if fy is not None else fx),
                cx=float(cx if cx is not None else width / 2.0),
                cy=float(cy if cy is not None else height / 2.0),
                width=int(width), height=int(height), znear=float(znear))


def _finish(types, means, log_scales, rots, opac_logit, sh):
    scales = np.exp(log_scales)
    scales[types == 0, 2] = 0.0
    return dict(means=np.ascontiguousarray(means, np.float32),
                scales=np.ascontiguousarray(scales, np.float32),
                rotations=np.ascontiguousarray(rots, np.float32),
                opacities=np.ascontiguousarray(_sigmoid(opac_logit), np.float32),
                sh=np.ascontiguousarray(sh, np.float32),
                types=np.ascontiguousarray(types, np.uint8),
                sh_degree=int(round(math.sqrt(sh.shape[1]))) - 1)


def _types(rng, n, n2d):
    t = np.ones(n, np.uint8)
    t[:n2d] = 0
    return t[rng.permutation(n)]


def _sh3(rng, n, sigma=0.3):
    return rng.normal(0.0, sigma, size=(n, 16, 3))


# --------------------------------------------------------------------------
# Workload 1: 10k Gaussians (5k 3D + 5k 2D) uniform in a cube, SH degree 0,
# 256x256 camera at distance 4.
# --------------------------------------------------------------------------
def scene_uniform_cube(n=10_000, n2d=5_000, seed=1):
    rng = _rng(seed)
    types = _types(rng, n, n2d)
    means = rng.uniform(-1.0, 1.0, size=(n, 3))
    log_s = rng.normal(-4.0, 0.5, size=(n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opac = rng.normal(size=n)
    sh = rng.uniform(-_SH0_HALF_RANGE, _SH0_HALF_RANGE, size=(n, 1, 3))
    return _finish(types, means, log_s, q, opac, sh)


def camera_cube():
    return look_at_camera((0.0, 0.0, -4.0), width=256, height=256, fx=256.0)


# --------------------------------------------------------------------------
# Surface scenes: surfels take their third axis from the surface normal at
# the un-noised sample; 3D Gaussians get random rotations.
# --------------------------------------------------------------------------
def _surface_scene(rng, n, n2d, pts, nrm, noise, log_mu=-5.0, log_sigma=0.5,
                   sh_degree=3):
    types = _types(rng, n, n2d)
    means = pts + rng.normal(0.0, noise, size=(n, 3))
    log_s = rng.normal(log_mu, log_sigma, size=(n, 3))
    q_rand = rng.normal(size=(n, 4))
    q_rand /= np.linalg.norm(q_rand, axis=1, keepdims=True)
    spin = rng.uniform(0.0, 2 * np.pi, size=n)
    q_surf = quats_aligning_z(nrm, spin)
    rots = np.where((types == 0)[:, None], q_surf, q_rand)
    opac = rng.normal(size=n)
    k = (sh_degree + 1) ** 2
    sh = _sh3(rng, n)[:, :k, :]
    return _finish(types, means, log_s, rots, opac, sh)


def _sphere_dirs(rng, n):
    d = rng.normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def scene_sphere(n=500_000, frac2d=0.7, seed=2, radius=1.0, noise=0.02):
    """Noisy sphere: centres on a sphere of ``radius`` plus N(0, noise^2)."""
    rng = _rng(seed)
    n2d = int(round(frac2d * n))
    d = _sphere_dirs(rng, n)
    return _surface_scene(rng, n, n2d, radius * d, d, noise)


def camera_sphere(width=1920, height=1080, f=1200.0, distance=3.0):
    return look_at_camera((0.0, 0.0, -distance), width=width, height=height, fx=f)


def torus_knot_points(phi, psi, tube=0.15):
    """(2,3) torus knot centre line c(phi) with a tube of radius ``tube``.
    Returns surface points and unit surface normals."""
    r = 1.0 + 0.4 * np.cos(3 * phi)
    c = np.stack([r * np.cos(2 * phi), r * np.sin(2 * phi), 0.4 * np.sin(3 * phi)], 1)
    dr = -1.2 * np.sin(3 * phi)
    tan = np.stack([dr * np.cos(2 * phi) - 2 * r * np.sin(2 * phi),
                    dr * np.sin(2 * phi) + 2 * r * np.cos(2 * phi),
                    1.2 * np.cos(3 * phi)], 1)
    tan /= np.linalg.norm(tan, axis=1, keepdims=True)
    n1 = np.cross(tan, np.array([0.0, 0.0, 1.0]))
    n1 /= np.linalg.norm(n1, axis=1, keepdims=True)
    n2 = np.cross(tan, n1)
    nrm = np.cos(psi)[:, None] * n1 + np.sin(psi)[:, None] * n2
    return c + tube * nrm, nrm


def scene_torus_knot(n=1_000_000, frac2d=0.5, seed=3, noise=0.01):
    rng = _rng(seed)
    n2d = int(round(frac2d * n))
    phi = rng.uniform(0.0, 2 * np.pi, size=n)
    psi = rng.uniform(0.0, 2 * np.pi, size=n)
    pts, nrm = torus_knot_points(phi, psi)
    return _surface_scene(rng, n, n2d, pts, nrm, noise)


def camera_torus_knot(width=1600, height=1064, f=1200.0, distance=4.0):
    return look_at_camera((0.0, 0.0, -distance), width=width, height=height, fx=f)


def camera_torus_knot_1080p():
    return camera_torus_knot(width=1920, height=1080)


def scene_multishell(n=6_000_000, frac2d=0.6, seed=5,
                     radii=(0.55, 0.80, 1.05, 1.30), noise=0.01):
    """Concentric noisy spheres, counts proportional to r^2."""
    rng = _rng(seed)
    radii = np.asarray(radii)
    w = radii ** 2 / np.sum(radii ** 2)
    counts = np.floor(w * n).astype(np.int64)
    counts[-1] += n - counts.sum()
    shell = np.repeat(np.arange(len(radii)), counts)
    d = _sphere_dirs(rng, n)
    pts = radii[shell][:, None] * d
    n2d = int(round(frac2d * n))
    return _surface_scene(rng, n, n2d, pts, d, noise)


def fibonacci_cameras(n_views=16, radius=3.5, width=3840, height=2160, f=2400.0):
    cams = []
    golden = math.pi * (3.0 - math.sqrt(5.0))
    for i in range(n_views):
        y = 1.0 - 2.0 * (i + 0.5) / n_views
        rr = math.sqrt(max(0.0, 1.0 - y * y))
        th = golden * i
        eye = radius * np.array([rr * math.cos(th), y, rr * math.sin(th)])
        cams.append(look_at_camera(eye, width=width, height=height, fx=f))
    return cams


# --------------------------------------------------------------------------
# Small random scenes for parity tests: a mix of types, orientations and
# sizes in front of the camera, including tilted and near edge-on surfels.
# --------------------------------------------------------------------------
def scene_random(n, seed, *, frac2d=0.5, box=1.0, log_mu=-3.0, log_sigma=0.6,
                 sh_degree=3, center=(0.0, 0.0, 0.0)):
    rng = _rng(seed)
    n2d = int(round(frac2d * n))
    types = _types(rng, n, n2d)
    means = rng.uniform(-box, box, size=(n, 3)) + np.asarray(center)
    log_s = rng.normal(log_mu, log_sigma, size=(n, 3))
    q = rng.normal(size=(n, 4))
    q *= rng.uniform(0.5, 2.0, size=(n, 1))      # non-unit quaternions
    opac = rng.normal(size=n)
    k = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, 0.3, size=(n, k, 3))
    return _finish(types, means, log_s, q, opac, sh)


def scene_gate(n, seed, *, theta_z, temp_z, log_mu=-3.0, box=1.0):
    """A random scene (half surfels) whose surfels carry a third scale s_z
    in the region of the scale-modulation gate (Sec. 3.2, Eq. 6-7): 40% of
    them uniform in theta_z +/- 5 temp_z, 20% far above the gate, uniform in
    [1.5 theta_z, 3 theta_z], and the rest at s_z = 0 (their initial value)."""
    sc = scene_random(n, seed, log_mu=log_mu, box=box)
    rng = _rng(seed + 1000)
    idx = np.nonzero(sc["types"] == 0)[0]
    pick = rng.permutation(idx)
    n_in, n_far = int(0.4 * len(idx)), int(0.2 * len(idx))
    sz = sc["scales"][:, 2].copy()
    sz[pick[:n_in]] = rng.uniform(theta_z - 5 * temp_z, theta_z + 5 * temp_z, n_in)
    sz[pick[n_in:n_in + n_far]] = rng.uniform(1.5 * theta_z, 3.0 * theta_z, n_far)
    sc["scales"][:, 2] = sz.astype(np.float32)
    return sc


def upstream_grads(n_views, height, width, seed):
    """N(0,1) cotangents for every output channel: rgb, alpha, depth, normal."""
    rng = _rng(seed)
    return dict(
        rgb=rng.normal(size=(n_views, 3, height, width)).astype(np.float32),
        alpha=rng.normal(size=(n_views, 1, height, width)).astype(np.float32),
        depth=rng.normal(size=(n_views, 1, height, width)).astype(np.float32),
        normal=rng.normal(size=(n_views, 3, height, width)).astype(np.float32))


def subset(scene, idx):
    out = {k: np.ascontiguousarray(scene[k][idx]) for k in SCENE_KEYS}
    out["sh_degree"] = scene["sh_degree"]
    return out


def crop_camera(cam, x0, y0, width, height):
    """The same pinhole camera restricted to the window [x0, x0+w) x [y0, y0+h)."""
    c = dict(cam)
    c["cx"] = cam["cx"] - x0
    c["cy"] = cam["cy"] - y0
    c["width"] = int(width)
    c["height"] = int(height)
    return c


def fd_subset(seed=33, n_each=32, crop=32):
    """Finite-difference workload: a 32x32 window of the torus-knot camera
    centred on the image of the knot's curve point at phi = 0, keeping the
    32 surfels and 32 3D Gaussians whose projected centres are nearest the
    window centre.  (The knot winds around the optical axis, so a window at
    the image centre would see nothing.)  Selection only; no rendering
    arithmetic."""
    scene = scene_torus_knot(n=200_000, seed=seed)
    cam = camera_torus_knot()
    V = cam["viewmat"].astype(np.float64)
    c0 = torus_knot_points(np.zeros(1), np.zeros(1), tube=0.0)[0][0]
    p0 = V[:3, :3] @ c0 + V[:3, 3]
    u0 = cam["fx"] * p0[0] / p0[2] + cam["cx"]
    v0 = cam["fy"] * p0[1] / p0[2] + cam["cy"]
    x0 = int(round(u0)) - crop // 2
    y0 = int(round(v0)) - crop // 2
    pc = scene["means"].astype(np.float64) @ V[:3, :3].T + V[:3, 3]
    u = cam["fx"] * pc[:, 0] / pc[:, 2] + cam["cx"]
    v = cam["fy"] * pc[:, 1] / pc[:, 2] + cam["cy"]
    dist = (u - (x0 + crop / 2)) ** 2 + (v - (y0 + crop / 2)) ** 2
    pick = []
    for t in (0, 1):
        cand = np.nonzero(scene["types"] == t)[0]
        pick.append(cand[np.argsort(dist[cand], kind="stable")[:n_each]])
    idx = np.sort(np.concatenate(pick))
    return subset(scene, idx), crop_camera(cam, x0, y0, crop, crop)


# ----- serving workload: four resident scenes and a Poisson request stream -----
SERVING_RESOLUTIONS = ((256, 256), (512, 512), (1280, 720), (1920, 1080))


def serving_scenes():
    """The four resident scenes of the serving workload, seeds 41-44:
    a 100k sphere (70% surfels), the 500k sphere, the 1M torus knot and a
    3M multi-shell (60% surfels), all SH degree 3."""
    return [scene_sphere(n=100_000, frac2d=0.7, seed=41),
            scene_sphere(n=500_000, frac2d=0.7, seed=42),
            scene_torus_knot(n=1_000_000, frac2d=0.5, seed=43),
            scene_multishell(n=3_000_000, frac2d=0.6, seed=44)]


def orbit_camera(radius, azimuth, elevation, width, height, vfov_deg=50.0):
    """Camera on an orbit around the origin, looking at it, with vertical
    field of view ``vfov_deg`` (f = H / (2 tan(vfov/2)))."""
    eye = radius * np.array([np.cos(elevation) * np.sin(azimuth), np.sin(elevation),
                             -np.cos(elevation) * np.cos(azimuth)])
    f = height / (2.0 * np.tan(np.deg2rad(vfov_deg) / 2.0))
    return look_at_camera(eye, width=width, height=height, fx=f)


def serving_requests(n, rate=200.0, seed=45, n_scenes=4):
    """``n`` requests: Poisson arrival times (s) at ``rate`` per second,
    scene index uniform, resolution uniform over SERVING_RESOLUTIONS,
    orbit radius U[3,5], azimuth U[0, 2 pi), elevation U[-20, 20] degrees.
    Returns a list of dicts (t, scene, camera)."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, n)
    t = np.cumsum(gaps)
    sc = rng.integers(0, n_scenes, n)
    res = rng.integers(0, len(SERVING_RESOLUTIONS), n)
    rad = rng.uniform(3.0, 5.0, n)
    az = rng.uniform(0.0, 2.0 * np.pi, n)
    el = np.deg2rad(rng.uniform(-20.0, 20.0, n))
    out = []
    for i in range(n):
        w, h = SERVING_RESOLUTIONS[res[i]]
        out.append(dict(t=float(t[i]), scene=int(sc[i]),
                        camera=orbit_camera(rad[i], az[i], el[i], w, h)))
    return out
