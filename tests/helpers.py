"""Small builders shared by the tests (scene assembly and packing only)."""
import numpy as np


def make_scene(means, scales, quats, opac, sh, types):
    means = np.asarray(means, np.float32).reshape(-1, 3)
    n = means.shape[0]
    sh = np.asarray(sh, np.float32).reshape(n, -1, 3)
    return dict(means=means, scales=np.asarray(scales, np.float32).reshape(n, 3),
                rotations=np.asarray(quats, np.float32).reshape(n, 4),
                opacities=np.asarray(opac, np.float32).reshape(n),
                sh=sh, types=np.asarray(types, np.uint8).reshape(n),
                sh_degree=int(round(np.sqrt(sh.shape[1]))) - 1)


def axis_camera(z=4.0, W=64, H=64, f=64.0, cx=None, cy=None):
    V = np.eye(4, dtype=np.float32)
    V[2, 3] = z
    return dict(viewmat=V, fx=float(f), fy=float(f), cx=float(W / 2 if cx is None else cx),
                cy=float(H / 2 if cy is None else cy), width=W, height=H, znear=0.2)


def pack_G(G, v=0):
    """[V,C,H,W] upstream gradient dict -> [P,8] in oracle pixel order."""
    rgb = G["rgb"][v].reshape(3, -1).T
    a = G["alpha"][v].reshape(1, -1).T
    d = G["depth"][v].reshape(1, -1).T
    n = G["normal"][v].reshape(3, -1).T
    return np.ascontiguousarray(np.concatenate([rgb, a, d, n], 1), np.float64)


def grad_close(g, ref, ref_abs, rtol=1e-3):
    """Per-element |g - ref| <= rtol (|ref| + sum|terms|)."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref) + np.asarray(ref_abs, np.float64)
    bad = np.abs(g - ref) > rtol * scale + 1e-12
    return bad


def rel_l2(g, ref):
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(np.asarray(g, np.float64) - ref) / (den if den > 0 else 1.0))


def central_fd(loss, base, key, g, j, ref_counts):
    """Fourth-order central difference of loss(params) with respect to
    base[key][g, j] at two step sizes, h and 2h with h = 1e-5 max(|x|, 1e-2):
    (-L(x+2h) + 8 L(x+h) - 8 L(x-h) + L(x-2h)) / 12h.  loss(params) returns
    (value, record); ref_counts(record) must equal ref_counts at the
    unperturbed point at every evaluation, else the coordinate crosses a
    discrete decision and None is returned.  Returns (fd_h, fd_2h)."""
    n = base[key].shape[0]
    x0 = float(base[key].reshape(n, -1)[g, j])
    h = 1e-5 * max(abs(x0), 1e-2)
    vals = {}
    for m in (-4, -2, -1, 1, 2, 4):
        p = {k: v.copy() for k, v in base.items()}
        p[key].reshape(n, -1)[g, j] = x0 + m * h
        val, rec = loss(p)
        if not ref_counts(rec):
            return None
        vals[m] = val

    def stencil(s):
        return (-vals[2 * s] + 8 * vals[s] - 8 * vals[-s] + vals[-2 * s]) / (12 * s * h)

    return stencil(1), stencil(2)
