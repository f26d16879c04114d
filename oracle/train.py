"""Training-step pieces, binary64: TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module.  It shares no code with the GPU library.

* The colour loss of Sec. 3.3, L_color = (1 - lambda) L1 + lambda D-SSIM,
  which the paper takes from 3DGS: L1 = mean |I^ - I|; D-SSIM = 1 - mean
  SSIM, with SSIM of Wang et al. (2004) per pixel and channel:
      SSIM = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2))
  where mu, s are local moments under an 11 x 11 Gaussian window of
  standard deviation 1.5 (normalised), C1 = 0.01^2, C2 = 0.03^2, and the
  window sums run over the image with zero padding ("same" size).  The
  gradient with respect to the rendered image is taken by PyTorch's
  autograd on the CPU in binary64 (the exact derivative of the expression
  above, a library primitive).
* Adam (Kingma and Ba, 2015) on the raw parameters of 3DGS: means,
  log-scales, quaternions, opacity logits and SH, with bias correction;
  the renderer's activated values are s = exp(s_raw), alpha =
  sigmoid(alpha_raw), and the chain from the activated-value gradients
  the rasterizer returns is dL/ds_raw = s dL/ds, dL/dalpha_raw =
  alpha (1 - alpha) dL/dalpha.
"""
from __future__ import annotations

import numpy as np

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def gauss_window(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    """Normalised 1D Gaussian window (the 2D window is its outer product)."""
    k = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return g / g.sum()


def _ssim_torch(x, y):
    import torch
    g = torch.from_numpy(gauss_window())
    w = (g[:, None] * g[None, :]).to(torch.float64)
    C = x.shape[1]
    win = w.expand(C, 1, WINDOW, WINDOW).contiguous()
    pad = WINDOW // 2
    conv = lambda t: torch.nn.functional.conv2d(t, win, padding=pad, groups=C)
    mx, my = conv(x), conv(y)
    sxx = conv(x * x) - mx * mx
    syy = conv(y * y) - my * my
    sxy = conv(x * y) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def ssim_map(render, target) -> np.ndarray:
    """Per-pixel, per-channel SSIM of [V, C, H, W] images (binary64)."""
    import torch
    x = torch.from_numpy(np.asarray(render, np.float64))
    y = torch.from_numpy(np.asarray(target, np.float64))
    return _ssim_torch(x, y).numpy()


def color_loss(render, target, lam: float = 0.2):
    """L_color and its gradient with respect to the rendered image.

    Returns dict(loss, l1, dssim, grad)."""
    import torch
    x = torch.from_numpy(np.array(render, np.float64)).requires_grad_(True)
    y = torch.from_numpy(np.asarray(target, np.float64))
    l1 = (x - y).abs().mean()
    dssim = 1.0 - _ssim_torch(x, y).mean()
    loss = (1.0 - lam) * l1 + lam * dssim
    loss.backward()
    return {"loss": float(loss.detach()), "l1": float(l1.detach()), "dssim": float(dssim.detach()),
            "grad": x.grad.numpy().copy()}


def ssim_brute(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """SSIM of two [H, W] planes by explicit window sums (tiny images)."""
    H, W = x.shape
    g = gauss_window()
    w = np.outer(g, g)
    r = WINDOW // 2
    out = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            mx = my = sxx = syy = sxy = 0.0
            for a in range(-r, r + 1):
                for b in range(-r, r + 1):
                    u, v = i + a, j + b
                    if 0 <= u < H and 0 <= v < W:
                        k = w[a + r, b + r]
                        mx += k * x[u, v]
                        my += k * y[u, v]
                        sxx += k * x[u, v] * x[u, v]
                        syy += k * y[u, v] * y[u, v]
                        sxy += k * x[u, v] * y[u, v]
            vx, vy, cxy = sxx - mx * mx, syy - my * my, sxy - mx * my
            out[i, j] = ((2 * mx * my + C1) * (2 * cxy + C2)) / \
                ((mx * mx + my * my + C1) * (vx + vy + C2))
    return out


ADAM_KEYS = ("means", "scales", "rotations", "opacities", "sh")


def adam_step(raw: dict, grads_act: dict, m: dict, v: dict, step: int, lr: dict,
              beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step (binary64) on raw 3DGS parameters from the gradients
    with respect to the activated values.  ``step`` is the 1-based step
    count.  Returns (raw', m', v', activated') as dicts of arrays."""
    raw = {k: np.asarray(raw[k], np.float64) for k in ADAM_KEYS}
    g = {k: np.asarray(grads_act[k], np.float64) for k in ADAM_KEYS}
    # chain to the raw parameters
    g["scales"] = g["scales"] * np.exp(raw["scales"])
    sig = 1.0 / (1.0 + np.exp(-raw["opacities"]))
    g["opacities"] = g["opacities"] * sig * (1.0 - sig)
    out_raw, out_m, out_v = {}, {}, {}
    for k in ADAM_KEYS:
        mk = beta1 * np.asarray(m[k], np.float64) + (1.0 - beta1) * g[k]
        vk = beta2 * np.asarray(v[k], np.float64) + (1.0 - beta2) * g[k] * g[k]
        mhat = mk / (1.0 - beta1 ** step)
        vhat = vk / (1.0 - beta2 ** step)
        lr_k = np.asarray(lr[k], np.float64)
        out_raw[k] = raw[k] - lr_k * mhat / (np.sqrt(vhat) + eps)
        out_m[k], out_v[k] = mk, vk
    act = dict(out_raw)
    act["scales"] = np.exp(out_raw["scales"])
    act["opacities"] = 1.0 / (1.0 + np.exp(-out_raw["opacities"]))
    return out_raw, out_m, out_v, act
