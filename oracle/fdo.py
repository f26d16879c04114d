"""Frequency-Decoupled Optimization, binary64: TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module.  It shares no code with the GPU library.

It follows Sec. 3.3 of the paper (frequency losses, Alg. 1) and the
appendices "Discrete Wavelet Transformation" and "Gradient Conflict
Analysis":

* The level-1 DWT with the Haar filters, written as the appendix writes it:
  analysis matrices L (low-pass l) and H (high-pass h) and the four
  sub-bands I^LL = L I L^T, I^LH = H I L^T, I^HL = L I H^T, I^HH = H I H^T.
  The row operator acts on the image's y index, the column operator on x.
  Haar: l = (1, 1)/sqrt 2, h = (1, -1)/sqrt 2.  An odd length is zero-padded
  at the end (the matrices simply have no column for the padded sample).
* L_low = ||I^_LL - I_LL||^2 and L_high = the same summed over LH, HL, HH,
  each squared norm averaged over the elements of its band (mean squared
  error).  Their cotangents on the rendered image come from the adjoint
  Y -> A^T Y B of each band map X -> A X B^T.
* Alg. 1, per primitive i: if g_low . g_high < 0, a 2D primitive (type 0)
  projects g_high onto the normal of g_low (Eq. 9), a 3D one projects g_low
  onto the normal of g_high (Eq. 10); the update is g_color + g_low +
  g_high.  g is the gradient with respect to all of the primitive's
  parameters, concatenated (means 3, scales 3, rotations 4, opacity 1,
  SH 3K), as the rasterizer's backward returns them.
"""
from __future__ import annotations

import numpy as np

PARAM_ORDER = ("means", "scales", "rotations", "opacities", "sh")


def haar_matrices(n: int):
    """Level-1 Haar analysis matrices (L, H), each ceil(n/2) x n."""
    m = (n + 1) // 2
    r = 1.0 / np.sqrt(2.0)
    L = np.zeros((m, n))
    H = np.zeros((m, n))
    for i in range(m):
        L[i, 2 * i] = r
        H[i, 2 * i] = r
        if 2 * i + 1 < n:
            L[i, 2 * i + 1] = r
            H[i, 2 * i + 1] = -r
    return L, H


def dwt(img):
    """Sub-bands of img [..., H, W] (binary64): dict LL, LH, HL, HH."""
    x = np.asarray(img, np.float64)
    Lr, Hr = haar_matrices(x.shape[-2])
    Lc, Hc = haar_matrices(x.shape[-1])
    return {"LL": Lr @ x @ Lc.T, "LH": Hr @ x @ Lc.T, "HL": Lr @ x @ Hc.T, "HH": Hr @ x @ Hc.T}


def dwt_adjoint(bands, shape):
    """Adjoint of :func:`dwt` applied to a dict of sub-band arrays (missing
    bands are zero); `shape` is the image's [..., H, W]."""
    Lr, Hr = haar_matrices(shape[-2])
    Lc, Hc = haar_matrices(shape[-1])
    out = np.zeros(shape)
    ops = {"LL": (Lr, Lc), "LH": (Hr, Lc), "HL": (Lr, Hc), "HH": (Hr, Hc)}
    for k, y in bands.items():
        A, B = ops[k]
        out = out + A.T @ np.asarray(y, np.float64) @ B
    return out


def fdo_losses(render, target, lambda_low=0.2, lambda_high=0.4):
    """Frequency losses of a rendered RGB image against a target, both
    [V, 3, H, W], and their weighted cotangents on the rendered image.

    Returns dict(low, high) = (L_low, L_high) unweighted, and
    grad_low = lambda_low dL_low/dI^, grad_high = lambda_high dL_high/dI^."""
    r = dwt(render)
    t = dwt(target)
    shape = np.asarray(render).shape
    res = {k: r[k] - t[k] for k in r}
    n = res["LL"].size
    low = float(np.sum(res["LL"] ** 2) / n)
    high = float(sum(np.sum(res[k] ** 2) / res[k].size for k in ("LH", "HL", "HH")))
    g_low = lambda_low * dwt_adjoint({"LL": 2.0 * res["LL"] / n}, shape)
    g_high = lambda_high * dwt_adjoint({k: 2.0 * res[k] / res[k].size for k in ("LH", "HL", "HH")},
                                       shape)
    return {"low": low, "high": high, "grad_low": g_low, "grad_high": g_high}


def pack(grads: dict, n: int):
    """Concatenate a gradient dict into [n, P] binary64 rows (PARAM_ORDER)."""
    cols = [np.asarray(grads[k], np.float64).reshape(n, -1) for k in PARAM_ORDER]
    return np.concatenate(cols, 1)


def fdo_project(types, g_color, g_low, g_high):
    """Alg. 1 on [n, P] gradient rows.  Returns dict(update, low, high,
    conflict): the summed update, the (possibly projected) g_low and g_high,
    and the conflict mask g_low . g_high < 0."""
    gc = np.asarray(g_color, np.float64)
    gl = np.array(g_low, np.float64)
    gh = np.array(g_high, np.float64)
    t = np.asarray(types)
    conflict = np.zeros(len(gl), bool)
    for i in range(len(gl)):
        d = float(np.dot(gl[i], gh[i]))
        if d < 0.0:
            conflict[i] = True
            if t[i] == 0:  # 2D: keep g_low, project g_high (Eq. 9)
                gh[i] = gh[i] - d / float(np.dot(gl[i], gl[i])) * gl[i]
            else:  # 3D: keep g_high, project g_low (Eq. 10)
                gl[i] = gl[i] - d / float(np.dot(gh[i], gh[i])) * gh[i]
    return {"update": gc + gl + gh, "low": gl, "high": gh, "conflict": conflict}
