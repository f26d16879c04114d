"""Adaptive Type Exchange on the GPU (hgs_type_exchange) against the oracle
(Sec. 3.2, Eq. 3; appendix "Effective Rank and Type Switch"): types and
scales bit-exact, rotations equal as rotations (unit quaternions up to sign,
within binary32 rounding of one quaternion product) and of unchanged length,
switch counts exact.  Primitives whose binary64 erank lies within 1e-12 of
theta_e are decided by either side's last-ulp log/exp and are checked for
validity only (either outcome of the rule, applied consistently)."""
import numpy as np
import pytest

import scenegen as sg
from gpu_common import IMG_KEYS, say

pytestmark = pytest.mark.gpu

QUAT_TOL = 1e-6
TIE = 1e-12


def _gaussians(n, seed, frac_flat=0.4):
    rng = np.random.default_rng(seed)
    s = np.exp(rng.normal(-3.0, 1.0, (n, 3))).astype(np.float32)
    flat = rng.random(n) < frac_flat
    s[flat, rng.integers(0, 3, int(flat.sum()))] *= rng.uniform(1e-4, 0.3, int(flat.sum())).astype(np.float32)
    q = (rng.normal(size=(n, 4)) * rng.uniform(0.5, 3.0, (n, 1))).astype(np.float32)
    t = (rng.random(n) < 0.5).astype(np.uint8)
    return s, q, t


def _run_gpu(s, q, t, theta):
    import torch
    from paper_2512_02932_amd.rasterizer import type_exchange
    S = torch.from_numpy(s.copy()).cuda()
    Q = torch.from_numpy(q.copy()).cuda()
    T = torch.from_numpy(t.copy()).cuda()
    counts = type_exchange(S, Q, T, theta)
    torch.cuda.synchronize()
    return S.cpu().numpy(), Q.cpu().numpy(), T.cpu().numpy(), counts.cpu().numpy()


def _canon(q):
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    return q * np.where(q[:, :1] < 0, -1.0, 1.0)


def _compare(s, q, t, theta):
    import oracle
    gs, gq, gt, counts = _run_gpu(s, q, t, theta)
    ref = oracle.type_exchange(s, q, t, theta)
    tie = np.abs(ref["erank"] - theta) <= TIE * theta
    ok = ~tie
    np.testing.assert_array_equal(gt[ok], ref["types"][ok])
    np.testing.assert_array_equal(gs[ok], ref["scales"][ok])
    err = np.abs(_canon(gq[ok]) - _canon(ref["quats"][ok]))
    # w = 0 rotations are equal up to sign too: compare |<q_gpu, q_ref>| = 1
    dots = np.abs(np.sum(_canon(gq[ok]) * _canon(ref["quats"][ok]), 1))
    assert (1.0 - dots).max() <= QUAT_TOL, (1.0 - dots).max()
    n0 = np.linalg.norm(q.astype(np.float64), axis=1)
    n1 = np.linalg.norm(gq.astype(np.float64), axis=1)
    assert np.abs(n1 / n0 - 1.0).max() <= 1e-6
    # untouched primitives keep their bytes
    keep = ok & (ref["moved"] == 0)
    np.testing.assert_array_equal(gq[keep], q[keep])
    # ties: either outcome, valid under the rule
    for i in np.flatnonzero(tie):
        assert gt[i] in (0, 1)
        assert sorted(gs[i].tolist()) == sorted(s[i].tolist())
    to2d = int(((t != 0) & (gt == 0)).sum())
    to3d = int(((t == 0) & (gt != 0)).sum())
    assert counts.tolist() == [to2d, to3d]
    ref2d = int(((t != 0) & (ref["types"] == 0))[ok].sum())
    ref3d = int(((t == 0) & (ref["types"] != 0))[ok].sum())
    assert to2d - int(tie.sum()) <= ref2d <= to2d + int(tie.sum())
    assert to3d - int(tie.sum()) <= ref3d <= to3d + int(tie.sum())
    say(f"[exchange] n={len(s)} theta={theta}: 3D->2D {to2d}, 2D->3D {to3d}, "
        f"moved {int((ref['moved'] != 0).sum())}, ties {int(tie.sum())}, "
        f"quat err {float(err.max()) if err.size else 0.0:.2e}")
    return gs, gq, gt, ref


@pytest.mark.parametrize("n,seed,theta", [(1, 1, 2.05), (255, 2, 2.05), (257, 3, 2.05),
                                          (100_003, 4, 2.05), (50_000, 5, 2.6), (50_000, 6, 1.5)])
def test_exchange_matches_oracle(n, seed, theta):
    _compare(*_gaussians(n, seed), theta)


def _near_threshold(n, theta, seed):
    """Scales whose erank lies within ~1e-3 of theta (both sides of both
    roots of erank(1, 1, z) = theta, then scaled, permuted and rotated), so
    that the kernel's binary32 pre-decision band and its binary64 fallback
    are both exercised."""
    import oracle
    f = lambda z: oracle.erank(1.0, 1.0, z) - theta
    roots = []
    for lo, hi in ((1e-6, 1.0), (1.0, 50.0)):
        if f(lo) * f(hi) < 0:
            for _ in range(100):
                mid = 0.5 * (lo + hi)
                lo, hi = (mid, hi) if f(lo) * f(mid) > 0 else (lo, mid)
            roots.append(lo)
    rng = np.random.default_rng(seed)
    z = np.array(roots)[rng.integers(0, len(roots), n)]
    z = z * (1.0 + rng.uniform(-2e-3, 2e-3, n) * rng.choice([1.0, 1e-2, 1e-4], n))
    s = np.stack([np.ones(n), np.ones(n), z], 1) * np.exp(rng.normal(-3.0, 1.5, (n, 1)))
    perm = np.argsort(rng.random((n, 3)), 1)
    s = np.take_along_axis(s, perm, 1).astype(np.float32)
    q = rng.normal(size=(n, 4)).astype(np.float32)
    t = (rng.random(n) < 0.5).astype(np.uint8)
    return s, q, t


@pytest.mark.parametrize("theta", [2.05, 2.6])
def test_exchange_near_threshold(theta):
    import oracle
    s, q, t = _near_threshold(200_000, theta, 17)
    e = oracle.type_exchange(s, q, t, theta)["erank"]
    band = np.abs(np.log(e) - np.log(theta)) < 1e-4
    say(f"[exchange] near threshold: {int(band.sum())} of {len(s)} inside the 1e-4 band of ln theta")
    assert band.sum() > 1000 and (~band).sum() > 1000
    _compare(s, q, t, theta)


def test_exchange_unaligned_arrays_take_the_scalar_path():
    """Scales at a 4-byte (not 16-byte) offset and types at an odd offset:
    the element-wise path gives the same result."""
    import torch
    import oracle
    from paper_2512_02932_amd.rasterizer import get_rasterizer
    from paper_2512_02932_amd import _hgs as H
    s, q, t = _gaussians(10_001, 8)
    ref = oracle.type_exchange(s, q, t, 2.05)
    S = torch.zeros(3 * len(s) + 1, device="cuda")
    S[1:] = torch.from_numpy(s.reshape(-1)).cuda()
    T = torch.zeros(len(t) + 1, dtype=torch.uint8, device="cuda")
    T[1:] = torch.from_numpy(t).cuda()
    Q = torch.from_numpy(q.copy()).cuda()
    counts = torch.zeros(2, dtype=torch.int32, device="cuda")
    rast = get_rasterizer(0)
    H.hgs_type_exchange(rast.ctx, len(s), S.data_ptr() + 4, Q.data_ptr(), T.data_ptr() + 1, 2.05,
                        counts.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    tie = np.abs(ref["erank"] - 2.05) <= TIE * 2.05
    gs = S[1:].cpu().numpy().reshape(-1, 3)
    gt = T[1:].cpu().numpy()
    np.testing.assert_array_equal(gt[~tie], ref["types"][~tie])
    np.testing.assert_array_equal(gs[~tie], ref["scales"][~tie])
    assert float(S[0]) == 0.0 and int(T[0]) == 0
    dots = np.abs(np.sum(_canon(Q.cpu().numpy()[~tie]) * _canon(ref["quats"][~tie]), 1))
    assert (1.0 - dots).max() <= QUAT_TOL


def test_exchange_edge_cases():
    # exact ties among the least scales, zero scales, erank exactly 1, 2, 3,
    # NaN, infinite, subnormal, near-overflow and negative scales
    s = np.array([[0.2, 0.2, 0.2], [0.1, 0.1, 0.5], [0.1, 0.5, 0.1], [0.5, 0.1, 0.1],
                  [0.0, 0.0, 0.0], [0.0, 0.3, 0.3], [0.4, 0.0, 0.0], [0.3, 0.3, 0.0],
                  [1e-30, 1e-30, 1e-30], [3e19, 1e-3, 2e19], [0.01, 0.5, 0.7], [0.5, 0.01, 0.7],
                  [np.nan, 0.3, 0.2], [0.3, np.nan, 0.2], [np.inf, 0.3, 0.2], [0.3, 0.2, np.inf],
                  [1e-40, 1e-40, 1e-41], [1e-40, 0.0, 0.0], [3e38, 3e38, 1e38], [-0.3, 0.2, -0.01]],
                 np.float32)
    n = len(s)
    q = np.tile(np.array([[0.3, -0.5, 0.7, 0.1]], np.float32), (n, 1))
    for t0 in (0, 1):
        t = np.full(n, t0, np.uint8)
        gs, gq, gt, ref = _compare(s, q, t, 2.05)
        if t0 == 1:
            # (0.1, 0.1, 0.5): s_x and s_y tie, s_z not least -> P_y; a z tying
            # for least moves nothing; x alone least -> P_x, y alone -> P_y
            np.testing.assert_array_equal(ref["moved"][[1, 2, 3, 10, 11]], [2, 0, 0, 1, 2])


def test_exchange_empty_and_bad_arguments():
    import torch
    from paper_2512_02932_amd import _hgs as H
    from paper_2512_02932_amd.rasterizer import get_rasterizer, type_exchange
    e = torch.zeros((0, 3), device="cuda")
    counts = type_exchange(e, torch.zeros((0, 4), device="cuda"),
                           torch.zeros(0, dtype=torch.uint8, device="cuda"))
    assert counts.cpu().tolist() == [0, 0]
    rast = get_rasterizer(0)
    buf = torch.zeros(64, device="cuda")
    p = buf.data_ptr()
    with pytest.raises(H.HGSError) as ex:
        H.hgs_type_exchange(rast.ctx, 1, p, p + 4, p, 2.05, 0, 0)  # misaligned rotations
    assert ex.value.status == H.HGS_EINVAL
    with pytest.raises(H.HGSError) as ex:
        H.hgs_type_exchange(rast.ctx, -1, p, p, p, 2.05, 0, 0)
    assert ex.value.status == H.HGS_EINVAL
    with pytest.raises(H.HGSError) as ex:
        H.hgs_type_exchange(rast.ctx, 4, p, p, p, float("nan"), 0, 0)
    assert ex.value.status == H.HGS_EINVAL


def test_exchange_full_size_scene_then_render_matches_oracle():
    """The 1M-primitive torus-knot scene at the paper's theta_e: exchange on
    the GPU equals the oracle's, and the exchanged scene renders like the
    oracle's render of the oracle-exchanged scene on sampled pixels."""
    import torch
    import oracle
    from paper_2512_02932_amd.rasterizer import get_rasterizer, to_device
    from gpu_common import compare_images
    scene = sg.scene_torus_knot(n=1_000_000, frac2d=0.5, seed=3)
    gs, gq, gt, ref = _compare(scene["scales"], scene["rotations"], scene["types"], 2.05)
    # small render of the exchanged scene
    ex = dict(scene)
    ex["scales"], ex["rotations"], ex["types"] = gs, gq, gt
    cam = sg.orbit_camera(3.2, 0.4, 0.1, 320, 200)
    rast = get_rasterizer(0)
    imgs, state = rast.render(to_device(ex), cam, want_state=True)
    torch.cuda.synchronize()
    imgs = {k: v.cpu().numpy() for k, v in imgs.items()}
    rng = np.random.default_rng(11)
    pix = np.stack([np.zeros(600, np.int32), rng.integers(0, 200, 600),
                    rng.integers(0, 320, 600)], 1).astype(np.int32)
    # the oracle renders the exchanged parameters as the GPU holds them
    res = oracle.forward(ex, cam, pix)
    _, _, rep = compare_images(imgs, state, res, pix, ex, cam)
    say(f"[exchange] render after exchange: {rep}")
    state.free()
