"""Pins of the oracle's training-step pieces: SSIM against explicit window
sums, its identities and constant-image closed form, the colour loss's
gradient against central differences, and Adam with the activation chain
against torch.optim.Adam driven through autograd (an independent route)."""
import numpy as np
import pytest

from oracle import train


def test_window():
    g = train.gauss_window()
    assert g.shape == (11,)
    assert g.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(g, g[::-1], atol=0)
    assert g[5] / g[6] == pytest.approx(np.exp(1.0 / (2 * 1.5 ** 2)), rel=1e-14)


@pytest.mark.parametrize("H,W", [(7, 9), (13, 12), (1, 5)])
def test_ssim_matches_explicit_window_sums(H, W):
    rng = np.random.default_rng(H * 31 + W)
    x = rng.uniform(0, 1, (H, W))
    y = np.clip(x + rng.normal(0, 0.2, (H, W)), 0, 1)
    got = train.ssim_map(x[None, None], y[None, None])[0, 0]
    np.testing.assert_allclose(got, train.ssim_brute(x, y), atol=1e-12)


def test_ssim_identities():
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, (2, 3, 20, 17))
    np.testing.assert_allclose(train.ssim_map(x, x), 1.0, atol=1e-12)
    # constant planes: away from the border the variances vanish
    a, b = 0.3, 0.7
    s = train.ssim_map(np.full((1, 1, 30, 30), a), np.full((1, 1, 30, 30), b))[0, 0]
    np.testing.assert_allclose(s[5:25, 5:25], (2 * a * b + train.C1) / (a * a + b * b + train.C1),
                               rtol=1e-12)
    # symmetric in its arguments
    y = rng.uniform(0, 1, x.shape)
    np.testing.assert_allclose(train.ssim_map(x, y), train.ssim_map(y, x), atol=1e-14)


def test_color_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (1, 3, 6, 8))
    y = rng.uniform(0, 1, (1, 3, 6, 8))
    r = train.color_loss(x, y, 0.2)
    eps = 1e-6
    for idx in [(0, 0, 0, 0), (0, 1, 3, 4), (0, 2, 5, 7), (0, 0, 2, 0)]:
        a = x.copy(); a[idx] += eps
        b = x.copy(); b[idx] -= eps
        fd = (train.color_loss(a, y, 0.2)["loss"] - train.color_loss(b, y, 0.2)["loss"]) / (2 * eps)
        assert fd == pytest.approx(r["grad"][idx], rel=1e-6, abs=1e-10)
    # lambda = 0 is the plain L1: sign / M
    r0 = train.color_loss(x, y, 0.0)
    np.testing.assert_allclose(r0["grad"], np.sign(x - y) / x.size, atol=1e-15)
    assert r["loss"] == pytest.approx(0.8 * r["l1"] + 0.2 * r["dssim"], rel=1e-14)


def _adam_case(n=50, K=16, seed=4):
    rng = np.random.default_rng(seed)
    raw = {"means": rng.normal(size=(n, 3)), "scales": rng.normal(-4, 1, (n, 3)),
           "rotations": rng.normal(size=(n, 4)), "opacities": rng.normal(size=(n,)),
           "sh": rng.normal(0, 0.3, (n, K, 3))}
    lr = {"means": 1.6e-4, "scales": 5e-3, "rotations": 1e-3, "opacities": 2.5e-2,
          "sh": np.array([2.5e-3] + [2.5e-3 / 20] * (K - 1))[:, None]}
    return raw, lr, rng


def test_adam_matches_torch_through_autograd():
    import torch
    raw, lr, rng = _adam_case()
    m = {k: np.zeros_like(v) for k, v in raw.items()}
    v = {k: np.zeros_like(x) for k, x in raw.items()}
    params = {k: torch.tensor(x, dtype=torch.float64, requires_grad=True) for k, x in raw.items()}
    groups = [{"params": [params["means"]], "lr": lr["means"]},
              {"params": [params["scales"]], "lr": lr["scales"]},
              {"params": [params["rotations"]], "lr": lr["rotations"]},
              {"params": [params["opacities"]], "lr": lr["opacities"]}]
    # SH: DC and rest at different rates, as separate tensors in torch
    sh_dc = torch.tensor(raw["sh"][:, :1], dtype=torch.float64, requires_grad=True)
    sh_rest = torch.tensor(raw["sh"][:, 1:], dtype=torch.float64, requires_grad=True)
    groups += [{"params": [sh_dc], "lr": 2.5e-3}, {"params": [sh_rest], "lr": 2.5e-3 / 20}]
    opt = torch.optim.Adam(groups, betas=(0.9, 0.999), eps=1e-15)
    cur = dict(raw)
    for step in range(1, 4):
        ga = {k: rng.normal(size=x.shape) for k, x in raw.items()}
        cur, m, v, act = train.adam_step(cur, ga, m, v, step, lr)
        opt.zero_grad()
        act_t = {"means": params["means"], "scales": torch.exp(params["scales"]),
                 "rotations": params["rotations"], "opacities": torch.sigmoid(params["opacities"])}
        loss = sum((act_t[k] * torch.from_numpy(ga[k])).sum() for k in act_t)
        loss = loss + (torch.cat([sh_dc, sh_rest], 1) * torch.from_numpy(ga["sh"])).sum()
        loss.backward()
        opt.step()
        for k in ("means", "scales", "rotations", "opacities"):
            np.testing.assert_allclose(cur[k], params[k].detach().numpy(), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(cur["sh"], torch.cat([sh_dc, sh_rest], 1).detach().numpy(),
                                   rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(act["scales"], np.exp(cur["scales"]), rtol=1e-15)


def test_adam_first_step_closed_form():
    raw, lr, rng = _adam_case(n=7)
    ga = {k: rng.normal(size=x.shape) for k, x in raw.items()}
    z = {k: np.zeros_like(x) for k, x in raw.items()}
    new, _, _, _ = train.adam_step(raw, ga, z, z, 1, lr)
    # bias-corrected first step: -lr g / (|g| + eps) = -lr sign(g) (up to eps)
    np.testing.assert_allclose(new["means"] - raw["means"], -lr["means"] * np.sign(ga["means"]),
                               rtol=1e-9)
