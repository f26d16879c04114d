"""Pins of the oracle's Frequency-Decoupled Optimization (Sec. 3.3, Alg. 1;
appendices on the DWT and on gradient conflicts): a worked 2x2 Haar example,
the sub-band of each elementary pattern, Parseval and perfect
reconstruction (Haar is orthonormal), the adjoint, closed-form losses,
cotangents against central finite differences, and the projection's
geometry (orthogonality, identity without conflict, which vector is kept)."""
import numpy as np
import pytest

from oracle import fdo


def test_haar_worked_2x2():
    # I = [[a, b], [c, d]]: LL = (a+b+c+d)/2, LH = (a+b-c-d)/2 (rows differ),
    # HL = (a-b+c-d)/2 (columns differ), HH = (a-b-c+d)/2
    b = fdo.dwt(np.array([[1.0, 2.0], [3.0, 4.0]]))
    assert b["LL"][0, 0] == pytest.approx(5.0, abs=1e-15)
    assert b["LH"][0, 0] == pytest.approx(-2.0, abs=1e-15)
    assert b["HL"][0, 0] == pytest.approx(-1.0, abs=1e-15)
    assert b["HH"][0, 0] == pytest.approx(0.0, abs=1e-15)


def test_elementary_patterns_land_in_one_band():
    H, W, c = 6, 8, 0.7
    y, x = np.mgrid[0:H, 0:W]
    pats = {"LL": np.full((H, W), c), "LH": c * (-1.0) ** y, "HL": c * (-1.0) ** x,
            "HH": c * (-1.0) ** (x + y)}
    for band, img in pats.items():
        b = fdo.dwt(img)
        for k in b:
            expect = 2.0 * c if k == band else 0.0
            np.testing.assert_allclose(np.abs(b[k]), expect, atol=1e-14, err_msg=(band, k))


@pytest.mark.parametrize("H,W", [(2, 2), (6, 10), (7, 5), (1, 3), (33, 64)])
def test_parseval_reconstruction_and_adjoint(H, W):
    rng = np.random.default_rng(H * 100 + W)
    x = rng.normal(size=(2, 3, H, W))
    b = fdo.dwt(x)
    energy = sum(np.sum(v ** 2) for v in b.values())
    assert energy == pytest.approx(np.sum(x ** 2), rel=1e-13)
    np.testing.assert_allclose(fdo.dwt_adjoint(b, x.shape), x, atol=1e-13)
    # <DWT x, y> = <x, DWT* y> band by band
    y = {k: rng.normal(size=v.shape) for k, v in b.items()}
    lhs = sum(np.sum(b[k] * y[k]) for k in b)
    rhs = np.sum(x * fdo.dwt_adjoint(y, x.shape))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_loss_closed_forms():
    H, W, d = 8, 12, 0.3
    tgt = np.random.default_rng(1).normal(size=(1, 3, H, W))
    y, x = np.mgrid[0:H, 0:W]
    r = fdo.fdo_losses(tgt + d, tgt)  # constant residual: LL = 2d only
    assert r["low"] == pytest.approx(4 * d * d, rel=1e-12)
    assert r["high"] == pytest.approx(0.0, abs=1e-20)
    r = fdo.fdo_losses(tgt + d * (-1.0) ** (x + y), tgt)  # checkerboard: HH = 2d only
    assert r["low"] == pytest.approx(0.0, abs=1e-20)
    assert r["high"] == pytest.approx(4 * d * d, rel=1e-12)


@pytest.mark.parametrize("H,W", [(4, 6), (5, 7)])
def test_cotangents_match_finite_differences(H, W):
    rng = np.random.default_rng(3)
    ren = rng.normal(size=(1, 3, H, W))
    tgt = rng.normal(size=(1, 3, H, W))
    lo, hi = 0.2, 0.4
    r = fdo.fdo_losses(ren, tgt, lo, hi)
    eps = 1e-6
    for idx in [(0, 0, 0, 0), (0, 1, H - 1, W - 1), (0, 2, H // 2, 1), (0, 0, 1, W // 2)]:
        a = ren.copy(); a[idx] += eps
        b = ren.copy(); b[idx] -= eps
        ra, rb = fdo.fdo_losses(a, tgt, lo, hi), fdo.fdo_losses(b, tgt, lo, hi)
        assert lo * (ra["low"] - rb["low"]) / (2 * eps) == pytest.approx(r["grad_low"][idx], rel=1e-6, abs=1e-10)
        assert hi * (ra["high"] - rb["high"]) / (2 * eps) == pytest.approx(r["grad_high"][idx], rel=1e-6, abs=1e-10)


def test_cotangents_sum_to_the_plain_residual():
    # LL and the three detail bands partition the image orthonormally and
    # have the same size, so g_low/l_low + g_high/l_high = 2 (I^ - I) / n_band
    rng = np.random.default_rng(4)
    ren = rng.normal(size=(2, 3, 9, 14))
    tgt = rng.normal(size=(2, 3, 9, 14))
    r = fdo.fdo_losses(ren, tgt, 0.2, 0.4)
    n_band = 2 * 3 * 5 * 7
    np.testing.assert_allclose(r["grad_low"] / 0.2 + r["grad_high"] / 0.4,
                               2.0 * (ren - tgt) / n_band, atol=1e-13)


def test_projection_worked_example():
    gc = np.zeros((2, 2))
    gl = np.array([[1.0, 0.0], [1.0, 0.0]])
    gh = np.array([[-1.0, 1.0], [-1.0, 1.0]])
    r = fdo.fdo_project(np.array([0, 1]), gc, gl, gh)
    assert r["conflict"].tolist() == [True, True]
    np.testing.assert_allclose(r["high"][0], [0.0, 1.0], atol=1e-15)  # 2D: g_high loses its g_low part
    np.testing.assert_allclose(r["low"][0], [1.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(r["low"][1], [0.5, 0.5], atol=1e-15)   # 3D: g_low loses its g_high part
    np.testing.assert_allclose(r["high"][1], [-1.0, 1.0], atol=1e-15)
    np.testing.assert_allclose(r["update"], [[1.0, 1.0], [-0.5, 1.5]], atol=1e-15)


def test_projection_properties():
    rng = np.random.default_rng(5)
    n, P = 2000, 59
    t = (rng.random(n) < 0.5).astype(np.uint8) * rng.integers(1, 3, n).astype(np.uint8)
    gc, gl, gh = (rng.normal(size=(n, P)) * rng.uniform(0.1, 10, (n, 1)) for _ in range(3))
    gl[:5] = 0.0  # zero vectors never conflict
    r = fdo.fdo_project(t, gc, gl, gh)
    dots = np.sum(gl * gh, 1)
    np.testing.assert_array_equal(r["conflict"], dots < 0)
    assert 0.3 < r["conflict"].mean() < 0.7
    c = r["conflict"]
    two = c & (t == 0)
    three = c & (t != 0)
    # the projected one is orthogonal to the kept one, which is unchanged
    assert np.abs(np.sum(r["high"][two] * gl[two], 1)).max() <= 1e-10 * np.max(np.abs(gl) ** 2) * P
    np.testing.assert_array_equal(r["low"][two], gl[two])
    assert np.abs(np.sum(r["low"][three] * gh[three], 1)).max() <= 1e-10 * np.max(np.abs(gh) ** 2) * P
    np.testing.assert_array_equal(r["high"][three], gh[three])
    # projection never lengthens; no conflict: identity
    assert (np.linalg.norm(r["high"][two], axis=1) <= np.linalg.norm(gh[two], axis=1) + 1e-12).all()
    np.testing.assert_array_equal(r["low"][~c], gl[~c])
    np.testing.assert_array_equal(r["high"][~c], gh[~c])
    np.testing.assert_allclose(r["update"], gc + r["low"] + r["high"], atol=0)
    # the update keeps the non-conflicting content: it equals the plain sum
    # minus the removed component along the kept vector
    plain = gc + gl + gh
    k2 = np.sum(gl[two] ** 2, 1)[:, None]
    np.testing.assert_allclose(r["update"][two], plain[two] - dots[two][:, None] / k2 * gl[two],
                               rtol=1e-12, atol=1e-12)


def test_orthogonal_gradients_are_not_a_conflict():
    gl = np.array([[1.0, 0.0, 0.0]])
    gh = np.array([[0.0, 2.0, 0.0]])
    r = fdo.fdo_project(np.array([0]), np.zeros((1, 3)), gl, gh)
    assert not r["conflict"][0]
    np.testing.assert_array_equal(r["update"], gl + gh)
