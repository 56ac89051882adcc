"""Pins of the background re-fit oracle (Sec. 3.1 eq. 1-3; Sec. 3.2 noise
model).  Each ties the oracle to something other than itself: torch's
bilinear resize, numpy's least squares, scipy's minimiser of the Huber loss,
the estimating equation of the Huber fit, exact models, and hand-checkable
noise/clipping cases."""
import math

import numpy as np
import pytest
import torch
from scipy import optimize

from oracle import refit


@pytest.mark.parametrize("ny,nx,H,W", [(16, 16, 64, 64), (7, 5, 50, 33), (1, 3, 9, 9), (8, 8, 8, 8)])
def test_upsample_is_torch_bilinear_half_pixel(ny, nx, H, W):
    g = np.random.default_rng(1)
    S = g.standard_normal((3, ny, nx))
    ref = torch.nn.functional.interpolate(torch.from_numpy(S)[None], size=(H, W), mode="bilinear",
                                          align_corners=False)[0].numpy()
    np.testing.assert_allclose(refit.upsample(S, H, W), ref, rtol=1e-12, atol=1e-12)


def test_upsample_reproduces_constants_and_interior_planes():
    S = np.full((2, 6, 6), 3.25)
    assert np.all(refit.upsample(S, 48, 48) == 3.25)
    # a plane in grid-point coordinates is reproduced between the outer grid points
    ny = nx = 8
    H = W = 64
    a = np.arange(ny)
    S = (2.0 * a[:, None] - 0.5 * a[None, :])[None].astype(np.float64)
    U = refit.upsample(S, H, W)[0]
    py = (np.arange(H) + 0.5) * ny / H - 0.5
    px = (np.arange(W) + 0.5) * nx / W - 0.5
    inner = (py >= 0) & (py <= ny - 1)
    innerx = (px >= 0) & (px <= nx - 1)
    plane = 2.0 * py[:, None] - 0.5 * px[None, :]
    np.testing.assert_allclose(U[np.ix_(inner, innerx)], plane[np.ix_(inner, innerx)], atol=1e-12)


def test_upsample_at_selected_pixels_matches_the_full_map():
    g = np.random.default_rng(3)
    S = g.standard_normal((4, 6, 9))
    full = refit.upsample(S, 41, 77)
    ys, xs = g.integers(0, 41, 30), g.integers(0, 77, 30)
    np.testing.assert_array_equal(refit.upsample_at(S, 41, 77, ys, xs), full[:, ys, xs])


def _problem(seed, T=60, H=5, W=7, outliers=0.0, noise=0.3):
    g = np.random.default_rng(seed)
    jit = np.column_stack([0.15 * np.sin(np.arange(T) / 7.0) + 0.05 * g.standard_normal(T),
                           0.12 * np.cos(np.arange(T) / 11.0) + 0.05 * g.standard_normal(T)])
    X = refit.basis(jit)
    beta = g.standard_normal((6, H * W)) * np.array([[50.0], [5.0], [5.0], [2.0], [2.0], [2.0]])
    S = g.standard_normal((T, 2, 3))
    U = refit.upsample(S, H, W).reshape(T, H * W)
    D = U + X @ beta + noise * g.standard_normal((T, H * W))
    if outliers:
        hit = g.random((T, H * W)) < outliers
        D = D + hit * g.uniform(20, 200, (T, H * W))
    return D.reshape(T, H, W), S, jit, beta.reshape(6, H, W)


def test_zero_rounds_is_least_squares():
    D, S, jit, _ = _problem(2)
    beta, resid = refit.refit(D, S, jit, delta=1.0, iterations=0)
    T, H, W = D.shape
    y = (D - refit.upsample(S, H, W)).reshape(T, -1)
    ls, *_ = np.linalg.lstsq(refit.basis(jit), y, rcond=None)
    np.testing.assert_allclose(beta.reshape(6, -1), ls, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(resid.reshape(T, -1), y - refit.basis(jit) @ ls, atol=1e-9)


def test_exact_model_is_recovered():
    D, S, jit, beta_true = _problem(3, noise=0.0)
    beta, resid = refit.refit(D, S, jit, delta=0.5, iterations=5)
    np.testing.assert_allclose(beta, beta_true, rtol=1e-9, atol=1e-8)
    assert np.abs(resid).max() < 1e-8


def test_no_clipping_keeps_least_squares():
    D, S, jit, _ = _problem(4, outliers=0.05)
    b0, _ = refit.refit(D, S, jit, delta=math.inf, iterations=0)
    b5, _ = refit.refit(D, S, jit, delta=math.inf, iterations=5)
    np.testing.assert_allclose(b5, b0, rtol=1e-12, atol=1e-9)


def test_converged_rounds_minimise_the_huber_loss():
    """Many rounds reach the minimiser of eq. 3's loss that scipy finds, and
    satisfy the Huber estimating equation sum_t x_t psi(r_t) = 0."""
    D, S, jit, _ = _problem(5, T=80, H=2, W=3, outliers=0.08)
    delta = 0.4
    beta, resid = refit.refit(D, S, jit, delta=delta, iterations=400)
    T, H, W = D.shape
    X = refit.basis(jit)
    y = (D - refit.upsample(S, H, W)).reshape(T, -1)
    for p in range(H * W):
        f = lambda b: float(refit.huber_loss(y[:, p] - X @ b, delta).sum())
        jac = lambda b: -X.T @ np.clip(y[:, p] - X @ b, -delta, delta)
        b0 = np.linalg.lstsq(X, y[:, p], rcond=None)[0]
        res = optimize.minimize(f, b0, jac=jac, method="BFGS", options={"gtol": 1e-11, "maxiter": 10000})
        bp = beta.reshape(6, -1)[:, p]
        assert f(bp) <= res.fun + 1e-9 * max(1.0, res.fun)
        np.testing.assert_allclose(bp, res.x, rtol=1e-5, atol=1e-5)
        psi = np.clip(resid.reshape(T, -1)[:, p], -delta, delta)
        assert np.abs(X.T @ psi).max() < 1e-8 * T
    # outliers pull least squares; the Huber fit has lower loss than it
    b_ls = np.linalg.lstsq(X, y, rcond=None)[0]
    assert refit.huber_loss(y - X @ b_ls, delta).sum() > refit.huber_loss(y - X @ beta.reshape(6, -1), delta).sum()


def test_each_round_lowers_the_loss():
    D, S, jit, _ = _problem(6, outliers=0.1)
    T, H, W = D.shape
    X = refit.basis(jit)
    y = (D - refit.upsample(S, H, W)).reshape(T, -1)
    prev = np.inf
    for it in range(6):
        beta, _ = refit.refit(D, S, jit, delta=0.5, iterations=it)
        loss = refit.huber_loss(y - X @ beta.reshape(6, -1), 0.5).sum()
        assert loss <= prev + 1e-9
        prev = loss


def test_huber_loss_closed_form():
    # eq. 3: continuous at |a| = delta, slope delta beyond
    d = 1.5
    assert refit.huber_loss(1.5, d) == pytest.approx(0.5 * 1.5 ** 2)
    assert refit.huber_loss(-4.0, d) == pytest.approx(1.5 * (4.0 - 0.75))
    assert refit.huber_loss(0.3, d) == pytest.approx(0.045)


def test_noise_model_hand_case():
    """99 residuals of +-1 and one of 10 in the kept pixel.  No rounds:
    sigma0 = sqrt((99 + 100) / 100) = 1.41; a 3-sigma clip zeroes the 10.
    One round: the 10 lies beyond 3 x 1.41, so sigma0 = sqrt(99/99) = 1 and
    stays there.  A bright pixel is masked whatever its residuals."""
    T = 100
    resid = np.ones((T, 1, 2))
    resid[::2, 0, 0] = -1.0
    resid[17, 0, 0] = 10.0
    resid[:, 0, 1] = 7.0
    beta = np.zeros((6, 1, 2))
    beta[0, 0, 1] = 1e4
    R, sigma, s0, nc, nm = refit.noise_and_clip(resid, beta, 5e3, 3.0, sigma_rounds=0)
    assert s0 == pytest.approx(math.sqrt(1.99), rel=1e-15)
    assert nc == 1 and nm == 1
    assert R[17, 0, 0] == 0.0 and np.count_nonzero(R[:, 0, 0]) == 99
    assert np.all(R[:, 0, 1] == 0.0)
    assert sigma[0, 0] == pytest.approx(math.sqrt(1.99)) and sigma[0, 1] == 0.0
    for rounds in (1, 4):
        R, sigma, s0, nc, nm = refit.noise_and_clip(resid, beta, 5e3, 3.0, sigma_rounds=rounds)
        assert s0 == 1.0 and nc == 1 and sigma[0, 0] == 1.0


def test_sigma_rounds_recover_gaussian_sigma_under_outliers():
    """Unit Gaussian samples with 0.5% gross outliers: the plain rms is far
    off, three clipped rounds at kappa = 5 recover sigma within 1% (a 5-sigma
    truncation lowers a Gaussian rms by under 1e-4)."""
    g = np.random.default_rng(9)
    r = g.standard_normal((4000, 1, 50))
    hit = g.random(r.shape) < 0.005
    r = r + hit * g.uniform(50, 500, r.shape)
    beta = np.zeros((6, 1, 50))
    _, _, s_plain, _, _ = refit.noise_and_clip(r, beta, np.inf, 5.0, sigma_rounds=0)
    R, _, s3, nc, _ = refit.noise_and_clip(r, beta, np.inf, 5.0, sigma_rounds=3)
    assert s_plain > 5.0
    assert abs(s3 - 1.0) < 0.01
    assert abs(nc - hit.sum()) <= 0.01 * hit.sum() + 5


def test_singular_basis_is_rejected():
    T, H, W = 10, 2, 2
    D = np.zeros((T, H, W))
    with pytest.raises(np.linalg.LinAlgError):
        refit.refit(D, None, np.zeros((T, 2)), 1.0, 1)
