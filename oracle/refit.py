"""Plain FP64 oracle of the per-pixel background re-fit that produces the
residual stack and noise map the matched filter reads (arXiv:2209.09848,
Sec. 3.1 and Sec. 3.2).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg are the only callers; the product never imports this module.

What it computes, step by step in the paper's order:
  * the forward model of Sec. 3.1 eq. 1, D_t = U(S_t) + B + B_theta theta_t^k,
    with the scattered light S_t held fixed (Sec. 3.1: solved beforehand at
    low resolution, then kept fixed while B and B_theta are re-estimated at
    full resolution);
  * U: bilinear upsampling of the low-resolution scattered-light grid, each
    full-resolution pixel a weighted combination of the four nearest grid
    points (Sec. 3.1).  Reading: grid cells tile the image, so grid point
    (a, b) sits at pixel coordinate ((a + 1/2) H/n_y - 1/2, (b + 1/2) W/n_x
    - 1/2); positions outside the outermost grid points take the edge value;
  * the basis of frame t: (1, x_t, y_t, x_t^2, y_t^2, x_t y_t), the constant
    background and the second-order Taylor terms in the jitter theta_t =
    (x_t, y_t) (Sec. 3.1);
  * every pixel regressed on the same basis, so one Gram (normal) matrix
    inverse serves all pixels (Sec. 3.1);
  * the Huber loss of eq. 3 (1/2 a^2 inside +-delta_0, delta_0 (|a| -
    delta_0/2) outside) minimised by repeated least-squares solves, each on the
    data with its residuals clipped to +-delta_0 (Sec. 3.1, after Huber 1977).
    Reading: start from the least-squares fit; one round = residuals
    r = y - X beta, pseudo-data y* = X beta + clip(r, -delta_0, delta_0), new
    beta = the least-squares fit to y*; a fixed number of rounds;
  * the noise model of Sec. 3.2: pixels whose background is bright are set to
    0 (masked: sigma 0), the rest share one Gaussian standard deviation.
    Readings: "bright" = fitted background B above a caller's threshold; the
    common sigma is the root mean square of the remaining residuals (the
    maximum-likelihood sigma of a mean-zero Gaussian), made robust to the
    transients it must flag by iterated clipping: after the first estimate,
    each round recomputes it over the samples within a caller's multiple
    kappa of the previous estimate; finally the samples beyond kappa times
    it are set to 0 (the clipping of unmodelled transients that Sec. 3.2
    calls for).
"""
from __future__ import annotations

import numpy as np

N_BASIS = 6


def upsample_axis(n_in: int, n_out: int):
    """Indices (i0, i1) and weights (w0, w1) of the two grid points each
    output position reads along one axis."""
    scale = n_in / n_out
    src = (np.arange(n_out, dtype=np.float64) + 0.5) * scale - 0.5
    src = np.maximum(src, 0.0)
    i0 = np.floor(src).astype(np.int64)
    i0 = np.minimum(i0, n_in - 1)
    i1 = np.minimum(i0 + 1, n_in - 1)
    w1 = src - i0
    w1 = np.where(i1 == i0, 0.0, w1)
    return i0, i1, 1.0 - w1, w1


def upsample(S, H: int, W: int) -> np.ndarray:
    """U(S): [T][ny][nx] -> [T][H][W] by bilinear interpolation (FP64)."""
    S = np.asarray(S, np.float64)
    T, ny, nx = S.shape
    y0, y1, wy0, wy1 = upsample_axis(ny, H)
    x0, x1, wx0, wx1 = upsample_axis(nx, W)
    top = S[:, y0][:, :, x0] * wx0 + S[:, y0][:, :, x1] * wx1
    bot = S[:, y1][:, :, x0] * wx0 + S[:, y1][:, :, x1] * wx1
    return top * wy0[None, :, None] + bot * wy1[None, :, None]


def upsample_at(S, H: int, W: int, ys, xs) -> np.ndarray:
    """U(S) of an H x W image at the listed pixels only: [T][len(ys)]."""
    S = np.asarray(S, np.float64)
    T, ny, nx = S.shape
    y0, y1, wy0, wy1 = (v[np.asarray(ys)] for v in upsample_axis(ny, H))
    x0, x1, wx0, wx1 = (v[np.asarray(xs)] for v in upsample_axis(nx, W))
    top = S[:, y0, x0] * wx0 + S[:, y0, x1] * wx1
    bot = S[:, y1, x0] * wx0 + S[:, y1, x1] * wx1
    return top * wy0 + bot * wy1


def basis(jitter) -> np.ndarray:
    """X [T][6]: (1, x, y, x^2, y^2, x y) of each frame's jitter (x, y)."""
    j = np.asarray(jitter, np.float64)
    x, y = j[:, 0], j[:, 1]
    return np.column_stack([np.ones_like(x), x, y, x * x, y * y, x * y])


def huber_loss(a, delta):
    """Eq. 3: 1/2 a^2 for |a| <= delta, delta (|a| - delta/2) beyond."""
    a = np.abs(np.asarray(a, np.float64))
    return np.where(a <= delta, 0.5 * a * a, delta * (a - 0.5 * delta))


def refit(D, S, jitter, delta, iterations):
    """Per-pixel Huber fit of y = D - U(S) on the jitter basis.

    D [T][H][W], S [T][ny][nx] or None, jitter [T][2].  Returns
    (beta [6][H][W], residuals [T][H][W]) in FP64; residuals = y - X beta
    with the final beta."""
    D = np.asarray(D, np.float64)
    T, H, W = D.shape
    y = D - upsample(S, H, W) if S is not None else D.copy()
    y = y.reshape(T, H * W)
    X = basis(jitter)
    G = X.T @ X                                  # the shared Gram matrix
    Ginv = np.linalg.inv(G)
    beta = Ginv @ (X.T @ y)                      # least-squares start
    for _ in range(int(iterations)):
        r = y - X @ beta
        ystar = X @ beta + np.clip(r, -delta, delta)
        beta = Ginv @ (X.T @ ystar)              # least squares on the clipped data
    resid = y - X @ beta
    return beta.reshape(N_BASIS, H, W), resid.reshape(T, H, W)


def noise_and_clip(resid, beta, bright_threshold, clip_sigma, sigma_rounds=3):
    """Sec. 3.2 noise model on the fitted residuals.

    Returns (R [T][H][W] float64, sigma [H][W], sigma0, n_clipped, n_masked):
    bright pixels (B = beta[0] > bright_threshold) are 0 in R with sigma 0;
    sigma0 = sqrt(mean r^2) over the other pixels and all frames, then
    `sigma_rounds` times over those samples with |r| <= clip_sigma * sigma0;
    samples with |r| > clip_sigma * sigma0 are set to 0."""
    resid = np.asarray(resid, np.float64)
    mask = np.asarray(beta)[0] > bright_threshold
    keep = ~mask
    rk = resid[:, keep]
    sigma0 = float(np.sqrt(np.mean(rk ** 2))) if rk.size else 0.0
    for _ in range(int(sigma_rounds)):
        inside = rk[np.abs(rk) <= clip_sigma * sigma0]
        sigma0 = float(np.sqrt(np.mean(inside ** 2))) if inside.size else 0.0
    out = np.where(mask[None], 0.0, resid)
    big = (np.abs(resid) > clip_sigma * sigma0) & keep[None]
    out = np.where(big, 0.0, out)
    sigma = np.where(mask, 0.0, sigma0)
    return out, sigma, sigma0, int(big.sum()), int(mask.sum())


def pipeline(D, S, jitter, delta, iterations, bright_threshold, clip_sigma, sigma_rounds=3):
    """The whole re-fit: returns dict beta, resid (unclipped), R, sigma,
    sigma0, n_clipped, n_masked."""
    beta, resid = refit(D, S, jitter, delta, iterations)
    R, sigma, sigma0, nc, nm = noise_and_clip(resid, beta, bright_threshold, clip_sigma,
                                              sigma_rounds)
    return {"beta": beta, "resid": resid, "R": R, "sigma": sigma, "sigma0": sigma0,
            "n_clipped": nc, "n_masked": nm}
