"""Brute force written from the paper's dense-filter form (Sec. 3.2): for each
hypothesis the filter F in R^{T x H x W} holds the PRF-weighted trajectory,
and the score is the dot product of F with the inverse-variance-weighted data
(eq. 4).  Independent of the oracle: its own offsets, profiles and loops, in
plain Python floats.  Only usable on tiny inputs."""
import math

import numpy as np


def anchor_phase(v, dt, th=0.0):
    d = v * dt + th
    a = math.floor(d + 0.5)
    return a, d - a


def profile(f, sigma_px, stamp, integrated=False):
    h = stamp // 2
    g = []
    for b in range(-h, h + 1):
        if integrated:
            lo = (b - 0.5 - f) / sigma_px
            hi = (b + 0.5 - f) / sigma_px
            g.append(0.5 * (math.erf(hi / math.sqrt(2)) - math.erf(lo / math.sqrt(2))))
        else:
            g.append(math.exp(-0.5 * ((b - f) / sigma_px) ** 2))
    s = sum(g)
    return [x / s for x in g]


def table_read(tab, q, stamp, uy, ux):
    """Tabulated PRF at offset (uy, ux): grid u = -(h+1) + i/q, read between
    the four surrounding grid points with weights linear in each axis."""
    r = stamp // 2 + 1
    py, px = (uy + r) * q, (ux + r) * q
    i, m = int(math.floor(py)), int(math.floor(px))
    sy, sx = py - i, px - m
    return ((1 - sy) * (1 - sx) * tab[i][m] + (1 - sy) * sx * tab[i][m + 1]
            + sy * (1 - sx) * tab[i + 1][m] + sy * sx * tab[i + 1][m + 1])


def dense_filter(j, y0, x0, T, H, W, times, t_ref, vel, sigma_px, stamp, integrated=False,
                 table=None, q=0, jitter=None):
    F = np.zeros((T, H, W))
    h = stamp // 2
    for k in range(T):
        thx, thy = (jitter[k][0], jitter[k][1]) if jitter is not None else (0.0, 0.0)
        ax, fx = anchor_phase(vel[j][0], times[k] - t_ref, thx)
        ay, fy = anchor_phase(vel[j][1], times[k] - t_ref, thy)
        if table is None:
            gx = profile(fx, sigma_px, stamp, integrated)
            gy = profile(fy, sigma_px, stamp, integrated)
        for a in range(-h, h + 1):
            for b in range(-h, h + 1):
                Y, X = y0 + ay + a, x0 + ax + b
                if 0 <= Y < H and 0 <= X < W:
                    if table is None:
                        F[k, Y, X] = gy[a + h] * gx[b + h]
                    else:
                        F[k, Y, X] = table_read(table, q, stamp, a - fy, b - fx)
    return F


def ivar_map(sigma):
    s = np.asarray(sigma, np.float64)
    ok = np.isfinite(s) & (s > 0)
    return np.where(ok, 1.0 / np.where(ok, s, 1.0) ** 2, 0.0)


def search(R, sigma, times, t_ref, vel, sigma_px=0.7, stamp=5, integrated=False, table=None,
           q=0, jitter=None):
    T, H, W = R.shape
    J = len(vel)
    iv = ivar_map(sigma)
    D = np.asarray(R, np.float64) * iv[None]
    nu = np.zeros((J, H, W))
    lam = np.zeros((J, H, W))
    for j in range(J):
        for y0 in range(H):
            for x0 in range(W):
                F = dense_filter(j, y0, x0, T, H, W, times, t_ref, vel, sigma_px, stamp,
                                 integrated, table, q, jitter)
                nu[j, y0, x0] = float(np.sum(F * D))
                lam[j, y0, x0] = float(np.sum(F * F * iv[None]))
    return nu, lam
