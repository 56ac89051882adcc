"""Seeded synthetic inputs shaped like the paper's TESS workloads.

This module generates data only: noise, per-pixel sigma maps, frame times,
trajectory banks and moving point sources drawn onto the stack by the forward
model (a moving object adds its flux times the PRF along its path; Sec. 2 and
Sec. 4.1, where injection adds "a filter times a flux").  It holds none of the
search's arithmetic and imports neither the search library nor the oracle;
both consume what it produces.

Conventions (the paper is silent on them):
* stack layout [T][H][W], x = column, y = row, pixel centres at integers;
* times in days (TESS-like epoch 2000.0, 30-minute cadence = 48 frames/day,
  Sec. 2); velocities in pixels per day; a config's "px/frame" is x48;
* seeds come from numpy.random.SeedSequence([2209, config_id, stream]) with
  stream 0 = sigma map, 1 = noise, 2 = sources, 3 = arrivals.  Large stacks
  are drawn on the GPU with torch's seeded generator instead (same streams).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FRAMES_PER_DAY = 48.0
T0_DAYS = 2000.0


def rng(config_id: int, stream: int, sub: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([2209, config_id, stream, sub]))


# ---------------------------------------------------------------- frame times

def times_uniform(T: int, t0: float = T0_DAYS, per_day: float = FRAMES_PER_DAY) -> np.ndarray:
    return t0 + np.arange(T, dtype=np.float64) / per_day


def times_with_gap(T: int, gap_after: int, gap_days: float = 1.0, t0: float = T0_DAYS,
                   per_day: float = FRAMES_PER_DAY) -> np.ndarray:
    """Uniform cadence with one downlink gap (Sec. 3.2, Fig. 3's time jump):
    frame gap_after follows frame gap_after-1 by gap_days instead of one cadence."""
    t = times_uniform(T, t0, per_day)
    t[gap_after:] += gap_days - 1.0 / per_day
    return t


# ---------------------------------------------------------------- noise maps

def sigma_lognormal(g: np.random.Generator, H: int, W: int, dex: float = 0.3) -> np.ndarray:
    """Per-pixel sigma, log-normal with median 1 and the given scatter in dex."""
    return (10.0 ** (dex * g.standard_normal((H, W)))).astype(np.float32)


# ---------------------------------------------------------------- trajectory banks

def grid_c1() -> np.ndarray:
    """3x3 velocity grid around (0.12, -0.05) px/frame; j = 3*i_vx + i_vy."""
    v = [(vx, vy) for vx in (0.10, 0.12, 0.14) for vy in (-0.07, -0.05, -0.03)]
    return np.array(v, np.float64) * FRAMES_PER_DAY


def grid_speeds_directions(n_speed: int = 10, n_dir: int = 10, vmin: float = 0.01,
                           vmax: float = 0.2) -> np.ndarray:
    """Speeds vmin*(vmax/vmin)^(m/(n_speed-1)) px/frame at directions d*360/n_dir
    degrees; j = n_dir*m + d."""
    out = []
    for m in range(n_speed):
        s = vmin * (vmax / vmin) ** (m / max(n_speed - 1, 1))
        for d in range(n_dir):
            th = math.radians(d * 360.0 / n_dir)
            out.append((s * math.cos(th), s * math.sin(th)))
    return np.array(out, np.float64) * FRAMES_PER_DAY


SHELLS_C4 = (512, 384, 320, 256, 192, 160, 128, 96)


def grid_shells(counts=SHELLS_C4, vfast: float = 0.3, vslow: float = 0.005,
                max_incl_deg: float = 60.0):
    """Uneven shells of trajectories (distance labels 30..300 AU; speeds
    geometric vfast..vslow px/frame).  Per shell: 4 speeds in [0.9,1.1]*v_s
    times n/4 directions spread evenly over [0, max_incl] degrees from the row
    axis.  Returns (vel [J][2] px/day, shell id [J])."""
    n = len(counts)
    vel, shell = [], []
    for i, c in enumerate(counts):
        vs = vfast * (vslow / vfast) ** (i / max(n - 1, 1))
        n_ang = max(c // 4, 1)
        for f in np.linspace(0.9, 1.1, 4):
            for a in np.linspace(0.0, max_incl_deg, n_ang):
                th = math.radians(a)
                vel.append((f * vs * math.cos(th), -f * vs * math.sin(th)))
                shell.append(i)
    return np.array(vel, np.float64) * FRAMES_PER_DAY, np.array(shell, np.int32)


# ---------------------------------------------------------------- moving sources

@dataclass
class Source:
    x: float          # column at t_ref
    y: float          # row at t_ref
    vx: float         # px/day
    vy: float         # px/day
    amp: float        # total in-stamp flux per frame (sigma units)
    traj: int = -1    # index of the bank trajectory it was drawn from, if any


def _prf_1d(offsets: np.ndarray, sigma_px: float, integrated: bool) -> np.ndarray:
    """Gaussian pixel response of a point at offset 0 seen by pixels at `offsets`."""
    if integrated:
        r2 = 1.0 / math.sqrt(2.0)
        lo = (offsets - 0.5) / sigma_px * r2
        hi = (offsets + 0.5) / sigma_px * r2
        from scipy.special import erf
        return 0.5 * (erf(hi) - erf(lo))
    return np.exp(-0.5 * (offsets / sigma_px) ** 2)


def render_sources(shape, times, t_ref, sources, sigma_px: float = 0.7, stamp: int = 5,
                   integrated: bool = False, jitter=None, psf=None):
    """Forward model of moving point sources: per frame, each source deposits
    amp * PRF on the stamp of pixels nearest its position (moved by the
    frame's pointing jitter [T][2] = (theta_x, theta_y) if given).  With the
    Gaussian PRF the stamp's response is normalised to unit sum; a `psf`
    object (see TabulatedPSF) gives each pixel's share as is.  Returns
    (k, y, x, value) arrays of the contributions that fall on the image
    (float64 values)."""
    T, H, W = shape
    h = stamp // 2
    ks, ys, xs, vs = [], [], [], []
    taps = np.arange(-h, h + 1, dtype=np.float64)
    for s in sources:
        for k in range(T):
            dt = float(times[k]) - t_ref
            px = s.x + s.vx * dt
            py = s.y + s.vy * dt
            if jitter is not None:
                px += float(jitter[k][0])
                py += float(jitter[k][1])
            cx = math.floor(px + 0.5)
            cy = math.floor(py + 0.5)
            if psf is not None:
                share = psf.pixel_share(taps[:, None] - (py - cy), taps[None, :] - (px - cx))
            else:
                rx = _prf_1d(taps - (px - cx), sigma_px, integrated)
                ry = _prf_1d(taps - (py - cy), sigma_px, integrated)
                share = np.outer(ry / ry.sum(), rx / rx.sum())
            for a in range(stamp):
                Y = cy - h + a
                if Y < 0 or Y >= H:
                    continue
                for b in range(stamp):
                    X = cx - h + b
                    if X < 0 or X >= W:
                        continue
                    ks.append(k)
                    ys.append(Y)
                    xs.append(X)
                    vs.append(s.amp * share[a, b])
    return (np.array(ks, np.int64), np.array(ys, np.int64), np.array(xs, np.int64),
            np.array(vs, np.float64))


def add_sources(R: np.ndarray, times, t_ref, sources, **kw) -> np.ndarray:
    """R (float64 or float32 [T][H][W]) plus the rendered sources, in float64."""
    out = np.array(R, dtype=np.float64, copy=True)
    k, y, x, v = render_sources(out.shape, times, t_ref, sources, **kw)
    np.add.at(out, (k, y, x), v)
    return out


def draw_sources(g: np.random.Generator, n: int, vel: np.ndarray, H: int, W: int, times,
                 t_ref: float, amp_lo: float, amp_hi: float, min_sep: float = 64.0,
                 margin: float = 3.0, max_tries: int = 100000):
    """n sources on random bank trajectories, sub-pixel starts chosen so the
    whole trail stays `margin` px inside the frame, starts >= min_sep apart."""
    t = np.asarray(times, np.float64)
    dts = np.array([t.min() - t_ref, t.max() - t_ref])
    out = []
    tries = 0
    while len(out) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place sources")
        j = int(g.integers(0, vel.shape[0]))
        vx, vy = vel[j]
        ex = vx * dts
        ey = vy * dts
        xlo, xhi = margin - min(ex.min(), 0.0), W - 1 - margin - max(ex.max(), 0.0)
        ylo, yhi = margin - min(ey.min(), 0.0), H - 1 - margin - max(ey.max(), 0.0)
        if xlo >= xhi or ylo >= yhi:
            continue
        x = float(g.uniform(xlo, xhi))
        y = float(g.uniform(ylo, yhi))
        if any((x - s.x) ** 2 + (y - s.y) ** 2 < min_sep ** 2 for s in out):
            continue
        out.append(Source(x, y, float(vx), float(vy), float(g.uniform(amp_lo, amp_hi)), j))
    return out


# ---------------------------------------------------------------- tabulated PRF and jitter

class TabulatedPSF:
    """A non-separable, slightly asymmetric point-spread function standing in
    for the TESS PRF model files (not available here): an elliptical Gaussian
    core, rotated off the pixel axes, plus a fainter displaced halo, both of
    unit integral.  `pixel_share(dy, dx)` is the fraction of a point source's
    flux that a pixel whose centre lies at offset (dy, dx) from the source
    records (midpoint rule over sub x sub points per pixel).  With the default
    shape 49% of the flux lands in the peak pixel of a centred source and 87%
    in the 2 x 2 pixels around a source on a pixel corner (Sec. 2 quotes
    about 50% and 90% for TESS)."""

    def __init__(self, core=(0.5, 0.38), angle_deg=35.0, halo_frac=0.15, halo_sigma=1.1,
                 halo_offset=(0.15, -0.1), sub=12):
        self.sa, self.sb = core
        self.th = math.radians(angle_deg)
        self.hf, self.hs = halo_frac, halo_sigma
        self.hoy, self.hox = halo_offset
        self.sub = sub

    def density(self, y, x):
        c, s = math.cos(self.th), math.sin(self.th)
        u = c * x + s * y
        v = -s * x + c * y
        core = np.exp(-0.5 * ((u / self.sa) ** 2 + (v / self.sb) ** 2)) / (2 * math.pi * self.sa * self.sb)
        yy, xx = y - self.hoy, x - self.hox
        halo = np.exp(-0.5 * (xx * xx + yy * yy) / self.hs ** 2) / (2 * math.pi * self.hs ** 2)
        return (1.0 - self.hf) * core + self.hf * halo

    def pixel_share(self, dy, dx):
        dy, dx = np.broadcast_arrays(np.asarray(dy, np.float64), np.asarray(dx, np.float64))
        n = self.sub
        o = (np.arange(n) + 0.5) / n - 0.5
        y = dy[..., None, None] + o[:, None]
        x = dx[..., None, None] + o[None, :]
        return self.density(y, x).mean(axis=(-1, -2))

    def table(self, stamp: int, q: int) -> np.ndarray:
        """pixel_share on the grid -(h+1) .. h+1 in steps of 1/q, [n][n], rows
        along y: the layout of a tabulated PRF."""
        h = stamp // 2
        u = -(h + 1) + np.arange((stamp + 1) * q + 1, dtype=np.float64) / q
        return self.pixel_share(u[:, None], u[None, :])


def jitter_series(g: np.random.Generator, T: int, amp: float = 0.15) -> np.ndarray:
    """Per-frame pointing jitter [T][2] = (theta_x, theta_y) in pixels: a
    smoothed random walk per axis, scaled so its largest excursion is `amp`
    (Sec. 2.1 shows up to +-0.15 px in Sector 5), referenced to frame 0."""
    out = np.zeros((T, 2))
    for ax in range(2):
        w = np.cumsum(g.standard_normal(T))
        k = max(1, T // 50)
        w = np.convolve(w, np.ones(k) / k, mode="same") + 0.3 * g.standard_normal(T)
        w = w - w[0]
        m = np.abs(w).max()
        out[:, ax] = w * (amp / m) if m > 0 else 0.0
    return out


# ---------------------------------------------------------------- configurations

@dataclass
class Problem:
    """One search problem: host arrays plus its metadata."""
    name: str
    R: np.ndarray            # [T][H][W] float32
    sigma: np.ndarray        # [H][W] float32
    times: np.ndarray        # [T] float64
    t_ref: float
    vel: np.ndarray          # [J][2] float64, px/day
    sigma_px: float = 0.7
    stamp: int = 5
    prf_kind: int = 0        # 0 sampled, 1 pixel-integrated
    top_k: int = 10
    sources: list = field(default_factory=list)


def make_c1(variant: str = "noisy", seed_sub: int = 0) -> Problem:
    """64x64 px x 50 frames, sigma = 1, iid N(0,1) residuals, uniform 30-min
    cadence, one source (A = 0.5; 4 for 'bright'; no noise for 'noise_free')
    at (x, y) = (20.3, 31.7) moving (0.12, -0.05) px/frame; 3x3 velocity grid."""
    H = W = 64
    T = 50
    times = times_uniform(T)
    t_ref = float(times[0])
    sigma = np.ones((H, W), np.float32)
    if variant == "noise_free":
        noise = np.zeros((T, H, W))
    else:
        noise = rng(1, 1, seed_sub).standard_normal((T, H, W))
    amp = 4.0 if variant == "bright" else 0.5
    src = [Source(20.3, 31.7, 0.12 * FRAMES_PER_DAY, -0.05 * FRAMES_PER_DAY, amp, 4)]
    R = add_sources(noise, times, t_ref, src).astype(np.float32)
    return Problem("c1_" + variant, R, sigma, times, t_ref, grid_c1(), top_k=10, sources=src)


def make_ffi_like(H: int, W: int, T: int, J_speeds: int = 10, J_dirs: int = 10,
                  n_sources: int = 30, amp=(0.05, 0.5), config_id: int = 2,
                  gap: bool = True, dex: float = 0.3, top_k: int = 100,
                  vmin: float = 0.01, vmax: float = 0.2) -> Problem:
    """FFI-shaped problem on the host (numpy): log-normal sigma (median 1,
    `dex` scatter), R = sigma*N(0,1) plus sources, a 1-day downlink gap half
    way, a speeds x directions bank.  Host memory ~ 12*T*H*W bytes."""
    times = times_with_gap(T, T // 2) if gap else times_uniform(T)
    t_ref = float(times[0])
    sigma = sigma_lognormal(rng(config_id, 0), H, W, dex)
    g = rng(config_id, 1)
    R = np.empty((T, H, W), np.float32)
    for k in range(T):
        R[k] = (sigma.astype(np.float64) * g.standard_normal((H, W))).astype(np.float32)
    vel = grid_speeds_directions(J_speeds, J_dirs, vmin, vmax)
    src = draw_sources(rng(config_id, 2), n_sources, vel, H, W, times, t_ref, amp[0], amp[1],
                       min_sep=min(64.0, 0.25 * min(H, W)))
    k, y, x, v = render_sources(R.shape, times, t_ref, src)
    lin = (k * H + y) * W + x
    uniq, inv = np.unique(lin, return_inverse=True)
    add = np.zeros(uniq.shape[0], np.float64)
    np.add.at(add, inv, v)      # trails may cross: sum coincident deposits first
    flat = R.reshape(-1)
    flat[uniq] = (flat[uniq].astype(np.float64) + add).astype(np.float32)
    return Problem("ffi_%dx%dx%d" % (H, W, T), R, sigma, times, t_ref, vel, top_k=top_k,
                   sources=src)


def make_ffi_like_torch(H: int, W: int, T: int, device, J_speeds: int = 10, J_dirs: int = 10,
                        n_sources: int = 30, amp=(0.05, 0.5), config_id: int = 2,
                        dex: float = 0.3, vmin: float = 0.01, vmax: float = 0.2,
                        seed: int = 0, bank=None):
    """FFI-shaped problem drawn on `device` with torch's seeded generator
    (for stacks too large to draw on the host quickly); `bank` replaces the
    speeds x directions grid.  Returns (R tensor [T][H][W] float32 on
    device, sigma numpy, times, t_ref, vel, sources)."""
    import torch
    times = times_with_gap(T, T // 2)
    t_ref = float(times[0])
    sigma = sigma_lognormal(rng(config_id, 0), H, W, dex)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(np.random.SeedSequence([2209, config_id, 1, seed]).generate_state(1)[0]))
    sig_t = torch.from_numpy(sigma).to(device)
    R = torch.empty((T, H, W), dtype=torch.float32, device=device)
    for k0 in range(0, T, 64):
        k1 = min(T, k0 + 64)
        R[k0:k1] = torch.randn((k1 - k0, H, W), generator=gen, device=device,
                               dtype=torch.float32) * sig_t
    vel = grid_speeds_directions(J_speeds, J_dirs, vmin, vmax) if bank is None else np.asarray(bank)
    src = draw_sources(rng(config_id, 2, seed), n_sources, vel, H, W, times, t_ref,
                       amp[0], amp[1], min_sep=min(64.0, 0.25 * min(H, W)))
    if src:
        k, y, x, v = render_sources((T, H, W), times, t_ref, src)
        idx = (torch.from_numpy(k).to(device), torch.from_numpy(y).to(device),
               torch.from_numpy(x).to(device))
        R.index_put_(idx, torch.from_numpy(v.astype(np.float32)).to(device), accumulate=True)
    return R, sigma, times, t_ref, vel, src


# ---------------------------------------------------------------- raw frames for the background re-fit

def scattered_light_field(tt, y, x, H: int, W: int):
    """A smooth scattered-light pattern (a few broad glows whose brightness
    drifts over the sector), evaluated at times tt [T] (days from the first
    frame) and pixel coordinates y [..], x [..] (broadcast).  Works on numpy
    arrays or torch tensors."""
    lib = np if isinstance(y, np.ndarray) else __import__("torch")
    L = float(max(H, W))
    out = 0.0
    for (cy, cx, s, a, per) in ((-0.3, 0.2, 0.6, 40.0, 13.7), (1.1, 0.9, 0.5, 25.0, 9.3),
                                (0.4, -0.4, 0.9, 15.0, 27.0)):
        g = lib.exp(-((y - cy * H) ** 2 + (x - cx * W) ** 2) / (2.0 * (s * L) ** 2))
        amp = a * (1.0 + 0.5 * lib.sin(2.0 * math.pi * tt / per))
        out = out + amp * g
    return out


def make_refit_problem(H: int, W: int, T: int, device="cpu", n_sl: int = 64,
                       n_stars: int | None = None, noise: float = 1.0,
                       cosmic_frac: float = 2e-4, n_streaks: int = 4, config_id: int = 7,
                       n_sources: int = 0, source_amp=(0.3, 1.0), J_speeds: int = 10,
                       J_dirs: int = 10, chunk: int = 64, source_min_speed: int = 0):
    """Raw TESS-like frames for the background re-fit (Sec. 3.1 eq. 1):
    smooth scattered light, a static sky with stars that move with the
    pointing jitter, Gaussian noise of standard deviation `noise`, cosmic-ray
    hits and a few fast asteroid streaks (the unmodelled transients of Sec.
    3.2), and optionally faint slow movers on bank trajectories (those of
    speed index >= source_min_speed).

    Returns dict: D (torch float32 [T][H][W] on `device`), S (numpy float32
    [T][n_sl][n_sl]: the scattered light sampled at the centres of an n_sl x
    n_sl grid of cells), jitter [T][2], times, t_ref, vel, sources, noise."""
    import torch
    times = times_with_gap(T, T // 2)
    t_ref = float(times[0])
    tt = times - times[0]
    jit = jitter_series(rng(config_id, 4), T, amp=0.15)
    g = rng(config_id, 5)
    if n_stars is None:
        n_stars = max(1, int(H * W / 800))
    sy = g.uniform(-3, H + 3, n_stars)
    sx = g.uniform(-3, W + 3, n_stars)
    sflux = noise * 10.0 ** g.uniform(1.0, 5.0, n_stars)
    # low-resolution samples of the scattered light at grid-cell centres
    gy = (np.arange(n_sl) + 0.5) * H / n_sl - 0.5
    gx = (np.arange(n_sl) + 0.5) * W / n_sl - 0.5
    S = scattered_light_field(tt[:, None, None], gy[None, :, None], gx[None, None, :], H, W)
    S = np.asarray(S, np.float32)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(np.random.SeedSequence([2209, config_id, 6]).generate_state(1)[0]))
    D = torch.empty((T, H, W), dtype=torch.float32, device=device)
    yy = torch.arange(H, device=device, dtype=torch.float64)[:, None]
    xx = torch.arange(W, device=device, dtype=torch.float64)[None, :]
    sky = 100.0 + 0.002 * yy - 0.001 * xx
    taps = torch.arange(-3, 4, device=device, dtype=torch.float64)
    sy_t = torch.from_numpy(sy).to(device)
    sx_t = torch.from_numpy(sx).to(device)
    sf_t = torch.from_numpy(sflux).to(device)
    r2 = 1.0 / math.sqrt(2.0)
    for k0 in range(0, T, chunk):
        k1 = min(T, k0 + chunk)
        n = k1 - k0
        tk = torch.from_numpy(tt[k0:k1]).to(device)[:, None, None]
        frame = scattered_light_field(tk, yy[None], xx[None], H, W) + sky[None]
        # stars at their jittered positions, Gaussian PSF (sigma 0.7) integrated over pixels
        jx = torch.from_numpy(jit[k0:k1, 0]).to(device)[:, None]
        jy = torch.from_numpy(jit[k0:k1, 1]).to(device)[:, None]
        px = sx_t[None] + jx
        py = sy_t[None] + jy
        cx = torch.floor(px + 0.5)
        cy = torch.floor(py + 0.5)
        def share(c, p):
            lo = (c[..., None] + taps - 0.5 - p[..., None]) / 0.7 * r2
            hi = (c[..., None] + taps + 0.5 - p[..., None]) / 0.7 * r2
            return 0.5 * (torch.erf(hi) - torch.erf(lo))
        wy = share(cy, py)                      # [n][stars][7]
        wx = share(cx, px)
        val = (sf_t[None, :, None, None] * wy[..., :, None] * wx[..., None, :])
        Y = (cy[..., None] + taps).long()[..., :, None].expand(val.shape)
        X = (cx[..., None] + taps).long()[..., None, :].expand(val.shape)
        K = torch.arange(n, device=device)[:, None, None, None].expand(val.shape)
        ok = (Y >= 0) & (Y < H) & (X >= 0) & (X < W)
        frame.index_put_((K[ok], Y[ok], X[ok]), val[ok], accumulate=True)
        frame += noise * torch.randn((n, H, W), generator=gen, device=device, dtype=torch.float64)
        hits = torch.rand((n, H, W), generator=gen, device=device) < cosmic_frac
        frame += hits * noise * (20.0 + 480.0 * torch.rand((n, H, W), generator=gen, device=device,
                                                            dtype=torch.float64))
        D[k0:k1] = frame.to(torch.float32)
    # fast asteroid streaks: bright, a few px per frame, over a stretch of frames
    for _ in range(n_streaks):
        k0 = int(g.integers(0, max(1, T - 40)))
        k1 = min(T, k0 + int(g.integers(10, 40)))
        y0, x0 = g.uniform(0, H), g.uniform(0, W)
        vy, vx = g.uniform(-6, 6), g.uniform(-6, 6)
        for k in range(k0, k1):
            yk, xk = int(round(y0 + vy * (k - k0))), int(round(x0 + vx * (k - k0)))
            if 0 <= yk < H and 0 <= xk < W:
                D[k, yk, xk] += float(noise * 300.0)
    vel = grid_speeds_directions(J_speeds, J_dirs)
    src = []
    if n_sources:
        j0 = source_min_speed * J_dirs
        src = draw_sources(rng(config_id, 2), n_sources, vel[j0:], H, W, times, t_ref,
                           source_amp[0], source_amp[1], min_sep=min(64.0, 0.25 * min(H, W)))
        for s_ in src:
            s_.traj += j0
        k, y, x, v = render_sources((T, H, W), times, t_ref, src, jitter=jit)
        D.index_put_((torch.from_numpy(k).to(device), torch.from_numpy(y).to(device),
                      torch.from_numpy(x).to(device)),
                     torch.from_numpy((v * noise).astype(np.float32)).to(device), accumulate=True)
    return {"D": D, "S": S, "jitter": jit, "times": times, "t_ref": t_ref, "vel": vel,
            "sources": src, "noise": noise}
