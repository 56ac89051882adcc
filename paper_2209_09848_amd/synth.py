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
    in the 2 x 2 pixels around a source on a pixel corner (Sec. 2.1 quotes
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
    (Sec. 2.2 shows up to +-0.15 px in Sector 5), referenced to frame 0."""
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
                        seed: int = 0):
    """FFI-shaped problem drawn on `device` with torch's seeded generator
    (for stacks too large to draw on the host quickly).  Returns
    (R tensor [T][H][W] float32 on device, sigma numpy, times, t_ref, vel, sources)."""
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
    vel = grid_speeds_directions(J_speeds, J_dirs, vmin, vmax)
    src = draw_sources(rng(config_id, 2, seed), n_sources, vel, H, W, times, t_ref,
                       amp[0], amp[1], min_sep=min(64.0, 0.25 * min(H, W)))
    if src:
        k, y, x, v = render_sources((T, H, W), times, t_ref, src)
        idx = (torch.from_numpy(k).to(device), torch.from_numpy(y).to(device),
               torch.from_numpy(x).to(device))
        R.index_put_(idx, torch.from_numpy(v.astype(np.float32)).to(device), accumulate=True)
    return R, sigma, times, t_ref, vel, src
