"""Plain FP64 CPU oracle of the matched-filter trajectory search (arXiv:2209.09848).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg are the only callers.  The product (the HIP library and its Python
binding) never imports this package, and this package never imports the
product.  The heavy loops live in ``oracle.c`` (built here with gcc, FP64,
``-ffp-contract=off``); the reductions (Sec. 3.2 "maximum score across the
filter bank", Sec. 3.3 "scores above a threshold") are written out in numpy.

Definitions follow Sec. 3.2 (filter = trajectory line convolved with the PRF;
score = dot product of filter and data at every start pixel, eq. 4; the score
estimates the total flux) with the inverse-variance weighting that makes the
dot product the maximum-likelihood estimate under the Sec. 3.2 Gaussian noise
model:  SNR = nu / sqrt(Lam),  flux = nu / Lam  (0 where Lam = 0).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")

PRF_SAMPLED = 0
PRF_INTEGRATED = 1
PRF_TABLE = 2

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into _build/liboracle.so (gcc, FP64, no contraction)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-std=c99", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.POINTER
            d, i32 = ctypes.c_double, ctypes.c_int32
            lib.oracle_offset.argtypes = [d, d, d, P(i32), P(d)]
            lib.oracle_profile.argtypes = [ctypes.c_int, d, ctypes.c_int, d, P(d)]
            lib.oracle_weights.argtypes = [ctypes.c_int, d, ctypes.c_int, P(d), ctypes.c_int,
                                           d, d, P(d)]
            lib.oracle_offsets.argtypes = [ctypes.c_int, P(d), d, ctypes.c_int, P(d), P(d),
                                           P(i32), P(i32), P(d), P(d)]
            lib.oracle_search.argtypes = [ctypes.c_int] * 3 + [P(ctypes.c_float)] * 2 + \
                [P(d), d, ctypes.c_int, P(d), P(d), ctypes.c_int, d, ctypes.c_int, P(d),
                 ctypes.c_int] + [ctypes.c_int] * 4 + [P(d), P(d)]
            lib.oracle_search.restype = ctypes.c_int
            lib.oracle_hypotheses.argtypes = [ctypes.c_int] * 3 + [P(ctypes.c_float)] * 2 + \
                [P(d), d, ctypes.c_int, P(d), P(d), ctypes.c_int, d, ctypes.c_int, P(d),
                 ctypes.c_int, ctypes.c_int, P(i32), P(i32), P(i32), P(d), P(d)]
            lib.oracle_hypotheses.restype = ctypes.c_int
            lib.oracle_threads.restype = ctypes.c_int
            lib.oracle_set_threads.argtypes = [ctypes.c_int]
            lib.oracle_set_threads.restype = None
            _lib = lib
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def threads() -> int:
    """OpenMP threads the oracle runs with."""
    return int(_load().oracle_threads())


def set_threads(n: int) -> None:
    """OpenMP threads for the following oracle calls."""
    _load().oracle_set_threads(int(n))


def resolve_t_ref(times, t_ref):
    """A NaN (or None) reference time means the first frame's time."""
    if t_ref is None or (isinstance(t_ref, float) and np.isnan(t_ref)):
        return float(np.asarray(times, dtype=np.float64)[0])
    return float(t_ref)


def offset(v: float, dt: float, th: float = 0.0):
    """Integer anchor floor(v*dt + th + 1/2) and phase v*dt + th - anchor (FP64)."""
    lib = _load()
    i = ctypes.c_int32()
    f = ctypes.c_double()
    lib.oracle_offset(float(v), float(dt), float(th), ctypes.byref(i), ctypes.byref(f))
    return int(i.value), float(f.value)


def profile(kind: int, sigma_px: float, stamp: int, f: float) -> np.ndarray:
    """Unit-sum 1-D PRF profile at sub-pixel phase f, taps -h..h."""
    g = np.zeros(stamp, dtype=np.float64)
    _load().oracle_profile(int(kind), float(sigma_px), int(stamp), float(f), _ptr(g, ctypes.c_double))
    return g


def table_size(stamp: int, q: int) -> int:
    """Side of a tabulated PRF grid: offsets -(h+1) .. h+1 in steps of 1/q."""
    return (stamp + 1) * q + 1


def _table(prf_table, stamp, q):
    if prf_table is None:
        return None
    t = np.ascontiguousarray(prf_table, dtype=np.float64)
    n = table_size(stamp, q)
    if t.shape != (n, n):
        raise ValueError("PRF table must be %dx%d for stamp %d, q %d" % (n, n, stamp, q))
    return t


def _opt(a, ctype):
    return None if a is None else _ptr(a, ctype)


def weights(kind: int, sigma_px: float, stamp: int, fy: float, fx: float, prf_table=None,
            prf_q: int = 0) -> np.ndarray:
    """Stamp weights W[a+h][b+h] at phase (fy, fx): the separable Gaussian
    product, or the tabulated PRF read at (a - fy, b - fx)."""
    t = _table(prf_table, stamp, prf_q)
    w = np.zeros((stamp, stamp), dtype=np.float64)
    _load().oracle_weights(int(kind), float(sigma_px), int(stamp), _opt(t, ctypes.c_double),
                           int(prf_q), float(fy), float(fx), _ptr(w, ctypes.c_double))
    return w


def _jitter(jitter, T):
    if jitter is None:
        return None
    j = np.ascontiguousarray(jitter, dtype=np.float64)
    if j.shape != (T, 2):
        raise ValueError("jitter must be [T][2] = (theta_x, theta_y)")
    return j


def offsets(times, t_ref, vel, jitter=None):
    """(iy, ix, fy, fx), each [J][T], for velocities vel [J][2] = (vx, vy) and
    optional per-frame jitter [T][2] = (theta_x, theta_y)."""
    times = np.ascontiguousarray(times, dtype=np.float64)
    vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 2)
    T, J = times.shape[0], vel.shape[0]
    jit = _jitter(jitter, T)
    iy = np.zeros((J, T), np.int32)
    ix = np.zeros((J, T), np.int32)
    fy = np.zeros((J, T), np.float64)
    fx = np.zeros((J, T), np.float64)
    _load().oracle_offsets(T, _ptr(times, ctypes.c_double), resolve_t_ref(times, t_ref), J,
                           _ptr(vel, ctypes.c_double), _opt(jit, ctypes.c_double),
                           _ptr(iy, ctypes.c_int32), _ptr(ix, ctypes.c_int32),
                           _ptr(fy, ctypes.c_double), _ptr(fx, ctypes.c_double))
    return iy, ix, fy, fx


def _finish(nu, lam):
    """SNR = nu/sqrt(Lam), flux = nu/Lam, both 0 where Lam = 0."""
    pos = lam > 0
    safe = np.where(pos, lam, 1.0)
    snr = np.where(pos, nu / np.sqrt(safe), 0.0)
    flux = np.where(pos, nu / safe, 0.0)
    return snr, flux


def search(R, sigma, times, t_ref, vel, prf_kind=PRF_SAMPLED, sigma_px=0.7, stamp=5,
           region=None, prf_table=None, prf_q=0, jitter=None):
    """Full FP64 search.  R [T][H][W] float32, sigma [H][W] float32.

    region = (y_lo, y_hi, x_lo, x_hi) restricts the start pixels (the frames
    are always read whole).  prf_kind PRF_TABLE reads prf_table
    [(stamp+1)q+1]^2 at oversampling prf_q; jitter is [T][2] or None.
    Returns dict of [J][ny][nx] float64 maps nu, lam, snr, flux.
    """
    R = np.ascontiguousarray(R, dtype=np.float32)
    sigma = np.ascontiguousarray(sigma, dtype=np.float32)
    times = np.ascontiguousarray(times, dtype=np.float64)
    vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 2)
    T, H, W = R.shape
    J = vel.shape[0]
    tab = _table(prf_table, stamp, prf_q)
    jit = _jitter(jitter, T)
    y_lo, y_hi, x_lo, x_hi = region if region is not None else (0, H, 0, W)
    ny, nx = y_hi - y_lo, x_hi - x_lo
    nu = np.zeros((J, ny, nx), np.float64)
    lam = np.zeros((J, ny, nx), np.float64)
    rc = _load().oracle_search(H, W, T, _ptr(R, ctypes.c_float), _ptr(sigma, ctypes.c_float),
                               _ptr(times, ctypes.c_double), resolve_t_ref(times, t_ref), J,
                               _ptr(vel, ctypes.c_double), _opt(jit, ctypes.c_double),
                               int(prf_kind), float(sigma_px), int(stamp),
                               _opt(tab, ctypes.c_double), int(prf_q), y_lo, y_hi, x_lo, x_hi,
                               _ptr(nu, ctypes.c_double), _ptr(lam, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_search rejected its arguments")
    snr, flux = _finish(nu, lam)
    return {"nu": nu, "lam": lam, "snr": snr, "flux": flux}


def hypotheses(R, sigma, times, t_ref, vel, hj, hy, hx, prf_kind=PRF_SAMPLED,
               sigma_px=0.7, stamp=5, prf_table=None, prf_q=0, jitter=None):
    """FP64 sums for an explicit list of hypotheses (j, y0, x0)."""
    R = np.ascontiguousarray(R, dtype=np.float32)
    sigma = np.ascontiguousarray(sigma, dtype=np.float32)
    times = np.ascontiguousarray(times, dtype=np.float64)
    vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 2)
    hj = np.ascontiguousarray(hj, dtype=np.int32)
    hy = np.ascontiguousarray(hy, dtype=np.int32)
    hx = np.ascontiguousarray(hx, dtype=np.int32)
    T, H, W = R.shape
    tab = _table(prf_table, stamp, prf_q)
    jit = _jitter(jitter, T)
    n = hj.shape[0]
    nu = np.zeros(n, np.float64)
    lam = np.zeros(n, np.float64)
    rc = _load().oracle_hypotheses(H, W, T, _ptr(R, ctypes.c_float), _ptr(sigma, ctypes.c_float),
                                   _ptr(times, ctypes.c_double), resolve_t_ref(times, t_ref),
                                   vel.shape[0], _ptr(vel, ctypes.c_double),
                                   _opt(jit, ctypes.c_double), int(prf_kind), float(sigma_px),
                                   int(stamp), _opt(tab, ctypes.c_double), int(prf_q), n,
                                   _ptr(hj, ctypes.c_int32), _ptr(hy, ctypes.c_int32),
                                   _ptr(hx, ctypes.c_int32), _ptr(nu, ctypes.c_double),
                                   _ptr(lam, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_hypotheses rejected its arguments")
    snr, flux = _finish(nu, lam)
    return {"nu": nu, "lam": lam, "snr": snr, "flux": flux}


# ---------------------------------------------------------------------------
# Reductions (Sec. 3.2: best trajectory per pixel by the maximum over the
# filter bank; Sec. 3.3: candidates are the highest scores).
# ---------------------------------------------------------------------------

def traj_max(snr, flux):
    """Per trajectory: argmax over start pixels, ties to the smallest y*W+x.
    Returns arrays snr[J], flux[J], y[J], x[J]."""
    J, H, W = snr.shape
    flat = snr.reshape(J, -1)
    arg = np.argmax(flat, axis=1)  # first occurrence = smallest flat index
    return (flat[np.arange(J), arg], flux.reshape(J, -1)[np.arange(J), arg],
            (arg // W).astype(np.int32), (arg % W).astype(np.int32))


def best_over_trajectories(snr, flux):
    """Per start pixel: maximum SNR over the bank, ties to the lowest j."""
    arg = np.argmax(snr, axis=0)  # first occurrence = lowest j
    best = np.take_along_axis(snr, arg[None], axis=0)[0]
    bflux = np.take_along_axis(flux, arg[None], axis=0)[0]
    return best, arg.astype(np.int32), bflux


def topk(snr, flux, k):
    """Global top-k over all (j, y0, x0): SNR descending, then flat index
    j*H*W + y0*W + x0 ascending.  Returns a list of (snr, flux, j, y, x)."""
    J, H, W = snr.shape
    s = snr.reshape(-1)
    idx = np.arange(s.size, dtype=np.int64)
    order = np.lexsort((idx, -s))[:k]
    f = flux.reshape(-1)
    out = []
    for o in order:
        j, p = divmod(int(o), H * W)
        out.append((float(s[o]), float(f[o]), j, p // W, p % W))
    return out


# ---------------------------------------------------------------------------
# Sec. 3.3: scores in units of the standard deviation of the scores in the
# box x box square centred on each pixel; candidates above a threshold.
# ---------------------------------------------------------------------------

def significance(best, box, pixels=None):
    """Each pixel's best score divided by the (population) standard deviation
    of the best scores in the box x box window centred on it, the window
    clipped at the image edges; 0 where that standard deviation is 0.
    Evaluated window by window; `pixels` = (ys, xs) restricts it to those
    pixels (returned as a 1-D array), else the whole map is returned."""
    b = np.asarray(best, np.float64)
    H, W = b.shape
    h = int(box) // 2
    if pixels is None:
        ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        ys, xs = ys.ravel(), xs.ravel()
    else:
        ys, xs = (np.asarray(v).ravel() for v in pixels)
    out = np.zeros(ys.size, np.float64)
    for i, (y, x) in enumerate(zip(ys, xs)):
        w = b[max(0, y - h):y + h + 1, max(0, x - h):x + h + 1]
        sd = w.std()
        out[i] = b[y, x] / sd if sd > 0 else 0.0
    return out.reshape(H, W) if pixels is None else out


def detections(sig, best, best_j, flux, threshold, k):
    """Pixels with significance >= threshold, ordered by significance
    descending then y*W + x ascending; the first k as (sig, snr, flux, j, y, x)."""
    H, W = sig.shape
    s = sig.reshape(-1)
    idx = np.arange(s.size)
    order = np.lexsort((idx, -s))
    out = []
    for o in order[:k]:
        if s[o] < threshold:
            break
        y, x = divmod(int(o), W)
        j = int(best_j[y, x])
        out.append((float(s[o]), float(best[y, x]), float(flux[j, y, x]), j, y, x))
    return out
