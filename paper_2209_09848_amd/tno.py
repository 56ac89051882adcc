"""Thin ctypes binding of libtno_search.so (include/tno_search.h).

Argument marshalling only: every step of the search runs in the library's HIP
kernels.  The functions keep the C names; `search_tensors` is a convenience
that fills the structs from torch tensors already on the GPU and runs one
request on torch's current stream.  Importing this module without the built
library raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtno_search.so")

TNO_OK = 0
TNO_PENDING = 1
TNO_E_INVAL = -1
TNO_E_NOMEM = -2
TNO_E_BUSY = -3
TNO_E_DEVICE = -4
TNO_E_TICKET = -5
TNO_E_CANCELLED = -6
TNO_E_INTERNAL = -7

TNO_F32, TNO_BF16, TNO_F16, TNO_FP8_E4M3 = 0, 1, 2, 3
TNO_PRF_GAUSS_SAMPLED, TNO_PRF_GAUSS_INTEGRATED, TNO_PRF_TABLE = 0, 1, 2
TNO_MAX_TABLE_Q = 64
TNO_CFG_GRAPHS = 1
TNO_CFG_AUTOTUNE = 2
TNO_CFG_BATCH = 4
TNO_CFG_RESERVE = 8
SEARCH_VARIANTS = ("w4c2", "w8c2", "w2c2", "w4c1", "w8c1", "w4c4", "w2c2r16", "w4c2r16", "ws", "ws4")
TNO_REQ_DEVICE_PTRS = 1
TNO_REQ_VALIDATE = 2
TNO_REQ_STAGE_FP32 = 4
TNO_MAX_TOPK = 1024
TNO_MAX_DETECTIONS = 1024
TNO_MAX_STAMP = 15
TNO_QTILE = 64
TNO_SCRATCH_BYTES = 128 << 20

DTYPE_CODE = {"f32": TNO_F32, "bf16": TNO_BF16, "f16": TNO_F16, "fp8_e4m3": TNO_FP8_E4M3}

_vp = ctypes.c_void_p


class tno_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("stream", _vp), ("tune_cache_path", ctypes.c_char_p),
                ("slab_bytes", ctypes.c_uint64)]


class tno_prf(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("stamp", ctypes.c_int32), ("sigma_px", ctypes.c_double),
                ("table", _vp), ("table_q", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class tno_request(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("n_frames", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("residuals", _vp), ("tile_scales", _vp), ("sigma", _vp), ("times", _vp),
                ("t_ref", ctypes.c_double), ("prf", tno_prf), ("n_traj", ctypes.c_int32),
                ("top_k", ctypes.c_int32), ("velocities", _vp), ("jitter", _vp),
                ("sig_box", ctypes.c_int32),
                ("sig_threshold", ctypes.c_float), ("stack_key", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class tno_peak(ctypes.Structure):
    _fields_ = [("snr", ctypes.c_float), ("flux", ctypes.c_float), ("y", ctypes.c_int32),
                ("x", ctypes.c_int32)]


class tno_candidate(ctypes.Structure):
    _fields_ = [("snr", ctypes.c_float), ("flux", ctypes.c_float), ("traj", ctypes.c_int32),
                ("y", ctypes.c_int32), ("x", ctypes.c_int32)]


class tno_detection(ctypes.Structure):
    _fields_ = [("significance", ctypes.c_float), ("snr", ctypes.c_float),
                ("flux", ctypes.c_float), ("traj", ctypes.c_int32), ("y", ctypes.c_int32),
                ("x", ctypes.c_int32)]


class tno_outputs(ctypes.Structure):
    _fields_ = [("snr", _vp), ("flux", _vp), ("best_snr", _vp), ("best_traj", _vp),
                ("traj_max", _vp), ("topk", _vp), ("significance", _vp), ("detections", _vp),
                ("max_detections", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class tno_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_topk", ctypes.c_int32),
                ("n_detections", ctypes.c_int32), ("n_above", ctypes.c_int32),
                ("updates", ctypes.c_uint64), ("queue_ms", ctypes.c_double),
                ("device_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("prep_ms", ctypes.c_double), ("table_ms", ctypes.c_double),
                ("lambda_ms", ctypes.c_double), ("search_ms", ctypes.c_double),
                ("reduce_ms", ctypes.c_double), ("message", ctypes.c_char * 160)]


class tno_refit_request(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32), ("n_frames", ctypes.c_int32),
                ("sl_height", ctypes.c_int32), ("sl_width", ctypes.c_int32), ("data", _vp),
                ("scattered", _vp), ("jitter", _vp), ("delta", ctypes.c_double),
                ("bright_threshold", ctypes.c_double), ("clip_sigma", ctypes.c_double),
                ("iterations", ctypes.c_int32), ("sigma_rounds", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class tno_refit_outputs(ctypes.Structure):
    _fields_ = [("residuals", _vp), ("sigma", _vp), ("coeffs", _vp), ("sigma0", ctypes.c_double),
                ("n_clipped", ctypes.c_int64), ("n_masked", ctypes.c_int64),
                ("device_ms", ctypes.c_double)]


class tno_stats(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("in_use_bytes", ctypes.c_uint64),
                ("held_bytes", ctypes.c_uint64), ("cached_bytes", ctypes.c_uint64),
                ("device_allocs", ctypes.c_uint64), ("inflight", ctypes.c_int32),
                ("resident_stacks", ctypes.c_int32), ("batch_steps", ctypes.c_uint64),
                ("batch_items", ctypes.c_uint64), ("batch_shared", ctypes.c_uint64),
                ("reserved", ctypes.c_uint64 * 1)]


EXPORTS = ("tno_search_create", "tno_search_submit", "tno_search_poll", "tno_search_destroy",
           "tno_search_cancel", "tno_search_stats", "tno_search_validate", "tno_search_footprint",
           "tno_search_last_error", "tno_quantize", "tno_refit", "tno_search_run_scratch")


class TnoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("tno status %d: %s" % (code, msg))
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libtno_search.so not built (run __graft_entry__.build() or "
                           "python -m paper_2209_09848_amd.build): %s" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.tno_search_create.argtypes = [P(tno_config), P(_vp)]
    lib.tno_search_create.restype = ctypes.c_int
    lib.tno_search_submit.argtypes = [_vp, P(tno_request), P(tno_outputs), P(ctypes.c_uint64)]
    lib.tno_search_submit.restype = ctypes.c_int
    lib.tno_search_poll.argtypes = [_vp, ctypes.c_uint64, ctypes.c_int32, P(tno_result)]
    lib.tno_search_poll.restype = ctypes.c_int
    lib.tno_search_destroy.argtypes = [_vp]
    lib.tno_search_destroy.restype = None
    lib.tno_search_cancel.argtypes = [_vp, ctypes.c_uint64]
    lib.tno_search_cancel.restype = ctypes.c_int
    lib.tno_search_stats.argtypes = [_vp, P(tno_stats)]
    lib.tno_search_stats.restype = ctypes.c_int
    lib.tno_search_validate.argtypes = [P(tno_request), P(tno_outputs), ctypes.c_char_p, ctypes.c_int32]
    lib.tno_search_validate.restype = ctypes.c_int
    lib.tno_search_footprint.argtypes = [P(tno_request), P(tno_outputs)]
    lib.tno_search_footprint.restype = ctypes.c_uint64
    lib.tno_search_last_error.argtypes = []
    lib.tno_search_last_error.restype = ctypes.c_char_p
    lib.tno_search_run_scratch.argtypes = [P(tno_request), P(tno_outputs), _vp, P(tno_result)]
    lib.tno_search_run_scratch.restype = ctypes.c_int
    lib.tno_quantize.argtypes = [ctypes.c_int32] * 4 + [_vp, _vp, _vp, _vp]
    lib.tno_quantize.restype = ctypes.c_int
    lib.tno_refit.argtypes = [P(tno_refit_request), P(tno_refit_outputs), _vp]
    lib.tno_refit.restype = ctypes.c_int
    _lib = lib
    return lib


# ------------------------------------------------------------------ C-named calls

def tno_search_last_error() -> str:
    return load().tno_search_last_error().decode(errors="replace")


def tno_search_create(cfg: tno_config):
    h = _vp()
    rc = load().tno_search_create(ctypes.byref(cfg), ctypes.byref(h))
    if rc != TNO_OK:
        raise TnoError(rc, tno_search_last_error())
    return h


def tno_search_submit(h, req: tno_request, out: tno_outputs):
    """Returns (status, ticket); ticket is None unless status == TNO_OK."""
    t = ctypes.c_uint64()
    rc = load().tno_search_submit(h, ctypes.byref(req), ctypes.byref(out), ctypes.byref(t))
    return rc, (t.value if rc == TNO_OK else None)


def tno_search_poll(h, ticket: int, timeout_ms: int = -1):
    """Returns (status, tno_result or None if pending)."""
    res = tno_result()
    rc = load().tno_search_poll(h, ctypes.c_uint64(ticket), int(timeout_ms), ctypes.byref(res))
    return rc, (None if rc == TNO_PENDING else res)


def tno_search_destroy(h) -> None:
    load().tno_search_destroy(h)


def tno_search_cancel(h, ticket: int) -> int:
    return int(load().tno_search_cancel(h, ctypes.c_uint64(ticket)))


def tno_search_stats(h) -> tno_stats:
    st = tno_stats()
    rc = load().tno_search_stats(h, ctypes.byref(st))
    if rc != TNO_OK:
        raise TnoError(rc, tno_search_last_error())
    return st


def tno_search_validate(req: tno_request, out: tno_outputs):
    buf = ctypes.create_string_buffer(256)
    rc = load().tno_search_validate(ctypes.byref(req), ctypes.byref(out), buf, 256)
    return rc, buf.value.decode(errors="replace")


def tno_search_footprint(req: tno_request, out: tno_outputs) -> int:
    return int(load().tno_search_footprint(ctypes.byref(req), ctypes.byref(out)))


def tno_search_run_scratch(req: tno_request, out: tno_outputs, stream=None):
    """The search as one synchronous call with no device allocation (its
    working memory is the library's fixed per-GPU array of
    TNO_SCRATCH_BYTES).  Returns (status, tno_result)."""
    res = tno_result()
    rc = int(load().tno_search_run_scratch(ctypes.byref(req), ctypes.byref(out),
                                           ctypes.c_void_p(stream) if stream else None, ctypes.byref(res)))
    return rc, res


def tno_quantize(T, H, W, dtype, residuals_ptr, codes_ptr, scales_ptr, stream=None) -> int:
    return int(load().tno_quantize(int(T), int(H), int(W), int(dtype), residuals_ptr, codes_ptr,
                                   scales_ptr, stream))


# ------------------------------------------------------------------ torch convenience

def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def make_request(R, sigma, times, vel, *, t_ref=float("nan"), dtype="f32", scales=None,
                 sigma_px=0.7, stamp=5, prf_kind=TNO_PRF_GAUSS_SAMPLED, top_k=10,
                 stack_key=0, flags=TNO_REQ_DEVICE_PTRS, shape=None, sig_box=0,
                 sig_threshold=5.0, prf_table=None, prf_q=0, jitter=None) -> tno_request:
    """A request over torch tensors on the GPU (device pointers).  R may be
    None (search the stack resident under stack_key) with shape=(T, H, W).
    prf_table (float64 [(stamp+1)q+1]^2, with prf_kind=TNO_PRF_TABLE and
    prf_q=q) and jitter (float64 [T][2]) are tensors on the same device."""
    T, H, W = (int(s) for s in (R.shape if R is not None else shape))
    req = tno_request()
    req.height, req.width, req.n_frames = H, W, T
    req.dtype = DTYPE_CODE[dtype] if isinstance(dtype, str) else int(dtype)
    req.residuals = _ptr(R)
    req.tile_scales = _ptr(scales)
    req.sigma = _ptr(sigma)
    req.times = _ptr(times)
    req.t_ref = float(t_ref) if t_ref is not None else float("nan")
    req.prf = tno_prf(int(prf_kind), int(stamp), float(sigma_px), _ptr(prf_table), int(prf_q), 0)
    req.n_traj = int(vel.shape[0])
    req.top_k = int(top_k)
    req.velocities = _ptr(vel)
    req.jitter = _ptr(jitter)
    req.sig_box = int(sig_box)
    req.sig_threshold = float(sig_threshold)
    req.stack_key = int(stack_key)
    req.flags = int(flags)
    req.reserved = 0
    return req


class Search:
    """One handle on torch's current stream of `device` (default cuda:0)."""

    def __init__(self, device: int = 0, max_inflight: int = 64, hbm_budget_bytes: int = 0,
                 stream=None, own_streams: bool = False, autotune: bool = False,
                 tune_cache_path: str | None = None, graphs: bool = False, batch: bool = False,
                 slab_bytes: int = 0, reserve: bool = False):
        """own_streams=True: the library runs requests on its own pool of streams
        (concurrent requests overlap; inputs must be complete before submit);
        otherwise every request runs on `stream` (default: torch's current).
        batch=True (implies own_streams): continuous batching of the searches
        of admitted requests into shared steps.  slab_bytes: device bytes of a
        trajectory slab (0: the library's default).  reserve=True: the HBM
        budget is reserved at creation and every device buffer carved from it."""
        import torch
        if own_streams or batch:
            stream = 0
        elif stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        cfg = tno_config()
        cfg.device = device
        cfg.max_inflight = max_inflight
        cfg.hbm_budget_bytes = hbm_budget_bytes
        cfg.flags = ((TNO_CFG_AUTOTUNE if autotune else 0) | (TNO_CFG_GRAPHS if graphs else 0) |
                     (TNO_CFG_BATCH if batch else 0) | (TNO_CFG_RESERVE if reserve else 0))
        cfg.reserved = 0
        cfg.stream = ctypes.c_void_p(stream) if stream else None
        self._path = tune_cache_path.encode() if tune_cache_path else None
        cfg.tune_cache_path = self._path
        cfg.slab_bytes = slab_bytes
        self.device = device
        self.h = tno_search_create(cfg)

    def close(self):
        if self.h is not None:
            tno_search_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, req: tno_request, out: tno_outputs) -> int:
        rc, t = tno_search_submit(self.h, req, out)
        if rc != TNO_OK:
            raise TnoError(rc, tno_search_last_error())
        return t

    def cancel(self, ticket: int) -> int:
        return tno_search_cancel(self.h, ticket)

    def stats(self) -> tno_stats:
        return tno_search_stats(self.h)

    def wait(self, ticket: int, timeout_ms: int = -1) -> tno_result:
        rc, res = tno_search_poll(self.h, ticket, timeout_ms)
        if rc == TNO_PENDING:
            raise TimeoutError("ticket %d still pending" % ticket)
        if rc != TNO_OK:
            msg = res.message.decode(errors="replace") if res is not None else tno_search_last_error()
            raise TnoError(rc, msg)
        return res


def shape_class(H, W, T, J, stamp=5, tabulated=False, direct=False) -> str:
    """Tuning-table key the library uses for a request shape; direct: a
    reduced-precision stack searched in place (stamps 1, 3, 5; W % 4 == 0)."""
    lg = lambda v: max(0, (int(v) - 1).bit_length())
    return "%s%s%d_H%d_W%d_J%d_T%d" % ("D" if direct else "", "P" if tabulated else "S", stamp, lg(H), lg(W),
                                       lg(J), lg(T))


def alloc_outputs(J, H, W, k, device="cuda", maps=True, detections=0):
    """Torch output buffers and the tno_outputs struct that points at them.
    detections > 0 also allocates the significance map and that many
    detection slots (the request needs sig_box > 0)."""
    import torch
    o = {}
    if maps:
        o["snr"] = torch.empty((J, H, W), dtype=torch.float32, device=device)
        o["flux"] = torch.empty((J, H, W), dtype=torch.float32, device=device)
    o["best_snr"] = torch.empty((H, W), dtype=torch.float32, device=device)
    o["best_traj"] = torch.empty((H, W), dtype=torch.int32, device=device)
    o["traj_max"] = torch.empty((J, 4), dtype=torch.int32, device=device)   # tno_peak
    o["topk"] = torch.empty((max(k, 1), 5), dtype=torch.int32, device=device)  # tno_candidate
    out = tno_outputs()
    out.snr = _ptr(o.get("snr"))
    out.flux = _ptr(o.get("flux"))
    out.best_snr = _ptr(o["best_snr"])
    out.best_traj = _ptr(o["best_traj"])
    out.traj_max = _ptr(o["traj_max"])
    out.topk = _ptr(o["topk"]) if k > 0 else None
    if detections > 0:
        o["significance"] = torch.empty((H, W), dtype=torch.float32, device=device)
        o["detections"] = torch.empty((detections, 6), dtype=torch.int32, device=device)
        out.significance = _ptr(o["significance"])
        out.detections = _ptr(o["detections"])
        out.max_detections = int(detections)
    return o, out


def decode_detections(t, n):
    """[m][6] int32 tensor of tno_detection -> list of (significance, snr, flux, traj, y, x)."""
    import numpy as np
    a = t.cpu().numpy()[:n]
    f = a[:, :3].copy().view(np.float32)
    return [(float(f[i, 0]), float(f[i, 1]), float(f[i, 2]), int(a[i, 3]), int(a[i, 4]),
             int(a[i, 5])) for i in range(n)]


def decode_peaks(t):
    """[J][4] int32 tensor of tno_peak -> (snr, flux, y, x) numpy arrays."""
    import numpy as np
    a = t.cpu().numpy()
    return (a[:, 0].view(np.float32).copy(), a[:, 1].view(np.float32).copy(),
            a[:, 2].copy(), a[:, 3].copy())


def decode_candidates(t, n):
    """[k][5] int32 tensor of tno_candidate -> list of (snr, flux, traj, y, x)."""
    import numpy as np
    a = t.cpu().numpy()[:n]
    s = a[:, 0].view(np.float32)
    f = a[:, 1].view(np.float32)
    return [(float(s[i]), float(f[i]), int(a[i, 2]), int(a[i, 3]), int(a[i, 4])) for i in range(n)]


def search_tensors(R, sigma, times, vel, *, top_k=10, maps=True, handle: Search | None = None,
                   detections=0, **kw):
    """Run one search over GPU tensors; returns (outputs dict, tno_result)."""
    T, H, W = (int(s) for s in R.shape)
    J = int(vel.shape[0])
    o, out = alloc_outputs(J, H, W, top_k, device=R.device, maps=maps, detections=detections)
    req = make_request(R, sigma, times, vel, top_k=top_k, **kw)
    own = handle is None
    h = Search(R.device.index or 0) if own else handle
    try:
        t = h.submit(req, out)
        res = h.wait(t)
    finally:
        if own:
            h.close()
    return o, res


# ------------------------------------------------------------------ background re-fit

def tno_refit(req: tno_refit_request, out: tno_refit_outputs, stream=None) -> int:
    return int(load().tno_refit(ctypes.byref(req), ctypes.byref(out),
                                ctypes.c_void_p(stream) if stream else None))


def refit_tensors(D, jitter, *, scattered=None, delta=1.345, iterations=5, bright_threshold=math.inf,
                  clip_sigma=5.0, sigma_rounds=3, coeffs=True, stream=None):
    """Per-pixel background re-fit of raw frames D (float32 [T][H][W] on the
    GPU) with jitter (float64 [T][2]) and optional low-resolution scattered
    light (float32 [T][ny][nx]), all device tensors.  Returns (dict with
    residuals, sigma, coeffs tensors, tno_refit_outputs)."""
    import torch
    T, H, W = (int(v) for v in D.shape)
    req = tno_refit_request()
    req.height, req.width, req.n_frames = H, W, T
    if scattered is not None:
        req.sl_height, req.sl_width = int(scattered.shape[1]), int(scattered.shape[2])
    req.data = _ptr(D)
    req.scattered = _ptr(scattered)
    req.jitter = _ptr(jitter)
    req.delta = float(delta)
    req.bright_threshold = float(bright_threshold)
    req.clip_sigma = float(clip_sigma)
    req.iterations = int(iterations)
    req.sigma_rounds = int(sigma_rounds)
    o = {"residuals": torch.empty((T, H, W), dtype=torch.float32, device=D.device),
         "sigma": torch.empty((H, W), dtype=torch.float32, device=D.device)}
    if coeffs:
        o["coeffs"] = torch.empty((6, H, W), dtype=torch.float64, device=D.device)
    out = tno_refit_outputs()
    out.residuals = _ptr(o["residuals"])
    out.sigma = _ptr(o["sigma"])
    out.coeffs = _ptr(o.get("coeffs"))
    if stream is None:
        stream = torch.cuda.current_stream(D.device).cuda_stream
    rc = tno_refit(req, out, stream)
    if rc != TNO_OK:
        raise TnoError(rc, tno_search_last_error())
    return o, out
