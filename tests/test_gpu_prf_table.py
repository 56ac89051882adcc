"""GPU parity of the tabulated (non-separable) PRF and the per-frame pointing
jitter (Sec. 2, 2.1, 3.1 and 3.2: the filter is the jittered trajectory
line convolved with the PRF) against the FP64 oracle, element by element on
small problems spanning several tiles and ragged edges, and on sampled start
pixels at the full FFI size."""
import ctypes
import math

import numpy as np
import pytest
import torch

from oracle import oracle
from paper_2209_09848_amd import synth, tno
from tests import parity

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _to(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _problem(seed, T, H, W, J, vmax=20.0):
    g = np.random.default_rng(seed)
    R = g.standard_normal((T, H, W)).astype(np.float32)
    sigma = synth.sigma_lognormal(g, H, W)
    for _ in range(max(1, H * W // 60)):
        sigma[g.integers(0, H), g.integers(0, W)] = g.choice([0.0, np.nan])
    times = synth.times_with_gap(T, T // 2, 0.9) if T > 2 else synth.times_uniform(T)
    vel = g.uniform(-vmax, vmax, size=(J, 2))
    return g, R, sigma, times, vel


def _run(R, sigma, times, vel, t_ref, top_k, stamp, kind, table=None, q=0, jitter=None,
         sigma_px=0.7, handle=None):
    kw = dict(t_ref=t_ref, top_k=top_k, stamp=stamp, prf_kind=kind, sigma_px=sigma_px)
    if table is not None:
        kw.update(prf_table=_to(table), prf_q=q)
    if jitter is not None:
        kw["jitter"] = _to(jitter)
    o, res = tno.search_tensors(_to(R), _to(sigma), _to(times), _to(vel), handle=handle, **kw)
    torch.cuda.synchronize()
    assert res.status == 0
    return {"snr": o["snr"].cpu().numpy(), "flux": o["flux"].cpu().numpy(),
            "best_snr": o["best_snr"].cpu().numpy(), "best_traj": o["best_traj"].cpu().numpy(),
            "traj_max": tno.decode_peaks(o["traj_max"]),
            "topk": tno.decode_candidates(o["topk"], res.n_topk) if top_k else []}, res


def _check(R, sigma, times, vel, t_ref, stamp, kind, table=None, q=0, jitter=None, top_k=20,
           sigma_px=0.7):
    print("prf case: T,H,W=%s J=%d stamp=%d kind=%d q=%d jitter=%s" %
          (tuple(R.shape), vel.shape[0], stamp, kind, q, jitter is not None), flush=True)
    g, res = _run(R, sigma, times, vel, t_ref, top_k, stamp, kind, table, q, jitter, sigma_px)
    o = oracle.search(R, sigma, times, t_ref, vel, prf_kind=kind, stamp=stamp, sigma_px=sigma_px,
                      prf_table=table, prf_q=q, jitter=jitter)
    parity.check_maps(g["snr"], g["flux"], o)
    parity.check_best(g["best_snr"], g["best_traj"], o["snr"])
    parity.check_traj_max(g["traj_max"], o["snr"], o["flux"])
    if top_k:
        parity.check_topk(g["topk"], o["snr"], top_k)
    return g, o


@pytest.mark.parametrize("T,H,W,J,stamp,q,jit", [
    (12, 70, 200, 4, 5, 9, True),      # TESS-like oversampling, several tiles, ragged
    (12, 70, 200, 4, 5, 9, False),
    (9, 37, 133, 3, 3, 3, True),
    (7, 45, 150, 3, 7, 4, True),
    (5, 40, 140, 2, 15, 2, True),      # widest stamp: 225 weights per frame
    (5, 33, 129, 2, 1, 5, True),
    (300, 34, 40, 2, 5, 6, True),      # many frame chunks
])
def test_tabulated_psf_parity(T, H, W, J, stamp, q, jit):
    g, R, sigma, times, vel = _problem(200 + T + H + stamp, T, H, W, J)
    table = synth.TabulatedPSF().table(stamp, q)
    jitter = synth.jitter_series(g, T, amp=0.15) if jit else None
    _check(R, sigma, times, vel, float(times[0]), stamp, oracle.PRF_TABLE, table, q, jitter)


def test_asymmetric_random_table_parity():
    """A random table: any transposition, mirror or phase-sign slip between
    the table kernel and the oracle shows."""
    g, R, sigma, times, vel = _problem(230, 8, 50, 170, 3)
    q = 3
    n = 6 * q + 1
    table = g.random((n, n)) - 0.2
    jitter = synth.jitter_series(g, 8, amp=0.4)
    _check(R, sigma, times, vel, float(times[3]) - 0.01, 5, oracle.PRF_TABLE, table, q, jitter)


@pytest.mark.parametrize("kind", [0, 1])
def test_gaussian_prf_with_jitter_parity(kind):
    g, R, sigma, times, vel = _problem(240 + kind, 10, 60, 190, 4)
    jitter = synth.jitter_series(g, 10, amp=0.3)
    _check(R, sigma, times, vel, float(times[0]), 5, kind, jitter=jitter,
           sigma_px=0.9 if kind else 0.7)


def test_large_jitter_moves_trails_off_the_image():
    """Jitter of tens of pixels (integer and fractional parts) with fast
    trajectories: shifts leave the image and the staged border."""
    g, R, sigma, times, vel = _problem(250, 6, 40, 130, 3)
    vel = np.array([[3000.0, 10.0], [-300.0, 1500.0], [3.0, -4.0]])
    jitter = np.column_stack([g.uniform(-40, 40, 6), g.uniform(-25, 25, 6)])
    _check(R, sigma, times, vel, float(times[0]), 5, oracle.PRF_TABLE,
           synth.TabulatedPSF().table(5, 4), 4, jitter)
    _check(R, sigma, times, vel, float(times[0]), 5, oracle.PRF_SAMPLED, jitter=jitter)


def test_host_pointer_table_and_jitter_match_device_path():
    g, R, sigma, times, vel = _problem(260, 8, 36, 140, 3)
    T, H, W = R.shape
    J = vel.shape[0]
    table = synth.TabulatedPSF().table(5, 6)
    jitter = synth.jitter_series(g, T, amp=0.2)
    dev, _ = _run(R, sigma, times, vel, float(times[0]), 0, 5, oracle.PRF_TABLE, table, 6, jitter)
    snr = np.zeros((J, H, W), np.float32)
    flux = np.zeros((J, H, W), np.float32)
    req = tno.tno_request()
    req.height, req.width, req.n_frames, req.dtype = H, W, T, tno.TNO_F32
    req.residuals = R.ctypes.data_as(ctypes.c_void_p)
    req.sigma = sigma.ctypes.data_as(ctypes.c_void_p)
    req.times = times.ctypes.data_as(ctypes.c_void_p)
    req.t_ref = float(times[0])
    req.prf = tno.tno_prf(tno.TNO_PRF_TABLE, 5, 0.0, table.ctypes.data_as(ctypes.c_void_p), 6, 0)
    req.n_traj = J
    req.velocities = vel.ctypes.data_as(ctypes.c_void_p)
    req.jitter = jitter.ctypes.data_as(ctypes.c_void_p)
    out = tno.tno_outputs()
    out.snr = snr.ctypes.data_as(ctypes.c_void_p)
    out.flux = flux.ctypes.data_as(ctypes.c_void_p)
    with tno.Search(0) as h:
        res = h.wait(h.submit(req, out))
    assert res.status == 0
    assert np.array_equal(snr, dev["snr"]) and np.array_equal(flux, dev["flux"])


def test_injected_tabulated_source_recovered_at_truth():
    """A source drawn with the continuous PSF on a jittered trail: the
    search's best hypothesis is the true (trajectory, start pixel), and its
    flux estimate is within 1% of the injected flux."""
    T, H, W = 60, 64, 256
    g, R, sigma, times, vel = _problem(270, T, H, W, 6, vmax=15.0)
    R[:] = 0.0
    sigma[:] = 1.0
    jitter = synth.jitter_series(g, T, amp=0.15)
    psf = synth.TabulatedPSF()
    src = synth.Source(x=100.0, y=30.0, vx=vel[2, 0], vy=vel[2, 1], amp=3.0, traj=2)
    k, y, x, v = synth.render_sources((T, H, W), times, float(times[0]), [src], stamp=5,
                                      jitter=jitter, psf=psf)
    Rn = np.zeros((T, H, W))
    np.add.at(Rn, (k, y, x), v)
    Rn += 0.05 * g.standard_normal((T, H, W))
    R = Rn.astype(np.float32)
    gout, _ = _run(R, sigma, times, vel, float(times[0]), 5, 5, oracle.PRF_TABLE,
                   psf.table(5, 9), 9, jitter)
    c = gout["topk"][0]
    assert (c[2], c[3], c[4]) == (2, 30, 100)
    assert abs(c[1] - 3.0) < 0.03
    o = oracle.hypotheses(R, sigma, times, float(times[0]), vel, [2], [30], [100],
                          prf_kind=oracle.PRF_TABLE, stamp=5, prf_table=psf.table(5, 9), prf_q=9,
                          jitter=jitter)
    assert abs(c[0] - o["snr"][0]) <= 1e-5 * abs(o["snr"][0])


@pytest.mark.slow
def test_ffi_full_size_tabulated_with_jitter_sampled_parity():
    """2048x2048 px x 1000 frames, 100 trajectories, with the tabulated PSF
    (q = 9) and a +-0.15 px jitter series: oracle on sampled start pixels in
    a corner, an edge and the centre, and at every fifth top-k candidate."""
    H = W = 2048
    T = 1000
    print("generating FFI-size problem", flush=True)
    R, sigma, times, t_ref, vel, src = synth.make_ffi_like_torch(H, W, T, DEV)
    jitter = synth.jitter_series(synth.rng(1, 9), T, amp=0.15)
    table = synth.TabulatedPSF().table(5, 9)
    o, res = tno.search_tensors(R, _to(sigma), _to(times), _to(vel), t_ref=t_ref, top_k=100,
                                prf_kind=tno.TNO_PRF_TABLE, stamp=5, prf_table=_to(table), prf_q=9,
                                jitter=_to(jitter))
    torch.cuda.synchronize()
    assert res.status == 0
    print("tabulated search: device %.1f ms (search %.1f ms), %.3g updates/s" %
          (res.device_ms, res.search_ms, res.updates / (res.device_ms * 1e-3)), flush=True)
    snr, flux = o["snr"], o["flux"]
    margin = int(math.ceil(np.abs(vel).max() * (times.max() - t_ref))) + 5
    for (y0, x0) in [(0, 0), (1020, 1020), (700, 2042)]:
        y1, x1 = min(H, y0 + 6), min(W, x0 + 6)
        cy0, cy1 = max(0, y0 - margin), min(H, y1 + margin)
        cx0, cx1 = max(0, x0 - margin), min(W, x1 + margin)
        print("oracle region", y0, x0, flush=True)
        ora = oracle.search(R[:, cy0:cy1, cx0:cx1].cpu().numpy(), sigma[cy0:cy1, cx0:cx1], times,
                            t_ref, vel, prf_kind=oracle.PRF_TABLE, stamp=5, prf_table=table,
                            prf_q=9, jitter=jitter,
                            region=(y0 - cy0, y1 - cy0, x0 - cx0, x1 - cx0))
        parity.check_maps(snr[:, y0:y1, x0:x1].cpu().numpy(), flux[:, y0:y1, x0:x1].cpu().numpy(), ora)
    # top-k: values equal the map's largest, and every fifth candidate
    # matches the oracle at its own (trajectory, start pixel)
    cands = tno.decode_candidates(o["topk"], res.n_topk)
    tv = torch.topk(snr.reshape(-1), 100).values.cpu().numpy()
    assert np.array_equal(np.array([c[0] for c in cands], np.float32), tv)
    for c in cands[::5]:
        _, _, j, y, x = c
        cy0, cy1 = max(0, y - margin), min(H, y + 1 + margin)
        cx0, cx1 = max(0, x - margin), min(W, x + 1 + margin)
        ora = oracle.search(R[:, cy0:cy1, cx0:cx1].cpu().numpy(), sigma[cy0:cy1, cx0:cx1], times,
                            t_ref, vel[j:j + 1], prf_kind=oracle.PRF_TABLE, stamp=5, prf_table=table,
                            prf_q=9, jitter=jitter, region=(y - cy0, y + 1 - cy0, x - cx0, x + 1 - cx0))
        parity.check_maps(np.array([[[c[0]]]], np.float32), np.array([[[c[1]]]], np.float32), ora)


@pytest.mark.parametrize("kind,stamp", [(0, 5), (1, 7), ("table", 5), ("table", 7)])
def test_both_trail_orientations(kind, stamp):
    """A bank with horizontal, vertical, diagonal and standing trajectories:
    the normaliser stores a trail box by rows when it is wider than tall and
    by columns otherwise, and runs the two groups in separate launches; every
    map must match the oracle whichever way a trajectory was stored."""
    T, H, W = 40, 60, 150
    g, R, sigma, times, _ = _problem(300 + stamp, T, H, W, 1)
    vel = np.array([[40.0, 0.0], [-35.0, 3.0], [0.0, 30.0], [2.5, -28.0], [20.0, 20.0],
                    [-21.0, 19.0], [0.0, 0.0], [60.0, -1.0]])
    table, q = (synth.TabulatedPSF().table(stamp, 5), 5) if kind == "table" else (None, 0)
    jitter = synth.jitter_series(g, T, amp=0.15)
    _check(R, sigma, times, vel, float(times[0]), stamp, oracle.PRF_TABLE if kind == "table" else kind,
           table=table, q=q, jitter=jitter)
