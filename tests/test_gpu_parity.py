"""GPU parity: the HIP search through the C ABI against the FP64 oracle.

Full maps on small problems that still span several tiles and ragged edges;
sampled hypotheses and reduction properties at the full FFI size.
"""
import math

import numpy as np
import pytest
import torch

from oracle import codec, oracle
from paper_2209_09848_amd import synth, tno
from tests import parity

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _to(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def run_gpu(R, sigma, times, vel, t_ref, top_k=10, stamp=5, sigma_px=0.7, prf_kind=0,
            dtype="f32", scales=None, handle=None):
    Rt = R if isinstance(R, torch.Tensor) else _to(R)
    o, res = tno.search_tensors(Rt, _to(sigma), _to(times), _to(vel), t_ref=t_ref, top_k=top_k,
                                stamp=stamp, sigma_px=sigma_px, prf_kind=prf_kind, dtype=dtype,
                                scales=None if scales is None else (scales if isinstance(scales, torch.Tensor) else _to(scales)),
                                handle=handle)
    torch.cuda.synchronize()
    J = vel.shape[0]
    out = {
        "snr": o["snr"].cpu().numpy(), "flux": o["flux"].cpu().numpy(),
        "best_snr": o["best_snr"].cpu().numpy(), "best_traj": o["best_traj"].cpu().numpy(),
        "traj_max": tno.decode_peaks(o["traj_max"]),
        "topk": tno.decode_candidates(o["topk"], res.n_topk) if top_k > 0 else [],
    }
    assert res.status == 0 and res.updates == J * R.shape[0] * R.shape[1] * R.shape[2]
    return out, res


def full_check(R, sigma, times, vel, t_ref, top_k=10, **kw):
    print("case: T,H,W=%s J=%d k=%d %s" % (tuple(R.shape), vel.shape[0], top_k, kw), flush=True)
    g, res = run_gpu(R, sigma, times, vel, t_ref, top_k=top_k, **kw)
    okw = {k: v for k, v in kw.items() if k in ("stamp", "sigma_px", "prf_kind")}
    o = oracle.search(R, sigma, times, t_ref, vel, **okw)
    es, ef = parity.check_maps(g["snr"], g["flux"], o)
    parity.check_best(g["best_snr"], g["best_traj"], o["snr"])
    parity.check_traj_max(g["traj_max"], o["snr"], o["flux"])
    if top_k > 0:
        parity.check_topk(g["topk"], o["snr"], top_k)
    return g, o, (es, ef)


@pytest.mark.parametrize("variant", ["noisy", "noise_free", "bright"])
def test_c1_full_parity(variant):
    p = synth.make_c1(variant)
    g, o, err = full_check(p.R, p.sigma, p.times, p.vel, p.t_ref, top_k=p.top_k)
    if variant != "noisy":
        j, y, x = np.unravel_index(np.argmax(g["snr"]), g["snr"].shape)
        assert (j, y, x) == (4, 32, 20)
    if variant == "noise_free":
        assert abs(g["snr"][4, 32, 20] - 1.2986868495) < 2e-5


def _rand_problem(seed, T, H, W, J, vmax=20.0, mask=True, gap=True):
    g = np.random.default_rng(seed)
    R = g.standard_normal((T, H, W)).astype(np.float32)
    sigma = synth.sigma_lognormal(g, H, W)
    if mask and H * W > 8:
        for _ in range(max(1, H * W // 50)):
            sigma[g.integers(0, H), g.integers(0, W)] = g.choice([0.0, -1.0, np.nan, np.inf])
    times = synth.times_with_gap(T, T // 2, 0.9) if gap and T > 2 else synth.times_uniform(T)
    vel = g.uniform(-vmax, vmax, size=(J, 2))
    return R, sigma, times, vel


@pytest.mark.parametrize("T,H,W,J,stamp,kind", [
    (9, 37, 133, 4, 5, 0),       # ragged in both axes, several tiles
    (12, 70, 260, 3, 5, 1),      # integrated PRF
    (6, 33, 129, 2, 1, 0),       # single-tap stamp
    (6, 40, 70, 2, 3, 0),
    (5, 45, 50, 2, 7, 1),
    (5, 41, 150, 3, 9, 0),       # shared rows would cost a block per CU: per-wave halo rows
    (4, 39, 140, 2, 11, 1),      # S - 1 above the rows per lane: per-wave halo rows
    (4, 47, 131, 2, 13, 0),
    (4, 50, 140, 2, 15, 0),      # widest stamp
    (300, 34, 40, 3, 5, 0),      # many frame chunks
    (1, 1, 1, 1, 5, 0),          # a single pixel, a single frame
    (3, 2, 3, 2, 3, 0),          # fewer elements than top_k
])
def test_edge_shapes(T, H, W, J, stamp, kind):
    R, sigma, times, vel = _rand_problem(1000 + T + H, T, H, W, J)
    full_check(R, sigma, times, vel, float(times[0]), top_k=25, stamp=stamp, prf_kind=kind,
               sigma_px=0.9 if kind else 0.7)


def test_explicit_reference_time_and_negative_baselines():
    R, sigma, times, vel = _rand_problem(7, 10, 40, 150, 3)
    full_check(R, sigma, times, vel, float(times[6]) + 0.013, top_k=10)


def test_trails_leaving_the_image_and_the_padding():
    # 6000 px/day over 5 cadences moves ~625 px: beyond the image and the
    # staged stack's zero border; many start pixels have Lam = 0
    R, sigma, times, vel = _rand_problem(8, 6, 40, 130, 3)
    vel = np.array([[6000.0, 10.0], [-300.0, 2500.0], [3.0, -4.0]])
    full_check(R, sigma, times, vel, float(times[0]), top_k=10)


def test_all_zero_residuals_ties_go_to_smallest_index():
    R = np.zeros((4, 20, 30), np.float32)
    sigma = np.ones((20, 30), np.float32)
    times = synth.times_uniform(4)
    vel = np.array([[1.0, 0.0], [0.0, -1.0]])
    g, res = run_gpu(R, sigma, times, vel, float(times[0]), top_k=17)
    assert np.all(g["snr"] == 0)
    assert [(c[2], c[3], c[4]) for c in g["topk"]] == [(0, i // 30, i % 30) for i in range(17)]
    assert np.all(g["best_traj"] == 0)
    s, f, y, x = g["traj_max"]
    assert list(y) == [0, 0] and list(x) == [0, 0]


def test_deterministic_repeat():
    R, sigma, times, vel = _rand_problem(9, 20, 64, 200, 4)
    a, _ = run_gpu(R, sigma, times, vel, float(times[0]), top_k=50)
    b, _ = run_gpu(R, sigma, times, vel, float(times[0]), top_k=50)
    for k in ("snr", "flux", "best_snr", "best_traj"):
        assert np.array_equal(a[k], b[k])
    assert a["topk"] == b["topk"]


def test_host_pointer_path_matches_device_path():
    R, sigma, times, vel = _rand_problem(10, 8, 36, 140, 3)
    dev, _ = run_gpu(R, sigma, times, vel, float(times[0]), top_k=12)
    J, (T, H, W) = vel.shape[0], R.shape
    snr = np.zeros((J, H, W), np.float32)
    flux = np.zeros((J, H, W), np.float32)
    best = np.zeros((H, W), np.float32)
    bestj = np.zeros((H, W), np.int32)
    peaks = (tno.tno_peak * J)()
    cands = (tno.tno_candidate * 12)()
    import ctypes
    req = tno.tno_request()
    req.height, req.width, req.n_frames, req.dtype = H, W, T, tno.TNO_F32
    req.residuals = R.ctypes.data_as(ctypes.c_void_p)
    req.sigma = sigma.ctypes.data_as(ctypes.c_void_p)
    req.times = times.ctypes.data_as(ctypes.c_void_p)
    req.t_ref = float(times[0])
    req.prf = tno.tno_prf(0, 5, 0.7)
    req.n_traj = J
    req.top_k = 12
    req.velocities = vel.ctypes.data_as(ctypes.c_void_p)
    out = tno.tno_outputs()
    out.snr = snr.ctypes.data_as(ctypes.c_void_p)
    out.flux = flux.ctypes.data_as(ctypes.c_void_p)
    out.best_snr = best.ctypes.data_as(ctypes.c_void_p)
    out.best_traj = bestj.ctypes.data_as(ctypes.c_void_p)
    out.traj_max = ctypes.cast(peaks, ctypes.c_void_p)
    out.topk = ctypes.cast(cands, ctypes.c_void_p)
    with tno.Search(0) as h:
        t = h.submit(req, out)
        res = h.wait(t)
    assert res.status == 0 and res.n_topk == 12
    assert np.array_equal(snr, dev["snr"]) and np.array_equal(flux, dev["flux"])
    assert np.array_equal(best, dev["best_snr"]) and np.array_equal(bestj, dev["best_traj"])
    assert [(c.snr, c.traj, c.y, c.x) for c in cands] == [(c[0], c[2], c[3], c[4]) for c in dev["topk"]]


# ------------------------------------------------------------------ precision form

@pytest.mark.parametrize("dtype", ["bf16", "f16", "fp8_e4m3"])
def test_quantize_matches_oracle_codec_bit_exactly(dtype):
    g = np.random.default_rng(21)
    T, H, W = 5, 100, 150
    R = (g.standard_normal((T, H, W)) * np.exp(2 * g.standard_normal((T, H, W)))).astype(np.float32)
    R[2, 64:, :64] = 0.0
    R[3, 10, 10] = 2.0 ** -140  # FP32 subnormal input
    codes_o, scales_o = codec.quantize(R, dtype)
    Rt = _to(R)
    ct = torch.empty((T, H, W), dtype=torch.uint8 if dtype == "fp8_e4m3" else torch.int16, device=DEV)
    st = torch.empty((T, (H + 63) // 64, (W + 63) // 64), dtype=torch.float32, device=DEV)
    rc = tno.tno_quantize(T, H, W, tno.DTYPE_CODE[dtype], Rt.data_ptr(), ct.data_ptr(), st.data_ptr(),
                          None)
    assert rc == 0
    torch.cuda.synchronize()
    codes = ct.cpu().numpy().view(np.uint8 if dtype == "fp8_e4m3" else np.uint16)
    assert np.array_equal(st.cpu().numpy(), scales_o)
    assert np.array_equal(codes, codes_o)


@pytest.mark.parametrize("dtype", ["bf16", "f16", "fp8_e4m3"])
@pytest.mark.parametrize("case", [
    (12, 70, 140, 3, 5, 20.0, None),       # searched in place (W % 4 == 0), several quantization tiles
    (9, 37, 200, 2, 3, 60.0, None),        # stamp 3 in place; trails far off the image
    (7, 33, 124, 2, 1, 20.0, None),        # stamp 1 in place, exactly one tile wide
    (8, 45, 136, 3, 5, 20.0, "ws4"),       # in place, 4 rows per lane
    (10, 40, 142, 2, 5, 20.0, None),       # W % 4 != 0: staged FP32 copy
    (6, 41, 120, 2, 7, 20.0, None),        # stamp 7: staged FP32 copy
    (12, 70, 140, 3, 5, 20.0, "stage"),    # staged FP32 copy on request
])
def test_precision_search_parity_on_dequantized_values(tmp_path, dtype, case):
    T, H, W, J, stamp, vmax, variant = case
    R, sigma, times, vel = _rand_problem(30 + W + stamp, T, H, W, J, vmax=vmax)
    codes, scales = codec.quantize(R, dtype)
    deq = codec.dequantize(codes, scales, dtype)
    ct = _to(codes.view(np.int16) if dtype != "fp8_e4m3" else codes)
    print("precision case", dtype, case, flush=True)
    handle = None
    kw = {}
    if variant == "stage":
        kw["flags"] = tno.TNO_REQ_DEVICE_PTRS | tno.TNO_REQ_STAGE_FP32
    elif variant:
        direct = stamp in (1, 3, 5) and W % 4 == 0
        path = tmp_path / "tune.txt"
        path.write_text("%s %s %s %d 1.0\n" % (_arch(), tno.shape_class(H, W, T, J, stamp, direct=direct),
                                               variant, J))
        handle = tno.Search(0, tune_cache_path=str(path))
    try:
        o_, r_ = tno.search_tensors(ct, _to(sigma), _to(times), _to(vel), t_ref=float(times[0]), top_k=10,
                                    dtype=dtype, scales=_to(scales), stamp=stamp, handle=handle, **kw)
        torch.cuda.synchronize()
    finally:
        if handle:
            handle.close()
    assert r_.status == 0, r_.message
    o = oracle.search(deq, sigma, times, float(times[0]), vel, stamp=stamp)
    parity.check_maps(o_["snr"].cpu().numpy(), o_["flux"].cpu().numpy(), o)
    parity.check_topk(tno.decode_candidates(o_["topk"], r_.n_topk), o["snr"], 10)


# ------------------------------------------------------------------ API behaviour on the GPU

def _small_request(k=5):
    R, sigma, times, vel = _rand_problem(40, 6, 30, 40, 2)
    t = [_to(R), _to(sigma), _to(times), _to(vel)]
    req = tno.make_request(*t, t_ref=float(times[0]), top_k=k)
    o, out = tno.alloc_outputs(2, 30, 40, k)
    return req, out, (t, o)


def test_tickets_budget_and_backpressure():
    req, out, keep = _small_request()
    with tno.Search(0, max_inflight=1) as h:
        t1 = h.submit(req, out)
        rc, t2 = tno.tno_search_submit(h.h, req, out)
        assert rc == tno.TNO_E_BUSY and t2 is None
        res = h.wait(t1)
        assert res.status == 0
        rc, _ = tno.tno_search_poll(h.h, t1, 0)
        assert rc == tno.TNO_E_TICKET
        rc, _ = tno.tno_search_poll(h.h, 987654, 0)
        assert rc == tno.TNO_E_TICKET
    with tno.Search(0, hbm_budget_bytes=4096) as h:
        rc, t = tno.tno_search_submit(h.h, req, out)
        assert rc == tno.TNO_E_NOMEM
    bad = tno.make_request(*keep[0], top_k=5)
    bad.prf = tno.tno_prf(0, 4, 0.7)
    with tno.Search(0) as h:
        rc, t = tno.tno_search_submit(h.h, bad, out)
        assert rc == tno.TNO_E_INVAL
        # destroy with work still pending frees everything
        h.submit(req, out)


# ------------------------------------------------------------------ full FFI size, sampled

def _crop_oracle(R_dev, sigma, times, t_ref, vel, y0, y1, x0, x1, margin):
    T, H, W = R_dev.shape
    cy0, cy1 = max(0, y0 - margin), min(H, y1 + margin)
    cx0, cx1 = max(0, x0 - margin), min(W, x1 + margin)
    Rc = R_dev[:, cy0:cy1, cx0:cx1].cpu().numpy()
    o = oracle.search(Rc, sigma[cy0:cy1, cx0:cx1], times, t_ref, vel,
                      region=(y0 - cy0, y1 - cy0, x0 - cx0, x1 - cx0))
    return o


@pytest.mark.slow
def test_ffi_full_size_sampled_parity():
    """2048x2048 px x 1000 frames, 100 trajectories, 30 sources: the launch
    configuration the benchmark times.  Oracle on sampled start pixels (all
    trajectories) in a corner, an edge and the centre, at every fifth top-k
    candidate and at injected sources; reductions checked against torch ops
    on the GPU's own maps."""
    H = W = 2048
    T = 1000
    print("generating FFI-size problem", flush=True)
    R, sigma, times, t_ref, vel, src = synth.make_ffi_like_torch(H, W, T, DEV)
    J = vel.shape[0]
    k = 100
    o, res = tno.search_tensors(R, _to(sigma), _to(times), _to(vel), t_ref=t_ref, top_k=k)
    torch.cuda.synchronize()
    print("search done: device %.1f ms, %.3g updates/s" % (res.device_ms, res.updates / (res.device_ms * 1e-3)), flush=True)
    snr, flux = o["snr"], o["flux"]
    # reductions vs torch on the same FP32 maps
    best = snr.max(dim=0).values
    assert torch.equal(o["best_snr"], best)
    first = (snr == best[None]).to(torch.uint8).argmax(dim=0).to(torch.int32)
    assert torch.equal(o["best_traj"], first)
    del first
    fl = snr.reshape(J, -1)
    mx = fl.max(dim=1).values
    am = (fl == mx[:, None]).to(torch.uint8).argmax(dim=1).cpu().numpy()
    ps, pf, py, px = tno.decode_peaks(o["traj_max"])
    assert np.array_equal(ps, mx.cpu().numpy())
    assert np.array_equal(py * W + px, am)
    flat = snr.reshape(-1)
    tv = torch.topk(flat, k).values.cpu().numpy()
    cands = tno.decode_candidates(o["topk"], res.n_topk)
    assert np.array_equal(np.array([c[0] for c in cands], np.float32), tv)
    kth = tv[-1]
    gt = torch.nonzero(flat > float(kth)).reshape(-1).cpu().numpy()
    eq = torch.nonzero(flat == float(kth)).reshape(-1).cpu().numpy()
    want = set(gt.tolist()) | set(eq[:k - gt.size].tolist())
    got = {c[2] * H * W + c[3] * W + c[4] for c in cands}
    assert got == want
    # oracle on sampled start pixels, all trajectories
    margin = int(math.ceil(np.abs(vel).max() * (times.max() - t_ref))) + 4
    for (y0, x0) in [(0, 0), (1020, 1020), (2040, 1500), (700, 2042)]:
        y1, x1 = min(H, y0 + 8), min(W, x0 + 8)
        print("oracle region", y0, x0, flush=True)
        ora = _crop_oracle(R, sigma, times, t_ref, vel, y0, y1, x0, x1, margin)
        sub = {"snr": snr[:, y0:y1, x0:x1].cpu().numpy(), "flux": flux[:, y0:y1, x0:x1].cpu().numpy()}
        parity.check_maps(sub["snr"], sub["flux"], ora)
    # every fifth top-k candidate: its SNR and flux against the oracle at its
    # own (trajectory, start pixel)
    for c in cands[::5]:
        _, _, j, y, x = c
        ora = _crop_oracle(R, sigma, times, t_ref, vel[j:j + 1], y, y + 1, x, x + 1, margin)
        parity.check_maps(np.array([[[c[0]]]], np.float32), np.array([[[c[1]]]], np.float32), ora)
    # injected sources: truth trajectory around the rounded start
    for s in src[:6]:
        j = s.traj
        yr, xr = int(math.floor(s.y + 0.5)), int(math.floor(s.x + 0.5))
        y0, y1, x0, x1 = max(0, yr - 1), min(H, yr + 2), max(0, xr - 1), min(W, xr + 2)
        ora = _crop_oracle(R, sigma, times, t_ref, vel[j:j + 1], y0, y1, x0, x1, margin)
        parity.check_maps(snr[j:j + 1, y0:y1, x0:x1].cpu().numpy(),
                          flux[j:j + 1, y0:y1, x0:x1].cpu().numpy(), ora)


# ------------------------------------------------------------------ serving: residency, streams

def test_graph_mode_replays_match_eager():
    """TNO_CFG_GRAPHS: each request is captured as a graph that updates the
    cached executable graph of its structure.  Every replay gives the eager
    request's bits, with other GPU work and synchronisations in between and
    fresh output buffers each time; a second shape gets its own graph; two
    requests of one structure in flight at once each get an executable."""
    R, sigma, times, vel = _rand_problem(60, 12, 50, 170, 4)
    R2, sigma2, times2, vel2 = _rand_problem(61, 9, 37, 133, 3)
    ref, _ = run_gpu(R, sigma, times, vel, float(times[0]), top_k=10)
    ref2, _ = run_gpu(R2, sigma2, times2, vel2, float(times2[0]), top_k=10)

    def same(g, r):
        return (np.array_equal(g["snr"], r["snr"]) and np.array_equal(g["flux"], r["flux"])
                and np.array_equal(g["best_traj"], r["best_traj"]) and g["topk"] == r["topk"])

    with tno.Search(0, own_streams=True, graphs=True) as h:
        for rep in range(4):
            print("graph replay", rep, flush=True)
            g, res = run_gpu(R, sigma, times, vel, float(times[0]), top_k=10, handle=h)
            assert same(g, ref) and res.search_ms == 0.0 and res.device_ms > 0.0
            x = torch.randn((512, 512), device=DEV)
            float((x @ x).sum())
            torch.cuda.synchronize()
            g2, _ = run_gpu(R2, sigma2, times2, vel2, float(times2[0]), top_k=10, handle=h)
            assert same(g2, ref2)
        # two requests of the same structure in flight together
        Rt, st_, tt, vt = _to(R), _to(sigma), _to(times), _to(vel)
        outs = [tno.alloc_outputs(vel.shape[0], R.shape[1], R.shape[2], 10, device=DEV) for _ in range(2)]
        reqs = [tno.make_request(Rt, st_, tt, vt, t_ref=float(times[0]), top_k=10) for _ in range(2)]
        torch.cuda.synchronize()
        tickets = [h.submit(r, o[1]) for r, o in zip(reqs, outs)]
        for t in tickets:
            h.wait(t)
        for o, _ in outs:
            assert np.array_equal(o["snr"].cpu().numpy(), ref["snr"])


def test_resident_stack_reuse_and_key_errors():
    R, sigma, times, vel = _rand_problem(50, 10, 40, 150, 3)
    ref, _ = run_gpu(R, sigma, times, vel, float(times[0]), top_k=8)
    t = [_to(R), _to(sigma), _to(times), _to(vel)]
    J, (T, H, W) = 3, R.shape
    with tno.Search(0, own_streams=True) as h:
        torch.cuda.synchronize()
        o1, out1 = tno.alloc_outputs(J, H, W, 8)
        req = tno.make_request(*t, t_ref=float(times[0]), top_k=8, stack_key=77)
        h.wait(h.submit(req, out1))
        o2, out2 = tno.alloc_outputs(J, H, W, 8)
        req2 = tno.make_request(*t, t_ref=float(times[0]), top_k=8, stack_key=77)
        req2.residuals = None       # served from the resident copy
        h.wait(h.submit(req2, out2))
        torch.cuda.synchronize()
        for o in (o1, o2):
            assert np.array_equal(o["snr"].cpu().numpy(), ref["snr"])
        req3 = tno.make_request(*t, t_ref=float(times[0]), top_k=8, stack_key=78)
        req3.residuals = None
        rc, _ = tno.tno_search_submit(h.h, req3, out2)
        assert rc == tno.TNO_E_INVAL
        req4 = tno.make_request(t[0][:5], t[1], t[2][:5], t[3], top_k=8, stack_key=77)
        rc, _ = tno.tno_search_submit(h.h, req4, out2)
        assert rc == tno.TNO_E_INVAL      # same key, other shape


def test_concurrent_requests_match_alone():
    """Requests in flight together on the library's stream pool give the same
    bits as each request alone."""
    probs = [_rand_problem(60 + i, 6 + 3 * i, 40 + 7 * i, 130 + 20 * i, 2 + i) for i in range(4)]
    alone = [run_gpu(R, s, t, v, float(t[0]), top_k=5)[0] for (R, s, t, v) in probs]
    keep = []
    with tno.Search(0, own_streams=True) as h:
        tickets = []
        for i, (R, s, t, v) in enumerate(probs):
            tt = [_to(R), _to(s), _to(t), _to(v)]
            o, out = tno.alloc_outputs(v.shape[0], R.shape[1], R.shape[2], 5)
            torch.cuda.synchronize()
            keep.append((tt, o, out))
            tickets.append(h.submit(tno.make_request(*tt, t_ref=float(t[0]), top_k=5), out))
        for tk in reversed(tickets):
            h.wait(tk)
    for (tt, o, out), a in zip(keep, alone):
        assert np.array_equal(o["snr"].cpu().numpy(), a["snr"])
        assert np.array_equal(o["best_traj"].cpu().numpy(), a["best_traj"])


def test_lru_eviction_under_budget():
    R, sigma, times, vel = _rand_problem(70, 8, 64, 128, 2)
    t = [_to(R), _to(sigma), _to(times), _to(vel)]
    o, out = tno.alloc_outputs(2, 64, 128, 4)
    with tno.Search(0, own_streams=True) as h0:
        torch.cuda.synchronize()
        h0.wait(h0.submit(tno.make_request(*t, top_k=4, stack_key=1), out))
    stack_bytes = R.nbytes + sigma.nbytes + 1024
    with tno.Search(0, own_streams=True, hbm_budget_bytes=1) as tiny:
        rc, _ = tno.tno_search_submit(tiny.h, tno.make_request(*t, top_k=4), out)
        assert rc == tno.TNO_E_NOMEM
    import ctypes
    req = tno.make_request(*t, top_k=4)
    # footprint of the arena alone (device pointers: estimate from a host twin)
    hostreq = tno.tno_request()
    ctypes.memmove(ctypes.byref(hostreq), ctypes.byref(req), ctypes.sizeof(req))
    hostreq.flags = 0
    keep = [R, sigma, times, vel]
    hostreq.residuals = R.ctypes.data_as(ctypes.c_void_p)
    hostreq.sigma = sigma.ctypes.data_as(ctypes.c_void_p)
    hostreq.times = times.ctypes.data_as(ctypes.c_void_p)
    hostreq.velocities = vel.ctypes.data_as(ctypes.c_void_p)
    hostreq.stack_key = 5
    fp = tno.tno_search_footprint(hostreq, out)
    assert fp > 0
    # room for one request's arena and two resident stacks, not three
    with tno.Search(0, own_streams=True, hbm_budget_bytes=fp + stack_bytes) as h:
        for key in (1, 2, 3):
            h.wait(h.submit(tno.make_request(*t, top_k=4, stack_key=key), out))
        r1 = tno.make_request(*t, top_k=4, stack_key=1)
        r1.residuals = None
        rc, _ = tno.tno_search_submit(h.h, r1, out)
        assert rc == tno.TNO_E_INVAL            # key 1 was evicted (least recently used)
        r3 = tno.make_request(*t, top_k=4, stack_key=3)
        r3.residuals = None
        h.wait(h.submit(r3, out))               # key 3 is still resident


# ------------------------------------------------------------------ batched form: tile shapes, autotuner

def _arch():
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _forced(tmp_path, name, tb, H, W, T, J):
    """A tuning cache that forces search variant `name` with trajectory
    blocks of `tb` for problems of this shape class."""
    path = tmp_path / ("tune_%s_%d.txt" % (name, tb))
    path.write_text("%s %s %s %d 1.0\n" % (_arch(), tno.shape_class(H, W, T, J), name, tb))
    return str(path)


def test_every_tile_shape_and_block_gives_identical_bits(tmp_path):
    """The k_search shapes evaluate each output with the same operation
    order, so forcing any (tile shape, trajectory block) through the tuning
    cache reproduces the bits of the first shape; the wave-shift variants add
    the horizontal taps in another order: they match the oracle and give
    the same bits for both rows-per-lane shapes and every trajectory block."""
    R, sigma, times, vel = _rand_problem(80, 11, 70, 300, 5)
    T, H, W = R.shape
    J = vel.shape[0]
    o = oracle.search(R, sigma, times, float(times[0]), vel)
    refs = {}
    for name in tno.SEARCH_VARIANTS:
        fam = "ws" if name.startswith("ws") else "k_search"
        for tb in (J, 2):
            print("variant", name, "tblock", tb, flush=True)
            with tno.Search(0, tune_cache_path=_forced(tmp_path, name, tb, H, W, T, J)) as h:
                g, res = run_gpu(R, sigma, times, vel, float(times[0]), top_k=20, handle=h)
            if fam not in refs:
                parity.check_maps(g["snr"], g["flux"], o)
                refs[fam] = g
                continue
            ref = refs[fam]
            assert np.array_equal(g["snr"], ref["snr"]) and np.array_equal(g["flux"], ref["flux"])
            assert g["topk"] == ref["topk"]
            assert np.array_equal(g["best_traj"], ref["best_traj"])


def test_tabulated_stamp_tile_shapes_give_identical_bits(tmp_path):
    """The general 5 x 5 stamp (tabulated PRF, jitter) in every k_search tile
    shape and two trajectory blocks: the bits of the first shape, which
    matches the oracle."""
    R, sigma, times, vel = _rand_problem(83, 13, 75, 290, 5)
    T, H, W = R.shape
    J = vel.shape[0]
    q = 4
    tab = synth.TabulatedPSF().table(5, q)
    jit = synth.jitter_series(synth.rng(83, 9), T, amp=0.3)
    kw = dict(prf_kind=tno.TNO_PRF_TABLE, prf_table=_to(tab), prf_q=q, jitter=_to(jit))
    o = oracle.search(R, sigma, times, float(times[0]), vel, prf_kind=oracle.PRF_TABLE, prf_table=tab,
                      prf_q=q, jitter=jit)
    ref = None
    for name in tno.SEARCH_VARIANTS:
        if name.startswith("ws"):
            continue
        for tb in (J, 2):
            print("tabulated variant", name, "tblock", tb, flush=True)
            path = tmp_path / ("tune_p_%s_%d.txt" % (name, tb))
            path.write_text("%s %s %s %d 1.0\n" % (_arch(), tno.shape_class(H, W, T, J, tabulated=True), name, tb))
            with tno.Search(0, tune_cache_path=str(path)) as h:
                g, res = tno.search_tensors(_to(R), _to(sigma), _to(times), _to(vel), t_ref=float(times[0]),
                                            top_k=20, handle=h, **kw)
            torch.cuda.synchronize()
            assert res.status == 0, res.message
            snr, flux = g["snr"].cpu().numpy(), g["flux"].cpu().numpy()
            if ref is None:
                parity.check_maps(snr, flux, o)
                ref = (snr, flux, tno.decode_candidates(g["topk"], res.n_topk))
                continue
            assert np.array_equal(snr, ref[0]) and np.array_equal(flux, ref[1])
            assert tno.decode_candidates(g["topk"], res.n_topk) == ref[2]


@pytest.mark.parametrize("dtype", ["bf16", "f16", "fp8_e4m3"])
@pytest.mark.parametrize("kind", [0, "table"])
def test_in_place_k_search_gives_the_bits_of_the_staged_stack(tmp_path, dtype, kind):
    """k_search reading a reduced-precision stack in place stores decode x
    scale x ivar into its window -- the products the staging of Z forms -- so
    it must give the bits of the same shape searching the staged copy
    (TNO_REQ_STAGE_FP32), on a ragged image wider than a tile with trails
    leaving the frame; and match the oracle on the dequantized values."""
    R, sigma, times, vel = _rand_problem(940 + (kind == "table"), 17, 70, 388, 4)
    vel = vel * 3.0
    T, H, W = R.shape
    J = vel.shape[0]
    codes = torch.empty((T, H, W), device=DEV, dtype=torch.uint8 if dtype == "fp8_e4m3" else torch.int16)
    sc = torch.empty((T, (H + 63) // 64, (W + 63) // 64), device=DEV)
    Rt = _to(R)
    assert tno.tno_quantize(T, H, W, tno.DTYPE_CODE[dtype], Rt.data_ptr(), codes.data_ptr(), sc.data_ptr(),
                            None) == 0
    torch.cuda.synchronize()
    kw = dict(dtype=dtype, scales=sc, top_k=15)
    okw = {}
    if kind == "table":
        q = 4
        tab = synth.TabulatedPSF().table(5, q)
        kw.update(prf_kind=tno.TNO_PRF_TABLE, prf_table=_to(tab), prf_q=q)
        okw = dict(prf_kind=oracle.PRF_TABLE, prf_table=tab, prf_q=q)
    got = {}
    for stage in (False, True):
        cls = tno.shape_class(H, W, T, J, tabulated=kind == "table", direct=not stage)
        path = tmp_path / ("tune_%s_%d.txt" % (dtype, stage))
        path.write_text("%s %s w4c2 %d 1.0\n" % (_arch(), cls, J))
        flags = tno.TNO_REQ_DEVICE_PTRS | (tno.TNO_REQ_STAGE_FP32 if stage else 0)
        print("k_search", dtype, kind, "staged" if stage else "in place", flush=True)
        with tno.Search(0, tune_cache_path=str(path)) as h:
            g, res = tno.search_tensors(codes, _to(sigma), _to(times), _to(vel), t_ref=float(times[0]),
                                        handle=h, flags=flags, **kw)
        torch.cuda.synchronize()
        assert res.status == 0, res.message
        got[stage] = (g["snr"].cpu().numpy(), g["flux"].cpu().numpy(), tno.decode_candidates(g["topk"], res.n_topk))
    assert np.array_equal(got[False][0], got[True][0]) and np.array_equal(got[False][1], got[True][1])
    assert got[False][2] == got[True][2]
    npdt = np.uint8 if dtype == "fp8_e4m3" else np.uint16
    deq = codec.dequantize(codes.cpu().numpy().view(npdt), sc.cpu().numpy(), dtype)
    o = oracle.search(deq, sigma, times, float(times[0]), vel, **okw)
    parity.check_maps(got[False][0], got[False][1], o)


@pytest.mark.parametrize("variant", ["ws", "ws4"])
@pytest.mark.parametrize("stamp,kind", [(1, 0), (3, 0), (5, 0), (5, 1), (3, "table"), (5, "table")])
def test_wave_shift_variant_stamps_and_edges(tmp_path, stamp, kind, variant):
    """The wave-shift search for every stamp it serves, separable and
    tabulated, on an image narrower than one tile and one several tiles wide
    with a ragged edge, trails leaving the frame: against the oracle."""
    for (H, W, T, J, seed) in [(37, 50, 23, 3, 0), (70, 390, 41, 4, 1)]:
        R, sigma, times, vel = _rand_problem(900 + seed + 10 * stamp, T, H, W, J)
        vel = vel * 3.0                     # trails well off the image
        if kind == "table":
            q = 5
            tab = synth.TabulatedPSF().table(stamp, q)
            kw = dict(prf_kind=tno.TNO_PRF_TABLE, prf_table=_to(tab), prf_q=q, stamp=stamp)
            okw = dict(prf_kind=oracle.PRF_TABLE, prf_table=tab, prf_q=q, stamp=stamp)
        else:
            kw = dict(prf_kind=kind, stamp=stamp)
            okw = dict(prf_kind=kind, stamp=stamp)
        print(variant, "stamp", stamp, "kind", kind, "shape", (T, H, W), "J", J, flush=True)
        with tno.Search(0, tune_cache_path=_forced(tmp_path, variant, J, H, W, T, J)) as h:
            g, res = tno.search_tensors(_to(R), _to(sigma), _to(times), _to(vel), t_ref=float(times[0]),
                                        top_k=10, handle=h, **kw)
        torch.cuda.synchronize()
        assert res.status == 0, res.message
        o = oracle.search(R, sigma, times, float(times[0]), vel, **okw)
        parity.check_maps(g["snr"].cpu().numpy(), g["flux"].cpu().numpy(), o)
        parity.check_topk(tno.decode_candidates(g["topk"], res.n_topk), o["snr"], 10)


def test_autotune_writes_cache_and_keeps_results(tmp_path):
    """Autotuning (which times candidates on the request's own buffers) leaves
    the request's results as a plain run of the chosen variant gives them,
    and those match the oracle."""
    R, sigma, times, vel = _rand_problem(81, 60, 100, 260, 20)
    path = tmp_path / "tune.txt"
    with tno.Search(0, autotune=True, tune_cache_path=str(path)) as h:
        g, res = run_gpu(R, sigma, times, vel, float(times[0]), top_k=10, handle=h)
    lines = [l for l in path.read_text().splitlines() if not l.startswith("#")]
    assert len(lines) == 1
    arch, cls, name, tb, rate = lines[0].split()
    assert arch == _arch() and cls == tno.shape_class(100, 260, 60, 20)
    assert name in tno.SEARCH_VARIANTS and 1 <= int(tb) <= 20 and float(rate) > 0
    print("tuned", name, tb, flush=True)
    with tno.Search(0, tune_cache_path=_forced(tmp_path, name, int(tb), 100, 260, 60, 20)) as h:
        ref, _ = run_gpu(R, sigma, times, vel, float(times[0]), top_k=10, handle=h)
    assert np.array_equal(g["snr"], ref["snr"]) and np.array_equal(g["flux"], ref["flux"])
    assert g["topk"] == ref["topk"]
    o = oracle.search(R, sigma, times, float(times[0]), vel)
    parity.check_maps(g["snr"], g["flux"], o)


# ------------------------------------------------------------------ Sec. 3.3 significance (next row)

SIG_TOL = 3e-5   # SNR inputs within 1e-5 relative; the local std inherits the same order


def _sig_check(R, sigma, times, vel, box, thr, k=64, top_k=5):
    print("significance case: T,H,W=%s J=%d box=%d thr=%g" % (tuple(R.shape), vel.shape[0], box, thr), flush=True)
    o, res = tno.search_tensors(_to(R), _to(sigma), _to(times), _to(vel), t_ref=float(times[0]),
                                top_k=top_k, sig_box=box, sig_threshold=thr, detections=k)
    torch.cuda.synchronize()
    assert res.status == 0
    ora = oracle.search(R, sigma, times, float(times[0]), vel)
    best, bj, _ = oracle.best_over_trajectories(ora["snr"], ora["flux"])
    osig = oracle.significance(best, box)
    gsig = o["significance"].cpu().numpy()
    err = np.abs(gsig - osig) / np.maximum(1.0, np.abs(osig))
    assert err.max() <= SIG_TOL, err.max()
    assert res.n_above == int(np.sum(gsig >= thr))
    band = SIG_TOL * np.maximum(1.0, np.abs(osig))
    assert np.all((osig >= thr + band) <= (gsig >= thr)) and np.all((gsig >= thr) <= (osig >= thr - band))
    dets = tno.decode_detections(o["detections"], res.n_detections)
    assert res.n_detections == min(k, res.n_above)
    H, W = best.shape
    gflat = gsig.reshape(-1)
    ref_order = np.lexsort((np.arange(gflat.size), -gflat))[:res.n_detections]
    assert [d[4] * W + d[5] for d in dets] == ref_order.tolist()   # GPU order of its own map
    for d in dets:
        y, x = d[4], d[5]
        assert d[0] == gsig[y, x] and d[0] >= thr
        assert abs(d[1] - best[y, x]) <= 1e-5 * max(1.0, abs(best[y, x]))
        assert abs(ora["snr"][d[3], y, x] - best[y, x]) <= 2e-5 * max(1.0, abs(best[y, x]))
    return gsig, osig, dets


def test_significance_tiny_config():
    p = synth.make_c1("bright")
    gsig, osig, dets = _sig_check(p.R, p.sigma, p.times, p.vel, 31, 3.0)
    assert dets and abs(dets[0][4] - 32) <= 2 and abs(dets[0][5] - 20) <= 2


@pytest.mark.parametrize("box", [1, 15, 255])
def test_significance_ragged_and_clipped_windows(box):
    R, sigma, times, vel = _rand_problem(90 + box, 7, 45, 150, 3)
    sigma[10:30, 60:120] = 0.0          # masked block: Lam = 0, scores exactly 0
    R[:, 20, 40] += 50.0                # one bright pixel
    gsig, osig, dets = _sig_check(R, sigma, times, vel, box, 2.5)
    if box == 1:
        assert np.all(gsig == 0)


def test_significance_full_size_property():
    """FFI size: significance * (population std of the best map over the
    255 x 255 clipped window, computed here independently) = best score."""
    from scipy import ndimage
    H = W = 2048
    R, sigma, times, t_ref, vel, src = synth.make_ffi_like_torch(H, W, 1000, DEV)
    o, res = tno.search_tensors(R, _to(sigma), _to(times), _to(vel), t_ref=t_ref, top_k=10,
                                sig_box=255, sig_threshold=5.0, detections=256, maps=False)
    torch.cuda.synchronize()
    best = o["best_snr"].cpu().numpy().astype(np.float64)
    gsig = o["significance"].cpu().numpy()
    ones = np.ones_like(best)
    n = ndimage.uniform_filter(ones, 255, mode="constant") * 255 ** 2
    s1 = ndimage.uniform_filter(best, 255, mode="constant") * 255 ** 2
    s2 = ndimage.uniform_filter(best * best, 255, mode="constant") * 255 ** 2
    sd = np.sqrt(np.maximum(s2 / n - (s1 / n) ** 2, 0))
    ref = best / sd
    err = np.abs(gsig - ref) / np.maximum(1.0, np.abs(ref))
    assert err.max() <= 1e-5
    assert res.n_above == int(np.sum(gsig >= 5.0))
    dets = tno.decode_detections(o["detections"], res.n_detections)
    assert res.n_detections == min(256, res.n_above)
    # injected sources bright enough in SNR come out as detections near their start
    found = 0
    for s in src:
        yr, xr = int(round(s.y)), int(round(s.x))
        if gsig[max(0, yr - 1):yr + 2, max(0, xr - 1):xr + 2].max() >= 5.0:
            found += any(abs(d[4] - yr) <= 1 and abs(d[5] - xr) <= 1 for d in dets)
    print("sources detected at 5 sigma:", found, "of", len(src), "; pixels above:", res.n_above, flush=True)
