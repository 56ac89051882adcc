"""Trajectory slabs: a request searched a few trajectories at a time (runs
of its velocity-sorted search order; the normaliser and the SNR/flux maps
held for one slab only, rows copied out to maps the caller asked for; bank
maximum, per-trajectory peaks and top-k merged slab after slab) must give the
bits of the same request searched as one slab, with and
without caller maps, for staged FP32 and in-place BF16 stacks, eager and
batched; the slabbed result is also checked against the FP64 oracle, and an
all-tie case against the order the outputs define.
"""
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


def _run(R, sigma, times, vel, t_ref, *, slab_bytes, maps, k, box=0, ndet=0, dtype="f32", scales=None,
         batch=False, flux_map=True):
    T, H, W = (int(s) for s in R.shape)
    J = int(vel.shape[0])
    o, out = tno.alloc_outputs(J, H, W, k, device=DEV, maps=maps, detections=ndet)
    if maps and not flux_map:
        out.flux = None
        del o["flux"]
    req = tno.make_request(R, _to(sigma), _to(times), _to(vel), t_ref=t_ref, top_k=k, dtype=dtype,
                           scales=scales, sig_box=box, sig_threshold=3.0)
    with tno.Search(0, slab_bytes=slab_bytes, batch=batch) as h:
        res = h.wait(h.submit(req, out))
    torch.cuda.synchronize()
    assert res.status == 0, res.message
    g = {n: t.cpu().numpy() for n, t in o.items()}
    g["n_topk"] = res.n_topk
    g["n_det"] = res.n_detections
    return g


def _same(a, b, keys):
    for n in keys:
        if n in a and n in b:
            assert np.array_equal(a[n], b[n]), n
    assert a["n_topk"] == b["n_topk"] and a["n_det"] == b["n_det"]


CASES = [
    # (H, W, T, speeds, dirs, k, dtype): ragged tiles, short last slabs,
    # top-k beyond a slab's first trajectory
    (200, 260, 40, 6, 6, 700, "f32"),
    (136, 192, 48, 5, 5, 300, "bf16"),
]


@pytest.mark.parametrize("case", CASES, ids=["f32", "bf16"])
def test_slabs_give_the_bits_of_one_slab(case):
    H, W, T, ns, nd, k, dtype = case
    p = synth.make_ffi_like(H, W, T, J_speeds=ns, J_dirs=nd, n_sources=6, config_id=41)
    J = p.vel.shape[0]
    scales = None
    R = _to(p.R)
    if dtype != "f32":
        codes = torch.empty((T, H, W), device=DEV, dtype=torch.int16)
        sc = torch.empty((T, (H + 63) // 64, (W + 63) // 64), device=DEV)
        assert tno.tno_quantize(T, H, W, tno.DTYPE_CODE[dtype], R.data_ptr(), codes.data_ptr(),
                                sc.data_ptr(), None) == 0
        torch.cuda.synchronize()
        R, scales = codes, sc
    HW = H * W
    kw = dict(k=k, box=21, ndet=40, dtype=dtype, scales=scales)
    print("slab case: %dx%dx%d J=%d k=%d %s" % (H, W, T, J, k, dtype), flush=True)
    ref = _run(R, p.sigma, p.times, p.vel, p.t_ref, slab_bytes=0, maps=True, **kw)
    keys = ("best_snr", "best_traj", "traj_max", "topk", "significance", "detections", "snr", "flux")
    # slabs of 4, 3 and 2 trajectories (a slab holds 16 bytes per start pixel
    # and trajectory: Lam and its SNR and flux rows), without caller maps,
    # with both, with the SNR map only
    for maps, flux_map, sb in ((False, True, 4 * HW * 16), (True, True, 3 * HW * 16), (True, False, 2 * HW * 16)):
        print("  maps=%s flux=%s slab_bytes=%d" % (maps, flux_map, sb), flush=True)
        got = _run(R, p.sigma, p.times, p.vel, p.t_ref, slab_bytes=sb, maps=maps, flux_map=flux_map, **kw)
        _same(got, ref, keys)
    print("  batched, slabs of 4", flush=True)
    got = _run(R, p.sigma, p.times, p.vel, p.t_ref, slab_bytes=4 * HW * 16, maps=False, batch=True, **kw)
    _same(got, ref, keys)
    # the slabbed search against the FP64 oracle
    Rh = p.R
    if dtype != "f32":
        Rh = codec.dequantize(R.cpu().numpy().view(np.uint16), scales.cpu().numpy(), dtype)
    ora = oracle.search(Rh, p.sigma, p.times, p.t_ref, p.vel)
    parity.check_best(got["best_snr"], got["best_traj"], ora["snr"])
    parity.check_traj_max(tno.decode_peaks(torch.from_numpy(got["traj_max"])), ora["snr"], ora["flux"])
    parity.check_topk(tno.decode_candidates(torch.from_numpy(got["topk"]), got["n_topk"]), ora["snr"], k)
    assert J > 8


def test_slabs_keep_the_tie_order():
    """A zero stack scores 0 everywhere: the bank maximum goes to trajectory 0
    at every pixel, each trajectory's peak to pixel 0, and the top-k to the
    first k flat indices (trajectory 0's pixels in row-major order, then
    trajectory 1's) -- across slab boundaries too."""
    H, W, T = 24, 28, 12
    R = torch.zeros((T, H, W), device=DEV)
    sigma = np.ones((H, W), np.float32)
    times = synth.times_uniform(T)
    vel = synth.grid_speeds_directions(3, 3, 0.01, 0.2)
    k = H * W + 100          # beyond the first trajectory
    for sb in (0, 2 * H * W * 16):
        print("tie case slab_bytes=%d" % sb, flush=True)
        g = _run(R, sigma, times, vel, float(times[0]), slab_bytes=sb, maps=False, k=k)
        assert np.all(g["best_snr"] == 0) and np.all(g["best_traj"] == 0)
        _, _, py, px = tno.decode_peaks(torch.from_numpy(g["traj_max"]))
        assert np.all(py == 0) and np.all(px == 0)
        cands = tno.decode_candidates(torch.from_numpy(g["topk"]), g["n_topk"])
        want = [(i // (H * W), (i % (H * W)) // W, i % W) for i in range(k)]
        assert [(c[2], c[3], c[4]) for c in cands] == want
