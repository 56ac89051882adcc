"""tno_search_run_scratch: the search without device allocation (its working
memory is the library's fixed per-GPU array) against the ticketed search
(tno_search_submit / poll) on the same inputs: identical bits, on two calls in
a row (the second smaller, so it runs over what the first left in the array)
and one reduced-precision call whose maps stay inside the array; a request
whose normaliser and maps for all trajectories exceed the array runs in
trajectory slabs; a request whose working memory exceeds the array is
refused."""
import numpy as np
import pytest
import torch

from paper_2209_09848_amd import synth, tno

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _to(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _problem(seed, T, H, W, J):
    g = np.random.default_rng(seed)
    R = g.standard_normal((T, H, W)).astype(np.float32)
    sigma = synth.sigma_lognormal(g, H, W)
    sigma[g.integers(0, H), g.integers(0, W)] = 0.0          # a masked pixel
    times = synth.times_with_gap(T, T // 2, 0.9)
    vel = g.uniform(-20.0, 20.0, size=(J, 2))
    return R, sigma, times, vel


def _outputs(o, res, maps=True):
    d = {"best_snr": o["best_snr"].cpu().numpy(), "best_traj": o["best_traj"].cpu().numpy(),
         "traj_max": o["traj_max"].cpu().numpy(), "topk": o["topk"][:res.n_topk].cpu().numpy()}
    if maps:
        d["snr"] = o["snr"].cpu().numpy()
        d["flux"] = o["flux"].cpu().numpy()
    return d


def _same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def _compare(R, sigma, times, vel, k=10, maps=True, **kw):
    T, H, W = R.shape
    J = vel.shape[0]
    t = [R if isinstance(R, torch.Tensor) else _to(R), _to(sigma), _to(times), _to(vel)]
    # the ticketed search
    o_ref, r_ref = tno.search_tensors(*t, t_ref=float(times[0]), top_k=k, maps=maps, **kw)
    torch.cuda.synchronize()
    assert r_ref.status == 0, r_ref.message
    # the same request without allocation, on a stream of its own
    o, out = tno.alloc_outputs(J, H, W, k, device=DEV, maps=maps)
    req = tno.make_request(*t, t_ref=float(times[0]), top_k=k, **kw)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    rc, res = tno.tno_search_run_scratch(req, out, s.cuda_stream)
    assert rc == tno.TNO_OK, res.message
    assert res.status == 0 and res.n_topk == min(k, J * H * W) and res.updates == J * T * H * W
    _same(_outputs(o, res, maps), _outputs(o_ref, r_ref, maps))


def test_scratch_search_matches_ticketed_search():
    print("scratch search: call 1 (70 x 260 x 20 frames, 4 trajectories)", flush=True)
    _compare(*_problem(1, 20, 70, 260, 4), k=12)
    print("scratch search: call 2, smaller (37 x 133 x 9 frames, 3 trajectories)", flush=True)
    _compare(*_problem(2, 9, 37, 133, 3), k=7)
    print("scratch search: call 3, BF16 in place, maps only inside the array", flush=True)
    R, sigma, times, vel = _problem(3, 11, 40, 128, 3)
    T, H, W = R.shape
    Rt = _to(R)
    codes = torch.empty((T, H, W), dtype=torch.int16, device=DEV)
    scales = torch.empty((T, (H + 63) // 64, (W + 63) // 64), dtype=torch.float32, device=DEV)
    assert tno.tno_quantize(T, H, W, tno.TNO_BF16, Rt.data_ptr(), codes.data_ptr(), scales.data_ptr(),
                            None) == 0
    torch.cuda.synchronize()
    _compare(codes, sigma, times, vel, k=9, maps=False, dtype="bf16", scales=scales)


def test_scratch_search_in_trajectory_slabs():
    """A request whose normaliser and maps for all trajectories exceed the
    array runs in trajectory slabs of a quarter of it (here 3 slabs of at
    most 8 of 20 trajectories), with the bits of the ticketed search (one
    slab)."""
    print("scratch search: BF16 in place, 512 x 512 x 24 frames, 20 trajectories in slabs", flush=True)
    R, sigma, times, vel = _problem(4, 24, 512, 512, 20)
    T, H, W = R.shape
    Rt = _to(R)
    codes = torch.empty((T, H, W), dtype=torch.int16, device=DEV)
    scales = torch.empty((T, (H + 63) // 64, (W + 63) // 64), dtype=torch.float32, device=DEV)
    assert tno.tno_quantize(T, H, W, tno.TNO_BF16, Rt.data_ptr(), codes.data_ptr(), scales.data_ptr(),
                            None) == 0
    torch.cuda.synchronize()
    assert 20 * H * W * 16 > tno.TNO_SCRATCH_BYTES // 4
    _compare(codes, sigma, times, vel, k=40, maps=False, dtype="bf16", scales=scales)


def test_scratch_search_refuses_what_does_not_fit():
    T, H, W, J = 64, 512, 512, 8           # staged stack > 100 MiB, Lam 16 MiB, maps 16 MiB
    R = torch.zeros((T, H, W), dtype=torch.float32, device=DEV)
    sigma = torch.ones((H, W), dtype=torch.float32, device=DEV)
    times = _to(synth.times_uniform(T))
    vel = _to(np.full((J, 2), 10.0))
    req = tno.make_request(R, sigma, times, vel, top_k=5)
    o, out = tno.alloc_outputs(J, H, W, 5, device=DEV, maps=False)
    rc, res = tno.tno_search_run_scratch(req, out, None)
    assert rc == tno.TNO_E_NOMEM and res.status == tno.TNO_E_NOMEM
    assert b"working memory" in res.message
    # without device pointers the request is refused before any work
    req.flags = 0
    rc, res = tno.tno_search_run_scratch(req, out, None)
    assert rc == tno.TNO_E_INVAL
