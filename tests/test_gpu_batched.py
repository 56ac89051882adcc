"""Batched form: a 1024 x 1024 px x 1000-frame BF16 stack searched with 2048
trajectories in eight uneven shells (0.005-0.3 px/frame, inclinations 0-60
deg, 96-512 per shell) in one launch, tile shape and trajectory block chosen
by the autotuner.  Parity on sampled start pixels against the oracle on the
dequantized stack; reductions against torch on the GPU's own maps."""
import math

import numpy as np
import pytest
import torch

from oracle import codec, oracle
from paper_2209_09848_amd import synth, tno
from tests import parity

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

DEV = "cuda:0"


def _to(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def test_batched_shells_bf16_autotuned(tmp_path):
    H = W = 1024
    T = 1000
    bank, shell = synth.grid_shells()
    J = bank.shape[0]
    assert J == 2048 and np.bincount(shell).tolist() == [512, 384, 320, 256, 192, 160, 128, 96]
    print("generating the batched-form stack", flush=True)
    R, sigma, times, t_ref, vel, src = synth.make_ffi_like_torch(H, W, T, DEV, bank=bank, config_id=4,
                                                                 n_sources=20, amp=(0.1, 0.5))
    nq = (H + 63) // 64
    codes = torch.empty((T, H, W), dtype=torch.int16, device=DEV)
    scales = torch.empty((T, nq, nq), dtype=torch.float32, device=DEV)
    assert tno.tno_quantize(T, H, W, tno.TNO_BF16, R.data_ptr(), codes.data_ptr(), scales.data_ptr(),
                            torch.cuda.current_stream().cuda_stream) == 0
    torch.cuda.synchronize()
    cache = tmp_path / "tune.txt"
    with tno.Search(0, autotune=True, tune_cache_path=str(cache)) as h:
        o, res = tno.search_tensors(codes, _to(sigma), _to(times), _to(vel), t_ref=t_ref, top_k=100,
                                    dtype="bf16", scales=scales, handle=h)
        torch.cuda.synchronize()
        first = res.device_ms
        o, res = tno.search_tensors(codes, _to(sigma), _to(times), _to(vel), t_ref=t_ref, top_k=100,
                                    dtype="bf16", scales=scales, handle=h)
        torch.cuda.synchronize()
    lines = [l for l in cache.read_text().splitlines() if not l.startswith("#")]
    print("tuned:", lines, "first request %.1f ms (with tuning), then %.1f ms (search %.1f): %.3g updates/s"
          % (first, res.device_ms, res.search_ms, res.updates / (res.device_ms * 1e-3)), flush=True)
    assert len(lines) == 1 and lines[0].split()[1] == tno.shape_class(H, W, T, J, direct=True)
    snr, flux = o["snr"], o["flux"]
    # reductions on the GPU's own maps
    best = snr.max(dim=0).values
    assert torch.equal(o["best_snr"], best)
    # (J*H*W > INT_MAX: the top 100 of every trajectory's top 100)
    tv = torch.topk(torch.topk(snr.reshape(J, -1), 100, dim=1).values.reshape(-1), 100).values.cpu().numpy()
    cands = tno.decode_candidates(o["topk"], res.n_topk)
    assert np.array_equal(np.array([c[0] for c in cands], np.float32), tv)
    # oracle on the dequantized stack: 8x8 start pixels, one trajectory per
    # shell direction extreme, crops aligned to the quantisation tiles
    js = [0, 127, 511, 700, 1100, 1400, 1700, 2047]
    deq_full = None
    for (y0, x0) in [(500, 480), (8, 1000)]:
        y1, x1 = y0 + 8, x0 + 8
        vj = vel[js]
        margin = int(math.ceil(np.abs(vj).max() * (times.max() - t_ref))) + 4
        cy0, cy1 = max(0, (y0 - margin) // 64 * 64), min(H, -(-(y1 + margin) // 64) * 64)
        cx0, cx1 = max(0, (x0 - margin) // 64 * 64), min(W, -(-(x1 + margin) // 64) * 64)
        cc = codes[:, cy0:cy1, cx0:cx1].cpu().numpy().view(np.uint16)
        sc = scales[:, cy0 // 64:cy1 // 64 if cy1 % 64 == 0 else cy1 // 64 + 1,
                    cx0 // 64:cx1 // 64 if cx1 % 64 == 0 else cx1 // 64 + 1].cpu().numpy()
        deq = codec.dequantize(cc, sc, "bf16").astype(np.float32)
        print("oracle crop", (cy0, cy1, cx0, cx1), flush=True)
        ora = oracle.search(deq, sigma[cy0:cy1, cx0:cx1], times, t_ref, vj,
                            region=(y0 - cy0, y1 - cy0, x0 - cx0, x1 - cx0))
        parity.check_maps(snr[js, y0:y1, x0:x1].cpu().numpy(), flux[js, y0:y1, x0:x1].cpu().numpy(), ora)
