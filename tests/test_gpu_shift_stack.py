"""Shift-stack baseline vs the PRF matched filter (Sec. 3.2's "error about
sqrt(2) lower" remark, measured rather than pinned: the paper prints no number).

The shift-stack filter is the 1x1 stamp: one weight of 1 at the pixel nearest
the trajectory in every frame.  For the same injected sources, the ratio of
the matched filter's SNR to the shift-stack's SNR at the true hypothesis is
reported (noise-free: the deterministic ratio, checked against the oracle;
with noise: the ratio of the mean recovered SNRs).
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle
from paper_2209_09848_amd import synth, tno

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _to(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _truth_snr(R, sigma, times, t_ref, vel, src, stamp):
    o, res = tno.search_tensors(R, _to(sigma), _to(times), _to(vel), t_ref=t_ref, top_k=0,
                                stamp=stamp)
    torch.cuda.synchronize()
    snr = o["snr"]
    out = []
    for s in src:
        out.append(float(snr[s.traj, int(math.floor(s.y + 0.5)), int(math.floor(s.x + 0.5))]))
    return np.array(out)


def test_matched_filter_vs_shift_stack_ratio():
    H = W = 1024
    T = 500
    R, sigma, times, t_ref, vel, src = synth.make_ffi_like_torch(H, W, T, DEV, amp=(0.2, 1.0),
                                                                 config_id=6)
    # noise-free copy: the sources alone
    k, y, x, v = synth.render_sources((T, H, W), times, t_ref, src)
    Rn = torch.zeros((T, H, W), dtype=torch.float32, device=DEV)
    Rn.index_put_((torch.from_numpy(k).to(DEV), torch.from_numpy(y).to(DEV),
                   torch.from_numpy(x).to(DEV)), torch.from_numpy(v.astype(np.float32)).to(DEV),
                  accumulate=True)
    mf0 = _truth_snr(Rn, sigma, times, t_ref, vel, src, 5)
    ss0 = _truth_snr(Rn, sigma, times, t_ref, vel, src, 1)
    ratio0 = mf0 / ss0
    # the oracle's ratio on a few sources (crop around each trail)
    Rh = Rn.cpu().numpy()
    for i in range(4):
        s = src[i]
        yr, xr = int(math.floor(s.y + 0.5)), int(math.floor(s.x + 0.5))
        hyp = [s.traj], [yr], [xr]
        o5 = oracle.hypotheses(Rh, sigma, times, t_ref, vel, *hyp, stamp=5)["snr"][0]
        o1 = oracle.hypotheses(Rh, sigma, times, t_ref, vel, *hyp, stamp=1)["snr"][0]
        assert abs(mf0[i] - o5) <= 1e-5 * max(1.0, abs(o5))
        assert abs(ss0[i] - o1) <= 1e-5 * max(1.0, abs(o1))
    mf = _truth_snr(R, sigma, times, t_ref, vel, src, 5)
    ss = _truth_snr(R, sigma, times, t_ref, vel, src, 1)
    print("SHIFTSTACK noise-free ratio mean %.3f min %.3f max %.3f; noisy mean SNR %.2f vs %.2f "
          "(ratio %.3f); sqrt(2) = %.3f" % (ratio0.mean(), ratio0.min(), ratio0.max(), mf.mean(),
                                            ss.mean(), mf.mean() / ss.mean(), math.sqrt(2)), flush=True)
    # the full PRF filter gains over the one-pixel filter for every source;
    # on average the gain lies between the closed forms of a static source at
    # the centred phase (1.26) and at the half-pixel phase (2.0) in both axes
    # (single sources exceed 2.0 where the start sits near a pixel corner)
    assert np.all(ratio0 > 1.0)
    assert 1.26 < ratio0.mean() < 2.0
    assert 1.2 < mf.mean() / ss.mean() < 2.0
