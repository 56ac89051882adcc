"""Serving form with continuous batching: a Poisson stream of uneven requests
(cutouts 256-512 px, 60-160 frames, 8-48 trajectories of the shell bank, BF16
stacks resident under stack keys) arrives faster than it is served, so the
searches of admitted requests share steps (also with trajectory slabs of 8 MiB,
a request's slabs joining steps one after another).  Every result must be the result
of the same request run alone, bit for bit; two requests also go to the FP64
oracle on their dequantized stacks."""
import numpy as np
import pytest
import torch

from oracle import codec, oracle
from paper_2209_09848_amd import serve, synth, tno
from tests import parity

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
K = 16


def _alone(pool, spec, bank, dtype):
    codes, scales = pool.residuals(spec.key)
    sig, times = pool.inputs(spec.key)
    vel = torch.from_numpy(bank[spec.traj_idx]).to(DEV).contiguous()
    o, res = tno.search_tensors(codes, sig, times, vel, top_k=K, maps=False, dtype=dtype, scales=scales)
    torch.cuda.synchronize()
    assert res.status == 0, res.message
    return o, res, codes, scales, sig, times


@pytest.mark.parametrize("mode,slab_bytes", [("batch", 0), ("eager", 0), ("batch", 8 << 20)],
                         ids=["batch", "eager", "batch_slabs"])
def test_stream_results_equal_alone(mode, slab_bytes):
    bank, _ = synth.grid_shells()
    shapes = serve.draw_stack_shapes(5, seed=7, sides=[256, 384, 512], frames=(60, 160))
    specs = serve.draw_requests(20, shapes, bank.shape[0], seed=7, jrange=(8, 48))
    specs = serve.poisson_arrivals(specs, rate=400.0, seed=7)
    stats = {}
    print("serving 20 requests, mode", mode, flush=True)
    recs = serve.run_stream(specs, bank, dtype="bf16", mode=mode, keep=True, max_inflight=8, top_k=K,
                            stats=stats, slab_bytes=slab_bytes)
    print("stats", stats, flush=True)
    assert len(recs) == 20
    if mode == "batch":
        # every work item (128 x 32 tile, trajectory: the in-place BF16 search's
        # shape) went through a step, and steps served several requests at once
        items = sum(-(-r["side"] // 128) * -(-r["side"] // 32) * r["traj"] for r in recs)
        assert stats["batch_items"] == items
        assert stats["batch_steps"] > 0 and stats["batch_shared"] > 0
    pool = serve.StackPool(shapes, "bf16", DEV)
    checked = 0
    for r in sorted(recs, key=lambda x: (x["side"] * x["side"] * x["frames"] * x["traj"])):
        s = r["spec"]
        print("alone: key %d %dx%dx%d J=%d" % (s.key, s.side, s.side, s.frames, len(s.traj_idx)), flush=True)
        o, res, codes, scales, sig, times = _alone(pool, s, bank, "bf16")
        assert r["topk"] == tno.decode_candidates(o["topk"], res.n_topk)
        assert np.array_equal(r["traj_max"], o["traj_max"].cpu().numpy())
        assert np.array_equal(r["best_snr"], o["best_snr"].cpu().numpy())
        assert np.array_equal(r["best_traj"], o["best_traj"].cpu().numpy())
        if checked < 2 and mode == "batch":
            # the FP64 oracle on the dequantized stack
            cc = codes.cpu().numpy().view(np.uint16)
            deq = codec.dequantize(cc, scales.cpu().numpy(), "bf16")
            ora = oracle.search(deq, sig.cpu().numpy(), times.cpu().numpy(), float(times[0]),
                                bank[s.traj_idx])
            parity.check_topk(r["topk"], ora["snr"], K)
            peaks = tno.decode_peaks(torch.from_numpy(r["traj_max"]))
            parity.check_traj_max(peaks, ora["snr"], ora["flux"])
            checked += 1
    print("20 requests equal alone; %d checked against the oracle" % checked, flush=True)


def test_admission_accounts_the_blocks_it_holds():
    """Uneven requests under a tight HBM budget (requests wait for room):
    at every round of polls the bytes the handle counts as in use equal the
    device blocks that live requests and resident stacks hold, and in-use
    plus cached bytes stay within the budget."""
    bank, _ = synth.grid_shells()
    shapes = serve.draw_stack_shapes(4, seed=11, sides=[256, 384, 512], frames=(60, 160))
    specs = serve.draw_requests(16, shapes, bank.shape[0], seed=11, jrange=(8, 48))
    specs = serve.poisson_arrivals(specs, rate=1000.0, seed=11)
    seen = {"polls": 0, "max_in_use": 0}

    def check(h):
        st = tno.tno_search_stats(h.h)
        assert st.in_use_bytes == st.held_bytes, (st.in_use_bytes, st.held_bytes)
        assert st.in_use_bytes + st.cached_bytes <= st.budget_bytes
        seen["polls"] += 1
        seen["max_in_use"] = max(seen["max_in_use"], st.in_use_bytes)

    budget_gb = 0.6
    recs = serve.run_stream(specs, bank, dtype="bf16", budget_gb=budget_gb, max_inflight=8, top_k=K,
                            on_poll=check)
    assert len(recs) == 16 and seen["polls"] > 0
    print("polls %d, most bytes in use %.3g GB of %.3g" % (seen["polls"], seen["max_in_use"] / 1e9, budget_gb),
          flush=True)
