"""Serving driver: a Poisson stream of uneven search requests against one handle.

Requests differ in cutout size (256..2048 px, multiples of 256), frame count
(200..1000) and trajectory set (16..256 drawn from the uneven-shell bank).
Residual stacks live on the device under stack keys drawn from a pool (about
half the requests reuse a resident stack); the library's stream pool runs
admitted requests concurrently and its budget admission refuses work
(TNO_E_BUSY) until memory or slots free up, in which case the request waits
in this driver's FIFO.  Latency = completion seen by poll - arrival time.

The driver marshals requests only; the search runs in libtno_search.so.
"""
from __future__ import annotations

import argparse
import collections
import json
import math
import sys
import time
from dataclasses import dataclass

import numpy as np

from . import synth, tno


@dataclass
class Spec:
    key: int
    side: int
    frames: int
    traj_idx: np.ndarray     # rows of the shell bank
    arrival: float = 0.0


def draw_stack_shapes(n_keys: int, seed: int, sides=None, frames=(200, 1000)):
    g = synth.rng(5, 3, seed)
    sides = sides or [256 * i for i in range(1, 9)]
    return {k + 1: (int(g.choice(sides)), int(g.integers(frames[0], frames[1] + 1)))
            for k in range(n_keys)}


def draw_requests(n: int, shapes: dict, bank_size: int, seed: int, jrange=(16, 256),
                  reuse: float = 0.5):
    """n request specs; a request reuses the previous key with probability
    `reuse`, else draws a key from the pool."""
    g = synth.rng(5, 3, 1000 + seed)
    keys = sorted(shapes)
    out = []
    prev = None
    for _ in range(n):
        if prev is not None and g.random() < reuse:
            key = prev
        else:
            key = int(g.choice(keys))
        prev = key
        side, frames = shapes[key]
        J = int(g.integers(jrange[0], jrange[1] + 1))
        idx = np.sort(g.choice(bank_size, size=J, replace=False))
        out.append(Spec(key, side, frames, idx))
    return out


def poisson_arrivals(specs, rate: float, seed: int):
    g = synth.rng(5, 3, 2000 + seed)
    t = 0.0
    for s in specs:
        t += float(g.exponential(1.0 / rate))
        s.arrival = t
    return specs


class StackPool:
    """Device-side residual stacks by key, drawn on first use and handed to the
    library once (it keeps its own resident copy); later requests on the key
    pass no residuals."""

    def __init__(self, shapes, dtype, device):
        import torch
        self.torch = torch
        self.shapes = shapes
        self.dtype = dtype
        self.device = device
        self.sigma = {}
        self.times = {}

    def inputs(self, key):
        torch = self.torch
        side, frames = self.shapes[key]
        if key not in self.sigma:
            g = synth.rng(5, 0, key)
            self.sigma[key] = torch.from_numpy(synth.sigma_lognormal(g, side, side)).to(self.device)
            self.times[key] = torch.from_numpy(synth.times_with_gap(frames, frames // 2)).to(self.device)
        return self.sigma[key], self.times[key]

    def residuals(self, key):
        """Freshly drawn stack (and scales) for the first submission of `key`."""
        torch = self.torch
        side, frames = self.shapes[key]
        sig, _ = self.inputs(key)
        gen = torch.Generator(device=self.device)
        gen.manual_seed(key)
        R = torch.randn((frames, side, side), generator=gen, device=self.device)
        R.mul_(sig)   # in place: the draw holds one stack-sized buffer
        if self.dtype == "f32":
            return R, None
        codes = torch.empty((frames, side, side), device=self.device,
                            dtype=torch.uint8 if self.dtype == "fp8_e4m3" else torch.int16)
        scales = torch.empty((frames, (side + 63) // 64, (side + 63) // 64), device=self.device)
        rc = tno.tno_quantize(frames, side, side, tno.DTYPE_CODE[self.dtype], R.data_ptr(),
                              codes.data_ptr(), scales.data_ptr(),
                              torch.cuda.current_stream().cuda_stream)
        if rc != 0:
            raise tno.TnoError(rc, tno.tno_search_last_error())
        torch.cuda.current_stream().synchronize()
        del R
        return codes, scales


HANDOVERS = 2                  # requests in flight that hold a stack being handed over
MAX_SIDE = 1024                # largest cutout side of a mix this driver runs
RUNTIME_MARGIN = 8 << 30       # device bytes left to the HIP runtime (scratch, queues)


def run_stream(specs, bank, dtype="bf16", budget_gb=0.0, device="cuda:0", top_k=16,
               max_inflight=8, log=None, mode="eager", keep=False, stats=None, slab_bytes=0,
               stage_fp32=False, on_poll=None, reserve=True):
    """Serve `specs` in arrival order; mode "eager" (each request's kernels on
    a pool stream), "graphs" (each request as a HIP graph) or "batch" (the
    searches of admitted requests share steps).  Returns per-request records
    (keep=True: with each request's outputs and stack key, for checks); a
    `stats` dict receives the handle's statistics at the end; slab_bytes: the
    handle's trajectory slab size (0: the library's default); stage_fp32: a
    reduced-precision stack is decoded into an FP32 copy per request
    (TNO_REQ_STAGE_FP32) instead of searched in place; on_poll(handle) is
    called after every round of polls.

    Device memory: a key's first request hands its freshly drawn stack to
    the library by device pointer, and the stack stays allocated here until
    that request completes.  At most HANDOVERS such requests are in flight
    (a request that would hand over another stack waits; requests behind it
    on keys the library holds go ahead), and with budget_gb=0 the library's
    budget is the free memory less room for those stacks, one more draw and
    a margin for the HIP runtime.  reserve: the handle takes that budget at
    creation as one block (TNO_CFG_RESERVE), so that no submit waits on a
    device allocation."""
    import torch
    pool = StackPool({s.key: (s.side, s.frames) for s in specs}, dtype, device)
    if budget_gb == 0.0:
        free, _ = torch.cuda.mem_get_info(torch.device(device))
        draw = max(side * side * frames for side, frames in pool.shapes.values()) * 4
        budget_gb = max(free / 4, free - (HANDOVERS + 1) * draw - RUNTIME_MARGIN) / 1e9
    vel_all = torch.from_numpy(bank).to(device)
    known = set()
    staged = {}
    recs = []
    queue = collections.deque()
    pending = collections.deque(sorted(specs, key=lambda s: s.arrival))
    inflight = {}
    h = tno.Search(0, own_streams=True, max_inflight=max_inflight,
                   hbm_budget_bytes=int(budget_gb * 1e9), graphs=mode == "graphs", batch=mode == "batch",
                   slab_bytes=slab_bytes, reserve=reserve)
    t0 = time.perf_counter()
    retried = False
    try:
        while pending or queue or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            i = 0
            while i < len(queue):
                s = queue[i]
                R = scales = None
                if s.key not in known:
                    if sum(v[3] is not None for v in inflight.values()) >= HANDOVERS:
                        i += 1   # its stack waits for a hand-over to complete
                        continue
                sig, times = pool.inputs(s.key)
                vel = vel_all[torch.from_numpy(s.traj_idx).to(device)].contiguous()
                if s.key not in known:
                    if staged.get(s.key) is None:
                        staged[s.key] = pool.residuals(s.key)
                        # the draw is on torch's stream; the library's streams
                        # (non-blocking) keep running meanwhile
                        torch.cuda.current_stream().synchronize()
                    R, scales = staged[s.key]
                req = tno.make_request(R, sig if R is not None else None, times, vel, dtype=dtype,
                                       scales=scales, top_k=top_k, stack_key=s.key,
                                       shape=(s.frames, s.side, s.side),
                                       flags=tno.TNO_REQ_DEVICE_PTRS |
                                       (tno.TNO_REQ_STAGE_FP32 if stage_fp32 else 0))
                o, out = tno.alloc_outputs(vel.shape[0], s.side, s.side, top_k, device=device,
                                           maps=False)
                rc, ticket = tno.tno_search_submit(h.h, req, out)
                if rc == tno.TNO_E_BUSY:
                    break
                if rc == tno.TNO_E_INVAL and R is None:
                    known.discard(s.key)   # evicted by the library: hand the stack over again
                    continue
                if rc == tno.TNO_E_NOMEM and not retried:
                    # nothing in flight: device memory is held by torch's cache
                    # (stacks already handed over); return it and try once more
                    retried = True
                    torch.cuda.empty_cache()
                    continue
                if rc != tno.TNO_OK:
                    raise tno.TnoError(rc, tno.tno_search_last_error())
                retried = False
                known.add(s.key)
                staged.pop(s.key, None)
                inflight[ticket] = (s, o, vel, R, scales)
                del queue[i]
            done = []
            for ticket in list(inflight):
                rc, res = tno.tno_search_poll(h.h, ticket, 0)
                if rc == tno.TNO_PENDING:
                    continue
                if rc != tno.TNO_OK:
                    raise tno.TnoError(rc, res.message.decode(errors="replace"))
                s = inflight[ticket][0]
                t_done = time.perf_counter() - t0
                rec = {"key": s.key, "side": s.side, "frames": s.frames,
                       "traj": int(len(s.traj_idx)), "arrival": s.arrival, "done": t_done,
                       "latency_ms": (t_done - s.arrival) * 1e3, "device_ms": res.device_ms,
                       "prep_ms": res.prep_ms, "table_ms": res.table_ms, "lambda_ms": res.lambda_ms,
                       "search_ms": res.search_ms, "reduce_ms": res.reduce_ms, "queue_ms": res.queue_ms,
                       "updates": int(res.updates),
                       "topk": tno.decode_candidates(inflight[ticket][1]["topk"], res.n_topk)}
                if keep:
                    o = inflight[ticket][1]
                    rec["spec"] = s
                    rec["traj_max"] = o["traj_max"].cpu().numpy()
                    rec["best_snr"] = o["best_snr"].cpu().numpy()
                    rec["best_traj"] = o["best_traj"].cpu().numpy()
                recs.append(rec)
                done.append(ticket)
                if log:
                    log("done key %d %dx%dx%d J=%d latency %.1f ms" %
                        (s.key, s.side, s.side, s.frames, len(s.traj_idx), recs[-1]["latency_ms"]))
            for t in done:
                del inflight[t]
            if on_poll is not None:
                on_poll(h)
            if not done:
                time.sleep(0.0005)
        if stats is not None:
            st = tno.tno_search_stats(h.h)
            stats.update({f: getattr(st, f) for f, _ in st._fields_ if f != "reserved"})
    finally:
        h.close()
        # give the device memory of the stacks and outputs back, so that a
        # handle created next sees it free (its default budget is a share of
        # the free memory)
        del pool, staged, inflight, queue
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return recs


def summarize(recs, warm: int = 0):
    r = sorted(recs, key=lambda x: x["arrival"])[warm:]
    lat = np.array([x["latency_ms"] for x in r])
    span = max(x["done"] for x in r) - min(x["arrival"] for x in r)
    return {"requests": len(r), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "updates_per_s": float(sum(x["updates"] for x in r) / span)}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--requests", type=int, default=150)
    ap.add_argument("--warm", type=int, default=20)
    ap.add_argument("--keys", type=int, default=12)
    ap.add_argument("--load", type=float, default=0.7, help="arrival rate / back-to-back capacity")
    ap.add_argument("--budget-gb", type=float, default=0.0)
    ap.add_argument("--max-side", type=int, default=1024,
                    help="largest cutout side (at most 1024 px: larger mixes are disabled)")
    ap.add_argument("--dtypes", default="f32,bf16")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--modes", default="eager,batch",
                    help="eager launches, requests run as HIP graphs, and/or batched steps")
    args = ap.parse_args(argv)
    if args.max_side > MAX_SIDE:
        # with cutouts to 2048 px this driver's own stack copies and the
        # library's budget together exhausted device memory: the HIP runtime
        # aborted its queues (out of resources) and the run hung
        ap.error("cutouts above %d px are disabled: device memory of the driver's stack copies "
                 "and the library's budget is not yet bounded together" % MAX_SIDE)

    def log(m):
        print("[serve] " + m, file=sys.stderr, flush=True)

    bank, _ = synth.grid_shells()
    sides = [s for s in range(256, args.max_side + 1, 256)]
    shapes = draw_stack_shapes(args.keys, args.seed, sides=sides)
    specs = draw_requests(args.requests + args.warm, shapes, bank.shape[0], args.seed)
    # capacity: updates/s of the plain FP32 search back to back on a sample of
    # the mix; arrivals offer `load` times that in the mix's mean work
    cal = [Spec(s.key, s.side, s.frames, s.traj_idx, 0.0) for s in specs[:16]]
    log("calibrating back-to-back capacity on %d requests" % len(cal))
    crec = run_stream(cal, bank, dtype="f32", budget_gb=args.budget_gb, max_inflight=1)
    cap = sum(x["updates"] for x in crec) / (sum(x["device_ms"] for x in crec) * 1e-3)
    mean_u = float(np.mean([len(s.traj_idx) * s.side * s.side * s.frames for s in specs]))
    rate = args.load * cap / mean_u
    log("capacity %.3g updates/s, mean %.3g updates per request -> arrival rate %.2f req/s"
        % (cap, mean_u, rate))
    out = {"load": args.load, "arrival_rate_per_s": rate, "capacity_updates_per_s": cap, "forms": {}}
    for dt in args.dtypes.split(","):
        for mode in args.modes.split(","):
            sp = poisson_arrivals([Spec(s.key, s.side, s.frames, s.traj_idx) for s in specs], rate,
                                  args.seed)
            name = dt if mode == "eager" else dt + "+" + mode
            log("serving %d requests, %s" % (len(sp), name))
            recs = run_stream(sp, bank, dtype=dt, budget_gb=args.budget_gb, log=None, mode=mode)
            out["forms"][name] = summarize(recs, args.warm)
            log("%s: %s" % (name, json.dumps(out["forms"][name])))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
