#!/usr/bin/env python3
"""Benchmark of the matched-filter trajectory search on one MI355X.

One step = one complete search request through the C ABI (submit + poll):
inverse-variance weighting of the stack, the FP64 offset/PRF table and trail
kernels, the FP64 normaliser, the numerator gather-stencil with its SNR/flux
epilogue, and the reductions (bank maximum, per-trajectory maximum, exact
top-k).  Inputs are resident in HBM before timing starts.

Default workload: a synthetic TESS-FFI-shaped stack, 2048 x 2048 px x 1000
frames (FP32 residuals, log-normal per-pixel sigma, a 1-day downlink gap half
way), 100 trajectories (10 speeds 0.01-0.2 px/frame x 10 directions), 30
injected sources, top-100 candidates.

Prints one JSON line (see the "roofline" and "cpu_baseline" objects; "extras"
holds untimed side measurements: the same request with a tabulated PRF and
pointing jitter, and the background re-fit of raw frames of the same shape).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3        # MI355X FP32 vector: 256 CU x 4 SIMD x 64 lanes x 2 flop / 2 cycles x 2.4 GHz
PEAK_HBM_GBS = 8000.0
PAPER_UPDATES_PER_S = 100 * 1000 * 2048 * 2048 / 300.0   # 100 traj, 1000 frames, 5 min (A100)
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_search_ffi_2048x2048x1000_j100_pmc.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2209_09848_amd", "csrc", "tno_kernels.hip")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """SHA-256 (first 16 hex digits) of the kernel source with its // comments
    and all whitespace removed: comment edits keep the counters valid, any
    code change voids them."""
    import re
    with open(KERNEL_SOURCE) as f:
        src = f.read()
    code = re.sub(r"\s+", "", re.sub(r"//[^\n]*", "", src))
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def measured_traffic(updates_per_request):
    """HBM bytes of one request's k_search launches (one per trajectory slab)
    from the committed rocprofv3 PMC summary, if it was taken on the current
    kernel source; else None."""
    try:
        with open(PMC_SUMMARY) as f:
            s = json.load(f)
    except (OSError, ValueError):
        return None
    if s.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if s.get("updates_per_request") != updates_per_request:
        return None
    return s.get("hbm_bytes_per_request")


def measured_copy_GBs():
    """Bandwidth of a plain device copy (read + write bytes / time) recorded
    beside the traffic counters, or None."""
    try:
        with open(PMC_SUMMARY) as f:
            return json.load(f).get("copy_probe", {}).get("copy_GBs")
    except (OSError, ValueError):
        return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def percentile(v, q):
    v = sorted(v)
    if not v:
        return None
    i = min(len(v) - 1, max(0, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[i]


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--height", type=int, default=2048)
    ap.add_argument("--width", type=int, default=2048)
    ap.add_argument("--frames", type=int, default=1000)
    ap.add_argument("--speeds", type=int, default=10)
    ap.add_argument("--dirs", type=int, default=10)
    ap.add_argument("--top-k", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-region", type=int, default=256,
                    help="side of the start-pixel square the oracle times")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched form, untuned (default tile shape), and print its result")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving form and print its result")
    ap.add_argument("--serving-side", type=int, default=1024,
                    help="largest cutout side of the serving form (multiples of 256 from 256)")
    ap.add_argument("--serving-requests", type=int, default=300,
                    help="measured requests per serving form (after a tenth as many warm-up ones)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the untimed side measurements (tabulated PRF, background re-fit)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the search is measured on a single "
              "MI355X (requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    # the serving form runs first, in a process of its own (the same command
    # as --serving-only), started before this process touches the GPU: its
    # host loop, which launches the batched steps, shares the host with
    # nothing else of this run, and it has the device to itself
    serving = None
    if not (args.no_extras or args.batched_only or args.copy_probe or args.serving_only):
        serving = serving_subprocess()

    import numpy as np
    import torch

    from paper_2209_09848_amd import synth, tno

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.batched_only:
        print(json.dumps(batched_form(dev, autotune=False)))
        return
    if args.serving_only:
        print(json.dumps(serving_form(n_requests=args.serving_requests, warm=max(1, args.serving_requests // 10),
                                      max_side=args.serving_side)))
        return

    if args.copy_probe:
        # a plain device copy of known size: scales the traffic counters and
        # measures the copy bandwidth the chip reaches (read + write bytes / time)
        n = args.copy_probe * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        ev0.record()
        for _ in range(reps):
            b.copy_(a)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                          "launches": 3 + reps, "copy_ms": ms, "copy_GBs": 2 * n * 4 / (ms * 1e-3) / 1e9}))
        return

    H, W, T = args.height, args.width, args.frames
    log("drawing synthetic %dx%dx%d stack on the GPU" % (H, W, T))
    R, sigma, times, t_ref, vel, src = synth.make_ffi_like_torch(
        H, W, T, dev, J_speeds=args.speeds, J_dirs=args.dirs)
    J = vel.shape[0]
    sig_t = torch.from_numpy(sigma).to(dev)
    times_t = torch.from_numpy(times).to(dev)
    vel_t = torch.from_numpy(vel).to(dev)
    k = args.top_k
    o, out = tno.alloc_outputs(J, H, W, k, device=dev)
    req = tno.make_request(R, sig_t, times_t, vel_t, t_ref=t_ref, top_k=k)
    torch.cuda.synchronize()
    U = J * H * W * T
    workload = "ffi_%dx%dx%d_j%d_f32" % (H, W, T, J)

    results = []
    with tno.Search(0) as h:
        for i in range(args.warmup):
            res = h.wait(h.submit(req, out))
            log("warmup %d: device %.1f ms (search %.1f ms)" % (i, res.device_ms, res.search_ms))
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for i in range(args.steps):
            s0 = time.perf_counter()
            res = h.wait(h.submit(req, out))
            lat.append((time.perf_counter() - s0) * 1e3)
            results.append({f: getattr(res, f) for f in
                            ("device_ms", "prep_ms", "table_ms", "lambda_ms", "search_ms", "reduce_ms")})
            log("step %d: %.1f ms wall, device %.1f ms, search %.1f ms" %
                (i, lat[-1], res.device_ms, res.search_ms))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0

    value = U * args.steps / elapsed
    mean = {f: float(np.mean([r[f] for r in results])) for f in results[0]}
    search_s = mean["search_ms"] * 1e-3
    flop_per_update = 4 * 5                    # separable stamp: 2 x 5 FMAs per update
    achieved = flop_per_update * U / search_s / 1e12
    traffic = measured_traffic(U)
    copy_GBs = measured_copy_GBs()

    cpu = None
    cpu_err = None
    if not args.no_cpu:
        from oracle import oracle
        n = args.cpu_region
        y0, x0 = H // 2 - n // 2, W // 2 - n // 2
        M = int(math.ceil(np.abs(vel).max() * np.abs(times - t_ref).max())) + 5
        cy0, cy1, cx0, cx1 = max(0, y0 - M), min(H, y0 + n + M), max(0, x0 - M), min(W, x0 + n + M)
        log("oracle baseline: %dx%d start pixels, crop %dx%d x %d frames"
            % (n, n, cy1 - cy0, cx1 - cx0, T))
        Rc = R[:, cy0:cy1, cx0:cx1].contiguous().cpu().numpy()
        sc = np.ascontiguousarray(sigma[cy0:cy1, cx0:cx1])
        oracle.build()
        c0 = time.perf_counter()
        ora = oracle.search(Rc, sc, times, t_ref, vel,
                            region=(y0 - cy0, y0 - cy0 + n, x0 - cx0, x0 - cx0 + n))
        cdt = time.perf_counter() - c0
        cu = J * T * n * n
        cpu = {"value": cu / cdt, "unit": "updates/s", "cores": oracle.threads(), "kind": "oracle",
               "sample": "all %d trajectories x %d frames x %dx%d start pixels at the image centre "
                         "(%.3g updates, %.1f s, FP64)" % (J, T, n, n, cu, cdt),
               "cpu_model": cpu_model()}
        # the same oracle on one core, over a smaller square of the same sample
        n1 = max(8, n // 4)
        all_threads = oracle.threads()
        oracle.set_threads(1)
        try:
            c0 = time.perf_counter()
            oracle.search(Rc, sc, times, t_ref, vel,
                          region=(y0 - cy0, y0 - cy0 + n1, x0 - cx0, x0 - cx0 + n1))
            cdt1 = time.perf_counter() - c0
        finally:
            oracle.set_threads(all_threads)
        cu1 = J * T * n1 * n1
        cpu["value_1core"] = cu1 / cdt1
        cpu["sample_1core"] = ("all %d trajectories x %d frames x %dx%d start pixels at the image "
                               "centre (%.3g updates, %.1f s, FP64, 1 thread)" % (J, T, n1, n1, cu1, cdt1))
        log("oracle on 1 core: %.1f s -> %.3g updates/s" % (cdt1, cu1 / cdt1))
        g = o["snr"][:, y0:y0 + n, x0:x0 + n].cpu().numpy().astype(np.float64)
        cpu_err = float(np.max(np.abs(g - ora["snr"]) / np.maximum(1.0, np.abs(ora["snr"]))))
        log("oracle %.1f s -> %.3g updates/s; GPU vs oracle max SNR rel err %.2e" %
            (cdt, cu / cdt, cpu_err))

    extras = None
    if not args.no_extras:
        extras = side_measurements(h_args=(H, W, T), R=R, sig_t=sig_t, times_t=times_t, vel_t=vel_t,
                                   t_ref=t_ref, k=k, out=out, dev=dev, U=U)
        extras["serving"] = serving

    line = {
        "metric": "traj*pixel*frame updates/s",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": value / PAPER_UPDATES_PER_S,
        "dtype": "f32",
        "data": "synthetic (seeded TESS-FFI-shaped stack, random sigma map, injected sources)",
        "config": {"workload": workload, "height": H, "width": W, "frames": T, "trajectories": J,
                   "stamp": 5, "prf": "gaussian sigma 0.7 px", "top_k": k,
                   "sources": len(src)},
        "roofline": {
            "bound": "alu",
            "kernel": "k_search",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": traffic,
            "flop_per_update": flop_per_update,
            "kernel_ms": mean["search_ms"],
            "hbm_equiv_GBs": U * 4 / search_s / 1e9,
            "hbm_equiv_frac": U * 4 / search_s / 1e9 / PEAK_HBM_GBS,
            # rocprof traffic over the kernel time, against the HBM peak and a
            # measured plain copy
            "traffic_GBs": traffic / search_s / 1e9 if traffic else None,
            "traffic_frac_hbm": traffic / search_s / 1e9 / PEAK_HBM_GBS if traffic else None,
            "copy_GBs": copy_GBs,
            "traffic_frac_copy": traffic / search_s / 1e9 / copy_GBs if traffic and copy_GBs else None,
        },
        "cpu_baseline": cpu,
        "cpu_parity_max_rel_err": cpu_err,
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
        "phases_ms": mean,
        "paper_context": {"updates_per_s": PAPER_UPDATES_PER_S, "hardware": "1x NVIDIA A100",
                          "note": "100 trajectories on 1000 2048x2048 frames in ~5 min"},
        "extras": extras,
    }
    print(json.dumps(line), flush=True)


def side_measurements(h_args, R, sig_t, times_t, vel_t, t_ref, k, out, dev, U):
    """Untimed by the contract above: the same request with the tabulated PRF
    and pointing jitter, and the background re-fit of raw frames of the same
    shape.  Each is one warm-up plus two measured runs (HIP-event times)."""
    import numpy as np
    import torch

    from paper_2209_09848_amd import synth, tno
    H, W, T = h_args
    res = {}
    table = torch.from_numpy(synth.TabulatedPSF().table(5, 9)).to(dev)
    jit = torch.from_numpy(synth.jitter_series(synth.rng(1, 9), T, amp=0.15)).to(dev)
    req = tno.make_request(R, sig_t, times_t, vel_t, t_ref=t_ref, top_k=k,
                           prf_kind=tno.TNO_PRF_TABLE, prf_table=table, prf_q=9, jitter=jit)
    with tno.Search(0) as h:
        runs = [h.wait(h.submit(req, out)) for _ in range(3)][1:]
    sm = float(np.mean([r.search_ms for r in runs]))
    dm = float(np.mean([r.device_ms for r in runs]))
    res["tabulated_prf_jitter"] = {
        "prf": "tabulated 5x5, q = 9, non-separable", "jitter_px": 0.15,
        "search_ms": sm, "device_ms": dm, "updates_per_s": U / (dm * 1e-3),
        "fma_per_update": 25, "achieved_TFLOPs": 50 * U / (sm * 1e-3) / 1e12,
        "frac": 50 * U / (sm * 1e-3) / 1e12 / PEAK_FP32_TFLOPS}
    log("tabulated PRF + jitter: search %.1f ms, device %.1f ms" % (sm, dm))
    log("drawing raw %dx%dx%d frames for the background re-fit" % (H, W, T))
    p = synth.make_refit_problem(H, W, T, device=dev, n_sl=64, config_id=90)
    S = torch.from_numpy(p["S"]).to(dev)
    jt = torch.from_numpy(p["jitter"]).to(dev)
    iters, rounds = 5, 3
    kw = dict(scattered=S, delta=1.345, iterations=iters, bright_threshold=5000.0, clip_sigma=5.0,
              sigma_rounds=rounds)
    ms = []
    for _ in range(3):
        o, ro = tno.refit_tensors(p["D"], jt, **kw)
        ms.append(ro.device_ms)
        del o
    m = float(np.mean(ms[1:]))
    passes = 1 + iters + (rounds + 1) + 1
    nbytes = (passes + 1) * T * H * W * 4          # each pass reads D; the last also writes R
    res["background_refit"] = {
        "workload": "raw_%dx%dx%d_f32, scattered light 64x64, %d rounds, %d sigma rounds" % (H, W, T, iters, rounds),
        "ms": m, "frame_passes": passes, "algorithmic_bytes": nbytes,
        "GBs": nbytes / (m * 1e-3) / 1e9, "frac_hbm": nbytes / (m * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "sigma0": ro.sigma0, "n_clipped": int(ro.n_clipped), "n_masked": int(ro.n_masked)}
    log("background re-fit: %.1f ms (%.2f TB/s)" % (m, nbytes / (m * 1e-3) / 1e12))
    del p
    res["precision_forms"] = precision_forms(R, sig_t, times_t, vel_t, t_ref, k, out, dev, U)
    res["batched_shells"] = batched_form(dev)
    return res


def footprint_bytes(H, W, T, times, vel, dtype, stage=False, k=100, stamp=5):
    """tno_search_footprint of a request over a stack resident under a key
    (its codes, tile scales and sigma counted once) with the top-k and no
    caller maps: the device bytes the request holds while in flight."""
    import ctypes

    import numpy as np

    from paper_2209_09848_amd import tno
    times = np.ascontiguousarray(times, np.float64)
    vel = np.ascontiguousarray(vel, np.float64)
    req = tno.tno_request()
    req.height, req.width, req.n_frames, req.dtype = H, W, T, tno.DTYPE_CODE[dtype]
    req.times = times.ctypes.data_as(ctypes.c_void_p)
    req.velocities = vel.ctypes.data_as(ctypes.c_void_p)
    req.t_ref = float("nan")
    req.prf = tno.tno_prf(0, stamp, 0.7, None, 0, 0)
    req.n_traj = vel.shape[0]
    req.top_k = k
    req.stack_key = 1
    req.flags = tno.TNO_REQ_STAGE_FP32 if stage else 0
    req.reserved = 0
    topk = np.zeros((k, 5), np.int32)
    out = tno.tno_outputs()
    out.topk = topk.ctypes.data_as(ctypes.c_void_p)
    return int(tno.tno_search_footprint(req, out))


def precision_forms(R, sig_t, times_t, vel_t, t_ref, k, out, dev, U):
    """The FFI request with its stack stored as BF16, FP16 and FP8-e4m3
    (per-64x64-tile scales): searched in place (default) and, for BF16, from
    a staged FP32 copy; one warm-up and two measured requests each."""
    import numpy as np
    import torch

    from paper_2209_09848_amd import tno
    T, H, W = (int(v) for v in R.shape)
    times = times_t.cpu().numpy()
    vel = vel_t.cpu().numpy()
    res = {"f32": {"footprint_bytes": footprint_bytes(H, W, T, times, vel, "f32")}}
    for dtype, stage in (("bf16", False), ("bf16", True), ("f16", False), ("fp8_e4m3", False)):
        codes = torch.empty((T, H, W), device=dev, dtype=torch.uint8 if dtype == "fp8_e4m3" else torch.int16)
        scales = torch.empty((T, (H + 63) // 64, (W + 63) // 64), device=dev)
        assert tno.tno_quantize(T, H, W, tno.DTYPE_CODE[dtype], R.data_ptr(), codes.data_ptr(),
                                scales.data_ptr(), None) == 0
        torch.cuda.synchronize()
        flags = tno.TNO_REQ_DEVICE_PTRS | (tno.TNO_REQ_STAGE_FP32 if stage else 0)
        req = tno.make_request(codes, sig_t, times_t, vel_t, t_ref=t_ref, top_k=k, dtype=dtype,
                               scales=scales, flags=flags)
        with tno.Search(0) as h:
            runs = [h.wait(h.submit(req, out)) for _ in range(3)][1:]
        name = dtype + ("_staged_fp32" if stage else "_in_place")
        sm = float(np.mean([r.search_ms for r in runs]))
        dm = float(np.mean([r.device_ms for r in runs]))
        res[name] = {"search_ms": sm, "device_ms": dm, "updates_per_s": U / (dm * 1e-3),
                     "stack_bytes": T * H * W * codes.element_size() + scales.numel() * 4,
                     "footprint_bytes": footprint_bytes(H, W, T, times, vel, dtype, stage=stage)}
        log("precision form %s: search %.1f ms, device %.1f ms, footprint %.2f GB"
            % (name, sm, dm, res[name]["footprint_bytes"] / 1e9))
        del codes, scales
        torch.cuda.empty_cache()
    return res


def serving_subprocess(timeout_s=600):
    """serving_form() in a child process (bench.py --serving-only), started
    before the calling process initialises the GPU; its JSON result, or the
    error it ended with."""
    import subprocess
    try:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--serving-only"], stdout=subprocess.PIPE,
                           stderr=None, text=True, timeout=timeout_s)
    except subprocess.TimeoutExpired:
        return {"error": "serving form did not finish in %d s" % timeout_s}
    except OSError as e:
        return {"error": "serving form did not start: %s" % e}
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    if r.returncode != 0 or not lines:
        return {"error": "serving form exited with status %d" % r.returncode}
    return json.loads(lines[-1])


def serving_form(n_requests=300, warm=30, load=0.7, max_side=1024, n_keys=32, seed=0):
    """A Poisson stream of uneven requests (cutouts 256..max_side px, 200-1000
    frames, 16-256 trajectories of the shell bank; stacks resident under
    `n_keys` keys, about half the requests reusing the previous one) at `load`
    times the back-to-back capacity of the plain FP32 search on a sample of
    the mix; FP32, BF16 read in place and BF16 staged into FP32 per request,
    each with eager per-request launches and with continuous batching, at the
    same arrival rate."""
    import gc

    import numpy as np
    import torch

    from paper_2209_09848_amd import serve, synth
    if max_side > serve.MAX_SIDE:
        # with cutouts to 2048 px the serving driver's own stack copies and the
        # library's budget together exhausted device memory: the HIP runtime
        # aborted its queues (out of resources) and the run hung
        raise ValueError("serving cutouts above %d px are disabled: device memory of the driver's "
                         "stack copies and the library's budget is not yet bounded together" % serve.MAX_SIDE)
    gc.collect()
    torch.cuda.empty_cache()   # each form's handle takes its budget from the free memory
    bank, _ = synth.grid_shells()
    sides = list(range(256, max_side + 1, 256))
    shapes = serve.draw_stack_shapes(n_keys, seed, sides=sides)
    specs = serve.draw_requests(n_requests + warm, shapes, bank.shape[0], seed)
    # capacity: updates/s of the plain FP32 search back to back on a sample of
    # the mix; the arrival rate offers `load` times that in the mix's mean
    # updates per request
    cal = [serve.Spec(s.key, s.side, s.frames, s.traj_idx, 0.0) for s in specs[:16]]
    crec = serve.run_stream(cal, bank, dtype="f32", max_inflight=1)
    cap = sum(x["updates"] for x in crec) / (sum(x["device_ms"] for x in crec) * 1e-3)
    mean_u = float(np.mean([len(s.traj_idx) * s.side * s.side * s.frames for s in specs]))
    rate = load * cap / mean_u
    out = {"workload": "%d requests (+%d warm-up), cutouts 256-%d px, 200-1000 frames, 16-256 trajectories, "
                       "%d stack keys" % (n_requests, warm, max_side, n_keys),
           "load": load, "arrival_rate_per_s": rate, "capacity_updates_per_s": cap,
           "mean_updates_per_request": mean_u, "forms": {}}
    for dtype, stage in (("f32", False), ("bf16", False), ("bf16", True)):
        for mode in ("eager", "batch"):
            sp = serve.poisson_arrivals([serve.Spec(s.key, s.side, s.frames, s.traj_idx) for s in specs],
                                        rate, seed)
            recs = serve.run_stream(sp, bank, dtype=dtype, mode=mode, stage_fp32=stage)
            name = dtype + ("_staged" if stage else "") + "_" + mode
            out["forms"][name] = serve.summarize(recs, warm)
            log("serving %s: p50 %.1f ms, p99 %.1f ms, %.3g updates/s"
                % (name, out["forms"][name]["p50_ms"], out["forms"][name]["p99_ms"],
                   out["forms"][name]["updates_per_s"]))
    return out


def batched_form(dev, autotune=True):
    """1024x1024x1000 BF16 stack, 2048 trajectories in 8 uneven shells, one
    launch per request; the first request of the shape class runs the
    autotuner (timed apart; with autotune=False the default shape), two more
    are measured."""
    import tempfile

    import numpy as np
    import torch

    from paper_2209_09848_amd import synth, tno
    H = W = 1024
    T = 1000
    bank, _ = synth.grid_shells()
    log("drawing the batched-form stack (1024x1024x1000, 2048 trajectories)")
    R, sigma, times, t_ref, vel, _ = synth.make_ffi_like_torch(H, W, T, dev, bank=bank, config_id=4,
                                                               n_sources=20, amp=(0.1, 0.5))
    nq = (H + 63) // 64
    codes = torch.empty((T, H, W), dtype=torch.int16, device=dev)
    scales = torch.empty((T, nq, nq), dtype=torch.float32, device=dev)
    tno.tno_quantize(T, H, W, tno.TNO_BF16, R.data_ptr(), codes.data_ptr(), scales.data_ptr(),
                     torch.cuda.current_stream().cuda_stream)
    del R
    J = bank.shape[0]
    o, out = tno.alloc_outputs(J, H, W, 100, device=dev, maps=False)
    req = tno.make_request(codes, torch.from_numpy(sigma).to(dev), torch.from_numpy(times).to(dev),
                           torch.from_numpy(vel).to(dev), t_ref=t_ref, top_k=100, dtype="bf16",
                           scales=scales)
    U = J * H * W * T
    res = {"workload": "batched_1024x1024x1000_bf16_j2048_8shells"}
    for stage in (True, False):
        r = req
        if stage:
            r = tno.make_request(codes, torch.from_numpy(sigma).to(dev), torch.from_numpy(times).to(dev),
                                 torch.from_numpy(vel).to(dev), t_ref=t_ref, top_k=100, dtype="bf16",
                                 scales=scales, flags=tno.TNO_REQ_DEVICE_PTRS | tno.TNO_REQ_STAGE_FP32)
        with tempfile.TemporaryDirectory() as d:
            path = d + "/tune.txt"
            with tno.Search(0, autotune=autotune, tune_cache_path=path) as h:
                first = h.wait(h.submit(r, out))
                runs = [h.wait(h.submit(r, out)) for _ in range(2)]
            tuned = ([l for l in open(path).read().splitlines() if not l.startswith("#")]
                     if os.path.exists(path) else [])
        dm = float(np.mean([x.device_ms for x in runs]))
        sm = float(np.mean([x.search_ms for x in runs]))
        name = "staged_fp32" if stage else "in_place"
        log("batched form (%s): %.1f ms per request (search %.1f ms), tuning request %.1f ms, tuned %s"
            % (name, dm, sm, first.device_ms, tuned))
        lm = float(np.mean([x.lambda_ms for x in runs]))
        res[name] = {"device_ms": dm, "search_ms": sm, "lambda_ms": lm, "updates_per_s": U / (dm * 1e-3),
                     "search_TFLOPs": 20 * U / (sm * 1e-3) / 1e12,
                     "first_request_ms_with_autotune" if autotune else "first_request_ms": first.device_ms,
                     "tuned": tuned[0].split()[2:4] if tuned else None,
                     "footprint_bytes": footprint_bytes(H, W, T, times, vel, "bf16", stage=stage)}
    return res


if __name__ == "__main__":
    main()
