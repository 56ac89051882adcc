"""Write the oracle's top-k and per-trajectory maxima for the 2048x2048 px x
1000 frame, 100-trajectory problem (the full FFI-shaped workload) into
tests/golden/c2_ffi_2048x2048x1000_j100.json.

Calls only the seeded generator (paper_2209_09848_amd.synth, data only) and
the FP64 oracle (oracle/); nothing from the HIP path.  The stack is drawn on
the host with numpy (platform-independent), so a GPU test can draw the same
stack and compare its search with the stored values.  The oracle runs over
all start pixels in row bands (region=), keeping each band's highest scores
and each trajectory's highest scores, then merges them:

* Sec. 3.3 candidates: the global top-k, ordered by SNR descending then flat
  index j*H*W + y*W + x ascending, plus every further entry within the tie
  band of the k-th value (so the test can tell which swaps are ties);
* Sec. 3.2 maximum over start pixels per trajectory, with the entries inside
  its tie band.

Usage:  python tests/golden/make_golden_c2.py [--threads N] [--band ROWS]
Takes about 15-30 minutes on 8 cores and ~20 GB of host memory.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from paper_2209_09848_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "c2_ffi_2048x2048x1000_j100.json")
H = W = 2048
T = 1000
K = 100
TIE = 2e-5            # oracle values within TIE*max(1,|s|) may swap in FP32
KEEP = 192            # entries kept per band (>= K plus the tie band)
PER_J = 8             # entries kept per trajectory and band


def stack_digest(R: np.ndarray) -> str:
    """sha256 of the per-frame FP64 sums and sums of squares (cheap, exact for
    a given float32 stack)."""
    s1 = R.sum(axis=(1, 2), dtype=np.float64)
    s2 = np.einsum("kij,kij->k", R, R, dtype=np.float64)
    return hashlib.sha256(np.concatenate([s1, s2]).tobytes()).hexdigest()


def problem():
    """The FFI-shaped problem of the golden file (seeded, numpy)."""
    return synth.make_ffi_like(H, W, T)


def band_top(snr, flux, y_lo, n):
    """Highest n entries of one band's [J][rows][W] maps as
    (snr, flux, flat index over the whole [J][H][W] map)."""
    J, rows, _ = snr.shape
    s = snr.reshape(-1)
    part = np.argpartition(-s, n - 1)[:n] if s.size > n else np.arange(s.size)
    j, rem = np.divmod(part, rows * W)
    y, x = np.divmod(rem, W)
    flat = (j.astype(np.int64) * H + (y + y_lo)) * W + x
    return s[part], flux.reshape(-1)[part], flat


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--band", type=int, default=64)
    ap.add_argument("--rows", type=int, default=H, help="stop after this many rows (timing)")
    args = ap.parse_args()
    if args.threads:
        oracle.set_threads(args.threads)
    t0 = time.time()
    p = problem()
    print("stack drawn in %.1f s" % (time.time() - t0), flush=True)
    digest = stack_digest(p.R)
    J = p.vel.shape[0]
    top_s, top_f, top_i = [], [], []
    pj_s = [[] for _ in range(J)]
    pj_f = [[] for _ in range(J)]
    pj_i = [[] for _ in range(J)]
    t1 = time.time()
    for y_lo in range(0, args.rows, args.band):
        y_hi = min(H, y_lo + args.band)
        o = oracle.search(p.R, p.sigma, p.times, p.t_ref, p.vel, region=(y_lo, y_hi, 0, W))
        s, f, i = band_top(o["snr"], o["flux"], y_lo, KEEP)
        top_s.append(s)
        top_f.append(f)
        top_i.append(i)
        for j in range(J):
            sj, fj, ij = band_top(o["snr"][j:j + 1], o["flux"][j:j + 1], y_lo, PER_J)
            pj_s[j].append(sj)
            pj_f[j].append(fj)
            pj_i[j].append(ij + j * H * W)
        el = time.time() - t1
        print("rows %d..%d done, %.0f s (%.2e updates/s)"
              % (y_lo, y_hi, el, J * y_hi * W * T / el), flush=True)
    s = np.concatenate(top_s)
    f = np.concatenate(top_f)
    i = np.concatenate(top_i)
    order = np.lexsort((i, -s))
    sk = s[order[K - 1]]
    keep = order[s[order] >= sk - TIE * max(1.0, abs(sk))]
    assert keep.size < KEEP, "tie band wider than the kept entries"
    cands = [[float(s[o]), float(f[o]), int(i[o])] for o in keep]
    peaks = []
    for j in range(J):
        sj = np.concatenate(pj_s[j])
        fj = np.concatenate(pj_f[j])
        ij = np.concatenate(pj_i[j]) - j * H * W
        oj = np.lexsort((ij, -sj))
        m = sj[oj[0]]
        near = oj[sj[oj] >= m - TIE * max(1.0, abs(m))]
        assert near.size < PER_J * (args.rows // args.band), "tie band wider than kept"
        peaks.append({"snr": float(m), "flux": float(fj[oj[0]]), "pixel": int(ij[oj[0]]),
                      "near": [[float(sj[o]), int(ij[o])] for o in near]})
    rec = {
        "what": "FP64 oracle top-k and per-trajectory maxima of synth.make_ffi_like(2048, 2048, 1000)",
        "height": H, "width": W, "frames": T, "trajectories": J, "top_k": K,
        "tie": TIE, "stack_digest": digest, "rows_done": args.rows,
        "oracle_threads": oracle.threads(), "oracle_seconds": round(time.time() - t1, 1),
        "candidates": cands,      # [snr, flux, flat index j*H*W + y*W + x], ordered
        "traj_max": peaks,
    }
    out = OUT if args.rows == H else OUT + ".partial"
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=0)
    print("wrote", out, "in %.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
