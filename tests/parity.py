"""Comparison helpers of the GPU parity tests (HIP path vs the FP64 oracle).

Tolerances (derived from the arithmetic; the search's outputs are FP32):
* SNR:  |gpu - oracle| <= 1e-5 * max(1, |oracle|)  (SNR ~ N(0,1) under noise,
  so a pure relative bound is ill-posed near 0);
* flux: |gpu - oracle| <= 1e-5 * max(|oracle|, 1/sqrt(Lam))  (flux noise is
  1/sqrt(Lam));
* "ties": two oracle values within TIE = 2e-5 * max(1, |s|) may be ordered
  either way by the FP32 search; there every choice inside the band is valid.
"""
import numpy as np

SNR_TOL = 1e-5
TIE = 2e-5


def check_maps(snr, flux, ora, tol=SNR_TOL):
    so, fo, lam = ora["snr"], ora["flux"], ora["lam"]
    es = np.abs(snr.astype(np.float64) - so) / np.maximum(1.0, np.abs(so))
    assert es.max() <= tol, "SNR rel error %.3g at %s" % (es.max(), np.unravel_index(es.argmax(), es.shape))
    scale = np.where(lam > 0, np.maximum(np.abs(fo), 1.0 / np.sqrt(np.where(lam > 0, lam, 1.0))), 1.0)
    ef = np.abs(flux.astype(np.float64) - fo) / scale
    assert ef.max() <= tol, "flux rel error %.3g at %s" % (ef.max(), np.unravel_index(ef.argmax(), ef.shape))
    # where the normaliser is zero both maps are exactly zero
    assert np.all(snr[lam == 0] == 0) and np.all(flux[lam == 0] == 0)
    return float(es.max()), float(ef.max())


def band(s):
    return TIE * max(1.0, abs(s))


def check_best(best_snr, best_traj, ora_snr):
    """best_snr within tolerance; best_traj exact unless the top two of the
    bank are within the tie band, then any j inside the band."""
    J = ora_snr.shape[0]
    obest = ora_snr.max(axis=0)
    es = np.abs(best_snr - obest) / np.maximum(1.0, np.abs(obest))
    assert es.max() <= SNR_TOL
    chosen = np.take_along_axis(ora_snr, best_traj[None].astype(np.int64), axis=0)[0]
    assert np.all(best_traj >= 0) and np.all(best_traj < J)
    lim = TIE * np.maximum(1.0, np.abs(obest))
    assert np.all(obest - chosen <= lim)
    exact = np.argmax(ora_snr, axis=0)
    srt = np.sort(ora_snr, axis=0)
    clear = (srt[-1] - srt[-2] > lim) if J > 1 else np.ones_like(obest, bool)
    assert np.array_equal(best_traj[clear], exact[clear])


def check_traj_max(peaks, ora_snr, ora_flux):
    s, f, y, x = peaks
    J, H, W = ora_snr.shape
    for j in range(J):
        flat = ora_snr[j].reshape(-1)
        m = flat.max()
        got = ora_snr[j, y[j], x[j]]
        assert m - got <= band(m), (j, m, got)
        assert abs(s[j] - got) <= 1e-5 * max(1.0, abs(got))
        near = np.flatnonzero(flat >= m - band(m))
        if near.size == 1:
            assert y[j] * W + x[j] == near[0]


def check_topk(cands, ora_snr, k):
    """cands: list of (snr, flux, j, y, x) from the GPU; exact set and order
    apart from oracle near-ties."""
    J, H, W = ora_snr.shape
    N = J * H * W
    k = min(k, N)
    assert len(cands) == k
    flat = ora_snr.reshape(-1)
    idx = np.array([c[2] * H * W + c[3] * W + c[4] for c in cands], np.int64)
    assert len(set(idx.tolist())) == k, "duplicate candidates"
    vals = flat[idx]
    # each reported SNR matches the oracle value at that index
    for c, v in zip(cands, vals):
        assert abs(c[0] - v) <= 1e-5 * max(1.0, abs(v))
    # the reported order is (SNR desc, index asc) on the reported values
    for a, b in zip(cands[:-1], cands[1:]):
        ia, ib = a[2] * H * W + a[3] * W + a[4], b[2] * H * W + b[3] * W + b[4]
        assert a[0] > b[0] or (a[0] == b[0] and ia < ib)
    order = np.lexsort((np.arange(N), -flat))
    sk = flat[order[k - 1]]
    # every oracle candidate clearly above the k-th value is present
    must = order[:k][flat[order[:k]] > sk + band(sk)]
    assert set(must.tolist()) <= set(idx.tolist())
    # nothing reported is clearly below the k-th value
    assert np.all(vals >= sk - band(sk))
