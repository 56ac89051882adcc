"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exact
rational arithmetic, scipy library routines, closed forms, statistical
invariants, or the independent dense-filter brute force (tests/brute.py).
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import ndimage, stats

from paper_2209_09848_amd import synth
from tests import brute


# ------------------------------------------------------------------ offsets

def _exact_anchor_phase(v, dt):
    """floor(v*dt + 1/2) and the phase from exact rationals of the FP64
    product v*dt (the product itself is one IEEE rounding)."""
    d = Fraction(float(v) * float(dt))
    a = math.floor(d + Fraction(1, 2))
    return a, float(d - a)


@pytest.mark.parametrize("v,dt,anchor,phase", [
    (0.25, 2.0, 1, -0.5),      # exactly half way: rounds up, phase -1/2
    (-0.25, 2.0, 0, -0.5),
    (-1.5, 1.0, -1, -0.5),
    (0.75, 3.0, 2, 0.25),
    (0.125, 4.0, 1, -0.5),
    (1.0, 0.0, 0, 0.0),
    (-0.375, 4.0, -1, -0.5),
    (2.5, -3.0, -7, -0.5),
])
def test_offset_dyadic_closed_form(oracle_mod, v, dt, anchor, phase):
    a, f = oracle_mod.offset(v, dt)
    assert a == anchor and f == phase


def test_offset_matches_exact_rationals(oracle_mod):
    g = np.random.default_rng(7)
    times = synth.times_with_gap(200, 100)
    vel = g.uniform(-15, 15, size=(50, 2))
    iy, ix, fy, fx = oracle_mod.offsets(times, times[0], vel)
    for j in range(50):
        for k in range(0, 200, 7):
            dt = times[k] - times[0]
            a, f = _exact_anchor_phase(vel[j, 0], dt)
            assert ix[j, k] == a and abs(fx[j, k] - f) < 1e-15
            a, f = _exact_anchor_phase(vel[j, 1], dt)
            assert iy[j, k] == a and abs(fy[j, k] - f) < 1e-15
    assert np.all(fx >= -0.5) and np.all(fx < 0.5)


def test_fp32_time_arithmetic_would_be_visible(oracle_mod):
    """At a TESS-like epoch (t ~ 2000 d) a float32 time baseline moves the
    sub-pixel phase by far more than the FP64 one: the table must be FP64."""
    times = synth.times_uniform(1000)
    v = 0.3 * synth.FRAMES_PER_DAY
    _, _, _, fx = oracle_mod.offsets(times, times[0], np.array([[v, 0.0]]))
    t32 = times.astype(np.float32)
    d32 = np.float32(v) * (t32 - t32[0])
    f32 = d32 - np.floor(d32 + np.float32(0.5))
    assert np.max(np.abs(f32 - fx[0])) > 1e-4


# ------------------------------------------------------------------ profiles

@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("stamp", [1, 3, 5, 7, 15])
def test_profile_unit_sum_and_mirror(oracle_mod, kind, stamp):
    for f in (-0.5, -0.31, 0.0, 0.2, 0.4999):
        g = oracle_mod.profile(kind, 0.7, stamp, f)
        assert abs(g.sum() - 1.0) < 1e-15
        gm = oracle_mod.profile(kind, 0.7, stamp, -f)
        np.testing.assert_allclose(g, gm[::-1], rtol=1e-14, atol=1e-300)


def test_profile_sampled_is_normal_pdf(oracle_mod):
    """Sampled Gaussian = normal pdf at the tap offsets, renormalised."""
    for f in (-0.5, -0.12, 0.0, 0.33):
        taps = np.arange(-2, 3)
        ref = stats.norm.pdf(taps, loc=f, scale=0.7)
        np.testing.assert_allclose(oracle_mod.profile(0, 0.7, 5, f), ref / ref.sum(), rtol=1e-13)


def test_profile_integrated_is_normal_cdf_difference(oracle_mod):
    for f in (-0.5, -0.12, 0.0, 0.33):
        taps = np.arange(-7, 8)
        ref = stats.norm.cdf(taps + 0.5, loc=f, scale=0.7) - stats.norm.cdf(taps - 0.5, loc=f, scale=0.7)
        got = oracle_mod.profile(1, 0.7, 15, f)
        np.testing.assert_allclose(got[4:11], (ref / ref.sum())[4:11], rtol=1e-12)
        assert np.all(got > 0)


def test_peak_pixel_fraction_reading(oracle_mod):
    """sigma_px = 0.7 puts ~32% (sampled) / ~28% (integrated) of the stamp's
    flux in the centred peak pixel (broader than the TESS PRF of Sec. 2)."""
    g0 = oracle_mod.profile(0, 0.7, 5, 0.0)
    g1 = oracle_mod.profile(1, 0.7, 5, 0.0)
    assert 0.31 < g0[2] ** 2 < 0.34
    assert 0.27 < g1[2] ** 2 < 0.30


# ------------------------------------------------------------------ v = 0 special case

def _weights_f0(sigma_px, stamp):
    taps = np.arange(stamp) - stamp // 2
    g = np.exp(-0.5 * (taps / sigma_px) ** 2)
    g /= g.sum()
    return np.outer(g, g)


def test_zero_velocity_is_prf_correlated_frame_sum(oracle_mod):
    """v = 0: nu = W0 (x) sum_k R_k ivar and Lam = W0^2 (x) (T ivar), with (x)
    the zero-padded correlation of scipy.ndimage."""
    g = np.random.default_rng(3)
    T, H, W = 7, 23, 29
    R = g.standard_normal((T, H, W)).astype(np.float32)
    sigma = (0.5 + g.random((H, W))).astype(np.float32)
    sigma[3, 4] = 0.0
    sigma[10, 11] = np.inf
    sigma[20, 2] = np.nan
    times = synth.times_with_gap(T, 3)
    out = oracle_mod.search(R, sigma, times, times[0], np.zeros((1, 2)))
    iv = brute.ivar_map(sigma)
    W0 = _weights_f0(0.7, 5)
    nu_ref = ndimage.correlate((R.astype(np.float64) * iv[None]).sum(0), W0, mode="constant", cval=0.0)
    lam_ref = ndimage.correlate(T * iv, W0 ** 2, mode="constant", cval=0.0)
    np.testing.assert_allclose(out["nu"][0], nu_ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out["lam"][0], lam_ref, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------ impulse response

def test_impulse_response_gives_the_filter(oracle_mod):
    T, H, W = 9, 30, 31
    times = synth.times_with_gap(T, 5, 0.7)
    vel = np.array([[3.1, -1.7], [-2.2, 0.9]])
    k0, Y, X = 6, 14, 17
    R = np.zeros((T, H, W), np.float32)
    R[k0, Y, X] = 1.0
    sigma = np.ones((H, W), np.float32)
    out = oracle_mod.search(R, sigma, times, times[0], vel)
    for j in range(2):
        ax, fx = brute.anchor_phase(vel[j][0], times[k0] - times[0])
        ay, fy = brute.anchor_phase(vel[j][1], times[k0] - times[0])
        gx = brute.profile(fx, 0.7, 5)
        gy = brute.profile(fy, 0.7, 5)
        ref = np.zeros((H, W))
        for a in range(-2, 3):
            for b in range(-2, 3):
                y0, x0 = Y - ay - a, X - ax - b
                if 0 <= y0 < H and 0 <= x0 < W:
                    ref[y0, x0] = gy[a + 2] * gx[b + 2]
        np.testing.assert_allclose(out["nu"][j], ref, rtol=1e-14, atol=1e-15)


# ------------------------------------------------------------------ brute force

@pytest.mark.parametrize("integrated", [False, True])
def test_matches_dense_filter_brute_force(oracle_mod, integrated):
    """Paper's own dense-filter form on a tiny case with edges, masked pixels
    and a downlink gap."""
    g = np.random.default_rng(11)
    T, H, W = 6, 12, 10
    R = g.standard_normal((T, H, W)).astype(np.float32)
    sigma = (0.6 + g.random((H, W))).astype(np.float32)
    sigma[2, 3] = 0.0
    sigma[7, 8] = -1.0
    times = synth.times_with_gap(T, 3, 1.5)
    vel = np.array([[20.0, -9.0], [-13.0, 31.0], [0.0, 0.0]])
    out = oracle_mod.search(R, sigma, times, times[0], vel, prf_kind=int(integrated),
                            sigma_px=0.8, stamp=5)
    nu, lam = brute.search(R, sigma, times, times[0], vel, sigma_px=0.8, stamp=5,
                           integrated=integrated)
    np.testing.assert_allclose(out["nu"], nu, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(out["lam"], lam, rtol=1e-12, atol=1e-13)


def test_region_and_hypotheses_agree_with_full(oracle_mod):
    g = np.random.default_rng(5)
    T, H, W = 8, 20, 24
    R = g.standard_normal((T, H, W)).astype(np.float32)
    sigma = (0.5 + g.random((H, W))).astype(np.float32)
    times = synth.times_uniform(T)
    vel = np.array([[9.0, 4.0], [-6.0, 2.0], [1.0, -12.0]])
    full = oracle_mod.search(R, sigma, times, times[0], vel)
    part = oracle_mod.search(R, sigma, times, times[0], vel, region=(3, 17, 5, 21))
    np.testing.assert_array_equal(part["nu"], full["nu"][:, 3:17, 5:21])
    hj = g.integers(0, 3, 50)
    hy = g.integers(0, H, 50)
    hx = g.integers(0, W, 50)
    hyp = oracle_mod.hypotheses(R, sigma, times, times[0], vel, hj, hy, hx)
    np.testing.assert_allclose(hyp["snr"], full["snr"][hj, hy, hx], rtol=1e-13, atol=1e-13)


# ------------------------------------------------------------------ invariants

def test_linearity_scale_translation(oracle_mod):
    g = np.random.default_rng(9)
    T, H, W = 6, 32, 32
    times = synth.times_uniform(T)
    vel = np.array([[8.0, -3.0], [0.0, 5.0]])
    R1 = g.standard_normal((T, H, W)).astype(np.float32)
    R2 = g.standard_normal((T, H, W)).astype(np.float32)
    sigma = (0.5 + g.random((H, W))).astype(np.float32)
    o1 = oracle_mod.search(R1, sigma, times, times[0], vel)
    o2 = oracle_mod.search(R2, sigma, times, times[0], vel)
    o12 = oracle_mod.search(R1 + R2, sigma, times, times[0], vel)
    # R1 + R2 is rounded to float32 once; compare within that rounding
    np.testing.assert_allclose(o12["snr"], o1["snr"] + o2["snr"], atol=1e-5)
    # SNR is invariant under R -> cR, sigma -> c sigma (c a power of two: exact)
    oc = oracle_mod.search(R1 * 4, sigma * 4, times, times[0], vel)
    np.testing.assert_allclose(oc["snr"], o1["snr"], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(oc["flux"], 4 * o1["flux"], rtol=1e-13, atol=1e-13)
    # shifting the data by an integer offset shifts the interior maps
    Rs = np.roll(R1, (3, -2), axis=(1, 2))
    ss = np.roll(sigma, (3, -2), axis=(0, 1))
    os_ = oracle_mod.search(Rs, ss, times, times[0], vel)
    np.testing.assert_allclose(os_["snr"][:, 13:20, 10:17], o1["snr"][:, 10:17, 12:19],
                               rtol=1e-12, atol=1e-12)


def test_white_noise_snr_is_standard_normal(oracle_mod):
    """Pure Gaussian noise with any sigma map: every hypothesis' SNR is N(0,1)
    (Sec. 3.2 noise model; the normalisation is exact ML)."""
    T, H, W = 10, 48, 48
    times = synth.times_with_gap(T, 5)
    vel = np.array([[6.0, 2.0], [-3.0, -7.0], [10.0, 0.0]])
    sig = synth.sigma_lognormal(np.random.default_rng(1), H, W).astype(np.float32)
    sig[5, 5] = 0.0
    ys, xs = np.meshgrid(np.arange(8, 48, 16), np.arange(8, 48, 16), indexing="ij")
    hy, hx = ys.ravel().astype(np.int32), xs.ravel().astype(np.int32)
    vals = []
    for seed in range(240):
        g = np.random.default_rng(1000 + seed)
        R = (sig * g.standard_normal((T, H, W))).astype(np.float32)
        hj = ((np.arange(hy.size) + seed) % 3).astype(np.int32)
        vals.append(oracle_mod.hypotheses(R, sig, times, times[0], vel, hj, hy, hx)["snr"])
    v = np.concatenate(vals)
    n = v.size
    assert abs(v.mean()) < 4.0 / math.sqrt(n)
    assert abs(v.var() - 1.0) < 4.0 * math.sqrt(2.0 / n)
    assert stats.kstest(v, "norm").pvalue > 1e-3


# ------------------------------------------------------------------ injection closed forms

def _template_inner(times, t_ref, v, start_src, start_tmpl, sigma_px=0.7, stamp=5):
    """<w_src, w_tmpl> and |w_tmpl|^2 summed over frames (sigma = 1, interior)."""
    num = den = 0.0
    for t in times:
        dt = t - t_ref
        ws = {}
        for (px, py), store in (((start_src[0] + v[0] * dt, start_src[1] + v[1] * dt), "s"),
                                ((start_tmpl[0] + v[0] * dt, start_tmpl[1] + v[1] * dt), "t")):
            cx, cy = math.floor(px + 0.5), math.floor(py + 0.5)
            gx = brute.profile(px - cx, sigma_px, stamp)
            gy = brute.profile(py - cy, sigma_px, stamp)
            ws[store] = {(cy + a - 2, cx + b - 2): gy[a] * gx[b] for a in range(5) for b in range(5)}
        num += sum(w * ws["s"].get(p, 0.0) for p, w in ws["t"].items())
        den += sum(w * w for w in ws["t"].values())
    return num, den


def test_injected_source_on_grid_closed_form(oracle_mod):
    """Noise-free injection at an integer start on a bank trajectory: the
    argmax is the true (x0, y0, j) and the peak SNR is A*sqrt(Lam)."""
    p = synth.make_c1("noise_free")
    src = [synth.Source(20.0, 32.0, p.vel[4][0], p.vel[4][1], 0.5, 4)]
    R = synth.add_sources(np.zeros_like(p.R), p.times, p.t_ref, src).astype(np.float32)
    out = oracle_mod.search(R, p.sigma, p.times, p.t_ref, p.vel)
    j, y, x = np.unravel_index(np.argmax(out["snr"]), out["snr"].shape)
    assert (j, y, x) == (4, 32, 20)
    lam = out["lam"][4, 32, 20]
    # float32 storage of the injected values limits agreement to ~1e-7
    assert abs(out["snr"][4, 32, 20] - 0.5 * math.sqrt(lam)) < 1e-6 * 0.5 * math.sqrt(lam)
    assert abs(out["flux"][4, 32, 20] - 0.5) < 1e-6
    _, den = _template_inner(p.times, p.t_ref, p.vel[4], (20.0, 32.0), (20.0, 32.0))
    assert abs(lam - den) < 1e-12 * den


def test_injected_source_subpixel_closed_form(oracle_mod):
    """C1's sub-pixel start (20.3, 31.7): the peak sits at the rounded start
    on the true trajectory, at A <w_src, w_tmpl> / |w_tmpl| (~1.299)."""
    p = synth.make_c1("noise_free")
    out = oracle_mod.search(p.R, p.sigma, p.times, p.t_ref, p.vel)
    j, y, x = np.unravel_index(np.argmax(out["snr"]), out["snr"].shape)
    assert (j, y, x) == (4, 32, 20)
    num, den = _template_inner(p.times, p.t_ref, p.vel[4], (20.3, 31.7), (20.0, 32.0))
    ref = 0.5 * num / math.sqrt(den)
    assert abs(out["snr"][4, 32, 20] - ref) < 2e-6 * ref
    assert 1.29 < ref < 1.31
    assert abs(0.5 * math.sqrt(den) - 1.426) < 1e-3


def test_injected_source_with_noise_is_unit_normal_offset(oracle_mod):
    """With N(0,1) noise, SNR at the truth minus the noise-free value is N(0,1)."""
    p0 = synth.make_c1("noise_free")
    clean = oracle_mod.hypotheses(p0.R, p0.sigma, p0.times, p0.t_ref, p0.vel,
                                  [4], [32], [20])["snr"][0]
    d = []
    for s in range(120):
        p = synth.make_c1("noisy", seed_sub=s)
        d.append(oracle_mod.hypotheses(p.R, p.sigma, p.times, p.t_ref, p.vel,
                                       [4], [32], [20])["snr"][0] - clean)
    d = np.array(d)
    assert abs(d.mean()) < 4 / math.sqrt(d.size)
    assert abs(d.std() - 1.0) < 0.25


def test_bright_source_detected(oracle_mod):
    p = synth.make_c1("bright")
    out = oracle_mod.search(p.R, p.sigma, p.times, p.t_ref, p.vel)
    j, y, x = np.unravel_index(np.argmax(out["snr"]), out["snr"].shape)
    assert j == 4 and abs(y - 32) <= 1 and abs(x - 20) <= 1
    assert out["snr"].max() > 7


# ------------------------------------------------------------------ reductions

def test_reductions_against_plain_loops(oracle_mod):
    g = np.random.default_rng(2)
    J, H, W = 3, 5, 4
    snr = g.integers(-3, 4, size=(J, H, W)).astype(np.float64)  # many exact ties
    flux = g.standard_normal((J, H, W))
    s, f, y, x = oracle_mod.traj_max(snr, flux)
    for j in range(J):
        best = max((snr[j, yy, xx], -(yy * W + xx)) for yy in range(H) for xx in range(W))
        assert s[j] == best[0] and y[j] * W + x[j] == -best[1]
    b, bj, bf = oracle_mod.best_over_trajectories(snr, flux)
    for yy in range(H):
        for xx in range(W):
            jb = max(range(J), key=lambda j: (snr[j, yy, xx], -j))
            assert bj[yy, xx] == jb and b[yy, xx] == snr[jb, yy, xx]
    tk = oracle_mod.topk(snr, flux, 17)
    ref = sorted(((snr[j, yy, xx], j * H * W + yy * W + xx) for j in range(J)
                  for yy in range(H) for xx in range(W)), key=lambda t: (-t[0], t[1]))[:17]
    assert [(c[0], c[2] * H * W + c[3] * W + c[4]) for c in tk] == ref


# ------------------------------------------------------------------ Sec. 3.3 significance

@pytest.mark.parametrize("H,W,box", [(23, 31, 7), (17, 12, 63), (40, 40, 1), (33, 45, 15)])
def test_significance_is_local_std_definition(oracle_mod, H, W, box):
    """Direct definition: np.std over each clipped window."""
    g = np.random.default_rng(H * W + box)
    b = g.standard_normal((H, W)) * (1 + g.random((H, W)))
    got = oracle_mod.significance(b, box)
    h = box // 2
    for y in range(H):
        for x in range(W):
            w = b[max(0, y - h):y + h + 1, max(0, x - h):x + h + 1]
            sd = w.std()
            ref = b[y, x] / sd if sd > 0 else 0.0
            assert abs(got[y, x] - ref) <= 1e-10 * max(1.0, abs(ref))


def test_significance_interior_matches_uniform_filter(oracle_mod):
    g = np.random.default_rng(3)
    b = g.standard_normal((60, 70))
    box = 31
    m1 = ndimage.uniform_filter(b, box, mode="constant")
    m2 = ndimage.uniform_filter(b * b, box, mode="constant")
    sd = np.sqrt(m2 - m1 * m1)
    got = oracle_mod.significance(b, box)
    h = box // 2
    np.testing.assert_allclose(got[h:-h, h:-h], (b / sd)[h:-h, h:-h], rtol=1e-9)


@pytest.mark.parametrize("H,W,box", [(23, 31, 7), (17, 12, 63), (33, 45, 15), (9, 40, 21),
                                      (28, 19, 255), (12, 12, 1)])
def test_significance_whole_map_against_clipped_moments(oracle_mod, H, W, box):
    """Whole map, edges included, against a construction that shares nothing
    with the oracle's window loop: window sums of b and b^2 from
    scipy.ndimage.uniform_filter with zero padding, divided by the clipped
    window's pixel count (the same filter applied to ones), give the
    population mean and variance of the clipped window.  Boxes wider than the
    image and the one-pixel box (std 0 -> 0) are included."""
    g = np.random.default_rng(7 * H + W + box)
    b = g.standard_normal((H, W)) * (1 + g.random((H, W))) + 0.3
    got = oracle_mod.significance(b, box)
    ones = np.ones_like(b)
    n = ndimage.uniform_filter(ones, box, mode="constant", cval=0.0)
    s1 = ndimage.uniform_filter(b, box, mode="constant", cval=0.0) / n
    s2 = ndimage.uniform_filter(b * b, box, mode="constant", cval=0.0) / n
    var = np.maximum(s2 - s1 * s1, 0.0)
    h = box // 2
    cnt = np.array([[(min(H, y + h + 1) - max(0, y - h)) * (min(W, x + h + 1) - max(0, x - h))
                     for x in range(W)] for y in range(H)], np.float64)
    # the filter's count is the clipped window's size (a box of ones)
    np.testing.assert_allclose(n * box * box, cnt, rtol=1e-12)
    if box == 1:
        assert np.all(got == 0.0)
        return
    ref = b / np.sqrt(var)
    np.testing.assert_allclose(got, ref, rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("H,W,box", [(14, 11, 5), (10, 13, 31)])
def test_significance_whole_map_against_nan_padded_std(oracle_mod, H, W, box):
    """Whole map against scipy.ndimage.generic_filter(np.nanstd) over a
    NaN-padded image: the clipped window is the window with the off-image
    samples left out (not zero-filled)."""
    g = np.random.default_rng(H + 100 * W + box)
    b = g.standard_normal((H, W)) * 2.0 - 0.7
    got = oracle_mod.significance(b, box)
    sd = ndimage.generic_filter(b, np.nanstd, size=box, mode="constant", cval=np.nan)
    np.testing.assert_allclose(got, b / sd, rtol=1e-10)
    # a zero-padded window would give a different, wrong answer at the edges
    sd0 = ndimage.generic_filter(b, np.std, size=box, mode="constant", cval=0.0)
    assert not np.allclose(got[0, :], (b / sd0)[0, :], rtol=1e-6)


def test_significance_invariants(oracle_mod):
    g = np.random.default_rng(4)
    b = g.standard_normal((30, 30))
    s = oracle_mod.significance(b, 9)
    np.testing.assert_allclose(oracle_mod.significance(3.5 * b, 9), s, rtol=1e-12)
    assert np.all(oracle_mod.significance(np.full((10, 10), 2.0), 5) == 0)
    # a white-noise map's significance is ~ N(0,1) (sampled pixels)
    big = g.standard_normal((400, 400))
    ys, xs = np.meshgrid(np.arange(25, 375, 7), np.arange(25, 375, 7), indexing="ij")
    v = oracle_mod.significance(big, 51, pixels=(ys, xs))
    assert abs(v.mean()) < 0.05 and abs(v.std() - 1.0) < 0.05
    full = oracle_mod.significance(big[:40, :50], 9)
    np.testing.assert_allclose(oracle_mod.significance(big[:40, :50], 9, pixels=([3, 39], [0, 49])),
                               [full[3, 0], full[39, 49]], rtol=0)


def test_detections_order_and_threshold(oracle_mod):
    sig = np.array([[1.0, 5.0, 3.0], [5.0, 2.9, 4.0]])
    best = sig * 2
    bj = np.array([[0, 1, 0], [1, 1, 0]])
    flux = np.stack([sig, sig + 10])
    d = oracle_mod.detections(sig, best, bj, flux, 3.0, 10)
    assert [(t[4], t[5]) for t in d] == [(0, 1), (1, 0), (1, 2), (0, 2)]
    assert d[0][2] == 15.0 and d[2][2] == 4.0
    assert len(oracle_mod.detections(sig, best, bj, flux, 3.0, 2)) == 2


# ------------------------------------------------------------------ shift-stack vs matched filter

def _closed_form_ratio(f, sigma_px=0.7, stamp=5):
    """Noise-free SNR(matched filter) / SNR(shift-stack) for a source on the
    filter's own track, sigma = 1, one frame at phase f per axis:
    SNR_mf = A sqrt(sum W^2), SNR_ss = A W(anchor) (1-pixel filter of weight 1)."""
    taps = np.arange(stamp) - stamp // 2
    g = np.exp(-0.5 * ((taps - f) / sigma_px) ** 2)
    g /= g.sum()
    w2 = (g ** 2).sum() ** 2
    return math.sqrt(w2) / g[stamp // 2] ** 2


@pytest.mark.parametrize("f,expect", [(0.0, 1.26), (0.49, 2.0)])
def test_shift_stack_is_the_one_pixel_filter(oracle_mod, f, expect):
    """A 1x1 stamp is the shift-stack filter (one weight of 1 at the pixel
    nearest the track per frame, Sec. 3.2); on a noise-free source its SNR is
    below the full PRF filter's by the closed-form ratio."""
    T, H, W = 1, 15, 15
    v = f / (1.0 / 48.0) if f else 0.0
    times = np.array([2000.0 + 1.0 / 48.0]) if f else np.array([2000.0])
    t_ref = 2000.0
    src = [synth.Source(7.0, 7.0, v, v, 1.0)]
    R = synth.add_sources(np.zeros((T, H, W)), times, t_ref, src).astype(np.float32)
    sig = np.ones((H, W), np.float32)
    vel = np.array([[v, v]])
    mf = oracle_mod.hypotheses(R, sig, times, t_ref, vel, [0], [7], [7], stamp=5)["snr"][0]
    ss = oracle_mod.hypotheses(R, sig, times, t_ref, vel, [0], [7], [7], stamp=1)["snr"][0]
    ratio = mf / ss
    assert abs(ratio - _closed_form_ratio(f)) < 1e-6 * ratio
    assert abs(ratio - expect) < 0.05
