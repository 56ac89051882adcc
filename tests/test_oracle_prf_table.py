"""Pins of the oracle's tabulated PRF and pointing-jitter paths (Sec. 2:
the PRF is the share of a point source's flux each pixel records; Sec. 2.1
and 3.1: per-frame jitter theta_t of the pointing; Sec. 3.2: the filter is
the trajectory line, jitter included, convolved with the PRF).

Readings: the tabulated PRF P(u_y, u_x) is given on the grid
u = -(h+1) + i/q and read by bilinear interpolation; the stamp weight of
pixel (a, b) at phase (f_y, f_x) is P(a - f_y, b - f_x), used as given (not
renormalised); the jitter adds to the displacement, D = v (t - t_ref) + theta.

Each pin ties the oracle to something other than itself: functions that
bilinear interpolation reproduces exactly, grid points, scipy's correlation,
a shifted copy of the data, the interpolation error bound, and the
dense-filter brute force."""
import math

import numpy as np
import pytest
from scipy import ndimage

from paper_2209_09848_amd import synth

from tests import brute


def _grid(stamp, q):
    h = stamp // 2
    return -(h + 1) + np.arange((stamp + 1) * q + 1, dtype=np.float64) / q


@pytest.mark.parametrize("stamp,q", [(3, 1), (5, 4), (5, 9), (7, 3)])
def test_table_weights_reproduce_bilinear_functions(oracle_mod, stamp, q):
    """P(uy, ux) = c0 + c1 uy + c2 ux + c3 uy ux is interpolated exactly, so
    W(a, b) must equal it at (a - fy, b - fx): pins the grid origin, the step,
    the axis roles and the sign of the phase."""
    g = np.random.default_rng(11)
    c0, c1, c2, c3 = 0.3, -0.7, 1.9, 0.45
    u = _grid(stamp, q)
    tab = c0 + c1 * u[:, None] + c2 * u[None, :] + c3 * u[:, None] * u[None, :]
    h = stamp // 2
    a = np.arange(-h, h + 1, dtype=np.float64)
    for _ in range(20):
        fy, fx = g.uniform(-0.5, 0.5, 2)
        w = oracle_mod.weights(oracle_mod.PRF_TABLE, 0.0, stamp, fy, fx, tab, q)
        uy, ux = (a - fy)[:, None], (a - fx)[None, :]
        ref = c0 + c1 * uy + c2 * ux + c3 * uy * ux
        np.testing.assert_allclose(w, ref, rtol=0, atol=1e-12)
    # the phase -1/2 edge reaches u = h + 1/2, still inside the grid
    w = oracle_mod.weights(oracle_mod.PRF_TABLE, 0.0, stamp, -0.5, -0.5, tab, q)
    assert np.isclose(w[-1, -1], c0 + (c1 + c2) * (h + 0.5) + c3 * (h + 0.5) ** 2, atol=1e-12)


def test_table_weights_at_grid_points(oracle_mod):
    """Phases on the grid (q = 4, exact in binary) read single samples of an
    arbitrary, asymmetric table."""
    g = np.random.default_rng(12)
    stamp, q = 5, 4
    n = (stamp + 1) * q + 1
    tab = g.random((n, n))
    for fy, fx in [(0.0, 0.0), (-0.5, 0.25), (0.25, -0.25), (-0.25, 0.0)]:
        w = oracle_mod.weights(oracle_mod.PRF_TABLE, 0.0, stamp, fy, fx, tab, q)
        for a in range(-2, 3):
            for b in range(-2, 3):
                i = int(round((a - fy + 3) * q))
                m = int(round((b - fx + 3) * q))
                assert w[a + 2, b + 2] == tab[i, m]


def test_table_zero_velocity_is_correlation(oracle_mod):
    """v = 0, no jitter: the phase is 0, so nu = K (x) sum_k R_k ivar and
    Lam = K^2 (x) (T ivar) with K[a][b] = P(a, b) read off the grid, (x) being
    scipy's zero-padded correlation.  The random table is asymmetric, so a
    transposed or mirrored kernel fails."""
    g = np.random.default_rng(13)
    T, H, W = 6, 21, 26
    stamp, q = 5, 3
    n = (stamp + 1) * q + 1
    tab = g.random((n, n))
    R = g.standard_normal((T, H, W)).astype(np.float32)
    sigma = (0.5 + g.random((H, W))).astype(np.float32)
    sigma[2, 5] = 0.0
    times = synth.times_with_gap(T, 2)
    out = oracle_mod.search(R, sigma, times, times[0], np.zeros((1, 2)),
                            prf_kind=oracle_mod.PRF_TABLE, stamp=stamp, prf_table=tab, prf_q=q)
    K = tab[q::q, q::q][:stamp, :stamp]      # u = -2 .. 2
    iv = brute.ivar_map(sigma)
    nu_ref = ndimage.correlate((R.astype(np.float64) * iv[None]).sum(0), K, mode="constant", cval=0.0)
    lam_ref = ndimage.correlate(T * iv, K ** 2, mode="constant", cval=0.0)
    np.testing.assert_allclose(out["nu"][0], nu_ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out["lam"][0], lam_ref, rtol=1e-12, atol=1e-12)


def test_table_of_a_gaussian_within_interpolation_bound(oracle_mod):
    """A table sampled from the unnormalised Gaussian product g(uy) g(ux)
    (sigma 0.7) reproduces it to within the bilinear error bound
    (dy^2/8 max|d2/dy2| + dx^2/8 max|d2/dx2| = 2 / (8 q^2 sigma^2))."""
    sp, stamp, q = 0.7, 5, 32
    u = _grid(stamp, q)
    gg = np.exp(-0.5 * (u / sp) ** 2)
    tab = np.outer(gg, gg)
    bound = 2.0 / (8.0 * q * q * sp * sp)
    rng = np.random.default_rng(14)
    a = np.arange(-2, 3, dtype=np.float64)
    worst = 0.0
    for _ in range(30):
        fy, fx = rng.uniform(-0.5, 0.5, 2)
        w = oracle_mod.weights(oracle_mod.PRF_TABLE, 0.0, stamp, fy, fx, tab, q)
        ref = np.outer(np.exp(-0.5 * ((a - fy) / sp) ** 2), np.exp(-0.5 * ((a - fx) / sp) ** 2))
        worst = max(worst, float(np.abs(w - ref).max()))
    assert worst <= bound
    assert worst > bound / 50      # the bound is not vacuous here


def test_integer_jitter_equals_shifted_frames(oracle_mod):
    """An integer jitter theta_k moves the trail by theta_k in frame k: with
    uniform sigma it equals the search without jitter over frames shifted by
    -theta_k, at start pixels whose every stamp stays on the image."""
    g = np.random.default_rng(15)
    T, H, W = 8, 34, 37
    R = g.standard_normal((T, H, W)).astype(np.float32)
    sigma = np.ones((H, W), np.float32)
    times = synth.times_with_gap(T, 4, 0.5)
    vel = np.array([[3.3, -1.2], [-2.1, 2.6]])
    th = g.integers(-2, 3, size=(T, 2)).astype(np.float64)
    Rs = np.zeros_like(R)
    for k in range(T):
        tx, ty = int(th[k, 0]), int(th[k, 1])
        # Rs_k(Y, X) = R_k(Y + ty, X + tx)
        Rs[k] = np.roll(R[k], shift=(-ty, -tx), axis=(0, 1))
    M = 9
    reg = (M, H - M, M, W - M)
    for kind, tab, q in [(oracle_mod.PRF_SAMPLED, None, 0),
                         (oracle_mod.PRF_TABLE, synth.TabulatedPSF().table(5, 4), 4)]:
        a = oracle_mod.search(R, sigma, times, times[0], vel, prf_kind=kind, region=reg,
                              prf_table=tab, prf_q=q, jitter=th)
        b = oracle_mod.search(Rs, sigma, times, times[0], vel, prf_kind=kind, region=reg,
                              prf_table=tab, prf_q=q)
        np.testing.assert_allclose(a["nu"], b["nu"], rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(a["lam"], b["lam"], rtol=1e-13, atol=1e-13)
    # and the jitter does change the answer
    c = oracle_mod.search(R, sigma, times, times[0], vel, prf_kind=kind, region=reg,
                          prf_table=tab, prf_q=q)
    assert np.abs(c["nu"] - a["nu"]).max() > 0.1


def test_constant_jitter_equals_velocity_over_unit_time(oracle_mod):
    """With every frame one day after t_ref, a constant jitter theta on a
    standing trajectory gives the displacement of velocity theta without
    jitter, to the last bit (0*1 + theta = theta*1 + 0)."""
    g = np.random.default_rng(16)
    T, H, W = 5, 19, 22
    R = g.standard_normal((T, H, W)).astype(np.float32)
    sigma = (0.6 + g.random((H, W))).astype(np.float32)
    times = np.full(T, 2001.0)
    t_ref = 2000.0
    th = np.array([1.37, -0.62])
    jit = np.tile(th, (T, 1))
    for kind, tab, q in [(oracle_mod.PRF_INTEGRATED, None, 0),
                         (oracle_mod.PRF_TABLE, synth.TabulatedPSF().table(5, 5), 5)]:
        a = oracle_mod.search(R, sigma, times, t_ref, np.zeros((1, 2)), prf_kind=kind,
                              prf_table=tab, prf_q=q, jitter=jit)
        b = oracle_mod.search(R, sigma, times, t_ref, th[None, :], prf_kind=kind,
                              prf_table=tab, prf_q=q)
        assert np.array_equal(a["nu"], b["nu"]) and np.array_equal(a["lam"], b["lam"])
    iy, ix, fy, fx = oracle_mod.offsets(times, t_ref, np.zeros((1, 2)), jitter=jit)
    assert (ix == 1).all() and (iy == -1).all()
    assert np.allclose(fx, 0.37) and np.allclose(fy, 0.38)


@pytest.mark.parametrize("use_table", [False, True])
def test_table_and_jitter_match_dense_filter_brute_force(oracle_mod, use_table):
    g = np.random.default_rng(17)
    T, H, W = 4, 9, 10
    R = g.standard_normal((T, H, W)).astype(np.float32)
    sigma = (0.5 + g.random((H, W))).astype(np.float32)
    sigma[4, 4] = -1.0
    times = synth.times_with_gap(T, 2, 0.3)
    vel = np.array([[4.1, -2.3], [-1.7, 3.9], [0.0, 0.0]])
    jit = synth.jitter_series(g, T, amp=0.4)
    stamp, q = 5, 6
    tab = synth.TabulatedPSF().table(stamp, q) if use_table else None
    kind = oracle_mod.PRF_TABLE if use_table else oracle_mod.PRF_SAMPLED
    out = oracle_mod.search(R, sigma, times, times[0], vel, prf_kind=kind, stamp=stamp,
                            prf_table=tab, prf_q=q if use_table else 0, jitter=jit)
    nu, lam = brute.search(R, sigma, times, times[0], vel, stamp=stamp, table=tab, q=q,
                           jitter=jit)
    np.testing.assert_allclose(out["nu"], nu, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(out["lam"], lam, rtol=1e-11, atol=1e-11)


def test_tabulated_psf_flux_estimate(oracle_mod):
    """A noise-free source drawn with the continuous PSF the table samples,
    on a jittered trail starting on a pixel centre: at the true hypothesis
    the filter is the source's own image up to the table's interpolation
    error, so the flux estimate nu/Lam recovers the injected flux."""
    T, H, W = 40, 40, 60
    times = synth.times_with_gap(T, 20, 0.5)
    t_ref = times[0]
    vel = np.array([[11.3, 2.7]])
    jit = synth.jitter_series(np.random.default_rng(18), T, amp=0.15)
    psf = synth.TabulatedPSF()
    src = [synth.Source(x=17.0, y=20.0, vx=11.3, vy=2.7, amp=5.0, traj=0)]
    R = np.zeros((T, H, W))
    k, y, x, v = synth.render_sources((T, H, W), times, t_ref, src, stamp=5, jitter=jit, psf=psf)
    np.add.at(R, (k, y, x), v)
    sigma = np.ones((H, W), np.float32)
    out = oracle_mod.hypotheses(R.astype(np.float32), sigma, times, t_ref, vel, [0], [20], [17],
                                prf_kind=oracle_mod.PRF_TABLE, stamp=5,
                                prf_table=psf.table(5, 9), prf_q=9, jitter=jit)
    assert abs(out["flux"][0] - 5.0) < 0.005 * 5.0
    # without the jitter in the filter the estimate is lower
    nj = oracle_mod.hypotheses(R.astype(np.float32), sigma, times, t_ref, vel, [0], [20], [17],
                               prf_kind=oracle_mod.PRF_TABLE, stamp=5,
                               prf_table=psf.table(5, 9), prf_q=9)
    assert nj["snr"][0] < out["snr"][0]


def test_oracle_rejects_bad_table_arguments(oracle_mod):
    T, H, W = 2, 8, 8
    R = np.zeros((T, H, W), np.float32)
    sigma = np.ones((H, W), np.float32)
    times = synth.times_uniform(T)
    with pytest.raises(ValueError):
        oracle_mod.search(R, sigma, times, times[0], np.zeros((1, 2)),
                          prf_kind=oracle_mod.PRF_TABLE, stamp=5, prf_table=np.zeros((5, 5)),
                          prf_q=1)
    with pytest.raises(ValueError):
        oracle_mod.search(R, sigma, times, times[0], np.zeros((1, 2)),
                          prf_kind=oracle_mod.PRF_TABLE, stamp=5, prf_table=None, prf_q=1)
    with pytest.raises(ValueError):
        oracle_mod.search(R, sigma, times, times[0], np.zeros((1, 2)), jitter=np.zeros((3, 2)))
