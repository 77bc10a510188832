"""Pins of the oracle's aperture phase term (defocus), a complex generalised
antenna parameter (Eq. DA with complex a_i; Sec. 5.3 names aperture phase
terms as the first shape parameters to solve for).

A defocus delta multiplies the illumination by exp(i delta (r/R)^2), R = D/2,
so the pattern E becomes complex and the visibility carries E_i conj(E_j)
(Eq. ME).  The pins tie the oracle to things outside it: the Airy pattern and
the Gaussian at delta = 0 (closed forms and scipy's Bessel J1); direct
two-dimensional Fourier sums of the defocused illumination (no Bessel
functions, no Hankel reduction) for both the uniform disc and the Gaussian
aperture, whose closed form they also pin; central differences in delta of
the pattern, the visibilities and chi^2; Hermitian symmetry; and recovery of
injected defocus by the damped step.
"""
import math

import numpy as np
import pytest
from scipy.special import j1

ARCSEC = math.pi / 180 / 3600
C_LIGHT = 299792458.0


def _fourier_disc(dish, freq, delta, rho, n_t=2000, n_th=256):
    """E(rho) of the uniform disc with the defocus phase, as the direct
    two-dimensional Fourier sum of the illumination over the aperture (polar
    midpoint rule), normalised by the sum of the illumination."""
    lam = C_LIGHT / freq
    R = dish / 2
    t = (np.arange(n_t) + 0.5) / n_t
    th = 2 * np.pi * (np.arange(n_th) + 0.5) / n_th
    T, TH = np.meshgrid(t, th, indexing="ij")
    x, y = R * T * np.cos(TH), R * T * np.sin(TH)
    area = T  # polar element r dr dtheta, up to constants
    ap = np.exp(1j * delta * T ** 2)
    # the displacement along +l (the pattern is radial)
    return np.sum(ap * np.exp(-2j * np.pi * x * rho / lam) * area) / np.sum(area)


def _fourier_gauss(dish, freq, sigma_ld, delta, rho, n=801, extent=6.0):
    """E(rho) of the Gaussian aperture exp(-2 pi^2 s^2 |x|^2 / lambda^2) times
    the defocus phase exp(i delta |x|^2 / R^2), as a direct Cartesian Fourier
    sum (the aperture is negligible beyond `extent` of its widths), normalised
    to the sum of the illumination's magnitude."""
    lam = C_LIGHT / freq
    s = sigma_ld * lam / dish
    R = dish / 2
    width = lam / (2 * np.pi * s)  # the aperture's 1/e^{1/2} radius
    x = np.linspace(-extent * width, extent * width, n)
    X, Y = np.meshgrid(x, x, indexing="ij")
    r2 = X ** 2 + Y ** 2
    mag = np.exp(-2 * np.pi ** 2 * s ** 2 * r2 / lam ** 2)
    ap = mag * np.exp(1j * delta * r2 / R ** 2)
    return np.sum(ap * np.exp(-2j * np.pi * X * rho / lam)) / np.sum(mag)


def test_zero_defocus_is_the_real_pattern(oracle_lib):
    """delta = 0: the uniform disc gives 2 J1(x)/x (scipy's J1), the Gaussian
    mode exp(-rho^2/(2 s^2)), both real, and zero derivative's real part."""
    o = oracle_lib
    D, f = 25.0, 1.4e9
    k = math.pi * D * f / C_LIGHT
    for rho in np.linspace(1e-6, 12.0 / k, 23):
        e, de = o.efp_defocus(0, D, 1.0, f, 0.0, rho * 0.6, rho * 0.8)
        x = k * rho
        assert abs(e - 2 * j1(x) / x) < 1e-13
        s = 1.3 * C_LIGHT / f / D
        eg, _ = o.efp_defocus(1, D, 1.3, f, 0.0, rho * 0.6, rho * 0.8)
        assert abs(eg - math.exp(-rho ** 2 / (2 * s * s))) < 1e-14
    e0, _ = o.efp_defocus(0, D, 1.0, f, 0.0, 0.0, 0.0)
    assert abs(e0 - 1.0) < 1e-14


@pytest.mark.parametrize("delta", [0.4, -1.1, 2.5])
def test_disc_defocus_against_direct_fourier_sum(oracle_lib, delta):
    """The Hankel-transform quadrature against the two-dimensional Fourier sum
    of the defocused uniform disc: normalisation, the sign of delta and the
    argument of J0 all enter."""
    o = oracle_lib
    D, f = 25.0, 1.4e9
    k = math.pi * D * f / C_LIGHT
    for x in (0.0, 0.7, 2.2, 4.0, 6.5):
        rho = x / k
        e, _ = o.efp_defocus(0, D, 1.0, f, delta, 0.0, rho)
        ref = _fourier_disc(D, f, delta, rho)
        assert abs(e - ref) < 2e-6, (x, e, ref)


@pytest.mark.parametrize("delta", [0.3, -0.9, 1.7])
def test_gaussian_defocus_closed_form_against_direct_fourier_sum(oracle_lib, delta):
    """The closed form z exp(-z rho^2/(2 s^2)), z = 1/(1 - i kappa), kappa =
    2 delta/(pi^2 sigma_ld^2), against the Fourier sum of the defocused
    Gaussian aperture."""
    o = oracle_lib
    D, f, sl = 25.0, 1.6e9, 1.5
    s = sl * C_LIGHT / f / D
    for r in (0.0, 0.5, 1.2, 2.0):
        e, _ = o.efp_defocus(1, D, sl, f, delta, r * s, 0.0)
        ref = _fourier_gauss(D, f, sl, delta, r * s)
        assert abs(e - ref) < 1e-7, (r, e, ref)


@pytest.mark.parametrize("illum", [0, 1])
def test_pattern_defocus_derivative_central_differences(oracle_lib, illum):
    o = oracle_lib
    D, f, h = 25.0, 1.3e9, 1e-5
    for delta in (-0.8, 0.0, 0.45):
        for dl, dm in ((0.0, 0.0), (0.004, -0.002), (-0.007, 0.003)):
            _, de = o.efp_defocus(illum, D, 1.5, f, delta, dl, dm)
            ep, _ = o.efp_defocus(illum, D, 1.5, f, delta + h, dl, dm)
            em, _ = o.efp_defocus(illum, D, 1.5, f, delta - h, dl, dm)
            fd = (ep - em) / (2 * h)
            assert abs(de - fd) < 1e-8 * max(1.0, abs(de)), (delta, dl, dm, de, fd)


def _problem(o, illum=0, n_ant=4, n_time=3, seed=5, n_pol=2, swap=False):
    rng = np.random.default_rng(seed)
    i, j = np.triu_indices(n_ant, 1)
    ant1, ant2 = np.tile(i, n_time), np.tile(j, n_time)
    uv = rng.uniform(-2500.0, 2500.0, size=(ant1.size, 2))
    if swap:  # the same baselines stored the other way round, uv negated
        ant1, ant2, uv = ant2, ant1, -uv
    src_l, src_m = rng.uniform(-0.01, 0.01, 5), rng.uniform(-0.01, 0.01, 5)
    flux = rng.uniform(0.3, 1.5, 5)
    half = ant1.size // 2
    prob = o.Problem(src_l, src_m, flux, n_ant, ant1, ant2, uv, [0, half, ant1.size], [1.2e9, 1.7e9],
                     n_pol=n_pol, illum=illum, gauss_sigma_ld=1.5, squint_frac=0.03)
    offs = rng.normal(0.0, 30 * ARCSEC, size=prob.offsets_shape())
    dfc = rng.uniform(-0.6, 0.6, size=prob.offsets_shape()[:3])
    return prob, offs, dfc


@pytest.mark.parametrize("illum", [0, 1])
def test_visibility_hermitian_with_complex_patterns(oracle_lib, illum):
    """V_ji(-u) = conj V_ij(u) when each antenna keeps its own defocus."""
    o = oracle_lib
    p1, offs, dfc = _problem(o, illum)
    p2, _, _ = _problem(o, illum, swap=True)
    v1, _ = o.predict_defocus(p1, offs, dfc)
    v2, _ = o.predict_defocus(p2, offs, dfc)
    np.testing.assert_allclose(v2, np.conj(v1), rtol=0, atol=1e-13 * np.abs(v1).max())


def test_zero_defocus_matches_the_real_predict(oracle_lib):
    o = oracle_lib
    prob, offs, _ = _problem(o, 0)
    v0, _ = o.predict_defocus(prob, offs, 0.0)
    ref = o.predict(prob, offs)
    np.testing.assert_allclose(v0, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("illum", [0, 1])
def test_visibility_defocus_derivative_central_differences(oracle_lib, illum):
    o = oracle_lib
    prob, offs, dfc = _problem(o, illum)
    _, dv = o.predict_defocus(prob, offs, dfc)
    h = 1e-5
    for (s, pol, a) in ((0, 0, 1), (1, 1, 3), (0, 1, 0)):
        dp, dm = dfc.copy(), dfc.copy()
        dp[s, pol, a] += h
        dm[s, pol, a] -= h
        fd = (o.predict_defocus(prob, offs, dp)[0] - o.predict_defocus(prob, offs, dm)[0]) / (2 * h)
        # the analytic derivative of the rows of interval s touching antenna a at pol
        r0, r1 = prob.int_row_ptr[s], prob.int_row_ptr[s + 1]
        an = np.zeros_like(fd)
        for r in range(r0, r1):
            if prob.ant1[r] == a:
                an[r, :, pol] = dv[r, :, pol, 0]
            elif prob.ant2[r] == a:
                an[r, :, pol] = dv[r, :, pol, 1]
        np.testing.assert_allclose(an, fd, rtol=0, atol=2e-8 * np.abs(fd).max())


@pytest.mark.parametrize("illum", [0, 1])
def test_defocus_sums_against_chi2(oracle_lib, illum):
    """g = -1/2 dchi^2/ddelta_a by central differences of chi^2; H =
    sum w |dV/ddelta_a|^2 from the explicit derivatives; sum of chi over
    antennas = 2 chi^2."""
    o = oracle_lib
    prob, offs, dfc = _problem(o, illum)
    rng = np.random.default_rng(9)
    truth = dfc + rng.normal(0, 0.2, dfc.shape)
    vobs, _ = o.predict_defocus(prob, offs, truth)
    w = rng.uniform(0.5, 2.0, prob.vis_shape())
    acc = o.defocus_gradient(prob, offs, dfc, vobs, w)

    def chi2(d):
        v, _ = o.predict_defocus(prob, offs, d)
        return float(np.sum(w * np.abs(vobs - v) ** 2))

    h = 1e-5
    for (s, pol, a) in ((0, 0, 1), (1, 1, 2), (1, 0, 3)):
        dp, dm = dfc.copy(), dfc.copy()
        dp[s, pol, a] += h
        dm[s, pol, a] -= h
        g_fd = -0.5 * (chi2(dp) - chi2(dm)) / (2 * h)
        assert abs(acc[s, pol, a, 1] - g_fd) < 1e-6 * max(1.0, abs(g_fd)), (acc[s, pol, a, 1], g_fd)
    _, dv = o.predict_defocus(prob, offs, dfc)
    H = np.zeros(prob.offsets_shape()[:3])
    for r in range(prob.n_row):
        s = np.searchsorted(prob.int_row_ptr, r, side="right") - 1
        for end, a in ((0, prob.ant1[r]), (1, prob.ant2[r])):
            H[s, :, a] += np.sum(w[r] * np.abs(dv[r, :, :, end]) ** 2, axis=0)
    np.testing.assert_allclose(acc[..., 2], H, rtol=1e-12)
    v, _ = o.predict_defocus(prob, offs, dfc)
    np.testing.assert_allclose(acc[..., 0].sum(), 2 * np.sum(w * np.abs(vobs - v) ** 2), rtol=1e-12)


def test_defocus_step_edge_cases(oracle_lib):
    o = oracle_lib
    acc = np.zeros((2, 1, 3, 3))
    acc[0, 0, 0] = [1.0, 0.5, 2.0]
    acc[0, 0, 1] = [1.0, 0.5, 0.0]      # no curvature: kept, flagged
    acc[0, 0, 2] = [1.0, np.nan, 1.0]   # non-finite: kept, flagged
    acc[1, 0, :] = [1.0, -0.3, 3.0]
    d0 = np.full((2, 1, 3), 0.2)
    d, nu, mx = o.defocus_step(acc, 0.5, d0)
    assert d[0, 0, 0] == 0.2 + 0.5 * 0.5 / 2.0 and nu[0, 0, 0] == 0
    assert d[0, 0, 1] == 0.2 and nu[0, 0, 1] == 1
    assert d[0, 0, 2] == 0.2 and nu[0, 0, 2] == 1
    np.testing.assert_allclose(d[1, 0], 0.2 - 0.5 * 0.1)
    assert mx[0] == 0.125 and abs(mx[1] - 0.05) < 1e-15


@pytest.mark.parametrize("illum", [0, 1])
def test_defocus_recovery_noiseless(oracle_lib, illum):
    """Damped Gauss-Newton steps from a start 0.15 rad (rms) off the injected
    defocus, on noiseless data: chi^2 falls by four orders and every antenna
    moves to within 0.04 rad of its truth.  The rest converges slowly: within
    the main lobe a defocus common to all antennas nearly cancels in
    E_i conj(E_j) (to first order each pattern only gains the phase delta/2,
    and |E|^2 is even in delta), a direction along which the data give
    almost no curvature and the per-antenna steps creep."""
    o = oracle_lib
    prob, offs, truth = _problem(o, illum, n_ant=5, n_time=4)
    vobs, _ = o.predict_defocus(prob, offs, truth)
    rng = np.random.default_rng(3)
    pert = rng.normal(0, 0.15, truth.shape)
    pert -= pert.mean(axis=2, keepdims=True)
    d = truth + pert
    chi0 = float(o.defocus_gradient(prob, offs, d, vobs, 1.0)[..., 0].sum())
    for _ in range(20):
        acc = o.defocus_gradient(prob, offs, d, vobs, 1.0)
        d, _, mx = o.defocus_step(acc, 0.5, d)
    chi = float(o.defocus_gradient(prob, offs, d, vobs, 1.0)[..., 0].sum())
    assert chi < 1e-4 * chi0, (chi, chi0)
    assert np.abs(d - truth).max() < 0.04, np.abs(d - truth).max()
