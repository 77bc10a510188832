"""Pins of the oracle's beam-width scale, a generalised antenna parameter.

Eq. DA holds for any antenna parameter a_i, and Sec. 5.3 solves for the shape
of the primary beam with the same machinery as the pointing offsets.  The
first such parameter here is a width scale sigma per (interval, pol,
antenna): the pattern becomes E0(d / sigma).  These tests pin the oracle's
derivative with respect to sigma, the sums of Eq. DCHIDD built from it and
the damped update, against closed forms, finite differences and recovery.
"""
import math

import numpy as np
import pytest

from paper_1709_08681_amd import synth

ARCSEC = math.pi / 180 / 3600
C_LIGHT = 299792458.0


@pytest.fixture(scope="module")
def o():
    import oracle
    return oracle


def _problem(o, scale=None, illum=0, par_angle=None, aperture=None, seed=3, n_src=6, squint=0.03):
    rng = np.random.default_rng(seed)
    n_ant, n_time = 4, 4
    i, j = np.triu_indices(n_ant, 1)
    ant1, ant2 = np.tile(i, n_time), np.tile(j, n_time)
    uv = rng.uniform(-2500.0, 2500.0, size=(ant1.size, 2))
    sl, sm = rng.uniform(-0.012, 0.012, n_src), rng.uniform(-0.012, 0.012, n_src)
    flux = rng.uniform(0.2, 1.5, n_src)
    pa = None if par_angle is None else np.broadcast_to(par_angle, ant1.shape).astype(np.float64)
    return o.Problem(sl, sm, flux, n_ant, ant1, ant2, uv, [0, 2 * 6, ant1.size], [1.2e9, 1.7e9], n_pol=2,
                     squint_frac=squint, illum=illum, gauss_sigma_ld=1.0, par_angle=pa, aperture=aperture,
                     beam_scale=scale)


def _scales(o, seed=4, spread=0.05):
    base = _problem(o)
    return np.random.default_rng(seed).uniform(1 - spread, 1 + spread, base.offsets_shape()[:3])


def test_unit_scale_is_the_nominal_beam(o):
    base = _problem(o)
    ones = _problem(o, scale=np.ones(base.offsets_shape()[:3]))
    offs = np.random.default_rng(5).normal(0.0, 30 * ARCSEC, base.offsets_shape())
    v0, d0 = o.predict(base, offs, want_grad=True)
    v1, d1 = o.predict(ones, offs, want_grad=True)
    assert np.array_equal(v0, v1) and np.array_equal(d0, d1)


def test_gaussian_scale_derivative_closed_form(o):
    """One source, Gaussian main lobe E = exp(-|d|^2 / (2 s^2 sigma^2)): the
    visibility is flux E_i E_j e^{+2 pi i u.l}, so
    dV/dsigma_i = V |d_i|^2 / (s^2 sigma_i^3) with d_i = l - p_i."""
    f = np.array([1.4e9])
    lam = C_LIGHT / f[0]
    s = 1.0 * lam / 25.0
    l, m = 0.004, -0.0025
    uv = np.array([[800.0, -300.0], [1500.0, 900.0]])
    sig = np.array([[[0.93, 1.08]]])
    prob = o.Problem([l], [m], [1.3], 2, [0, 0], [1, 1], uv, [0, 2], f, illum=1, gauss_sigma_ld=1.0,
                     beam_scale=sig)
    offs = np.array([[[[0.0007, -0.0004], [-0.0003, 0.0009]]]])
    v, ds = o.predict_scale(prob, offs)
    for end in range(2):
        d2 = (l - offs[0, 0, end, 0]) ** 2 + (m - offs[0, 0, end, 1]) ** 2
        want = v[:, 0, 0] * d2 / (s * s * sig[0, 0, end] ** 3)
        np.testing.assert_allclose(ds[:, 0, 0, end], want, rtol=1e-12)


@pytest.mark.parametrize("mode", ["airy", "gauss", "mount", "aperture"])
def test_scale_derivative_matches_central_differences(o, mode):
    """dV/dsigma_a against central differences of V in sigma_a (h = 1e-6),
    each end of every baseline, two pols with squint."""
    kw = {}
    if mode == "gauss":
        kw["illum"] = 1
    if mode in ("mount", "aperture"):
        kw["par_angle"] = np.random.default_rng(6).uniform(-1.0, 1.0, _problem(o).n_row)
    if mode == "aperture":
        kw["illum"] = 2
        kw["aperture"] = synth.measured_aperture(seed=2)
    sc = _scales(o)
    prob = _problem(o, scale=sc, **kw)
    offs = np.random.default_rng(7).normal(0.0, 30 * ARCSEC, prob.offsets_shape())
    _, ds = o.predict_scale(prob, offs)
    h = 1e-6
    for s, pol, ant in [(0, 0, 1), (0, 1, 2), (1, 0, 3), (1, 1, 0)]:
        sp, sm = sc.copy(), sc.copy()
        sp[s, pol, ant] += h
        sm[s, pol, ant] -= h
        fd = (o.predict(_problem(o, scale=sp, **kw), offs) - o.predict(_problem(o, scale=sm, **kw), offs))
        fd = fd[..., pol] / (2 * h)
        r0, r1 = prob.int_row_ptr[s], prob.int_row_ptr[s + 1]
        rows = np.arange(prob.n_row)
        inside = (rows >= r0) & (rows < r1)
        an = np.where((inside & (prob.ant1 == ant))[:, None], ds[:, :, pol, 0], 0) + \
            np.where((inside & (prob.ant2 == ant))[:, None], ds[:, :, pol, 1], 0)
        assert np.linalg.norm(fd - an) <= 1e-7 * np.linalg.norm(an), (mode, s, pol, ant)


def test_scale_sums_match_chi2_and_jacobian(o):
    """g_sigma = -1/2 d chi^2 / d sigma by central differences, and H_sigma =
    sum w |dV/dsigma|^2 from the explicit per-visibility derivatives."""
    sc = _scales(o)
    prob = _problem(o, scale=sc)
    rng = np.random.default_rng(8)
    offs = rng.normal(0.0, 30 * ARCSEC, prob.offsets_shape())
    vobs = o.predict(_problem(o, scale=sc * rng.uniform(0.97, 1.03, sc.shape)), offs)
    w = rng.uniform(0.5, 2.0, vobs.shape)
    acc = o.scale_gradient(prob, offs, vobs, w)
    h = 1e-6
    for s, pol, ant in [(0, 0, 1), (0, 1, 3), (1, 0, 0), (1, 1, 2)]:
        sp, sm = sc.copy(), sc.copy()
        sp[s, pol, ant] += h
        sm[s, pol, ant] -= h
        chi = [float((w * np.abs(vobs - o.predict(_problem(o, scale=x), offs)) ** 2).sum()) for x in (sp, sm)]
        fd = (chi[0] - chi[1]) / (2 * h)
        assert abs(-0.5 * fd - acc[s, pol, ant, 1]) <= 1e-6 * abs(acc[s, pol, ant, 1]) + 1e-9
    _, ds = o.predict_scale(prob, offs)
    H = np.zeros(acc.shape[:3])
    for r in range(prob.n_row):
        s = np.searchsorted(prob.int_row_ptr, r, side="right") - 1
        for end, a in ((0, prob.ant1[r]), (1, prob.ant2[r])):
            H[s, :, a] += (w[r] * np.abs(ds[r, :, :, end]) ** 2).sum(axis=0)
    np.testing.assert_allclose(acc[..., 2], H, rtol=1e-12)
    # chi is the same per-antenna sum as the offsets' gradient gives
    np.testing.assert_allclose(acc[..., 0], o.gradient(prob, offs, vobs, w)[..., 0], rtol=1e-13)


def test_scale_step_cases(o):
    acc = np.zeros((1, 1, 4, 3))
    acc[0, 0, 0] = [1.0, 0.02, 4.0]      # ordinary: +gain * g / H
    acc[0, 0, 1] = [1.0, 0.02, 0.0]      # no data
    acc[0, 0, 2] = [1.0, -50.0, 1.0]     # step would make sigma negative
    acc[0, 0, 3] = [1.0, np.nan, 2.0]    # non-finite
    s, nu, mx = o.scale_step(acc, 0.5, np.ones((1, 1, 4)))
    assert s[0, 0, 0] == 1.0 + 0.5 * 0.02 / 4.0
    assert np.array_equal(s[0, 0, 1:], np.ones(3))
    assert nu.tolist() == [[[0, 1, 1, 1]]]
    assert mx[0] == pytest.approx(0.5 * 0.02 / 4.0, rel=1e-12)


def test_scale_recovered_from_noiseless_data(o):
    """Injected scales (3% spread), true offsets: iterating the scale step
    from sigma = 1 with loop gain 0.5 recovers them.  (All antennas move
    together from sums taken at the previous iterate, as for the offsets;
    with gain 1 the two ends of each baseline overshoot together and the
    iteration stalls, which the loop gain of Eq. SelfCal avoids.)"""
    truth = _scales(o, seed=9, spread=0.03)
    offs = np.random.default_rng(10).normal(0.0, 30 * ARCSEC, truth.shape + (2,))
    vobs = o.predict(_problem(o, scale=truth), offs)
    s = np.ones_like(truth)
    for _ in range(80):
        acc = o.scale_gradient(_problem(o, scale=s), offs, vobs, 1.0)
        s, nu, mx = o.scale_step(acc, 0.5, s)
        if mx.max() < 1e-12:
            break
    assert np.abs(s - truth).max() < 1e-8


def test_offset_sums_with_scales_match_chi2_differences(o):
    """With widened and narrowed beams, the offsets' sums still equal
    -1/2 d chi^2 / d p (central differences, h = 0.01 arcsec), sky and
    mount frame."""
    sc = _scales(o, seed=11, spread=0.08)
    rng = np.random.default_rng(12)
    for pa in (None, rng.uniform(-1.0, 1.0, _problem(o).n_row)):
        prob = _problem(o, scale=sc, par_angle=pa)
        offs = rng.normal(0.0, 30 * ARCSEC, prob.offsets_shape())
        vobs = o.predict(prob, offs + rng.normal(0.0, 20 * ARCSEC, offs.shape))
        acc = o.gradient(prob, offs, vobs, 1.0)
        h = 0.01 * ARCSEC
        for s, pol, ant, ax in [(0, 0, 1, 0), (0, 1, 2, 1), (1, 0, 3, 1), (1, 1, 0, 0)]:
            op, om = offs.copy(), offs.copy()
            op[s, pol, ant, ax] += h
            om[s, pol, ant, ax] -= h
            fd = (float((np.abs(vobs - o.predict(prob, op)) ** 2).sum()) -
                  float((np.abs(vobs - o.predict(prob, om)) ** 2).sum())) / (2 * h)
            g = acc[s, pol, ant, 1 + ax]
            assert abs(-0.5 * fd - g) <= 1e-6 * abs(g) + 1e-9, (pa is None, s, pol, ant, ax)
