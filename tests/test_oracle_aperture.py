"""Pins of the oracle's measured-aperture mode (illum 2).

The far-field pattern of a dish is the Fourier transform of its aperture
illumination (Sec. 1 and Sec. 3; the VLA beam model of Sec. 4.2 is such a
transform of a simulated illumination with blockage and taper), and it is
fixed to the antenna mount, so it turns on the sky with the parallactic angle
(Sec. 1).  These tests pin the oracle's direct-sum transform to closed forms
and limits, and its mount-frame handling to the geometry of a joint rotation.
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


def _cells(n):
    return (np.arange(n) - 0.5 * (n - 1)) / n


def _problem(o, aperture, par_angle=None, seed=5, squint=0.03, src=None, uv=None, n_time=4):
    rng = np.random.default_rng(seed)
    n_ant = 4
    i, j = np.triu_indices(n_ant, 1)
    ant1, ant2 = np.tile(i, n_time), np.tile(j, n_time)
    uv_r = rng.uniform(-2500.0, 2500.0, size=(ant1.size, 2))
    sl, sm = rng.uniform(-0.012, 0.012, 6), rng.uniform(-0.012, 0.012, 6)
    flux = rng.uniform(0.2, 1.5, 6)
    if src is not None:
        sl, sm = src
    if uv is not None:
        uv_r = uv
    pa = None if par_angle is None else np.broadcast_to(par_angle, ant1.shape).astype(np.float64)
    return o.Problem(sl, sm, flux, n_ant, ant1, ant2, uv_r, [0, 2 * 6, ant1.size], [1.2e9, 1.7e9],
                     n_pol=2, squint_frac=squint, par_angle=pa, illum=2, aperture=aperture)


def test_rectangular_aperture_is_a_product_of_dirichlet_kernels(o):
    """Cells filled in rows [a0, n - 1 - a0] (x) and every column (y): the
    transform is the product of two Dirichlet kernels, sin(k pi t)/(k sin(pi t))
    with t = cell d / lambda, k = n - 2 a0 along l and n along m.  Pins the
    cell positions, the scale D/lambda and which array axis is l."""
    D, f = 25.0, 1.4e9
    lam = C_LIGHT / f
    for n, a0 in [(16, 5), (15, 3)]:
        A = np.zeros((n, n))
        A[a0:n - a0, :] = 1.0
        kx, ky = n - 2 * a0, n
        cell = D / n
        for dl, dm in [(0.3, 0.1), (-0.7, 0.45), (1.3, -0.2), (0.05, 1.9)]:
            dl_r, dm_r = dl * lam / D, dm * lam / D
            tx, ty = cell * dl_r / lam, cell * dm_r / lam
            want = (math.sin(kx * math.pi * tx) / (kx * math.sin(math.pi * tx)) *
                    math.sin(ky * math.pi * ty) / (ky * math.sin(math.pi * ty)))
            got = o.efp_aperture(A, D, f, dl_r, dm_r)[0]
            assert abs(got - want) <= 1e-13, (n, dl, dm, got, want)


def test_aperture_derivatives_match_central_differences(o):
    """dE/dc (c the beam centre, d = l - c) against central differences of E
    in d, h = 1e-4 lambda/D, on the synthetic blocked aperture."""
    D, f = 25.0, 1.6e9
    lam = C_LIGHT / f
    A = synth.measured_aperture(seed=3)
    h = 1e-4 * lam / D
    for dl, dm in [(0.2, 0.0), (0.6, -0.4), (-1.1, 0.7), (0.0, 1.4), (1.9, 1.2)]:
        dl_r, dm_r = dl * lam / D, dm * lam / D
        e = o.efp_aperture(A, D, f, dl_r, dm_r)
        fd_l = (o.efp_aperture(A, D, f, dl_r + h, dm_r)[0] - o.efp_aperture(A, D, f, dl_r - h, dm_r)[0]) / (2 * h)
        fd_m = (o.efp_aperture(A, D, f, dl_r, dm_r + h)[0] - o.efp_aperture(A, D, f, dl_r, dm_r - h)[0]) / (2 * h)
        scale = np.abs(e[1:]).max()
        assert abs(e[1] + fd_l) <= 1e-7 * scale and abs(e[2] + fd_m) <= 1e-7 * scale, (dl, dm)
    assert o.efp_aperture(A, D, f, 0.0, 0.0)[0] == 1.0


def test_uniform_disc_aperture_approaches_the_airy_pattern(o):
    """A uniformly illuminated disc sampled on n x n cells tends to
    2 J1(x)/x as n grows (the stair-stepped rim is the only difference):
    the largest difference in E and in dE/dc over the main lobe and first
    sidelobes shrinks roughly as 1/n."""
    D, f = 25.0, 1.4e9
    lam = C_LIGHT / f

    def err(n):
        x = _cells(n)
        X, Y = np.meshgrid(x, x, indexing="ij")
        A = (np.hypot(X, Y) <= 0.5).astype(float)
        worst = 0.0
        for d in np.linspace(0.25, 2.5, 10):
            for ang in (0.0, 0.3, 0.785):
                dl, dm = d * lam / D * math.cos(ang), d * lam / D * math.sin(ang)
                e = o.efp_aperture(A, D, f, dl, dm)
                a = o.efp(0, D, 1.0, f, dl, dm)
                worst = max(worst, abs(e[0] - a[0]), np.abs(e[1:] - a[1:]).max() / np.abs(a[1:]).max())
        return worst

    e64, e128, e256 = err(64), err(128), err(256)
    assert e64 > e128 > e256
    assert e128 / e256 > 1.8
    assert e256 < 8e-3


def test_mount_frame_joint_rotation(o):
    """Rotating the sky and every baseline by b and adding b to every
    parallactic angle rotates the whole system: with the pattern fixed to the
    mount and the offsets (and squint) in the mount frame, every visibility and
    every mount-frame derivative is unchanged.  The blocked aperture is not
    circular, so a pattern turned the wrong way would fail this."""
    A = synth.measured_aperture(seed=4)
    rng = np.random.default_rng(9)
    base = _problem(o, A, par_angle=0.0)
    chi = rng.uniform(-1.0, 1.0, base.n_row)
    p1 = _problem(o, A, par_angle=chi)
    b = 0.83
    c, s = math.cos(b), math.sin(b)
    rl = c * p1.src_l - s * p1.src_m
    rm = s * p1.src_l + c * p1.src_m
    ruv = np.stack([c * p1.uv_m[:, 0] - s * p1.uv_m[:, 1], s * p1.uv_m[:, 0] + c * p1.uv_m[:, 1]], -1)
    p2 = _problem(o, A, par_angle=chi + b, src=(rl, rm), uv=ruv)
    offs = rng.normal(0.0, 40 * ARCSEC, size=p1.offsets_shape())
    v1, d1 = o.predict(p1, offs, want_grad=True)
    v2, d2 = o.predict(p2, offs, want_grad=True)
    np.testing.assert_allclose(v2, v1, rtol=0, atol=1e-12 * np.abs(v1).max())
    np.testing.assert_allclose(d2, d1, rtol=0, atol=1e-11 * np.abs(d1).max())
    # and the pattern does turn: the same sky and uv at the turned angles differ
    p3 = _problem(o, A, par_angle=chi + b)
    assert np.abs(o.predict(p3, offs) - v1).max() > 1e-3 * np.abs(v1).max()


def test_mount_frame_zero_angle_is_the_sky_frame(o):
    A = synth.measured_aperture(seed=4)
    sky = _problem(o, A)
    mnt = _problem(o, A, par_angle=0.0)
    offs = np.random.default_rng(10).normal(0.0, 30 * ARCSEC, size=sky.offsets_shape())
    v1, d1 = o.predict(sky, offs, want_grad=True)
    v2, d2 = o.predict(mnt, offs, want_grad=True)
    assert np.array_equal(v1, v2) and np.array_equal(d1, d2)
    vobs = v1 * 1.1 + 0.05
    pl, pm = np.array([0.0, 0.004, -0.009]), np.array([0.003, -0.006, 0.001])
    np.testing.assert_allclose(o.image_gradient(mnt, offs, vobs, 1.0, pl, pm),
                               o.image_gradient(sky, offs, vobs, 1.0, pl, pm), rtol=1e-13, atol=0.0)


def test_aperture_sums_match_chi2_differences(o):
    """Per-row parallactic angle, two pols with squint: the sums against
    central differences of chi^2 in the mount-frame offsets (h = 0.01 arcsec),
    and the image gradient against central differences in a pixel's flux."""
    A = synth.measured_aperture(seed=5)
    rng = np.random.default_rng(11)
    base = _problem(o, A)
    chi = rng.uniform(-1.2, 1.2, base.n_row)
    prob = _problem(o, A, par_angle=chi)
    offs = rng.normal(0.0, 30 * ARCSEC, size=prob.offsets_shape())
    vobs = o.predict(prob, offs + rng.normal(0.0, 20 * ARCSEC, offs.shape))
    w = rng.uniform(0.5, 2.0, size=vobs.shape)
    acc = o.gradient(prob, offs, vobs, w)

    def chi2(of):
        return float((w * np.abs(vobs - o.predict(prob, of)) ** 2).sum())

    h = 0.01 * ARCSEC
    for s, pol, ant, ax in [(0, 0, 1, 0), (0, 1, 2, 1), (1, 0, 3, 1), (1, 1, 0, 0)]:
        op, om = offs.copy(), offs.copy()
        op[s, pol, ant, ax] += h
        om[s, pol, ant, ax] -= h
        fd = (chi2(op) - chi2(om)) / (2 * h)
        g = acc[s, pol, ant, 1 + ax]
        assert abs(-0.5 * fd - g) <= 1e-6 * abs(g) + 1e-9, (s, pol, ant, ax, fd, g)
    src_l, src_m = np.append(prob.src_l, 0.005), np.append(prob.src_m, -0.007)
    flux = np.append(prob.src_flux, 0.0)

    def with_flux(fl):
        return o.Problem(src_l, src_m, fl, prob.n_ant, prob.ant1, prob.ant2, prob.uv_m, prob.int_row_ptr,
                         prob.freq_hz, n_pol=2, squint_frac=0.03, par_angle=chi, illum=2, aperture=A)

    g = o.image_gradient(with_flux(flux), offs, vobs, w, src_l, src_m)
    hf = 1e-3
    for k in range(flux.size):
        fp, fm = flux.copy(), flux.copy()
        fp[k] += hf
        fm[k] -= hf
        c2 = [float((w * np.abs(vobs - o.predict(with_flux(x), offs)) ** 2).sum()) for x in (fp, fm)]
        fd = (c2[0] - c2[1]) / (2 * hf)
        assert abs(fd - g[k]) <= 1e-8 * max(abs(fd), 1e-6), (k, fd, g[k])


def test_aperture_must_be_even(o):
    A = synth.measured_aperture(seed=6)
    A[3, 5] += 0.1  # its mirror cell (n-4, n-6) keeps the old value
    prob = _problem(o, A)
    with pytest.raises(RuntimeError):
        o.predict(prob, np.zeros(prob.offsets_shape()))


def test_generator_aperture_is_even_and_not_circular(o):
    """The synthetic aperture is even (so its pattern is real) and its feed-leg
    shadows make the pattern differ between directions at equal distance."""
    A = synth.measured_aperture(seed=7)
    assert np.array_equal(A, A[::-1, ::-1])
    D, f = 25.0, 1.4e9
    lam = C_LIGHT / f
    d = 1.2 * lam / D
    e = [o.efp_aperture(A, D, f, d * math.cos(t), d * math.sin(t))[0] for t in np.linspace(0, math.pi, 9)]
    assert max(e) - min(e) > 1e-3
