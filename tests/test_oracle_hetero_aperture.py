"""Pins of the oracle's heterogeneous array: each antenna with its own
measured aperture (Sec. 3 extends the measurement equation to arrays whose
antennas differ; a baseline then carries E_i of antenna i's illumination and
E_j of antenna j's).

The pins hold without retyping the measurement equation:
- a stack of identical apertures under any assignment is the homogeneous
  array, exactly;
- for a one-source sky the visibility factors into one pattern per antenna,
  so exchanging the two antennas' apertures and multiplying gives the
  product of the two homogeneous arrays' visibilities (a pattern taken from
  the wrong antenna breaks it);
- relabelling the antennas, with their offsets and apertures, changes
  nothing;
- the derivatives and the sums match central differences of the
  prediction and of chi^2 on a mixed array, in the sky and the mount frame.
"""
import math

import numpy as np
import pytest

from paper_1709_08681_amd import synth

ARCSEC = math.pi / 180 / 3600


@pytest.fixture(scope="module")
def o():
    import oracle
    return oracle


def _apertures():
    """Three different illuminations: the blocked, four-legged stand-in, a
    three-legged one with a larger blockage and rotated legs, and an
    unblocked, more strongly tapered dish."""
    return np.stack([synth.measured_aperture(seed=21),
                     synth.measured_aperture(seed=22, blockage_frac=0.15, n_legs=3, leg_angle_deg=10.0),
                     synth.measured_aperture(seed=23, blockage_frac=0.0, n_legs=0, edge_taper=0.1)])


def _problem(o, stack, ant_ap, n_ant=5, n_time=3, seed=7, src=None, par_angle=None, squint=0.03, n_pol=2):
    rng = np.random.default_rng(seed)
    i, j = np.triu_indices(n_ant, 1)
    ant1, ant2 = np.tile(i, n_time), np.tile(j, n_time)
    uv = rng.uniform(-2500.0, 2500.0, size=(ant1.size, 2))
    if src is None:
        sl, sm = rng.uniform(-0.012, 0.012, 6), rng.uniform(-0.012, 0.012, 6)
        flux = rng.uniform(0.2, 1.5, 6)
    else:
        sl, sm, flux = src
    pa = None if par_angle is None else rng.uniform(-1.2, 1.2, ant1.size)
    ptr = [0, i.size * (n_time // 2 + 1), ant1.size]
    return o.Problem(sl, sm, flux, n_ant, ant1, ant2, uv, ptr, [1.2e9, 1.7e9], n_pol=n_pol,
                     squint_frac=squint, par_angle=pa, illum=2, aperture=stack,
                     ant_aperture=None if ant_ap is None else np.asarray(ant_ap, np.int32))


def _offsets(prob, seed=8, sigma=40.0):
    return np.random.default_rng(seed).normal(0.0, sigma * ARCSEC, size=prob.offsets_shape())


def test_identical_stack_is_the_homogeneous_array(o):
    A = _apertures()[0]
    hom = _problem(o, A, None)
    het = _problem(o, np.stack([A, A, A]), [2, 0, 1, 1, 2])
    offs = _offsets(hom)
    v = o.predict(hom, offs)
    assert np.array_equal(o.predict(het, offs), v)
    vobs = o.predict(hom, offs + _offsets(hom, 9, 20.0))
    assert np.array_equal(o.gradient(het, offs, vobs, 1.0), o.gradient(hom, offs, vobs, 1.0))


@pytest.mark.parametrize("mount", [False, True])
def test_one_source_visibility_factors_per_antenna(o, mount):
    """One source: V(i: A, j: B) V(i: B, j: A) = V(all A) V(all B) on every
    baseline, row, channel and polarisation (each side a product of one
    pattern per antenna and the same fringe)."""
    stack = _apertures()
    src = (np.array([0.004]), np.array([-0.003]), np.array([1.3]))
    n_ant = 4
    A, B = stack[0], stack[1]
    pa = True if mount else None
    all_a = _problem(o, A, None, n_ant=n_ant, src=src, par_angle=pa)
    all_b = _problem(o, B, None, n_ant=n_ant, src=src, par_angle=pa)
    # antennas 0, 2 take A and 1, 3 take B; then the reverse
    ab = _problem(o, np.stack([A, B]), [0, 1, 0, 1], n_ant=n_ant, src=src, par_angle=pa)
    ba = _problem(o, np.stack([A, B]), [1, 0, 1, 0], n_ant=n_ant, src=src, par_angle=pa)
    offs = _offsets(all_a)
    lhs = o.predict(ab, offs) * o.predict(ba, offs)
    rhs = o.predict(all_a, offs) * o.predict(all_b, offs)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-15 * np.abs(rhs).max())
    # the mixed baselines differ from both homogeneous arrays
    mixed = all_a.ant1 % 2 != all_a.ant2 % 2
    assert np.abs(o.predict(ab, offs) - o.predict(all_a, offs))[mixed].max() > 1e-3 * np.abs(rhs).max() ** 0.5


def test_relabelling_antennas_changes_nothing(o):
    stack = _apertures()
    ant_ap = np.array([0, 2, 1, 2, 0])
    prob = _problem(o, stack, ant_ap)
    offs = _offsets(prob)
    v = o.predict(prob, offs)
    perm = np.array([3, 0, 4, 1, 2])  # new label of old antenna a is perm[a]
    inv = np.argsort(perm)
    a1, a2 = perm[prob.ant1], perm[prob.ant2]
    # keep ant1 < ant2: a swapped pair is the conjugate baseline
    swap = a1 > a2
    uv = np.where(swap[:, None], -prob.uv_m, prob.uv_m)
    rel = o.Problem(prob.src_l, prob.src_m, prob.src_flux, prob.n_ant, np.where(swap, a2, a1),
                    np.where(swap, a1, a2), uv, prob.int_row_ptr, prob.freq_hz, n_pol=2, squint_frac=0.03,
                    illum=2, aperture=stack, ant_aperture=ant_ap[inv])
    v2 = o.predict(rel, offs[:, :, inv, :])
    v2 = np.where(swap[:, None, None], np.conj(v2), v2)
    np.testing.assert_allclose(v2, v, rtol=1e-12, atol=1e-14 * np.abs(v).max())


@pytest.mark.parametrize("mount", [False, True])
def test_mixed_array_sums_match_chi2_differences(o, mount):
    stack = _apertures()
    prob = _problem(o, stack, [1, 0, 2, 0, 1], par_angle=True if mount else None)
    offs = _offsets(prob)
    vobs = o.predict(prob, offs + _offsets(prob, 10, 20.0))
    w = np.random.default_rng(12).uniform(0.5, 2.0, size=vobs.shape)
    acc = o.gradient(prob, offs, vobs, w)

    def chi2(of):
        return float((w * np.abs(vobs - o.predict(prob, of)) ** 2).sum())

    h = 0.01 * ARCSEC
    for s, pol, ant, ax in [(0, 0, 0, 0), (0, 1, 2, 1), (1, 0, 4, 0), (1, 1, 1, 1), (0, 0, 3, 1)]:
        op, om = offs.copy(), offs.copy()
        op[s, pol, ant, ax] += h
        om[s, pol, ant, ax] -= h
        fd = (chi2(op) - chi2(om)) / (2 * h)
        g = acc[s, pol, ant, 1 + ax]
        assert abs(-0.5 * fd - g) <= 1e-6 * abs(g) + 1e-9, (s, pol, ant, ax, fd, g)


@pytest.mark.parametrize("mount", [False, True])
def test_mixed_array_derivatives_match_central_differences(o, mount):
    """dV/dp of both ends against central differences (h = 0.01 arcsec) of
    the prediction on a mixed array: a derivative taken from the other
    antenna's aperture would break it."""
    stack = _apertures()
    prob = _problem(o, stack, [2, 1, 0, 1, 2], par_angle=True if mount else None)
    offs = _offsets(prob)
    _, dv = o.predict(prob, offs, want_grad=True)
    h = 0.01 * ARCSEC
    rows = slice(0, prob.int_row_ptr[1])  # the first interval's rows
    for ant in range(prob.n_ant):
        for pol in range(2):
            for ax in range(2):
                op, om = offs.copy(), offs.copy()
                op[0, pol, ant, ax] += h
                om[0, pol, ant, ax] -= h
                fd = ((o.predict(prob, op) - o.predict(prob, om))[:, :, pol] / (2 * h))[rows]
                an = np.zeros_like(fd)
                an += np.where((prob.ant1[rows] == ant)[:, None], dv[rows, :, pol, 0 + ax], 0)
                an += np.where((prob.ant2[rows] == ant)[:, None], dv[rows, :, pol, 2 + ax], 0)
                err = np.linalg.norm(fd - an) / np.linalg.norm(an)
                assert err < 1e-6, (ant, pol, ax, err)


def test_bad_aperture_index_is_refused(o):
    stack = _apertures()[:2]
    prob = _problem(o, stack, [0, 1, 2, 0, 1])
    with pytest.raises(Exception):
        o.predict(prob, _offsets(prob))
