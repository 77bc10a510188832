"""Float32 against float64 accumulation of the per-antenna sums on the large
workload (Eq. DCHIDD and the 2 x 2 normal matrix, summed over every baseline
of an antenna).

The GPU path forms each visibility's terms w Re(conj(x) y) in float32 and adds
them to float64 running sums.  This test reproduces that on the CPU from the
oracle's per-visibility model and derivatives, and reports what float32
running sums would have cost instead: the relative error of chi^2, g and H per
antenna, and the offset step that the damped update (Algorithm 1) takes from
them.  It runs on a subset of the large workload (32 antennas, one solution
interval, 16 channels, both polarisations).
"""
import math

import numpy as np
import pytest

from paper_1709_08681_amd import synth

ARCSEC = math.pi / 180 / 3600


def per_vis_terms(obs, vm, dv, vobs, w):
    """Terms [n_row, n_chan, n_pol, 2 ends, 6] of the per-antenna sums, in
    float64: chi, g_l, g_m, H_ll, H_lm, H_mm = w Re(conj(x) y) for (x, y) =
    (R,R) (R,dl) (R,dm) (dl,dl) (dl,dm) (dm,dm), R = V^Obs - V^M."""
    r = vobs - vm
    out = np.empty(vm.shape + (2, 6))
    for end in range(2):
        dl, dm = dv[..., 2 * end], dv[..., 2 * end + 1]
        pairs = [(r, r), (r, dl), (r, dm), (dl, dl), (dl, dm), (dm, dm)]
        for k, (x, y) in enumerate(pairs):
            out[..., end, k] = w * (x.real * y.real + x.imag * y.imag)
    return out


def accumulate(obs, terms, dtype):
    """Sequential sums per (interval, pol, antenna) in rows-then-channels
    order, with running sums of the given dtype."""
    n_int, n_pol, n_ant = obs.n_int, obs.n_pol, obs.n_ant
    acc = np.zeros((n_int, n_pol, n_ant, 6))
    for it in range(n_int):
        r0, r1 = obs.int_row_ptr[it], obs.int_row_ptr[it + 1]
        for p in range(n_pol):
            for end, ants in ((0, obs.ant1), (1, obs.ant2)):
                for a in range(n_ant):
                    rows = np.nonzero(ants[r0:r1] == a)[0] + r0
                    if rows.size == 0:
                        continue
                    t = terms[rows, :, p, end, :].reshape(-1, 6).astype(dtype)
                    part = np.cumsum(t, axis=0, dtype=dtype)[-1]
                    # the two ends of an antenna's baselines go to one sum
                    acc[it, p, a] = (acc[it, p, a].astype(dtype) + part).astype(np.float64)
    return acc


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def large_subset():
    import oracle
    full = synth.make_config(5)
    nt = full.wl.interval_lengths[0]
    obs = full.subset(ants=range(32), times=range(nt), chans=range(0, 256, 16))
    prob = oracle.Problem.from_observation(obs)
    v_true = oracle.predict(prob, obs.offsets_true)
    noise, w = synth.noise(v_true, 100.0, 5)
    return obs, prob, v_true + noise, w


@pytest.mark.parametrize("where", ["start", "truth"])
def test_float32_against_float64_accumulation(large_subset, where):
    """At a start 5 arcsec (rms) from the true offsets, and at the true
    offsets, where only the noise drives the gradient."""
    import oracle
    obs, prob, vobs, w = large_subset
    at = synth.perturbed_offsets(obs, 5.0, 6) if where == "start" else obs.offsets_true
    vm, dv = oracle.predict(prob, at, want_grad=True)
    wv = np.full(vm.shape, w)
    terms = per_vis_terms(obs, vm, dv, vobs, wv)
    # the term definitions reproduce the oracle's own float64 sums
    ref = oracle.gradient(prob, at, vobs, w)
    exact = accumulate(obs, terms, np.float64)
    assert rel(exact, ref) <= 1e-12
    # float32 terms into float64 sums (the GPU's arrangement)
    t32 = terms.astype(np.float32).astype(np.float64)
    acc64 = accumulate(obs, t32, np.float64)
    acc32 = accumulate(obs, t32, np.float32)
    e64 = [rel(acc64[..., k], ref[..., k]) for k in range(6)]
    e32 = [rel(acc32[..., k], ref[..., k]) for k in range(6)]
    step64, _, _ = oracle.solve_step(acc64, 0.5, at)
    step32, _, _ = oracle.solve_step(acc32, 0.5, at)
    stepref, _, _ = oracle.solve_step(ref, 0.5, at)
    d64 = float(np.abs(step64 - stepref).max() / ARCSEC)
    d32 = float(np.abs(step32 - stepref).max() / ARCSEC)
    n_terms = int(np.bincount(np.concatenate([obs.ant1, obs.ant2])).max()) * obs.n_chan
    print(f"\n{where}: terms per antenna sum {n_terms}")
    print("float64 sums, rel. error chi g_l g_m H_ll H_lm H_mm:", " ".join(f"{e:.1e}" for e in e64))
    print("float32 sums, rel. error chi g_l g_m H_ll H_lm H_mm:", " ".join(f"{e:.1e}" for e in e32))
    print(f"offset step difference: float64 sums {d64:.2e} arcsec, float32 sums {d32:.2e} arcsec")
    # float32 terms summed in float64 stay within the gradient tolerance
    assert max(e64) <= 1e-6
    assert d64 <= 1e-4
    # float32 running sums lose accuracy against them
    assert max(e32) > max(e64)
