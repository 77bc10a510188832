"""Error handling and degenerate data through the C ABI on the GPU: the plan
rejects malformed observations with PSC_E_ARG, calls made in the wrong order
return PSC_E_STATE, a non-finite weight leaves its antennas unchanged and
flagged, an all-flagged interval yields zero sums, and an observation with no
rows runs every entry point."""
import math

import numpy as np
import pytest

import oracle
from paper_1709_08681_amd import synth

pytestmark = pytest.mark.gpu
ARCSEC = math.pi / 180 / 3600


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_08681_amd import psc
    psc.load()
    return torch


def _desc(torch, obs, **bad):
    """Device arrays and an ObsDesc for `obs`, with fields replaced by `bad`."""
    from paper_1709_08681_amd import psc
    arrs = dict(int_row_ptr=np.asarray(obs.int_row_ptr, np.int64), ant1=np.asarray(obs.ant1, np.int32),
                ant2=np.asarray(obs.ant2, np.int32), uv_m=np.asarray(obs.uv_m, np.float64),
                freq_hz=np.asarray(obs.freq_hz, np.float64))
    arrs.update(bad)
    dev = {k: torch.as_tensor(np.ascontiguousarray(v), device="cuda") for k, v in arrs.items()}
    d = psc.ObsDesc(obs.n_ant, len(arrs["freq_hz"]), obs.n_pol, obs.n_int, len(arrs["ant1"]),
                    dev["int_row_ptr"].data_ptr(), dev["ant1"].data_ptr(), dev["ant2"].data_ptr(),
                    dev["uv_m"].data_ptr(), dev["freq_hz"].data_ptr())
    return d, dev


@pytest.mark.parametrize("case", ["ant_order", "ant_range", "row_ptr", "uv_nan", "freq", "support"])
def test_obs_create_rejects_malformed_plans(torch_dev, case):
    torch = torch_dev
    from paper_1709_08681_amd import psc
    obs = synth.make_config(1)
    ctx = psc.psc_create(psc.config_for(obs))
    try:
        a1, a2 = obs.ant1.copy(), obs.ant2.copy()
        bad = {}
        if case == "ant_order":
            a1[3], a2[3] = a2[3], a1[3]
            bad = dict(ant1=a1, ant2=a2)
        elif case == "ant_range":
            a2[5] = obs.n_ant
            bad = dict(ant2=a2)
        elif case == "row_ptr":
            bad = dict(int_row_ptr=np.array([0, obs.n_row + 1], np.int64))
        elif case == "uv_nan":
            uv = obs.uv_m.copy()
            uv[7, 1] = np.nan
            bad = dict(uv_m=uv)
        elif case == "freq":
            bad = dict(freq_hz=np.array([-1.4e9]))
        elif case == "support":
            # at 20 GHz both 25 m apertures no longer fit the 16-cell kernel
            bad = dict(freq_hz=np.array([2.0e10]))
        d, keep = _desc(torch, obs, **bad)
        with pytest.raises(psc.PscError) as ei:
            psc.psc_obs_create(ctx, d)
        assert ei.value.status == psc.PSC_E_ARG
        assert psc.load().psc_last_error(ctx)
    finally:
        psc.psc_destroy(ctx)


def test_calls_before_model_are_state_errors(torch_dev):
    torch = torch_dev
    from paper_1709_08681_amd import psc
    obs = synth.make_config(1)
    ctx = psc.psc_create(psc.config_for(obs))
    try:
        d, keep = _desc(torch, obs)
        h = psc.psc_obs_create(ctx, d)
        off = torch.zeros((obs.n_int, obs.n_pol, obs.n_ant, 2), dtype=torch.float64, device="cuda")
        out = torch.empty((obs.n_row, obs.n_chan, obs.n_pol), dtype=torch.complex64, device="cuda")
        with pytest.raises(psc.PscError) as ei:
            psc.psc_predict(ctx, h, off, out)
        assert ei.value.status == psc.PSC_E_STATE
        psc.psc_obs_destroy(h)
    finally:
        psc.psc_destroy(ctx)


def test_nonfinite_weight_flags_its_antennas(torch_dev):
    """A NaN weight makes both antennas' sums non-finite: the update leaves
    them unchanged and flags them, as the oracle's update does."""
    torch = torch_dev
    from paper_1709_08681_amd.psc import Session
    obs = synth.make_config(1)
    prob = oracle.Problem.from_observation(obs)
    s = Session(obs, device=0)
    try:
        v = oracle.predict(prob, obs.offsets_true)
        w = np.ones(s.vis_shape)
        w[4, 0, 0] = np.nan
        i, j = int(obs.ant1[4]), int(obs.ant2[4])
        start = synth.perturbed_offsets(obs, 20.0, 31)
        acc = s.gradient(s.offsets(start), torch.as_tensor(v.astype(np.complex64), device=s.dev),
                         torch.as_tensor(w.astype(np.float32), device=s.dev))
        a = acc.cpu().numpy()
        assert not np.isfinite(a[0, 0, i]).all() and not np.isfinite(a[0, 0, j]).all()
        off = s.offsets(start)
        nu, mx = s.solve_step(acc, 0.5, off)
        ref_off, ref_nu, _ = oracle.solve_step(a, 0.5, start)
        assert np.array_equal(nu.cpu().numpy(), ref_nu)
        assert nu.cpu().numpy()[0, 0, i] == 1 and nu.cpu().numpy()[0, 0, j] == 1
        o = off.cpu().numpy()
        assert np.array_equal(o[0, 0, i], start[0, 0, i]) and np.array_equal(o[0, 0, j], start[0, 0, j])
        assert np.abs(o - ref_off).max() / ARCSEC <= 1e-6
    finally:
        s.close()


def test_all_flagged_interval_and_empty_observation(torch_dev):
    torch = torch_dev
    from paper_1709_08681_amd import psc
    from paper_1709_08681_amd.psc import Session
    lengths = [4, 3]
    wl = synth.workload(1, n_ant=5, n_time=sum(lengths), interval_lengths=lengths, n_src=3)
    obs = synth.make_observation(wl, 41)
    prob = oracle.Problem.from_observation(obs)
    s = Session(obs, device=0)
    try:
        v = oracle.predict(prob, obs.offsets_true)
        w = np.ones(s.vis_shape)
        w[obs.int_row_ptr[1]:] = 0.0  # every sample of interval 1 flagged
        start = synth.perturbed_offsets(obs, 20.0, 32)
        acc = s.gradient(s.offsets(start), torch.as_tensor(v.astype(np.complex64), device=s.dev),
                         torch.as_tensor(w.astype(np.float32), device=s.dev)).cpu().numpy()
        assert np.all(acc[1] == 0.0) and np.all(acc[0, :, :, 3] > 0)
        off = s.offsets(start)
        nu, _ = s.solve_step(torch.as_tensor(acc, device=s.dev), 0.5, off)
        assert np.all(nu.cpu().numpy()[1] == 1)
        assert np.array_equal(off.cpu().numpy()[1], start[1])
    finally:
        s.close()
    # no rows at all: every entry point runs and returns zeros
    empty = obs.subset(times=[])
    s = Session(empty, device=0)
    try:
        assert s.info()[2] == 0
        z = s.predict(np.zeros(s.off_shape))
        assert z.numel() == 0
        acc = s.gradient(s.offsets(np.zeros(s.off_shape)),
                         torch.zeros(s.vis_shape, dtype=torch.complex64, device=s.dev),
                         torch.zeros(s.vis_shape, dtype=torch.float32, device=s.dev))
        assert torch.count_nonzero(acc) == 0
        off = s.offsets(np.zeros(s.off_shape))
        its = s.solve(torch.zeros(s.vis_shape, dtype=torch.complex64, device=s.dev),
                      torch.zeros(s.vis_shape, dtype=torch.float32, device=s.dev), off,
                      gain=0.5, n_max=3, tol_rad=1e-3 * ARCSEC, form=psc.SOLVE_GRAPH)
        assert torch.count_nonzero(off) == 0
        assert its.shape[0] == empty.n_int
        vz = torch.zeros(s.vis_shape, dtype=torch.complex64, device=s.dev)
        wz = torch.zeros(s.vis_shape, dtype=torch.float32, device=s.dev)
        img = s.image_gradient(off, vz, wz)
        assert torch.count_nonzero(img) == 0
        # beam scales on no rows: zero sums, no step, scales unchanged
        s.set_beam_scale(np.full(s.off_shape[:3], 1.02))
        sacc = s.scale_gradient(off, vz, wz)
        assert torch.count_nonzero(sacc) == 0
        nu, mx = s.scale_step(sacc, 0.5)
        assert torch.all(nu == 1) and torch.count_nonzero(mx) == 0
        sits = s.solve_beam_scale(off, vz, wz, n_max=3)
        assert sits.shape[0] == empty.n_int
        assert torch.all(s.beam_scale() == 1.02)
        assert torch.count_nonzero(s.image_gradient(off, vz, wz)) == 0
        s.set_beam_scale(None)
    finally:
        s.close()
    # a measured aperture on no rows
    s = Session(empty, device=0, aperture=synth.measured_aperture(n=16, seed=1), mount_frame=True)
    try:
        off = s.offsets(np.zeros(s.off_shape))
        vz = torch.zeros(s.vis_shape, dtype=torch.complex64, device=s.dev)
        wz = torch.zeros(s.vis_shape, dtype=torch.float32, device=s.dev)
        assert s.predict(off).numel() == 0
        assert torch.count_nonzero(s.gradient(off, vz, wz)) == 0
        assert torch.count_nonzero(s.image_gradient(off, vz, wz)) == 0
    finally:
        s.close()
