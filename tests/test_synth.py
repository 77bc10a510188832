"""Geometry of the synthetic workloads: the (u, v, w) of every row is the
local east-north baseline rotated into the frame of the phase centre, so its
length is the baseline's; towards the celestial pole w is the baseline's
polar component north cos(lat), zero for an east-west baseline."""
import numpy as np

from paper_1709_08681_amd import synth


def test_uvw_is_a_rotation_of_the_baseline():
    for k in (1, 2):
        obs = synth.make_config(k)
        e = obs.ant_pos[obs.ant2, 0] - obs.ant_pos[obs.ant1, 0]
        n = obs.ant_pos[obs.ant2, 1] - obs.ant_pos[obs.ant1, 1]
        b2 = obs.uv_m[:, 0] ** 2 + obs.uv_m[:, 1] ** 2 + obs.w_m ** 2
        np.testing.assert_allclose(b2, e * e + n * n, rtol=1e-12, atol=1e-6)


def test_w_vanishes_for_east_west_baselines_towards_the_pole():
    wl = synth.workload(1, n_ant=6, n_time=9, dec_deg=90.0)
    obs = synth.make_observation(wl, 3)
    # source at the celestial pole: w = Z = north cos(lat), independent of time
    n = obs.ant_pos[obs.ant2, 1] - obs.ant_pos[obs.ant1, 1]
    np.testing.assert_allclose(obs.w_m, n * np.cos(np.radians(wl.lat_deg)), rtol=1e-12, atol=1e-9)
