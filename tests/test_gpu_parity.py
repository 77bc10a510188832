"""GPU parity: libpsc (HIP, gfx950) against the FP64 direct-summation oracle.

Tolerances (per result):
  visibilities  ||dV|| / ||V||        <= 1e-5
  chi, g, H     ||d acc|| / ||acc||   <= 1e-4 (at perturbed offsets, |g| >> 0)
  offsets       max |p_gpu - p_oracle| <= 0.1 arcsec after the same iterations
Integer/plan work (iteration counts, flags) must match exactly.
"""
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


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def elem_err(a, b):
    """Largest single-visibility error relative to the rms visibility of the
    set: max_k |a_k - b_k| / rms |b|."""
    a, b = np.asarray(a).ravel(), np.asarray(b).ravel()
    return float(np.abs(a - b).max() / np.sqrt(np.mean(np.abs(b) ** 2)))


def per_antenna_err(acc, ref):
    """Worst per-antenna relative error of each kind of sum: chi, the
    gradient (g_l, g_m) and the normal matrix (H_ll, H_lm, H_mm), each
    ||d||/||ref|| over one (interval, pol, antenna) entry; entries whose sums
    are zero on the oracle side (no data) must be zero on the GPU side too."""
    acc, ref = np.asarray(acc).reshape(-1, 6), np.asarray(ref).reshape(-1, 6)
    out = []
    for cols in ((0,), (1, 2), (3, 4, 5)):
        d = np.linalg.norm(acc[:, cols] - ref[:, cols], axis=1)
        n = np.linalg.norm(ref[:, cols], axis=1)
        live = n > 0
        assert np.all(d[~live] == 0.0)
        out.append(float((d[live] / n[live]).max()) if live.any() else 0.0)
    return out


# Per-element bounds.  Each visibility is a float32 sum of S^2 taps (or, in
# the window form, an S-point transform pair and an M^2 image-sample sum),
# whose rounding error is of order sqrt(terms) * 2^-24 of the sum of the
# terms' magnitudes; with the taper's kernel that sum stays within a few
# times rms |V|, so one visibility's error stays near 1e-6 of rms |V|.  The
# bound below is ten times the set-wide tolerance: a single visibility wrong
# at 1e-4 of rms |V| fails it, which the norm over millions would hide.
ELEM_VIS_TOL = 1e-4
# per (interval, pol, antenna) entry: the set-wide sum tolerance, applied to
# every antenna alone
ANT_SUM_TOL = 1e-4


def session(obs, **kw):
    from paper_1709_08681_amd.psc import Session
    return Session(obs, device=0, **kw)


def c64(torch, s, a):
    return torch.as_tensor(np.ascontiguousarray(a).astype(np.complex64), device=s.dev)


def f32(torch, s, a, shape):
    return torch.as_tensor(np.ascontiguousarray(np.broadcast_to(a, shape)).astype(np.float32),
                           device=s.dev)


# ---------------------------------------------------------------------------
# tiny array (config 1), every result
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def cfg1(torch_dev):
    obs = synth.make_config(1)
    prob = oracle.Problem.from_observation(obs)
    s = session(obs)
    yield obs, prob, s
    s.close()


def test_predict_cfg1(torch_dev, cfg1):
    obs, prob, s = cfg1
    print("case: predict cfg1", flush=True)
    for seed in (1, 2):
        off = synth.perturbed_offsets(obs, 20.0, seed)
        ref = oracle.predict(prob, off)
        got = s.predict(off).cpu().numpy()
        assert rel(got, ref) <= 1e-5
        assert np.abs(got - ref).max() / np.abs(ref).max() <= 1e-5


def test_gradient_cfg1(torch_dev, cfg1):
    torch = torch_dev
    obs, prob, s = cfg1
    print("case: gradient cfg1", flush=True)
    v = oracle.predict(prob, obs.offsets_true)
    nz, w = synth.noise(v, 100.0, 3)
    vo = v + nz
    start = synth.perturbed_offsets(obs, 20.0, 4)
    ref, vm_ref = oracle.gradient(prob, start, vo, w, want_model=True)
    acc, vm = s.gradient(s.offsets(start), c64(torch, s, vo), f32(torch, s, w, s.vis_shape),
                         want_model=True)
    acc = acc.cpu().numpy()
    assert rel(vm.cpu().numpy(), vm_ref) <= 1e-5
    for k, name in enumerate(["chi", "g_l", "g_m", "H_ll", "H_lm", "H_mm"]):
        assert rel(acc[..., k], ref[..., k]) <= 1e-4, name


def test_gradient_is_deterministic(torch_dev, cfg1):
    torch = torch_dev
    obs, prob, s = cfg1
    v = s.predict(obs.offsets_true)
    w = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
    off = s.offsets(synth.perturbed_offsets(obs, 20.0, 5))
    a1 = s.gradient(off, v, w)
    a2 = s.gradient(off, v, w)
    assert torch.equal(a1, a2)


def test_hermitian_symmetry_gpu(torch_dev, cfg1):
    """V_ji(-u) = conj V_ij(u): rows reversed and negated give conjugates."""
    obs, prob, s = cfg1
    from paper_1709_08681_amd.psc import Session
    flip = synth.Observation(obs.wl, obs.ant_pos, obs.ant1, obs.ant2, obs.time_idx, -obs.uv_m,
                             obs.int_row_ptr, obs.freq_hz, obs.grid_n, obs.cell_rad, obs.src_pix,
                             obs.src_flux, obs.offsets_true)
    # a baseline with its antennas swapped is the same baseline with uv negated
    # and the model conjugated; with equal offsets at both ends the products
    # E_i E_j are symmetric, so V(-u) must be conj V(u).
    off = np.repeat(obs.offsets_true[:, :, :1, :], obs.n_ant, axis=2)
    s2 = Session(flip, device=0)
    try:
        a = s.predict(off).cpu().numpy()
        b = s2.predict(off).cpu().numpy()
    finally:
        s2.close()
    assert rel(b, np.conj(a)) <= 1e-5


def test_vjp_matches_oracle(torch_dev, cfg1):
    torch = torch_dev
    obs, prob, s = cfg1
    print("case: vjp cfg1", flush=True)
    off = synth.perturbed_offsets(obs, 20.0, 6)
    rng = np.random.default_rng(7)
    G = rng.normal(size=s.vis_shape) + 1j * rng.normal(size=s.vis_shape)
    G = G.astype(np.complex64)
    _, dv = oracle.predict(prob, off, want_grad=True)
    ref = np.zeros(s.off_shape)
    for r in range(obs.n_row):
        i, j = obs.ant1[r], obs.ant2[r]
        for c in range(obs.n_chan):
            for p in range(obs.n_pol):
                g = G[r, c, p].astype(np.complex128)
                for ax in range(2):
                    ref[0, p, i, ax] += (np.conj(g) * dv[r, c, p, ax]).real
                    ref[0, p, j, ax] += (np.conj(g) * dv[r, c, p, 2 + ax]).real
    got = s.vjp(s.offsets(off), torch.as_tensor(G, device=s.dev)).cpu().numpy()
    assert rel(got, ref) <= 1e-4


def test_autograd_chi2_gradient(torch_dev, cfg1):
    """d chi^2 / d p through the autograd Function equals -2 g of psc_gradient
    and the oracle's."""
    torch = torch_dev
    from paper_1709_08681_amd.autograd import predict
    obs, prob, s = cfg1
    v = oracle.predict(prob, obs.offsets_true)
    vo = c64(torch, s, v)
    start = synth.perturbed_offsets(obs, 20.0, 8)
    off = s.offsets(start).requires_grad_(True)
    model = predict(off, s)
    loss = ((vo - model).abs() ** 2).sum()
    loss.backward()
    ref = oracle.gradient(prob, start, v, 1.0)
    assert rel(off.grad.cpu().numpy(), -2 * ref[..., 1:3]) <= 1e-4


def test_solve_step_matches_oracle(torch_dev, cfg1):
    torch = torch_dev
    obs, prob, s = cfg1
    rng = np.random.default_rng(9)
    acc = np.zeros((3, 2, 5, 6))
    acc[..., 1:3] = rng.normal(size=(3, 2, 5, 2))
    A = rng.normal(size=(3, 2, 5, 2, 2))
    H = A @ np.swapaxes(A, -1, -2) + 0.1 * np.eye(2)
    acc[..., 3], acc[..., 4], acc[..., 5] = H[..., 0, 0], H[..., 0, 1], H[..., 1, 1]
    acc[1, 0, 2, 3:] = 0.0  # no data
    acc[2, 1, 4, 3:] = [1.0, 1.0, 1.0]  # singular
    off0 = rng.normal(size=(3, 2, 5, 2)) * 1e-4
    from paper_1709_08681_amd import psc
    for mu in (0.0, 0.3, 1e6):
        ref, nu_ref, mx_ref = oracle.solve_step(acc, 0.5, off0, mu=mu)
        offs = torch.as_tensor(off0, device=s.dev)
        nu = torch.empty((3, 2, 5), dtype=torch.int32, device=s.dev)
        mx = torch.empty(3, dtype=torch.float64, device=s.dev)
        psc.psc_solve_step(s.ctx, 3, 2, 5, torch.as_tensor(acc, device=s.dev), 0.5, mu, offs, nu, mx)
        np.testing.assert_allclose(offs.cpu().numpy(), ref, rtol=1e-12, atol=1e-18)
        assert np.array_equal(nu.cpu().numpy(), nu_ref)
        np.testing.assert_allclose(mx.cpu().numpy(), mx_ref, rtol=1e-12)


def test_solve_forms_match_oracle(torch_dev, cfg1):
    """Algorithm 1 at SNR 100: GPU offsets within 0.1 arcsec of the oracle's
    after the same iterations, and the three execution forms bit-identical."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    obs, prob, s = cfg1
    print("case: solve cfg1", flush=True)
    v = oracle.predict(prob, obs.offsets_true)
    nz, w = synth.noise(v, 100.0, 10)
    vo = v + nz
    start = synth.perturbed_offsets(obs, 20.0, 11)
    ref, its_ref = oracle.solve(prob, vo, w, start, gain=0.5, n_max=10, tol_rad=1e-3 * ARCSEC)
    vo_d = c64(torch, s, vo)
    w_d = f32(torch, s, w, s.vis_shape)
    outs = []
    for form in (psc.SOLVE_PLAIN, psc.SOLVE_BATCHED, psc.SOLVE_GRAPH, psc.SOLVE_GRAPH):
        off = s.offsets(start)
        its = s.solve(vo_d, w_d, off, gain=0.5, n_max=10, tol_rad=1e-3 * ARCSEC, form=form)
        outs.append((off.cpu().numpy(), its.cpu().numpy()))
    # the library timed its capture and instantiation of the graph
    assert psc.psc_obs_launch_info(s.handle)["capture_ms"] > 0.0
    for o, its in outs:
        assert np.array_equal(its, its_ref)
        assert np.abs(o - ref).max() / ARCSEC <= 0.1
    for o, its in outs[1:]:
        assert np.array_equal(o, outs[0][0])


def test_recovers_injected_offsets(torch_dev, cfg1):
    torch = torch_dev
    obs, prob, s = cfg1
    v = oracle.predict(prob, obs.offsets_true)
    vo = c64(torch, s, v)
    w = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
    off = s.offsets(synth.perturbed_offsets(obs, 20.0, 12))
    s.solve(vo, w, off, gain=0.5, n_max=80, tol_rad=1e-5 * ARCSEC)
    err = np.abs(off.cpu().numpy() - obs.offsets_true).max() / ARCSEC
    assert err <= 0.05, err


# ---------------------------------------------------------------------------
# ragged intervals, two polarisations with squint, flagged data, empty interval
# ---------------------------------------------------------------------------

def test_ragged_intervals_two_pols(torch_dev):
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print("case: ragged intervals, 2 pols", flush=True)
    lengths = [3, 0, 7, 1, 5]
    wl = synth.workload(1, n_ant=7, n_time=sum(lengths), interval_lengths=lengths, n_pol=2,
                        squint_frac=0.03, freqs_hz=np.array([1.2e9, 1.45e9, 1.7e9]), n_src=5)
    obs = synth.make_observation(wl, 77)
    prob = oracle.Problem.from_observation(obs)
    s = session(obs)
    try:
        start = synth.perturbed_offsets(obs, 25.0, 13)
        ref = oracle.predict(prob, start)
        got = s.predict(start).cpu().numpy()
        assert rel(got, ref) <= 1e-5
        v = oracle.predict(prob, obs.offsets_true)
        w = np.ones(s.vis_shape)
        # flag every sample of antenna 3 in interval 2
        r0, r1 = obs.int_row_ptr[2], obs.int_row_ptr[3]
        rows = np.arange(r0, r1)
        flag = rows[(obs.ant1[rows] == 3) | (obs.ant2[rows] == 3)]
        w[flag] = 0.0
        acc_ref = oracle.gradient(prob, start, v, w)
        acc = s.gradient(s.offsets(start), c64(torch, s, v), f32(torch, s, w, s.vis_shape))
        acc = acc.cpu().numpy()
        assert rel(acc, acc_ref) <= 1e-4
        assert np.all(acc[1] == 0.0)  # empty interval
        assert np.all(acc[2, :, 3] == 0.0)  # flagged antenna
        ref_off, its_ref = oracle.solve(prob, v, w, start, gain=0.5, n_max=8, tol_rad=1e-3 * ARCSEC)
        for form in (psc.SOLVE_PLAIN, psc.SOLVE_GRAPH):
            off = s.offsets(start)
            its = s.solve(c64(torch, s, v), f32(torch, s, w, s.vis_shape), off, gain=0.5, n_max=8,
                          tol_rad=1e-3 * ARCSEC, form=form)
            assert np.array_equal(its.cpu().numpy(), its_ref)
            o = off.cpu().numpy()
            assert np.abs(o - ref_off).max() / ARCSEC <= 0.1
            assert np.array_equal(o[2, :, 3], start[2, :, 3])  # not updated
    finally:
        s.close()


# ---------------------------------------------------------------------------
# single interval at full size (config 2: 2,021,760 visibilities)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant", ["vector", "matrix_core"])
def test_cfg2_full_size_parity(torch_dev, variant):
    """Single-interval workload at full size (2,021,760 visibilities), table
    form on the vector units and on the matrix cores: every visibility and
    every per-antenna sum against the oracle, set-wide and element by
    element."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print(f"case: cfg2 full size, table form, {variant}", flush=True)
    obs = synth.make_config(2)
    prob = oracle.Problem.from_observation(obs)
    s = session(obs)
    try:
        psc.psc_set_degrid(s.handle, psc.DEGRID_VALU if variant == "vector" else psc.DEGRID_MFMA)
        start = synth.perturbed_offsets(obs, 30.0, 14)
        v_true = oracle.predict(prob, obs.offsets_true)
        ref_acc, ref_vm = oracle.gradient(prob, start, v_true, 1.0, want_model=True)
        w = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        acc, vm = s.gradient(s.offsets(start), c64(torch, s, v_true), w, want_model=True)
        vm, acc = vm.cpu().numpy(), acc.cpu().numpy()
        e_v = rel(vm, ref_vm)
        e_a = [rel(acc[..., k], ref_acc[..., k]) for k in range(6)]
        e_el, e_ant = elem_err(vm, ref_vm), per_antenna_err(acc, ref_acc)
        print(f"cfg2 {variant}: vis rel {e_v:.2e}, acc rel {max(e_a):.2e}, max element {e_el:.2e}, "
              f"per antenna {max(e_ant):.2e}", flush=True)
        assert e_v <= 1e-5
        assert max(e_a) <= 1e-4
        assert e_el <= ELEM_VIS_TOL
        assert max(e_ant) <= ANT_SUM_TOL
    finally:
        s.close()


# ---------------------------------------------------------------------------
# subsets of the batched and differentiation workloads
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant", ["vector", "window"])
def test_cfg3_subset_ragged_intervals(torch_dev, variant):
    """Batched workload (2048^2 grid, uneven intervals): 6 antennas, the first
    five intervals (45 timesteps, so 45 samples per item on average: the
    window form's two-wavefront blocks, as on the whole workload), all 16
    channels.  Prediction, gradient sums, the adjoint, and Algorithm 1 in the
    plain, batched and graph forms, in the table form and the window form."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print(f"case: cfg3 subset, {variant}", flush=True)
    full = synth.make_config(3)
    nt = sum(full.wl.interval_lengths[:5])
    obs = full.subset(ants=range(6), times=range(nt))
    prob = oracle.Problem.from_observation(obs)
    s = session(obs)
    try:
        if variant == "window":
            psc.psc_set_degrid(s.handle, psc.DEGRID_WINDOW)
            info = psc.psc_obs_launch_info(s.handle)
            assert info["degrid"] == psc.DEGRID_WINDOW
            assert 16 <= info["samples_per_item"] < 128
            assert info["window_waves"] == 2, info
        start = synth.perturbed_offsets(obs, 30.0, 15)
        v = oracle.predict(prob, obs.offsets_true)
        vp = s.predict(start).cpu().numpy()
        vp_ref = oracle.predict(prob, start)
        assert rel(vp, vp_ref) <= 1e-5 and elem_err(vp, vp_ref) <= ELEM_VIS_TOL
        ref, ref_vm = oracle.gradient(prob, start, v, 1.0, want_model=True)
        w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        acc, vm = s.gradient(s.offsets(start), c64(torch, s, v), w1, want_model=True)
        acc, vm = acc.cpu().numpy(), vm.cpu().numpy()
        assert rel(vm, ref_vm) <= 1e-5 and elem_err(vm, ref_vm) <= ELEM_VIS_TOL
        live = obs.int_row_ptr[1:] > obs.int_row_ptr[:-1]
        for k in range(6):
            assert rel(acc[live][..., k], ref[live][..., k]) <= 1e-4, k
        assert max(per_antenna_err(acc, ref)) <= ANT_SUM_TOL
        # adjoint: sum Re(conj(G) dV/dp) for a seeded cotangent
        G = np.random.default_rng(16).normal(size=s.vis_shape) + 1j * np.random.default_rng(17).normal(
            size=s.vis_shape)
        gv = s.vjp(s.offsets(start), c64(torch, s, G)).cpu().numpy()
        gv_ref = vjp_reference(obs, prob, start, G, s.off_shape)
        assert rel(gv[live], gv_ref[live]) <= 1e-4
        ref_off, its_ref = oracle.solve(prob, v, 1.0, start, gain=0.5, n_max=6, tol_rad=1e-3 * ARCSEC)
        outs = []
        for form in (psc.SOLVE_PLAIN, psc.SOLVE_BATCHED, psc.SOLVE_GRAPH):
            off = s.offsets(start)
            its = s.solve(c64(torch, s, v), w1, off, gain=0.5, n_max=6, tol_rad=1e-3 * ARCSEC,
                          form=form)
            assert np.array_equal(its.cpu().numpy(), its_ref)
            outs.append(off.cpu().numpy())
            assert np.abs(outs[-1] - ref_off).max() / ARCSEC <= 0.1
        assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    finally:
        s.close()


def test_cfg3_full_size_tuned_sampled_rows(torch_dev):
    """The whole batched workload (256 uneven intervals, 93 M visibilities)
    after the autotuner, in the launch configuration the bench times: the
    model of every 83rd timestep and the per-antenna sums with the weights
    zero elsewhere, against the oracle on those rows; then Algorithm 1 in the
    graph form over all intervals against the oracle's solve of the same
    rows (iteration counts equal, offsets within 0.1 arcsec)."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    every = 83
    print(f"case: cfg3 full size after psc_tune, every {every}th timestep", flush=True)
    obs = synth.make_config(3)
    times = np.unique(obs.time_idx)[::every]
    rows = np.nonzero(np.isin(obs.time_idx, times))[0]
    sub = obs.subset(times=times)
    prob = oracle.Problem.from_observation(sub)
    s = session(obs)
    try:
        start = synth.perturbed_offsets(obs, 30.0, 19)
        v_sub = oracle.predict(prob, obs.offsets_true)
        vobs = np.zeros(s.vis_shape, np.complex64)
        vobs[rows] = v_sub
        w = np.zeros(s.vis_shape, np.float32)
        w[rows] = 1.0
        g_vobs, g_w = c64(torch, s, vobs), f32(torch, s, w, s.vis_shape)
        del vobs, w
        off = s.offsets(start)
        psc.psc_tune(s.ctx, s.handle, off, g_vobs, g_w, 1, None)
        info = psc.psc_obs_launch_info(s.handle)
        print(f"cfg3 full: tuned degrid {info}", flush=True)
        vp = s.predict(start)[torch.as_tensor(rows, device=s.dev)].cpu().numpy()
        vp_ref = oracle.predict(prob, start)
        acc = s.gradient(off, g_vobs, g_w).cpu().numpy()
        ref = oracle.gradient(prob, start, v_sub, 1.0)
        e_v, e_el = rel(vp, vp_ref), elem_err(vp, vp_ref)
        e_a = [rel(acc[..., k], ref[..., k]) for k in range(6)]
        e_ant = per_antenna_err(acc, ref)
        print(f"cfg3 full: vis rel {e_v:.2e}, max element {e_el:.2e}, acc rel {max(e_a):.2e}, "
              f"per antenna {max(e_ant):.2e} ({len(rows)} of {obs.n_row} rows)", flush=True)
        assert e_v <= 1e-5 and e_el <= ELEM_VIS_TOL
        assert max(e_a) <= 1e-4 and max(e_ant) <= ANT_SUM_TOL
        ref_off, its_ref = oracle.solve(prob, v_sub, 1.0, start, gain=0.5, n_max=3, tol_rad=1e-3 * ARCSEC)
        its = s.solve(g_vobs, g_w, off, gain=0.5, n_max=3, tol_rad=1e-3 * ARCSEC, form=psc.SOLVE_GRAPH)
        assert np.array_equal(its.cpu().numpy(), its_ref)
        d = np.abs(off.cpu().numpy() - ref_off).max() / ARCSEC
        print(f"cfg3 full: graph solve offsets within {d:.2e} arcsec of the oracle", flush=True)
        assert d <= 0.1
    finally:
        s.close()


def test_cfg4_subset_with_diffuse_emission(torch_dev):
    """Differentiation workload (1000 sources plus a 5 arcmin Gaussian of
    ~3.7e5 pixels): 4 antennas, every 8th timestep, every 8th channel."""
    torch = torch_dev
    print("case: cfg4 subset", flush=True)
    full = synth.make_config(4)
    obs = full.subset(ants=[0, 1, 2, 3], times=range(0, 240, 8), chans=range(0, 64, 8))
    prob = oracle.Problem.from_observation(obs)
    s = session(obs)
    try:
        start = synth.perturbed_offsets(obs, 30.0, 16)
        v_true = oracle.predict(prob, obs.offsets_true)
        ref_acc, ref_vm = oracle.gradient(prob, start, v_true, 1.0, want_model=True)
        w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        acc, vm = s.gradient(s.offsets(start), c64(torch, s, v_true), w1, want_model=True)
        assert rel(vm.cpu().numpy(), ref_vm) <= 1e-5
        acc = acc.cpu().numpy()
        for k in range(6):
            assert rel(acc[..., k], ref_acc[..., k]) <= 1e-4, k
    finally:
        s.close()


def test_cfg4_subset_autograd_against_finite_differences(torch_dev):
    """Differentiation workload: the autograd backward (the adjoint kernel,
    kernels rebuilt in the backward pass) against the oracle's analytic
    gradient, which is itself checked by FP64 central differences at
    h = 0.01 arcsec on the same 4-antenna subset."""
    torch = torch_dev
    from paper_1709_08681_amd.autograd import predict
    print("case: cfg4 subset autograd vs finite differences", flush=True)
    full = synth.make_config(4)
    obs = full.subset(ants=[0, 1, 2, 3], times=range(0, 240, 24), chans=range(0, 64, 16))
    prob = oracle.Problem.from_observation(obs)
    v_obs = oracle.predict(prob, obs.offsets_true)
    start = synth.perturbed_offsets(obs, 30.0, 24)
    g = oracle.gradient(prob, start, v_obs, 1.0)[..., 1:3]  # -1/2 d chi^2 / dp
    h = 0.01 * ARCSEC

    def chi2(off):
        r = v_obs - oracle.predict(prob, off)
        return float(np.sum(np.abs(r) ** 2))

    for ant, ax in [(1, 0), (3, 1)]:
        up, dn = start.copy(), start.copy()
        up[0, 0, ant, ax] += h
        dn[0, 0, ant, ax] -= h
        fd = (chi2(up) - chi2(dn)) / (2 * h)
        assert abs(fd - (-2 * g[0, 0, ant, ax])) <= 1e-6 * abs(fd), (ant, ax)
    s = session(obs)
    try:
        vo = c64(torch, s, v_obs)
        off = s.offsets(start).requires_grad_(True)
        loss = ((vo - predict(off, s)).abs() ** 2).sum()
        loss.backward()
        got = off.grad.cpu().numpy()
        live = np.abs(g).sum(axis=-1) > 0
        assert rel(got[live], -2 * g[live]) <= 1e-4
    finally:
        s.close()


def test_gaussian_mode_parity(torch_dev):
    """The Gaussian main-lobe model of Sec. 3 on both sides (illum = 1).  A
    Gaussian aperture has no compact support; its kernel fits the S-cell window
    (to e^-23 at the edge) for sigma >= 1.5 lambda/D."""
    torch = torch_dev
    obs = synth.make_config(1)
    prob = oracle.Problem.from_observation(obs, illum=1, gauss_sigma_ld=1.5)
    s = session(obs, illum=1, gauss_sigma_ld=1.5)
    try:
        start = synth.perturbed_offsets(obs, 20.0, 17)
        v_true = oracle.predict(prob, obs.offsets_true)
        ref_acc, ref_vm = oracle.gradient(prob, start, v_true, 1.0, want_model=True)
        w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        acc, vm = s.gradient(s.offsets(start), c64(torch, s, v_true), w1, want_model=True)
        assert rel(vm.cpu().numpy(), ref_vm) <= 1e-5
        assert rel(acc.cpu().numpy(), ref_acc) <= 1e-4
    finally:
        s.close()


@pytest.mark.parametrize("m", [20, 32])
def test_image_sample_counts(torch_dev, m):
    """Kernel construction with fewer / more image-plane samples per axis."""
    obs = synth.make_config(1)
    prob = oracle.Problem.from_observation(obs)
    s = session(obs, image_samples=m)
    try:
        off = synth.perturbed_offsets(obs, 20.0, 18)
        assert rel(s.predict(off).cpu().numpy(), oracle.predict(prob, off)) <= 1e-5
    finally:
        s.close()


# ---------------------------------------------------------------------------
# every degrid variant: table form on the vector units and on the matrix
# cores, and the window form
# ---------------------------------------------------------------------------

def vjp_reference(obs, prob, off, G, off_shape):
    """Re(conj(G) dV/dp) summed per (interval, pol, antenna, axis), from the
    oracle's analytic derivatives."""
    _, dv = oracle.predict(prob, off, want_grad=True)
    gref = np.zeros(off_shape)
    for r in range(obs.n_row):
        it = np.searchsorted(obs.int_row_ptr, r, side="right") - 1
        i, j = obs.ant1[r], obs.ant2[r]
        for c in range(obs.n_chan):
            for p in range(obs.n_pol):
                g = np.complex128(G[r, c, p])
                for ax in range(2):
                    gref[it, p, i, ax] += (np.conj(g) * dv[r, c, p, ax]).real
                    gref[it, p, j, ax] += (np.conj(g) * dv[r, c, p, 2 + ax]).real
    return gref


def small_ragged_obs(seed, **overrides):
    """8 antennas, intervals of 6, 2 and 9 times, two polarisations with
    squint, two channels (workload fields overridable: the oracle rounds uv to
    the workload's own oversampling lattice)."""
    lengths = [6, 2, 9]
    wl = synth.workload(1, n_ant=8, n_time=sum(lengths), interval_lengths=lengths, n_pol=2,
                        squint_frac=0.03, freqs_hz=np.array([1.1e9, 1.6e9]), n_src=6, **overrides)
    return synth.make_observation(wl, seed)


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_degrid_variants_gradient_and_vjp(torch_dev, variant):
    """Prediction, gradient sums and the adjoint with each degrid variant, on
    ragged intervals with two polarisations (offset pairs f, -f in every item)."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    obs = small_ragged_obs(91)
    prob = oracle.Problem.from_observation(obs)
    s = session(obs)
    try:
        psc.psc_set_degrid(s.handle, variant)
        assert psc.psc_get_degrid(s.handle) == variant
        start = synth.perturbed_offsets(obs, 25.0, 19)
        v = oracle.predict(prob, obs.offsets_true)
        assert rel(s.predict(obs.offsets_true).cpu().numpy(), v) <= 1e-5
        ref, vm_ref = oracle.gradient(prob, start, v, 1.0, want_model=True)
        w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        acc, vm = s.gradient(s.offsets(start), c64(torch, s, v), w1, want_model=True)
        assert rel(vm.cpu().numpy(), vm_ref) <= 1e-5
        acc = acc.cpu().numpy()
        for k in range(6):
            assert rel(acc[..., k], ref[..., k]) <= 1e-4, k
        rng = np.random.default_rng(20)
        G = (rng.normal(size=s.vis_shape) + 1j * rng.normal(size=s.vis_shape)).astype(np.complex64)
        gref = vjp_reference(obs, prob, start, G, s.off_shape)
        got = s.vjp(s.offsets(start), torch.as_tensor(G, device=s.dev)).cpu().numpy()
        assert rel(got, gref) <= 1e-4
    finally:
        s.close()


@pytest.mark.parametrize("m,over", [(32, 4), (64, 2), (48, 8)])
def test_support32_image_sample_extremes(torch_dev, m, over):
    """Support 32, where a wavefront handles each sample and its two halves
    split the 32-point transforms and the image-sample m indices, at M = S
    (half the lanes of each half idle), M = 2S (none idle) and the default
    3S/2: prediction, gradient sums and the adjoint against the oracle."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    obs = small_ragged_obs(93, support=32, oversample=over)
    prob = oracle.Problem.from_observation(obs)
    print(f"case: support 32, M {m}, O {over}", flush=True)
    s = session(obs, image_samples=m)
    try:
        assert psc.psc_get_degrid(s.handle) == psc.DEGRID_WINDOW
        start = synth.perturbed_offsets(obs, 25.0, 37)
        v = oracle.predict(prob, obs.offsets_true)
        assert rel(s.predict(obs.offsets_true).cpu().numpy(), v) <= 1e-5
        ref, vm_ref = oracle.gradient(prob, start, v, 1.0, want_model=True)
        w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        acc, vm = s.gradient(s.offsets(start), c64(torch, s, v), w1, want_model=True)
        assert rel(vm.cpu().numpy(), vm_ref) <= 1e-5
        acc = acc.cpu().numpy()
        for k in range(6):
            assert rel(acc[..., k], ref[..., k]) <= 1e-4, k
        rng = np.random.default_rng(21)
        G = (rng.normal(size=s.vis_shape) + 1j * rng.normal(size=s.vis_shape)).astype(np.complex64)
        got = s.vjp(s.offsets(start), torch.as_tensor(G, device=s.dev)).cpu().numpy()
        assert rel(got, vjp_reference(obs, prob, start, G, s.off_shape)) <= 1e-4
    finally:
        s.close()


def test_autotuner_picks_a_variant(torch_dev, cfg1):
    torch = torch_dev
    from paper_1709_08681_amd import psc
    obs, prob, s = cfg1
    v = s.predict(obs.offsets_true)
    w = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
    off = s.offsets(synth.perturbed_offsets(obs, 20.0, 21))
    t = psc.psc_tune(s.ctx, s.handle, off, v, w, repeats=2)
    assert len(t) == 3 and min(t) > 0
    assert psc.psc_get_degrid(s.handle) == int(np.argmin(t))
    psc.psc_set_degrid(s.handle, psc.DEGRID_VALU)


# ---------------------------------------------------------------------------
# the window form at full size and at support 32 (large workload)
# ---------------------------------------------------------------------------

def test_cfg2_full_size_window_form(torch_dev):
    """Window-form gradient at the full single-interval size against the
    oracle, on every visibility and every per-antenna sum."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print("case: cfg2 full size, window form", flush=True)
    obs = synth.make_config(2)
    prob = oracle.Problem.from_observation(obs)
    s = session(obs)
    try:
        psc.psc_set_degrid(s.handle, psc.DEGRID_WINDOW)
        start = synth.perturbed_offsets(obs, 30.0, 14)
        v_true = oracle.predict(prob, obs.offsets_true)
        ref_acc, ref_vm = oracle.gradient(prob, start, v_true, 1.0, want_model=True)
        w = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        acc, vm = s.gradient(s.offsets(start), c64(torch, s, v_true), w, want_model=True)
        vm, acc = vm.cpu().numpy(), acc.cpu().numpy()
        e_v = rel(vm, ref_vm)
        e_a = [rel(acc[..., k], ref_acc[..., k]) for k in range(6)]
        e_el, e_ant = elem_err(vm, ref_vm), per_antenna_err(acc, ref_acc)
        print(f"cfg2 window: vis rel {e_v:.2e}, acc rel {max(e_a):.2e}, max element {e_el:.2e}, "
              f"per antenna {max(e_ant):.2e}", flush=True)
        assert e_v <= 1e-5
        assert max(e_a) <= 1e-4
        assert e_el <= ELEM_VIS_TOL
        assert max(e_ant) <= ANT_SUM_TOL
    finally:
        s.close()


@pytest.mark.parametrize("what", ["mount_frame", "measured_aperture", "beam_scale", "w_term", "w_stack"])
def test_cfg2_full_size_extensions_sampled_rows(torch_dev, what):
    """The extension kernels on the full single-interval array, in the launch
    configuration the bench times them in (360 samples per item, blocks of
    four wavefronts), in the mount frame (the w-term, like the bench, in the
    sky frame on the array shrunk to arms of 1 km): the model visibilities of every
    36th timestep (every 180th for the measured aperture, whose oracle sums
    the aperture's cells for every pixel and row), and the per-antenna sums
    with the weights zero outside those timesteps, against the oracle on
    those rows alone."""
    torch = torch_dev
    every = 180 if what == "measured_aperture" else 36
    print(f"case: cfg2 full size, {what}, every {every}th timestep", flush=True)
    # w_term: the array shrunk to arms of 1 km (one kernel holds the w-term);
    # w_stack: the array as configured, arms to 21 km (w-stacked)
    obs = synth.make_config(2, layout_radius_m=1000.0) if what == "w_term" else synth.make_config(2)
    times = np.unique(obs.time_idx)[::every]
    rows = np.nonzero(np.isin(obs.time_idx, times))[0]
    sub = obs.subset(times=times)
    kw, okw = dict(mount_frame=True), dict(mount_frame=True)
    if what in ("w_term", "w_stack"):
        kw, okw = dict(w_term=True), dict(w_term=True)
    if what == "measured_aperture":
        A = synth.measured_aperture()
        kw["aperture"] = A
        okw.update(illum=2, aperture=A)
    scale = None
    if what == "beam_scale":
        scale = np.random.default_rng(0).uniform(0.97, 1.03, (obs.n_int, obs.n_pol, obs.n_ant))
        okw["beam_scale"] = scale
    prob = oracle.Problem.from_observation(sub, **okw)
    s = session(obs, **kw)
    try:
        if scale is not None:
            s.set_beam_scale(scale)
        start = synth.perturbed_offsets(obs, 30.0, 14)
        v_sub = oracle.predict(prob, obs.offsets_true)
        vobs = np.zeros(s.vis_shape, np.complex128)
        vobs[rows] = v_sub
        w = np.zeros(s.vis_shape)
        w[rows] = 1.0
        vp = s.predict(start).cpu().numpy()[rows]
        vp_ref = oracle.predict(prob, start)
        e_v, e_el = rel(vp, vp_ref), elem_err(vp, vp_ref)
        if what == "beam_scale":
            acc = s.scale_gradient(s.offsets(start), c64(torch, s, vobs), f32(torch, s, w, s.vis_shape))
            ref = oracle.scale_gradient(prob, start, v_sub, 1.0)
        else:
            acc = s.gradient(s.offsets(start), c64(torch, s, vobs), f32(torch, s, w, s.vis_shape))
            ref = oracle.gradient(prob, start, v_sub, 1.0)
        acc = acc.cpu().numpy()
        e_a = [rel(acc[..., k], ref[..., k]) for k in range(ref.shape[-1])]
        e_ant = per_antenna_err(acc, ref) if ref.shape[-1] == 6 else [0.0]
        print(f"cfg2 {what}: vis rel {e_v:.2e}, acc rel {max(e_a):.2e}, max element {e_el:.2e}, "
              f"per antenna {max(e_ant):.2e} ({len(rows)} of {obs.n_row} rows)", flush=True)
        assert e_v <= 1e-5
        assert max(e_a) <= 1e-4
        assert e_el <= ELEM_VIS_TOL
        assert max(e_ant) <= ANT_SUM_TOL
    finally:
        s.close()


@pytest.fixture(scope="module")
def cfg5_subset(torch_dev):
    """Large workload (4096^2 grid, support 32, oversampling 8, two
    polarisations with opposite squint, random-walk offsets): 6 antennas, the
    first four solution intervals, every 32nd channel."""
    full = synth.make_config(5)
    nt = sum(full.wl.interval_lengths[:4])
    obs = full.subset(ants=range(6), times=range(nt), chans=range(0, 256, 32))
    prob = oracle.Problem.from_observation(obs)
    s = session(obs)
    yield obs, prob, s
    s.close()


def test_cfg5_subset_predict_gradient(torch_dev, cfg5_subset):
    torch = torch_dev
    from paper_1709_08681_amd import psc
    obs, prob, s = cfg5_subset
    print("case: cfg5 subset predict/gradient", flush=True)
    assert psc.psc_get_degrid(s.handle) == psc.DEGRID_WINDOW
    for variant in (psc.DEGRID_VALU, psc.DEGRID_MFMA):
        with pytest.raises(psc.PscError) as ei:
            psc.psc_set_degrid(s.handle, variant)
        assert ei.value.status == -4
    start = synth.perturbed_offsets(obs, 30.0, 22)
    ref = oracle.predict(prob, start)
    got = s.predict(start).cpu().numpy()
    assert rel(got, ref) <= 1e-5
    v = oracle.predict(prob, obs.offsets_true)
    ref_acc, ref_vm = oracle.gradient(prob, start, v, 1.0, want_model=True)
    w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
    acc, vm = s.gradient(s.offsets(start), c64(torch, s, v), w1, want_model=True)
    assert rel(vm.cpu().numpy(), ref_vm) <= 1e-5
    acc = acc.cpu().numpy()
    live = obs.int_row_ptr[1:] > obs.int_row_ptr[:-1]
    for k in range(6):
        assert rel(acc[live][..., k], ref_acc[live][..., k]) <= 1e-4, k


def test_cfg5_subset_solve(torch_dev, cfg5_subset):
    """Algorithm 1 on the support-32 workload: offsets within 0.1 arcsec of the
    oracle's, iteration counts equal, plain and graph forms bit-identical."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    obs, prob, s = cfg5_subset
    print("case: cfg5 subset solve", flush=True)
    v = oracle.predict(prob, obs.offsets_true)
    start = synth.perturbed_offsets(obs, 30.0, 23)
    ref_off, its_ref = oracle.solve(prob, v, 1.0, start, gain=0.5, n_max=5, tol_rad=1e-3 * ARCSEC)
    w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
    outs = []
    for form in (psc.SOLVE_PLAIN, psc.SOLVE_GRAPH):
        off = s.offsets(start)
        its = s.solve(c64(torch, s, v), w1, off, gain=0.5, n_max=5, tol_rad=1e-3 * ARCSEC, form=form)
        assert np.array_equal(its.cpu().numpy(), its_ref)
        outs.append(off.cpu().numpy())
        assert np.abs(outs[-1] - ref_off).max() / ARCSEC <= 0.1
    assert np.array_equal(outs[0], outs[1])


def test_cfg5_share_full_size_sampled_rows(torch_dev):
    """One GPU's share of the large workload at full size (its first 32 of
    256 channels: 312 M visibilities in 64 uneven intervals, support 32), in
    the launch configuration the bench times, where a whole-batch launch
    gives each block 32 consecutive items and one interval's launch one: the
    model of every 200th timestep and the per-antenna sums with the weights
    zero elsewhere against the oracle on those rows; then two iterations of
    Algorithm 1 in the plain form (a launch per interval) and the batched
    form (one launch), iteration counts and offsets bit-identical."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    every = 200
    print(f"case: cfg5 32-channel share at full size, every {every}th timestep", flush=True)
    obs = synth.make_config(5).subset(chans=range(32))
    times = np.unique(obs.time_idx)[::every]
    rows = np.nonzero(np.isin(obs.time_idx, times))[0]
    sub = obs.subset(times=times)
    prob = oracle.Problem.from_observation(sub)
    s = session(obs)
    try:
        assert psc.psc_get_degrid(s.handle) == psc.DEGRID_WINDOW
        start = synth.perturbed_offsets(obs, 30.0, 24)
        v_sub = oracle.predict(prob, obs.offsets_true)
        vobs = np.zeros(s.vis_shape, np.complex64)
        vobs[rows] = v_sub
        w = np.zeros(s.vis_shape, np.float32)
        w[rows] = 1.0
        g_vobs, g_w = c64(torch, s, vobs), f32(torch, s, w, s.vis_shape)
        del vobs, w
        off = s.offsets(start)
        vp = s.predict(start)[torch.as_tensor(rows, device=s.dev)].cpu().numpy()
        vp_ref = oracle.predict(prob, start)
        acc = s.gradient(off, g_vobs, g_w).cpu().numpy()
        ref = oracle.gradient(prob, start, v_sub, 1.0)
        e_v, e_el = rel(vp, vp_ref), elem_err(vp, vp_ref)
        e_a = [rel(acc[..., k], ref[..., k]) for k in range(6)]
        e_ant = per_antenna_err(acc, ref)
        print(f"cfg5 share: vis rel {e_v:.2e}, max element {e_el:.2e}, acc rel {max(e_a):.2e}, "
              f"per antenna {max(e_ant):.2e} ({len(rows)} of {obs.n_row} rows)", flush=True)
        assert e_v <= 1e-5 and e_el <= ELEM_VIS_TOL
        assert max(e_a) <= 1e-4 and max(e_ant) <= ANT_SUM_TOL
        outs = []
        for form in (psc.SOLVE_PLAIN, psc.SOLVE_BATCHED):
            o = s.offsets(start)
            its = s.solve(g_vobs, g_w, o, gain=0.5, n_max=2, tol_rad=1e-3 * ARCSEC, form=form)
            outs.append((its.cpu().numpy(), o.cpu().numpy()))
        assert np.array_equal(outs[0][0], outs[1][0])
        assert np.array_equal(outs[0][1], outs[1][1])
        assert not np.array_equal(outs[0][1], start)
    finally:
        s.close()


def test_support32_multi_item_blocks_ragged(torch_dev):
    """Blocks of 32 items (sky frame, support 32, a launch of at least 2^19
    items) on a ragged item count: 127 antennas of the large workload (8001
    baselines), 31 channels, one timestep in each of its first three
    intervals: 744,093 items, so the whole-batch launch ends on a block of
    29 and has blocks that straddle two intervals.  Every visibility, every
    per-antenna sum and the adjoint against the oracle at perturbed offsets;
    then
    Algorithm 1 with the first interval starting at the true offsets (done
    after one step, so the later whole-batch launches skip its items inside
    blocks shared with the second interval): plain (one item per block),
    batched and graph forms bit-identical."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print("case: support-32 blocks of 32 items, ragged count", flush=True)
    full = synth.make_config(5)
    starts = np.concatenate([[0], np.cumsum(full.wl.interval_lengths)])[:3]
    obs = full.subset(ants=range(127), times=starts, chans=range(31))
    live = np.nonzero(obs.int_row_ptr[1:] > obs.int_row_ptr[:-1])[0]
    assert list(live) == [0, 1, 2]
    prob = oracle.Problem.from_observation(obs)
    s = session(obs)
    try:
        n_items = psc.psc_obs_info(s.handle)[0]
        info = psc.psc_obs_launch_info(s.handle)
        assert n_items == 3 * 8001 * 31 and n_items % 32 == 29
        assert info["degrid"] == psc.DEGRID_WINDOW and info["items_per_block"] == 32
        start = synth.perturbed_offsets(obs, 30.0, 25)
        v = oracle.predict(prob, obs.offsets_true)
        vp = s.predict(start).cpu().numpy()
        vp_ref, dv = oracle.predict(prob, start, want_grad=True)
        w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        g_v = c64(torch, s, v)
        acc = s.gradient(s.offsets(start), g_v, w1).cpu().numpy()
        ref = oracle.gradient(prob, start, v, 1.0)
        e_v, e_el = rel(vp, vp_ref), elem_err(vp, vp_ref)
        e_a = [rel(acc[live][..., k], ref[live][..., k]) for k in range(6)]
        e_ant = per_antenna_err(acc[live], ref[live])
        # the adjoint: sum over visibilities of Re(conj(G) dV/dp) per end
        rng = np.random.default_rng(26)
        G = (rng.normal(size=s.vis_shape) + 1j * rng.normal(size=s.vis_shape)).astype(np.complex64)
        gc = G.astype(np.complex128).conj()
        ti = (gc[..., None] * dv[..., 0:2]).real.sum(axis=1)  # [row][pol][axis], end i
        tj = (gc[..., None] * dv[..., 2:4]).real.sum(axis=1)
        row_int = np.searchsorted(obs.int_row_ptr, np.arange(obs.n_row), side="right") - 1
        vjp_ref = np.zeros(s.off_shape)
        for p in range(obs.n_pol):
            np.add.at(vjp_ref[:, p], (row_int, obs.ant1), ti[:, p, :])
            np.add.at(vjp_ref[:, p], (row_int, obs.ant2), tj[:, p, :])
        vjp = s.vjp(s.offsets(start), torch.as_tensor(G, device=s.dev)).cpu().numpy()
        e_j = rel(vjp[live], vjp_ref[live])
        print(f"multi-item blocks: vis rel {e_v:.2e}, max element {e_el:.2e}, acc rel {max(e_a):.2e}, "
              f"per antenna {max(e_ant):.2e}, adjoint rel {e_j:.2e}", flush=True)
        assert e_v <= 1e-5 and e_el <= ELEM_VIS_TOL
        assert max(e_a) <= 1e-4 and max(e_ant) <= ANT_SUM_TOL
        assert e_j <= 1e-4
        # the first interval from the true offsets: its step is the model's
        # error alone, far below the tolerance
        start[0] = obs.offsets_true[0]
        outs = []
        for form in (psc.SOLVE_PLAIN, psc.SOLVE_BATCHED, psc.SOLVE_GRAPH):
            o = s.offsets(start)
            its = s.solve(g_v, w1, o, gain=0.5, n_max=4, tol_rad=1e-2 * ARCSEC, form=form)
            outs.append((its.cpu().numpy(), o.cpu().numpy()))
        its = outs[0][0]
        print(f"multi-item blocks: iterations per live interval {its[live]}", flush=True)
        assert its[0] == 1 and its[1] == 4 and its[2] == 4
        for its_f, off_f in outs[1:]:
            assert np.array_equal(its_f, its) and np.array_equal(off_f, outs[0][1])
    finally:
        s.close()


# ---------------------------------------------------------------------------
# image gradient: the adjoint of predict with respect to the model image
# ---------------------------------------------------------------------------

def _check_image_gradient(torch, obs, prob, s, start, vo, w, n_rand, seed, tol=1e-4):
    n = obs.grid_n
    rng = np.random.default_rng(seed)
    ix, iy, _ = obs.sky_pixels()
    rx = rng.integers(n // 4, 3 * n // 4, n_rand)
    ry = rng.integers(n // 4, 3 * n // 4, n_rand)
    px = np.concatenate([ix, rx])
    py = np.concatenate([iy, ry])
    l = (px - n // 2) * obs.cell_rad
    m = (py - n // 2) * obs.cell_rad
    ref = oracle.image_gradient(prob, start, vo, w, l, m)
    G = s.image_gradient(s.offsets(start), c64(torch, s, vo), f32(torch, s, w, s.vis_shape))
    got = G.cpu().numpy()[px, py]
    err = rel(got, ref)
    print(f"image gradient: rel {err:.2e} over {px.size} pixels", flush=True)
    assert err <= tol
    return G


def test_image_gradient_cfg1(torch_dev, cfg1):
    """d chi^2 / d I on the model grid against the oracle's direct sum, at
    every model pixel and at random pixels of the central half; a second run
    agrees to float64 rounding (float64 atomics)."""
    torch = torch_dev
    obs, prob, s = cfg1
    print("case: image gradient cfg1", flush=True)
    v = oracle.predict(prob, obs.offsets_true)
    nz, w = synth.noise(v, 100.0, 25)
    vo = v + nz
    start = synth.perturbed_offsets(obs, 20.0, 26)
    G1 = _check_image_gradient(torch, obs, prob, s, start, vo, w, 96, 27)
    G2 = s.image_gradient(s.offsets(start), c64(torch, s, vo), f32(torch, s, w, s.vis_shape))
    assert rel(G2.cpu().numpy(), G1.cpu().numpy()) <= 1e-12


def test_image_gradient_cfg2_full_size(torch_dev):
    torch = torch_dev
    print("case: image gradient cfg2 full size", flush=True)
    obs = synth.make_config(2)
    prob = oracle.Problem.from_observation(obs)
    s = session(obs)
    try:
        start = synth.perturbed_offsets(obs, 30.0, 28)
        v = oracle.predict(prob, obs.offsets_true)
        _check_image_gradient(torch, obs, prob, s, start, v, 1.0, 56, 29)
    finally:
        s.close()


@pytest.mark.parametrize("over,dt", [(2, 30.0), (4, 600.0), (8, 30.0)])
def test_image_gradient_scatter_paths(torch_dev, over, dt):
    """The image gradient through each scatter: LDS patches at oversampling 2;
    10-minute steps at oversampling 4, whose chunks span more than a patch and
    add their taps directly; the one-pass table-form scatter at oversampling
    8, where an item's sub-tables do not fit in LDS."""
    torch = torch_dev
    print(f"case: image gradient scatter, O {over}, dt {dt}", flush=True)
    obs = small_ragged_obs(95, oversample=over, dt_s=dt)
    prob = oracle.Problem.from_observation(obs)
    s = session(obs)
    try:
        v = oracle.predict(prob, obs.offsets_true)
        nz, w = synth.noise(v, 100.0, 31)
        start = synth.perturbed_offsets(obs, 20.0, 32)
        _check_image_gradient(torch, obs, prob, s, start, v + nz, w, 64, 33)
    finally:
        s.close()


@pytest.mark.parametrize("over,dt", [(8, 30.0), (4, 600.0)])
def test_image_gradient_support32(torch_dev, over, dt):
    """Support 32: a kernel built per sample and scattered through an item
    patch (30 s steps) or tap by tap (10-minute steps, items wider than a
    patch)."""
    torch = torch_dev
    print(f"case: image gradient support 32, O {over}, dt {dt}", flush=True)
    obs = small_ragged_obs(97, support=32, oversample=over, dt_s=dt)
    prob = oracle.Problem.from_observation(obs)
    s = session(obs)
    try:
        v = oracle.predict(prob, obs.offsets_true)
        nz, w = synth.noise(v, 100.0, 34)
        start = synth.perturbed_offsets(obs, 20.0, 35)
        G1 = _check_image_gradient(torch, obs, prob, s, start, v + nz, w, 64, 36)
        G2 = s.image_gradient(s.offsets(start), c64(torch, s, v + nz), f32(torch, s, w, s.vis_shape))
        assert rel(G2.cpu().numpy(), G1.cpu().numpy()) <= 1e-12
    finally:
        s.close()


def test_image_gradient_cfg5_subset(torch_dev, cfg5_subset):
    torch = torch_dev
    obs, prob, s = cfg5_subset
    print("case: image gradient cfg5 subset", flush=True)
    v = oracle.predict(prob, obs.offsets_true)
    start = synth.perturbed_offsets(obs, 30.0, 37)
    _check_image_gradient(torch, obs, prob, s, start, v, 1.0, 48, 38)


# ---------------------------------------------------------------------------
# the w-term (each row's w in the measurement equation, window form)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("S,over,mount", [(16, 4, False), (32, 8, False), (16, 4, True)])
def test_w_term_predict_gradient_vjp_image(torch_dev, S, over, mount):
    """Baselines to 3 km, so that leaving w out is a 2-3% error: prediction,
    gradient sums, the adjoint and the image gradient against the oracle
    with the w-term, at both supports and with mount-frame offsets."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print(f"case: w-term, S {S}, O {over}, mount {mount}", flush=True)
    obs = small_ragged_obs(99, support=S, oversample=over, fov_frac=0.85, layout_radius_m=3000.0)
    prob = oracle.Problem.from_observation(obs, w_term=True, mount_frame=mount)
    s = session(obs, w_term=True, mount_frame=mount)
    try:
        assert psc.psc_get_degrid(s.handle) == psc.DEGRID_WINDOW
        with pytest.raises(psc.PscError):
            psc.psc_set_degrid(s.handle, psc.DEGRID_VALU)
        v = oracle.predict(prob, obs.offsets_true)
        v_no_w = oracle.predict(oracle.Problem.from_observation(obs, mount_frame=mount), obs.offsets_true)
        assert rel(v_no_w, v) > 1e-3  # the w-term matters here
        assert rel(s.predict(obs.offsets_true).cpu().numpy(), v) <= 1e-5
        start = synth.perturbed_offsets(obs, 25.0, 43)
        nz, w = synth.noise(v, 100.0, 44)
        ref, vm_ref = oracle.gradient(prob, start, v + nz, w, want_model=True)
        acc, vm = s.gradient(s.offsets(start), c64(torch, s, v + nz), f32(torch, s, w, s.vis_shape),
                             want_model=True)
        assert rel(vm.cpu().numpy(), vm_ref) <= 1e-5
        acc = acc.cpu().numpy()
        for k in range(6):
            assert rel(acc[..., k], ref[..., k]) <= 1e-4, k
        rng = np.random.default_rng(45)
        G = (rng.normal(size=s.vis_shape) + 1j * rng.normal(size=s.vis_shape)).astype(np.complex64)
        got = s.vjp(s.offsets(start), torch.as_tensor(G, device=s.dev)).cpu().numpy()
        assert rel(got, vjp_reference(obs, prob, start, G, s.off_shape)) <= 1e-4
        _check_image_gradient(torch, obs, prob, s, start, v + nz, w, 48, 46)
    finally:
        s.close()


@pytest.mark.parametrize("S,over,mount", [(16, 4, False), (32, 8, False), (16, 4, True)])
def test_w_stacking_predict_gradient_vjp_solve(torch_dev, S, over, mount):
    """Baselines to 24 km: |w| FoV / D up to several uv cells, more than one
    kernel holds, so the observation is w-stacked (each sample reads the
    model grid of the w-plane nearest its w and carries the rest in its
    kernel).  Prediction, gradient sums, the adjoint and Algorithm 1 against
    the oracle's exact w phase; the image gradient is refused."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print(f"case: w-stacking, S {S}, O {over}, mount {mount}", flush=True)
    obs = small_ragged_obs(99, support=S, oversample=over, layout_radius_m=24000.0)
    assert np.abs(obs.w_m).max() * obs.fov / obs.wl.dish_diam_m > 1.5
    prob = oracle.Problem.from_observation(obs, w_term=True, mount_frame=mount)
    s = session(obs, w_term=True, mount_frame=mount)
    try:
        info = psc.psc_obs_launch_info(s.handle)
        print(f"w-stacking: {info['w_planes']} planes", flush=True)
        assert info["w_planes"] > 1
        v = oracle.predict(prob, obs.offsets_true)
        vp = s.predict(obs.offsets_true).cpu().numpy()
        assert rel(vp, v) <= 1e-5 and elem_err(vp, v) <= ELEM_VIS_TOL
        start = synth.perturbed_offsets(obs, 25.0, 43)
        nz, w = synth.noise(v, 100.0, 44)
        ref, vm_ref = oracle.gradient(prob, start, v + nz, w, want_model=True)
        acc, vm = s.gradient(s.offsets(start), c64(torch, s, v + nz), f32(torch, s, w, s.vis_shape),
                             want_model=True)
        vm, acc = vm.cpu().numpy(), acc.cpu().numpy()
        assert rel(vm, vm_ref) <= 1e-5 and elem_err(vm, vm_ref) <= ELEM_VIS_TOL
        for k in range(6):
            assert rel(acc[..., k], ref[..., k]) <= 1e-4, k
        assert max(per_antenna_err(acc, ref)) <= ANT_SUM_TOL
        rng = np.random.default_rng(45)
        G = (rng.normal(size=s.vis_shape) + 1j * rng.normal(size=s.vis_shape)).astype(np.complex64)
        got = s.vjp(s.offsets(start), torch.as_tensor(G, device=s.dev)).cpu().numpy()
        assert rel(got, vjp_reference(obs, prob, start, G, s.off_shape)) <= 1e-4
        ref_off, its_ref = oracle.solve(prob, v + nz, w, start, gain=0.5, n_max=5, tol_rad=1e-3 * ARCSEC)
        off = s.offsets(start)
        its = s.solve(c64(torch, s, v + nz), f32(torch, s, w, s.vis_shape), off, gain=0.5, n_max=5,
                      tol_rad=1e-3 * ARCSEC, form=psc.SOLVE_GRAPH)
        assert np.array_equal(its.cpu().numpy(), its_ref)
        assert np.abs(off.cpu().numpy() - ref_off).max() / ARCSEC <= 0.1
        with pytest.raises(psc.PscError) as ei:
            s.image_gradient(s.offsets(start), c64(torch, s, v), f32(torch, s, w, s.vis_shape))
        assert ei.value.status == psc.PSC_E_UNSUPPORTED
    finally:
        s.close()


def test_w_stacking_follows_the_model(torch_dev):
    """A w-stacked observation planned before the model is set, then given
    two different models in turn: its w-planes follow each one."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print("case: w-stacking follows psc_set_model", flush=True)
    obs = small_ragged_obs(98, layout_radius_m=24000.0)
    s = session(obs, w_term=True)
    try:
        assert psc.psc_obs_launch_info(s.handle)["w_planes"] > 1
        for scale, seed in ((2.0, 0), (0.5, 1)):
            img = obs.image() * scale
            # move one source by a pixel, so the models differ in more than scale
            ix, iy = np.nonzero(img)
            img[ix[seed] + 1, iy[seed]] = img[ix[seed], iy[seed]]
            img[ix[seed], iy[seed]] = 0.0
            psc.psc_set_model(s.ctx, torch.as_tensor(img, device=s.dev))
            n = obs.grid_n
            l, m = (np.nonzero(img)[0] - n // 2) * obs.cell_rad, (np.nonzero(img)[1] - n // 2) * obs.cell_rad
            prob = oracle.Problem(l, m, img[np.nonzero(img)], obs.n_ant, obs.ant1, obs.ant2, obs.uv_m,
                                  obs.int_row_ptr, obs.freq_hz, n_pol=obs.n_pol,
                                  dish_diam_m=obs.wl.dish_diam_m, squint_frac=obs.wl.squint_frac,
                                  snap_scale=obs.snap_scale, w_m=obs.w_m)
            v = oracle.predict(prob, obs.offsets_true)
            assert rel(s.predict(obs.offsets_true).cpu().numpy(), v) <= 1e-5
    finally:
        s.close()


def test_pattern_tables_only_where_an_interval_fits(torch_dev):
    """Per-antenna pattern tables: used by the sky frame at support 16 while
    one interval's tables (pols x channels x antennas x M^2 x 8 bytes) fit
    8 MiB; the mount frame, support 32 and larger arrays evaluate patterns
    per item.  Both paths agree with the oracle (the parity tests above run
    each); here the rule itself."""
    from paper_1709_08681_amd import psc
    print("case: pattern-table rule", flush=True)
    small = synth.make_config(3).subset(ants=range(6), times=range(20))  # 1 x 16 x 6 x 576 x 8 B
    s = session(small)
    try:
        assert psc.psc_obs_launch_info(s.handle)["pattern_tables"] == 1
    finally:
        s.close()
    s = session(small, mount_frame=True)
    try:
        assert psc.psc_obs_launch_info(s.handle)["pattern_tables"] == 0
    finally:
        s.close()
    # 64 antennas x 64 channels: 18.9 MB per interval
    big = synth.make_config(4).subset(times=range(2))
    s = session(big)
    try:
        assert psc.psc_obs_launch_info(s.handle)["pattern_tables"] == 0
    finally:
        s.close()


def test_w_stacking_beyond_its_limit_is_refused(torch_dev):
    """Baselines of 10,000 km: the w-planes would need far more than 2 GiB of
    model grids; refused, while the same observation without w plans."""
    from paper_1709_08681_amd import psc
    print("case: w-stacking refused", flush=True)
    obs = small_ragged_obs(97, layout_radius_m=1.0e7)
    with pytest.raises(psc.PscError) as ei:
        session(obs, w_term=True)
    assert ei.value.status == psc.PSC_E_UNSUPPORTED
    session(obs).close()


def test_w_term_solve(torch_dev):
    """Algorithm 1 with the w-term: the same iterations and offsets as the
    oracle's solve on noisy data, and recovery of the injected offsets from
    noiseless data (without the w-term the model error would bias them)."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print("case: w-term solve", flush=True)
    obs = small_ragged_obs(101, fov_frac=0.85, layout_radius_m=3000.0)
    prob = oracle.Problem.from_observation(obs, w_term=True)
    s = session(obs, w_term=True)
    try:
        v = oracle.predict(prob, obs.offsets_true)
        start = synth.perturbed_offsets(obs, 20.0, 47)
        nz, w = synth.noise(v, 100.0, 48)
        ref, its_ref = oracle.solve(prob, v + nz, w, start, gain=0.5, n_max=8, tol_rad=1e-3 * ARCSEC)
        off = s.offsets(start)
        its = s.solve(c64(torch, s, v + nz), f32(torch, s, w, s.vis_shape), off, gain=0.5, n_max=8,
                      tol_rad=1e-3 * ARCSEC, form=psc.SOLVE_GRAPH)
        assert np.array_equal(its.cpu().numpy(), its_ref)
        assert np.abs(off.cpu().numpy() - ref).max() / ARCSEC <= 0.1
        w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        off = s.offsets(start)
        s.solve(c64(torch, s, v), w1, off, gain=0.5, n_max=80, tol_rad=1e-5 * ARCSEC)
        assert np.abs(off.cpu().numpy() - obs.offsets_true).max() / ARCSEC <= 0.05
    finally:
        s.close()


# ---------------------------------------------------------------------------
# offsets in the antenna mount frame (per-row parallactic angle)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def mount(torch_dev):
    """Ten-minute timesteps over 2.3 hours (the parallactic angle sweeps
    tens of degrees), two polarisations with squint, uneven intervals."""
    lengths = [5, 3, 6]
    wl = synth.workload(1, n_ant=7, n_time=sum(lengths), dt_s=600.0, interval_lengths=lengths, n_pol=2,
                        squint_frac=0.03, freqs_hz=np.array([1.2e9, 1.6e9]), n_src=5)
    obs = synth.make_observation(wl, 93)
    prob = oracle.Problem.from_observation(obs, mount_frame=True)
    s = session(obs, mount_frame=True)
    yield obs, prob, s
    s.close()


def test_mount_frame_predict_gradient_vjp(torch_dev, mount):
    torch = torch_dev
    from paper_1709_08681_amd import psc
    obs, prob, s = mount
    print("case: mount frame predict/gradient/vjp", flush=True)
    pa = obs.par_angle
    assert np.ptp(pa) > 0.3
    assert psc.psc_get_degrid(s.handle) == psc.DEGRID_WINDOW
    for variant in (psc.DEGRID_VALU, psc.DEGRID_MFMA):
        with pytest.raises(psc.PscError) as ei:
            psc.psc_set_degrid(s.handle, variant)
        assert ei.value.status == psc.PSC_E_UNSUPPORTED
    start = synth.perturbed_offsets(obs, 25.0, 33)
    assert rel(s.predict(start).cpu().numpy(), oracle.predict(prob, start)) <= 1e-5
    v = oracle.predict(prob, obs.offsets_true)
    ref, vm_ref = oracle.gradient(prob, start, v, 1.0, want_model=True)
    w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
    acc, vm = s.gradient(s.offsets(start), c64(torch, s, v), w1, want_model=True)
    assert rel(vm.cpu().numpy(), vm_ref) <= 1e-5
    acc = acc.cpu().numpy()
    for k in range(6):
        assert rel(acc[..., k], ref[..., k]) <= 1e-4, k
    rng = np.random.default_rng(34)
    G = (rng.normal(size=s.vis_shape) + 1j * rng.normal(size=s.vis_shape)).astype(np.complex64)
    _, dv = oracle.predict(prob, start, want_grad=True)
    gref = np.zeros(s.off_shape)
    for r in range(obs.n_row):
        it = np.searchsorted(obs.int_row_ptr, r, side="right") - 1
        i, j = obs.ant1[r], obs.ant2[r]
        for c in range(obs.n_chan):
            for p in range(obs.n_pol):
                g = np.complex128(G[r, c, p])
                for ax in range(2):
                    gref[it, p, i, ax] += (np.conj(g) * dv[r, c, p, ax]).real
                    gref[it, p, j, ax] += (np.conj(g) * dv[r, c, p, 2 + ax]).real
    got = s.vjp(s.offsets(start), torch.as_tensor(G, device=s.dev)).cpu().numpy()
    assert rel(got, gref) <= 1e-4


def test_mount_frame_solve(torch_dev, mount):
    """Algorithm 1 solving for mount-frame offsets: offsets within 0.1 arcsec
    of the oracle's after the same iterations, plain and graph forms equal,
    and noiseless recovery of the injected offsets."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    obs, prob, s = mount
    print("case: mount frame solve", flush=True)
    v = oracle.predict(prob, obs.offsets_true)
    start = synth.perturbed_offsets(obs, 25.0, 35)
    ref_off, its_ref = oracle.solve(prob, v, 1.0, start, gain=0.5, n_max=8, tol_rad=1e-3 * ARCSEC)
    w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
    outs = []
    for form in (psc.SOLVE_PLAIN, psc.SOLVE_GRAPH):
        off = s.offsets(start)
        its = s.solve(c64(torch, s, v), w1, off, gain=0.5, n_max=8, tol_rad=1e-3 * ARCSEC, form=form)
        assert np.array_equal(its.cpu().numpy(), its_ref)
        outs.append(off.cpu().numpy())
        assert np.abs(outs[-1] - ref_off).max() / ARCSEC <= 0.1
    assert np.array_equal(outs[0], outs[1])
    off = s.offsets(start)
    s.solve(c64(torch, s, v), w1, off, gain=0.5, n_max=80, tol_rad=1e-5 * ARCSEC)
    assert np.abs(off.cpu().numpy() - obs.offsets_true).max() / ARCSEC <= 0.05


def test_mount_frame_image_gradient(torch_dev, mount):
    """d chi^2 / d I with mount-frame offsets (every row's beams rotated by
    its parallactic angle): a kernel built per sample."""
    torch = torch_dev
    obs, prob, s = mount
    print("case: mount frame image gradient", flush=True)
    v = oracle.predict(prob, obs.offsets_true)
    nz, w = synth.noise(v, 100.0, 39)
    start = synth.perturbed_offsets(obs, 20.0, 40)
    _check_image_gradient(torch, obs, prob, s, start, v + nz, w, 48, 41)


def test_mount_frame_support32(torch_dev, cfg5_subset):
    """Mount-frame offsets on the support-32 large-workload subset."""
    torch = torch_dev
    obs, _, s0 = cfg5_subset
    print("case: mount frame support 32", flush=True)
    prob = oracle.Problem.from_observation(obs, mount_frame=True)
    s = session(obs, mount_frame=True)
    try:
        start = synth.perturbed_offsets(obs, 30.0, 36)
        assert rel(s.predict(start).cpu().numpy(), oracle.predict(prob, start)) <= 1e-5
        v = oracle.predict(prob, obs.offsets_true)
        ref = oracle.gradient(prob, start, v, 1.0)
        w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        acc = s.gradient(s.offsets(start), c64(torch, s, v), w1).cpu().numpy()
        live = obs.int_row_ptr[1:] > obs.int_row_ptr[:-1]
        for k in range(6):
            assert rel(acc[live][..., k], ref[live][..., k]) <= 1e-4, k
        _check_image_gradient(torch, obs, prob, s, start, v, 1.0, 32, 42)
    finally:
        s.close()


# ---------------------------------------------------------------------------
# measured aperture (illum 2): a non-circular pattern fixed to the mount,
# from a table of the aperture's transform
# ---------------------------------------------------------------------------

def _aperture_obs(support, oversample):
    """Ten-minute timesteps over 2.3 hours, two polarisations with squint,
    uneven intervals."""
    lengths = [5, 3, 6]
    wl = synth.workload(1, n_ant=7, n_time=sum(lengths), dt_s=600.0, interval_lengths=lengths, n_pol=2,
                        squint_frac=0.03, freqs_hz=np.array([1.2e9, 1.6e9]), n_src=5, support=support,
                        oversample=oversample)
    return synth.make_observation(wl, 95)


@pytest.mark.parametrize("S,over,mount", [(16, 4, True), (16, 4, False), (32, 8, True)])
def test_measured_aperture_predict_gradient_vjp_image(torch_dev, S, over, mount):
    """A blocked, tapered aperture with feed-leg shadows: prediction, model,
    sums, the adjoint and the image gradient against the oracle's direct
    Fourier sum over the aperture, in the mount frame (angle per row) and in
    the sky frame, at both supports."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print(f"case: measured aperture, S {S}, O {over}, mount {mount}", flush=True)
    obs = _aperture_obs(S, over)
    A = synth.measured_aperture(seed=11)
    prob = oracle.Problem.from_observation(obs, mount_frame=mount, illum=2, aperture=A)
    s = session(obs, mount_frame=mount, aperture=A)
    try:
        assert psc.psc_get_degrid(s.handle) == psc.DEGRID_WINDOW
        for variant in (psc.DEGRID_VALU, psc.DEGRID_MFMA):
            with pytest.raises(psc.PscError) as ei:
                psc.psc_set_degrid(s.handle, variant)
            assert ei.value.status == psc.PSC_E_UNSUPPORTED
        v = oracle.predict(prob, obs.offsets_true)
        v_dish = oracle.predict(oracle.Problem.from_observation(obs, mount_frame=mount), obs.offsets_true)
        assert rel(v_dish, v) > 1e-2  # not the uniform dish
        start = synth.perturbed_offsets(obs, 25.0, 51)
        assert rel(s.predict(start).cpu().numpy(), oracle.predict(prob, start)) <= 1e-5
        nz, w = synth.noise(v, 100.0, 52)
        ref, vm_ref = oracle.gradient(prob, start, v + nz, w, want_model=True)
        acc, vm = s.gradient(s.offsets(start), c64(torch, s, v + nz), f32(torch, s, w, s.vis_shape),
                             want_model=True)
        assert rel(vm.cpu().numpy(), vm_ref) <= 1e-5
        acc = acc.cpu().numpy()
        for k in range(6):
            assert rel(acc[..., k], ref[..., k]) <= 1e-4, k
        rng = np.random.default_rng(53)
        G = (rng.normal(size=s.vis_shape) + 1j * rng.normal(size=s.vis_shape)).astype(np.complex64)
        got = s.vjp(s.offsets(start), torch.as_tensor(G, device=s.dev)).cpu().numpy()
        assert rel(got, vjp_reference(obs, prob, start, G, s.off_shape)) <= 1e-4
        _check_image_gradient(torch, obs, prob, s, start, v + nz, w, 48, 54)
    finally:
        s.close()


def _aperture_stack():
    """Three different illuminations for a heterogeneous array."""
    return np.stack([synth.measured_aperture(seed=31),
                     synth.measured_aperture(seed=32, blockage_frac=0.15, n_legs=3, leg_angle_deg=10.0),
                     synth.measured_aperture(seed=33, blockage_frac=0.0, n_legs=0, edge_taper=0.1)])


@pytest.mark.parametrize("S,over,mount", [(16, 4, True), (16, 4, False), (32, 8, True)])
def test_heterogeneous_apertures_predict_gradient_vjp_image(torch_dev, S, over, mount):
    """Each antenna with one of three measured apertures (Sec. 3, the
    heterogeneous array): prediction, model, sums, the adjoint and the image
    gradient against the oracle, mount and sky frame, both supports."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print(f"case: heterogeneous apertures, S {S}, O {over}, mount {mount}", flush=True)
    obs = _aperture_obs(S, over)
    stack = _aperture_stack()
    ant_ap = np.array([2, 0, 1, 1, 0, 2, 1], np.int32)[:obs.n_ant]
    prob = oracle.Problem.from_observation(obs, mount_frame=mount, illum=2, aperture=stack, ant_aperture=ant_ap)
    s = session(obs, mount_frame=mount, aperture=stack, ant_aperture=ant_ap)
    try:
        assert psc.psc_get_degrid(s.handle) == psc.DEGRID_WINDOW
        v = oracle.predict(prob, obs.offsets_true)
        v_one = oracle.predict(oracle.Problem.from_observation(obs, mount_frame=mount, illum=2, aperture=stack[0]),
                               obs.offsets_true)
        assert rel(v_one, v) > 1e-3  # the assignment matters
        start = synth.perturbed_offsets(obs, 25.0, 71)
        assert rel(s.predict(start).cpu().numpy(), oracle.predict(prob, start)) <= 1e-5
        nz, w = synth.noise(v, 100.0, 72)
        ref, vm_ref = oracle.gradient(prob, start, v + nz, w, want_model=True)
        acc, vm = s.gradient(s.offsets(start), c64(torch, s, v + nz), f32(torch, s, w, s.vis_shape),
                             want_model=True)
        assert rel(vm.cpu().numpy(), vm_ref) <= 1e-5
        vm = vm.cpu().numpy()
        assert elem_err(vm, vm_ref) <= ELEM_VIS_TOL
        acc = acc.cpu().numpy()
        for k in range(6):
            assert rel(acc[..., k], ref[..., k]) <= 1e-4, k
        rng = np.random.default_rng(73)
        G = (rng.normal(size=s.vis_shape) + 1j * rng.normal(size=s.vis_shape)).astype(np.complex64)
        got = s.vjp(s.offsets(start), torch.as_tensor(G, device=s.dev)).cpu().numpy()
        assert rel(got, vjp_reference(obs, prob, start, G, s.off_shape)) <= 1e-4
        _check_image_gradient(torch, obs, prob, s, start, v + nz, w, 32, 74)
        # beam scales below 1 rebuild every aperture's table (0.9: above the
        # floor of both supports, about 0.68 at 16 and 0.86 at 32 here)
        sc = np.random.default_rng(75).uniform(0.9, 1.05, (obs.n_int, obs.n_pol, obs.n_ant))
        s.set_beam_scale(sc)
        prob_s = oracle.Problem.from_observation(obs, mount_frame=mount, illum=2, aperture=stack,
                                                 ant_aperture=ant_ap, beam_scale=sc)
        assert rel(s.predict(start).cpu().numpy(), oracle.predict(prob_s, start)) <= 1e-5
    finally:
        s.close()


def test_heterogeneous_aperture_map_errors(torch_dev):
    from paper_1709_08681_amd import psc
    print("case: heterogeneous aperture map validation", flush=True)
    obs = _aperture_obs(16, 4)
    stack = _aperture_stack()
    bad = np.zeros(obs.n_ant, np.int32)
    bad[3] = 3  # three apertures: 0..2
    with pytest.raises(psc.PscError) as ei:
        session(obs, aperture=stack, ant_aperture=bad)
    assert ei.value.status == psc.PSC_E_ARG
    with pytest.raises(psc.PscError) as ei:
        session(obs, ant_aperture=np.zeros(obs.n_ant, np.int32))  # no measured aperture
    assert ei.value.status == psc.PSC_E_ARG
    odd = stack.copy()
    odd[1, 2, 5] += 0.5  # the second aperture is not even
    with pytest.raises(psc.PscError) as ei:
        session(obs, aperture=odd, ant_aperture=np.zeros(obs.n_ant, np.int32))
    assert ei.value.status == psc.PSC_E_ARG


def test_measured_aperture_solve(torch_dev):
    """Algorithm 1 with the measured aperture in the mount frame: the same
    iterations and offsets as the oracle's solve, plain and graph forms
    equal, and noiseless recovery of the injected offsets."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print("case: measured aperture solve", flush=True)
    obs = _aperture_obs(16, 4)
    A = synth.measured_aperture(seed=12)
    prob = oracle.Problem.from_observation(obs, mount_frame=True, illum=2, aperture=A)
    s = session(obs, mount_frame=True, aperture=A)
    try:
        v = oracle.predict(prob, obs.offsets_true)
        start = synth.perturbed_offsets(obs, 25.0, 55)
        ref_off, its_ref = oracle.solve(prob, v, 1.0, start, gain=0.5, n_max=8, tol_rad=1e-3 * ARCSEC)
        w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        outs = []
        for form in (psc.SOLVE_PLAIN, psc.SOLVE_GRAPH):
            off = s.offsets(start)
            its = s.solve(c64(torch, s, v), w1, off, gain=0.5, n_max=8, tol_rad=1e-3 * ARCSEC, form=form)
            assert np.array_equal(its.cpu().numpy(), its_ref)
            outs.append(off.cpu().numpy())
            assert np.abs(outs[-1] - ref_off).max() / ARCSEC <= 0.1
        assert np.array_equal(outs[0], outs[1])
        off = s.offsets(start)
        s.solve(c64(torch, s, v), w1, off, gain=0.5, n_max=80, tol_rad=1e-5 * ARCSEC)
        assert np.abs(off.cpu().numpy() - obs.offsets_true).max() / ARCSEC <= 0.05
    finally:
        s.close()


@pytest.mark.parametrize("n,mount", [(256, False), (256, True), (2, True), (1, False), (1, True)])
def test_measured_aperture_size_limits(torch_dev, n, mount):
    """The largest illumination the library takes (256 cells per side), the
    smallest that is not flat (2 x 2 cells) and a single cell, whose pattern
    is 1 everywhere: prediction and the sums against the oracle; with one
    cell the offsets' sums and curvatures are exactly zero on both sides."""
    torch = torch_dev
    print(f"case: measured aperture of {n} x {n} cells, mount {mount}", flush=True)
    obs = _aperture_obs(16, 4)
    A = synth.measured_aperture(n=n, seed=3) if n > 2 else np.ones((n, n))
    prob = oracle.Problem.from_observation(obs, mount_frame=mount, illum=2, aperture=A)
    s = session(obs, mount_frame=mount, aperture=A)
    try:
        start = synth.perturbed_offsets(obs, 25.0, 51)
        v = oracle.predict(prob, obs.offsets_true)
        assert rel(s.predict(start).cpu().numpy(), oracle.predict(prob, start)) <= 1e-5
        # noisy data, so that chi is not zero where the beam is flat
        nz, w = synth.noise(v, 100.0, 52)
        ref = oracle.gradient(prob, start, v + nz, w)
        acc = s.gradient(s.offsets(start), c64(torch, s, v + nz), f32(torch, s, w, s.vis_shape)).cpu().numpy()
        if n == 1:
            assert rel(acc[..., 0], ref[..., 0]) <= 1e-4
            assert np.all(ref[..., 1:] == 0) and np.all(acc[..., 1:] == 0)
        else:
            for k in range(6):
                assert rel(acc[..., k], ref[..., k]) <= 1e-4, k
    finally:
        s.close()


def test_measured_aperture_must_be_even(torch_dev):
    from paper_1709_08681_amd import psc
    print("case: measured aperture validation", flush=True)
    obs = _aperture_obs(16, 4)
    A = synth.measured_aperture(seed=13)
    A[2, 7] += 0.5
    with pytest.raises(psc.PscError) as ei:
        session(obs, aperture=A)
    assert ei.value.status == psc.PSC_E_ARG


# ---------------------------------------------------------------------------
# beam-width scales: a generalised antenna parameter beside the offsets
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("S,over,mount,ap", [(16, 4, False, False), (16, 4, True, False),
                                             (32, 8, True, False), (16, 4, True, True)])
def test_beam_scale_predict_gradients_image(torch_dev, S, over, mount, ap):
    """Scales within 5% of nominal: prediction, the offsets' sums, the scale
    sums, the adjoint and the image gradient against the oracle, sky and
    mount frame, both supports, and with a measured aperture."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print(f"case: beam scale, S {S}, O {over}, mount {mount}, aperture {ap}", flush=True)
    obs = _aperture_obs(S, over)
    A = synth.measured_aperture(seed=14) if ap else None
    sc = np.random.default_rng(61).uniform(0.95, 1.05, (obs.n_int, obs.n_pol, obs.n_ant))
    kw = dict(illum=2, aperture=A) if ap else {}
    prob = oracle.Problem.from_observation(obs, mount_frame=mount, beam_scale=sc, **kw)
    s = session(obs, mount_frame=mount, aperture=A)
    try:
        s.set_beam_scale(sc)
        assert np.array_equal(s.beam_scale().cpu().numpy(), sc)
        assert psc.psc_get_degrid(s.handle) == psc.DEGRID_WINDOW
        with pytest.raises(psc.PscError) as ei:
            psc.psc_set_degrid(s.handle, psc.DEGRID_VALU)
        assert ei.value.status == psc.PSC_E_UNSUPPORTED
        v = oracle.predict(prob, obs.offsets_true)
        v_nom = oracle.predict(oracle.Problem.from_observation(obs, mount_frame=mount, **kw), obs.offsets_true)
        assert rel(v_nom, v) > 1e-3  # the scales matter
        start = synth.perturbed_offsets(obs, 25.0, 62)
        assert rel(s.predict(start).cpu().numpy(), oracle.predict(prob, start)) <= 1e-5
        nz, w = synth.noise(v, 100.0, 63)
        vo_d, w_d = c64(torch, s, v + nz), f32(torch, s, w, s.vis_shape)
        ref, vm_ref = oracle.gradient(prob, start, v + nz, w, want_model=True)
        acc, vm = s.gradient(s.offsets(start), vo_d, w_d, want_model=True)
        assert rel(vm.cpu().numpy(), vm_ref) <= 1e-5
        acc = acc.cpu().numpy()
        for k in range(6):
            assert rel(acc[..., k], ref[..., k]) <= 1e-4, k
        ref3 = oracle.scale_gradient(prob, start, v + nz, w)
        acc3 = s.scale_gradient(s.offsets(start), vo_d, w_d).cpu().numpy()
        for k in range(3):
            assert rel(acc3[..., k], ref3[..., k]) <= 1e-4, k
        rng = np.random.default_rng(64)
        G = (rng.normal(size=s.vis_shape) + 1j * rng.normal(size=s.vis_shape)).astype(np.complex64)
        got = s.vjp(s.offsets(start), torch.as_tensor(G, device=s.dev)).cpu().numpy()
        assert rel(got, vjp_reference(obs, prob, start, G, s.off_shape)) <= 1e-4
        _check_image_gradient(torch, obs, prob, s, start, v + nz, w, 32, 65)
        # dropping the scales gives the nominal beams again
        s.set_beam_scale(None)
        nominal = oracle.Problem.from_observation(obs, mount_frame=mount, **kw)
        assert rel(s.predict(start).cpu().numpy(), oracle.predict(nominal, start)) <= 1e-5
    finally:
        s.close()


def test_beam_scale_solve(torch_dev):
    """Injected scales (3% spread) at the true offsets, noiseless data: the
    damped scale steps from sigma = 1 follow the oracle's and recover them."""
    torch = torch_dev
    print("case: beam scale solve", flush=True)
    obs = _aperture_obs(16, 4)
    truth = np.random.default_rng(66).uniform(0.97, 1.03, (obs.n_int, obs.n_pol, obs.n_ant))
    v = oracle.predict(oracle.Problem.from_observation(obs, beam_scale=truth), obs.offsets_true)
    s = session(obs)
    try:
        w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        vo = c64(torch, s, v)
        off = s.offsets(obs.offsets_true)
        s.set_beam_scale(np.ones_like(truth))
        ref = np.ones_like(truth)
        for it in range(60):
            acc = s.scale_gradient(off, vo, w1)
            nu, mx = s.scale_step(acc, 0.5)
            if it < 8:
                a3 = oracle.scale_gradient(oracle.Problem.from_observation(obs, beam_scale=ref), obs.offsets_true,
                                           v, 1.0)
                ref, _, _ = oracle.scale_step(a3, 0.5, ref)
                if it == 7:
                    assert np.abs(s.beam_scale().cpu().numpy() - ref).max() <= 1e-5
        assert int(nu.sum()) == 0
        assert np.abs(s.beam_scale().cpu().numpy() - truth).max() <= 1e-4
    finally:
        s.close()


def test_beam_scale_errors(torch_dev):
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print("case: beam scale errors", flush=True)
    obs = _aperture_obs(16, 4)
    s = session(obs)
    try:
        w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        vo = torch.zeros(s.vis_shape, dtype=torch.complex64, device=s.dev)
        with pytest.raises(psc.PscError) as ei:
            s.scale_gradient(s.offsets(obs.offsets_true), vo, w1)
        assert ei.value.status == psc.PSC_E_STATE
        bad = np.ones((obs.n_int, obs.n_pol, obs.n_ant))
        bad[1, 0, 2] = 0.0
        with pytest.raises(psc.PscError) as ei:
            s.set_beam_scale(bad)
        assert ei.value.status == psc.PSC_E_ARG
        assert psc.psc_get_degrid(s.handle) == psc.DEGRID_VALU  # unchanged
        # a beam narrowed to 0.6 widens the aperture past what the support
        # holds (8 of 16 cells at sigma = 1 here); 0.75 still fits
        narrow = np.ones((obs.n_int, obs.n_pol, obs.n_ant))
        narrow[2, 1, 4] = 0.6
        with pytest.raises(psc.PscError) as ei:
            s.set_beam_scale(narrow)
        assert ei.value.status == psc.PSC_E_UNSUPPORTED
        assert psc.psc_get_degrid(s.handle) == psc.DEGRID_VALU
        narrow[2, 1, 4] = 0.75
        s.set_beam_scale(narrow)
        prob = oracle.Problem.from_observation(obs, beam_scale=narrow)
        start = synth.perturbed_offsets(obs, 25.0, 57)
        assert rel(s.predict(start).cpu().numpy(), oracle.predict(prob, start)) <= 1e-5
        # the step does not narrow a beam past the same bound: 0.75 - 0.15
        # is refused and flagged, 1 - 0.15 taken
        acc = np.zeros((obs.n_int, obs.n_pol, obs.n_ant, 3))
        acc[..., 2] = 1.0
        acc[2, 1, 4, 1] = acc[2, 1, 3, 1] = -0.15
        nu, _ = s.scale_step(torch.as_tensor(acc, device=s.dev), 1.0)
        got, nu = s.beam_scale().cpu().numpy(), nu.cpu().numpy()
        assert nu[2, 1, 4] == 1 and got[2, 1, 4] == 0.75
        assert nu[2, 1, 3] == 0 and got[2, 1, 3] == pytest.approx(0.85, abs=1e-15)
    finally:
        s.close()


@pytest.mark.parametrize("mount,ap", [(False, False), (True, True)])
def test_beam_scale_tables_cover_narrow_beams(torch_dev, mount, ap):
    """A scale below 1 stretches every pattern lookup to |l - p| / sigma: the
    first psc_set_beam_scale rebuilds the Airy table (and a measured
    aperture's) over the range at the narrowest scale the support allows, and
    beams narrowed to 0.75 with offsets up to 0.15 of the field of view per
    axis (within the quarter the tables allow for) still match the oracle's
    direct evaluation."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print(f"case: beam scale tables, mount {mount}, aperture {ap}", flush=True)
    obs = _aperture_obs(16, 4)
    A = synth.measured_aperture(seed=15) if ap else None
    kw = dict(illum=2, aperture=A) if ap else {}
    s = session(obs, mount_frame=mount, aperture=A)
    try:
        n0 = psc.psc_obs_launch_info(s.handle)["tab_nodes"]
        sc = np.full((obs.n_int, obs.n_pol, obs.n_ant), 0.75)
        s.set_beam_scale(sc)
        n1 = psc.psc_obs_launch_info(s.handle)["tab_nodes"]
        assert n1 >= (n0 - 3) / 0.75 + 2
        s.set_beam_scale(np.ones_like(sc))  # no second rebuild
        assert psc.psc_obs_launch_info(s.handle)["tab_nodes"] == n1
        s.set_beam_scale(sc)
        rng = np.random.default_rng(67)
        far = obs.offsets_true + rng.uniform(-0.15, 0.15, obs.offsets_true.shape) * obs.fov
        prob = oracle.Problem.from_observation(obs, mount_frame=mount, beam_scale=sc, **kw)
        v = oracle.predict(prob, obs.offsets_true)
        assert rel(s.predict(far).cpu().numpy(), oracle.predict(prob, far)) <= 1e-5
        w = np.ones(v.shape)
        ref = oracle.gradient(prob, far, v, w)
        acc = s.gradient(s.offsets(far), c64(torch, s, v), f32(torch, s, w, s.vis_shape)).cpu().numpy()
        for k in range(6):
            assert rel(acc[..., k], ref[..., k]) <= 1e-4, k
        ref3 = oracle.scale_gradient(prob, far, v, w)
        acc3 = s.scale_gradient(s.offsets(far), c64(torch, s, v), f32(torch, s, w, s.vis_shape)).cpu().numpy()
        for k in range(3):
            assert rel(acc3[..., k], ref3[..., k]) <= 1e-4, k
    finally:
        s.close()


def test_offsets_solve_with_beam_scales(torch_dev):
    """Algorithm 1 for the offsets with the beams widened or narrowed: the
    same iterations and offsets as the oracle's solve, in the plain and the
    graph forms; a graph captured before the scales were set, or before they
    were dropped, is rebuilt."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print("case: offsets solve with beam scales", flush=True)
    obs = _aperture_obs(16, 4)
    sc = np.random.default_rng(67).uniform(0.95, 1.05, (obs.n_int, obs.n_pol, obs.n_ant))
    prob = oracle.Problem.from_observation(obs, beam_scale=sc)
    nominal = oracle.Problem.from_observation(obs)
    v = oracle.predict(prob, obs.offsets_true)
    start = synth.perturbed_offsets(obs, 25.0, 68)
    kw = dict(gain=0.5, n_max=8, tol_rad=1e-3 * ARCSEC)
    ref, its_ref = oracle.solve(prob, v, 1.0, start, **kw)
    ref0, its0 = oracle.solve(nominal, v, 1.0, start, **kw)
    s = session(obs)
    try:
        w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        vo = c64(torch, s, v)
        off = s.offsets(start)
        s.solve(vo, w1, off, form=psc.SOLVE_GRAPH, **kw)  # captured on the nominal beams
        s.set_beam_scale(sc)
        for form in (psc.SOLVE_PLAIN, psc.SOLVE_GRAPH):
            off = s.offsets(start)
            its = s.solve(vo, w1, off, form=form, **kw)
            assert np.array_equal(its.cpu().numpy(), its_ref)
            assert np.abs(off.cpu().numpy() - ref).max() / ARCSEC <= 0.1
        s.set_beam_scale(None)
        off = s.offsets(start)
        its = s.solve(vo, w1, off, form=psc.SOLVE_GRAPH, **kw)
        assert np.array_equal(its.cpu().numpy(), its0)
        assert np.abs(off.cpu().numpy() - ref0).max() / ARCSEC <= 0.1
    finally:
        s.close()


def test_scale_step_matches_oracle(torch_dev):
    """The damped scale step on random sums against the oracle's, with an
    antenna without data, one whose step would turn sigma negative, and a
    non-finite sum; the scales live on the observation."""
    torch = torch_dev
    print("case: scale step", flush=True)
    obs = _aperture_obs(16, 4)
    shape = (obs.n_int, obs.n_pol, obs.n_ant)
    rng = np.random.default_rng(69)
    sc0 = rng.uniform(0.9, 1.1, shape)
    acc = np.zeros(shape + (3,))
    acc[..., 0] = rng.uniform(1.0, 2.0, shape)
    acc[..., 1] = rng.normal(0.0, 0.05, shape)
    acc[..., 2] = rng.uniform(0.5, 2.0, shape)
    acc[0, 0, 1, 2] = 0.0          # no data
    acc[1, 1, 3, 1:] = [-40.0, 1.0]  # sigma would turn negative
    acc[2, 0, 5, 1] = np.nan        # non-finite
    ref, nu_ref, mx_ref = oracle.scale_step(acc, 0.5, sc0)
    s = session(obs)
    try:
        s.set_beam_scale(sc0)
        nu, mx = s.scale_step(torch.as_tensor(acc, device=s.dev), 0.5)
        np.testing.assert_allclose(s.beam_scale().cpu().numpy(), ref, rtol=1e-15, atol=0.0)
        assert np.array_equal(nu.cpu().numpy(), nu_ref)
        np.testing.assert_allclose(mx.cpu().numpy(), mx_ref, rtol=1e-12)
    finally:
        s.close()


@pytest.mark.parametrize("mount", [False, True])
def test_extensions_together(torch_dev, mount):
    """The measured aperture, beam scales and the w-term at once (baselines
    to 3 km, field at 0.85 of the support's limit): prediction, the offsets'
    sums, the scale sums and the image gradient against the oracle."""
    torch = torch_dev
    print(f"case: aperture + scales + w-term, mount {mount}", flush=True)
    lengths = [5, 3, 6]
    wl = synth.workload(1, n_ant=7, n_time=sum(lengths), dt_s=600.0, interval_lengths=lengths, n_pol=2,
                        squint_frac=0.03, freqs_hz=np.array([1.2e9, 1.6e9]), n_src=5, fov_frac=0.85,
                        layout_radius_m=3000.0)
    obs = synth.make_observation(wl, 97)
    A = synth.measured_aperture(seed=15)
    sc = np.random.default_rng(70).uniform(0.96, 1.04, (obs.n_int, obs.n_pol, obs.n_ant))
    prob = oracle.Problem.from_observation(obs, mount_frame=mount, w_term=True, illum=2, aperture=A,
                                           beam_scale=sc)
    s = session(obs, mount_frame=mount, w_term=True, aperture=A)
    try:
        s.set_beam_scale(sc)
        start = synth.perturbed_offsets(obs, 25.0, 71)
        assert rel(s.predict(start).cpu().numpy(), oracle.predict(prob, start)) <= 1e-5
        v = oracle.predict(prob, obs.offsets_true)
        nz, w = synth.noise(v, 100.0, 72)
        vo_d, w_d = c64(torch, s, v + nz), f32(torch, s, w, s.vis_shape)
        ref = oracle.gradient(prob, start, v + nz, w)
        acc = s.gradient(s.offsets(start), vo_d, w_d).cpu().numpy()
        for k in range(6):
            assert rel(acc[..., k], ref[..., k]) <= 1e-4, k
        ref3 = oracle.scale_gradient(prob, start, v + nz, w)
        acc3 = s.scale_gradient(s.offsets(start), vo_d, w_d).cpu().numpy()
        for k in range(3):
            assert rel(acc3[..., k], ref3[..., k]) <= 1e-4, k
        _check_image_gradient(torch, obs, prob, s, start, v + nz, w, 32, 73)
    finally:
        s.close()


def test_solve_beam_scale(torch_dev):
    """psc_solve_scale: with tol 0 it equals as many separate scale-gradient
    and step calls, bit for bit; with a tolerance, the steps per interval and
    the scales follow the oracle's loop under the same stopping rule, and the
    injected scales are recovered."""
    torch = torch_dev
    print("case: beam scale solve on the device", flush=True)
    obs = _aperture_obs(16, 4)
    shape = (obs.n_int, obs.n_pol, obs.n_ant)
    truth = np.random.default_rng(74).uniform(0.97, 1.03, shape)
    v = oracle.predict(oracle.Problem.from_observation(obs, beam_scale=truth), obs.offsets_true)
    s = session(obs)
    try:
        off = s.offsets(obs.offsets_true)
        vo = c64(torch, s, v)
        w1 = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        s.set_beam_scale(np.ones(shape))
        s.solve_beam_scale(off, vo, w1, gain=0.5, n_max=6, tol=0.0)
        solved = s.beam_scale().clone()
        s.set_beam_scale(np.ones(shape))
        for _ in range(6):
            s.scale_step(s.scale_gradient(off, vo, w1), 0.5)
        assert torch.equal(solved, s.beam_scale())
        tol = 1e-4
        s.set_beam_scale(np.ones(shape))
        its = s.solve_beam_scale(off, vo, w1, gain=0.5, n_max=60, tol=tol).cpu().numpy()
        ref = np.ones(shape)
        done = np.zeros(obs.n_int, bool)
        its_ref = np.zeros(obs.n_int, np.int32)
        for _ in range(60):
            if done.all():
                break
            a3 = oracle.scale_gradient(oracle.Problem.from_observation(obs, beam_scale=ref), obs.offsets_true, v,
                                       1.0)
            new, _, mx = oracle.scale_step(a3, 0.5, ref)
            new[done] = ref[done]
            its_ref[~done] += 1
            ref = new
            done |= mx < tol
        assert np.abs(its - its_ref).max() <= 1, (its, its_ref)
        got = s.beam_scale().cpu().numpy()
        assert np.abs(got - ref).max() <= 2e-4
        assert np.abs(got - truth).max() <= 5e-4
    finally:
        s.close()


# ---------------------------------------------------------------------------
# aperture defocus: a complex generalised antenna parameter
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("S,over,illum", [(16, 4, 0), (16, 4, 1), (32, 8, 0)])
def test_defocus_predict_sums_step(torch_dev, S, over, illum):
    """Aperture defocus per (interval, pol, antenna) (Eq. DA with complex
    a_i; Sec. 5.3): complex patterns E_i conj(E_j) in the window form against
    the oracle (uniform disc by its Hankel quadrature, Gaussian aperture in
    closed form): prediction, the defocus sums, the damped step, five rounds of
    sums + step, back to real patterns, and the calls refused meanwhile."""
    torch = torch_dev
    from paper_1709_08681_amd import psc
    print(f"case: defocus, S {S}, O {over}, illum {illum}", flush=True)
    obs = small_ragged_obs(77, support=S, oversample=over)
    kw = dict(illum=1, gauss_sigma_ld=1.5) if illum == 1 else {}
    prob = oracle.Problem.from_observation(obs, **kw)
    s = session(obs, **kw)
    rng = np.random.default_rng(78)
    truth = rng.uniform(-0.8, 0.8, s.off_shape[:3])
    start = truth + rng.normal(0.0, 0.1, truth.shape)
    try:
        with pytest.raises(psc.PscError) as ei:
            s.defocus()
        assert ei.value.status == psc.PSC_E_STATE
        psc.psc_set_degrid(s.handle, psc.DEGRID_WINDOW)  # as with the defocus set
        v_real = s.predict(obs.offsets_true).cpu().numpy()
        s.set_defocus(truth)
        assert np.array_equal(s.defocus().cpu().numpy(), truth)
        v_ref, _ = oracle.predict_defocus(prob, obs.offsets_true, truth)
        vp = s.predict(obs.offsets_true).cpu().numpy()
        e_v = rel(vp, v_ref)
        print(f"defocus predict rel {e_v:.2e}, effect {rel(v_real, v_ref):.2e}", flush=True)
        assert e_v <= 1e-5 and elem_err(vp, v_ref) <= ELEM_VIS_TOL
        assert rel(v_real, v_ref) > 1e-3  # the defocus matters here
        # sums at a perturbed defocus, data from the truth with noise
        nz, w = synth.noise(v_ref, 100.0, 79)
        s.set_defocus(start)
        off = s.offsets(obs.offsets_true)
        acc = s.defocus_gradient(off, c64(torch, s, v_ref + nz), f32(torch, s, w, s.vis_shape)).cpu().numpy()
        ref = oracle.defocus_gradient(prob, obs.offsets_true, start, v_ref + nz, w)
        e_a = [rel(acc[..., k], ref[..., k]) for k in range(3)]
        print(f"defocus sums rel {max(e_a):.2e}", flush=True)
        assert max(e_a) <= 1e-4
        # the step on the oracle's own sums
        nu, mx = s.defocus_step(torch.as_tensor(ref, device=s.dev), 0.5)
        d_ref, nu_ref, mx_ref = oracle.defocus_step(ref, 0.5, start)
        np.testing.assert_allclose(s.defocus().cpu().numpy(), d_ref, rtol=0, atol=1e-12)
        assert np.array_equal(nu.cpu().numpy(), nu_ref)
        np.testing.assert_allclose(mx.cpu().numpy(), mx_ref, rtol=1e-12)
        # five rounds of sums + step on each side
        s.set_defocus(start)
        d_o = start.copy()
        vo = c64(torch, s, v_ref + nz)
        wt = f32(torch, s, w, s.vis_shape)
        for _ in range(5):
            s.defocus_step(s.defocus_gradient(off, vo, wt), 0.5)
            d_o, _, _ = oracle.defocus_step(oracle.defocus_gradient(prob, obs.offsets_true, d_o, v_ref + nz, w),
                                            0.5, d_o)
        d_g = s.defocus().cpu().numpy()
        print(f"defocus after 5 rounds: {np.abs(d_g - d_o).max():.2e} rad from the oracle's", flush=True)
        assert np.abs(d_g - d_o).max() <= 1e-5
        # the calls that take real patterns only are refused meanwhile
        for call in (lambda: s.gradient(off, vo, wt), lambda: s.vjp(off, vo),
                     lambda: s.solve(vo, wt, s.offsets(obs.offsets_true), n_max=1)):
            with pytest.raises(psc.PscError) as ei:
                call()
            assert ei.value.status == psc.PSC_E_UNSUPPORTED
        with pytest.raises(psc.PscError) as ei:
            s.set_defocus(np.full(s.off_shape[:3], 3.2))
        assert ei.value.status == psc.PSC_E_ARG
        s.set_defocus(None)
        assert np.array_equal(s.predict(obs.offsets_true).cpu().numpy(), v_real)
    finally:
        s.close()


def test_defocus_full_size_sampled_rows(torch_dev):
    """Aperture defocus on the full single-interval array (360 samples per
    item, four-wavefront blocks): the model of every 36th timestep and the
    defocus sums with the weights zero elsewhere, against the oracle on those
    rows."""
    torch = torch_dev
    every = 36
    print(f"case: cfg2 full size, defocus, every {every}th timestep", flush=True)
    obs = synth.make_config(2)
    times = np.unique(obs.time_idx)[::every]
    rows = np.nonzero(np.isin(obs.time_idx, times))[0]
    sub = obs.subset(times=times)
    prob = oracle.Problem.from_observation(sub)
    s = session(obs)
    try:
        rng = np.random.default_rng(80)
        truth = rng.uniform(-1.0, 1.0, s.off_shape[:3])
        start = truth + rng.normal(0.0, 0.1, truth.shape)
        v_sub, _ = oracle.predict_defocus(prob, obs.offsets_true, truth)
        s.set_defocus(start)
        vp = s.predict(obs.offsets_true).cpu().numpy()[rows]
        vp_ref, _ = oracle.predict_defocus(prob, obs.offsets_true, start)
        vobs = np.zeros(s.vis_shape, np.complex128)
        vobs[rows] = v_sub
        w = np.zeros(s.vis_shape)
        w[rows] = 1.0
        acc = s.defocus_gradient(s.offsets(obs.offsets_true), c64(torch, s, vobs),
                                 f32(torch, s, w, s.vis_shape)).cpu().numpy()
        ref = oracle.defocus_gradient(prob, obs.offsets_true, start, v_sub, 1.0)
        e_v, e_el = rel(vp, vp_ref), elem_err(vp, vp_ref)
        e_a = [rel(acc[..., k], ref[..., k]) for k in range(3)]
        print(f"cfg2 defocus: vis rel {e_v:.2e}, max element {e_el:.2e}, sums rel {max(e_a):.2e}", flush=True)
        assert e_v <= 1e-5 and e_el <= ELEM_VIS_TOL
        assert max(e_a) <= 1e-4
    finally:
        s.close()
