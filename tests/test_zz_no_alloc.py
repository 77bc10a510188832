"""The allocation-free gradient (psc_gradient_noalloc) against psc_gradient,
through the C ABI: two calls in a row on one GPU, the second on a smaller
observation, in the table form and the window form, and the refusal of an
observation whose partial sums exceed the fixed scratch."""
import numpy as np
import pytest

from paper_1709_08681_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_08681_amd import psc
    psc.load()
    return torch


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _pair(torch, s, obs, variant, seed):
    """(psc_gradient, psc_gradient_noalloc) sums and model visibilities on the
    same data."""
    from paper_1709_08681_amd import psc as P
    P.psc_set_degrid(s.handle, variant)
    off = s.offsets(synth.perturbed_offsets(obs, 30.0, seed))
    v = s.predict(s.offsets(obs.offsets_true))
    w = torch.rand(s.vis_shape, dtype=torch.float32, device=s.dev, generator=torch.Generator(
        device=s.dev).manual_seed(seed)) + 0.5
    out = []
    for fn in (P.psc_gradient, P.psc_gradient_noalloc):
        acc = torch.full(s.off_shape[:3] + (6,), float("nan"), dtype=torch.float64, device=s.dev)
        vm = torch.zeros(s.vis_shape, dtype=torch.complex64, device=s.dev)
        fn(s.ctx, s.handle, off, v, w, acc, vm, None)
        torch.cuda.synchronize()
        out.append((acc.cpu().numpy(), vm.cpu().numpy()))
    return out


@pytest.mark.parametrize("variant_name", ["vector", "window"])
def test_noalloc_gradient_matches_gradient_two_calls(torch_dev, variant_name):
    torch = torch_dev
    from paper_1709_08681_amd import psc as P
    variant = P.DEGRID_VALU if variant_name == "vector" else P.DEGRID_WINDOW
    big = synth.make_config(2)  # 5616 work items
    small = synth.make_config(1)  # 45 work items, after the big one
    for obs, seed in ((big, 3), (small, 4)):
        print(f"case: no-alloc gradient, {variant_name}, {obs.n_vis} visibilities", flush=True)
        s = P.Session(obs, device=0)
        try:
            (a_ref, v_ref), (a_na, v_na) = _pair(torch, s, obs, variant, seed)
        finally:
            s.close()
        assert np.all(np.isfinite(a_na))
        # the same kernels in the same order: identical, and within the sums' tolerance
        assert _rel(a_na, a_ref) <= 1e-4 and _rel(v_na, v_ref) <= 1e-5
        assert np.array_equal(a_na, a_ref) and np.array_equal(v_na, v_ref)


def test_noalloc_gradient_refuses_beyond_its_scratch(torch_dev):
    """The batched workload has 1,437,696 work items: 138 MB of partial sums,
    beyond the 64 MiB scratch; refused before any launch."""
    torch = torch_dev
    from paper_1709_08681_amd import psc as P
    obs = synth.make_config(3)
    s = P.Session(obs, device=0)
    try:
        n_items = P.psc_obs_info(s.handle)[0]
        assert n_items * obs.n_pol * 12 * 8 > 64 << 20
        off = s.offsets(obs.offsets_true)
        v = torch.zeros(s.vis_shape, dtype=torch.complex64, device=s.dev)
        w = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        acc = torch.zeros(s.off_shape[:3] + (6,), dtype=torch.float64, device=s.dev)
        with pytest.raises(P.PscError) as ei:
            P.psc_gradient_noalloc(s.ctx, s.handle, off, v, w, acc, None, None)
        assert ei.value.status == P.PSC_E_UNSUPPORTED
        assert float(acc.abs().sum()) == 0.0
    finally:
        s.close()
