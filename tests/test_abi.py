"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/psc.h, and rejects invalid configurations before touching
a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psc.h")


@pytest.fixture(scope="module")
def psc():
    from paper_1709_08681_amd import psc as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1709_08681_amd import build
        build.build()
    m.load()
    return m


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"PSC_API\s+[\w\s\*]+?\b(psc_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["psc_create", "psc_destroy", "psc_set_model", "psc_obs_create", "psc_predict",
              "psc_gradient", "psc_predict_vjp", "psc_solve_step", "psc_solve"]:
        assert n in names


def test_library_exports_every_declared_symbol(psc):
    lib = C.CDLL(psc.LIB_PATH)
    for n in declared():
        assert hasattr(lib, n), n
    assert sorted(psc.EXPORTS) == declared()


def test_version_string(psc):
    assert "gfx950" in psc.psc_version()


def _cfg(psc, **kw):
    c = psc.Config(grid_n=1024, support=16, oversample=4, image_samples=0, cell_rad=7e-6,
                   dish_diam_m=25.0, illum=0, gauss_sigma_ld=1.0, squint_frac=0.0, taper_width=8,
                   taper_beta=0.0, device=0)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


@pytest.mark.parametrize("bad", [
    dict(grid_n=1000), dict(grid_n=32), dict(support=12), dict(oversample=0),
    dict(image_samples=15), dict(image_samples=40), dict(cell_rad=0.0), dict(dish_diam_m=-1.0),
    dict(illum=2), dict(illum=3), dict(taper_width=16), dict(illum=1, gauss_sigma_ld=0.0),
])
def test_create_rejects_invalid_config(psc, bad):
    with pytest.raises(psc.PscError) as ei:
        psc.psc_create(_cfg(psc, **bad))
    assert ei.value.status == -1


@pytest.mark.parametrize("over", [1, 2, 4, 8, 16])
def test_support32_fits_every_image_sample_count(psc, over):
    """Support 32 at the most image samples (M = 2S) fits the window form's LDS
    at every oversampling: create gets past its configuration checks (here,
    without a GPU, to the device selection)."""
    try:
        ctx = psc.psc_create(_cfg(psc, support=32, oversample=over, image_samples=64))
    except psc.PscError as e:
        assert e.status != -4, str(e)
        assert "device" in str(e)
    else:
        psc.psc_destroy(ctx)


def _aperture_cfg(psc, ap, **kw):
    ap = np.ascontiguousarray(ap, dtype=np.float64)
    return _cfg(psc, illum=2, aperture_n=ap.shape[0], aperture=ap.ctypes.data, **kw), ap


def test_measured_aperture_validation(psc):
    """illum 2 takes a real, even aperture with a positive sum and at most
    256 cells per side; a valid one gets past the configuration checks
    (here, without a GPU, to the device selection)."""
    from paper_1709_08681_amd import synth
    good = synth.measured_aperture(seed=1)
    uneven = good.copy()
    uneven[4, 9] += 0.25
    nonfinite = good.copy()
    nonfinite[0, 0] = nonfinite[-1, -1] = np.nan
    for bad in (uneven, nonfinite, -good, np.zeros((8, 8)), np.ones((257, 257))):
        cfg, keep = _aperture_cfg(psc, bad)
        with pytest.raises(psc.PscError) as ei:
            psc.psc_create(cfg)
        assert ei.value.status == -1
    cfg, keep = _aperture_cfg(psc, good)
    try:
        ctx = psc.psc_create(cfg)
    except psc.PscError as e:
        assert e.status != -1 or "device" in str(e), str(e)
    else:
        psc.psc_destroy(ctx)


def test_null_arguments(psc):
    lib = psc.load()
    assert lib.psc_create(None, None) == -1
    assert lib.psc_destroy(None) == 0
    assert lib.psc_obs_destroy(None) == 0
    assert lib.psc_set_model(None, None, None) == -1
    assert lib.psc_predict(None, None, None, None, None) == -1
    assert lib.psc_last_error(None) is not None
    assert lib.psc_set_beam_scale(None, None, None, None) == -1
    assert lib.psc_get_beam_scale(None, None, None, None) == -1
    assert lib.psc_scale_gradient(None, None, None, None, None, None, None) == -1
    assert lib.psc_scale_step(None, None, None, 0.5, None, None, None) == -1
    assert lib.psc_image_gradient(None, None, None, None, None, None, None, None) == -1
