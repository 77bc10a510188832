"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/psc.h, and rejects invalid configurations before touching
a GPU."""
import ctypes as C
import os
import re

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
    dict(illum=2), dict(taper_width=16), dict(illum=1, gauss_sigma_ld=0.0),
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


def test_null_arguments(psc):
    lib = psc.load()
    assert lib.psc_create(None, None) == -1
    assert lib.psc_destroy(None) == 0
    assert lib.psc_obs_destroy(None) == 0
    assert lib.psc_set_model(None, None, None) == -1
    assert lib.psc_predict(None, None, None, None, None) == -1
    assert lib.psc_last_error(None) is not None
