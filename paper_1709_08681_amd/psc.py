"""Python binding of libpsc (ctypes), plus a small session helper.

Every function named ``psc_*`` marshals arguments for the C entry point of
the same name in ``include/psc.h``; all computation happens in the HIP
kernels of libpsc.so.  PyTorch is used only to own device memory and to pick
the stream.  There is no fallback: if the library has not been built, or no
GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsc.so")

PSC_OK = 0
PSC_E_ARG, PSC_E_HIP, PSC_E_OOM, PSC_E_UNSUPPORTED, PSC_E_STATE = -1, -2, -3, -4, -5
STATUS = {0: "PSC_OK", -1: "PSC_E_ARG", -2: "PSC_E_HIP", -3: "PSC_E_OOM", -4: "PSC_E_UNSUPPORTED",
          -5: "PSC_E_STATE"}
SOLVE_PLAIN, SOLVE_BATCHED, SOLVE_GRAPH = 0, 1, 2
DEGRID_VALU, DEGRID_MFMA, DEGRID_WINDOW = 0, 1, 2
ARCSEC = math.pi / (180.0 * 3600.0)

EXPORTS = ["psc_version", "psc_create", "psc_destroy", "psc_last_error", "psc_set_model",
           "psc_obs_create", "psc_obs_destroy", "psc_obs_info", "psc_obs_launch_info", "psc_predict",
           "psc_gradient", "psc_gradient_noalloc", "psc_predict_vjp", "psc_solve_step", "psc_solve", "psc_set_degrid", "psc_get_degrid",
           "psc_tune", "psc_image_gradient", "psc_set_beam_scale", "psc_get_beam_scale",
           "psc_scale_gradient", "psc_scale_step", "psc_solve_scale", "psc_set_defocus", "psc_get_defocus",
           "psc_defocus_gradient", "psc_defocus_step"]


class PscError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [
        ("grid_n", C.c_int32), ("support", C.c_int32), ("oversample", C.c_int32),
        ("image_samples", C.c_int32), ("cell_rad", C.c_double), ("dish_diam_m", C.c_double),
        ("illum", C.c_int32), ("gauss_sigma_ld", C.c_double), ("squint_frac", C.c_double),
        ("taper_width", C.c_int32), ("taper_beta", C.c_double), ("device", C.c_int32),
        ("aperture_n", C.c_int32), ("aperture", C.c_void_p), ("aperture_count", C.c_int32),
    ]


class LaunchInfo(C.Structure):
    _fields_ = [("degrid", C.c_int32), ("window_waves", C.c_int32), ("samples_per_item", C.c_double),
                ("plan_ms", C.c_double), ("w_planes", C.c_int32), ("tab_nodes", C.c_int32), ("capture_ms", C.c_double),
                ("pattern_tables", C.c_int32), ("items_per_block", C.c_int32)]


class ObsDesc(C.Structure):
    _fields_ = [
        ("n_ant", C.c_int32), ("n_chan", C.c_int32), ("n_pol", C.c_int32), ("n_int", C.c_int32),
        ("n_row", C.c_int64), ("int_row_ptr", C.c_void_p), ("ant1", C.c_void_p),
        ("ant2", C.c_void_p), ("uv_m", C.c_void_p), ("freq_hz", C.c_void_p),
        ("par_angle", C.c_void_p), ("w_m", C.c_void_p), ("ant_aperture", C.c_void_p),
    ]


_lib = None
_lock = threading.Lock()


def load():
    """Load libpsc.so (built in-tree by ``paper_1709_08681_amd.build``)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m "
                               "paper_1709_08681_amd.build` (no CPU fallback exists)")
        lib = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "psc_version": ([], C.c_char_p),
            "psc_create": ([C.POINTER(Config), C.POINTER(vp)], C.c_int),
            "psc_destroy": ([vp], C.c_int),
            "psc_last_error": ([vp], C.c_char_p),
            "psc_set_model": ([vp, vp, vp], C.c_int),
            "psc_obs_create": ([vp, C.POINTER(ObsDesc), C.POINTER(vp)], C.c_int),
            "psc_obs_destroy": ([vp], C.c_int),
            "psc_obs_info": ([vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)], C.c_int),
            "psc_obs_launch_info": ([vp, C.POINTER(LaunchInfo)], C.c_int),
            "psc_predict": ([vp, vp, vp, vp, vp], C.c_int),
            "psc_gradient": ([vp, vp, vp, vp, vp, vp, vp, vp], C.c_int),
            "psc_gradient_noalloc": ([vp, vp, vp, vp, vp, vp, vp, vp], C.c_int),
            "psc_predict_vjp": ([vp, vp, vp, vp, vp, vp], C.c_int),
            "psc_solve_step": ([vp, i32, i32, i32, vp, dbl, dbl, vp, vp, vp, vp], C.c_int),
            "psc_solve": ([vp, vp, vp, vp, vp, dbl, i32, dbl, i32, vp, vp], C.c_int),
            "psc_set_degrid": ([vp, i32], C.c_int),
            "psc_get_degrid": ([vp, C.POINTER(i32)], C.c_int),
            "psc_tune": ([vp, vp, vp, vp, vp, i32, C.POINTER(dbl), vp], C.c_int),
            "psc_image_gradient": ([vp, vp, vp, vp, vp, vp, vp, vp], C.c_int),
            "psc_set_beam_scale": ([vp, vp, vp, vp], C.c_int),
            "psc_get_beam_scale": ([vp, vp, vp, vp], C.c_int),
            "psc_scale_gradient": ([vp, vp, vp, vp, vp, vp, vp], C.c_int),
            "psc_scale_step": ([vp, vp, vp, dbl, vp, vp, vp], C.c_int),
            "psc_solve_scale": ([vp, vp, vp, vp, vp, dbl, i32, dbl, vp, vp], C.c_int),
            "psc_set_defocus": ([vp, vp, vp, vp], C.c_int),
            "psc_get_defocus": ([vp, vp, vp, vp], C.c_int),
            "psc_defocus_gradient": ([vp, vp, vp, vp, vp, vp, vp], C.c_int),
            "psc_defocus_step": ([vp, vp, vp, dbl, vp, vp, vp], C.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
        return lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _check(rc, ctx=None):
    if rc != PSC_OK:
        msg = load().psc_last_error(ctx)
        raise PscError(rc, (msg or b"").decode())


# ---------------------------------------------------------------------------
# thin wrappers, one per C entry point
# ---------------------------------------------------------------------------

def psc_version() -> str:
    return load().psc_version().decode()


def psc_create(cfg: Config):
    h = C.c_void_p()
    _check(load().psc_create(C.byref(cfg), C.byref(h)))
    return h


def psc_destroy(ctx):
    _check(load().psc_destroy(ctx))


def psc_set_model(ctx, image_dev, stream=None):
    _check(load().psc_set_model(ctx, _ptr(image_dev), _stream(stream)), ctx)


def psc_obs_create(ctx, desc: ObsDesc):
    h = C.c_void_p()
    _check(load().psc_obs_create(ctx, C.byref(desc), C.byref(h)), ctx)
    return h


def psc_obs_destroy(obs):
    _check(load().psc_obs_destroy(obs))


def psc_obs_info(obs):
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    _check(load().psc_obs_info(obs, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def psc_obs_launch_info(obs):
    """dict(degrid, window_waves, samples_per_item, plan_ms, w_planes, tab_nodes, capture_ms,
    pattern_tables, items_per_block)."""
    li = LaunchInfo()
    _check(load().psc_obs_launch_info(obs, C.byref(li)))
    return {"degrid": li.degrid, "window_waves": li.window_waves,
            "samples_per_item": li.samples_per_item, "plan_ms": li.plan_ms, "w_planes": li.w_planes,
            "tab_nodes": li.tab_nodes, "capture_ms": li.capture_ms, "pattern_tables": li.pattern_tables,
            "items_per_block": li.items_per_block}


def psc_predict(ctx, obs, offsets_dev, vis_out_dev, stream=None):
    _check(load().psc_predict(ctx, obs, _ptr(offsets_dev), _ptr(vis_out_dev), _stream(stream)), ctx)


def psc_gradient(ctx, obs, offsets_dev, vis_obs_dev, weight_dev, acc_out_dev, vis_model_dev=None,
                 stream=None):
    _check(load().psc_gradient(ctx, obs, _ptr(offsets_dev), _ptr(vis_obs_dev), _ptr(weight_dev),
                               _ptr(acc_out_dev), _ptr(vis_model_dev), _stream(stream)), ctx)


def psc_gradient_noalloc(ctx, obs, offsets_dev, vis_obs_dev, weight_dev, acc_out_dev, vis_model_dev=None,
                         stream=None):
    _check(load().psc_gradient_noalloc(ctx, obs, _ptr(offsets_dev), _ptr(vis_obs_dev), _ptr(weight_dev),
                                       _ptr(acc_out_dev), _ptr(vis_model_dev), _stream(stream)), ctx)


def psc_predict_vjp(ctx, obs, offsets_dev, grad_vis_dev, grad_offsets_dev, stream=None):
    _check(load().psc_predict_vjp(ctx, obs, _ptr(offsets_dev), _ptr(grad_vis_dev),
                                  _ptr(grad_offsets_dev), _stream(stream)), ctx)


def psc_solve_step(ctx, n_int, n_pol, n_ant, acc_dev, gain, lm_mu, offsets_dev, not_updated_dev=None,
                   max_step_dev=None, stream=None):
    _check(load().psc_solve_step(ctx, n_int, n_pol, n_ant, _ptr(acc_dev), float(gain), float(lm_mu),
                                 _ptr(offsets_dev), _ptr(not_updated_dev), _ptr(max_step_dev),
                                 _stream(stream)), ctx)


def psc_solve(ctx, obs, vis_obs_dev, weight_dev, offsets_dev, gain, n_max, tol_rad, form,
              iters_dev=None, stream=None):
    _check(load().psc_solve(ctx, obs, _ptr(vis_obs_dev), _ptr(weight_dev), _ptr(offsets_dev),
                            float(gain), int(n_max), float(tol_rad), int(form), _ptr(iters_dev),
                            _stream(stream)), ctx)


def psc_set_degrid(obs, variant):
    _check(load().psc_set_degrid(obs, int(variant)))


def psc_get_degrid(obs):
    v = C.c_int32()
    _check(load().psc_get_degrid(obs, C.byref(v)))
    return v.value


def psc_image_gradient(ctx, obs, offsets_dev, vis_obs_dev, weight_dev, image_grad_out_dev,
                       vis_model_dev=None, stream=None):
    _check(load().psc_image_gradient(ctx, obs, _ptr(offsets_dev), _ptr(vis_obs_dev), _ptr(weight_dev),
                                     _ptr(image_grad_out_dev), _ptr(vis_model_dev), _stream(stream)),
           ctx)


def psc_set_beam_scale(ctx, obs, scale_dev, stream=None):
    _check(load().psc_set_beam_scale(ctx, obs, _ptr(scale_dev), _stream(stream)), ctx)


def psc_get_beam_scale(ctx, obs, scale_out_dev, stream=None):
    _check(load().psc_get_beam_scale(ctx, obs, _ptr(scale_out_dev), _stream(stream)), ctx)


def psc_scale_gradient(ctx, obs, offsets_dev, vis_obs_dev, weight_dev, acc_out_dev, stream=None):
    _check(load().psc_scale_gradient(ctx, obs, _ptr(offsets_dev), _ptr(vis_obs_dev), _ptr(weight_dev),
                                     _ptr(acc_out_dev), _stream(stream)), ctx)


def psc_scale_step(ctx, obs, acc_dev, gain, not_updated_dev=None, max_step_dev=None, stream=None):
    _check(load().psc_scale_step(ctx, obs, _ptr(acc_dev), float(gain), _ptr(not_updated_dev),
                                 _ptr(max_step_dev), _stream(stream)), ctx)


def psc_solve_scale(ctx, obs, offsets_dev, vis_obs_dev, weight_dev, gain, n_max, tol, iters_dev=None,
                    stream=None):
    _check(load().psc_solve_scale(ctx, obs, _ptr(offsets_dev), _ptr(vis_obs_dev), _ptr(weight_dev), float(gain),
                                  int(n_max), float(tol), _ptr(iters_dev), _stream(stream)), ctx)


def psc_set_defocus(ctx, obs, defocus_dev, stream=None):
    _check(load().psc_set_defocus(ctx, obs, _ptr(defocus_dev), _stream(stream)), ctx)


def psc_get_defocus(ctx, obs, defocus_out_dev, stream=None):
    _check(load().psc_get_defocus(ctx, obs, _ptr(defocus_out_dev), _stream(stream)), ctx)


def psc_defocus_gradient(ctx, obs, offsets_dev, vis_obs_dev, weight_dev, acc_out_dev, stream=None):
    _check(load().psc_defocus_gradient(ctx, obs, _ptr(offsets_dev), _ptr(vis_obs_dev), _ptr(weight_dev),
                                       _ptr(acc_out_dev), _stream(stream)), ctx)


def psc_defocus_step(ctx, obs, acc_dev, gain, not_updated_dev=None, max_step_dev=None, stream=None):
    _check(load().psc_defocus_step(ctx, obs, _ptr(acc_dev), float(gain), _ptr(not_updated_dev),
                                   _ptr(max_step_dev), _stream(stream)), ctx)


def psc_tune(ctx, obs, offsets_dev, vis_obs_dev, weight_dev, repeats=3, stream=None):
    """Returns the mean launch time (us) of each degrid variant (-1 where the
    support does not allow it); the observation keeps the fastest."""
    t = (C.c_double * 3)()
    _check(load().psc_tune(ctx, obs, _ptr(offsets_dev), _ptr(vis_obs_dev), _ptr(weight_dev),
                           int(repeats), t, _stream(stream)), ctx)
    return list(t)


# ---------------------------------------------------------------------------
# session: one context + one planned observation, from a synthetic Observation
# ---------------------------------------------------------------------------

def config_for(obs, device=0, aperture=None, **kw) -> Config:
    """Config of a synthetic observation; ``aperture`` (a square float64
    array, or a stack [count, n, n] of them, kept alive by the caller until
    psc_create returns) selects the measured-aperture mode (illum 2)."""
    wl = obs.wl
    cfg = Config(grid_n=obs.grid_n, support=wl.support, oversample=wl.oversample, image_samples=0,
                 cell_rad=obs.cell_rad, dish_diam_m=wl.dish_diam_m, illum=0, gauss_sigma_ld=1.0,
                 squint_frac=wl.squint_frac, taper_width=wl.es_width, taper_beta=0.0, device=device,
                 aperture_n=0, aperture=None, aperture_count=0)
    if aperture is not None:
        cfg.illum = 2
        cfg.aperture_n = int(aperture.shape[-1])
        cfg.aperture = aperture.ctypes.data
        cfg.aperture_count = int(aperture.shape[0]) if aperture.ndim == 3 else 1
    for k, v in kw.items():
        setattr(cfg, k, v)
    return cfg


class Session:
    """Context + planned observation living on one GPU.

    ``obs`` is a :class:`paper_1709_08681_amd.synth.Observation`.  Device
    tensors of the geometry are kept alive for the session's lifetime.  With
    ``mount_frame`` the offsets are in the antenna mount frame and every row's
    parallactic angle (``obs.par_angle``) carries them onto the sky; with
    ``w_term`` every row's w (``obs.w_m``) enters the measurement equation;
    ``aperture`` (square, real, even) gives every antenna that measured
    aperture illumination, whose pattern turns with the mount; a stack
    [count, n, n] with ``ant_aperture`` [n_ant] gives each antenna its own
    (a heterogeneous array).
    """

    def __init__(self, obs, device=0, image=None, mount_frame=False, w_term=False, aperture=None,
                 ant_aperture=None, **cfg_overrides):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libpsc needs a ROCm GPU; none is visible")
        self.torch = torch
        self.dev = torch.device("cuda", device)
        self.obs = obs
        ap = None if aperture is None else np.ascontiguousarray(aperture, dtype=np.float64)
        if ap is not None and (ap.ndim not in (2, 3) or ap.shape[-2] != ap.shape[-1]):
            raise ValueError("aperture must be a square array or a stack of them")
        self.cfg = config_for(obs, device=device, aperture=ap, **cfg_overrides)
        self.ctx = psc_create(self.cfg)
        self.cfg.aperture = None  # read by psc_create only
        self.handle = None
        try:
            img = obs.image() if image is None else image
            self.image = torch.as_tensor(np.ascontiguousarray(img), dtype=torch.float64, device=self.dev)
            psc_set_model(self.ctx, self.image)
            t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=self.dev)
            self.g_ptr = t(obs.int_row_ptr, torch.int64)
            self.g_a1 = t(obs.ant1, torch.int32)
            self.g_a2 = t(obs.ant2, torch.int32)
            self.g_uv = t(obs.uv_m, torch.float64)
            self.g_fr = t(obs.freq_hz, torch.float64)
            # mount-frame offsets: every row's parallactic angle
            self.g_pa = t(obs.par_angle, torch.float64) if mount_frame else None
            self.g_w = t(obs.w_m, torch.float64) if w_term else None
            self.g_apa = None if ant_aperture is None else t(ant_aperture, torch.int32)
            desc = ObsDesc(obs.n_ant, obs.n_chan, obs.n_pol, obs.n_int, obs.n_row,
                           self.g_ptr.data_ptr(), self.g_a1.data_ptr(), self.g_a2.data_ptr(),
                           self.g_uv.data_ptr(), self.g_fr.data_ptr(),
                           self.g_pa.data_ptr() if mount_frame else None,
                           self.g_w.data_ptr() if w_term else None,
                           None if self.g_apa is None else self.g_apa.data_ptr())
            self.handle = psc_obs_create(self.ctx, desc)
        except Exception:
            self.close()
            raise

    # shapes
    @property
    def vis_shape(self):
        return (self.obs.n_row, self.obs.n_chan, self.obs.n_pol)

    @property
    def off_shape(self):
        return (self.obs.n_int, self.obs.n_pol, self.obs.n_ant, 2)

    def info(self):
        return psc_obs_info(self.handle)

    def tensor(self, a, dtype):
        return self.torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=self.dev)

    def offsets(self, a):
        t = self.tensor(a, self.torch.float64)
        if tuple(t.shape) != self.off_shape:
            raise ValueError(f"offsets shape {tuple(t.shape)} != {self.off_shape}")
        return t

    def predict(self, offsets, out=None):
        torch = self.torch
        off = offsets if isinstance(offsets, torch.Tensor) else self.offsets(offsets)
        if out is None:
            out = torch.empty(self.vis_shape, dtype=torch.complex64, device=self.dev)
        psc_predict(self.ctx, self.handle, off, out)
        return out

    def gradient(self, offsets, vis_obs, weight, want_model=False):
        torch = self.torch
        off = offsets if isinstance(offsets, torch.Tensor) else self.offsets(offsets)
        acc = torch.empty(self.off_shape[:3] + (6,), dtype=torch.float64, device=self.dev)
        vm = torch.empty(self.vis_shape, dtype=torch.complex64, device=self.dev) if want_model else None
        psc_gradient(self.ctx, self.handle, off, vis_obs, weight, acc, vm)
        return (acc, vm) if want_model else acc

    def vjp(self, offsets, grad_vis):
        torch = self.torch
        off = offsets if isinstance(offsets, torch.Tensor) else self.offsets(offsets)
        g = torch.empty(self.off_shape, dtype=torch.float64, device=self.dev)
        psc_predict_vjp(self.ctx, self.handle, off, grad_vis.contiguous(), g)
        return g

    def set_beam_scale(self, scale):
        """Beam-width scales [n_int, n_pol, n_ant] (array or device tensor), or
        None for the nominal beams."""
        torch = self.torch
        if scale is None:
            psc_set_beam_scale(self.ctx, self.handle, None)
            return
        sc = scale if isinstance(scale, torch.Tensor) else torch.as_tensor(
            np.ascontiguousarray(scale, dtype=np.float64), device=self.dev)
        psc_set_beam_scale(self.ctx, self.handle, sc.contiguous())

    def beam_scale(self):
        out = self.torch.empty(self.off_shape[:3], dtype=self.torch.float64, device=self.dev)
        psc_get_beam_scale(self.ctx, self.handle, out)
        return out

    def scale_gradient(self, offsets, vis_obs, weight):
        torch = self.torch
        off = offsets if isinstance(offsets, torch.Tensor) else self.offsets(offsets)
        acc = torch.empty(self.off_shape[:3] + (3,), dtype=torch.float64, device=self.dev)
        psc_scale_gradient(self.ctx, self.handle, off, vis_obs, weight, acc)
        return acc

    def scale_step(self, acc, gain=0.5):
        """Returns (not_updated, max_step per interval)."""
        torch = self.torch
        nu = torch.empty(self.off_shape[:3], dtype=torch.int32, device=self.dev)
        mx = torch.empty(self.obs.n_int, dtype=torch.float64, device=self.dev)
        psc_scale_step(self.ctx, self.handle, acc, gain, nu, mx)
        return nu, mx

    def solve_beam_scale(self, offsets, vis_obs, weight, gain=0.5, n_max=30, tol=1e-6):
        """Solve for the beam scales at fixed offsets; returns the steps taken
        per interval (the scales stay on the observation)."""
        torch = self.torch
        off = offsets if isinstance(offsets, torch.Tensor) else self.offsets(offsets)
        its = torch.zeros(self.obs.n_int, dtype=torch.int32, device=self.dev)
        psc_solve_scale(self.ctx, self.handle, off, vis_obs, weight, gain, n_max, tol, its)
        return its

    def set_defocus(self, defocus):
        """Every antenna's aperture defocus [n_int, n_pol, n_ant] (radians at
        the rim), or None for real patterns again."""
        if defocus is None:
            psc_set_defocus(self.ctx, self.handle, None)
            return
        d = self.tensor(np.array(np.broadcast_to(defocus, self.off_shape[:3])), self.torch.float64)
        psc_set_defocus(self.ctx, self.handle, d)

    def defocus(self):
        out = self.torch.empty(self.off_shape[:3], dtype=self.torch.float64, device=self.dev)
        psc_get_defocus(self.ctx, self.handle, out)
        return out

    def defocus_gradient(self, offsets, vis_obs, weight):
        torch = self.torch
        off = offsets if isinstance(offsets, torch.Tensor) else self.offsets(offsets)
        acc = torch.empty(self.off_shape[:3] + (3,), dtype=torch.float64, device=self.dev)
        psc_defocus_gradient(self.ctx, self.handle, off, vis_obs, weight, acc)
        return acc

    def defocus_step(self, acc, gain=0.5):
        torch = self.torch
        nu = torch.empty(self.off_shape[:3], dtype=torch.int32, device=self.dev)
        mx = torch.empty(self.obs.n_int, dtype=torch.float64, device=self.dev)
        psc_defocus_step(self.ctx, self.handle, acc, gain, nu, mx)
        return nu, mx

    def image_gradient(self, offsets, vis_obs, weight):
        """d chi^2 / d I on the model grid, [N][N] float64."""
        torch = self.torch
        off = offsets if isinstance(offsets, torch.Tensor) else self.offsets(offsets)
        n = self.obs.grid_n
        out = torch.empty((n, n), dtype=torch.float64, device=self.dev)
        psc_image_gradient(self.ctx, self.handle, off, vis_obs, weight, out)
        return out

    def solve_step(self, acc, gain, offsets, lm_mu=0.0):
        torch = self.torch
        nu = torch.empty(self.off_shape[:3], dtype=torch.int32, device=self.dev)
        mx = torch.empty(self.obs.n_int, dtype=torch.float64, device=self.dev)
        psc_solve_step(self.ctx, self.obs.n_int, self.obs.n_pol, self.obs.n_ant, acc, gain, lm_mu,
                       offsets, nu, mx)
        return nu, mx

    def solve(self, vis_obs, weight, offsets, gain=0.5, n_max=10, tol_rad=1e-3 * ARCSEC,
              form=SOLVE_GRAPH):
        torch = self.torch
        its = torch.zeros(self.obs.n_int, dtype=torch.int32, device=self.dev)
        psc_solve(self.ctx, self.handle, vis_obs, weight, offsets, gain, n_max, tol_rad, form, its)
        return its

    def close(self):
        if getattr(self, "handle", None):
            psc_obs_destroy(self.handle)
            self.handle = None
        if getattr(self, "ctx", None):
            psc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
