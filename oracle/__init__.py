"""FP64 direct-summation oracle for the Pointing SelfCal hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product library never does.  It
shares no code with the HIP path.  The C source (psc_oracle.c) is compiled
with gcc into ``oracle/_build/liboracle.so`` by :func:`build`.

Every function here is a thin ctypes marshaller around the C oracle, which
evaluates the measurement equation (Sec. 2, Eq. ME / Eq. MEDD) by direct
summation over sky pixels, its analytic offset derivative (Eq. DA), the
per-antenna sums of Eq. DCHIDD and the damped update of Sec. 2.2.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "psc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, FP64, no fast-math)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Problem(C.Structure):
    _fields_ = [
        ("n_src", C.c_int32),
        ("src_l", C.POINTER(C.c_double)),
        ("src_m", C.POINTER(C.c_double)),
        ("src_flux", C.POINTER(C.c_double)),
        ("n_ant", C.c_int32), ("n_chan", C.c_int32), ("n_pol", C.c_int32), ("n_int", C.c_int32),
        ("n_row", C.c_int64),
        ("int_row_ptr", C.POINTER(C.c_int64)),
        ("ant1", C.POINTER(C.c_int32)),
        ("ant2", C.POINTER(C.c_int32)),
        ("uv_m", C.POINTER(C.c_double)),
        ("freq_hz", C.POINTER(C.c_double)),
        ("dish_diam_m", C.c_double),
        ("illum", C.c_int32),
        ("gauss_sigma_ld", C.c_double),
        ("squint_frac", C.c_double),
        ("snap_scale", C.c_double),
        ("par_angle", C.POINTER(C.c_double)),
        ("w_m", C.POINTER(C.c_double)),
        ("aperture_n", C.c_int32),
        ("aperture", C.POINTER(C.c_double)),
        ("n_apertures", C.c_int32),
        ("ant_aperture", C.POINTER(C.c_int32)),
        ("beam_scale", C.POINTER(C.c_double)),
    ]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build(force=False)
            lib = C.CDLL(_LIB_PATH)
            P = C.POINTER(_Problem)
            dp = C.POINTER(C.c_double)
            ip = C.POINTER(C.c_int32)
            lib.oracle_efp.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                       C.c_double, dp]
            lib.oracle_efp_aperture.argtypes = [C.c_int, dp, C.c_double, C.c_double, C.c_double,
                                                C.c_double, dp]
            lib.oracle_hpbw.argtypes = [C.c_double, C.c_double]
            lib.oracle_hpbw.restype = C.c_double
            lib.oracle_snap_uv.argtypes = [P, C.c_int64, C.c_int, dp]
            lib.oracle_predict.argtypes = [P, dp, dp, dp]
            lib.oracle_predict_scale.argtypes = [P, dp, dp, dp]
            lib.oracle_scale_gradient.argtypes = [P, dp, dp, dp, dp]
            lib.oracle_scale_step.argtypes = [C.c_int, C.c_int, C.c_int, dp, C.c_double, dp, ip, dp]
            lib.oracle_gradient.argtypes = [P, dp, dp, dp, dp, dp]
            lib.oracle_image_gradient.argtypes = [P, dp, dp, dp, C.c_int, dp, dp, dp]
            lib.oracle_solve_step.argtypes = [C.c_int, C.c_int, C.c_int, dp, C.c_double, C.c_double, dp, ip,
                                              dp, ip]
            lib.oracle_solve.argtypes = [P, dp, dp, dp, C.c_double, C.c_int, C.c_double, ip]
            lib.oracle_efp_defocus.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                               C.c_double, C.c_double, dp]
            lib.oracle_predict_defocus.argtypes = [P, dp, dp, dp, dp]
            lib.oracle_defocus_gradient.argtypes = [P, dp, dp, dp, dp, dp]
            lib.oracle_defocus_step.argtypes = [C.c_int, C.c_int, C.c_int, dp, C.c_double, dp, ip, dp]
            for name in ("oracle_predict", "oracle_predict_scale", "oracle_scale_gradient", "oracle_scale_step",
                         "oracle_gradient", "oracle_image_gradient",
                         "oracle_solve_step", "oracle_solve", "oracle_predict_defocus",
                         "oracle_defocus_gradient", "oracle_defocus_step",
                         "oracle_num_threads"):
                getattr(lib, name).restype = C.c_int
            _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32)) if a is not None else None


class Problem:
    """Plain-array description of a data set for the oracle.

    ``src_l, src_m, src_flux``: non-zero sky pixels; ``uv_m``: [n_row, 2];
    ``int_row_ptr``: [n_int+1]; ``freq_hz``: [n_chan].  ``snap_scale`` > 0
    rounds uv (in wavelengths) to the lattice 1/snap_scale.  ``w_m``: [n_row]
    baseline w in metres for the w-term (None: w = 0).  ``aperture``: a
    square, real, even aperture illumination across the dish for the
    measured-aperture mode (illum 2), or a stack [n_ap, n, n] of them for a
    heterogeneous array with ``ant_aperture`` [n_ant] naming each antenna's
    (None: the first for all).  ``beam_scale``: [n_int, n_pol, n_ant]
    beam-width scale sigma of each antenna, E = E0(d / sigma) (None: 1).
    """

    def __init__(self, src_l, src_m, src_flux, n_ant, ant1, ant2, uv_m, int_row_ptr, freq_hz,
                 n_pol=1, dish_diam_m=25.0, illum=0, gauss_sigma_ld=1.0, squint_frac=0.0,
                 snap_scale=0.0, par_angle=None, w_m=None, aperture=None, beam_scale=None,
                 ant_aperture=None):
        self.src_l = np.ascontiguousarray(src_l, np.float64)
        self.src_m = np.ascontiguousarray(src_m, np.float64)
        self.src_flux = np.ascontiguousarray(src_flux, np.float64)
        self.ant1 = np.ascontiguousarray(ant1, np.int32)
        self.ant2 = np.ascontiguousarray(ant2, np.int32)
        self.uv_m = np.ascontiguousarray(uv_m, np.float64).reshape(-1, 2)
        self.int_row_ptr = np.ascontiguousarray(int_row_ptr, np.int64)
        self.freq_hz = np.ascontiguousarray(freq_hz, np.float64)
        self.n_ant = int(n_ant)
        self.n_pol = int(n_pol)
        self.n_int = int(self.int_row_ptr.shape[0] - 1)
        self.n_row = int(self.ant1.shape[0])
        self.n_chan = int(self.freq_hz.shape[0])
        # per-row parallactic angle: offsets are then in the mount frame
        self.par_angle = None if par_angle is None else np.ascontiguousarray(par_angle, np.float64)
        if self.par_angle is not None and self.par_angle.shape != (self.n_row,):
            raise ValueError("par_angle must have one value per row")
        self.w_m = None if w_m is None else np.ascontiguousarray(w_m, np.float64)
        if self.w_m is not None and self.w_m.shape != (self.n_row,):
            raise ValueError("w_m must have one value per row")
        self.aperture = None if aperture is None else np.ascontiguousarray(aperture, np.float64)
        if (self.aperture is not None) != (int(illum) == 2):
            raise ValueError("the measured-aperture mode (illum 2) takes an aperture, and only it")
        if self.aperture is not None and self.aperture.ndim == 2:
            self.aperture = self.aperture[None]
        if self.aperture is not None and (self.aperture.ndim != 3 or
                                          self.aperture.shape[1] != self.aperture.shape[2]):
            raise ValueError("aperture must be square, or a stack of square apertures")
        self.ant_aperture = None if ant_aperture is None else np.ascontiguousarray(ant_aperture, np.int32)
        if self.ant_aperture is not None and (self.aperture is None or self.ant_aperture.shape != (self.n_ant,)):
            raise ValueError("ant_aperture takes one index per antenna, with an aperture stack")
        self.beam_scale = None if beam_scale is None else np.ascontiguousarray(beam_scale, np.float64)
        if self.beam_scale is not None and self.beam_scale.shape != (self.n_int, self.n_pol, self.n_ant):
            raise ValueError("beam_scale must be [n_int, n_pol, n_ant]")
        self._s = _Problem(
            int(self.src_flux.shape[0]), _dp(self.src_l), _dp(self.src_m), _dp(self.src_flux),
            self.n_ant, self.n_chan, self.n_pol, self.n_int, self.n_row,
            self.int_row_ptr.ctypes.data_as(C.POINTER(C.c_int64)), _ip(self.ant1), _ip(self.ant2),
            _dp(self.uv_m), _dp(self.freq_hz), float(dish_diam_m), int(illum), float(gauss_sigma_ld),
            float(squint_frac), float(snap_scale),
            None if self.par_angle is None else _dp(self.par_angle),
            None if self.w_m is None else _dp(self.w_m),
            0 if self.aperture is None else int(self.aperture.shape[1]),
            None if self.aperture is None else _dp(self.aperture),
            0 if self.aperture is None else int(self.aperture.shape[0]),
            None if self.ant_aperture is None else _ip(self.ant_aperture),
            None if self.beam_scale is None else _dp(self.beam_scale))

    @classmethod
    def from_observation(cls, obs, snap=True, mount_frame=False, w_term=False, **kw):
        """mount_frame: offsets in the antenna mount frame, carried onto the
        sky by each row's parallactic angle; w_term: with each row's w."""
        l, m, f = obs.sky_lm()
        args = dict(n_pol=obs.n_pol, dish_diam_m=obs.wl.dish_diam_m, squint_frac=obs.wl.squint_frac,
                    snap_scale=obs.snap_scale if snap else 0.0,
                    par_angle=obs.par_angle if mount_frame else None,
                    w_m=obs.w_m if w_term else None)
        args.update(kw)
        return cls(l, m, f, obs.n_ant, obs.ant1, obs.ant2, obs.uv_m, obs.int_row_ptr, obs.freq_hz,
                   **args)

    @property
    def ref(self):
        return C.byref(self._s)

    def offsets_shape(self):
        return (self.n_int, self.n_pol, self.n_ant, 2)

    def vis_shape(self):
        return (self.n_row, self.n_chan, self.n_pol)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def efp(illum, dish_diam_m, gauss_sigma_ld, freq_hz, dl, dm):
    """(E, dE/dp_l, dE/dp_m) of one antenna at sky offset (dl, dm) = l - p."""
    lib = _load()
    out = np.zeros(3)
    lib.oracle_efp(int(illum), float(dish_diam_m), float(gauss_sigma_ld), float(freq_hz),
                   float(dl), float(dm), _dp(out))
    return out


def efp_aperture(aperture, dish_diam_m, freq_hz, dl, dm):
    """(E, dE/dc_l, dE/dc_m) of a measured aperture's pattern at displacement
    (dl, dm) from the beam centre c, in the mount frame."""
    lib = _load()
    ap = np.ascontiguousarray(aperture, np.float64)
    out = np.zeros(3)
    lib.oracle_efp_aperture(int(ap.shape[0]), _dp(ap), float(dish_diam_m), float(freq_hz), float(dl),
                            float(dm), _dp(out))
    return out


def hpbw(freq_hz, dish_diam_m):
    return _load().oracle_hpbw(float(freq_hz), float(dish_diam_m))


def snap_uv(prob: Problem, row: int, chan: int):
    out = np.zeros(2)
    _load().oracle_snap_uv(prob.ref, int(row), int(chan), _dp(out))
    return out


def _offs(prob, offsets):
    o = np.ascontiguousarray(offsets, np.float64)
    if o.shape != prob.offsets_shape():
        raise ValueError(f"offsets shape {o.shape} != {prob.offsets_shape()}")
    return o


def predict(prob: Problem, offsets, want_grad=False):
    """Model visibilities [n_row, n_chan, n_pol] complex128 and, if asked, their
    derivatives [n_row, n_chan, n_pol, 4] (d/dl_i, d/dm_i, d/dl_j, d/dm_j)."""
    lib = _load()
    o = _offs(prob, offsets)
    vis = np.zeros(prob.vis_shape() + (2,))
    dvis = np.zeros(prob.vis_shape() + (4, 2)) if want_grad else None
    _check(lib.oracle_predict(prob.ref, _dp(o), _dp(vis), _dp(dvis)), "predict")
    v = vis[..., 0] + 1j * vis[..., 1]
    if want_grad:
        return v, dvis[..., 0] + 1j * dvis[..., 1]
    return v


def gradient(prob: Problem, offsets, vis_obs, weight, want_model=False):
    """Per-antenna sums [n_int, n_pol, n_ant, 6] = chi, g_l, g_m, H_ll, H_lm, H_mm."""
    lib = _load()
    o = _offs(prob, offsets)
    vo = np.ascontiguousarray(np.broadcast_to(vis_obs, prob.vis_shape()), np.complex128)
    vo2 = np.ascontiguousarray(vo.view(np.float64))
    w = np.ascontiguousarray(np.broadcast_to(weight, prob.vis_shape()), np.float64)
    acc = np.zeros(prob.offsets_shape()[:3] + (6,))
    vm = np.zeros(prob.vis_shape() + (2,)) if want_model else None
    _check(lib.oracle_gradient(prob.ref, _dp(o), _dp(vo2), _dp(w), _dp(acc), _dp(vm)), "gradient")
    if want_model:
        return acc, vm[..., 0] + 1j * vm[..., 1]
    return acc


def image_gradient(prob: Problem, offsets, vis_obs, weight, pix_l, pix_m):
    """d chi^2 / d I at the sky positions (pix_l[k], pix_m[k]) (direction
    cosines): minus twice the weighted residual seen through both offset
    beams, summed over every visibility."""
    lib = _load()
    o = _offs(prob, offsets)
    vo = np.ascontiguousarray(np.broadcast_to(vis_obs, prob.vis_shape()), np.complex128)
    vo2 = np.ascontiguousarray(vo.view(np.float64))
    w = np.ascontiguousarray(np.broadcast_to(weight, prob.vis_shape()), np.float64)
    pl = np.ascontiguousarray(pix_l, np.float64).reshape(-1)
    pm = np.ascontiguousarray(pix_m, np.float64).reshape(-1)
    out = np.zeros(pl.shape[0])
    _check(lib.oracle_image_gradient(prob.ref, _dp(o), _dp(vo2), _dp(w), int(pl.shape[0]), _dp(pl),
                                     _dp(pm), _dp(out)), "image_gradient")
    return out


def solve_step(acc, gain, offsets, done=None, mu=0.0):
    """Returns (new offsets, not_updated [n_int,n_pol,n_ant], max_step [n_int]).
    mu >= 0 damps the diagonal of each 2x2 normal matrix (H + mu diag H)."""
    lib = _load()
    acc = np.ascontiguousarray(acc, np.float64)
    n_int, n_pol, n_ant = acc.shape[:3]
    o = np.array(offsets, dtype=np.float64, copy=True, order="C")
    nu = np.zeros((n_int, n_pol, n_ant), np.int32)
    mx = np.zeros(n_int)
    d = None if done is None else np.ascontiguousarray(done, np.int32)
    _check(lib.oracle_solve_step(n_int, n_pol, n_ant, _dp(acc), float(gain), float(mu), _dp(o), _ip(nu),
                                 _dp(mx), _ip(d)), "solve_step")
    return o, nu, mx


def predict_scale(prob: Problem, offsets):
    """Model visibilities and their derivatives with respect to the two
    antennas' beam-width scales, [n_row, n_chan, n_pol, 2] (d/dsigma_i,
    d/dsigma_j)."""
    lib = _load()
    o = _offs(prob, offsets)
    vis = np.zeros(prob.vis_shape() + (2,))
    ds = np.zeros(prob.vis_shape() + (2, 2))
    _check(lib.oracle_predict_scale(prob.ref, _dp(o), _dp(vis), _dp(ds)), "predict_scale")
    return vis[..., 0] + 1j * vis[..., 1], ds[..., 0] + 1j * ds[..., 1]


def scale_gradient(prob: Problem, offsets, vis_obs, weight):
    """Per-antenna sums [n_int, n_pol, n_ant, 3] = chi, g_sigma, H_sigma for the
    beam-width scales the problem carries."""
    lib = _load()
    o = _offs(prob, offsets)
    vo = np.ascontiguousarray(np.broadcast_to(vis_obs, prob.vis_shape()), np.complex128)
    vo2 = np.ascontiguousarray(vo.view(np.float64))
    w = np.ascontiguousarray(np.broadcast_to(weight, prob.vis_shape()), np.float64)
    acc = np.zeros(prob.offsets_shape()[:3] + (3,))
    _check(lib.oracle_scale_gradient(prob.ref, _dp(o), _dp(vo2), _dp(w), _dp(acc)), "scale_gradient")
    return acc


def scale_step(acc3, gain, scale):
    """Returns (new scales, not_updated, max_step [n_int])."""
    lib = _load()
    acc3 = np.ascontiguousarray(acc3, np.float64)
    n_int, n_pol, n_ant = acc3.shape[:3]
    s = np.array(scale, dtype=np.float64, copy=True, order="C")
    nu = np.zeros((n_int, n_pol, n_ant), np.int32)
    mx = np.zeros(n_int)
    _check(lib.oracle_scale_step(n_int, n_pol, n_ant, _dp(acc3), float(gain), _dp(s), _ip(nu), _dp(mx)),
           "scale_step")
    return s, nu, mx


def solve(prob: Problem, vis_obs, weight, offsets0, gain=0.5, n_max=10, tol_rad=None):
    """Algorithm 1: returns (offsets, iterations per interval)."""
    from math import pi
    lib = _load()
    if tol_rad is None:
        tol_rad = 1e-3 * pi / (180 * 3600)
    o = np.array(_offs(prob, offsets0), dtype=np.float64, copy=True, order="C")
    vo = np.ascontiguousarray(np.broadcast_to(vis_obs, prob.vis_shape()), np.complex128)
    vo2 = np.ascontiguousarray(vo.view(np.float64))
    w = np.ascontiguousarray(np.broadcast_to(weight, prob.vis_shape()), np.float64)
    its = np.zeros(prob.n_int, np.int32)
    _check(lib.oracle_solve(prob.ref, _dp(vo2), _dp(w), _dp(o), float(gain), int(n_max),
                            float(tol_rad), _ip(its)), "solve")
    return o, its


def efp_defocus(illum, dish_diam_m, gauss_sigma_ld, freq_hz, delta, dl, dm):
    """(E, dE/ddelta) of the pattern with an aperture defocus delta (radians
    at the rim), complex, at displacement (dl, dm) from the beam centre."""
    out = np.zeros(4)
    _load().oracle_efp_defocus(int(illum), float(dish_diam_m), float(gauss_sigma_ld), float(freq_hz),
                               float(delta), float(dl), float(dm), _dp(out))
    return out[0] + 1j * out[1], out[2] + 1j * out[3]


def _defocus(prob, defocus):
    return np.ascontiguousarray(np.broadcast_to(defocus, prob.offsets_shape()[:3]), np.float64)


def predict_defocus(prob: Problem, offsets, defocus):
    """Model visibilities with every antenna's defocus [n_int, n_pol, n_ant]
    and their derivatives [n_row, n_chan, n_pol, 2] (d/ddelta_i, d/ddelta_j)."""
    lib = _load()
    o = _offs(prob, offsets)
    d = _defocus(prob, defocus)
    vis = np.zeros(prob.vis_shape() + (2,))
    dd = np.zeros(prob.vis_shape() + (2, 2))
    _check(lib.oracle_predict_defocus(prob.ref, _dp(o), _dp(d), _dp(vis), _dp(dd)), "predict_defocus")
    return vis[..., 0] + 1j * vis[..., 1], dd[..., 0] + 1j * dd[..., 1]


def defocus_gradient(prob: Problem, offsets, defocus, vis_obs, weight):
    """Per-antenna sums [n_int, n_pol, n_ant, 3] = chi, g_delta, H_delta."""
    lib = _load()
    o = _offs(prob, offsets)
    d = _defocus(prob, defocus)
    vo = np.ascontiguousarray(np.broadcast_to(vis_obs, prob.vis_shape()), np.complex128)
    vo2 = np.ascontiguousarray(vo.view(np.float64))
    w = np.ascontiguousarray(np.broadcast_to(weight, prob.vis_shape()), np.float64)
    acc = np.zeros(prob.offsets_shape()[:3] + (3,))
    _check(lib.oracle_defocus_gradient(prob.ref, _dp(o), _dp(d), _dp(vo2), _dp(w), _dp(acc)),
           "defocus_gradient")
    return acc


def defocus_step(acc3, gain, defocus):
    """Returns (new defocus, not_updated, max_step [n_int])."""
    lib = _load()
    acc3 = np.ascontiguousarray(acc3, np.float64)
    n_int, n_pol, n_ant = acc3.shape[:3]
    d = np.array(defocus, dtype=np.float64, copy=True, order="C")
    nu = np.zeros((n_int, n_pol, n_ant), np.int32)
    mx = np.zeros(n_int)
    _check(lib.oracle_defocus_step(n_int, n_pol, n_ant, _dp(acc3), float(gain), _dp(d), _ip(nu), _dp(mx)),
           "defocus_step")
    return d, nu, mx


def num_threads():
    return _load().oracle_num_threads()
