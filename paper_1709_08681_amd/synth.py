"""Seeded synthetic workloads for the Pointing SelfCal hot path.

This module makes inputs only: antenna layouts, baseline (u, v) tracks,
frequencies, solution-interval cut points, a pixelised sky model and the
injected pointing offsets.  It holds none of the method's arithmetic (no
beams, no prediction, no gradients); the oracle and the HIP library both take
what it returns as plain arrays.

The workloads mirror the paper's test setting (Sec. 4.1: a 27-antenna array
at L band, a sky of compact sources spread over the primary beam, pointing
offsets of about 1% of the beam width, 10 s integrations, solution intervals
of tens of seconds) at the sizes of the five benchmark configurations.  The
paper's own sky model and data are not available, so every input is drawn
from a stated random recipe instead.

Conventions
-----------
* Pixel (ix, iy) of the N x N model image sits at direction cosines
  l = (ix - N/2) * cell, m = (iy - N/2) * cell; the image array is indexed
  [ix, iy].
* Baseline vector of row (i, j) is position_j - position_i, projected with the
  standard equatorial transform for hour angle H and declination dec at the
  array latitude; w is returned separately (``Observation.w_m``) and used
  only when the w-term is asked for.
* The field of view FoV = N * cell is chosen from the kernel support:
  FoV = 0.98 (S - W_c) lambda_min / (2 D), so that the support of one
  baseline's uv kernel plus the anti-aliasing taper fits in S cells.
* Sources lie on pixel centres inside the central half of the image.
* Offsets are in radians, shaped [n_int, n_pol, n_ant, 2] (l, m).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

C_LIGHT = 299792458.0
ARCSEC = math.pi / (180.0 * 3600.0)
OMEGA_EARTH = 7.2921159e-5  # rad / s, sidereal rate


@dataclass
class Workload:
    """Recipe for one synthetic workload (sizes and distributions)."""

    name: str
    n_ant: int
    layout: str  # "disk" (uniform in area) or "y" (three log-spaced arms)
    layout_radius_m: float
    n_time: int
    dt_s: float
    freqs_hz: np.ndarray
    n_pol: int = 1
    dec_deg: float = 30.0
    lat_deg: float = 34.08
    interval_lengths: list | None = None  # timesteps per interval; None = one interval
    grid_n: int = 1024
    support: int = 16
    oversample: int = 4
    es_width: int = 8
    dish_diam_m: float = 25.0
    n_src: int = 4
    flux_model: str = "unit"  # "unit" (1 Jy each) or "lognormal" (median 10 mJy)
    src_radius: str = "safe"  # "hpbw2": within HPBW/2 at the first channel; "safe": central half
    offset_sigma_arcsec: float = 20.0
    # if set, offsets drift as a per-antenna random walk (arcsec per axis per
    # sqrt(minute)) and each interval's true offset is the walk's mean over it
    offset_walk_arcsec_per_min: float | None = None
    squint_frac: float = 0.0
    snr: float | None = None
    diffuse_fwhm_arcmin: float | None = None
    diffuse_peak_jy: float = 1e-3
    fov_frac: float = 1.0

    @property
    def n_bl(self) -> int:
        return self.n_ant * (self.n_ant - 1) // 2


def _chan_freqs(n: int, lo: float = 1.0e9, bw: float = 1.0e9) -> np.ndarray:
    return lo + (np.arange(n) + 0.5) * bw / n


def workload(k: int, **overrides) -> Workload:
    """The five benchmark workloads (k = 1..5)."""
    if k == 1:
        w = Workload("tiny", n_ant=10, layout="disk", layout_radius_m=1000.0, n_time=20, dt_s=30.0,
                     freqs_hz=np.array([1.4e9]), n_src=4, flux_model="unit", src_radius="hpbw2",
                     offset_sigma_arcsec=20.0, snr=100.0)
    elif k == 2:
        w = Workload("single_interval", n_ant=27, layout="y", layout_radius_m=21000.0, n_time=360,
                     dt_s=10.0, freqs_hz=_chan_freqs(16), n_src=200, flux_model="lognormal",
                     offset_sigma_arcsec=30.0)
    elif k == 3:
        w = Workload("batched", n_ant=27, layout="y", layout_radius_m=21000.0, n_time=0, dt_s=10.0,
                     freqs_hz=_chan_freqs(16), grid_n=2048, n_src=200, flux_model="lognormal",
                     offset_sigma_arcsec=30.0)
        rng = np.random.default_rng(1000 + k)
        w.interval_lengths = [int(x) for x in rng.integers(10, 121, size=256)]
    elif k == 4:
        w = Workload("differentiation", n_ant=64, layout="disk", layout_radius_m=5000.0, n_time=240,
                     dt_s=10.0, freqs_hz=_chan_freqs(64), grid_n=2048, n_src=1000,
                     flux_model="lognormal", offset_sigma_arcsec=30.0, diffuse_fwhm_arcmin=5.0)
    elif k == 5:
        w = Workload("large", n_ant=128, layout="disk", layout_radius_m=5000.0, n_time=600, dt_s=10.0,
                     freqs_hz=_chan_freqs(256), n_pol=2, grid_n=4096, support=32, oversample=8,
                     n_src=1000, flux_model="lognormal", offset_walk_arcsec_per_min=5.0,
                     squint_frac=0.03)
        rng = np.random.default_rng(1000 + k)
        cuts = np.sort(rng.choice(np.arange(1, 600), size=63, replace=False))
        w.interval_lengths = [int(x) for x in np.diff(np.concatenate([[0], cuts, [600]]))]
    else:
        raise ValueError(f"no workload {k}")
    for key, val in overrides.items():
        if not hasattr(w, key):
            raise AttributeError(key)
        setattr(w, key, val)
    if w.interval_lengths is not None:
        w.n_time = int(sum(w.interval_lengths))
    return w


@dataclass
class Observation:
    """Arrays of one synthetic workload (host, numpy)."""

    wl: Workload
    ant_pos: np.ndarray  # [n_ant, 2] east, north (m)
    ant1: np.ndarray  # [n_row] int32
    ant2: np.ndarray  # [n_row] int32
    time_idx: np.ndarray  # [n_row] int32
    uv_m: np.ndarray  # [n_row, 2] float64
    int_row_ptr: np.ndarray  # [n_int+1] int64
    freq_hz: np.ndarray  # [n_chan]
    grid_n: int
    cell_rad: float
    src_pix: np.ndarray  # [n_src, 2] int pixel indices (ix, iy)
    src_flux: np.ndarray  # [n_src]
    offsets_true: np.ndarray  # [n_int, n_pol, n_ant, 2] rad
    extra_pix: np.ndarray | None = None  # diffuse component pixels [n, 2]
    extra_flux: np.ndarray | None = None
    seed: int = 0

    # --- derived views -----------------------------------------------------
    @property
    def n_ant(self) -> int:
        return self.wl.n_ant

    @property
    def n_row(self) -> int:
        return int(self.ant1.shape[0])

    @property
    def n_chan(self) -> int:
        return int(self.freq_hz.shape[0])

    @property
    def n_pol(self) -> int:
        return self.wl.n_pol

    @property
    def n_int(self) -> int:
        return int(self.int_row_ptr.shape[0] - 1)

    @property
    def n_vis(self) -> int:
        return self.n_row * self.n_chan * self.n_pol

    @property
    def fov(self) -> float:
        return self.grid_n * self.cell_rad

    @property
    def w_m(self) -> np.ndarray:
        """Baseline w (m) of every row: the component along the phase centre,
        w = cos(dec) cos(H) X - cos(dec) sin(H) Y + sin(dec) Z for the
        equatorial baseline (X, Y, Z) of the local east-north baseline
        (the companion of u and v in the synthesis tracks)."""
        wl = self.wl
        east = self.ant_pos[self.ant2, 0] - self.ant_pos[self.ant1, 0]
        north = self.ant_pos[self.ant2, 1] - self.ant_pos[self.ant1, 1]
        lat, dec = np.radians(wl.lat_deg), np.radians(wl.dec_deg)
        X, Y, Z = -north * np.sin(lat), east, north * np.cos(lat)
        h = OMEGA_EARTH * (self.time_idx - 0.5 * (wl.n_time - 1)) * wl.dt_s
        return np.cos(dec) * np.cos(h) * X - np.cos(dec) * np.sin(h) * Y + np.sin(dec) * Z

    @property
    def par_angle(self) -> np.ndarray:
        """Parallactic angle of every row (rad), from its hour angle, the
        declination and the latitude (textbook spherical astronomy):
        tan q = sin H cos(lat) / (sin(lat) cos(dec) - cos(lat) sin(dec) cos H)."""
        wl = self.wl
        t = (self.time_idx - 0.5 * (wl.n_time - 1)) * wl.dt_s
        h = OMEGA_EARTH * t
        lat, dec = np.radians(wl.lat_deg), np.radians(wl.dec_deg)
        return np.arctan2(np.sin(h) * np.cos(lat),
                          np.sin(lat) * np.cos(dec) - np.cos(lat) * np.sin(dec) * np.cos(h))

    @property
    def snap_scale(self) -> float:
        """uv lattice density (per wavelength): oversample * FoV."""
        return self.wl.oversample * self.fov

    def sky_pixels(self):
        """All non-zero pixels: (ix, iy, flux) with duplicates merged."""
        pix = self.src_pix
        flux = self.src_flux
        if self.extra_pix is not None:
            pix = np.concatenate([pix, self.extra_pix])
            flux = np.concatenate([flux, self.extra_flux])
        key = pix[:, 0].astype(np.int64) * self.grid_n + pix[:, 1]
        uniq, inv = np.unique(key, return_inverse=True)
        f = np.zeros(uniq.shape[0])
        np.add.at(f, inv, flux)
        return (uniq // self.grid_n).astype(np.int64), (uniq % self.grid_n).astype(np.int64), f

    def sky_lm(self):
        """Direction cosines and flux of every non-zero pixel."""
        ix, iy, f = self.sky_pixels()
        n2 = self.grid_n // 2
        return (ix - n2) * self.cell_rad, (iy - n2) * self.cell_rad, f

    def image(self) -> np.ndarray:
        """Dense N x N float64 model image, indexed [ix, iy]."""
        ix, iy, f = self.sky_pixels()
        img = np.zeros((self.grid_n, self.grid_n), dtype=np.float64)
        img[ix, iy] = f
        return img

    def subset(self, ants=None, times=None, chans=None) -> "Observation":
        """A smaller observation: keep rows whose antennas and time index are
        in the given sets and the given channels (interval structure kept)."""
        keep = np.ones(self.n_row, dtype=bool)
        if ants is not None:
            aset = np.asarray(ants)
            keep &= np.isin(self.ant1, aset) & np.isin(self.ant2, aset)
        if times is not None:
            keep &= np.isin(self.time_idx, np.asarray(times))
        rows = np.nonzero(keep)[0]
        row_int = np.searchsorted(self.int_row_ptr, rows, side="right") - 1
        counts = np.bincount(row_int, minlength=self.n_int)
        ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        freq = self.freq_hz if chans is None else self.freq_hz[np.asarray(chans)]
        return Observation(self.wl, self.ant_pos, self.ant1[rows].copy(), self.ant2[rows].copy(),
                           self.time_idx[rows].copy(), self.uv_m[rows].copy(), ptr, freq.copy(),
                           self.grid_n, self.cell_rad, self.src_pix, self.src_flux,
                           self.offsets_true, self.extra_pix, self.extra_flux, self.seed)


def _layout(wl: Workload, rng: np.random.Generator) -> np.ndarray:
    if wl.layout == "disk":
        r = wl.layout_radius_m * np.sqrt(rng.uniform(0.0, 1.0, wl.n_ant))
        th = rng.uniform(0.0, 2 * np.pi, wl.n_ant)
        return np.stack([r * np.sin(th), r * np.cos(th)], axis=1)
    if wl.layout == "y":
        per_arm = wl.n_ant // 3
        if per_arm * 3 != wl.n_ant:
            raise ValueError("Y layout needs a multiple of 3 antennas")
        kk = np.arange(per_arm)
        radii = 50.0 * (wl.layout_radius_m / 50.0) ** (kk / max(per_arm - 1, 1))
        pos = []
        for az in (0.0, 120.0, 240.0):
            a = np.radians(az)
            pos.append(np.stack([radii * np.sin(a), radii * np.cos(a)], axis=1))
        return np.concatenate(pos)
    raise ValueError(wl.layout)


def _uv_tracks(wl: Workload, ant_pos: np.ndarray):
    """Rows (time-major, baseline-minor) with (u, v) in metres."""
    i, j = np.triu_indices(wl.n_ant, k=1)
    east = ant_pos[j, 0] - ant_pos[i, 0]
    north = ant_pos[j, 1] - ant_pos[i, 1]
    lat = np.radians(wl.lat_deg)
    dec = np.radians(wl.dec_deg)
    # local (east, north, up=0) -> equatorial (X, Y, Z)
    X = -north * np.sin(lat)
    Y = east
    Z = north * np.cos(lat)
    t = (np.arange(wl.n_time) - 0.5 * (wl.n_time - 1)) * wl.dt_s
    H = OMEGA_EARTH * t
    sH, cH = np.sin(H)[:, None], np.cos(H)[:, None]
    u = sH * X[None, :] + cH * Y[None, :]
    v = -np.sin(dec) * cH * X[None, :] + np.sin(dec) * sH * Y[None, :] + np.cos(dec) * Z[None, :]
    n_bl = i.shape[0]
    ant1 = np.tile(i, wl.n_time).astype(np.int32)
    ant2 = np.tile(j, wl.n_time).astype(np.int32)
    tidx = np.repeat(np.arange(wl.n_time), n_bl).astype(np.int32)
    uv = np.stack([u.reshape(-1), v.reshape(-1)], axis=1)
    return ant1, ant2, tidx, uv


def fov_for(wl: Workload) -> float:
    """Field of view: the widest whose aperture autocorrelation plus the
    anti-aliasing taper fits the support, times fov_frac (below 1 leaves room
    in the support for the w-term's kernel)."""
    lam_min = C_LIGHT / float(np.max(wl.freqs_hz))
    return wl.fov_frac * 0.98 * (wl.support - wl.es_width) * lam_min / (2.0 * wl.dish_diam_m)


def make_observation(wl: Workload, seed: int) -> Observation:
    rng = np.random.default_rng(seed)
    ant_pos = _layout(wl, rng)
    ant1, ant2, tidx, uv = _uv_tracks(wl, ant_pos)
    n_bl = wl.n_bl
    lengths = wl.interval_lengths or [wl.n_time]
    ptr = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64) * n_bl
    fov = fov_for(wl)
    n = wl.grid_n
    cell = fov / n
    # sources: uniform in area inside a disk, snapped to pixel centres
    if wl.src_radius == "hpbw2":
        rmax = 0.5 * 1.02899 * (C_LIGHT / float(wl.freqs_hz[0])) / wl.dish_diam_m
    else:
        rmax = 0.95 * fov / 4.0
    rmax = min(rmax, 0.95 * fov / 4.0)
    r = rmax * np.sqrt(rng.uniform(0.0, 1.0, wl.n_src))
    th = rng.uniform(0.0, 2 * np.pi, wl.n_src)
    pix = np.stack([np.rint(r * np.cos(th) / cell), np.rint(r * np.sin(th) / cell)], axis=1)
    pix = pix.astype(np.int64) + n // 2
    if wl.flux_model == "unit":
        flux = np.ones(wl.n_src)
    else:
        flux = 0.01 * np.exp(rng.normal(0.0, 1.0, wl.n_src))
    extra_pix = extra_flux = None
    if wl.diffuse_fwhm_arcmin:
        hp = 0.5 * 1.02899 * (C_LIGHT / float(np.mean(wl.freqs_hz))) / wl.dish_diam_m
        rc = min(hp, 0.5 * fov / 4.0) * math.sqrt(rng.uniform())
        tc = rng.uniform(0.0, 2 * np.pi)
        cx, cy = rc * math.cos(tc) / cell, rc * math.sin(tc) / cell
        sig = wl.diffuse_fwhm_arcmin * 60.0 * ARCSEC / (2.0 * math.sqrt(2.0 * math.log(2.0))) / cell
        rcut = sig * math.sqrt(2.0 * math.log(1e9))
        lim = int(math.ceil(rcut)) + 1
        gx, gy = np.meshgrid(np.arange(-lim, lim + 1) + int(round(cx)),
                             np.arange(-lim, lim + 1) + int(round(cy)), indexing="ij")
        d2 = (gx - cx) ** 2 + (gy - cy) ** 2
        val = wl.diffuse_peak_jy * np.exp(-0.5 * d2 / sig ** 2)
        ok = (val >= 1e-9 * wl.diffuse_peak_jy) & (np.abs(gx) < n // 4) & (np.abs(gy) < n // 4)
        extra_pix = np.stack([gx[ok], gy[ok]], axis=1).astype(np.int64) + n // 2
        extra_flux = val[ok]
    n_int = len(lengths)
    if wl.offset_walk_arcsec_per_min:
        step = wl.offset_walk_arcsec_per_min * ARCSEC * math.sqrt(wl.dt_s / 60.0)
        walk = np.cumsum(rng.normal(0.0, step, size=(wl.n_time, wl.n_ant, 2)), axis=0)
        t_ptr = np.concatenate([[0], np.cumsum(lengths)])
        offs = np.stack([walk[t_ptr[s]:t_ptr[s + 1]].mean(axis=0) for s in range(n_int)])[:, None]
    else:
        offs = rng.normal(0.0, wl.offset_sigma_arcsec * ARCSEC, size=(n_int, 1, wl.n_ant, 2))
    offs = np.repeat(offs, wl.n_pol, axis=1)  # mechanical offsets: same for both pols
    return Observation(wl, ant_pos, ant1, ant2, tidx, uv, ptr, np.asarray(wl.freqs_hz, np.float64),
                       n, cell, pix, flux, np.ascontiguousarray(offs), extra_pix, extra_flux, seed)


def make_config(k: int, seed: int | None = None, **overrides) -> Observation:
    """Workload k (1..5) with its default seed (k) unless given."""
    wl = workload(k, **overrides)
    return make_observation(wl, k if seed is None else seed)


def noise(vis: np.ndarray, snr: float, seed: int):
    """Complex Gaussian noise at the given SNR (sigma = rms|vis| / snr), and the
    matching inverse-variance weight 1 / sigma^2."""
    rng = np.random.default_rng(seed)
    sigma = float(np.sqrt(np.mean(np.abs(vis) ** 2))) / snr
    nz = (rng.normal(size=vis.shape) + 1j * rng.normal(size=vis.shape)) * (sigma / math.sqrt(2.0))
    return nz, 1.0 / sigma ** 2


def measured_aperture(n: int = 32, seed: int = 0, blockage_frac: float = 0.08, n_legs: int = 4,
                      leg_width_frac: float = 0.03, leg_angle_deg: float = 45.0, edge_taper: float = 0.3,
                      ripple: float = 0.05) -> np.ndarray:
    """A stand-in for a measured aperture illumination (the paper's VLA beam
    model comes from a simulation of the illumination with blockage and
    taper, which is not available): n x n cells over the square of side D
    centred on the dish axis, [x][y], x along the mount frame's l axis.

    Inside the rim: a parabolic taper falling to ``edge_taper`` at the rim,
    zero inside the central blockage (diameter ``blockage_frac`` D) and
    under ``n_legs`` feed-leg shadows (radial strips of width
    ``leg_width_frac`` D, the first at ``leg_angle_deg`` from +x), and a
    seeded ripple of relative amplitude ``ripple`` standing in for
    measurement noise.  The result is made even, A[a][b] =
    A[n-1-a][n-1-b], so that the far-field pattern is real; the legs make it
    non-circular.
    """
    rng = np.random.default_rng(seed)
    x = (np.arange(n) - 0.5 * (n - 1)) / n  # cell centres in units of D
    X, Y = np.meshgrid(x, x, indexing="ij")
    r = np.hypot(X, Y)
    amp = 1.0 - (1.0 - edge_taper) * (2.0 * r) ** 2
    amp *= 1.0 + ripple * rng.standard_normal((n, n))
    amp[r > 0.5] = 0.0
    amp[r < 0.5 * blockage_frac] = 0.0
    for k in range(n_legs):
        ang = np.radians(leg_angle_deg) + 2.0 * np.pi * k / n_legs
        along = X * np.cos(ang) + Y * np.sin(ang)
        across = -X * np.sin(ang) + Y * np.cos(ang)
        amp[(along > 0.0) & (np.abs(across) < 0.5 * leg_width_frac)] = 0.0
    return 0.5 * (amp + amp[::-1, ::-1])


def perturbed_offsets(obs: Observation, sigma_arcsec: float, seed: int) -> np.ndarray:
    """Truth plus an independent Gaussian perturbation (a starting point)."""
    rng = np.random.default_rng(seed)
    return obs.offsets_true + rng.normal(0.0, sigma_arcsec * ARCSEC, size=obs.offsets_true.shape)
