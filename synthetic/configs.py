"""The five benchmark workloads as seeded synthetic observations (inputs only).

Every quantity is fixed by BASE_SEED + the workload index; independent sub-streams
are spawned for the layout, the sky, the noise and the sample excitations so that
changing one does not shift the others.

Workloads (sizes follow the paper's observation tables, Sec. 4):
  0  tiny coplanar: 27 antennas uniform in a 10 km-across disc, 64 integrations
     over 1 h, w := 0, 128^2 sky at 1 arcsec, 22,464 rows, complex128.
  1  VLA-like: 27 antennas on a Y with 21 km arms, 8 h at 10 s (1,010,880 rows),
     w rescaled so max|w| = 0.05 max|uv|, 512^2 sky at 0.05 deg/1024.
  2  as 1 with a batch of 8 log-sky samples.
  3  MeerKAT-like: 64 antennas (core + 3 spirals), 8 h at 8 s (7,257,600 rows),
     16 channels over 0.9-1.7 GHz, 4096^2 sky per channel at 1 arcsec.
  4  served mix: jobs drawn from the layouts above with images in
     {128, 256, 512, 1024, 2048}^2 and 5e4..5e6 visibilities.
"""

from dataclasses import dataclass, field

import numpy as np

from .layouts import (
    C_LIGHT,
    earth_rotation_uvw,
    layout_meerkat_like,
    layout_uniform_disc,
    layout_vla_y,
    n_baselines,
)
from .skies import correlated_field, gaussian_blob, point_sources

BASE_SEED = 240609144
ARCSEC = np.pi / (180.0 * 3600.0)


def config_rng(cfg, stream):
    """Independent generator for (workload, sub-stream)."""
    names = {"layout": 0, "sky": 1, "noise": 2, "samples": 3, "misc": 4}
    ss = np.random.SeedSequence(BASE_SEED + cfg).spawn(8)[names[stream]]
    return np.random.default_rng(ss)


@dataclass
class Observation:
    cfg: int
    uvw: np.ndarray            # [n_row, 3] float64, metres
    freq: np.ndarray           # [n_chan] float64, Hz
    nx: int
    ny: int
    dx: float                  # pixel size, radians
    dy: float
    coplanar: bool
    sky: np.ndarray = None     # [n_chan, nx, ny] float64 (None when too large)
    meta: dict = field(default_factory=dict)

    @property
    def n_row(self):
        return self.uvw.shape[0]

    @property
    def n_chan(self):
        return self.freq.shape[0]

    @property
    def n_vis(self):
        return self.n_row * self.n_chan


def _hour_angles(n_int, span_h):
    # integrations uniformly covering [-span/2, +span/2) hours, in radians
    return (np.arange(n_int) * (span_h / n_int) - span_h / 2.0) * (np.pi / 12.0)


def _rescale_w(uvw, frac=0.05):
    uvmax = np.sqrt(uvw[:, 0] ** 2 + uvw[:, 1] ** 2).max()
    wmax = np.abs(uvw[:, 2]).max()
    out = uvw.copy()
    out[:, 2] *= frac * uvmax / wmax
    return out


def make_config(cfg, n=None, n_int=None, with_sky=True, n_chan=None):
    """Build workload `cfg`; `n` (image side) and `n_int` (integrations) may be
    reduced for small test variants of the same layout."""
    rng_l = config_rng(cfg, "layout")
    rng_s = config_rng(cfg, "sky")
    if cfg == 0:
        enu = layout_uniform_disc(rng_l, 27, 5_000.0)
        n_int = n_int or 64
        uvw = earth_rotation_uvw(enu, np.deg2rad(-30.0), np.deg2rad(-45.0), _hour_angles(n_int, 1.0))
        uvw[:, 2] = 0.0
        n = n or 128
        freq = np.array([1.4e9])
        dx = dy = 1.0 * ARCSEC
        coplanar = True
        sky = None
        if with_sky:
            inner = max(8, n // 2)
            sky = point_sources(rng_s, n, n, 5, inner=inner) + gaussian_blob(rng_s, n, n, 3.0, 1.0, inner=inner)
            sky = sky[None]
    elif cfg in (1, 2):
        enu = layout_vla_y(rng_l)
        n_int = n_int or 2880
        uvw = earth_rotation_uvw(enu, np.deg2rad(34.1), np.deg2rad(40.0), _hour_angles(n_int, 8.0))
        uvw = _rescale_w(uvw, 0.05)
        n = n or 512
        freq = np.array([2.052e9])
        # keep the paper's Cyg A pixel at full size; scale up for reduced images so
        # the field of view (and hence the w-phase) stays comparable
        dx = dy = (0.05 / 1024.0) * (np.pi / 180.0) * (512 / n)
        coplanar = False
        sky = None
        if with_sky:
            s = correlated_field(rng_s, n, n)
            sky = np.exp(s - s.max()) + point_sources(rng_s, n, n, 20, inner=n // 2)
            sky = sky[None]
    elif cfg == 3:
        enu = layout_meerkat_like(rng_l)
        n_int = n_int or 3600
        uvw = earth_rotation_uvw(enu, np.deg2rad(-30.7), np.deg2rad(-60.0), _hour_angles(n_int, 8.0))
        uvw = _rescale_w(uvw, 0.05)
        n = n or 4096
        nc = n_chan or 16
        freq = np.linspace(0.9e9, 1.7e9, 16)[:nc] if nc <= 16 else np.linspace(0.9e9, 1.7e9, nc)
        dx = dy = 1.0 * ARCSEC * (4096 / n)
        coplanar = False
        sky = None
        if with_sky:
            s = correlated_field(rng_s, n, n)
            base = np.exp(s - s.max()) + point_sources(rng_s, n, n, 20, inner=n // 2)
            sky = np.stack([base * (f / freq[0]) ** -0.7 for f in freq])
    else:
        raise ValueError("make_config covers workloads 0-3; workload 4 is built by serving_jobs()")
    return Observation(cfg=cfg, uvw=uvw, freq=freq, nx=n, ny=n, dx=dx, dy=dy,
                       coplanar=coplanar, sky=sky,
                       meta={"n_int": n_int, "n_bl": uvw.shape[0] // n_int})


def noise_from_model(rng, model_vis, rel=0.1):
    """Noise with sigma = rel * rms|model|; returns (noise, weight = 1/sigma^2)."""
    sigma = rel * float(np.sqrt(np.mean(np.abs(model_vis) ** 2)))
    noise = sigma * (rng.standard_normal(model_vis.shape) + 1j * rng.standard_normal(model_vis.shape))
    return noise, np.full(model_vis.shape, 1.0 / sigma ** 2)


def serving_jobs(n_jobs=16, max_vis=5_000_000, min_vis=50_000):
    """Job descriptors for the served mix (workload 4): layout source, image side,
    visibility count and the pixel size giving u_max * dl = 0.4."""
    rng = config_rng(4, "misc")
    jobs = []
    sides = [128, 256, 512, 1024, 2048]
    for j in range(n_jobs):
        src = int(rng.integers(0, 4)) if j >= 4 else j % 4
        src = {0: 0, 1: 1, 2: 1, 3: 3}[src]
        n = int(sides[rng.integers(0, len(sides))])
        nvis = int(np.exp(rng.uniform(np.log(min_vis), np.log(max_vis))))
        jobs.append({"job": j, "layout": src, "n": n, "n_vis": nvis})
    return jobs


def serving_observation(job):
    """Realise one served job: its layout's track with the integration count set
    to give about job['n_vis'] rows, single channel, pixel size so u_max*dl = 0.4."""
    src = job["layout"]
    rng_l = config_rng(src, "layout")
    if src == 0:
        enu = layout_uniform_disc(rng_l, 27, 5_000.0)
        lat, dec, span, f = -30.0, -45.0, 1.0, 1.4e9
    elif src == 1:
        enu = layout_vla_y(rng_l)
        lat, dec, span, f = 34.1, 40.0, 8.0, 2.052e9
    else:
        enu = layout_meerkat_like(rng_l)
        lat, dec, span, f = -30.7, -60.0, 8.0, 1.3e9
    nbl = n_baselines(len(enu))
    n_int = max(1, job["n_vis"] // nbl)
    uvw = earth_rotation_uvw(enu, np.deg2rad(lat), np.deg2rad(dec), _hour_angles(n_int, span))
    if src == 0:
        uvw[:, 2] = 0.0
    else:
        uvw = _rescale_w(uvw, 0.05)
    freq = np.array([f])
    uvmax = np.sqrt(uvw[:, 0] ** 2 + uvw[:, 1] ** 2).max() * f / C_LIGHT
    dl = 0.4 / uvmax
    return Observation(cfg=4, uvw=uvw, freq=freq, nx=job["n"], ny=job["n"], dx=dl, dy=dl,
                       coplanar=(src == 0), sky=None, meta={"n_int": n_int, "n_bl": nbl})
