"""Synthetic skies, prior power spectra and noise realisations (inputs only).

The diffuse component is an exponentiated Gaussian random field, the prior family
the paper builds on (Sec. 3.1.1).  Its spectrum is a proposal, since the paper
defers the correlated-field hyperparameters to earlier work:

    P(k) = A (1 + (|k|/k0)^2)^-2      (asymptotic slope -4)

with |k| in integer FFT frequency units on the N_x x N_y periodic grid and A chosen
so that the field has unit standard deviation.  A field is drawn as
s = Re ifft2(sqrt(P) fft2(eta)), eta ~ N(0, 1) per pixel.
"""

import numpy as np


def _kmag(nx, ny):
    kx = np.fft.fftfreq(nx) * nx
    ky = np.fft.fftfreq(ny) * ny
    return np.sqrt(kx[:, None] ** 2 + ky[None, :] ** 2)


def power_spectrum(nx, ny, k0=2.0):
    """Full [nx, ny] spectrum P(k), normalised to unit field variance."""
    p = (1.0 + (_kmag(nx, ny) / k0) ** 2) ** -2
    # var(s) = sum_k P_k / (nx ny) for s = ifft2(sqrt(P) fft2(eta)).
    return p * (nx * ny / p.sum())


def inv_power_half(nx, ny, k0=2.0):
    """1/P(k) on the r2c half-spectrum layout [nx, ny//2 + 1]."""
    return 1.0 / power_spectrum(nx, ny, k0)[:, : ny // 2 + 1]


def correlated_field(rng, nx, ny, k0=2.0, eta=None):
    if eta is None:
        eta = rng.standard_normal((nx, ny))
    P = power_spectrum(nx, ny, k0)
    return np.real(np.fft.ifft2(np.sqrt(P) * np.fft.fft2(eta)))


def point_sources(rng, nx, ny, n_src, inner=None, mu=0.0, sigma=1.0):
    """n_src lognormal point sources at integer pixels uniform in the inner box."""
    img = np.zeros((nx, ny))
    ix0 = (nx - (inner or nx)) // 2
    iy0 = (ny - (inner or ny)) // 2
    xs = ix0 + rng.integers(0, inner or nx, n_src)
    ys = iy0 + rng.integers(0, inner or ny, n_src)
    flux = rng.lognormal(mu, sigma, n_src)
    np.add.at(img, (xs, ys), flux)
    return img


def gaussian_blob(rng, nx, ny, sigma_px=3.0, peak=1.0, inner=None):
    ix0 = (nx - (inner or nx)) // 2
    iy0 = (ny - (inner or ny)) // 2
    cx = ix0 + rng.random() * (inner or nx)
    cy = iy0 + rng.random() * (inner or ny)
    x = np.arange(nx)[:, None]
    y = np.arange(ny)[None, :]
    return peak * np.exp(-0.5 * ((x - cx) ** 2 + (y - cy) ** 2) / sigma_px ** 2)


def complex_noise(rng, shape, sigma):
    """Complex Gaussian noise: real and imaginary parts each N(0, sigma^2)."""
    return sigma * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
