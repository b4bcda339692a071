"""Pins of the oracle's prior-covariance inverse S^-1 = F^-1 diag(1/P) F (the
Gaussian-process prior of Sec. 3.1.1 on the periodic grid), against facts that do
not go through the FFT it is written with:

  * a single Fourier mode cos(2 pi (k i/nx + q j/ny)) is an eigenvector, with
    eigenvalue 1/P(k, q) of its own frequency (an even spectrum takes the same
    value at (k, q) and (-k, -q));
  * S^-1 is the circulant matrix of the correlation function F^-1(1/P), whose
    entries are written out here as plain cosine sums (Wiener-Khinchin).

An anisotropic spectrum makes a transposed axis, a spectrum shifted by half the
grid or an inverted factor fail every test."""

import numpy as np
import pytest

import oracle as O
from synthetic.skies import power_spectrum


def even_anisotropic_inv_power(nx, ny):
    """1/P(k) = 1 + 0.3 k_x^2 + 2.1 k_y^2 + 0.05 k_x^2 k_y^2 with signed integer
    frequencies: even in (k_x, k_y) jointly and in each axis, different along the
    two axes."""
    kx = np.fft.fftfreq(nx) * nx
    ky = np.fft.fftfreq(ny) * ny
    return 1.0 + 0.3 * kx[:, None] ** 2 + 2.1 * ky[None, :] ** 2 + 0.05 * kx[:, None] ** 2 * ky[None, :] ** 2


@pytest.mark.parametrize("nx,ny", [(8, 8), (16, 8), (12, 20)])
@pytest.mark.parametrize("k,q", [(0, 0), (1, 0), (0, 1), (2, 3), (3, -2)])
def test_fourier_mode_is_eigenvector(nx, ny, k, q):
    i = np.arange(nx)[:, None]
    j = np.arange(ny)[None, :]
    ph = 2.0 * np.pi * (k * i / nx + q * j / ny)
    ip = even_anisotropic_inv_power(nx, ny)
    lam = 1.0 + 0.3 * k ** 2 + 2.1 * q ** 2 + 0.05 * k ** 2 * q ** 2  # 1/P at (k, q), by hand
    for x in (np.cos(ph), np.sin(ph) if (k, q) != (0, 0) else None):
        if x is None:
            continue
        y = O.prior_inv_apply(x, ip)
        np.testing.assert_allclose(y, lam * x, rtol=0, atol=1e-12 * lam)


def test_fourier_mode_with_the_synthetic_spectrum():
    """The same eigen-relation with the isotropic prior spectrum of the synthetic
    skies, whose value at |k| is written out from its formula here."""
    n = 16
    P = power_spectrum(n, n)
    k0, scale = 2.0, P[0, 0]  # P = scale (1 + (|k|/k0)^2)^-2, P[0, 0] = scale
    for k, q in [(1, 2), (4, 0), (5, 7)]:
        i = np.arange(n)[:, None]
        j = np.arange(n)[None, :]
        x = np.cos(2 * np.pi * (k * i + q * j) / n)
        lam = 1.0 / (scale * (1.0 + (k * k + q * q) / k0 ** 2) ** -2)
        np.testing.assert_allclose(O.prior_inv_apply(x, 1.0 / P), lam * x, rtol=1e-12, atol=1e-12 * lam)


def test_dense_circulant_of_the_correlation_function():
    """S^-1 x = sum_i'j' c[(i - i') mod nx, (j - j') mod ny] x[i', j'] with
    c[a, b] = (1/N) sum_kq (1/P)[k, q] cos(2 pi (k a/nx + q b/ny)) summed directly."""
    nx, ny = 6, 10
    ip = even_anisotropic_inv_power(nx, ny)
    kx = np.arange(nx)
    ky = np.arange(ny)
    c = np.zeros((nx, ny))
    for a in range(nx):
        for b in range(ny):
            c[a, b] = np.sum(ip * np.cos(2 * np.pi * (kx[:, None] * a / nx + ky[None, :] * b / ny))) / (nx * ny)
    M = np.zeros((nx * ny, nx * ny))
    for i in range(nx):
        for j in range(ny):
            for i2 in range(nx):
                for j2 in range(ny):
                    M[i * ny + j, i2 * ny + j2] = c[(i - i2) % nx, (j - j2) % ny]
    rng = np.random.default_rng(3)
    for _ in range(3):
        x = rng.standard_normal((nx, ny))
        np.testing.assert_allclose(O.prior_inv_apply(x, ip).ravel(), M @ x.ravel(), rtol=0,
                                   atol=1e-12 * np.abs(M @ x.ravel()).max())
    # symmetric positive definite, as an inverse covariance must be
    np.testing.assert_allclose(M, M.T, atol=1e-12)
    assert np.linalg.eigvalsh(M).min() > 0


def test_inverse_of_the_covariance_map():
    """S^-1 undoes S: the map F^-1 diag(P) F x written with explicit numpy FFTs
    here, then the oracle's S^-1, returns x."""
    n = 16
    P = power_spectrum(n, n)
    x = np.random.default_rng(5).standard_normal((n, n))
    Sx = np.real(np.fft.ifft2(np.fft.fft2(x) * P))
    np.testing.assert_allclose(O.prior_inv_apply(Sx, 1.0 / P), x, atol=1e-10)
