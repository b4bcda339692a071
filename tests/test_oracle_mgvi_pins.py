"""Pins of the oracle's MGVI pieces (minor cycle of Sec. 3.3.5 in standardised
coordinates, Gaussian-process prior of Sec. 3.1.1) against facts other than the
formulas themselves: the covariance of the GP map against the circulant matrix of
its correlation function (Wiener-Khinchin), the metric against J^T N'^-1 J + 1 with
J from finite differences, the draw's covariance against the metric, the gradient
against finite differences, and the CG sample against a dense solve."""

import numpy as np
import pytest

import oracle as O
from synthetic import make_config
from synthetic.skies import power_spectrum


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _dense(op, n):
    cols = []
    for k in range(n * n):
        e = np.zeros(n * n)
        e[k] = 1.0
        cols.append(np.ravel(op(e.reshape(n, n))))
    return np.array(cols).T


def _setup(n=8, seed=31):
    obs = make_config(1, n=n, n_int=6, with_sky=False)
    rng = np.random.default_rng(seed)
    wt = rng.uniform(0.5, 2.0, obs.n_row)
    psf = O.psf0(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, wt)
    K = O.response_kernel(psf)
    KN = O.noise_kernel(psf, 1e-2 * psf.max())
    a = O.n_factor(n, n, obs.dx, obs.dy)
    power = power_spectrum(n, n)
    xi = 0.5 * rng.standard_normal((n, n))
    d = O.psf_conv_fft(np.exp(O.gp_apply(rng.standard_normal((n, n)), power)), K, a)
    return n, K, KN, a, power, xi, d, rng


def test_gp_map_covariance_is_the_circulant_of_the_correlation(oracle_lib):
    """For white xi, s = A xi has covariance A A^T; by Wiener-Khinchin it is the
    circulant matrix C[i - j] of the correlation function C = F^-1 P."""
    n, K, KN, a, power, xi, d, rng = _setup()
    A = _dense(lambda x: O.gp_apply(x, power), n)
    C = np.real(np.fft.ifft2(power))
    idx = np.arange(n)
    S = np.empty((n * n, n * n))
    for i in range(n):
        for j in range(n):
            S[i * n + j] = C[(i - idx[:, None]) % n, (j - idx[None, :]) % n].ravel()
    assert rel(A @ A.T, S) < 1e-12
    assert rel(A, A.T) < 1e-12  # real even spectrum: symmetric
    Ai = _dense(lambda x: O.gp_apply(x, power, inverse=True), n)
    assert rel(Ai @ A, np.eye(n * n)) < 1e-10


def test_mgvi_gradient_matches_finite_differences(oracle_lib):
    n, K, KN, a, power, xi, d, rng = _setup()
    H, g = O.mgvi_hamiltonian(xi, d, K, KN, power, a)
    h = 1e-6
    for _ in range(3):
        u = rng.standard_normal((n, n))
        u /= np.linalg.norm(u)
        Hp, _ = O.mgvi_hamiltonian(xi + h * u, d, K, KN, power, a)
        Hm, _ = O.mgvi_hamiltonian(xi - h * u, d, K, KN, power, a)
        fd = (Hp - Hm) / (2 * h)
        assert abs(fd - float(np.sum(g * u))) < 1e-6 * np.linalg.norm(g)


def test_mgvi_metric_is_gauss_newton_of_the_residual(oracle_lib):
    """M = 1 + J^T N'^-1 J with J = dr/dxi taken by central differences of
    r(xi) = d - R' exp(A xi): pins the order of the factors in the metric."""
    n, K, KN, a, power, xi, d, rng = _setup()
    D = np.exp(O.gp_apply(xi, power))
    M = _dense(lambda x: O.mgvi_metric_apply(x, K, KN, power, D, a), n)

    def resid(z):
        return d - O.psf_conv_fft(np.exp(O.gp_apply(z, power)), K, a)

    h = 1e-6
    J = np.empty((n * n, n * n))
    for k in range(n * n):
        e = np.zeros(n * n)
        e[k] = h
        J[:, k] = (resid(xi + e.reshape(n, n)) - resid(xi - e.reshape(n, n))).ravel() / (2 * h)
    Ninv = _dense(lambda x: O.noise_inv_apply(x, KN), n)
    M_gn = np.eye(n * n) + J.T @ Ninv @ J
    assert rel(M, M_gn) < 1e-6
    assert rel(M, M.T) < 1e-12
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() >= 1.0 - 1e-9


def test_mgvi_draw_has_the_metric_as_covariance(oracle_lib):
    n, K, KN, a, power, xi, d, rng = _setup()
    D = np.exp(O.gp_apply(xi, power))
    M = _dense(lambda x: O.mgvi_metric_apply(x, K, KN, power, D, a), n)
    B = _dense(lambda e: O.mgvi_draw(np.zeros((n, n)), e, K, KN, power, D, a), n)
    assert rel(np.eye(n * n) + B @ B.T, M) < 1e-10
    e0 = rng.standard_normal((n, n))
    assert rel(O.mgvi_draw(e0, np.zeros((n, n)), K, KN, power, D, a), e0) < 1e-15


def test_mgvi_sample_is_the_metric_solve(oracle_lib):
    """x = M^-1 (draw): CG to convergence equals the dense solve, so x has
    covariance M^-1 M M^-1 = M^-1."""
    n, K, KN, a, power, xi, d, rng = _setup()
    D = np.exp(O.gp_apply(xi, power))
    M = _dense(lambda x: O.mgvi_metric_apply(x, K, KN, power, D, a), n)
    e0, e1 = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    x, hist = O.mgvi_sample(e0, e1, K, KN, power, D, maxiter=4 * n * n, a=a, rtol=1e-13)
    draw = O.mgvi_draw(e0, e1, K, KN, power, D, a)
    assert rel(x.ravel(), np.linalg.solve(M, draw.ravel())) < 1e-9
    assert hist[-1] <= 1e-13 * hist[0] * 1.0001
