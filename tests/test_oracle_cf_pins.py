"""Pins of the oracle's correlated-field amplitude model (the inferred power
spectrum of the Gaussian-process prior of Sec. 3.1.1, hyperparameters as in the
prior-parameter appendices), on the CPU:

  * with zero flexibility and asperity the spectrum is a pure power law: the
    amplitude goes as |k|^slope, the power as |k|^(2 slope);
  * whatever the flexibility and asperity, the average log-log slope of the
    amplitude between the first and last frequency bin is the given slope;
  * the fluctuations parameter sets the standard deviation of the field without
    its zero mode, exactly in expectation (sum of the spectrum) and in a Monte
    Carlo ensemble of fields; the zero mode adds its own variance;
  * the lognormal hyperparameters have the stated mean and standard deviation;
  * the local-slope process is a Wiener process: its variance after a log-frequency
    span T is flexibility^2 T."""

import numpy as np
import pytest

import oracle as O

PRIOR = dict(offset=13.0, zm_mean=1.0, zm_std=0.1, fluct_mean=3.0, fluct_std=1.0, slope_mean=-2.4,
             slope_std=0.1, flex_mean=1.2, flex_std=0.4, asp_mean=0.2, asp_std=0.2)


def test_bins_cover_the_grid():
    vals, mult, idx = O.cf_bins(16, 32)
    assert mult.sum() == 16 * 32 - 1 and np.all(np.diff(vals) > 0)
    kx = np.fft.fftfreq(16) * 16
    ky = np.fft.fftfreq(32) * 32
    k2 = kx[:, None] ** 2 + ky[None, :] ** 2
    assert idx[0, 0] == -1
    assert np.all(vals[idx[k2 > 0]] == k2[k2 > 0])


def test_zero_flexibility_and_asperity_give_a_power_law():
    p = dict(PRIOR, flex_mean=0.0, asp_mean=0.0)
    nx = ny = 32
    vals, _, _ = O.cf_bins(nx, ny)
    rng = np.random.default_rng(1)
    xi_h = rng.standard_normal(5)
    P = O.cf_power(nx, ny, p, xi_h, rng.standard_normal(len(vals)), rng.standard_normal(len(vals)))
    slope = p["slope_mean"] + p["slope_std"] * xi_h[2]
    kx = np.fft.fftfreq(nx) * nx
    ky = np.fft.fftfreq(ny) * ny
    k2 = kx[:, None] ** 2 + ky[None, :] ** 2
    m = k2 > 0
    ratio = P[m] / P[0, 1]  # P(k) / P(|k| = 1)
    assert np.allclose(ratio, k2[m] ** slope, rtol=1e-12, atol=0)


def test_average_slope_is_the_given_slope():
    vals, _, _ = O.cf_bins(64, 64)
    t = 0.5 * np.log(vals.astype(np.float64))
    rng = np.random.default_rng(2)
    for flex, asp in ((1.2, 0.2), (0.1, 0.01), (3.0, 1.0)):
        logA, v, y = O.cf_log_amplitude(t, -2.2, flex, asp, rng.standard_normal(len(t)),
                                        rng.standard_normal(len(t)))
        assert abs((logA[-1] - logA[0]) - (-2.2) * (t[-1] - t[0])) < 1e-12 * (t[-1] - t[0])
        assert np.std(np.diff(y)) > 0  # the deviation is not trivially zero


def test_fluctuations_set_the_field_standard_deviation():
    nx = ny = 32
    vals, _, _ = O.cf_bins(nx, ny)
    rng = np.random.default_rng(3)
    xi_h = rng.standard_normal(5)
    P = O.cf_power(nx, ny, PRIOR, xi_h, rng.standard_normal(len(vals)), rng.standard_normal(len(vals)))
    zm, fluct = O.cf_hyper(PRIOR, xi_h)[:2]
    # exact: var of a pixel without the zero mode = sum_{k != 0} P / N; the zero mode adds zm^2
    assert abs(np.sum(P) / (nx * ny) - P[0, 0] / (nx * ny) - fluct ** 2) < 1e-12 * fluct ** 2
    assert abs(P[0, 0] / (nx * ny) - zm ** 2) < 1e-12 * zm ** 2
    # Monte Carlo: ensemble variance of the field at every pixel
    n_s = 4000
    s = np.stack([O.cf_logsky(P, rng.standard_normal((nx, ny)), PRIOR["offset"]) for _ in range(n_s)])
    var = np.var(s, axis=0).mean()
    assert abs(var / (zm ** 2 + fluct ** 2) - 1.0) < 0.06
    assert abs(s.mean() - PRIOR["offset"]) < 5 * np.sqrt((zm ** 2 + fluct ** 2) / n_s)


@pytest.mark.parametrize("mean,std", [(1.0, 0.1), (3.0, 1.0), (1.2, 0.4), (0.2, 0.2)])
def test_lognormal_moments(mean, std):
    x = O.lognormal_from_moments(mean, std, np.random.default_rng(4).standard_normal(400_000))
    assert abs(x.mean() / mean - 1) < 0.01
    assert abs(x.std() / std - 1) < 0.02
    assert np.all(x > 0)


def test_local_slope_is_a_wiener_process():
    vals, _, _ = O.cf_bins(64, 64)
    t = 0.5 * np.log(vals.astype(np.float64))
    rng = np.random.default_rng(5)
    flex = 1.5
    vJ = np.array([O.cf_log_amplitude(t, 0.0, flex, 0.0, rng.standard_normal(len(t)), np.zeros(len(t)))[1][-1]
                   for _ in range(3000)])
    assert abs(vJ.var() / (flex ** 2 * (t[-1] - t[0])) - 1) < 0.08
