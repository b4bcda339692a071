"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed form, a
library routine on a special case, an invariant, brute force on a tiny input, or a
numerical optimiser.  Chosen so a dropped term, a wrong sign, a wrong index or a
transposed operand in the oracle fails at least one of them.
"""

import numpy as np
import pytest

import oracle as O
from synthetic import layouts, make_config
from synthetic.skies import power_spectrum

RTOL_TIGHT = 1e-12


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def small_obs(rng, n_vis=200, w_scale=1.0, uvmax=None, nx=16, ny=16, dx=None, dy=None):
    nx_, ny_ = nx, ny
    dx = dx or 1e-3
    dy = dy or 1.3e-3
    uvmax = uvmax or 0.45 / dx
    freq = np.array([1.0e9])
    lam = O.C_LIGHT_M_S / freq[0]
    uvw = np.empty((n_vis, 3))
    uvw[:, 0] = rng.uniform(-uvmax, uvmax, n_vis) * lam
    uvw[:, 1] = rng.uniform(-uvmax, uvmax, n_vis) * lam
    uvw[:, 2] = rng.uniform(-1, 1, n_vis) * w_scale * uvmax * lam
    return uvw, freq, nx_, ny_, dx, dy


# ------------------------------------------------------------------ R (degrid)
def test_point_source_at_phase_centre_is_constant(oracle_lib):
    """A point source of flux S at the phase centre gives V = S for every
    baseline, whatever u, v, w (the w-term and 1/n vanish there)."""
    rng = np.random.default_rng(1)
    uvw, freq, nx, ny, dx, dy = small_obs(rng, w_scale=3.0)
    img = np.zeros((nx, ny))
    img[nx // 2, ny // 2] = 2.5
    V = O.degrid(uvw, freq, nx, ny, dx, dy, img, divide_by_n=True)[:, 0]
    assert np.max(np.abs(V - 2.5)) < 1e-13


def test_point_source_off_centre_closed_form(oracle_lib):
    """Off-centre point source: |V| = S/n0 and arg V = -2 pi (u l0 + v m0 + w (n0 - 1)),
    on a wide field so that 1/n0 and the w-phase are far from trivial."""
    rng = np.random.default_rng(2)
    dx, dy = 0.05, 0.04
    uvw, freq, nx, ny, _, _ = small_obs(rng, dx=dx, dy=dy, w_scale=2.0)
    i0, j0 = 2, 14
    img = np.zeros((nx, ny))
    img[i0, j0] = 1.7
    V = O.degrid(uvw, freq, nx, ny, dx, dy, img, divide_by_n=True)[:, 0]
    l0, m0 = (i0 - nx // 2) * dx, (j0 - ny // 2) * dy
    n0 = np.sqrt(1 - l0 ** 2 - m0 ** 2)
    u, v, w = (uvw * freq[0] / O.C_LIGHT_M_S).T
    expect = 1.7 / n0 * np.exp(-2j * np.pi * (u * l0 + v * m0 + w * (n0 - 1)))
    assert np.max(np.abs(V - expect)) < 1e-12
    assert n0 < 0.97  # the 1/n factor is not trivially 1 here


def test_on_grid_uv_equals_numpy_fft(oracle_lib):
    """w = 0, no 1/n, and u = p/(nx dx), v = q/(ny dy) on grid frequencies:
    R reduces to numpy's fft2 of the image with its centre moved to index 0."""
    rng = np.random.default_rng(3)
    nx, ny, dx, dy = 16, 8, 1e-3, 2e-3
    img = rng.standard_normal((nx, ny))
    p = rng.integers(-nx // 2, nx // 2, 100)
    q = rng.integers(-ny // 2, ny // 2, 100)
    freq = np.array([1.0e9])
    lam = O.C_LIGHT_M_S / freq[0]
    uvw = np.stack([p / (nx * dx) * lam, q / (ny * dy) * lam, np.zeros(100)], axis=1)
    V = O.degrid(uvw, freq, nx, ny, dx, dy, img, divide_by_n=False)[:, 0]
    F = np.fft.fft2(np.fft.ifftshift(img))
    assert rel(V, F[p % nx, q % ny]) < 1e-12


def test_hermitian_symmetry_and_linearity(oracle_lib):
    rng = np.random.default_rng(4)
    uvw, freq, nx, ny, dx, dy = small_obs(rng, dx=0.01, dy=0.01, w_scale=1.0)
    img1 = rng.standard_normal((nx, ny))
    img2 = rng.standard_normal((nx, ny))
    V = O.degrid(uvw, freq, nx, ny, dx, dy, img1)[:, 0]
    Vm = O.degrid(-uvw, freq, nx, ny, dx, dy, img1)[:, 0]
    assert rel(Vm, np.conj(V)) < 1e-13
    V2 = O.degrid(uvw, freq, nx, ny, dx, dy, img2)[:, 0]
    V12 = O.degrid(uvw, freq, nx, ny, dx, dy, 2.0 * img1 - 0.5 * img2)[:, 0]
    assert rel(V12, 2.0 * V - 0.5 * V2) < 1e-13


@pytest.mark.parametrize("divide_by_n", [True, False])
def test_adjointness(oracle_lib, divide_by_n):
    """Re <R x, y> = <x, R^+ y> in the real inner product."""
    rng = np.random.default_rng(5)
    uvw, freq, nx, ny, dx, dy = small_obs(rng, dx=0.01, dy=0.012, w_scale=2.0)
    x = rng.standard_normal((nx, ny))
    y = rng.standard_normal(len(uvw)) + 1j * rng.standard_normal(len(uvw))
    Rx = O.degrid(uvw, freq, nx, ny, dx, dy, x, divide_by_n)[:, 0]
    Ry = O.grid(uvw, freq, nx, ny, dx, dy, y, None, divide_by_n)[0]
    lhs = np.real(np.vdot(Rx, y))
    rhs = float(np.sum(x * Ry))
    assert abs(lhs - rhs) < 1e-13 * max(abs(lhs), 1.0) * 10


def test_grid_pixels_matches_grid(oracle_lib):
    rng = np.random.default_rng(6)
    uvw, freq, nx, ny, dx, dy = small_obs(rng, dx=0.01, dy=0.01, w_scale=1.0)
    y = rng.standard_normal(len(uvw)) + 1j * rng.standard_normal(len(uvw))
    full = O.grid(uvw, freq, nx, ny, dx, dy, y)[0]
    pix = rng.choice(nx * ny, 20, replace=False)
    assert rel(O.grid_pixels(uvw, freq, nx, ny, dx, dy, y, pix), full.ravel()[pix]) < 1e-14


def test_degrid_rows_matches_degrid(oracle_lib):
    obs = make_config(3, n=16, n_int=4, n_chan=3)
    rng = np.random.default_rng(7)
    img = rng.standard_normal((3, 16, 16))
    full = O.degrid(obs.uvw, obs.freq, 16, 16, obs.dx, obs.dy, img)
    rows = rng.integers(0, obs.n_row, 30)
    chans = rng.integers(0, 3, 30)
    part = O.degrid_rows(obs.uvw, obs.freq, 16, 16, obs.dx, obs.dy, img, rows, chans)
    assert rel(part, full[rows, chans]) < 1e-14


# ------------------------------------------------------------------ PSF
def _psf_setup(seed=8, n=16, n_int=6):
    obs = make_config(1, n=n, n_int=n_int, with_sky=False)
    rng = np.random.default_rng(seed)
    wt = rng.uniform(0.5, 2.0, obs.n_row)
    return obs, wt


def test_dirty_image_of_point_source_is_shifted_psf(oracle_lib):
    """Coplanar data of a point source at (i0, j0): R^+ N^-1 V = S PSF0 shifted to
    (i0, j0) -- the PSF relation of Sec. 3.2 holding exactly when w = 0."""
    obs, wt = _psf_setup()
    uvw = obs.uvw.copy()
    uvw[:, 2] = 0.0
    n = obs.nx
    i0, j0 = 5, 11
    img = np.zeros((n, n))
    img[i0, j0] = 3.0
    V = O.degrid(uvw, obs.freq, n, n, obs.dx, obs.dy, img, divide_by_n=False)
    D = O.dirty_image(uvw, obs.freq, n, n, obs.dx, obs.dy, V, wt[:, None], divide_by_n=False)[0]
    psf = O.psf0(uvw, obs.freq, n, n, obs.dx, obs.dy, wt, zero_edge=False)
    expect = 3.0 * psf[n - i0: 2 * n - i0, n - j0: 2 * n - j0]
    assert rel(D, expect) < 1e-12


def test_psf_symmetries(oracle_lib):
    obs, wt = _psf_setup()
    n = obs.nx
    psf = O.psf0(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, wt)
    raw = O.psf0(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, wt, zero_edge=False)
    assert abs(psf[n, n] - wt.sum()) < 1e-12 * wt.sum()
    assert np.max(np.abs(raw)) <= wt.sum() * (1 + 1e-14)
    # periodically even after zeroing: psf[(2n - i) % 2n, (2n - j) % 2n] == psf[i, j] about (n, n)
    sh = np.fft.ifftshift(psf)
    flip = np.roll(sh[::-1, ::-1], (1, 1), axis=(0, 1))
    assert np.max(np.abs(flip - sh)) < 1e-12 * wt.sum()
    full = np.fft.fft2(sh)
    assert np.max(np.abs(full.imag)) < 1e-12 * np.max(np.abs(full.real))
    K = O.response_kernel(psf)
    assert K.shape == (2 * n, n + 1)
    assert np.max(np.abs(K - full.real[:, : n + 1])) < 1e-12 * np.max(np.abs(K))
    # K(-k) = K(k) on the full spectrum; in the half spectrum the two
    # self-conjugate columns (0 and n) are mirror-symmetric along the rows
    neg = np.roll(full.real[::-1, ::-1], (1, 1), axis=(0, 1))
    assert np.max(np.abs(neg - full.real)) < 1e-12 * np.max(np.abs(K))
    for j in (0, n):
        assert np.max(np.abs(K[1:, j][::-1] - K[1:, j])) < 1e-12 * np.max(np.abs(K))
    # without zeroing the edge the spectrum is genuinely complex
    fr = np.fft.fft2(np.fft.ifftshift(raw))
    assert np.max(np.abs(fr.imag)) > 1e-3 * np.max(np.abs(fr.real))


def test_psf_conv_fft_equals_direct(oracle_lib):
    obs, wt = _psf_setup(n=16)
    n = obs.nx
    psf = O.psf0(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, wt)
    K = O.response_kernel(psf)
    rng = np.random.default_rng(9)
    x = rng.standard_normal((n, n))
    a = O.n_factor(n, n, obs.dx, obs.dy)
    assert rel(O.psf_conv_fft(x, K, a), O.psf_conv_direct(x, psf, a)) < 1e-12
    pix = rng.choice(n * n, 17, replace=False)
    assert rel(O.psf_conv_direct(x, psf, a, pix=pix), O.psf_conv_direct(x, psf, a).ravel()[pix]) < 1e-14


@pytest.mark.parametrize("h,p", [((3, 3), (19, 19)), ((3, 6), (20, 24)), ((8, 8), (24, 24)),
                                 ((5, 2), (21, 40)), ((15, 15), (31, 31)), ((0, 0), (16, 16))])
def test_reduced_psf_conv_equals_direct_truncated(oracle_lib, h, p):
    """Sec. 3.3.2, reduced PSF: with the sidelobes beyond (hx, hy) dropped, padding
    to px >= nx + hx, py >= ny + hy gives the linear convolution with the truncated
    PSF, checked against the direct O(N^4) sum (which knows nothing of padding),
    at odd, even, non-power-of-two and anisotropic sizes."""
    obs, wt = _psf_setup(n=16)
    n = obs.nx
    psf = O.psf0(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, wt)
    (hx, hy), (px, py) = h, p
    Kp = O.response_kernel_padded(psf, hx, hy, px, py)
    assert Kp.shape == (px, py // 2 + 1)
    rng = np.random.default_rng(21)
    x = rng.standard_normal((n, n))
    a = O.n_factor(n, n, obs.dx, obs.dy)
    tr = O.psf_truncate(psf, hx, hy)
    direct = O.psf_conv_direct(x, tr, a)
    assert rel(O.psf_conv_fft_padded(x, Kp, px, py, a), direct) < 1e-12
    # the truncated PSF keeps exactly the (2hx + 1)(2hy + 1) central offsets
    assert np.count_nonzero(tr) == np.count_nonzero(psf[n - hx: n + hx + 1, n - hy: n + hy + 1])
    assert np.all(tr[n - hx: n + hx + 1, n - hy: n + hy + 1] == psf[n - hx: n + hx + 1, n - hy: n + hy + 1])
    # a single pixel at the centre picks out the truncated PSF itself
    e = np.zeros((n, n))
    e[n // 2, n // 2] = 1.0
    y = O.psf_conv_fft_padded(e, Kp, px, py)
    assert np.max(np.abs(y - tr[n - n // 2: n + n // 2, n - n // 2: n + n // 2])) < 1e-12 * psf.max()


def test_reduced_psf_padding_bound_is_tight(oracle_lib):
    """One row or column less than nx + hx (ny + hy) and the periodic wrap reaches
    the cropped window."""
    obs, wt = _psf_setup(n=16)
    n = obs.nx
    psf = O.psf0(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, wt)
    rng = np.random.default_rng(22)
    x = rng.standard_normal((n, n))
    hx, hy = 6, 4
    direct = O.psf_conv_direct(x, O.psf_truncate(psf, hx, hy))
    for px, py in ((n + hx - 1, n + hy), (n + hx, n + hy - 1)):
        y = O.psf_conv_fft_padded(x, O.response_kernel_padded(psf, hx, hy, px, py), px, py)
        assert rel(y, direct) > 1e-3


def test_reduced_psf_full_support_is_the_doubled_grid(oracle_lib):
    """hx = nx - 1, hy = ny - 1 on the 2nx x 2ny grid keeps every offset but the
    zeroed -n row and column: the kernel is K_R itself."""
    obs, wt = _psf_setup(n=16)
    n = obs.nx
    psf = O.psf0(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, wt)
    K = O.response_kernel(psf)
    Kp = O.response_kernel_padded(psf, n - 1, n - 1, 2 * n, 2 * n)
    assert np.max(np.abs(Kp - K)) < 1e-12 * np.max(np.abs(K))


def test_reduced_psf_error_vanishes_with_support(oracle_lib):
    """The neglected sidelobes are all that separates the reduced R' from the full
    one: the error is the convolution with the dropped part, and it is zero once
    nothing is dropped."""
    obs, wt = _psf_setup(n=16)
    n = obs.nx
    psf = O.psf0(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, wt)
    rng = np.random.default_rng(23)
    x = rng.standard_normal((n, n))
    full = O.psf_conv_fft(x, O.response_kernel(psf))
    for h in (2, 5, 9):
        red = O.psf_conv_fft_padded(x, O.response_kernel_padded(psf, h, h, n + h, n + h), n + h, n + h)
        dropped = O.psf_conv_direct(x, psf - O.psf_truncate(psf, h, h))
        assert rel(full - red, dropped) < 1e-10
    h = n - 1
    red = O.psf_conv_fft_padded(x, O.response_kernel_padded(psf, h, h, n + h, n + h), n + h, n + h)
    assert rel(red, full) < 1e-12


@pytest.mark.parametrize("divide_by_n", [True, False])
def test_psf_conv_exact_for_coplanar(oracle_lib, divide_by_n):
    """Sec. 3.3.2: the PSF convolution is exact for a coplanar array."""
    obs, wt = _psf_setup(n=16)
    uvw = obs.uvw.copy()
    uvw[:, 2] = 0.0
    n = obs.nx
    psf = O.psf0(uvw, obs.freq, n, n, obs.dx, obs.dy, wt)
    K = O.response_kernel(psf)
    a = O.n_factor(n, n, obs.dx, obs.dy, divide_by_n)
    rng = np.random.default_rng(10)
    x = rng.standard_normal((n, n))
    exact = O.rnr_exact(uvw, obs.freq, n, n, obs.dx, obs.dy, x, wt[:, None], divide_by_n)[0]
    assert rel(O.psf_conv_fft(x, K, a), exact) < 1e-12


def test_psf_conv_not_exact_with_w(oracle_lib):
    """...and only for coplanar ones: a wide field with large w breaks it."""
    rng = np.random.default_rng(11)
    uvw, freq, nx, ny, dx, dy = small_obs(rng, n_vis=300, dx=0.02, dy=0.02, w_scale=3.0)
    wt = np.ones(len(uvw))
    psf = O.psf0(uvw, freq, nx, ny, dx, dy, wt)
    K = O.response_kernel(psf)
    a = O.n_factor(nx, ny, dx, dy)
    x = rng.standard_normal((nx, ny))
    exact = O.rnr_exact(uvw, freq, nx, ny, dx, dy, x, wt[:, None])[0]
    assert rel(O.psf_conv_fft(x, K, a), exact) > 1e-3


def test_psf_conv_symmetric_psd(oracle_lib):
    obs, wt = _psf_setup(n=16)
    n = obs.nx
    psf = O.psf0(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, wt)
    K = O.response_kernel(psf)
    a = O.n_factor(n, n, obs.dx, obs.dy)
    rng = np.random.default_rng(12)
    for _ in range(5):
        x, y = rng.standard_normal((2, n, n))
        Rx, Ry = O.psf_conv_fft(x, K, a), O.psf_conv_fft(y, K, a)
        assert abs(np.sum(Rx * y) - np.sum(x * Ry)) < 1e-12 * np.linalg.norm(Rx) * np.linalg.norm(y)
        assert np.sum(x * Rx) >= -1e-12 * np.linalg.norm(Rx) * np.linalg.norm(x)


# ------------------------------------------------------------------ noise kernel
def test_noise_kernel_properties_and_optimality(oracle_lib):
    from scipy.optimize import minimize

    obs, wt = _psf_setup(n=16)
    n = obs.nx
    psf = O.psf0(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, wt)
    eps = 1e-3 * psf.max()
    K = O.noise_kernel(psf, eps)
    assert K.shape == (n, n) and np.all(np.isreal(K)) and np.all(K >= eps)
    f0 = O.noise_kernel_objective(psf, eps, K)
    rng = np.random.default_rng(13)
    for _ in range(20):
        Kp = np.maximum(K * np.exp(0.05 * rng.standard_normal(K.shape)), eps * (1 + 1e-9))
        assert O.noise_kernel_objective(psf, eps, Kp) >= f0 - 1e-10 * max(f0, 1.0)
    # the paper's argmin over xi solved by a generic optimiser (image-space objective)
    scale = psf.max()

    def obj(xi):
        Kx = np.exp(xi).reshape(n, n) * scale + eps
        return O.noise_kernel_objective(psf, eps, Kx) / scale ** 2

    xi0 = np.log(np.maximum(K - eps, 1e-3 * scale) / scale).ravel() + 0.1 * rng.standard_normal(n * n)
    res = minimize(obj, xi0, method="L-BFGS-B", options={"maxiter": 2000, "ftol": 1e-16, "gtol": 1e-14})
    assert f0 / scale ** 2 <= res.fun + 1e-10


def test_noise_kernel_exact_for_even_positive_crop(oracle_lib):
    """A PSF whose crop is periodically even with a positive spectrum T is
    reproduced exactly: K = T + eps and the objective is zero."""
    n = 16
    k = np.fft.fftfreq(n) * n
    T = 1.0 + 0.4 * np.cos(2 * np.pi * k[:, None] / n) + 0.3 * np.cos(4 * np.pi * k[None, :] / n)
    crop = np.fft.fftshift(np.real(np.fft.ifft2(T)))
    psf = np.zeros((2 * n, 2 * n))
    psf[n - n // 2: n + n // 2, n - n // 2: n + n // 2] = crop
    eps = 1e-4
    K = O.noise_kernel(psf, eps)
    assert np.max(np.abs(K - (T + eps))) < 1e-12
    assert O.noise_kernel_objective(psf, eps, K) < 1e-24


def test_noise_inv_is_inverse(oracle_lib):
    rng = np.random.default_rng(14)
    K = rng.uniform(0.5, 2.0, (8, 8))
    K = 0.5 * (K + np.roll(K[::-1, ::-1], (1, 1), axis=(0, 1)))  # even -> real operator
    x = rng.standard_normal((8, 8))
    assert rel(O.noise_apply(O.noise_inv_apply(x, K), K), x) < 1e-13


# ------------------------------------------------------------------ likelihoods
def _lik_setup(seed=15, n=16):
    obs = make_config(1, n=n, n_int=5, with_sky=False)
    rng = np.random.default_rng(seed)
    wt = rng.uniform(0.5, 2.0, (obs.n_row, 1))
    V = rng.standard_normal((obs.n_row, 1)) + 1j * rng.standard_normal((obs.n_row, 1))
    s = 0.3 * rng.standard_normal((n, n))
    fwd = lambda I: O.degrid(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, I)
    adj = lambda y: O.grid(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, y)[0]
    return obs, wt, V, s, fwd, adj, rng


def test_exact_likelihood_quadratic_identity(oracle_lib):
    """H = 1/2 I^T R' I - I^T I_D + 1/2 V^H N^-1 V (expansion of eq. ham)."""
    obs, wt, V, s, fwd, adj, rng = _lik_setup()
    n = obs.nx
    H, _ = O.likelihood_exact(s, V, wt, fwd, adj)
    I = np.exp(s)
    RI = O.rnr_exact(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, I, wt)[0]
    ID = O.dirty_image(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, V, wt)[0]
    H2 = 0.5 * np.sum(I * RI) - np.sum(I * ID) + 0.5 * np.sum(wt * np.abs(V) ** 2)
    assert abs(H - H2) < 1e-10 * abs(H)


def test_exact_likelihood_gradient_fd(oracle_lib):
    obs, wt, V, s, fwd, adj, rng = _lik_setup()
    n = obs.nx
    inv_power = 1.0 / power_spectrum(n, n)
    ifix = np.zeros((n, n))
    ifix[3, 4] = 2.0
    H, g = O.likelihood_exact(s, V, wt, fwd, adj, i_fixed=ifix, inv_power=inv_power)
    for _ in range(3):
        d = rng.standard_normal((n, n))
        d /= np.linalg.norm(d)
        h = 1e-6
        Hp, _ = O.likelihood_exact(s + h * d, V, wt, fwd, adj, ifix, inv_power)
        Hm, _ = O.likelihood_exact(s - h * d, V, wt, fwd, adj, ifix, inv_power)
        fd = (Hp - Hm) / (2 * h)
        assert abs(fd - np.sum(g * d)) < 1e-7 * max(abs(fd), np.linalg.norm(g))


def _dense(op, n):
    cols = []
    for k in range(n * n):
        e = np.zeros(n * n)
        e[k] = 1.0
        cols.append(op(e.reshape(n, n)).ravel())
    return np.array(cols).T


def test_fast_likelihood_dense_brute_force(oracle_lib):
    """On 16^2: assemble R'_approx (direct convolution) and N'^-1 (inverse-kernel
    convolution) as dense matrices; H and g from matrix products must equal the
    FFT forms.  g_s = -exp(s) * R'^T N'^-1 (d - R' I)."""
    obs, wt, V, s, fwd, adj, rng = _lik_setup(n=16)
    n = obs.nx
    psf = O.psf0(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, wt[:, 0])
    K = O.response_kernel(psf)
    KN = O.noise_kernel(psf, 1e-2 * psf.max())
    a = O.n_factor(n, n, obs.dx, obs.dy)
    Rm = _dense(lambda x: O.psf_conv_direct(x, psf, a), n)
    Nm = _dense(lambda x: O.noise_inv_apply(x, KN), n)
    d = rng.standard_normal((n, n))
    ifix = np.zeros((n, n))
    ifix[7, 2] = 1.5
    H, g = O.likelihood_fast(s, d, K, KN, a, i_fixed=ifix)
    I = (np.exp(s) + ifix).ravel()
    r = d.ravel() - Rm @ I
    H2 = 0.5 * r @ Nm @ r
    g2 = -np.exp(s).ravel() * (Rm.T @ (Nm @ r))
    assert abs(H - H2) < 1e-12 * abs(H2)
    assert rel(g.ravel(), g2) < 1e-12


def test_fast_likelihood_reduced_psf_dense_brute_force(oracle_lib):
    """The FAST likelihood with a reduced-support kernel on a smaller padded grid
    equals the dense form with the direct convolution by the truncated PSF."""
    obs, wt, V, s, fwd, adj, rng = _lik_setup(n=16)
    n = obs.nx
    psf = O.psf0(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, wt[:, 0])
    hx, hy, px, py = 5, 3, 21, 20
    Kp = O.response_kernel_padded(psf, hx, hy, px, py)
    KN = O.noise_kernel(psf, 1e-2 * psf.max())
    a = O.n_factor(n, n, obs.dx, obs.dy)
    tr = O.psf_truncate(psf, hx, hy)
    Rm = _dense(lambda x: O.psf_conv_direct(x, tr, a), n)
    Nm = _dense(lambda x: O.noise_inv_apply(x, KN), n)
    d = rng.standard_normal((n, n))
    H, g = O.likelihood_fast(s, d, Kp, KN, a, pad=(px, py))
    I = np.exp(s).ravel()
    r = d.ravel() - Rm @ I
    H2 = 0.5 * r @ Nm @ r
    g2 = -np.exp(s).ravel() * (Rm.T @ (Nm @ r))
    assert abs(H - H2) < 1e-12 * abs(H2)
    assert rel(g.ravel(), g2) < 1e-12


def test_fast_likelihood_gradient_fd(oracle_lib):
    obs, wt, V, s, fwd, adj, rng = _lik_setup(n=16)
    n = obs.nx
    psf = O.psf0(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, wt[:, 0])
    K = O.response_kernel(psf)
    KN = O.noise_kernel(psf, 1e-2 * psf.max())
    a = O.n_factor(n, n, obs.dx, obs.dy)
    d = rng.standard_normal((n, n))
    inv_power = 1.0 / power_spectrum(n, n)
    H, g = O.likelihood_fast(s, d, K, KN, a, inv_power=inv_power)
    dd = rng.standard_normal((n, n))
    dd /= np.linalg.norm(dd)
    h = 1e-6
    fd = (O.likelihood_fast(s + h * dd, d, K, KN, a, inv_power=inv_power)[0]
          - O.likelihood_fast(s - h * dd, d, K, KN, a, inv_power=inv_power)[0]) / (2 * h)
    assert abs(fd - np.sum(g * dd)) < 1e-7 * max(abs(fd), np.linalg.norm(g))


# ------------------------------------------------------------------ CG
def test_cg_matches_dense_cholesky(oracle_lib):
    obs, wt, V, s, fwd, adj, rng = _lik_setup(n=8)
    n = obs.nx
    psf = O.psf0(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, wt[:, 0])
    K = O.response_kernel(psf) / psf.max()
    inv_power = 1.0 / power_spectrum(n, n)
    inv_power = inv_power / inv_power.max() + 0.05
    a = O.n_factor(n, n, obs.dx, obs.dy)
    diag = np.exp(0.2 * rng.standard_normal((n, n)))
    op = lambda x: O.metric_apply(x, K, inv_power, a, diag)
    A = _dense(op, n)
    assert np.max(np.abs(A - A.T)) < 1e-13 * np.max(np.abs(A))
    b = rng.standard_normal(n * n)
    L = np.linalg.cholesky(A)
    xs = np.linalg.solve(L.T, np.linalg.solve(L, b))
    x, hist = O.cg(op, b.reshape(n, n), maxiter=400, rtol=1e-14)
    assert rel(x.ravel(), xs) < 1e-10
    # A-norm of the error never increases
    errs = []
    for k in range(1, 40):
        xk, _ = O.cg(op, b.reshape(n, n), maxiter=k)
        e = xk.ravel() - xs
        errs.append(e @ A @ e)
    floor = 1e-24 * errs[0]  # once converged the error sits at rounding level
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-9) + floor for i in range(len(errs) - 1))
    assert errs[5] < errs[0]
    assert hist[0] == pytest.approx(np.linalg.norm(b))


# ------------------------------------------------------------------ synthetic shapes
@pytest.mark.parametrize("cfg,rows", [(0, 22_464), (1, 1_010_880), (3, 7_257_600)])
def test_baseline_counts(cfg, rows):
    n_ant = {0: 27, 1: 27, 3: 64}[cfg]
    n_int = {0: 64, 1: 2880, 3: 3600}[cfg]
    assert layouts.n_baselines(n_ant) * n_int == rows
    if cfg != 3:
        obs = make_config(cfg, with_sky=False)
        assert obs.n_row == rows
