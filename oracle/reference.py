"""FP64 oracle: plain definitions of everything the response-operator path computes.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Sections cited are those of
Roth et al., "fast-resolve: Fast Bayesian Radio Interferometric Imaging"
(arXiv 2406.09144).

Readings of points the paper leaves open (listed with reasons in the design notes):
  * pixel sum for the sky integral, phase centre at pixel (nx/2, ny/2), first image
    axis <-> l <-> u, image in flux per pixel;
  * gains G = 1 (calibrated data);
  * real sky, so R^+ y = Re(R^H y) and adjointness holds in the real inner product
    <p, q> = Re sum conj(p) q;
  * the PSF is the coplanar one (w := 0, no 1/n), on the doubled grid, with the
    unpaired offset -N row and column zeroed; D = diag(1/n) is applied on both sides
    of the convolution when divide_by_n is set;
  * the noise-kernel argmin is solved in closed form (noise_kernel below);
  * conjugate gradients: Hestenes-Stiefel, x0 = 0, no preconditioner.
"""

import ctypes

import numpy as np

from .build import build, lib_path

C_LIGHT_M_S = 299_792_458.0

_lib = None


def _c():
    global _lib
    if _lib is None:
        import os
        if not os.path.exists(lib_path()):
            build()
        _lib = ctypes.CDLL(lib_path())
        i64, dbl, ip = ctypes.c_int64, ctypes.c_double, ctypes.c_int
        P = ctypes.c_void_p
        _lib.oracle_degrid.argtypes = [i64, i64, dbl, dbl, ip, P, i64, P, P, P, P]
        _lib.oracle_grid.argtypes = [i64, i64, dbl, dbl, ip, i64, P, P, P, P, P]
        _lib.oracle_grid_pixels.argtypes = [i64, i64, dbl, dbl, ip, i64, P, P, P, P, i64, P, P]
        _lib.oracle_psf0.argtypes = [i64, i64, dbl, dbl, i64, P, P, P, P]
        _lib.oracle_psf_conv_direct.argtypes = [i64, i64, P, P, i64, P, P]
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- O1 coordinates
def lmn(nx, ny, dx, dy):
    """Pixel direction cosines (Sec. 2): l_i = (i - nx/2) dx, m_j = (j - ny/2) dy,
    n = sqrt(1 - l^2 - m^2).  Returns l [nx], m [ny], n [nx, ny]."""
    l = (np.arange(nx) - nx // 2) * dx
    m = (np.arange(ny) - ny // 2) * dy
    n = np.sqrt(1.0 - l[:, None] ** 2 - m[None, :] ** 2)
    return l, m, n


def n_factor(nx, ny, dx, dy, divide_by_n=True):
    """a_ij = 1/n_ij (the 1/sqrt(1 - l^2) of C(l, w), Sec. 2) or ones."""
    if not divide_by_n:
        return np.ones((nx, ny))
    return 1.0 / lmn(nx, ny, dx, dy)[2]


def uvw_lambda(uvw_m, freq_hz):
    """Baseline coordinates in units of the wavelength (Sec. 2): u = uvw nu / c.
    Returns u, v, w each [n_row, n_chan]."""
    uvw_m = _f64(uvw_m)
    s = _f64(freq_hz)[None, :] / C_LIGHT_M_S
    return uvw_m[:, 0:1] * s, uvw_m[:, 1:2] * s, uvw_m[:, 2:3] * s


# ---------------------------------------------------------------- O2 / O3
def degrid(uvw_m, freq_hz, nx, ny, dx, dy, img, divide_by_n=True):
    """R, the measurement equation of Sec. 2 (Eq. 1) with G = 1, written as a pixel sum.
    img [n_chan, nx, ny] (or [nx, ny] for one channel) -> vis [n_row, n_chan] complex."""
    img = _f64(img)
    if img.ndim == 2:
        img = img[None]
    u, v, w = uvw_lambda(uvw_m, freq_hz)
    n_row, n_chan = u.shape
    out = np.empty((n_row, n_chan), np.complex128)
    for c in range(n_chan):
        uc, vc, wc = _f64(u[:, c]), _f64(v[:, c]), _f64(w[:, c])
        buf = np.empty((n_row, 2))
        _c().oracle_degrid(nx, ny, dx, dy, int(divide_by_n), _p(_f64(img[c])), n_row,
                           _p(uc), _p(vc), _p(wc), _p(buf))
        out[:, c] = buf[:, 0] + 1j * buf[:, 1]
    return out


def degrid_rows(uvw_m, freq_hz, nx, ny, dx, dy, img, rows, chans, divide_by_n=True):
    """R evaluated only at the listed (row, channel) pairs."""
    img = _f64(img)
    if img.ndim == 2:
        img = img[None]
    u, v, w = uvw_lambda(uvw_m, freq_hz)
    rows = np.asarray(rows)
    chans = np.asarray(chans)
    out = np.empty(len(rows), np.complex128)
    for c in np.unique(chans):
        sel = np.nonzero(chans == c)[0]
        r = rows[sel]
        buf = np.empty((len(r), 2))
        _c().oracle_degrid(nx, ny, dx, dy, int(divide_by_n), _p(_f64(img[c])), len(r),
                           _p(_f64(u[r, c])), _p(_f64(v[r, c])), _p(_f64(w[r, c])), _p(buf))
        out[sel] = buf[:, 0] + 1j * buf[:, 1]
    return out


def grid(uvw_m, freq_hz, nx, ny, dx, dy, vis, weight=None, divide_by_n=True):
    """R^+ (Sec. 3.2, adjoint of R; real sky so R^+ y = Re R^H y), applied to
    weight * vis.  vis [n_row, n_chan] -> img [n_chan, nx, ny]."""
    vis = np.asarray(vis, np.complex128)
    if vis.ndim == 1:
        vis = vis[:, None]
    if weight is not None:
        vis = vis * np.asarray(weight, np.float64).reshape(vis.shape)
    u, v, w = uvw_lambda(uvw_m, freq_hz)
    n_row, n_chan = u.shape
    out = np.empty((n_chan, nx, ny))
    for c in range(n_chan):
        y = _f64(np.stack([vis[:, c].real, vis[:, c].imag], axis=1))
        img = np.empty((nx, ny))
        _c().oracle_grid(nx, ny, dx, dy, int(divide_by_n), n_row, _p(_f64(u[:, c])),
                         _p(_f64(v[:, c])), _p(_f64(w[:, c])), _p(y), _p(img))
        out[c] = img
    return out


def grid_pixels(uvw_m, freq_hz, nx, ny, dx, dy, vis, pix, chan=0, weight=None, divide_by_n=True):
    """R^+ of channel `chan` evaluated only at flat pixel indices `pix`."""
    vis = np.asarray(vis, np.complex128)
    if vis.ndim == 1:
        vis = vis[:, None]
    if weight is not None:
        vis = vis * np.asarray(weight, np.float64).reshape(vis.shape)
    u, v, w = uvw_lambda(uvw_m, freq_hz)
    c = chan
    y = _f64(np.stack([vis[:, c].real, vis[:, c].imag], axis=1))
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    out = np.empty(len(pix))
    _c().oracle_grid_pixels(nx, ny, dx, dy, int(divide_by_n), u.shape[0], _p(_f64(u[:, c])),
                            _p(_f64(v[:, c])), _p(_f64(w[:, c])), _p(y), len(pix), _p(pix), _p(out))
    return out


def dirty_image(uvw_m, freq_hz, nx, ny, dx, dy, vis, weight, divide_by_n=True):
    """I_D = R^+ N^-1 V with N^-1 = diag(weight) (Sec. 3.1.2, Sec. 3.2)."""
    return grid(uvw_m, freq_hz, nx, ny, dx, dy, vis, weight, divide_by_n)


# ---------------------------------------------------------------- O6 / O7 PSF
def psf0(uvw_m, freq_hz, nx, ny, dx, dy, weight, chan=0, zero_edge=True):
    """Coplanar PSF on the doubled grid (Sec. 3.3.2: the PSF must be twice the
    field of view): PSF0[i, j] = sum_k wt_k cos(2 pi [u_k (i - nx) dx + v_k (j - ny) dy]),
    i.e. R0^+ N^-1 R0 applied to a delta, with R0 = R at w = 0 without 1/n.
    With zero_edge, the offset -nx row and -ny column are set to zero: they never
    enter the cropped linear convolution, and zeroing them makes the array
    periodically even so its FFT is real."""
    u, v, _ = uvw_lambda(uvw_m, freq_hz)
    wt = np.asarray(weight, np.float64).reshape(u.shape)[:, chan]
    out = np.empty((2 * nx, 2 * ny))
    _c().oracle_psf0(nx, ny, dx, dy, u.shape[0], _p(_f64(u[:, chan])), _p(_f64(v[:, chan])),
                     _p(_f64(wt)), _p(out))
    if zero_edge:
        out[0, :] = 0.0
        out[:, 0] = 0.0
    return out


def response_kernel(psf):
    """K_R = FFT[I_PSF] of Sec. 3.3.2: rfft2 of the PSF moved so offset 0 sits at
    index 0.  The PSF is periodically even, so the transform is real; returns the
    real part, shape [2nx, ny + 1]."""
    return np.real(np.fft.rfft2(np.fft.ifftshift(psf)))


# ---------------------------------------------------------------- O8 / O9
def psf_conv_fft(x, K_R, a=None):
    """R' I ~ P^+ FFT^-1[FFT[I_PSF] FFT[P I]] (Sec. 3.3.2), with D = diag(a) on both
    sides; P pads nx x ny into the top-left of 2nx x 2ny, P^+ crops it back."""
    x = _f64(x)
    nx, ny = x.shape[-2:]
    if a is not None:
        x = x * a
    xp = np.zeros(x.shape[:-2] + (2 * nx, 2 * ny))
    xp[..., :nx, :ny] = x
    y = np.fft.irfft2(K_R * np.fft.rfft2(xp), s=(2 * nx, 2 * ny))[..., :nx, :ny]
    return y * a if a is not None else y


def psf_conv_direct(x, psf, a=None, pix=None):
    """The same linear convolution summed directly (O(N^4)):
    y_ij = a_ij sum_{i'j'} PSF0[nx + i - i', ny + j - j'] a_{i'j'} x_{i'j'}."""
    x = _f64(x)
    nx, ny = x.shape
    xin = _f64(x * a) if a is not None else x
    psf = _f64(psf)
    if pix is None:
        y = np.empty((nx, ny))
        _c().oracle_psf_conv_direct(nx, ny, _p(psf), _p(xin), 0, None, _p(y))
        return y * a if a is not None else y
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    y = np.empty(len(pix))
    _c().oracle_psf_conv_direct(nx, ny, _p(psf), _p(xin), len(pix), _p(pix), _p(y))
    return y * a.reshape(-1)[pix] if a is not None else y


# ---------------------------------------------------------------- reduced PSF
def psf_truncate(psf, hx, hy):
    """The doubled-grid PSF with the sidelobes beyond offsets |dx| > hx, |dy| > hy
    neglected (Sec. 3.3.2: a smaller PSF needs less zero padding, at the price of
    a less accurate R').  0 <= hx < nx, 0 <= hy < ny."""
    nx, ny = psf.shape[0] // 2, psf.shape[1] // 2
    assert 0 <= hx < nx and 0 <= hy < ny
    out = np.zeros_like(_f64(psf))
    wx = slice(nx - hx, nx + hx + 1)
    wy = slice(ny - hy, ny + hy + 1)
    out[wx, wy] = psf[wx, wy]
    return out


def response_kernel_padded(psf, hx, hy, px, py):
    """FFT[I_PSF] of the truncated PSF on a px x py periodic grid: offset (dx, dy)
    sits at index (dx mod px, dy mod py).  Returns the real part of the r2c half,
    [px, py // 2 + 1].  The convolution of an nx x ny image cropped back to
    nx x ny is linear (no wrapped term reaches the window) iff px >= nx + hx and
    py >= ny + hy."""
    nx, ny = psf.shape[0] // 2, psf.shape[1] // 2
    assert px >= 2 * hx + 1 and py >= 2 * hy + 1
    ox = np.arange(-hx, hx + 1)
    oy = np.arange(-hy, hy + 1)
    z = np.zeros((px, py))
    z[np.ix_(ox % px, oy % py)] = _f64(psf)[np.ix_(nx + ox, ny + oy)]
    return np.real(np.fft.rfft2(z))


def psf_conv_fft_padded(x, K, px, py, a=None):
    """P^+ FFT^-1[K FFT[P I]] with P padding nx x ny into the top-left of
    px x py (Sec. 3.3.2 with a reduced padding), D = diag(a) on both sides."""
    x = _f64(x)
    nx, ny = x.shape[-2:]
    if a is not None:
        x = x * a
    xp = np.zeros(x.shape[:-2] + (px, py))
    xp[..., :nx, :ny] = x
    y = np.fft.irfft2(K * np.fft.rfft2(xp), s=(px, py))[..., :nx, :ny]
    return y * a if a is not None else y


def rnr_exact(uvw_m, freq_hz, nx, ny, dx, dy, x, weight, divide_by_n=True):
    """R' x = R^+ N^-1 R x evaluated exactly (Sec. 3.3.1; major cycle, Sec. 3.3.4)."""
    vis = degrid(uvw_m, freq_hz, nx, ny, dx, dy, x, divide_by_n)
    return grid(uvw_m, freq_hz, nx, ny, dx, dy, vis, weight, divide_by_n)


# ---------------------------------------------------------------- O10 / O11
def crop_psf(psf):
    """The nx x ny window of the doubled-grid PSF holding offsets [-n/2, n/2):
    N' applied to a delta at the field centre (Sec. 3.3.3), without the epsilon."""
    nx, ny = psf.shape[0] // 2, psf.shape[1] // 2
    return psf[nx - nx // 2: nx + nx // 2, ny - ny // 2: ny + ny // 2]


def noise_kernel(psf, eps):
    """K = exp(xi) + eps with xi the argmin of Sec. 3.3.3, in closed form.

    With I_delta at the field centre, |FFT(I_delta)| = 1 and Parseval turn the
    objective into (1/N^2) sum_k |T_k + eps - (exp(xi_k) + eps)|^2 with
    T = fft2(ifftshift(crop)), which separates per frequency: exp(xi_k) = Re T_k
    where Re T_k > 0; elsewhere the infimum is approached as xi_k -> -inf, i.e.
    K_k = eps.  Returns the full [nx, ny] real kernel."""
    T = np.fft.fft2(np.fft.ifftshift(crop_psf(psf)))
    return eps + np.maximum(T.real, 0.0)


def noise_kernel_objective(psf, eps, K):
    """The squared residual of Sec. 3.3.3 for a candidate kernel K (= exp(xi) + eps),
    evaluated in image space exactly as written (not through Parseval)."""
    nx, ny = psf.shape[0] // 2, psf.shape[1] // 2
    delta = np.zeros((nx, ny))
    delta[nx // 2, ny // 2] = 1.0
    target = crop_psf(psf) + eps * delta
    approx = np.real(np.fft.ifft2(K * np.fft.fft2(delta)))
    return float(np.sum((target - approx) ** 2))


def noise_inv_apply(x, K_N):
    """N'^-1 x ~ FFT^-1[K^-1 FFT x] on the periodic nx x ny grid (Sec. 3.3.3)."""
    return np.real(np.fft.ifft2(np.fft.fft2(_f64(x)) / K_N))


def noise_apply(x, K_N):
    return np.real(np.fft.ifft2(np.fft.fft2(_f64(x)) * K_N))


# ---------------------------------------------------------------- O14 prior
def prior_inv_apply(x, inv_power):
    """S^-1 x = F^-1 diag(1/P) F x on the periodic grid; inv_power is the full
    [nx, ny] array 1/P(k)."""
    return np.real(np.fft.ifft2(np.fft.fft2(_f64(x)) * inv_power))


# ---------------------------------------------------------------- O12 / O13
def likelihood_exact(s, vis, weight, fwd, adj, i_fixed=None, inv_power=None):
    """Eq. (ham) of Sec. 3.1.2 without the constant log-determinant, as a function
    of the log-sky s with I = exp(s) (+ fixed sources):
        H = 1/2 sum w |V - R I|^2,   g = exp(s) * R^+ [w (R I - V)].
    fwd(img) -> vis and adj(vis) -> img are the exact operators.  An optional
    prior term 1/2 s^T S^-1 s adds S^-1 s to the gradient."""
    s = _f64(s)
    I = np.exp(s) + (i_fixed if i_fixed is not None else 0.0)
    res = fwd(I) - vis
    H = 0.5 * float(np.sum(weight * np.abs(res) ** 2))
    g = np.exp(s) * adj(weight * res)
    if inv_power is not None:
        Ss = prior_inv_apply(s, inv_power)
        H += 0.5 * float(np.sum(s * Ss))
        g = g + Ss
    return H, g


def likelihood_fast(s, d, K_R, K_N, a=None, i_fixed=None, inv_power=None, pad=None):
    """Eq. (ham_new) of Sec. 3.3.1 with R' replaced by the PSF convolution
    (Sec. 3.3.2) and N'^-1 by the inverse-kernel convolution (Sec. 3.3.3):
        r = d - R' I,  q = N'^-1 r,  H = 1/2 <r, q>,  g = -exp(s) * R' q.
    pad = (px, py): K_R is a reduced-support kernel on that padded grid."""
    def rconv(x):
        return psf_conv_fft(x, K_R, a) if pad is None else psf_conv_fft_padded(x, K_R, pad[0], pad[1], a)
    s = _f64(s)
    I = np.exp(s) + (i_fixed if i_fixed is not None else 0.0)
    r = _f64(d) - rconv(I)
    q = noise_inv_apply(r, K_N)
    H = 0.5 * float(np.sum(r * q))
    g = -np.exp(s) * rconv(q)
    if inv_power is not None:
        Ss = prior_inv_apply(s, inv_power)
        H += 0.5 * float(np.sum(s * Ss))
        g = g + Ss
    return H, g


# ---------------------------------------------------------------- O15 CG
def cg(apply_A, b, maxiter, rtol=0.0):
    """Conjugate gradients (Hestenes-Stiefel), x0 = 0, no preconditioner, FP64.
    The solve MGVI uses to apply an inverse metric (minor cycle, Sec. 3.3.5).
    Returns x and the residual-norm history ||r_k|| (k = 0 .. iterations)."""
    b = _f64(b)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(np.sum(r * r))
    hist = [np.sqrt(rr)]
    stop = rtol * np.sqrt(rr)
    for _ in range(maxiter):
        if np.sqrt(rr) <= stop:
            break
        Ap = apply_A(p)
        alpha = rr / float(np.sum(p * Ap))
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = float(np.sum(r * r))
        hist.append(np.sqrt(rr_new))
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, np.array(hist)


# ---------------------------------------------------------------- MGVI (standardised coordinates)
def gp_apply(x, power, inverse=False):
    """Standardised excitations -> log-sky: A x = F^-1 diag(sqrt P) F x on the
    periodic grid, the Gaussian process of the diffuse-emission prior (Sec. 3.1.1:
    correlated pixels, exponentiated for positivity), so s = A xi has covariance
    S = F^-1 diag(P) F for white xi.  power: full [nx, ny] array P(k) > 0.
    inverse: apply A^-1 instead."""
    f = np.sqrt(power)
    if inverse:
        f = 1.0 / f
    return np.real(np.fft.ifft2(np.fft.fft2(_f64(x)) * f))


def noise_inv_sqrt_apply(x, K_N):
    """N'^-1/2 x = F^-1 diag(K^-1/2) F x (square root of the Sec. 3.3.3 kernel)."""
    return np.real(np.fft.ifft2(np.fft.fft2(_f64(x)) / np.sqrt(K_N)))


def mgvi_hamiltonian(xi, d, K_R, K_N, power, a=None):
    """Eq. (ham_new) in standardised coordinates with the Gaussian-process prior
    (the minor-cycle posterior of Sec. 3.3.5): s = A xi, I = exp(s),
        r = d - R' I,  H = 1/2 r^T N'^-1 r + 1/2 xi^T xi,
        dH/dxi = -A D R' N'^-1 r + xi,  D = diag(I)."""
    xi = _f64(xi)
    I = np.exp(gp_apply(xi, power))
    r = _f64(d) - psf_conv_fft(I, K_R, a)
    q = noise_inv_apply(r, K_N)
    H = 0.5 * float(np.sum(r * q)) + 0.5 * float(np.sum(xi * xi))
    g = -gp_apply(I * psf_conv_fft(q, K_R, a), power) + xi
    return H, g


def mgvi_metric_apply(x, K_R, K_N, power, diag, a=None):
    """M x = x + A D R' N'^-1 R' D A x: the Fisher metric of mgvi_hamiltonian
    (J^T N'^-1 J + 1 with J = dr/dxi = -R' D A), which MGVI inverts to draw its
    samples (Sec. 3.3.5).  diag = exp(s) at the expansion point."""
    u = psf_conv_fft(diag * gp_apply(x, power), K_R, a)
    u = diag * psf_conv_fft(noise_inv_apply(u, K_N), K_R, a)
    return _f64(x) + gp_apply(u, power)


def mgvi_draw(eta0, eta1, K_R, K_N, power, diag, a=None):
    """A vector with covariance M from two white ones: eta0 + A D R' N'^-1/2 eta1
    (covariance 1 + A D R' N'^-1 R' D A, every factor symmetric)."""
    u = diag * psf_conv_fft(noise_inv_sqrt_apply(eta1, K_N), K_R, a)
    return _f64(eta0) + gp_apply(u, power)


def mgvi_sample(eta0, eta1, K_R, K_N, power, diag, maxiter, a=None, rtol=0.0):
    """An MGVI sample offset x = M^-1 (draw with covariance M), so x ~ N(0, M^-1),
    by CG; returns x and the residual history."""
    xi = mgvi_draw(eta0, eta1, K_R, K_N, power, diag, a)
    return cg(lambda p: mgvi_metric_apply(p, K_R, K_N, power, diag, a), xi, maxiter, rtol)


def metric_apply(x, K_R, inv_power, a=None, diag=None):
    """A x = D_s R' D_s x + S^-1 x with R' the PSF convolution and D_s = diag(diag)."""
    y = x if diag is None else diag * x
    y = psf_conv_fft(y, K_R, a)
    if diag is not None:
        y = diag * y
    return y + prior_inv_apply(x, inv_power)


# ---------------------------------------------------------------- Algorithm 1
def algorithm1(uvw_m, freq_hz, nx, ny, dx, dy, vis, weight, K_R, K_N, a, inv_power, s0, n_major, n_minor,
               cg_iters, lam, max_step):
    """The major/minor scheme of Algorithm 1 (Sec. 3.3.4) for one channel, with a
    fixed minor-cycle schedule:

        I_D = R^+ N^-1 V  (exact);  d_0 = I_D
        for each major cycle i:
            minor cycle on d_i = I_PSF * (I - I_i-1) + n' (FAST likelihood, eq. ham_new,
            with the prior 1/2 s^T S^-1 s): n_minor damped Gauss-Newton steps
                (D R' D + S^-1 + lam) ds = -g,   s <- s + t ds,   D = diag(exp s),
            each solved by cg_iters conjugate-gradient iterations, with
            t = min(1, max_step / max|ds|) bounding the change of the log-sky
            (exp is nonlinear);
            I_i = exp(s);  d_i+1 = I_D - R^+ N^-1 R I_i  (exact).

    The Gauss-Newton metric D R' D stands in for D R' N'^-1 R' D (reading of the
    minor cycle: the paper runs MGVI there).  K_R [2nx, ny + 1] and K_N [nx, ny]
    (full) as response_kernel and noise_kernel; inv_power the full [nx, ny] 1/P.
    Returns the log-sky after the last minor cycle, the residual images d_1 ..
    d_n_major, the FAST H after each minor cycle and the log-sky after each."""
    I_D = dirty_image(uvw_m, freq_hz, nx, ny, dx, dy, vis, weight)[0]
    d = I_D
    s = _f64(s0)
    I_prev = None
    ds_out, Hs, s_out = [], [], []
    for _ in range(n_major):
        for _ in range(n_minor):
            ifix = None if I_prev is None else -I_prev
            _, g = likelihood_fast(s, d, K_R, K_N, a, i_fixed=ifix, inv_power=inv_power)
            D = np.exp(s)
            ds, _ = cg(lambda p: metric_apply(p, K_R, inv_power + lam, a, D), -g, cg_iters)
            s = s + min(1.0, max_step / np.max(np.abs(ds))) * ds
        Hs.append(likelihood_fast(s, d, K_R, K_N, a, i_fixed=None if I_prev is None else -I_prev,
                                  inv_power=inv_power)[0])
        s_out.append(s)
        I_prev = np.exp(s)
        d = I_D - rnr_exact(uvw_m, freq_hz, nx, ny, dx, dy, I_prev, weight)[0]
        ds_out.append(d)
    return s, ds_out, Hs, s_out


# ---------------------------------------------------------------- correlated-field amplitude model
# The diffuse-emission prior is an exponentiated Gaussian process (Sec. 3.1.1)
# whose power spectrum is itself inferred, with the hyperparameters listed in the
# prior-parameter appendices (zero mode offset; zero mode, fluctuations,
# loglogavgslope, flexibility and asperity, each with a mean and a standard
# deviation).  The paper defers their definition to earlier work; the reading
# written out here:
#   * positive hyperparameters (zero-mode std, fluctuations, flexibility,
#     asperity) are lognormal with the given mean and standard deviation
#     (x = exp(mu + sigma xi), sigma^2 = ln(1 + std^2/mean^2), mu = ln mean -
#     sigma^2 / 2); a mean of 0 gives exactly 0; the average slope is normal;
#   * on the log of the spatial frequency, t = ln|k| over the distinct non-zero
#     |k| of the grid, the log-amplitude is the average slope times (t - t_0) plus
#     a deviation: a Wiener process v (the local slope, variance flexibility^2
#     per unit t) integrated over t, plus a rougher Wiener part scaled by
#     flexibility * asperity, with its straight line between the first and last
#     bin removed (so loglogavgslope is the average log-log slope of the
#     amplitude);
#   * the power is the squared amplitude, normalised so that the variance of the
#     field without its zero mode is fluctuations^2; the zero mode has variance
#     (zero-mode std)^2; the log-sky is offset + F^-1 sqrt(P) F xi_field.
CF_PRIOR_KEYS = ("offset", "zm_mean", "zm_std", "fluct_mean", "fluct_std", "slope_mean", "slope_std",
                 "flex_mean", "flex_std", "asp_mean", "asp_std")


def lognormal_from_moments(mean, std, xi):
    """exp(mu + sigma xi) with mean `mean` and standard deviation `std` (0 if mean is 0)."""
    if mean == 0.0:
        return 0.0 * np.asarray(xi, np.float64)
    s2 = np.log1p((std / mean) ** 2)
    return np.exp(np.log(mean) - 0.5 * s2 + np.sqrt(s2) * np.asarray(xi, np.float64))


def cf_bins(nx, ny):
    """Distinct non-zero |k|^2 of the nx x ny grid (integer frequency units), their
    multiplicity over the full grid, and the bin of every full-grid frequency (-1
    for k = 0)."""
    kx = np.fft.fftfreq(nx) * nx
    ky = np.fft.fftfreq(ny) * ny
    k2 = np.rint(kx[:, None] ** 2 + ky[None, :] ** 2).astype(np.int64)
    vals, inv, counts = np.unique(k2, return_inverse=True, return_counts=True)
    assert vals[0] == 0
    return vals[1:], counts[1:], inv.reshape(nx, ny) - 1


def cf_hyper(prior, xi_h):
    """(zero-mode std, fluctuations, slope, flexibility, asperity) from the standardised
    excitations xi_h[0..4]."""
    return (float(lognormal_from_moments(prior["zm_mean"], prior["zm_std"], xi_h[0])),
            float(lognormal_from_moments(prior["fluct_mean"], prior["fluct_std"], xi_h[1])),
            float(prior["slope_mean"] + prior["slope_std"] * xi_h[2]),
            float(lognormal_from_moments(prior["flex_mean"], prior["flex_std"], xi_h[3])),
            float(lognormal_from_moments(prior["asp_mean"], prior["asp_std"], xi_h[4])))


def cf_log_amplitude(t, slope, flex, asp, xi_v, xi_y):
    """The log-amplitude on the log-frequencies t (ascending) and its two Wiener
    processes: v_j = flex sum_{i<=j} sqrt(d_i) xi_v_i (local slope),
    y_j = sum_{i<=j} [(v_i-1 + v_i) d_i / 2 + flex asp sqrt(d_i) xi_y_i], d_i = t_i - t_i-1
    (d_0 = 0), and logA = slope (t - t_0) + y - y_J (t - t_0) / (t_J - t_0)."""
    t = _f64(t)
    d = np.concatenate([[0.0], np.diff(t)])
    v = flex * np.cumsum(np.sqrt(d) * xi_v)
    v_prev = np.concatenate([[0.0], v[:-1]])
    y = np.cumsum(0.5 * (v_prev + v) * d + flex * asp * np.sqrt(d) * xi_y)
    span = t[-1] - t[0]
    frac = (t - t[0]) / span if span > 0 else np.zeros_like(t)
    return slope * (t - t[0]) + y - y[-1] * frac, v, y


def cf_power(nx, ny, prior, xi_h, xi_v, xi_y):
    """Full [nx, ny] power spectrum P(k) of the correlated field for the given
    excitations (xi_h: 5 hyperparameter excitations; xi_v, xi_y: one per bin)."""
    vals, mult, idx = cf_bins(nx, ny)
    zm, fluct, slope, flex, asp = cf_hyper(prior, xi_h)
    t = 0.5 * np.log(vals.astype(np.float64))
    logA, _, _ = cf_log_amplitude(t, slope, flex, asp, _f64(xi_v), _f64(xi_y))
    a2 = np.exp(2.0 * (logA - logA.max()))  # the normalisation removes any common factor
    P_bin = fluct ** 2 * (nx * ny) * a2 / np.sum(mult * a2)
    P = np.empty((nx, ny))
    P[idx >= 0] = P_bin[idx[idx >= 0]]
    P[0, 0] = zm ** 2 * (nx * ny)
    return P


def cf_logsky(P, xi_field, offset):
    """offset + F^-1 sqrt(P) F xi: the Gaussian-process log-sky."""
    return offset + gp_apply(xi_field, P)
