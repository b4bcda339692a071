"""Parity of the PSF machinery and of the 32-plane configuration at the workloads'
full shapes, on outputs the oracle computes one by one.

  * make_psf_kernel on the VLA-like plan (512^2 image, 1024^2 PSF grid gridded from
    1,010,880 weights) and on a MeerKAT-like plan (4096^2 per channel, 8192^2 PSF
    grid, three channels across the band): the GPU response kernel K_R, transformed
    back to the PSF with numpy, is compared at sampled offsets with the oracle's
    dirty image of unit visibilities on the doubled field (w := 0, no 1/n), which is
    the PSF's definition.  Bound: the plan's eps on the sampled relative L2 error.
  * apply_RNR_approx at 4096^2 per channel with an 8192^2 kernel per channel (two
    channels): the brute-force linear convolution on sampled output pixels.  The
    kernel is the oracle's rfft2 of a synthetic periodically even PSF (the
    convolution machinery is what is tested; the PSF values are those of a PSF
    with a sharp peak and decaying random sidelobes).  Bound 1e-6, as at 512^2:
    FP32 FFT rounding grows only like u32 sqrt(log2 L) on average with twiddles
    rounded once from FP64 (measured 2.7e-7 with 8192-long lines in both passes).
  * the MeerKAT-like workload at its stated 32 improved-w-stacking planes
    (7,257,600 rows x 16 channels): sampled degridding and gridding against the
    direct sums on three channels, bound eps = 1e-5.
"""

import numpy as np
import pytest

import oracle as O
from synthetic import make_config

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def gpu_psf0(psf, chan):
    """PSF0 [2nx, 2ny] (peak at (nx, ny)) from the GPU kernel K_R = rfft2(ifftshift(PSF0))."""
    KR, _ = psf.kernels()
    K = KR[chan].cpu().numpy().astype(np.float64)
    return np.fft.fftshift(np.fft.irfft2(K, s=(2 * psf.nx, 2 * psf.ny)))


def oracle_psf0_at(obs, wt, chan, flat_idx):
    """PSF0 at flat indices of the doubled grid: the dirty image of unit visibilities
    with weights wt on the 2nx x 2ny field, w := 0 and no 1/n (the PSF's definition)."""
    uvw0 = obs.uvw.copy()
    uvw0[:, 2] = 0.0
    ones = np.ones((obs.n_row, obs.n_chan), np.complex128)
    return O.grid_pixels(uvw0, obs.freq, 2 * obs.nx, 2 * obs.ny, obs.dx, obs.dy, ones, flat_idx, chan=chan,
                         weight=wt, divide_by_n=False)


def sampled_offsets(rng, nx, ny, k):
    """k flat indices of the doubled grid away from the zeroed offset -n row/column,
    plus the peak."""
    i = rng.integers(1, 2 * nx, k)
    j = rng.integers(1, 2 * ny, k)
    flat = i * (2 * ny) + j
    return np.concatenate([flat, [nx * 2 * ny + ny]])


def _psf_check(obs, chans, n_samp, seed, eps=1e-5):
    import torch
    from paper_2406_09144_amd import api
    rng = np.random.default_rng(seed)
    n = obs.nx
    print(f"[psf-full] {obs.n_row} rows x {obs.n_chan} channel(s), {n}^2, PSF grid {2 * n}^2", flush=True)
    pl = api.Plan(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, eps=eps)
    wt = rng.uniform(0.5, 2.0, (obs.n_row, obs.n_chan))
    psf = api.make_psf_kernel(pl, torch.from_numpy(wt).float().cuda(), eps_noise=-1e-4)
    torch.cuda.synchronize()
    for c in chans:
        p_gpu = gpu_psf0(psf, c)
        idx = sampled_offsets(rng, n, n, n_samp)
        ref = oracle_psf0_at(obs, wt, c, idx)
        got = p_gpu.ravel()[idx]
        e = rel(got, ref)
        e_side = rel(got[:-1], ref[:-1])
        print(f"[psf-full] channel {c}: peak {got[-1]:.6e} (sum w {wt[:, c].sum():.6e}), sampled rel err "
              f"{e:.2e}, sidelobes only {e_side:.2e}", flush=True)
        assert abs(got[-1] - wt[:, c].sum()) <= eps * wt[:, c].sum()
        assert e_side < eps
        # the zeroed offset -n row and column
        assert np.all(p_gpu[0, :] == 0) or np.max(np.abs(p_gpu[0, :])) < 1e-6 * wt[:, c].sum()


def test_make_psf_kernel_vla_like_full_size():
    obs = make_config(1, with_sky=False)
    assert obs.n_row == 1_010_880
    _psf_check(obs, [0], n_samp=256, seed=41)


def test_make_psf_kernel_meerkat_like_8192_grid_three_channels():
    obs = make_config(3, n_int=400, with_sky=False)
    assert obs.nx == 4096 and obs.n_chan == 16
    _psf_check(obs, [0, 7, 15], n_samp=96, seed=42)


def even_psf(rng, nx, ny):
    """A periodically even PSF-like array on the 2nx x 2ny grid (peak at (nx, ny),
    offset -n row and column zero): unit peak plus random sidelobes decaying as
    1 / (1 + r / 64)."""
    gx = np.fft.fftfreq(2 * nx) * 2 * nx
    gy = np.fft.fftfreq(2 * ny) * 2 * ny
    r = np.sqrt(gx[:, None] ** 2 + gy[None, :] ** 2)
    g = rng.standard_normal((2 * nx, 2 * ny)).astype(np.float64) * (0.05 / (1.0 + r / 64.0))
    # even about index 0 (periodically): g[d] + g[-d]
    g = g + np.roll(g[::-1, ::-1], (1, 1), axis=(0, 1))
    g[0, 0] = 1.0
    p = np.fft.fftshift(g)  # peak to (nx, ny)
    p[0, :] = 0.0
    p[:, 0] = 0.0
    return p


def test_psf_apply_4096_per_channel_8192_kernel_sampled_pixels():
    import torch
    from paper_2406_09144_amd import api
    n, n_chan = 4096, 2
    rng = np.random.default_rng(43)
    psfs = [even_psf(rng, n, n) for _ in range(n_chan)]
    K = np.stack([O.response_kernel(p) for p in psfs]).astype(np.float32)
    print(f"[psf-full] apply 4096^2 x {n_chan} channels, kernels {K.shape}", flush=True)
    obs = make_config(3, n_int=2, with_sky=False)
    a = O.n_factor(n, n, obs.dx, obs.dy)
    psf = api.PSF.from_kernels(torch.from_numpy(K).cuda(), nfac=torch.from_numpy(a).float().cuda())
    x = rng.standard_normal((1, n_chan, n, n)).astype(np.float32)
    y = api.apply_RNR_approx(psf, torch.from_numpy(x).cuda()).cpu().numpy()
    for c in range(n_chan):
        pix = rng.choice(n * n, 48, replace=False)
        ref = O.psf_conv_direct(x[0, c].astype(np.float64), psfs[c], a, pix=pix)
        e = rel(y[0, c].ravel()[pix], ref)
        print(f"[psf-full] apply channel {c}: sampled rel err {e:.2e}", flush=True)
        assert e < 1e-6


def test_meerkat_like_32_wplanes():
    import torch
    from paper_2406_09144_amd import api
    obs = make_config(3, with_sky=False)
    assert obs.n_row == 7_257_600 and obs.n_chan == 16
    rng = np.random.default_rng(44)
    n = obs.nx
    pl = api.Plan(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, eps=1e-5, n_wplanes=32)
    info = pl.info
    print(f"[32 planes] W={info['support']} planes={info['n_planes']} w_support={info['w_support']}", flush=True)
    assert info["n_planes"] == 32
    chans = [0, 7, 15]
    sky = torch.randn((obs.n_chan, n, n), device="cuda")
    vis = api.degrid(pl, sky)
    torch.cuda.synchronize()
    rows = rng.choice(obs.n_row, 256, replace=False)
    ch = rng.choice(chans, 256)
    got = vis.cpu().numpy()[rows, ch]
    skyh = sky.cpu().numpy().astype(np.float64)
    ref = O.degrid_rows(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, skyh, rows, ch)
    e = rel(got, ref)
    print(f"[32 planes] degrid sampled rel err {e:.2e}", flush=True)
    assert e < 1e-5
    del vis
    y = torch.randn((obs.n_row, obs.n_chan), dtype=torch.complex64, device="cuda")
    w = torch.rand((obs.n_row, obs.n_chan), device="cuda") + 0.5
    img = api.grid(pl, y, w).cpu().numpy()
    yh = y.cpu().numpy().astype(np.complex128)
    wh = w.cpu().numpy().astype(np.float64)
    for c in chans:
        pix = rng.choice(n * n, 16, replace=False)
        refp = O.grid_pixels(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, yh, pix, chan=c, weight=wh)
        e = rel(img[c].ravel()[pix], refp)
        print(f"[32 planes] grid channel {c} sampled rel err {e:.2e}", flush=True)
        assert e < 1e-5
