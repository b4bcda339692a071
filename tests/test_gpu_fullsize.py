"""Parity at the workloads' full sizes, in the launch configuration the benchmark
times, on outputs the oracle computes one by one:

  * VLA-like 512^2, 1,010,880 visibilities with w (FP32, eps = 1e-5): degridding
    on a random sample of visibilities, gridding on a random sample of pixels,
    the PSF-convolution response on a sample of output pixels (brute force);
  * the same VLA-like workload with an FP64 plan at eps = 1e-11 (bound 1e-10);
  * MeerKAT-like 4096^2 x 16 channels, 7,257,600 rows (116 M visibilities): the
    same samples on three channels.

The sampled relative error is ||gpu - oracle|| / ||oracle|| over the sample; the
bound is the eps the plan was made for.
"""

import numpy as np
import pytest

import oracle as O
from synthetic import make_config

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _check_plan(obs, chans, n_vis_sample=2048, n_pix_sample=96, seed=0, fp64=False, eps=1e-5, bound=1e-5):
    import torch
    from paper_2406_09144_amd import api
    rng = np.random.default_rng(seed)
    n = obs.nx
    rd, cd = (torch.float64, torch.complex128) if fp64 else (torch.float32, torch.complex64)
    print(f"[fullsize] {obs.n_vis} visibilities, {n}x{n}, {obs.n_chan} channel(s), fp64={fp64}", flush=True)
    pl = api.Plan(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, eps=eps, fp64=fp64)
    info = pl.info
    print(f"[fullsize] plan: W={info['support']} planes={info['n_planes']} items={info['n_workitems']}", flush=True)
    sky = torch.from_numpy(obs.sky).to(rd).cuda() if obs.sky is not None else \
        torch.from_numpy(rng.standard_normal((obs.n_chan, n, n))).to(rd).cuda()
    vis = api.degrid(pl, sky)
    torch.cuda.synchronize()
    rows = rng.choice(obs.n_row, n_vis_sample, replace=False)
    ch = rng.choice(chans, n_vis_sample)
    skyh = sky.cpu().numpy().astype(np.float64)
    got = vis.cpu().numpy()[rows, ch]
    ref = O.degrid_rows(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, skyh, rows, ch)
    e_deg = rel(got, ref)
    print(f"[fullsize] degrid sampled rel err {e_deg:.2e}", flush=True)
    assert e_deg < bound
    # gridding: random data and weights, sampled pixels per channel
    y = torch.randn((obs.n_row, obs.n_chan), dtype=cd, device="cuda")
    w = torch.rand((obs.n_row, obs.n_chan), dtype=rd, device="cuda") + 0.5
    img = api.grid(pl, y, w).cpu().numpy()
    yh = y.cpu().numpy().astype(np.complex128)
    wh = w.cpu().numpy().astype(np.float64)
    for c in chans:
        pix = rng.choice(n * n, n_pix_sample, replace=False)
        refp = O.grid_pixels(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, yh, pix, chan=c, weight=wh)
        e_grid = rel(img[c].ravel()[pix], refp)
        print(f"[fullsize] grid channel {c} sampled rel err {e_grid:.2e}", flush=True)
        assert e_grid < bound
    return pl


def test_vla_like_full_size():
    obs = make_config(1)
    assert obs.n_vis == 1_010_880
    pl = _check_plan(obs, chans=[0])
    # the coverage leaves whole tile columns of the uv grid empty, so the parity
    # above is that of the w-plane transforms restricted to the active columns
    info = pl.info
    ntu, ntv = info["nu"] // info["tile"], info["nv"] // info["tile"]
    print(f"[fullsize] active tiles {info['active_tiles']} of {ntu * ntv}, tile columns "
          f"{info['active_tile_cols']} of {ntv}", flush=True)
    assert 0 < info["active_tile_cols"] < ntv
    assert 0 < info["active_tiles"] < ntu * ntv


def test_vla_like_full_size_fp64():
    """The FP64 plain form at full size: FP64 plan at eps = 1e-11, bound 1e-10."""
    obs = make_config(1)
    _check_plan(obs, chans=[0], n_vis_sample=1024, n_pix_sample=64, fp64=True, eps=1e-11, bound=1e-10)


def test_meerkat_like_full_size():
    obs = make_config(3, with_sky=False)
    assert obs.n_row == 7_257_600 and obs.n_chan == 16 and obs.nx == 4096
    _check_plan(obs, chans=[0, 7, 15], n_vis_sample=256, n_pix_sample=16)


def test_psf_apply_full_size_batch8_sampled_pixels():
    """N = 512, B = 8, kernel from the oracle PSF of a subset of the tracks; the
    brute-force convolution on a sample of output pixels."""
    import torch
    from paper_2406_09144_amd import api
    n = 512
    o = make_config(2, n=n, n_int=16, with_sky=False)
    rng = np.random.default_rng(3)
    wt = rng.uniform(0.5, 2.0, o.n_row)
    p0 = O.psf0(o.uvw, o.freq, n, n, o.dx, o.dy, wt)
    K = O.response_kernel(p0)
    a = O.n_factor(n, n, o.dx, o.dy)
    psf = api.PSF.from_kernels(torch.from_numpy(K[None]).float().cuda(), nfac=torch.from_numpy(a).float().cuda())
    x = rng.standard_normal((8, 1, n, n))
    y = api.apply_RNR_approx(psf, torch.from_numpy(x).float().cuda()).cpu().numpy()
    for b in (0, 7):
        pix = rng.choice(n * n, 64, replace=False)
        ref = O.psf_conv_direct(x[b, 0], p0, a, pix=pix)
        assert rel(y[b, 0].ravel()[pix], ref) < 1e-6
