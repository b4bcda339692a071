"""apply_RNR_approx (zero-padded PSF convolution, Sec. 3.3.2) against the FP64
oracle, with the oracle's response kernel as input."""

import numpy as np
import pytest

import oracle as O
from synthetic import make_config

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def oracle_kernels(n, n_int=8, seeds=(0,), ny=None):
    obs = make_config(1, n=n, n_int=n_int, with_sky=False)
    ny = ny or n
    Ks, psfs = [], []
    for sd in seeds:
        wt = np.random.default_rng(100 + sd).uniform(0.5, 2.0, obs.n_row)
        psf = O.psf0(obs.uvw, obs.freq, n, ny, obs.dx, obs.dy, wt)
        psfs.append(psf)
        Ks.append(O.response_kernel(psf))
    a = O.n_factor(n, ny, obs.dx * 40, obs.dy * 40)  # a non-trivial diagonal
    return np.stack(Ks), psfs, a


@pytest.mark.parametrize("n,ny", [(16, 16), (32, 64), (64, 32), (128, 128), (256, 256)])
@pytest.mark.parametrize("fp64", [False, True])
def test_apply_rnr_approx_vs_oracle(n, ny, fp64):
    import torch
    from paper_2406_09144_amd import api
    K, psfs, a = oracle_kernels(n, ny=ny, seeds=(0, 1))
    rd = torch.float64 if fp64 else torch.float32
    psf = api.PSF.from_kernels(torch.from_numpy(K).to(rd).cuda(), nfac=torch.from_numpy(a).to(rd).cuda())
    rng = np.random.default_rng(n + ny)
    B = 3
    x = rng.standard_normal((B, 2, n, ny))
    y = api.apply_RNR_approx(psf, torch.from_numpy(x).to(rd).cuda())
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    for b in range(B):
        for c in range(2):
            ref = O.psf_conv_fft(x[b, c], K[c], a)
            err = rel(y[b, c], ref)
            assert err < (1e-12 if fp64 else 1e-6), (b, c, err)
    # one image against the brute-force convolution as well
    ref_direct = O.psf_conv_direct(x[0, 1], psfs[1], a)
    assert rel(y[0, 1], ref_direct) < (1e-12 if fp64 else 1e-6)


def test_apply_rnr_approx_512_batch8():
    """The bench shape (N = 512, B = 8) against the oracle."""
    import torch
    from paper_2406_09144_amd import api
    K, _, _ = oracle_kernels(512, n_int=4)
    psf = api.PSF.from_kernels(torch.from_numpy(K).float().cuda())
    rng = np.random.default_rng(5)
    x = rng.standard_normal((8, 1, 512, 512))
    y = api.apply_RNR_approx(psf, torch.from_numpy(x).float().cuda()).cpu().numpy()
    for b in (0, 7):
        assert rel(y[b, 0], O.psf_conv_fft(x[b, 0], K[0])) < 1e-6


def test_apply_rnr_approx_errors():
    import torch
    from paper_2406_09144_amd import api, FrError
    K, _, _ = oracle_kernels(16)
    psf = api.PSF.from_kernels(torch.from_numpy(K).float().cuda())
    x = torch.zeros((1, 1, 16, 16), device="cuda")
    with pytest.raises(FrError):
        api.apply_RNR_approx(psf, x, out=x)
    y = api.apply_RNR_approx(psf, torch.zeros((0, 1, 16, 16), device="cuda"))
    assert y.shape[0] == 0
