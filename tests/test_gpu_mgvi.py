"""MGVI pieces of the minor cycle (Sec. 3.3.5) in standardised coordinates against
the FP64 oracle: the periodic convolutions (kernel, inverse, square roots), the
metric M = 1 + A D R' N'^-1 R' D A, draws with covariance M, and the CG solve
whose output on a draw is an MGVI sample offset.

Tolerances: FP64 1e-10 (1e-11 for single applies); FP32 1e-5 relative L2, CG
iterates for k <= 10 at a metric condition number below ~1e2 (as cg_solve)."""

import numpy as np
import pytest

import oracle as O
from synthetic import make_config
from synthetic.skies import power_spectrum

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def tdev(x, fp64):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.float64 if fp64 else torch.float32).cuda()


def system(n=32, n_chan=1, seed=51):
    """Kernels scaled so the metric's condition number stays below ~1e2."""
    o = make_config(1, n=n, n_int=24, with_sky=False)
    rng = np.random.default_rng(seed)
    Ks, KNs = [], []
    for c in range(n_chan):
        wt = rng.uniform(0.5, 2.0, o.n_row)
        p0 = O.psf0(o.uvw, o.freq, n, n, o.dx, o.dy, wt)
        p0 = p0 / p0.max()
        K = O.response_kernel(p0)
        scale = np.abs(K).max()
        Ks.append(K / scale)
        KNs.append(O.noise_kernel(p0 / scale, 0.1))
    a = O.n_factor(n, n, o.dx, o.dy)
    power = power_spectrum(n, n)
    power = power / power.max()
    xi = 0.5 * rng.standard_normal((n_chan, n, n))
    diag = np.exp(np.stack([O.gp_apply(xi[c], power) for c in range(n_chan)]))
    return np.stack(Ks), np.stack(KNs), a, power, diag, rng


def make_psf(K, KN, a, fp64):
    from paper_2406_09144_amd import api
    n = KN.shape[-2]
    return api.PSF.from_kernels(tdev(K, fp64), tdev(KN[..., : n // 2 + 1], fp64), tdev(a, fp64))


@pytest.mark.parametrize("n", [32, 64])
@pytest.mark.parametrize("fp64", [False, True])
def test_periodic_conv_modes_vs_oracle(n, fp64):
    from paper_2406_09144_amd import api
    from paper_2406_09144_amd import _lib as L
    K, KN, a, power, diag, rng = system(n, n_chan=2)
    x = rng.standard_normal((3, 2, n, n))
    half = lambda k: k[..., : n // 2 + 1]
    tol = 1e-11 if fp64 else 1e-5
    refs = {
        L.FR_CONV_MUL: lambda v, c: O.noise_apply(v, KN[c]),
        L.FR_CONV_DIV: lambda v, c: O.noise_inv_apply(v, KN[c]),
        L.FR_CONV_DIV_SQRT: lambda v, c: O.noise_inv_sqrt_apply(v, KN[c]),
    }
    for mode, ref in refs.items():
        y = api.periodic_conv(tdev(half(KN), fp64), tdev(x, fp64), mode).cpu().numpy()
        for b in range(3):
            for c in range(2):
                assert rel(y[b, c], ref(x[b, c], c)) < tol, (mode, b, c)
    # the Gaussian-process map and its inverse, one shared spectrum
    y = api.periodic_conv(tdev(half(power), fp64), tdev(x, fp64), L.FR_CONV_MUL_SQRT).cpu().numpy()
    z = api.periodic_conv(tdev(half(power), fp64), tdev(y, fp64), L.FR_CONV_DIV_SQRT).cpu().numpy()
    for b in range(3):
        for c in range(2):
            assert rel(y[b, c], O.gp_apply(x[b, c], power)) < tol
            assert rel(z[b, c], x[b, c]) < 10 * tol


@pytest.mark.parametrize("n,n_chan", [(32, 1), (64, 2)])
@pytest.mark.parametrize("fp64", [False, True])
def test_mgvi_metric_and_draw_vs_oracle(n, n_chan, fp64):
    from paper_2406_09144_amd import api
    K, KN, a, power, diag, rng = system(n, n_chan)
    psf = make_psf(K, KN, a, fp64)
    pw = tdev(power[:, : n // 2 + 1], fp64)
    x = rng.standard_normal((n_chan, n, n))
    e0, e1 = rng.standard_normal((n_chan, n, n)), rng.standard_normal((n_chan, n, n))
    y = api.mgvi_metric_apply(psf, pw, tdev(diag, fp64), tdev(x, fp64)).cpu().numpy()
    xi = api.mgvi_draw(psf, pw, tdev(diag, fp64), tdev(e0, fp64), tdev(e1, fp64)).cpu().numpy()
    tol = 1e-11 if fp64 else 1e-5
    for c in range(n_chan):
        assert rel(y[c], O.mgvi_metric_apply(x[c], K[c], KN[c], power, diag[c], a)) < tol, c
        assert rel(xi[c], O.mgvi_draw(e0[c], e1[c], K[c], KN[c], power, diag[c], a)) < tol, c
    # diag = NULL is D = 1
    y1 = api.mgvi_metric_apply(psf, pw, None, tdev(x, fp64)).cpu().numpy()
    assert rel(y1[0], O.mgvi_metric_apply(x[0], K[0], KN[0], power, np.ones((n, n)), a)) < tol


@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("k", [1, 5, 10])
def test_mgvi_solve_iterates_vs_oracle(fp64, k):
    import torch
    from paper_2406_09144_amd import api
    n = 32
    K, KN, a, power, diag, rng = system(n)
    psf = make_psf(K, KN, a, fp64)
    pw = tdev(power[:, : n // 2 + 1], fp64)
    e0, e1 = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    xi = api.mgvi_draw(psf, pw, tdev(diag, fp64), tdev(e0[None], fp64), tdev(e1[None], fp64))
    x, hist, it = api.mgvi_solve(psf, pw, tdev(diag, fp64), xi, maxiter=k)
    torch.cuda.synchronize()
    xr, hr = O.mgvi_sample(e0, e1, K[0], KN[0], power, diag[0], maxiter=k, a=a)
    tol = 1e-10 if fp64 else 1e-5
    assert int(it) == k
    assert rel(x.cpu().numpy()[0], xr) < tol
    assert rel(hist.cpu().numpy(), hr) < tol


def test_mgvi_sample_fp64_converges_to_the_dense_solve():
    import torch
    from paper_2406_09144_amd import api
    n = 16
    K, KN, a, power, diag, rng = system(n)
    psf = make_psf(K, KN, a, True)
    pw = tdev(power[:, : n // 2 + 1], True)
    e0, e1 = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    xi = api.mgvi_draw(psf, pw, tdev(diag, True), tdev(e0[None], True), tdev(e1[None], True))
    x, hist, it = api.mgvi_solve(psf, pw, tdev(diag, True), xi, maxiter=300, rtol=1e-12)
    torch.cuda.synchronize()
    cols = []
    for q in range(n * n):
        e = np.zeros(n * n)
        e[q] = 1
        cols.append(O.mgvi_metric_apply(e.reshape(n, n), K[0], KN[0], power, diag[0], a).ravel())
    M = np.array(cols).T
    draw = O.mgvi_draw(e0, e1, K[0], KN[0], power, diag[0], a)
    assert rel(x.cpu().numpy().ravel(), np.linalg.solve(M, draw.ravel())) < 1e-10
    assert 0 < int(it) < 300


def test_mgvi_metric_512_bench_shape():
    """The VLA-like 512 x 512 shape (doubled-grid PSF of a real plan-free kernel)."""
    from paper_2406_09144_amd import api
    n = 512
    o = make_config(1, n=n, n_int=4, with_sky=False)
    rng = np.random.default_rng(9)
    p0 = O.psf0(o.uvw, o.freq, n, n, o.dx, o.dy, np.ones(o.n_row))
    K = O.response_kernel(p0)
    KN = O.noise_kernel(p0, 1e-1 * p0.max())
    power = power_spectrum(n, n)
    diag = np.exp(0.2 * rng.standard_normal((n, n)))
    psf = make_psf(K[None], KN[None], np.ones((n, n)), False)
    x = rng.standard_normal((n, n))
    y = api.mgvi_metric_apply(psf, tdev(power[:, : n // 2 + 1], False), tdev(diag[None], False),
                              tdev(x[None], False)).cpu().numpy()
    assert rel(y[0], O.mgvi_metric_apply(x, K, KN, power, diag)) < 1e-5


def test_mgvi_errors():
    import torch
    from paper_2406_09144_amd import api, FrError
    n = 16
    K, KN, a, power, diag, rng = system(n)
    no_kn = api.PSF.from_kernels(tdev(K, False))
    pw = tdev(power[:, : n // 2 + 1], False)
    x = torch.zeros((1, n, n), device="cuda")
    with pytest.raises(FrError):
        api.mgvi_metric_apply(no_kn, pw, None, x)
    with pytest.raises(FrError):
        api.mgvi_draw(no_kn, pw, None, x, x)
    psf = make_psf(K, KN, a, False)
    with pytest.raises(FrError):
        api.mgvi_solve(psf, pw, None, x, maxiter=-1)
    with pytest.raises(FrError):
        api.periodic_conv(pw, torch.zeros((2, n, n), device="cuda"), mode=7)
