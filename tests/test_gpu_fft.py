"""The hand-written LDS Stockham FFT against numpy (FP64 on the host)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("shape", [(2, 2), (16, 32), (64, 64), (3, 256, 128), (1024, 1024), (8, 2048),
                                   (2, 4096, 8), (2, 8192), (16384, 2), (2, 16384),
                                   # mixed radix: 3 2^p and 5 2^p (reduced PSF padding)
                                   (3, 5), (6, 10), (2, 12, 40), (48, 80), (3, 96, 160), (640, 768),
                                   (1280, 24), (2, 12288), (10240, 2), (2, 6144), (5120, 4),
                                   # 8192-long columns in strips of two
                                   (8192, 4), (2, 8192, 6)])
@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft2_matches_numpy(shape, fp64, sign):
    import torch
    from paper_2406_09144_amd import api
    if fp64 and max(shape[-2:]) > 8192:
        pytest.skip("FP64 lines are limited to 8192")
    rng = np.random.default_rng(sum(shape) + 7 * fp64 + sign)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    dt = torch.complex128 if fp64 else torch.complex64
    t = torch.from_numpy(x).to(dt).cuda().contiguous()
    api.fft2(t, sign=sign)
    torch.cuda.synchronize()
    ref = np.fft.fft2(x) if sign < 0 else np.fft.ifft2(x) * (shape[-1] * shape[-2])
    err = rel(t.cpu().numpy(), ref)
    assert err < (1e-13 if fp64 else 2e-6), err


@pytest.mark.parametrize("shape", [(9, 16), (15, 16), (16, 7), (16, 24576)])
def test_fft2_rejects_unsupported_lengths(shape):
    import torch
    from paper_2406_09144_amd import api, FrError
    t = torch.zeros(shape, dtype=torch.complex64, device="cuda")
    with pytest.raises(FrError):
        api.fft2(t)
