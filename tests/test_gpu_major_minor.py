"""Algorithm 1 (Sec. 3.3.4) over the library: the exact major-cycle residual
||d_i|| = ||I_D - R^+ N^-1 R I_i|| shrinks from cycle to cycle, and the exact
likelihood of the final sky is far below that of the starting sky."""

import numpy as np
import pytest

from synthetic import make_config
from synthetic.configs import config_rng, noise_from_model
from synthetic.skies import inv_power_half

pytestmark = pytest.mark.gpu


def test_major_minor_reduces_residual():
    import torch
    from paper_2406_09144_amd import api, major_minor
    from paper_2406_09144_amd._lib import FR_LIK_EXACT
    n = 64
    obs = make_config(1, n=n, n_int=240)
    pl = api.Plan(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, eps=1e-5)
    sky = torch.from_numpy(obs.sky).float().cuda()
    model = api.degrid(pl, sky).cpu().numpy().astype(np.complex128)
    noise, wt = noise_from_model(config_rng(1, "noise"), model, rel=0.05)
    V = torch.from_numpy(model + noise).to(torch.complex64).cuda()
    w = torch.from_numpy(wt).float().cuda()
    psf = api.make_psf_kernel(pl, w, eps_noise=-1e-4)
    ip = torch.from_numpy(inv_power_half(n, n)).float().cuda()
    s0 = torch.full((1, n, n), float(np.log(obs.sky.mean())), device="cuda")
    lines = []
    s, I, norms = major_minor.reconstruct(pl, psf, V, w, ip, n_major=3, n_minor=4, cg_iters=20, s0=s0,
                                          log=lines.append)
    print("\n".join(lines))
    print("||d_i||:", norms)
    assert norms[1] < 0.5 * norms[0]
    assert norms[-1] <= norms[1] * 1.05
    H0, _ = api.likelihood_grad(FR_LIK_EXACT, s0[None].contiguous(), V, plan=pl, weight=w)
    H1, _ = api.likelihood_grad(FR_LIK_EXACT, s[None].contiguous(), V, plan=pl, weight=w)
    print("exact H:", float(H0), "->", float(H1))
    assert float(H1) < 0.1 * float(H0)
