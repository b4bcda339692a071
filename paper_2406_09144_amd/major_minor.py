"""The fast-resolve inference scheme (Algorithm 1, Sec. 3.3.4) over the library.

    I_D <- R^+ N^-1 V                   (exact gridding, once)
    d_0 <- I_D
    for i in 0 .. n_major - 1:
        minor cycle: estimate the sky from d_i = I_PSF * (I - I_{i-1}) + n'
        I_i <- the estimate
        major cycle: d_{i+1} <- I_D - R^+ N^-1 R I_i   (exact operators)

The minor cycle here is a maximum-a-posteriori estimate of the log-sky s
(I = exp s) under the FAST likelihood (eq. ham_new with the PSF and noise-kernel
convolutions) and the Gaussian prior 1/2 s^T S^-1 s.  Each step is a damped
Gauss-Newton (Levenberg-Marquardt) step: the likelihood's metric
D R' N'^-1 R' D (D = diag(exp s)) is replaced by D R' D, which it equals wherever
the PSF spectrum dominates the regulariser (N' = R' + eps), so the step solves
(D R' D + S^-1 + lambda 1) ds = -g with the library's CG (lambda enters as a
constant added to the prior spectrum), with lambda lowered after an accepted
step and raised after a rejected one.  The paper uses MGVI/geoVI for this
cycle; the MAP step exercises the same operators (the FAST likelihood gradient
and the metric CG solve) without the sampling machinery.  The driver is host
orchestration: the vector updates between library calls are plain torch ops.
"""

import torch

from . import api
from ._lib import FR_LIK_FAST


def _H_and_grad(psf, s, d, i_fixed, inv_power):
    return api.likelihood_grad(FR_LIK_FAST, s, d, psf=psf, i_fixed=i_fixed, inv_power=inv_power)


def minor_cycle(psf, d, s, i_prev, inv_power, lam, n_steps=8, cg_iters=20, max_step=2.0, log=None):
    """Damped Gauss-Newton MAP steps on the FAST likelihood; d is the minor cycle's
    data image, i_prev the sky the previous major cycle subtracted (None at first).
    Returns the log-sky, its FAST H and the damping to continue with."""
    ifix = None if i_prev is None else (-i_prev).contiguous()
    sb = s[None].contiguous()
    H, g = _H_and_grad(psf, sb, d, ifix, inv_power)
    for k in range(n_steps):
        D = torch.exp(sb[0])
        ip = (inv_power + lam).contiguous()
        ds, _, _ = api.cg_solve((-g[0]).contiguous(), psf=psf, inv_power=ip, diag=D, maxiter=cg_iters)
        dmax = float(ds.abs().max())
        if not dmax > 0:
            break
        t = min(1.0, max_step / dmax)  # exp(s) is nonlinear: bound the log-sky change
        cand = (sb + t * ds[None]).contiguous()
        Hc, gc = _H_and_grad(psf, cand, d, ifix, inv_power)
        accepted = float(Hc[0]) <= float(H[0])
        if accepted:
            sb, H, g = cand, Hc, gc
            lam *= 0.3
        else:
            lam *= 10.0
        if log is not None:
            log(f"  minor step {k}: H {float(H[0]):.6e} ({'accepted' if accepted else 'rejected'}, "
                f"t = {t:.3g}, lambda -> {lam:.3g})")
    return sb[0], float(H[0]), lam


def reconstruct(plan, psf, vis, weight, inv_power, n_major=3, n_minor=8, cg_iters=20, s0=None, lam0=None,
                log=None):
    """Run the major/minor scheme; returns the log-sky, the sky and the norms of the
    major-cycle residual images ||d_i|| (i = 0 .. n_major)."""
    I_D = api.grid(plan, vis, weight)
    d = I_D
    norms = [float(torch.linalg.vector_norm(d.double()))]
    s = s0 if s0 is not None else torch.zeros_like(I_D)
    lam = lam0 if lam0 is not None else 1e-2 * float(psf.kernels()[0].abs().max())
    I_prev = None
    for i in range(n_major):
        s, H, lam = minor_cycle(psf, d, s, I_prev, inv_power, lam, n_steps=n_minor, cg_iters=cg_iters, log=log)
        I = torch.exp(s)
        # major cycle: exact residual against the dirty image
        d = (I_D - api.apply_RNR_exact(plan, I, weight)).contiguous()
        norms.append(float(torch.linalg.vector_norm(d.double())))
        if log is not None:
            log(f"major {i}: H_fast {H:.6e}, ||d|| {norms[-2]:.6e} -> {norms[-1]:.6e}")
        I_prev = I
    return s, torch.exp(s), norms
