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


def minor_cycle(psf, d, s, i_prev, inv_power, lam, n_steps=8, cg_iters=20, max_step=2.0, log=None,
                adaptive=True):
    """Damped Gauss-Newton MAP steps on the FAST likelihood; d is the minor cycle's
    data image, i_prev the sky the previous major cycle subtracted (None at first).
    Returns the log-sky, its FAST H and the damping to continue with.  With
    adaptive=False the schedule is fixed: every step is taken (no acceptance
    test) and lambda stays as given."""
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
        accepted = (not adaptive) or float(Hc[0]) <= float(H[0])
        if accepted:
            sb, H, g = cand, Hc, gc
            if adaptive:
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


def mgvi_minor_cycle(psf, d, xi, power, s0=None, i_fixed=None, n_samples=2, n_iter=4, cg_iters=20, seed=0,
                     log=None):
    """MGVI (Sec. 3.3.5) on the FAST posterior in standardised coordinates: the
    log-sky is s = s0 + A xi (A = F^-1 sqrt(P) F, the Gaussian process of the
    prior; xi has the white prior 1/2 xi^T xi).  Each iteration draws n_samples
    antithetic pairs +-x_j, x_j = M^-1 (a draw with covariance M) at the current
    mean, estimates the KL and its gradient by the sample average of H and dH/dxi,
    and takes the natural-gradient step -M^-1 g, halved until the estimate drops.
    power: [nx, ny/2+1] P(k); d: [n_chan, nx, ny].  Returns xi, the last KL
    estimate and the samples of the last iteration (offsets of xi)."""
    from ._lib import FR_CONV_MUL_SQRT
    gen = torch.Generator(device=d.device).manual_seed(seed)
    shape = tuple(d.shape)

    def logsky(z):
        s = api.periodic_conv(power, z.contiguous(), FR_CONV_MUL_SQRT)
        return s if s0 is None else s + s0

    def kl(z, samples):
        X = torch.stack([z + x for x in samples]).contiguous()  # [2S, n_chan, nx, ny]
        H, g_s = api.likelihood_grad(FR_LIK_FAST, logsky(X), d, psf=psf, i_fixed=i_fixed)
        g = api.periodic_conv(power, g_s.contiguous(), FR_CONV_MUL_SQRT) + X
        prior = 0.5 * (X.double() ** 2).sum(dim=(1, 2, 3))
        return float((H + prior).mean()), g.mean(dim=0).contiguous()

    H = None
    samples = []
    for it in range(n_iter):
        D = torch.exp(logsky(xi)).contiguous()
        samples = []
        for _ in range(n_samples):
            eta0 = torch.randn(shape, generator=gen, device=d.device, dtype=d.dtype)
            eta1 = torch.randn(shape, generator=gen, device=d.device, dtype=d.dtype)
            x, _, _ = api.mgvi_solve(psf, power, D, api.mgvi_draw(psf, power, D, eta0, eta1), maxiter=cg_iters)
            samples += [x, -x]
        H, g = kl(xi, samples)
        step, _, _ = api.mgvi_solve(psf, power, D, (-g).contiguous(), maxiter=cg_iters)
        t, accepted = 1.0, False
        while t >= 1.0 / 64:
            cand = (xi + t * step).contiguous()
            Hc, _ = kl(cand, samples)
            if Hc < H:
                xi, H, accepted = cand, Hc, True
                break
            t *= 0.5
        if log is not None:
            log(f"  MGVI iteration {it}: KL estimate {H:.6e} ({'step ' + format(t, '.3g') if accepted else 'no step'})")
    return xi, H, samples
