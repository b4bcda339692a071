"""The serving loop on the GPU.

  * Every request's result in the concurrent, batched mix equals the same request
    computed alone, bit for bit: all operations are deterministic (fixed-order
    reductions, gridding through integer fixed-point tiles and an owner-computes
    assembly), and batched and single launches share their kernels.
  * Every served result matches the FP64 oracle: PSF applies and the FAST
    likelihood gradient (FFT rounding: 1e-5 and 2e-5), degridding and gridding on sampled
    outputs (epsilon 1e-5), and the 20-iteration CG against the oracle's FP64 CG
    (FP32 vectors drift from FP64 iterates at about kappa * u32 per iteration;
    with the prior floored at 1e-3 of the PSF spectrum peak the drift after 20
    iterations stays near 1e-5: tolerance 1e-3).  The jobs' PSF kernels,
    visibilities and dirty images come from the oracle and the seeded inputs, so
    nothing the oracle sees was computed by the GPU.
  * Footprint admission keeps the in-flight scratch within the budget."""

import numpy as np
import pytest

import oracle as O
from synthetic import make_config
from synthetic.skies import correlated_field, power_spectrum

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a, np.complex128).ravel(), np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def build_jobs(api, torch):
    from paper_2406_09144_amd.serving import ServedJob
    jobs, orc = [], []
    for k, (cfg, n, n_int) in enumerate([(0, 64, 12), (1, 64, 16), (3, 32, 2)]):
        o = make_config(cfg, n=n, n_int=n_int, with_sky=False, n_chan=1)
        freq = o.freq[:1]
        rng = np.random.default_rng(50 + k)
        pl = api.Plan(o.uvw, freq, n, n, o.dx, o.dy, eps=1e-5)
        wt = rng.uniform(0.5, 2.0, (o.n_row, 1))
        psf0 = O.psf0(o.uvw, freq, n, n, o.dx, o.dy, wt)
        K = O.response_kernel(psf0)
        KN = O.noise_kernel(psf0, 1e-3 * psf0.max())
        a = O.n_factor(n, n, o.dx, o.dy)
        psf = api.PSF.from_kernels(torch.from_numpy(K[None]).float().cuda(),
                                   torch.from_numpy(np.ascontiguousarray(KN[:, : n // 2 + 1])[None]).float().cuda(),
                                   torch.from_numpy(a).float().cuda())
        sky = np.exp(correlated_field(rng, n, n))
        V = O.degrid(o.uvw, freq, n, n, o.dx, o.dy, sky[None])
        d = O.grid(o.uvw, freq, n, n, o.dx, o.dy, V, wt)
        imgs = rng.standard_normal((6, 1, n, n))
        logs = 0.3 * rng.standard_normal((6, 1, n, n))
        # prior floor at 1e-3 of the PSF spectrum peak (as in the 512^2 CG test):
        # FP32 CG iterates follow the FP64 ones only while kappa * u32 stays small,
        # and with the unscaled slope -4 spectrum kappa(A) reaches ~1e8 at 64^2
        ip_full = 1.0 / power_spectrum(n, n)
        ip_full = ip_full * (np.abs(K).max() * 1e-3 / ip_full.min())
        ip = torch.from_numpy(np.ascontiguousarray(ip_full[:, : n // 2 + 1])).float().cuda()
        jobs.append(ServedJob(pl, psf, torch.from_numpy(V).to(torch.complex64).cuda(),
                              torch.from_numpy(wt).float().cuda(), torch.from_numpy(d).float().cuda(), ip,
                              torch.from_numpy(imgs).float().cuda(), torch.from_numpy(logs).float().cuda()))
        orc.append(dict(o=o, freq=freq, n=n, wt=wt, K=K, KN=KN, a=a, V=V, d=d, imgs=imgs, logs=logs, ip=ip_full))
    return jobs, orc


def alone(api, J, r):
    from paper_2406_09144_amd._lib import FR_LIK_FAST
    import torch
    P = J.images.shape[0]
    if r.op == "psf_apply":
        return api.apply_RNR_approx(J.psf, J.images[r.rid % P][None])
    if r.op == "lik_fast":
        s = torch.stack([J.logsky[(r.rid + k) % P] for k in range(r.size)])
        return api.likelihood_grad(FR_LIK_FAST, s, J.dirty, psf=J.psf, inv_power=J.inv_power)[1]
    if r.op == "degrid":
        return api.degrid(J.plan, J.images[r.rid % P])
    if r.op == "grid":
        return api.grid(J.plan, J.vis, J.weight)
    return api.cg_solve(J.images[r.rid % P], psf=J.psf, inv_power=J.inv_power, maxiter=20)[0]


def oracle_check(q, r, got, rng):
    """Relative error of the served result `got` (host) against the oracle."""
    o, n, P = q["o"], q["n"], q["imgs"].shape[0]
    if r.op == "psf_apply":
        ref = O.psf_conv_fft(q["imgs"][r.rid % P, 0], q["K"], q["a"])
        return rel(got.reshape(n, n), ref), 1e-5
    if r.op == "lik_fast":
        errs = []
        for k in range(r.size):
            _, g = O.likelihood_fast(q["logs"][(r.rid + k) % P, 0], q["d"][0], q["K"], q["KN"], q["a"],
                                     inv_power=q["ip"])
            errs.append(rel(got.reshape(r.size, n, n)[k], g))
        return max(errs), 2e-5
    if r.op == "degrid":
        rows = np.sort(rng.choice(o.n_row, min(64, o.n_row), replace=False))
        ref = O.degrid_rows(o.uvw, q["freq"], n, n, o.dx, o.dy, q["imgs"][r.rid % P], rows, np.zeros_like(rows))
        return rel(got.reshape(-1)[rows], ref), 2e-5
    if r.op == "grid":
        pix = np.sort(rng.choice(n * n, 64, replace=False))
        ref = O.grid_pixels(o.uvw, q["freq"], n, n, o.dx, o.dy, q["V"], pix, weight=q["wt"])
        return rel(got.reshape(-1)[pix], ref), 2e-5
    x, _ = O.cg(lambda p: O.metric_apply(p, q["K"], q["ip"], q["a"]), q["imgs"][r.rid % P, 0], 20)
    return rel(got.reshape(n, n), x), 1e-3


def run_mix(api, torch, jobs, keep=True):
    from paper_2406_09144_amd.serving import GpuExecutor, Server, make_trace
    trace = make_trace(len(jobs), 2000.0, 0.04, seed=9)
    assert len(trace) > 40
    ex = GpuExecutor(jobs, n_slots=3, keep_outputs=keep)
    budget = 3 * max(ex.footprint(j, op, 8) for j in range(len(jobs)) for op in ("psf_apply", "lik_fast", "cg20"))
    srv = Server(ex, n_slots=3, hbm_budget=budget, max_batch=8)
    out = srv.run(trace, realtime=False)
    torch.cuda.synchronize()
    assert srv.peak_bytes <= budget
    assert any(n > 1 for _, _, n, _, _ in srv.launches), "no request was coalesced"
    return ex, srv, out


def test_results_alone_equal_results_in_the_mix_and_the_oracle():
    import torch
    from paper_2406_09144_amd import api
    from paper_2406_09144_amd.serving import latency_stats
    jobs, orc = build_jobs(api, torch)
    ex, srv, out = run_mix(api, torch, jobs)
    rng = np.random.default_rng(17)
    worst = {}
    for r in out:
        got = ex.results[r.rid]
        ref = alone(api, jobs[r.job], r)
        torch.cuda.synchronize()
        got = got.reshape(ref.shape)
        assert torch.equal(got, ref), (r.rid, r.op)
        err, tol = oracle_check(orc[r.job], r, got.cpu().numpy(), rng)
        assert err < tol, (r.rid, r.op, err)
        worst[r.op] = max(worst.get(r.op, 0.0), err)
    print("worst relative error against the oracle per op:", worst, flush=True)
    assert set(worst) == {"psf_apply", "lik_fast", "degrid", "grid", "cg20"}
    st = latency_stats(out, from_release=True)
    assert st["p99_ms"] >= st["p50_ms"]
