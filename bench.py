#!/usr/bin/env python3
"""Benchmark of the interferometric response-operator hot path on one MI355X.

Workload: the VLA-like single-channel observation (27 antennas on a Y with 21 km
arms, 8 h at 10 s: 1,010,880 visibilities with w up to 5% of |uv|max), 512 x 512
sky, FP32 at eps = 1e-5, synthetic seeded data; the PSF-convolution rows use the
batch of 8 log-sky samples of the differentiated-likelihood workload.

One step is one pass over every hot-path operation, inputs resident in HBM:
  degrid (R), grid (R^+ N^-1), PSF-convolution R' apply (B = 8), exact R' (B = 1),
  FAST likelihood + gradient (B = 8), EXACT likelihood + gradient (B = 1),
  50-iteration CG on D R' D + S^-1.
Plan creation and the PSF/noise kernels are built once before timing (resident).

`value` is the (de)gridding rate: 2 n_vis / (device time of degrid + grid), from
hipEvents on the launch stream over the timed steps; the other operations are
reported under "components".  "roofline" covers the kernel with the largest
device time inside the (de)gridding the metric is quoted on (the gridding
spread, a contraction on the matrix cores: algorithmic FLOPs against the FP32
MFMA peak),
from the library's per-kernel hipEvent timing over a second pass of the same
steps (per-launch event brackets are kept out of the step timings);
"roofline_hbm" lists the memory-bound kernels of the same path against HBM, and
the whole degrid and grid calls and the batch-8 PSF apply on the bytes the method
must move (every w-plane written once by its FFT and read once; x, y and the
kernel once per apply); "roofline_lds" rates the degridding kernel against the LDS
(every visibility reads its W^2 Ww footprint values from LDS).
PSF applies/s is the sustained rate of back-to-back batch-8 applies;
"psf_apply_4096" times the apply at the MeerKAT-like channel shape (16 x 4096^2,
8192^2 kernels), the HBM-bound size.  "meerkat_like" is the multi-channel
(de)gridding with the w-planes derived from eps, "meerkat_like_stated_wplanes" the
same with the 32 planes the workload states, each with its HBM fractions.
"served" runs the served mix for 60 s of a Poisson trace at 200 req/s (FP32
continuous batching on 4 streams, with the device overlap of their launches),
replays it unbatched and serially on the plain FP64 form, then sweeps the rate
towards saturation.
"reduced_psf" measures the PSF cut to |offset| <= h on the n + h padded grid:
applies/s, accuracy against the exact R^+ N^-1 R, and the major cycles of the
major/minor scheme it needs.  "mgvi" times the MGVI metric apply, a draw and a
sample (draw + 20-iteration metric CG) of the minor cycle.  "taylor_w" is the
same (de)gridding with the w-term as a Taylor series instead of w-stacking (the
plan option for small w-phases; `value` stays on improved w-stacking).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "vis/s (de)gridding at eps=1e-5; PSF-conv R^dagger N^-1 R applies/s; p99 latency"
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3  # dense FP32 matrix-core peak of the MI355X
# LDS: 128 bytes per clock per CU, 256 CUs at 2.4 GHz
LDS_PEAK_GBS = 128 * 256 * 2.4
PSF_APPLY_REPS = 20
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "grid_traffic.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def grid_flops(info, n_vis):
    """Algorithmic FLOPs of one gridding spread: every visibility adds y * psi to
    W x W x Ww cells, one complex-by-real multiply-add (4 FLOPs) each."""
    W = info["support"]
    Ww = info["w_support"]
    return 4.0 * W * W * Ww * n_vis


def gridder_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in ("gridder.hip", "eskernel.h", "workitem.h"):
        with open(os.path.join(ROOT, "paper_2406_09144_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when the gridder sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = {}
            for line in fh:
                if "=" in line and not line.lstrip().startswith("#"):
                    k, v = line.split("=", 1)
                    rec[k.strip()] = v.strip()
    except OSError:
        return None
    if rec.get("source_digest") != gridder_source_digest() or rec.get("kernel") != kernel:
        return None
    return int(float(rec["hbm_bytes_per_launch"]))


def active_fractions(info):
    """Fractions of the uv tiles that can be non-zero (the only ones degridding reads
    and the assembly writes) and of the tile columns holding one (the only columns
    the w-plane transforms touch); the rest of every plane is zero or unread."""
    tile, n_chan = info["tile"], info["n_chan"]
    ntu, ntv = info["nu"] // tile, info["nv"] // tile
    return info["active_tiles"] / (n_chan * ntu * ntv), info["active_tile_cols"] / (n_chan * ntv)


def algorithmic_bytes(name, info, n_vis, n_row, B_conv, nx, ny):
    """Bytes one launch of kernel `name` must move at minimum (FP32): the w-plane
    figures count only the active tiles and the tile columns holding one."""
    planes = info["n_planes"] * info["nu"] * info["nv"] * 8
    f_tiles, f_cols = active_fractions(info)
    if name == "degrid":
        return planes * f_tiles + 8 * n_vis + 24 * n_row    # active tiles read once, vis written, uvw
    if name == "grid":
        return 12 * n_vis + 24 * n_row                  # vis + weights read (spread into per-item tiles)
    if name == "grid_assemble":
        return planes * f_tiles                         # every active plane cell written once
    if name in ("wplane_rows_fwd",):
        return 4 * nx * ny + info["n_planes"] * nx * info["nv"] * 8 * f_cols
    if name in ("wplane_cols_fwd", "wplane_cols_inv"):
        # band rows of the active columns one way, the active tiles the other
        return info["n_planes"] * 8 * (nx * info["nv"] * f_cols + info["nu"] * info["nv"] * f_tiles)
    if name == "wplane_rows_inv":
        return info["n_planes"] * nx * info["nv"] * 8 * f_cols + 4 * nx * ny
    if name == "psfconv_rows_r2c":
        return B_conv * (4 * nx * ny + 8 * nx * ny)
    if name == "psfconv_cols":
        return B_conv * 2 * 8 * nx * ny + 4 * 2 * nx * (ny + 1)
    if name == "psfconv_rows_c2r":
        return B_conv * (8 * nx * ny + 4 * nx * ny)
    return None


def call_bytes(op, info, n_vis_per_chan, n_row, nx, ny, n_chan=1):
    """Bytes a whole (de)gridding call must move (FP32): the image, every w-plane
    grid written once by its FFT and read once, the visibilities (and weights for
    gridding) and uvw, per channel.  This full-grid figure over-counts what the
    calls move when the uv coverage leaves tiles empty (they touch only the active
    tiles and the tile columns holding one)."""
    per = 4 * nx * ny + info["n_planes"] * 2 * 8 * info["nu"] * info["nv"] + 8 * n_vis_per_chan + 24 * n_row
    if op == "grid":
        per += 4 * n_vis_per_chan
    return n_chan * per


def psf_apply_bytes(n, B, n_chan=1):
    """Bytes of a batch-B PSF-convolution apply per channel kernel (FP32): x and y
    (4 N^2 each per image) and the real half-spectrum kernel K_R, 4 2N (N + 1),
    read once per call: (8 + 8/B) N^2 per image."""
    return n_chan * (B * 8 * n * n + 4 * 2 * n * (n + 1))


def hbm_entry(name, byts, ms):
    ach = byts / (ms * 1e-3) / 1e9
    return {"kernel": name, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_launch": int(byts), "avg_launch_ms": round(ms, 5)}


def psf_apply_4096(api, torch, n=4096, n_chan=16, reps=5):
    """The PSF-convolution apply at the MeerKAT-like channel shape (4096^2 per
    channel, per-channel 8192^2 kernels, 16 channels, B = 1): the HBM-bound size.
    Kernel values do not change the work; they are random positive numbers."""
    g = torch.Generator(device="cuda").manual_seed(12)
    K = torch.rand((n_chan, 2 * n, n + 1), device="cuda", generator=g) + 0.5
    psf = api.PSF.from_kernels(K)
    del K
    x = torch.rand((1, n_chan, n, n), device="cuda", generator=g)
    y = api.apply_RNR_approx(psf, x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        api.apply_RNR_approx(psf, x, out=y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    api.profile_reset()
    api.profile_enable(True)
    for _ in range(reps):
        api.apply_RNR_approx(psf, x, out=y)
    torch.cuda.synchronize()
    api.profile_enable(False)
    kern = {}
    for kname in ("psfconv_rows_r2c", "psfconv_cols", "psfconv_rows_c2r"):
        cnt, tot = api.profile_query(kname)
        if cnt:
            kern[kname] = round(tot / cnt, 4)
    byts = psf_apply_bytes(n, 1, n_chan)
    res = {"workload": f"{n_chan} channels x {n}x{n}, per-channel {2 * n}x{2 * n} kernels, B = 1, FP32",
           "call_ms": round(ms, 4), "applies_per_s": round(n_chan / (ms * 1e-3), 1), "kernels_ms": kern,
           "hbm": hbm_entry("psf_apply_call_4096", byts, ms),
           "two_pass_bytes": int(byts + n_chan * 32 * n * n)}
    del psf, x, y
    torch.cuda.empty_cache()
    return res


def scale_workload(api, torch, steps=3, n_wplanes=0):
    """(De)gridding on the MeerKAT-like multi-channel workload (7,257,600 rows x 16
    channels = 116,121,600 visibilities, 4096 x 4096 per channel, FP32, eps 1e-5):
    the HBM-bound regime at the paper's data scale."""
    import numpy as np
    from synthetic import make_config
    t0 = time.time()
    obs = make_config(3, with_sky=False)
    t_gen = time.time() - t0
    t0 = time.time()
    plan = api.Plan(obs.uvw, obs.freq, obs.nx, obs.ny, obs.dx, obs.dy, eps=1e-5, n_wplanes=n_wplanes)
    torch.cuda.synchronize()
    t_plan = time.time() - t0
    info = plan.info
    g = torch.Generator(device="cuda").manual_seed(11)
    sky = torch.rand((obs.n_chan, obs.nx, obs.ny), device="cuda", generator=g)
    w = torch.rand((obs.n_row, obs.n_chan), device="cuda", generator=g) + 0.5
    vis = api.degrid(plan, sky)
    img = api.grid(plan, vis, w)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(steps):
        api.degrid(plan, sky, out=vis)
    e[1].record()
    for _ in range(steps):
        api.grid(plan, vis, w, out=img)
    e[2].record()
    torch.cuda.synchronize()
    dg = e[0].elapsed_time(e[1]) / steps
    gr = e[1].elapsed_time(e[2]) / steps
    n_vis = obs.n_row * obs.n_chan
    res = {"workload": f"MeerKAT-like: {obs.n_row} rows x {obs.n_chan} channels, {obs.nx}x{obs.ny} per channel, "
                       f"eps=1e-5, FP32, " + (f"{n_wplanes} w-planes (as stated)" if n_wplanes else
                                              "w-planes derived from eps"),
           "n_vis": n_vis, "support": info["support"], "n_planes": info["n_planes"],
           "degrid_ms": dg, "grid_ms": gr, "vis_per_s": 2 * n_vis / ((dg + gr) * 1e-3),
           "plan_create_s": t_plan, "inputs_generated_s": t_gen,
           "hbm": [hbm_entry("degrid_call", call_bytes("degrid", info, obs.n_row, obs.n_row, obs.nx, obs.ny,
                                                       obs.n_chan), dg),
                   hbm_entry("grid_call", call_bytes("grid", info, obs.n_row, obs.n_row, obs.nx, obs.ny,
                                                     obs.n_chan), gr)]}
    del plan, sky, w, vis, img
    torch.cuda.empty_cache()
    return res


def reduced_psf_tradeoff(api, torch, plan, w, V, x8, inv_power, s0, supports=(128, 256, 384, 511),
                         cycle_supports=(384, 256, 128), n_major=6, reps=20):
    """Reduced PSF support (Sec. 3.3.2): speed and accuracy of R' with the PSF cut
    to |offset| <= h on the n + h padded grid, and the effect on the major cycles
    of Algorithm 1 (exact likelihood after each cycle; the count is the number of
    major cycles to reach the value the full PSF reaches after two)."""
    from paper_2406_09144_amd import major_minor
    from paper_2406_09144_amd._lib import FR_LIK_EXACT
    psf = api.make_psf_kernel(plan, w, eps_noise=-1e-1)
    full_y = api.apply_RNR_approx(psf, x8)
    exact = api.apply_RNR_exact(plan, x8[0].contiguous(), w)[0]

    def nrm(t):
        return float(torch.linalg.vector_norm(t.double()))

    rows = []
    for h in (None,) + tuple(supports):
        p = psf if h is None else psf.reduce(h)
        y = api.apply_RNR_approx(p, x8)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            api.apply_RNR_approx(p, x8, out=y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        rows.append({"support": h if h is not None else "full", "padded": [p.px, p.py], "b8_ms": round(ms, 5),
                     "applies_per_s": round(x8.shape[0] / (ms * 1e-3)),
                     "rel_err_vs_exact": nrm(y[0, 0] - exact) / nrm(exact),
                     "rel_err_vs_full_psf": nrm(y - full_y) / nrm(full_y)})

    def H_exact(s):
        return float(api.likelihood_grad(FR_LIK_EXACT, s[None].contiguous(), V, plan=plan, weight=w,
                                         inv_power=inv_power)[0])

    I_D = api.grid(plan, V, w)
    lam0 = 1e-2 * float(psf.kernels()[0].abs().max())
    cycles = {}
    for h in (None,) + tuple(cycle_supports):
        p = psf if h is None else psf.reduce(h)
        d, s, lam, I_prev = I_D, s0, lam0, None
        Hs = [H_exact(s0)]
        for _ in range(n_major):
            s, _, lam = major_minor.minor_cycle(p, d, s, I_prev, inv_power, lam, n_steps=8, cg_iters=20)
            I_prev = torch.exp(s)
            d = (I_D - api.apply_RNR_exact(plan, I_prev, w)).contiguous()
            Hs.append(H_exact(s))
        cycles["full" if h is None else h] = Hs
    target = cycles["full"][2]
    counts = {str(k): next((i for i, v in enumerate(Hs) if v <= target * (1 + 1e-6)), None)
              for k, Hs in cycles.items()}
    return {"workload": "VLA-like 512x512, 1,010,880 visibilities, batch 8, eps_noise 0.1 of the PSF peak",
            "apply": rows, "major_cycles_to_full_psf_H_after_2": counts, "n_major": n_major,
            "exact_H_per_major_cycle": {str(k): [round(v, 1) for v in Hs] for k, Hs in cycles.items()}}


def mgvi_timing(api, torch, plan, w, n, reps=5, cg_iters=20):
    """MGVI pieces at the VLA-like 512 x 512 shape (Sec. 3.3.5, standardised
    coordinates): one metric apply M x, one draw, and one sample (draw + a
    20-iteration CG solve of M x = draw), device time per call."""
    import numpy as np
    from synthetic.skies import power_spectrum
    psf = api.make_psf_kernel(plan, w, eps_noise=-1e-1)
    power = torch.from_numpy(power_spectrum(n, n)[:, : n // 2 + 1]).float().cuda().contiguous()
    g = torch.Generator(device="cuda").manual_seed(5)
    D = torch.exp(0.1 * torch.randn((1, n, n), device="cuda", generator=g)).contiguous()
    e0 = torch.randn((1, n, n), device="cuda", generator=g)
    e1 = torch.randn((1, n, n), device="cuda", generator=g)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    metric_ms = timed(lambda: api.mgvi_metric_apply(psf, power, D, e0))
    draw_ms = timed(lambda: api.mgvi_draw(psf, power, D, e0, e1))
    sample_ms = timed(lambda: api.mgvi_solve(psf, power, D, api.mgvi_draw(psf, power, D, e0, e1),
                                             maxiter=cg_iters))
    return {"workload": f"VLA-like {n}x{n}, PSF-convolution metric, FP32", "metric_apply_ms": round(metric_ms, 5),
            "draw_ms": round(draw_ms, 5), "sample_ms": round(sample_ms, 4), "cg_iters": cg_iters,
            "samples_per_s": round(1e3 / sample_ms, 1)}


def taylor_timing(api, torch, obs, sky, V, w, n, steps=5):
    """The same (de)gridding with the w-term as a Taylor series (FR_W_TAYLOR:
    3 terms instead of 7 w-planes at eps 1e-5 on this array), device time per
    call and the rate."""
    pl = api.Plan(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, eps=1e-5, w_taylor=True)
    vis = api.degrid(pl, sky)
    img = api.grid(pl, V, w)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(steps):
        api.degrid(pl, sky, out=vis)
    e[1].record()
    for _ in range(steps):
        api.grid(pl, V, w, out=img)
    e[2].record()
    torch.cuda.synchronize()
    dg, gr = e[0].elapsed_time(e[1]) / steps, e[1].elapsed_time(e[2]) / steps
    info = pl.info
    return {"w_taylor": info["w_taylor"], "n_planes": info["n_planes"], "support": info["support"],
            "degrid_ms": round(dg, 5), "grid_ms": round(gr, 5), "vis_per_s": 2 * obs.n_vis / ((dg + gr) * 1e-3)}


def build_served_jobs(api, torch, n_jobs, fp64):
    """Resident jobs of the served mix: plan, PSF kernels, data, input pools."""
    import numpy as np
    from paper_2406_09144_amd.serving import ServedJob
    from synthetic.configs import serving_jobs, serving_observation
    from synthetic.skies import correlated_field, inv_power_half
    rd, cd = (torch.float64, torch.complex128) if fp64 else (torch.float32, torch.complex64)
    jobs = []
    for jd in serving_jobs(n_jobs):
        o = serving_observation(jd)
        rng = np.random.default_rng(1000 + jd["job"])
        n = o.nx
        pl = api.Plan(o.uvw, o.freq, n, n, o.dx, o.dy, eps=1e-5, fp64=fp64)
        wt = torch.from_numpy(rng.uniform(0.5, 2.0, (o.n_row, 1))).to(rd).cuda()
        psf = api.make_psf_kernel(pl, wt, eps_noise=-1e-6)
        sky = torch.from_numpy(np.exp(correlated_field(rng, n, n))[None]).to(rd).cuda()
        V = api.degrid(pl, sky)
        d = api.grid(pl, V, wt)
        P = 4
        imgs = torch.exp(torch.from_numpy(0.3 * rng.standard_normal((P, 1, n, n)))).to(rd).cuda()
        logs = torch.from_numpy(0.3 * rng.standard_normal((P, 1, n, n))).to(rd).cuda()
        ip = torch.from_numpy(inv_power_half(n, n)).to(rd).cuda() * float(wt.sum()) * 1e-6
        jobs.append(ServedJob(pl, psf, V.to(cd), wt, d, ip, imgs, logs))
    torch.cuda.synchronize()
    return jobs


def served_workload(api, torch, seconds, rate, n_jobs, fp64_requests, sweep_rates=(), sweep_requests=2000):
    """p50/p99 of the served mix (FP32, continuous batching, 4 streams) against the
    same trace replayed unbatched and serially on the plain FP64 form; the device
    intervals of the FP32 launches give their overlap across streams; then a rate
    sweep towards saturation."""
    from paper_2406_09144_amd.serving import GpuExecutor, Server, latency_stats, make_trace, overlap_stats
    t0 = time.time()
    jobs = build_served_jobs(api, torch, n_jobs, fp64=False)
    log(f"[bench] served jobs built in {time.time() - t0:.1f}s")
    trace = make_trace(len(jobs), rate, seconds)
    ex = GpuExecutor(jobs, n_slots=4, timeline=True)
    srv = Server(ex, n_slots=4, hbm_budget=64 << 30, max_batch=8)
    out = srv.run(trace, realtime=True)
    torch.cuda.synchronize()
    st = latency_stats(out)
    st["launches"] = len(srv.launches)
    st["peak_scratch_GB"] = srv.peak_bytes / 2 ** 30
    iv = ex.timeline_intervals()
    st["device"] = {k: (round(v, 3) if isinstance(v, float) else v)
                    for k, v in overlap_stats([(a, b) for _, _, a, b in iv]).items()}
    st["device"]["busy_fraction"] = round(st["device"]["busy_ms"] / (seconds * 1e3), 4)
    st["coalesced_requests_per_launch"] = round(sum(n for _, _, n, _, _ in srv.launches) / max(1, len(srv.launches)), 3)
    st["per_op"] = {op: {k: round(v, 3) for k, v in latency_stats([r for r in out if r.op == op]).items()
                         if k in ("n", "p50_ms", "p99_ms")}
                    for op in sorted({r.op for r in out})}
    log(f"[bench] served FP32: {json.dumps(st)}")
    res = {"fp32_batched": st, "rate_hz": rate, "seconds": seconds, "n_jobs": n_jobs}
    del ex, srv
    jobs64 = None
    if fp64_requests >= 0:
        jobs64 = build_served_jobs(api, torch, n_jobs, fp64=True)
        trace64 = make_trace(len(jobs64), rate, seconds)
        if fp64_requests > 0:
            trace64 = trace64[:fp64_requests]
        ex64 = GpuExecutor(jobs64, n_slots=1)
        srv64 = Server(ex64, n_slots=1, hbm_budget=64 << 30, max_batch=1)
        out64 = srv64.run(trace64, realtime=True)
        torch.cuda.synchronize()
        st64 = latency_stats(out64)
        log(f"[bench] served FP64 unbatched serial: {json.dumps(st64)}")
        res["fp64_unbatched_serial"] = st64
        del ex64, srv64
    # rate sweep to saturation: the same mix at higher Poisson rates, a fixed
    # number of requests per point, FP32 continuous batching against the plain
    # FP64 form served unbatched and serially
    sweep = []
    for r_hz in sweep_rates:
        tr = make_trace(len(jobs), r_hz, sweep_requests / r_hz, seed=240609149)
        ex = GpuExecutor(jobs, n_slots=4)
        srv = Server(ex, n_slots=4, hbm_budget=64 << 30, max_batch=8)
        o32 = srv.run(tr, realtime=True)
        torch.cuda.synchronize()
        s32 = latency_stats(o32)
        point = {"rate_hz": r_hz, "fp32_batched": {k: round(v, 3) for k, v in s32.items()}}
        if jobs64 is not None:
            tr = make_trace(len(jobs64), r_hz, sweep_requests / r_hz, seed=240609149)
            ex = GpuExecutor(jobs64, n_slots=1)
            srv = Server(ex, n_slots=1, hbm_budget=64 << 30, max_batch=1)
            o64 = srv.run(tr, realtime=True)
            torch.cuda.synchronize()
            point["fp64_unbatched_serial"] = {k: round(v, 3) for k, v in latency_stats(o64).items()}
        log(f"[bench] served sweep: {json.dumps(point)}")
        sweep.append(point)
    res["rate_sweep"] = sweep
    res["sweep_requests_per_point"] = sweep_requests
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=32768,
                    help="visibilities of the oracle CPU-baseline sample (0 disables)")
    ap.add_argument("--fp64-steps", type=int, default=3, help="timed (de)grid passes of the plain FP64 form")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="served-mix trace length (0 disables)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-sweep", type=str, default="1000,3000,10000",
                    help="Poisson rates (req/s) of the saturation sweep, comma-separated ('' disables)")
    ap.add_argument("--serve-sweep-requests", type=int, default=2000, help="requests per sweep point")
    ap.add_argument("--psf4096", type=int, default=1,
                    help="time the PSF apply at 16 x 4096^2 with 8192^2 kernels (0 disables)")
    ap.add_argument("--serve-jobs", type=int, default=16)
    ap.add_argument("--serve-fp64-requests", type=int, default=0,
                    help="requests of the FP64 replay (0: the whole trace, -1: skip it)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run 5 plain copies of this many bytes (counter calibration)")
    ap.add_argument("--scale-steps", type=int, default=2,
                    help="timed (de)grid passes of the MeerKAT-like workload (0 disables)")
    ap.add_argument("--scale-wplanes", type=int, default=32,
                    help="w-planes of the MeerKAT-like workload as stated (0: derive from eps only)")
    ap.add_argument("--reduced-psf", type=int, default=1,
                    help="measure the reduced-PSF-support trade-off (0 disables)")
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--n-int", type=int, default=2880)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU sharding is a "
              f"design, not a measured path", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration > 0:
        # a plain device-to-device copy of known size: the reference for scaling
        # the HBM byte counters (FETCH_SIZE / WRITE_SIZE) of the other kernels
        import torch
        nb = int(args.copy_calibration)
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nb, "copies": 5}), flush=True)
        return

    import numpy as np
    import torch

    from paper_2406_09144_amd import api
    from paper_2406_09144_amd._lib import FR_LIK_EXACT, FR_LIK_FAST
    from synthetic import make_config
    from synthetic.configs import config_rng, noise_from_model
    from synthetic.skies import correlated_field, inv_power_half

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    n = args.n
    t0 = time.time()
    obs = make_config(1, n=n, n_int=args.n_int)
    log(f"[bench] workload: {obs.n_vis} visibilities, {n}x{n} sky, generated in {time.time() - t0:.1f}s")
    t0 = time.time()
    plan = api.Plan(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, eps=1e-5)
    torch.cuda.synchronize()
    t_plan = time.time() - t0
    info = plan.info
    log(f"[bench] plan {t_plan:.2f}s: W={info['support']} planes={info['n_planes']} work items={info['n_workitems']}")

    sky = torch.from_numpy(obs.sky).float().to(dev)
    model = api.degrid(plan, sky)
    noise, wt = noise_from_model(config_rng(1, "noise"), model.cpu().numpy().astype(np.complex128))
    V = (model + torch.from_numpy(noise).to(torch.complex64).to(dev)).contiguous()
    w = torch.from_numpy(wt).float().to(dev)
    t0 = time.time()
    psf = api.make_psf_kernel(plan, w, eps_noise=-1e-6)
    torch.cuda.synchronize()
    t_psf = time.time() - t0
    d = api.grid(plan, V, w)
    # 8 MGVI-style log-sky samples around the log of the true sky
    rng_s = config_rng(2, "samples")
    sbar = np.log(np.maximum(obs.sky[0], 1e-6 * obs.sky.max()))
    samples = np.stack([sbar + 0.1 * correlated_field(rng_s, n, n) for _ in range(8)])[:, None]
    s8 = torch.from_numpy(samples).float().to(dev).contiguous()
    s1 = s8[:1].contiguous()
    ip = torch.from_numpy(inv_power_half(n, n)).float().to(dev)
    KR = psf.kernels()[0]
    ip_cg = (ip * (float(KR.abs().max()) * 1e-3)).contiguous()
    x8 = torch.exp(s8).contiguous()
    x1 = x8[:1].contiguous()
    diag = torch.exp(s1[0]).contiguous()
    b = d.clone()
    out_vis = torch.empty_like(V)
    out_img = torch.empty_like(d)
    y8 = torch.empty_like(x8)
    y1 = torch.empty_like(x1)

    names = ["degrid", "grid", "rnr_approx_b8", "rnr_exact_b1", "lik_fast_b8", "lik_exact_b1", "cg50"]
    calls = {
        "degrid": lambda: api.degrid(plan, sky, out=out_vis),
        "grid": lambda: api.grid(plan, V, w, out=out_img),
        "rnr_approx_b8": lambda: api.apply_RNR_approx(psf, x8, out=y8),
        "rnr_exact_b1": lambda: api.apply_RNR_exact(plan, x1, w, out=y1),
        "lik_fast_b8": lambda: api.likelihood_grad(FR_LIK_FAST, s8, d, psf=psf, inv_power=ip),
        "lik_exact_b1": lambda: api.likelihood_grad(FR_LIK_EXACT, s1, V, plan=plan, weight=w, inv_power=ip),
        "cg50": lambda: api.cg_solve(b, psf=psf, inv_power=ip_cg, diag=diag, maxiter=50),
    }

    def step(ev=None):
        for k in names:
            if ev is not None:
                ev[k][0].record()
            calls[k]()
            if ev is not None:
                ev[k][1].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [{k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for k in names}
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
        log(f"[bench] step {i + 1}/{args.steps} enqueued")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    comp = {k: float(np.mean([e[k][0].elapsed_time(e[k][1]) for e in evs])) for k in names}
    ms_per_step = 1e3 * t_total / args.steps
    n_vis = obs.n_vis
    degrid_grid_ms = comp["degrid"] + comp["grid"]
    value = 2 * n_vis / (degrid_grid_ms * 1e-3)

    # per-kernel device time: the same steps again with every library launch
    # bracketed by hipEvents on its stream (the brackets add gaps between
    # launches, so the step timings above are taken without them)
    api.profile_reset()
    api.profile_enable(True)
    torch.cuda.synchronize()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    api.profile_enable(False)
    kern = {}
    for kname in api.PROFILED_KERNELS:
        cnt, tot = api.profile_query(kname)
        if cnt:
            kern[kname] = {"launches": cnt, "avg_ms": tot / cnt, "total_ms": tot}
    roof = None
    if "grid" in kern:
        fl = grid_flops(info, n_vis)
        ach = fl / (kern["grid"]["avg_ms"] * 1e-3) / 1e12
        roof = {"kernel": "grid", "bound": "mfma", "achieved": round(ach, 3), "peak": FP32_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / FP32_MFMA_PEAK_TFLOPS, 5),
                "traffic": measured_traffic("grid"), "flops_per_launch": fl,
                "avg_launch_ms": round(kern["grid"]["avg_ms"], 5)}
    roof_hbm = []
    for kname in ("degrid", "grid_assemble", "wplane_rows_fwd", "wplane_cols_fwd", "wplane_cols_inv",
                  "wplane_rows_inv"):
        if kname in kern:
            byts = algorithmic_bytes(kname, info, n_vis, obs.n_row, 1, n, n)
            ach = byts / (kern[kname]["avg_ms"] * 1e-3) / 1e9
            roof_hbm.append({"kernel": kname, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_launch": int(byts),
                             "avg_launch_ms": round(kern[kname]["avg_ms"], 5)})
    # whole calls on the method's bytes (every w-plane written once by its FFT and
    # read once, image, visibilities, weights, uvw)
    roof_hbm.append(hbm_entry("degrid_call", call_bytes("degrid", info, n_vis, obs.n_row, n, n), comp["degrid"]))
    roof_hbm.append(hbm_entry("grid_call", call_bytes("grid", info, n_vis, obs.n_row, n, n), comp["grid"]))
    # the degridding kernel against the LDS: every thread slot (a visibility, or a
    # pair of visibilities of one base cell when the plan pairs them) reads its
    # W^2 Ww complex footprint values from the LDS tile, and every item writes its
    # planes' tiles (halo included) once
    lds = None
    if "degrid" in kern:
        W, Ww = info["support"], info["w_support"]
        ts = info["tile"] + W - 1
        lds_bytes = info["degrid_slots"] * W * W * Ww * 8 + info["n_workitems"] * Ww * ts * ts * 8
        ach = lds_bytes / (kern["degrid"]["avg_ms"] * 1e-3) / 1e9
        lds = {"kernel": "degrid", "bound": "lds", "achieved": round(ach, 1), "peak": round(LDS_PEAK_GBS, 1),
               "unit": "GB/s", "frac": round(ach / LDS_PEAK_GBS, 4), "bytes_per_launch": int(lds_bytes),
               "avg_launch_ms": round(kern["degrid"]["avg_ms"], 5)}
    log("[bench] per-kernel: " + json.dumps({k: round(v["avg_ms"], 4) for k, v in kern.items()}))

    # sustained PSF-convolution applies (batch 8, back to back), then the same
    # loop with per-launch event brackets for the kernel times
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(PSF_APPLY_REPS):
        api.apply_RNR_approx(psf, x8, out=y8)
    e1.record()
    torch.cuda.synchronize()
    psf_ms = e0.elapsed_time(e1) / PSF_APPLY_REPS
    roof_hbm.append(hbm_entry("psf_apply_call_b8", psf_apply_bytes(n, 8), psf_ms))
    api.profile_reset()
    api.profile_enable(True)
    for _ in range(PSF_APPLY_REPS):
        api.apply_RNR_approx(psf, x8, out=y8)
    torch.cuda.synchronize()
    api.profile_enable(False)
    for kname in ("psfconv_rows_r2c", "psfconv_cols", "psfconv_rows_c2r"):
        cnt, tot = api.profile_query(kname)
        if cnt:
            byts = algorithmic_bytes(kname, info, n_vis, obs.n_row, 8, n, n)
            ach = byts / (tot / cnt * 1e-3) / 1e9
            roof_hbm.append({"kernel": kname + "_b8", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_launch": int(byts),
                             "avg_launch_ms": round(tot / cnt, 5)})

    # plain FP64 form of the same (de)gridding at eps = 1e-5
    fp64 = None
    if args.fp64_steps > 0:
        plan64 = api.Plan(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, eps=1e-5, fp64=True)
        sky64, V64, w64 = sky.double(), V.to(torch.complex128), w.double()
        api.degrid(plan64, sky64)
        api.grid(plan64, V64, w64)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.fp64_steps):
            api.degrid(plan64, sky64)
            api.grid(plan64, V64, w64)
        e1.record()
        torch.cuda.synchronize()
        ms64 = e0.elapsed_time(e1) / args.fp64_steps
        fp64 = {"degrid_grid_ms": round(ms64, 4), "vis_per_s": 2 * n_vis / (ms64 * 1e-3),
                "support": plan64.info["support"], "n_planes": plan64.info["n_planes"]}
        del plan64

    scale = scale32 = None
    if args.scale_steps > 0:
        scale = scale_workload(api, torch, args.scale_steps)
        log(f"[bench] MeerKAT-like: {json.dumps(scale)}")
        if args.scale_wplanes > 0:
            scale32 = scale_workload(api, torch, args.scale_steps, n_wplanes=args.scale_wplanes)
            log(f"[bench] MeerKAT-like, {args.scale_wplanes} planes: {json.dumps(scale32)}")
    psf4096 = None
    if args.psf4096:
        psf4096 = psf_apply_4096(api, torch)
        log(f"[bench] PSF apply 4096^2: {json.dumps(psf4096)}")

    reduced = None
    if args.reduced_psf:
        s0 = torch.full((1, n, n), float(np.log(max(float(obs.sky.mean()), 1e-12))), device=dev)
        reduced = reduced_psf_tradeoff(api, torch, plan, w, V, x8, ip, s0)
        log(f"[bench] reduced PSF: {json.dumps(reduced)}")

    taylor = taylor_timing(api, torch, obs, sky, V, w, n)
    log(f"[bench] Taylor in w: {json.dumps(taylor)}")
    mgvi = mgvi_timing(api, torch, plan, w, n)
    log(f"[bench] MGVI: {json.dumps(mgvi)}")

    served = None
    if args.serve_seconds > 0:
        rates = [float(r) for r in args.serve_sweep.split(",") if r.strip()]
        served = served_workload(api, torch, args.serve_seconds, args.serve_rate, args.serve_jobs,
                                 args.serve_fp64_requests, sweep_rates=rates,
                                 sweep_requests=args.serve_sweep_requests)

    cpu = None
    if args.cpu_sample > 0:
        import oracle as O
        O.build(force=False)
        rng = np.random.default_rng(7)
        rows = np.sort(rng.choice(obs.n_row, args.cpu_sample, replace=False))
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        O.degrid_rows(obs.uvw, obs.freq, n, n, obs.dx, obs.dy, obs.sky, rows, np.zeros_like(rows))
        tc = time.perf_counter() - t0
        cpu = {"value": args.cpu_sample / tc, "unit": "vis/s", "cores": cores, "kind": "oracle",
               "sample": f"direct-DFT R of {args.cpu_sample} of the {n_vis} visibilities on the {n}x{n} sky "
                         f"({tc:.1f} s, FP64, OpenMP)"}

    out = {
        "metric": METRIC, "value": value, "unit": "vis/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"VLA-like single channel, {n}x{n} sky, {n_vis} visibilities with w "
                               f"(improved w-stacking), eps=1e-5; PSF rows batch 8",
                   "n_vis": n_vis, "image": [n, n], "eps": 1e-5, "support": info["support"],
                   "n_planes": info["n_planes"], "psf_batch": 8, "cg_iters": 50},
        "components": {
            "degrid_ms": comp["degrid"], "grid_ms": comp["grid"],
            "degrid_vis_per_s": n_vis / (comp["degrid"] * 1e-3), "grid_vis_per_s": n_vis / (comp["grid"] * 1e-3),
            "psf_applies_per_s": 8 / (psf_ms * 1e-3), "psf_apply_b8_sustained_ms": psf_ms,
            "rnr_approx_b8_ms": comp["rnr_approx_b8"], "rnr_exact_b1_ms": comp["rnr_exact_b1"],
            "lik_fast_b8_ms": comp["lik_fast_b8"], "lik_exact_b1_ms": comp["lik_exact_b1"],
            "cg50_ms": comp["cg50"], "plan_create_s": t_plan, "make_psf_s": t_psf,
            "fp64_plain_form": fp64,
            "meerkat_like": scale,
            "meerkat_like_stated_wplanes": scale32,
            "psf_apply_4096": psf4096,
            "reduced_psf": reduced,
            "mgvi": mgvi,
            "taylor_w": taylor,
            "served": served,
        },
        "kernels_ms": {k: round(v["avg_ms"], 5) for k, v in kern.items()},
        "roofline": roof,
        "roofline_hbm": roof_hbm,
        "roofline_lds": lds,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
