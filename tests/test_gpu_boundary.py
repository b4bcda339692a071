"""The C-ABI boundary on the GPU:

  * fr_degrid_weighted is N^-1 R: the weights applied by the library equal the
    weights applied afterwards, bit for bit;
  * fr_query_footprint bounds the scratch every operation really takes from its
    stream's arena (the arena's high-water mark, read through fr_scratch_stats),
    at batch 1 and batch 8, and fr_scratch_trim returns the arena;
  * an injected device-allocation failure makes plan creation, an operator call
    and the PSF-kernel build return FR_ENOMEM, releases what the call had taken,
    and leaves the library usable (the next call gives the right result)."""

import numpy as np
import pytest

from synthetic import make_config
from synthetic.skies import inv_power_half

pytestmark = pytest.mark.gpu


def setup(fp64=False, n=64, n_int=20, cfg=1, n_chan=None):
    import torch
    from paper_2406_09144_amd import api
    kw = {} if n_chan is None else {"n_chan": n_chan}
    o = make_config(cfg, n=n, n_int=n_int, with_sky=False, **kw)
    rd = torch.float64 if fp64 else torch.float32
    cd = torch.complex128 if fp64 else torch.complex64
    pl = api.Plan(o.uvw, o.freq, n, n, o.dx, o.dy, eps=1e-10 if fp64 else 1e-5, fp64=fp64)
    rng = np.random.default_rng(7)
    wt = torch.from_numpy(rng.uniform(0.5, 2.0, (o.n_row, len(o.freq)))).to(rd).cuda()
    img = torch.from_numpy(rng.standard_normal((len(o.freq), n, n))).to(rd).cuda()
    vis = torch.from_numpy(rng.standard_normal((o.n_row, len(o.freq))) +
                           1j * rng.standard_normal((o.n_row, len(o.freq)))).to(cd).cuda()
    return o, pl, wt, img, vis


@pytest.mark.parametrize("fp64", [False, True])
def test_weighted_degrid_is_weights_times_degrid(fp64):
    from paper_2406_09144_amd import api
    import torch
    o, pl, wt, img, vis = setup(fp64, cfg=3, n_chan=2, n_int=3)
    a = api.degrid(pl, img, weight=wt)
    b = api.degrid(pl, img) * wt
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def _ops(api, pl, psf, wt, img, vis, B, ip):
    from paper_2406_09144_amd import _lib as L
    import torch
    x = img.expand(B, *img.shape).contiguous()
    s = (0.1 * x).contiguous()
    d = api.grid(pl, vis, wt)
    torch.cuda.synchronize()
    return [
        (L.FR_OP_DEGRID, dict(plan=pl), lambda st: api.degrid(pl, img, stream=st)),
        (L.FR_OP_GRID, dict(plan=pl), lambda st: api.grid(pl, vis, wt, stream=st)),
        (L.FR_OP_RNR_APPROX, dict(psf=psf), lambda st: api.apply_RNR_approx(psf, x, stream=st)),
        (L.FR_OP_RNR_EXACT, dict(plan=pl), lambda st: api.apply_RNR_exact(pl, x, wt, stream=st)),
        (L.FR_OP_LIK_FAST, dict(psf=psf),
         lambda st: api.likelihood_grad(L.FR_LIK_FAST, s, d, psf=psf, inv_power=ip, stream=st)),
        (L.FR_OP_LIK_EXACT, dict(plan=pl),
         lambda st: api.likelihood_grad(L.FR_LIK_EXACT, s, vis, plan=pl, weight=wt, inv_power=ip, stream=st)),
        (L.FR_OP_CG, dict(psf=psf), lambda st: api.cg_solve(d, psf=psf, inv_power=ip, diag=img, maxiter=3,
                                                             stream=st)),
        (L.FR_OP_CG, dict(plan=pl), lambda st: api.cg_solve(d, plan=pl, weight=wt, inv_power=ip, diag=img,
                                                             maxiter=2, stream=st)),
        (L.FR_OP_MAKE_PSF, dict(plan=pl), lambda st: api.make_psf_kernel(pl, wt, eps_noise=-1e-4, stream=st)),
    ]


@pytest.mark.parametrize("B", [1, 8])
@pytest.mark.parametrize("fp64", [False, True])
def test_footprint_bounds_the_scratch_each_op_takes(B, fp64):
    import torch
    from paper_2406_09144_amd import api
    o, pl, wt, img, vis = setup(fp64, n=64, n_int=20)
    psf = api.make_psf_kernel(pl, wt, eps_noise=-1e-4)
    rd = torch.float64 if fp64 else torch.float32
    ip = torch.from_numpy(inv_power_half(64, 64)).to(rd).cuda()
    for op, obj, call in _ops(api, pl, psf, wt, img, vis, B, ip):
        print(f"footprint: op {op} {list(obj)} B={B} fp64={fp64}", flush=True)
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        api.scratch_stats(st, reset=True)
        with torch.cuda.stream(st):
            call(st)
        st.synchronize()
        peak, held = api.scratch_stats(st)
        fp, _ = api.query_footprint(op, B, **obj)
        assert peak <= fp, (op, peak, fp)
        assert peak > 0 and held >= peak
        if op != 7:  # the PSF build's bound counts its sub-plan and a worst-case item count
            assert fp <= 2 * peak + 8192, (op, peak, fp)
        api.scratch_trim(st)
        assert api.scratch_stats(st)[1] == 0


def test_injected_allocation_failures_return_enomem_and_release():
    import torch
    from paper_2406_09144_amd import api
    from paper_2406_09144_amd._lib import FR_ENOMEM, FrError
    # 300k visibilities: a leaked plan or sub-plan would hold tens of MB
    o, pl, wt, img, vis = setup(False, n=128, n_int=855)
    ref = api.grid(pl, vis, wt)
    torch.cuda.synchronize()

    def free():
        torch.cuda.synchronize()
        return torch.cuda.mem_get_info()[0]

    # plan creation: fail at the 1st, 4th and 9th device allocation
    for after in (0, 3, 8):
        f0 = free()
        api.inject_alloc_failure(after)
        with pytest.raises(FrError) as e:
            api.Plan(o.uvw, o.freq, 128, 128, o.dx, o.dy, eps=1e-5)
        assert e.value.status == FR_ENOMEM
        assert abs(free() - f0) <= 2 << 20, f"plan build after {after} allocations leaked"
    # an operator call on a fresh stream: the arena's first chunk fails
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    out = torch.empty_like(ref)
    api.inject_alloc_failure(0)
    with pytest.raises(FrError) as e:
        api.grid(pl, vis, wt, out=out, stream=st)
    assert e.value.status == FR_ENOMEM
    assert api.scratch_stats(st)[1] == 0
    with torch.cuda.stream(st):
        api.grid(pl, vis, wt, out=out, stream=st)
    st.synchronize()
    assert torch.equal(out, ref)
    # the PSF build (arena warmed by one good build; its sub-plan fails part-way)
    good = api.make_psf_kernel(pl, wt, eps_noise=-1e-4)
    KR0, KN0 = good.kernels()
    del good
    for after in (2, 6):
        f0 = free()
        api.inject_alloc_failure(after)
        with pytest.raises(FrError) as e:
            api.make_psf_kernel(pl, wt, eps_noise=-1e-4)
        assert e.value.status == FR_ENOMEM
        assert abs(free() - f0) <= 2 << 20, f"PSF build after {after} allocations leaked"
    api.inject_alloc_failure(-1)
    again = api.make_psf_kernel(pl, wt, eps_noise=-1e-4)
    KR1, KN1 = again.kernels()
    torch.cuda.synchronize()
    assert torch.equal(KR0, KR1) and torch.equal(KN0, KN1)
