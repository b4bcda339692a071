"""Degridding R and gridding R^+ (ES kernel + improved w-stacking) against the
FP64 direct-DFT oracle, element by element, and adjointness of the GPU pair.

Tolerances (relative L2 over all elements): 1e-5 for FP32 plans at eps = 1e-5,
1e-10 for FP64 plans at eps = 1e-11.  The pair is an exact transpose whatever
eps is, so <R x, y> = <x, R^+ y> holds to rounding (FP32 ~1e-6, FP64 ~1e-13).
"""

import numpy as np
import pytest

import oracle as O
from synthetic import make_config

pytestmark = pytest.mark.gpu

LAM_1GHZ = O.C_LIGHT_M_S / 1.0e9


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def wide_field(seed=3, n=64, nvis=3000, dx=0.008, wfac=2.0):
    """Random uv inside and beyond the pixel Nyquist band, large w, wide field."""
    rng = np.random.default_rng(seed)
    uvmax = 0.7 / dx  # beyond |u| dx = 1/2: exercises the wrap
    uvw = np.empty((nvis, 3))
    uvw[:, 0] = rng.uniform(-uvmax, uvmax, nvis) * LAM_1GHZ
    uvw[:, 1] = rng.uniform(-uvmax, uvmax, nvis) * LAM_1GHZ
    uvw[:, 2] = rng.uniform(-1, 1, nvis) * wfac * uvmax * LAM_1GHZ
    return dict(uvw=uvw, freq=np.array([1.0e9]), nx=n, ny=n, dx=dx, dy=dx * 1.1)


def offset_w_field(seed=4, n=64, nvis=3000, dx=0.008, w0=5000.0, span=300.0):
    """Every |w| far from zero: w uniform in +-[w0, w0 + span] wavelengths on a wide
    field, so the plane phases w_p ((n - 1) - yc) reach about 85 cycles and their
    rounding must happen after the reduction modulo one cycle."""
    rng = np.random.default_rng(seed)
    uvmax = 0.45 / dx
    uvw = np.empty((nvis, 3))
    uvw[:, 0] = rng.uniform(-uvmax, uvmax, nvis) * LAM_1GHZ
    uvw[:, 1] = rng.uniform(-uvmax, uvmax, nvis) * LAM_1GHZ
    sign = np.where(rng.uniform(size=nvis) < 0.5, -1.0, 1.0)
    uvw[:, 2] = sign * rng.uniform(w0, w0 + span, nvis) * LAM_1GHZ
    return dict(uvw=uvw, freq=np.array([1.0e9]), nx=n, ny=n, dx=dx, dy=dx)


def case(name):
    if name == "cfg0_coplanar":
        o = make_config(0, n=64, n_int=16, with_sky=False)
    elif name == "cfg1_wstack":
        o = make_config(1, n=64, n_int=20, with_sky=False)
    elif name == "cfg3_multichan":
        o = make_config(3, n=64, n_int=3, n_chan=3, with_sky=False)
    elif name == "wide_w":
        return wide_field()
    elif name == "offset_w":
        return offset_w_field()
    elif name == "rect":
        o = make_config(1, n=32, n_int=12, with_sky=False)
        return dict(uvw=o.uvw, freq=o.freq, nx=32, ny=64, dx=o.dx * 2, dy=o.dy)
    return dict(uvw=o.uvw, freq=o.freq, nx=o.nx, ny=o.ny, dx=o.dx, dy=o.dy)


CASES = ["cfg0_coplanar", "cfg1_wstack", "cfg3_multichan", "wide_w", "offset_w", "rect"]


def _plan(c, fp64, eps=None, divide_by_n=True):
    from paper_2406_09144_amd import api
    eps = eps or (1e-11 if fp64 else 1e-5)
    return api.Plan(c["uvw"], c["freq"], c["nx"], c["ny"], c["dx"], c["dy"], eps=eps, fp64=fp64,
                    divide_by_n=divide_by_n)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("fp64", [False, True])
def test_degrid_vs_oracle(name, fp64):
    import torch
    from paper_2406_09144_amd import api
    c = case(name)
    pl = _plan(c, fp64)
    rng = np.random.default_rng(11)
    nchan = len(c["freq"])
    img = rng.standard_normal((nchan, c["nx"], c["ny"]))
    rd = torch.float64 if fp64 else torch.float32
    vis = api.degrid(pl, torch.from_numpy(img).to(rd).cuda()).cpu().numpy()
    ref = O.degrid(c["uvw"], c["freq"], c["nx"], c["ny"], c["dx"], c["dy"], img)
    err = rel(vis, ref)
    print(name, fp64, pl.info["support"], pl.info["n_planes"], err)
    assert err < (1e-10 if fp64 else 1e-5), (err, pl.info)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("fp64", [False, True])
def test_grid_vs_oracle(name, fp64):
    import torch
    from paper_2406_09144_amd import api
    c = case(name)
    pl = _plan(c, fp64)
    rng = np.random.default_rng(12)
    nrow, nchan = c["uvw"].shape[0], len(c["freq"])
    vis = rng.standard_normal((nrow, nchan)) + 1j * rng.standard_normal((nrow, nchan))
    wt = rng.uniform(0.2, 3.0, (nrow, nchan))
    cd, rd = (torch.complex128, torch.float64) if fp64 else (torch.complex64, torch.float32)
    img = api.grid(pl, torch.from_numpy(vis).to(cd).cuda(), torch.from_numpy(wt).to(rd).cuda()).cpu().numpy()
    ref = O.grid(c["uvw"], c["freq"], c["nx"], c["ny"], c["dx"], c["dy"], vis, wt)
    err = rel(img, ref)
    print(name, fp64, pl.info["support"], pl.info["n_planes"], err)
    assert err < (1e-10 if fp64 else 1e-5), (err, pl.info)


@pytest.mark.parametrize("name", ["cfg1_wstack", "wide_w"])
@pytest.mark.parametrize("fp64", [False, True])
def test_gpu_pair_is_adjoint(name, fp64):
    import torch
    from paper_2406_09144_amd import api
    c = case(name)
    pl = _plan(c, fp64, eps=1e-3)  # exact transpose at any accuracy
    rng = np.random.default_rng(13)
    nrow, nchan = c["uvw"].shape[0], len(c["freq"])
    x = rng.standard_normal((nchan, c["nx"], c["ny"]))
    y = rng.standard_normal((nrow, nchan)) + 1j * rng.standard_normal((nrow, nchan))
    cd, rd = (torch.complex128, torch.float64) if fp64 else (torch.complex64, torch.float32)
    Rx = api.degrid(pl, torch.from_numpy(x).to(rd).cuda()).cpu().numpy().astype(np.complex128)
    Ry = api.grid(pl, torch.from_numpy(y).to(cd).cuda()).cpu().numpy().astype(np.float64)
    lhs = np.real(np.vdot(Rx, y))
    rhs = float(np.sum(x * Ry))
    scale = np.linalg.norm(Rx) * np.linalg.norm(y)
    assert abs(lhs - rhs) < (1e-13 if fp64 else 2e-6) * scale, (lhs, rhs)


@pytest.mark.parametrize("eps", [1e-3, 1e-4, 1e-6])
def test_accuracy_tracks_epsilon(eps):
    import torch
    from paper_2406_09144_amd import api
    c = case("cfg1_wstack")
    fp64 = eps < 1e-5
    pl = _plan(c, fp64, eps=eps)
    rng = np.random.default_rng(14)
    img = rng.standard_normal((1, c["nx"], c["ny"]))
    rd = torch.float64 if fp64 else torch.float32
    vis = api.degrid(pl, torch.from_numpy(img).to(rd).cuda()).cpu().numpy()
    ref = O.degrid(c["uvw"], c["freq"], c["nx"], c["ny"], c["dx"], c["dy"], img)
    assert rel(vis, ref) < eps


def test_divide_by_n_off_and_coplanar_flag():
    import torch
    from paper_2406_09144_amd import api
    c = case("wide_w")
    rng = np.random.default_rng(15)
    img = rng.standard_normal((1, c["nx"], c["ny"]))
    pl = api.Plan(c["uvw"], c["freq"], c["nx"], c["ny"], c["dx"], c["dy"], eps=1e-11, fp64=True,
                  divide_by_n=False, coplanar=True)
    assert pl.info["coplanar"] == 1 and pl.info["n_planes"] == 1
    vis = api.degrid(pl, torch.from_numpy(img).cuda()).cpu().numpy()
    uvw0 = c["uvw"].copy()
    uvw0[:, 2] = 0
    ref = O.degrid(uvw0, c["freq"], c["nx"], c["ny"], c["dx"], c["dy"], img, divide_by_n=False)
    assert rel(vis, ref) < 1e-10


def test_empty_plan():
    import torch
    from paper_2406_09144_amd import api
    pl = api.Plan(np.zeros((0, 3)), np.array([1e9]), 16, 16, 1e-3, 1e-3)
    img = api.grid(pl, torch.zeros((0, 1), dtype=torch.complex64, device="cuda"))
    assert float(img.abs().max()) == 0.0
    vis = api.degrid(pl, torch.ones((1, 16, 16), device="cuda"))
    assert vis.shape == (0, 1)


def test_plan_rejects_bad_arguments():
    from paper_2406_09144_amd import api, FrError
    uvw = np.zeros((4, 3))
    for kw in [dict(nx=24), dict(eps=1e-8), dict(dx=-1.0), dict(dx=0.2)]:
        args = dict(uvw=uvw, freq=np.array([1e9]), nx=16, ny=16, dx=1e-3, dy=1e-3, eps=1e-5)
        args.update(kw)
        with pytest.raises(FrError):
            api.Plan(**args)


@pytest.mark.parametrize("fp64", [False, True])
def test_grid_is_bitwise_reproducible_and_scale_exact(fp64):
    """Gridding sums in 64-bit fixed point, in an order fixed by the stable sort:
    the same input gives the same bits (same plan, and a plan rebuilt from the same
    uvw), and scaling the visibilities by 2^k scales the image by exactly 2^k (the
    fixed-point exponent follows the bound)."""
    import torch
    from paper_2406_09144_amd import api
    c = case("cfg1_wstack")
    rng = np.random.default_rng(21)
    nrow = c["uvw"].shape[0]
    vis = rng.standard_normal((nrow, 1)) + 1j * rng.standard_normal((nrow, 1))
    wt = rng.uniform(0.2, 3.0, (nrow, 1))
    cd, rd = (torch.complex128, torch.float64) if fp64 else (torch.complex64, torch.float32)
    V = torch.from_numpy(vis).to(cd).cuda()
    w = torch.from_numpy(wt).to(rd).cuda()
    pl = _plan(c, fp64)
    a = api.grid(pl, V, w).cpu()
    b = api.grid(pl, V, w).cpu()
    c2 = api.grid(_plan(c, fp64), V, w).cpu()
    assert torch.equal(a, b) and torch.equal(a, c2)
    for k in (-40, 40):
        s = api.grid(pl, V * 2.0 ** k, w).cpu() * 2.0 ** -k
        assert torch.equal(s, a), k


def test_grid_wide_dynamic_range_vs_oracle():
    """Visibility amplitudes over eight decades and weights over four: the error
    stays within the FP32 bound relative to the image norm (the fixed-point
    resolution is set by the largest contribution)."""
    import torch
    from paper_2406_09144_amd import api
    c = case("wide_w")
    rng = np.random.default_rng(22)
    nrow = c["uvw"].shape[0]
    amp = 10.0 ** rng.uniform(-4, 4, (nrow, 1))
    vis = amp * (rng.standard_normal((nrow, 1)) + 1j * rng.standard_normal((nrow, 1)))
    wt = 10.0 ** rng.uniform(-2, 2, (nrow, 1))
    pl = _plan(c, False)
    img = api.grid(pl, torch.from_numpy(vis).to(torch.complex64).cuda(),
                   torch.from_numpy(wt).float().cuda()).cpu().numpy()
    ref = O.grid(c["uvw"], c["freq"], c["nx"], c["ny"], c["dx"], c["dy"], vis, wt)
    assert rel(img, ref) < 1e-5


@pytest.mark.parametrize("name", ["cfg1_wstack", "cfg3_multichan", "rect"])
@pytest.mark.parametrize("fp64", [False, True])
def test_taylor_w_vs_oracle(name, fp64):
    """FR_W_TAYLOR: the w-term as a Taylor series (terms = 2-D planes times
    (-i t/h)^j, weights (2 pi w h)^j / j!) meets the same tolerance against the
    direct sums, with fewer planes than w-stacking on the VLA-like layout."""
    import torch
    from paper_2406_09144_amd import api
    c = case(name)
    eps = 1e-11 if fp64 else 1e-5
    pl = api.Plan(c["uvw"], c["freq"], c["nx"], c["ny"], c["dx"], c["dy"], eps=eps, fp64=fp64, w_taylor=True)
    ws = api.Plan(c["uvw"], c["freq"], c["nx"], c["ny"], c["dx"], c["dy"], eps=eps, fp64=fp64)
    info = pl.info
    print(name, fp64, "taylor", info["w_taylor"], info["n_planes"], "w-stacking planes", ws.info["n_planes"])
    if name == "cfg1_wstack":
        assert info["w_taylor"] == 1 and info["n_planes"] < ws.info["n_planes"]
    rng = np.random.default_rng(13)
    nrow, nchan = c["uvw"].shape[0], len(c["freq"])
    img = rng.standard_normal((nchan, c["nx"], c["ny"]))
    cd, rd = (torch.complex128, torch.float64) if fp64 else (torch.complex64, torch.float32)
    vis = api.degrid(pl, torch.from_numpy(img).to(rd).cuda()).cpu().numpy()
    ref = O.degrid(c["uvw"], c["freq"], c["nx"], c["ny"], c["dx"], c["dy"], img)
    tol = 1e-10 if fp64 else 1e-5
    assert rel(vis, ref) < tol, (rel(vis, ref), info)
    y = rng.standard_normal((nrow, nchan)) + 1j * rng.standard_normal((nrow, nchan))
    wt = rng.uniform(0.2, 3.0, (nrow, nchan))
    im = api.grid(pl, torch.from_numpy(y).to(cd).cuda(), torch.from_numpy(wt).to(rd).cuda()).cpu().numpy()
    ref = O.grid(c["uvw"], c["freq"], c["nx"], c["ny"], c["dx"], c["dy"], y, wt)
    assert rel(im, ref) < tol, (rel(im, ref), info)
    # the GPU pair stays an exact transpose
    x = rng.standard_normal((nchan, c["nx"], c["ny"]))
    Rx = api.degrid(pl, torch.from_numpy(x).to(rd).cuda()).cpu().numpy().astype(np.complex128)
    Ry = api.grid(pl, torch.from_numpy(y).to(cd).cuda()).cpu().numpy().astype(np.float64)
    lhs = np.real(np.vdot(Rx, y))
    rhs = float(np.sum(x * Ry))
    scale = np.linalg.norm(Rx) * np.linalg.norm(y)
    assert abs(lhs - rhs) < (1e-13 if fp64 else 2e-6) * scale, (lhs, rhs)


def test_taylor_w_falls_back_to_w_stacking_for_large_w():
    from paper_2406_09144_amd import api
    c = case("wide_w")
    pl = api.Plan(c["uvw"], c["freq"], c["nx"], c["ny"], c["dx"], c["dy"], eps=1e-5, w_taylor=True)
    assert pl.info["w_taylor"] == 0
    assert pl.info["n_planes"] == api.Plan(c["uvw"], c["freq"], c["nx"], c["ny"], c["dx"], c["dy"],
                                           eps=1e-5).info["n_planes"]


def dense_tracks(n=64, n_bl=12):
    """VLA-like tracks sampled every 10 s on a few baselines: consecutive records of
    a baseline stay in one uv cell, so the sorted records come in long runs."""
    o = make_config(1, n=n, n_int=2880, with_sky=False)
    nbl = 27 * 26 // 2  # rows are time-major over the 351 baselines
    assert o.uvw.shape[0] % nbl == 0
    sel = (np.arange(o.uvw.shape[0]) % nbl) < n_bl
    return dict(uvw=o.uvw[sel], freq=o.freq, nx=n, ny=n, dx=o.dx, dy=o.dy)


@pytest.mark.parametrize("kind", ["dense_tracks", "random_uv"])
def test_both_spread_kernels_vs_oracle(kind):
    """Long runs take the matrix-core spread and the paired degridding, single-record
    runs the vector spread and one record per thread (the plan reports which); all
    meet the FP32 bound against the oracle."""
    import torch
    from paper_2406_09144_amd import api
    c = dense_tracks() if kind == "dense_tracks" else wide_field()
    pl = _plan(c, False)
    info = pl.info
    long_runs = kind == "dense_tracks"
    assert (info["records_per_run"] >= 4.0) == long_runs, info
    assert info["matrix_spread"] == (1 if long_runs else 0), info
    assert _plan(c, True).info["matrix_spread"] == 0  # FP64 always on the vector units
    rng = np.random.default_rng(21)
    nrow = c["uvw"].shape[0]
    vis = rng.standard_normal((nrow, 1)) + 1j * rng.standard_normal((nrow, 1))
    wt = rng.uniform(0.2, 3.0, (nrow, 1))
    img = api.grid(pl, torch.from_numpy(vis).to(torch.complex64).cuda(),
                   torch.from_numpy(wt).to(torch.float32).cuda()).cpu().numpy()
    ref = O.grid(c["uvw"], c["freq"], c["nx"], c["ny"], c["dx"], c["dy"], vis, wt)
    err = rel(img, ref)
    print(kind, info["records_per_run"], info["matrix_spread"], err)
    assert err < 1e-5, (err, info)
    # degridding on the same layouts: long runs two records of a base cell per thread
    assert info["paired_degrid"] == (1 if long_runs else 0), info
    sky = rng.standard_normal((1, c["nx"], c["ny"]))
    got = api.degrid(pl, torch.from_numpy(sky).to(torch.float32).cuda()).cpu().numpy()
    dref = O.degrid(c["uvw"], c["freq"], c["nx"], c["ny"], c["dx"], c["dy"], sky)
    derr = rel(got, dref)
    print(kind, "degrid", derr)
    assert derr < 1e-5, (derr, info)


def test_vector_spread_flag_same_plan_both_kernels():
    """FR_VECTOR_SPREAD makes a plan whose runs would take the matrix cores grid on
    the vector units: the two kernels on the same layout agree with each other and
    with the oracle to the FP32 bound, and each is bitwise reproducible."""
    import torch
    from paper_2406_09144_amd import api
    c = dense_tracks()
    args = (c["uvw"], c["freq"], c["nx"], c["ny"], c["dx"], c["dy"])
    pm = api.Plan(*args, eps=1e-5)
    pv = api.Plan(*args, eps=1e-5, vector_spread=True)
    assert pm.info["matrix_spread"] == 1 and pv.info["matrix_spread"] == 0
    assert pm.info["n_planes"] == pv.info["n_planes"]
    rng = np.random.default_rng(22)
    nrow = c["uvw"].shape[0]
    vis = rng.standard_normal((nrow, 1)) + 1j * rng.standard_normal((nrow, 1))
    wt = rng.uniform(0.2, 3.0, (nrow, 1))
    vd = torch.from_numpy(vis).to(torch.complex64).cuda()
    wd = torch.from_numpy(wt).to(torch.float32).cuda()
    im = api.grid(pm, vd, wd)
    iv = api.grid(pv, vd, wd)
    assert torch.equal(im, api.grid(pm, vd, wd)) and torch.equal(iv, api.grid(pv, vd, wd))
    ref = O.grid(*args, vis, wt)
    em, ev = rel(im.cpu().numpy(), ref), rel(iv.cpu().numpy(), ref)
    ed = rel(im.cpu().numpy(), iv.cpu().numpy().astype(np.float64))
    print("matrix", em, "vector", ev, "between", ed)
    assert em < 1e-5 and ev < 1e-5 and ed < 1e-5
