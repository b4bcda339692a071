"""Plan bucketing (hot-path step a1) read back through fr_plan_export_order and
compared bit for bit with numpy:

  * the record order is numpy's stable argsort of the exported keys;
  * the first record of every bucket (from the plan's own work items, which the
    export checks tile each bucket exactly) is numpy's searchsorted of the sorted
    buckets;
  * the keys themselves agree with the coordinate formula evaluated in numpy
    (u = uvw nu / c, wrapped onto the 2n grid, base cell ceil(k - W/2), first
    w-plane ceil((w - w0)/dw - Ww/2)), apart from keys whose coordinate sits on a
    cell boundary to within rounding.

Layouts: coplanar, w-stacked, three channels, random wide-field uv beyond the
Nyquist band, a 300k-visibility plan (many sort tiles, ragged last tile), a plan
with 32 w-planes, and an empty plan."""

import numpy as np
import pytest

import oracle as O
from synthetic import make_config

pytestmark = pytest.mark.gpu


def layout(name):
    if name == "cfg0_coplanar":
        o = make_config(0, n=64, n_int=16, with_sky=False)
    elif name == "cfg1_wstack":
        o = make_config(1, n=64, n_int=20, with_sky=False)
    elif name == "cfg3_multichan":
        o = make_config(3, n=64, n_int=3, n_chan=3, with_sky=False)
    elif name == "wide_random":
        rng = np.random.default_rng(4)
        n, dx, m = 64, 0.008, 5000
        lam = O.C_LIGHT_M_S / 1e9
        uvw = np.stack([rng.uniform(-0.7 / dx, 0.7 / dx, m) * lam, rng.uniform(-0.7 / dx, 0.7 / dx, m) * lam,
                        rng.uniform(-1, 1, m) * 1.4 / dx * lam], axis=1)
        return dict(uvw=uvw, freq=np.array([1e9]), nx=n, ny=n, dx=dx, dy=dx * 1.1, n_wplanes=0)
    elif name == "cfg1_300k":
        o = make_config(1, n=256, n_int=855, with_sky=False)
    elif name == "cfg1_32planes":
        o = make_config(1, n=64, n_int=20, with_sky=False)
        return dict(uvw=o.uvw, freq=o.freq, nx=64, ny=64, dx=o.dx, dy=o.dy, n_wplanes=32)
    elif name == "empty":
        return dict(uvw=np.zeros((0, 3)), freq=np.array([1.4e9]), nx=32, ny=32, dx=1e-5, dy=1e-5, n_wplanes=0)
    return dict(uvw=o.uvw, freq=o.freq, nx=o.nx, ny=o.ny, dx=o.dx, dy=o.dy, n_wplanes=0)


def numpy_keys(c, info):
    """Sort keys from the coordinate formula, and the distance of each visibility's
    decision values to their rounding boundaries (in cells / planes)."""
    u, v, w = O.uvw_lambda(c["uvw"], c["freq"])
    u, v, w = u.ravel(), v.ravel(), w.ravel()
    if info["coplanar"]:
        w = np.zeros_like(w)
    neg = w < 0
    u, v, w = np.where(neg, -u, u), np.where(neg, -v, v), np.where(neg, -w, w)
    nu, nv, W, Ww = info["nu"], info["nv"], info["support"], info["w_support"]
    ku = u * nu * c["dx"]
    ku -= np.floor(ku / nu) * nu
    kv = v * nv * c["dy"]
    kv -= np.floor(kv / nv) * nv
    a0 = (np.ceil(ku - 0.5 * W).astype(np.int64) + nu) % nu
    b0 = (np.ceil(kv - 0.5 * W).astype(np.int64) + nv) % nv
    near = np.minimum(np.abs(ku - 0.5 * W - np.rint(ku - 0.5 * W)), np.abs(kv - 0.5 * W - np.rint(kv - 0.5 * W)))
    near = np.minimum(near, np.abs(ku / nu - np.rint(ku / nu)) * nu)
    near = np.minimum(near, np.abs(kv / nv - np.rint(kv / nv)) * nv)
    n_p0 = info["n_planes"] - Ww + 1
    p0 = np.zeros_like(a0)
    if not info["coplanar"]:
        kw = (w - info["w0"]) / info["dw"]
        p0 = np.clip(np.ceil(kw - 0.5 * Ww).astype(np.int64), 0, n_p0 - 1)
        near = np.minimum(near, np.abs(kw - 0.5 * Ww - np.rint(kw - 0.5 * Ww)))
    ntv = nv // 32
    n_tiles = (nu // 32) * ntv
    n_chan = len(c["freq"])
    chan = np.tile(np.arange(n_chan), len(c["uvw"]))
    bucket = (chan * n_p0 + p0) * n_tiles + (a0 // 32) * ntv + b0 // 32
    key = (bucket.astype(np.uint64) << np.uint64(10)) | ((a0 % 32) * 32 + b0 % 32).astype(np.uint64)
    return key, near, n_chan * n_p0 * n_tiles


@pytest.mark.parametrize("name", ["cfg0_coplanar", "cfg1_wstack", "cfg3_multichan", "wide_random", "cfg1_300k",
                                  "cfg1_32planes", "empty"])
@pytest.mark.parametrize("fp64", [False, True])
def test_plan_order_is_the_stable_sort_of_the_keys(name, fp64):
    from paper_2406_09144_amd import api
    c = layout(name)
    print(f"plan order: {name} fp64={fp64} n_vis={len(c['uvw']) * len(c['freq'])}", flush=True)
    pl = api.Plan(c["uvw"], c["freq"], c["nx"], c["ny"], c["dx"], c["dy"], eps=1e-10 if fp64 else 1e-5, fp64=fp64,
                  n_wplanes=c["n_wplanes"])
    info = pl.info
    keys, perm, bs = pl.export_order()
    n = len(keys)
    assert n == len(c["uvw"]) * len(c["freq"])
    # bit-exact record order and bucket offsets
    np.testing.assert_array_equal(perm, np.argsort(keys, kind="stable").astype(np.uint32))
    buckets = keys[perm] >> np.uint64(10)
    expect = np.searchsorted(buckets, np.arange(len(bs), dtype=np.uint64), side="left")
    np.testing.assert_array_equal(bs, expect)
    assert bs[-1] == n
    if n == 0:
        return
    # the keys follow the coordinate formula
    ref, near, n_keys = numpy_keys(c, info)
    assert len(bs) == n_keys + 1
    bad = keys != ref
    assert np.all(near[bad] < 1e-6), f"{int(bad.sum())} keys differ away from a rounding boundary"
    assert bad.mean() < 1e-3
    if name == "cfg1_32planes":
        assert info["n_planes"] == 32
