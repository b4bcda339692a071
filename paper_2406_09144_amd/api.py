"""Thin torch-facing layer over the C ABI: argument checks and marshalling only.

Every numerical step runs in libfrmi's HIP kernels.  Tensors must live on the
GPU, be contiguous and have the precision of the plan/PSF they are used with
(float32/complex64, or float64/complex128 for FP64 objects).
"""

import ctypes

import torch

from . import _lib as L


def _lib():
    return L.load()


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _real_dtype(fp64):
    return torch.float64 if fp64 else torch.float32


def _cplx_dtype(fp64):
    return torch.complex128 if fp64 else torch.complex64


def _need(t, dtype, shape, name):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Context:
    _by_device = {}

    def __init__(self, device):
        h = ctypes.c_void_p()
        L.check(_lib().fr_ctx_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = int(device)

    @classmethod
    def get(cls, device=None):
        d = torch.cuda.current_device() if device is None else int(device)
        if d not in cls._by_device:
            cls._by_device[d] = Context(d)
        return cls._by_device[d]

    def __del__(self):
        try:
            if self.handle:
                _lib().fr_ctx_destroy(self.handle)
        except Exception:
            pass


class PSF:
    """Response kernel K_R [n_chan, px, py/2+1] on the px x py padded grid (2nx x 2ny,
    smaller for a reduced support) and noise kernel K_N [n_chan, nx, ny/2+1]."""

    def __init__(self, handle, nx, ny, n_chan, fp64, ctx):
        self.handle = handle
        self.nx, self.ny, self.n_chan, self.fp64 = nx, ny, n_chan, fp64
        self.ctx = ctx
        px, py = ctypes.c_int64(), ctypes.c_int64()
        L.check(_lib().fr_psf_get_padding(handle, ctypes.byref(px), ctypes.byref(py)))
        self.px, self.py = px.value, py.value

    def reduce(self, hx, hy=None, stream=None):
        """A new PSF object whose response kernel keeps the offsets |dx| <= hx,
        |dy| <= hy of this one's PSF, on the smaller padded grid (Sec. 3.3.2)."""
        hy = hx if hy is None else hy
        h = ctypes.c_void_p()
        L.check(_lib().fr_psf_reduce(self.handle, int(hx), int(hy), ctypes.byref(h), _stream(stream)))
        return PSF(h, self.nx, self.ny, self.n_chan, self.fp64, self.ctx)

    @classmethod
    def from_kernels(cls, K_R, K_N=None, nfac=None, ctx=None, stream=None):
        ctx = ctx or Context.get(K_R.device.index)
        fp64 = K_R.dtype == torch.float64
        if K_R.dim() == 2:
            K_R = K_R[None]
        n_chan, two_nx, nyp1 = K_R.shape
        nx, ny = two_nx // 2, nyp1 - 1
        rd = _real_dtype(fp64)
        K_R = _need(K_R.contiguous(), rd, (n_chan, 2 * nx, ny + 1), "K_R")
        if K_N is not None:
            K_N = _need(K_N.reshape(n_chan, nx, ny // 2 + 1).contiguous(), rd, (n_chan, nx, ny // 2 + 1), "K_N")
        if nfac is not None:
            nfac = _need(nfac.contiguous(), rd, (nx, ny), "nfac")
        h = ctypes.c_void_p()
        L.check(_lib().fr_psf_create(ctx.handle, nx, ny, n_chan, _ptr(K_R), _ptr(K_N), _ptr(nfac),
                                     L.FR_FP64 if fp64 else 0, ctypes.byref(h), _stream(stream)))
        return cls(h, nx, ny, n_chan, fp64, ctx)

    def kernels(self, stream=None):
        rd = _real_dtype(self.fp64)
        dev = torch.device("cuda", self.ctx.device)
        KR = torch.empty((self.n_chan, self.px, self.py // 2 + 1), dtype=rd, device=dev)
        KN = torch.empty((self.n_chan, self.nx, self.ny // 2 + 1), dtype=rd, device=dev)
        try:
            L.check(_lib().fr_psf_get_kernels(self.handle, _ptr(KR), _ptr(KN), _stream(stream)))
        except L.FrError:
            L.check(_lib().fr_psf_get_kernels(self.handle, _ptr(KR), None, _stream(stream)))
            KN = None
        return KR, KN

    def __del__(self):
        try:
            if self.handle:
                _lib().fr_psf_destroy(self.handle)
        except Exception:
            pass


def apply_RNR_approx(psf, x, out=None, stream=None):
    """R' x by the zero-padded PSF convolution; x [B, n_chan, nx, ny] or [n_chan, nx, ny]."""
    squeeze = x.dim() == 3
    xb = x[None] if squeeze else x
    B = xb.shape[0]
    _need(xb, _real_dtype(psf.fp64), (B, psf.n_chan, psf.nx, psf.ny), "x")
    y = out if out is not None else torch.empty_like(xb)
    L.check(_lib().fr_apply_RNR_approx(psf.handle, _ptr(xb), _ptr(y), B, _stream(stream)))
    return y[0] if squeeze and out is None else y


def fft2(x, sign=-1, ctx=None, stream=None):
    """In-place unnormalised 2D FFT of a contiguous complex tensor [..., n0, n1]."""
    ctx = ctx or Context.get(x.device.index)
    if not x.is_contiguous() or x.dtype not in (torch.complex64, torch.complex128):
        raise ValueError("x must be a contiguous complex64/complex128 GPU tensor")
    n0, n1 = x.shape[-2:]
    batch = x.numel() // (n0 * n1)
    L.check(_lib().fr_fft2(ctx.handle, _ptr(x), batch, n0, n1, int(sign),
                           int(x.dtype == torch.complex128), _stream(stream)))
    return x


class Plan:
    """Visibilities of one observation bucketed on the oversampled uv grid.

    uvw: host float64 [n_row, 3] metres; freq: host float64 [n_chan] Hz;
    nx, ny image size; dx, dy pixel sizes (radians); eps requested accuracy;
    w_taylor: expand the w-term in a Taylor series when that needs fewer planes
    than improved w-stacking (FR_W_TAYLOR); vector_spread: grid on the vector units
    even where the matrix-core spread applies (FR_VECTOR_SPREAD)."""

    def __init__(self, uvw, freq, nx, ny, dx, dy, eps=1e-5, fp64=False, divide_by_n=True,
                 coplanar=False, n_wplanes=0, w_taylor=False, vector_spread=False, ctx=None, device=None):
        import numpy as np
        self.ctx = ctx or Context.get(device)
        uvw = np.ascontiguousarray(uvw, dtype=np.float64).reshape(-1, 3)
        freq = np.ascontiguousarray(np.atleast_1d(freq), dtype=np.float64)
        flags = (L.FR_FP64 if fp64 else 0) | (L.FR_DIVIDE_BY_N if divide_by_n else 0) | \
            (L.FR_COPLANAR if coplanar else 0) | (L.FR_W_TAYLOR if w_taylor else 0) | \
            (L.FR_VECTOR_SPREAD if vector_spread else 0)
        h = ctypes.c_void_p()
        L.check(_lib().fr_plan_create(self.ctx.handle, uvw.ctypes.data_as(ctypes.c_void_p), uvw.shape[0],
                                      freq.ctypes.data_as(ctypes.c_void_p), freq.shape[0], int(nx), int(ny),
                                      float(dx), float(dy), float(eps), flags, int(n_wplanes), ctypes.byref(h)))
        self.handle = h
        self.nx, self.ny = int(nx), int(ny)
        self.n_row, self.n_chan = uvw.shape[0], freq.shape[0]
        self.fp64 = bool(fp64)
        self.divide_by_n = bool(divide_by_n)

    @property
    def info(self):
        inf = L.fr_plan_info()
        L.check(_lib().fr_plan_get_info(self.handle, ctypes.byref(inf)))
        return inf.as_dict()

    @property
    def device(self):
        return torch.device("cuda", self.ctx.device)

    def export_order(self):
        """The plan's bucketing as host numpy arrays: the sort key of every
        visibility (input order), the record order perm (perm[k] = visibility of
        record k) and the first record of every bucket (n_keys + 1 entries)."""
        import numpy as np
        nk = ctypes.c_int64()
        L.check(_lib().fr_plan_export_order(self.handle, None, None, None, ctypes.byref(nk)))
        n = self.n_row * self.n_chan
        keys = np.empty(n, np.uint64)
        perm = np.empty(n, np.uint32)
        bs = np.empty(nk.value + 1, np.int64)
        L.check(_lib().fr_plan_export_order(self.handle, keys.ctypes.data_as(ctypes.c_void_p),
                                            perm.ctypes.data_as(ctypes.c_void_p),
                                            bs.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nk)))
        return keys, perm, bs

    def img_shape(self, B=None):
        s = (self.n_chan, self.nx, self.ny)
        return s if B is None else (B,) + s

    def __del__(self):
        try:
            if self.handle:
                _lib().fr_plan_destroy(self.handle)
        except Exception:
            pass


def _img3(plan, img, name):
    if img.dim() == 2:
        img = img[None]
    return _need(img, _real_dtype(plan.fp64), plan.img_shape(), name)


def degrid(plan, img, out=None, stream=None, weight=None):
    """R: image [n_chan, nx, ny] (or [nx, ny]) -> visibilities [n_row, n_chan] complex;
    with weight [n_row, n_chan], N^-1 R (weights applied by the library as it stores)."""
    img = _img3(plan, img, "img")
    vis = out if out is not None else torch.empty((plan.n_row, plan.n_chan), dtype=_cplx_dtype(plan.fp64),
                                                  device=img.device)
    _need(vis, _cplx_dtype(plan.fp64), (plan.n_row, plan.n_chan), "vis")
    if weight is None:
        L.check(_lib().fr_degrid(plan.handle, _ptr(img), _ptr(vis), _stream(stream)))
    else:
        weight = _need(weight.reshape(plan.n_row, plan.n_chan), _real_dtype(plan.fp64),
                       (plan.n_row, plan.n_chan), "weight")
        L.check(_lib().fr_degrid_weighted(plan.handle, _ptr(img), _ptr(weight), _ptr(vis), _stream(stream)))
    return vis


def grid(plan, vis, weight=None, out=None, stream=None):
    """R^+ N^-1: visibilities [n_row, n_chan] complex (weights real, optional) -> image [n_chan, nx, ny]."""
    vis = _need(vis.reshape(plan.n_row, plan.n_chan), _cplx_dtype(plan.fp64), (plan.n_row, plan.n_chan), "vis")
    if weight is not None:
        weight = _need(weight.reshape(plan.n_row, plan.n_chan), _real_dtype(plan.fp64),
                       (plan.n_row, plan.n_chan), "weight")
    img = out if out is not None else torch.empty(plan.img_shape(), dtype=_real_dtype(plan.fp64), device=vis.device)
    _need(img, _real_dtype(plan.fp64), plan.img_shape(), "img")
    L.check(_lib().fr_grid(plan.handle, _ptr(vis), _ptr(weight), _ptr(img), _stream(stream)))
    return img


class Degrid(torch.autograd.Function):
    """V = R I.  For a real loss, torch hands backward g = dL/dRe V + i dL/dIm V,
    and dL/dI = Re R^H g = R^+ g, i.e. fr_grid without weights."""

    @staticmethod
    def forward(ctx, img, plan):
        ctx.plan = plan
        return degrid(plan, img.contiguous())

    @staticmethod
    def backward(ctx, g):
        gi = grid(ctx.plan, g.contiguous())
        return gi, None


class Grid(torch.autograd.Function):
    """I = R^+ (w V).  The gradient with respect to V in torch's convention is
    w (R g): fr_degrid_weighted (fr_degrid without weights)."""

    @staticmethod
    def forward(ctx, vis, plan, weight=None):
        ctx.plan = plan
        ctx.weight = weight
        return grid(plan, vis.contiguous(), weight)

    @staticmethod
    def backward(ctx, g):
        w = None if ctx.weight is None else ctx.weight.contiguous()
        return degrid(ctx.plan, g.contiguous(), weight=w), None, None


def make_psf_kernel(plan, weight=None, eps_noise=-1e-6, stream=None):
    """Response kernel K_R and noise kernel K_N of `plan` (weights [n_row, n_chan] or None).
    eps_noise > 0 is the absolute regulariser; < 0 is relative to the PSF peak."""
    if weight is not None:
        weight = _need(weight.reshape(plan.n_row, plan.n_chan), _real_dtype(plan.fp64),
                       (plan.n_row, plan.n_chan), "weight")
    h = ctypes.c_void_p()
    L.check(_lib().fr_make_psf_kernel(plan.handle, _ptr(weight), float(eps_noise), ctypes.byref(h),
                                      _stream(stream)))
    return PSF(h, plan.nx, plan.ny, plan.n_chan, plan.fp64, plan.ctx)


def apply_RNR_exact(plan, x, weight=None, out=None, stream=None):
    """R^+ N^-1 R x exactly; x [B, n_chan, nx, ny] or [n_chan, nx, ny]."""
    squeeze = x.dim() == 3
    xb = x[None] if squeeze else x
    B = xb.shape[0]
    _need(xb, _real_dtype(plan.fp64), plan.img_shape(B), "x")
    if weight is not None:
        weight = _need(weight.reshape(plan.n_row, plan.n_chan), _real_dtype(plan.fp64),
                       (plan.n_row, plan.n_chan), "weight")
    y = out if out is not None else torch.empty_like(xb)
    L.check(_lib().fr_apply_RNR_exact(plan.handle, _ptr(weight), _ptr(xb), _ptr(y), B, _stream(stream)))
    return y[0] if squeeze and out is None else y


def likelihood_grad(mode, s, data, plan=None, psf=None, weight=None, i_fixed=None, inv_power=None,
                    stream=None):
    """(H [B] float64, grad [B, n_chan, nx, ny]) of the EXACT (data = visibilities) or FAST
    (data = dirty image) likelihood with respect to the log-sky s [B, n_chan, nx, ny]."""
    obj = plan if mode == L.FR_LIK_EXACT else psf
    fp64 = obj.fp64
    rd = _real_dtype(fp64)
    B = s.shape[0]
    n_chan = obj.n_chan
    _need(s, rd, (B, n_chan, obj.nx, obj.ny), "s")
    if mode == L.FR_LIK_EXACT:
        _need(data, _cplx_dtype(fp64), (plan.n_row, plan.n_chan), "data")
        if weight is not None:
            weight = _need(weight.reshape(plan.n_row, plan.n_chan), rd, (plan.n_row, plan.n_chan), "weight")
    else:
        data = _need(data.reshape(n_chan, obj.nx, obj.ny), rd, (n_chan, obj.nx, obj.ny), "data")
    if i_fixed is not None:
        i_fixed = _need(i_fixed.reshape(n_chan, obj.nx, obj.ny), rd, (n_chan, obj.nx, obj.ny), "i_fixed")
    if inv_power is not None:
        inv_power = _need(inv_power, rd, (obj.nx, obj.ny // 2 + 1), "inv_power")
    g = torch.empty_like(s)
    H = torch.empty(B, dtype=torch.float64, device=s.device)
    L.check(_lib().fr_likelihood_grad(plan.handle if plan is not None else None,
                                      psf.handle if psf is not None else None, int(mode), _ptr(s), _ptr(i_fixed),
                                      _ptr(data), _ptr(weight), _ptr(inv_power), B, _ptr(g), _ptr(H),
                                      _stream(stream)))
    return H, g


def cg_solve(b, psf=None, plan=None, weight=None, inv_power=None, diag=None, maxiter=50, rtol=0.0,
             stream=None):
    """Solve (D R' D + S^-1) x = b by conjugate gradients; R' is the PSF convolution
    of `psf`, or the exact operator of `plan` when psf is None.  b [n_chan, nx, ny].
    Returns x, the residual-norm history [maxiter + 1] (float64) and the
    iteration count (0-d int32 tensor), all on the device."""
    obj = psf if psf is not None else plan
    rd = _real_dtype(obj.fp64)
    shape = (obj.n_chan, obj.nx, obj.ny)
    b = _need(b.reshape(shape), rd, shape, "b")
    if diag is not None:
        diag = _need(diag.reshape(shape), rd, shape, "diag")
    if inv_power is not None:
        inv_power = _need(inv_power, rd, (obj.nx, obj.ny // 2 + 1), "inv_power")
    if weight is not None:
        weight = _need(weight.reshape(plan.n_row, plan.n_chan), rd, (plan.n_row, plan.n_chan), "weight")
    x = torch.empty_like(b)
    hist = torch.zeros(maxiter + 1, dtype=torch.float64, device=b.device)
    iters = torch.zeros((), dtype=torch.int32, device=b.device)
    L.check(_lib().fr_cg_solve(plan.handle if plan is not None else None,
                               psf.handle if psf is not None else None, _ptr(weight), _ptr(inv_power), _ptr(diag),
                               _ptr(b), _ptr(x), int(maxiter), float(rtol), _ptr(hist), _ptr(iters),
                               _stream(stream)))
    return x, hist, iters


def periodic_conv(K, x, mode=L.FR_CONV_MUL, out=None, ctx=None, stream=None):
    """y = F^-1 diag(f(K)) F x on the periodic grid, f = K, 1/K, sqrt K, 1/sqrt K
    (FR_CONV_MUL / _DIV / _MUL_SQRT / _DIV_SQRT); K [nk, nx, ny/2+1] or [nx, ny/2+1]
    (image g uses K[g % nk]), x [..., nx, ny]."""
    ctx = ctx or Context.get(x.device.index)
    nx, ny = x.shape[-2:]
    fp64 = x.dtype == torch.float64
    rd = _real_dtype(fp64)
    Kb = K if K.dim() == 3 else K[None]
    Kb = _need(Kb.contiguous(), rd, (Kb.shape[0], nx, ny // 2 + 1), "K")
    xc = _need(x.contiguous(), rd, tuple(x.shape), "x")
    y = out if out is not None else torch.empty_like(xc)
    n_img = xc.numel() // (nx * ny)
    L.check(_lib().fr_periodic_conv(ctx.handle, _ptr(Kb), Kb.shape[0], int(mode), _ptr(xc), _ptr(y), n_img, nx, ny,
                                    int(fp64), _stream(stream)))
    return y


def _mgvi_args(psf, power, diag):
    rd = _real_dtype(psf.fp64)
    shape = (psf.n_chan, psf.nx, psf.ny)
    power = _need(power, rd, (psf.nx, psf.ny // 2 + 1), "power")
    if diag is not None:
        diag = _need(diag.reshape(shape), rd, shape, "diag")
    return rd, shape, power, diag


def mgvi_metric_apply(psf, power, diag, x, stream=None):
    """M x = x + A D R' N'^-1 R' D A x (MGVI metric in standardised coordinates)."""
    rd, shape, power, diag = _mgvi_args(psf, power, diag)
    x = _need(x.reshape(shape), rd, shape, "x")
    y = torch.empty_like(x)
    L.check(_lib().fr_mgvi_metric_apply(psf.handle, _ptr(power), _ptr(diag), _ptr(x), _ptr(y), _stream(stream)))
    return y


def mgvi_draw(psf, power, diag, eta0, eta1, stream=None):
    """eta0 + A D R' N'^-1/2 eta1: covariance M for white eta0, eta1."""
    rd, shape, power, diag = _mgvi_args(psf, power, diag)
    eta0 = _need(eta0.reshape(shape), rd, shape, "eta0")
    eta1 = _need(eta1.reshape(shape), rd, shape, "eta1")
    xi = torch.empty_like(eta0)
    L.check(_lib().fr_mgvi_draw(psf.handle, _ptr(power), _ptr(diag), _ptr(eta0), _ptr(eta1), _ptr(xi),
                                _stream(stream)))
    return xi


def mgvi_solve(psf, power, diag, b, maxiter=20, rtol=0.0, stream=None):
    """M x = b by CG; returns x, the residual history and the iteration count."""
    rd, shape, power, diag = _mgvi_args(psf, power, diag)
    b = _need(b.reshape(shape), rd, shape, "b")
    x = torch.empty_like(b)
    hist = torch.zeros(maxiter + 1, dtype=torch.float64, device=b.device)
    iters = torch.zeros((), dtype=torch.int32, device=b.device)
    L.check(_lib().fr_mgvi_solve(psf.handle, _ptr(power), _ptr(diag), _ptr(b), _ptr(x), int(maxiter), float(rtol),
                                 _ptr(hist), _ptr(iters), _stream(stream)))
    return x, hist, iters


def query_footprint(op, B=1, plan=None, psf=None):
    """(scratch_bytes, resident_bytes) of one call of `op` (host-only)."""
    s, r = ctypes.c_size_t(), ctypes.c_size_t()
    L.check(_lib().fr_query_footprint(plan.handle if plan is not None else None,
                                      psf.handle if psf is not None else None, int(op), int(B),
                                      ctypes.byref(s), ctypes.byref(r)))
    return s.value, r.value


def scratch_stats(stream=None, reset=False, ctx=None):
    """(peak bytes in use since the last reset, bytes held) of the library's scratch
    arena for `stream` (default: torch's current stream) on ctx's device."""
    ctx = ctx or Context.get()
    peak, held = ctypes.c_size_t(), ctypes.c_size_t()
    L.check(_lib().fr_scratch_stats(ctx.handle, _stream(stream), int(bool(reset)), ctypes.byref(peak),
                                    ctypes.byref(held)))
    return peak.value, held.value


def scratch_trim(stream=None, ctx=None):
    """Synchronise `stream` and return its arena's device memory."""
    ctx = ctx or Context.get()
    L.check(_lib().fr_scratch_trim(ctx.handle, _stream(stream)))


def inject_alloc_failure(after):
    """Make the library's device allocation after the next `after` fail (tests)."""
    L.check(_lib().fr_inject_alloc_failure(int(after)))


def profile_enable(on=True):
    """Turn the library's per-kernel hipEvent timing on or off (process-wide)."""
    L.check(_lib().fr_profile_enable(int(bool(on))))


def profile_reset():
    L.check(_lib().fr_profile_reset())


def profile_query(name):
    """(launches, total milliseconds) recorded for kernel `name` since the last reset."""
    n, ms = ctypes.c_int64(), ctypes.c_double()
    L.check(_lib().fr_profile_query(name.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


PROFILED_KERNELS = ["degrid", "grid", "grid_assemble", "zero", "wplane_rows_fwd", "wplane_cols_fwd", "wplane_cols_inv",
                    "wplane_rows_inv", "psfconv_rows_r2c", "psfconv_cols", "psfconv_rows_c2r",
                    "pconv_rows_r2c", "pconv_cols", "pconv_rows_c2r"]


class CorrelatedField:
    """Amplitude model of the correlated-field prior on an nx x ny grid
    (fr_cf_*): `power` turns hyperparameter excitations into the r2c half power
    spectrum [nx, ny/2+1], `logsky` turns field excitations into log-skies."""

    PRIOR_KEYS = ("offset", "zm_mean", "zm_std", "fluct_mean", "fluct_std", "slope_mean", "slope_std",
                  "flex_mean", "flex_std", "asp_mean", "asp_std")

    def __init__(self, nx, ny, ctx=None, device=None):
        self.ctx = ctx or Context.get(device)
        h = ctypes.c_void_p()
        L.check(_lib().fr_cf_create(self.ctx.handle, int(nx), int(ny), ctypes.byref(h)))
        self.handle = h
        self.nx, self.ny = int(nx), int(ny)
        J = ctypes.c_int64()
        L.check(_lib().fr_cf_num_bins(h, ctypes.byref(J)))
        self.n_bins = J.value

    def power(self, prior, xi_hyper, xi_v, xi_y, fp64=False, stream=None):
        import numpy as np
        pr = np.ascontiguousarray([float(prior[k]) for k in self.PRIOR_KEYS], dtype=np.float64)
        dev = torch.device("cuda", self.ctx.device)
        xi_hyper = _need(xi_hyper.to(dev).contiguous(), torch.float64, (5,), "xi_hyper")
        xi_v = _need(xi_v.to(dev).contiguous(), torch.float64, (self.n_bins,), "xi_v")
        xi_y = _need(xi_y.to(dev).contiguous(), torch.float64, (self.n_bins,), "xi_y")
        P = torch.empty((self.nx, self.ny // 2 + 1), dtype=_real_dtype(fp64), device=dev)
        L.check(_lib().fr_cf_power(self.handle, pr.ctypes.data_as(ctypes.c_void_p), _ptr(xi_hyper), _ptr(xi_v),
                                   _ptr(xi_y), _ptr(P), int(fp64), _stream(stream)))
        return P

    def logsky(self, power, offset, xi, stream=None):
        fp64 = power.dtype == torch.float64
        rd = _real_dtype(fp64)
        power = _need(power, rd, (self.nx, self.ny // 2 + 1), "power")
        shape = tuple(xi.shape)
        xi = _need(xi.reshape(-1, self.nx, self.ny).contiguous(), rd, (xi.numel() // (self.nx * self.ny),
                                                                      self.nx, self.ny), "xi")
        s = torch.empty_like(xi)
        L.check(_lib().fr_cf_logsky(self.handle, _ptr(power), float(offset), _ptr(xi), _ptr(s), xi.shape[0],
                                    int(fp64), _stream(stream)))
        return s.reshape(shape)

    def __del__(self):
        try:
            if self.handle:
                _lib().fr_cf_destroy(self.handle)
        except Exception:
            pass
