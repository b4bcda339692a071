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
    """Response kernel K_R [n_chan, 2nx, ny+1] and noise kernel K_N [n_chan, nx, ny/2+1]."""

    def __init__(self, handle, nx, ny, n_chan, fp64, ctx):
        self.handle = handle
        self.nx, self.ny, self.n_chan, self.fp64 = nx, ny, n_chan, fp64
        self.ctx = ctx

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
        KR = torch.empty((self.n_chan, 2 * self.nx, self.ny + 1), dtype=rd, device=dev)
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
