"""Error behaviour of the C ABI that needs no GPU: every entry point validates its
handles and arguments first and reports FR_EINVAL with a message, without
touching a device."""

import ctypes

import pytest

from paper_2406_09144_amd import _lib as L


@pytest.fixture(scope="module")
def lib():
    return L.load(import_torch=False)


def test_null_handles_are_rejected(lib):
    out = ctypes.c_void_p()
    freq = (ctypes.c_double * 1)(1e9)
    rc = lib.fr_plan_create(None, None, 0, ctypes.cast(freq, ctypes.c_void_p), 1, 16, 16, 1e-3, 1e-3, 1e-5, 0, 0,
                            ctypes.byref(out))
    assert rc == L.FR_EINVAL
    assert b"ctx" in lib.fr_last_error()
    assert lib.fr_degrid(None, None, None, None) == L.FR_EINVAL
    assert lib.fr_grid(None, None, None, None, None) == L.FR_EINVAL
    assert lib.fr_apply_RNR_approx(None, None, None, 1, None) == L.FR_EINVAL
    assert lib.fr_apply_RNR_exact(None, None, None, None, 1, None) == L.FR_EINVAL
    assert lib.fr_make_psf_kernel(None, None, 1.0, ctypes.byref(out), None) == L.FR_EINVAL
    assert lib.fr_likelihood_grad(None, None, 7, None, None, None, None, None, 1, None, None, None) == L.FR_EINVAL
    assert b"mode" in lib.fr_last_error()
    assert lib.fr_likelihood_grad(None, None, L.FR_LIK_FAST, None, None, None, None, None, 1, None, None,
                                  None) == L.FR_EINVAL
    assert lib.fr_cg_solve(None, None, None, None, None, None, None, 5, 0.0, None, None, None) == L.FR_EINVAL
    s, r = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.fr_query_footprint(None, None, L.FR_OP_DEGRID, 1, ctypes.byref(s), ctypes.byref(r)) == L.FR_EINVAL
    assert lib.fr_fft2(None, None, 1, 8, 8, -1, 0, None) == L.FR_EINVAL
    assert lib.fr_psf_create(None, 16, 16, 1, None, None, None, 0, ctypes.byref(out), None) == L.FR_EINVAL


def test_destroy_accepts_null(lib):
    lib.fr_plan_destroy(None)
    lib.fr_psf_destroy(None)
    lib.fr_ctx_destroy(None)


def test_profiler_api_without_gpu(lib):
    assert lib.fr_profile_enable(0) == L.FR_OK
    n, ms = ctypes.c_int64(), ctypes.c_double()
    assert lib.fr_profile_query(b"degrid", ctypes.byref(n), ctypes.byref(ms)) == L.FR_OK
    assert n.value == 0 and ms.value == 0.0
    assert lib.fr_profile_reset() == L.FR_OK
    assert lib.fr_profile_query(None, ctypes.byref(n), ctypes.byref(ms)) == L.FR_EINVAL


def test_error_status_names():
    e = L.FrError(L.FR_EINVAL, "x")
    assert "FR_EINVAL" in str(e) and e.status == L.FR_EINVAL
