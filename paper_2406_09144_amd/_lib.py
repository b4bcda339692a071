"""ctypes binding of libfrmi.so: the C ABI of include/frmi.h, same names, no logic.

torch is imported before the library is loaded so that both share the HIP
runtime torch already brought into the process (one runtime, one set of
streams and allocations).  There is no fallback: if libfrmi.so has not been
built, loading raises.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfrmi.so")

FR_OK, FR_EINVAL, FR_ENOMEM, FR_EHIP, FR_EUNSUPPORTED, FR_EBUSY = 0, -1, -2, -3, -4, -5
FR_FP64, FR_DIVIDE_BY_N, FR_COPLANAR, FR_W_TAYLOR, FR_VECTOR_SPREAD = 1, 2, 4, 8, 16
FR_LIK_EXACT, FR_LIK_FAST = 0, 1
FR_CONV_MUL, FR_CONV_DIV, FR_CONV_MUL_SQRT, FR_CONV_DIV_SQRT = 0, 1, 2, 3
(FR_OP_DEGRID, FR_OP_GRID, FR_OP_RNR_APPROX, FR_OP_RNR_EXACT, FR_OP_LIK_EXACT,
 FR_OP_LIK_FAST, FR_OP_CG, FR_OP_MAKE_PSF) = range(8)

FR_NOALLOC_SCRATCH_BYTES = 64 << 20

_STATUS = {FR_EINVAL: "FR_EINVAL", FR_ENOMEM: "FR_ENOMEM", FR_EHIP: "FR_EHIP",
           FR_EUNSUPPORTED: "FR_EUNSUPPORTED", FR_EBUSY: "FR_EBUSY"}


class FrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class fr_plan_info(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
        ("nu", ctypes.c_int64), ("nv", ctypes.c_int64),
        ("n_row", ctypes.c_int64), ("n_chan", ctypes.c_int64),
        ("precision", ctypes.c_int), ("support", ctypes.c_int),
        ("beta", ctypes.c_double), ("coplanar", ctypes.c_int),
        ("n_planes", ctypes.c_int), ("w_support", ctypes.c_int),
        ("w_beta", ctypes.c_double), ("w0", ctypes.c_double), ("dw", ctypes.c_double),
        ("eps_bound", ctypes.c_double), ("tile", ctypes.c_int),
        ("n_workitems", ctypes.c_int64), ("resident_bytes", ctypes.c_size_t),
        ("w_taylor", ctypes.c_int),
        ("records_per_run", ctypes.c_double), ("matrix_spread", ctypes.c_int),
        ("paired_degrid", ctypes.c_int), ("degrid_slots", ctypes.c_int64),
        ("active_tiles", ctypes.c_int64), ("active_tile_cols", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I = ctypes.c_int
_D = ctypes.c_double
_PP = ctypes.POINTER(ctypes.c_void_p)

SIGNATURES = {
    "fr_version": ([], ctypes.c_char_p),
    "fr_last_error": ([], ctypes.c_char_p),
    "fr_ctx_create": ([_I, _PP], _I),
    "fr_ctx_destroy": ([_P], None),
    "fr_plan_create": ([_P, _P, _I64, _P, _I64, _I64, _I64, _D, _D, _D, _I, _I, _PP], _I),
    "fr_plan_destroy": ([_P], None),
    "fr_plan_get_info": ([_P, ctypes.POINTER(fr_plan_info)], _I),
    "fr_degrid": ([_P, _P, _P, _P], _I),
    "fr_degrid_weighted": ([_P, _P, _P, _P, _P], _I),
    "fr_plan_export_order": ([_P, _P, _P, _P, ctypes.POINTER(_I64)], _I),
    "fr_grid": ([_P, _P, _P, _P, _P], _I),
    "fr_make_psf_kernel": ([_P, _P, _D, _PP, _P], _I),
    "fr_psf_create": ([_P, _I64, _I64, _I64, _P, _P, _P, _I, _PP, _P], _I),
    "fr_psf_reduce": ([_P, _I64, _I64, _PP, _P], _I),
    "fr_psf_get_padding": ([_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)], _I),
    "fr_psf_get_kernels": ([_P, _P, _P, _P], _I),
    "fr_psf_destroy": ([_P], None),
    "fr_apply_RNR_approx": ([_P, _P, _P, _I64, _P], _I),
    "fr_apply_RNR_approx_noalloc": ([_P, _P, _P, _I64, _P], _I),
    "fr_apply_RNR_exact": ([_P, _P, _P, _P, _I64, _P], _I),
    "fr_likelihood_grad": ([_P, _P, _I, _P, _P, _P, _P, _P, _I64, _P, _P, _P], _I),
    "fr_cg_solve": ([_P, _P, _P, _P, _P, _P, _P, _I, _D, _P, _P, _P], _I),
    "fr_periodic_conv": ([_P, _P, _I64, _I, _P, _P, _I64, _I64, _I64, _I, _P], _I),
    "fr_mgvi_metric_apply": ([_P, _P, _P, _P, _P, _P], _I),
    "fr_mgvi_draw": ([_P, _P, _P, _P, _P, _P, _P], _I),
    "fr_mgvi_solve": ([_P, _P, _P, _P, _P, _I, _D, _P, _P, _P], _I),
    "fr_cf_create": ([_P, _I64, _I64, _PP], _I),
    "fr_cf_num_bins": ([_P, ctypes.POINTER(_I64)], _I),
    "fr_cf_power": ([_P, _P, _P, _P, _P, _P, _I, _P], _I),
    "fr_cf_logsky": ([_P, _P, _D, _P, _P, _I64, _I, _P], _I),
    "fr_cf_destroy": ([_P], None),
    "fr_query_footprint": ([_P, _P, _I, _I64, ctypes.POINTER(ctypes.c_size_t),
                            ctypes.POINTER(ctypes.c_size_t)], _I),
    "fr_scratch_stats": ([_P, _P, _I, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)], _I),
    "fr_scratch_trim": ([_P, _P], _I),
    "fr_inject_alloc_failure": ([_I64], _I),
    "fr_fft2": ([_P, _P, _I64, _I64, _I64, _I, _I, _P], _I),
    "fr_profile_enable": ([_I], _I),
    "fr_profile_reset": ([], _I),
    "fr_profile_query": ([ctypes.c_char_p, ctypes.POINTER(_I64), ctypes.POINTER(_D)], _I),
}

_lib = None


def load(import_torch=True):
    """Load libfrmi.so (after torch, so both use one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if import_torch:
        import torch  # noqa: F401  (brings the process's HIP runtime in first)
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libfrmi.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(status):
    if status != FR_OK:
        msg = _lib.fr_last_error().decode(errors="replace") if _lib is not None else ""
        raise FrError(status, msg)
    return status
