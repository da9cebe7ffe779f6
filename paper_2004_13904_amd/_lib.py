"""ctypes binding of libfastfocus (argument marshalling only; all compute runs in HIP).

The names mirror the C ABI in include/fastfocus.h.  Torch tensors are passed as raw device
pointers on torch's current HIP stream.  There is no CPU fallback: if the library or a GPU is
missing every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libfastfocus.so")

FF_OK = 0
FF_EINVAL, FF_ESHAPE, FF_EDTYPE, FF_ENOMEM, FF_EHIP, FF_EDEVICE, FF_ENOTIMPL = -1, -2, -3, -4, -5, -6, -7
FF_F32, FF_F64 = 0, 1
FF_GRAVITY_GZ, FF_MAGNETIC_TFA = 0, 1
STATUS = {0: "FF_OK", -1: "FF_EINVAL", -2: "FF_ESHAPE", -3: "FF_EDTYPE", -4: "FF_ENOMEM",
          -5: "FF_EHIP", -6: "FF_EDEVICE", -7: "FF_ENOTIMPL"}

EXPORTS = ["build_spectra", "ff_free_spectra", "ff_spectra_info", "ff_kernel_table", "apply_G",
           "apply_GT", "apply_G_block", "ff_workspace_size", "gkb_project", "rsvd_project",
           "irls_step", "ff_get_tuning", "ff_set_tuning", "ff_profile_begin", "ff_profile_end", "ff_time_pass",
           "ff_multi_create", "ff_multi_apply", "ff_multi_time_pass", "ff_multi_free", "ff_spectra_save", "ff_spectra_load",
           "ff_spectra_geometry", "ff_solver_stats", "ff_focusing_loss", "ff_focusing_grad", "ff_fft_1d",
           "ff_apply_block_noalloc", "ff_last_error"]


class FFGeometry(C.Structure):
    _fields_ = [("sx", C.c_int32), ("sy", C.c_int32), ("nz", C.c_int32),
                ("pad_xl", C.c_int32), ("pad_xr", C.c_int32), ("pad_yl", C.c_int32),
                ("pad_yr", C.c_int32), ("dx", C.c_double), ("dy", C.c_double),
                ("z_edges", C.POINTER(C.c_double)), ("kernel", C.c_int32),
                ("incl_deg", C.c_double), ("decl_deg", C.c_double), ("field_nT", C.c_double),
                ("nfft_x", C.c_int32), ("nfft_y", C.c_int32)]


class FFIrlsParams(C.Structure):
    _fields_ = [("solver", C.c_int32), ("t", C.c_int32), ("tp", C.c_int32), ("k", C.c_int32),
                ("lam", C.c_double), ("eps2", C.c_double), ("beta_depth", C.c_double),
                ("m_min", C.c_double), ("m_max", C.c_double), ("alpha_fixed", C.c_double),
                ("power_iters", C.c_int32), ("seed", C.c_uint64), ("basis_dtype", C.c_int32)]


class FFTuning(C.Structure):
    _fields_ = [("lg_G", C.c_int32), ("lg_GT", C.c_int32), ("row_tile", C.c_int32), ("batch", C.c_int32),
                ("col_batched", C.c_int32), ("rsvd_qr", C.c_int32), ("pair_fused", C.c_int32),
                ("gkb_graph", C.c_int32), ("fft_plan_x", C.c_int32), ("fft_plan_y", C.c_int32),
                ("gkb_onesided", C.c_int32)]


class FastFocusError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} -> {STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load(path=None):
    """Load the shared library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise FastFocusError("load", -7, f"{path} is missing; run python -m paper_2004_13904_amd.build")
    lib = C.CDLL(path)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    sig = {
        "build_spectra": [C.POINTER(FFGeometry), i32, vp, C.POINTER(vp)],
        "ff_free_spectra": [vp],
        "ff_spectra_info": [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i32), C.POINTER(i32),
                            C.POINTER(i32)],
        "ff_kernel_table": [vp, vp, vp],
        "apply_G": [vp, vp, vp, vp, vp, vp],
        "apply_GT": [vp, vp, vp, vp, vp, vp],
        "apply_G_block": [vp, i32, i64, vp, i64, vp, i64, vp, vp, vp],
        "ff_apply_block_noalloc": [vp, i32, i64, vp, i64, vp, i64, vp, vp, vp],
        "ff_workspace_size": [vp, i32, i32, i32, i32, C.POINTER(C.c_size_t)],
        "gkb_project": [vp, vp, vp, vp, i32, i32, i32, i32, vp, dp, vp, vp, C.c_size_t, vp],
        "rsvd_project": [vp, vp, vp, vp, i32, i32, vp, C.c_uint64, i32, i32, i32, vp, dp, vp, vp, C.c_size_t, vp],
        "irls_step": [vp, C.POINTER(FFIrlsParams), vp, vp, vp, vp, vp, vp, dp, dp, vp, C.c_size_t,
                      vp],
        "ff_get_tuning": [vp, C.POINTER(FFTuning)],
        "ff_set_tuning": [vp, C.POINTER(FFTuning)],
        "ff_profile_begin": [vp, i32],
        "ff_time_pass": [vp, i32, i32, i32, vp, vp, vp],
        "ff_profile_end": [vp, dp, C.POINTER(i64)],
        "ff_multi_create": [i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                            C.POINTER(vp)],
        "ff_multi_apply": [vp, vp],
        "ff_multi_time_pass": [vp, i32, i32, vp],
        "ff_multi_free": [vp],
        "ff_spectra_save": [vp, C.c_char_p],
        "ff_spectra_load": [C.c_char_p, vp, C.POINTER(vp)],
        "ff_spectra_geometry": [vp, C.POINTER(FFGeometry), C.POINTER(C.c_double)],
        "ff_solver_stats": [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)],
        "ff_focusing_loss": [vp, i64, vp, vp, vp, C.c_double, C.c_double, vp, vp, vp],
        "ff_focusing_grad": [vp, i64, vp, vp, C.c_double, C.c_double, vp, vp, vp],
        "ff_fft_1d": [i32, i32, i32, i32, i64, vp, vp, vp, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = i32
    lib.ff_last_error.argtypes = []
    lib.ff_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def check(fn, code):
    if code != FF_OK:
        msg = load().ff_last_error().decode(errors="replace")
        raise FastFocusError(fn, code, msg)


def call(name, *args):
    lib = load()
    check(name, getattr(lib, name)(*args))


def make_geometry(s, nfft=(0, 0)):
    """FFGeometry from a survey dict (keys as in workloads.survey).  Returns (struct, keepalive)."""
    z = (C.c_double * len(s["z_edges"]))(*s["z_edges"])
    kern = FF_GRAVITY_GZ if s.get("kernel", "gravity") == "gravity" else FF_MAGNETIC_TFA
    g = FFGeometry(s["sx"], s["sy"], s["nz"], s.get("pad_xl", 0), s.get("pad_xr", 0),
                   s.get("pad_yl", 0), s.get("pad_yr", 0), float(s["dx"]), float(s["dy"]),
                   C.cast(z, C.POINTER(C.c_double)), kern, float(s.get("incl_deg", 90.0)),
                   float(s.get("decl_deg", 0.0)), float(s.get("field_nT", 50000.0)),
                   int(nfft[0]), int(nfft[1]))
    return g, z
