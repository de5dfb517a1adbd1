"""ctypes declarations of the C ABI in include/tdvp.h."""
from __future__ import annotations

import ctypes as C
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtdvp.so")
_lib = None

STATUS = {
    0: "TDVP_OK", 1: "TDVP_E_ARG", 2: "TDVP_E_SHAPE", 3: "TDVP_E_DTYPE", 4: "TDVP_E_NOMEM",
    5: "TDVP_E_HIP", 6: "TDVP_E_NOCONV", 7: "TDVP_E_NUMERIC", 8: "TDVP_E_STATE", 9: "TDVP_E_SOLVER",
}

TDVP_C64 = 0
TDVP_C128 = 1

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class MpoSpec(C.Structure):
    _fields_ = [
        ("N", C.c_int), ("d", C.c_int), ("n_terms", C.c_int),
        ("g", C.POINTER(C.c_double)), ("A_ops", C.POINTER(C.c_double)), ("B_ops", C.POINTER(C.c_double)),
        ("K", C.c_int), ("c", C.POINTER(C.c_double)), ("lam", C.POINTER(C.c_double)),
        ("coupling", C.POINTER(C.c_double)), ("onsite", C.POINTER(C.c_double)), ("h", C.c_double),
        ("alpha", C.c_double), ("fit_rmax", C.c_int), ("fit_refine", C.c_int),
    ]


class Opts(C.Structure):
    _fields_ = [
        ("compute", C.c_int), ("krylov_max", C.c_int), ("krylov_tol", C.c_double),
        ("chi_max", C.c_int), ("w_max", C.c_double), ("eps_rel", C.c_double),
        ("multiplet_guard", C.c_int), ("strict", C.c_int), ("gemm_form", C.c_int),
        ("svd_mode", C.c_int), ("imaginary", C.c_int), ("exp_method", C.c_int), ("u1_block_min", C.c_int),
    ]


class SegOpts(C.Structure):
    _fields_ = [
        ("compute", C.c_int), ("krylov_k", C.c_int), ("chi_max", C.c_int), ("w_max", C.c_double),
        ("eps_rel", C.c_double), ("multiplet_guard", C.c_int), ("static_shapes", C.c_int),
        ("batched", C.c_int), ("use_graph", C.c_int), ("svd_mode", C.c_int), ("one_site", C.c_int),
        ("max_phases", C.c_int),
    ]


class HeffDesc(C.Structure):
    _fields_ = [
        ("nsite", C.c_int), ("chil", C.c_int), ("chir", C.c_int), ("d", C.c_int), ("wl", C.c_int),
        ("wm", C.c_int), ("wr", C.c_int), ("L", C.c_void_p), ("W1", C.c_void_p), ("W2", C.c_void_p),
        ("R", C.c_void_p), ("theta", C.c_void_p), ("out", C.c_void_p),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("w_step", C.c_double), ("w_total", C.c_double), ("seconds", C.c_double), ("flops", C.c_double),
        ("chi_peak", C.c_int), ("matvecs", C.c_int), ("krylov_max_used", C.c_int), ("flags", C.c_int),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_P = C.c_void_p
_I = C.c_int
_D = C.c_double
_PI = C.POINTER(C.c_int)
_PD = C.POINTER(C.c_double)

SIGNATURES = {
    "tdvp_version": (C.c_char_p, []),
    "tdvp_ctx_create": (_I, [_I, _P, ALLOC_FN, FREE_FN, _P, C.POINTER(_P)]),
    "tdvp_ctx_destroy": (_I, [_P]),
    "tdvp_last_error": (C.c_char_p, [_P]),
    "tdvp_ctx_sync": (_I, [_P]),
    "mpo_longrange": (_I, [_P, C.POINTER(MpoSpec), C.POINTER(_P), _PD]),
    "tdvp_fit_exponentials": (_I, [_PD, _I, _I, _I, _PD, _PD, _PD]),
    "tdvp_fit_power_law": (_I, [_D, _I, _I, _I, _PD, _PD, _PD]),
    "mpo_from_tensors": (_I, [_P, _I, _I, _PI, _PD, C.POINTER(_P)]),
    "mpo_get_info": (_I, [_P, _PI, _PI, _PI]),
    "mpo_get_tensor": (_I, [_P, _I, _PD]),
    "mpo_destroy": (_I, [_P]),
    "mpo_set_charges": (_I, [_P, _PI]),
    "mps_set_charges": (_I, [_P, _PI, _PI]),
    "mps_get_charges": (_I, [_P, _PI, _PI]),
    "mps_init": (_I, [_P, _I, _I, _PI, _PI, C.c_uint64, C.POINTER(_P)]),
    "mps_get_info": (_I, [_P, _PI, _PI, _PI]),
    "mps_get_tensor": (_I, [_P, _I, _PD]),
    "mps_set_tensor": (_I, [_P, _I, _PD, _I, _I]),
    "mps_right_canonicalize": (_I, [_P, _P]),
    "mps_destroy": (_I, [_P]),
    "tdvp_opts_default": (_I, [C.POINTER(Opts)]),
    "tdvp1_step": (_I, [_P, _P, _P, _D, C.POINTER(Opts), C.POINTER(Stats)]),
    "tdvp2_step": (_I, [_P, _P, _P, _D, C.POINTER(Opts), C.POINTER(Stats)]),
    "tdvp_hybrid_step": (_I, [_P, _P, _P, _D, C.POINTER(Opts), C.POINTER(Stats), C.POINTER(_I)]),
    "dmrg2_sweep": (_I, [_P, _P, _P, C.POINTER(Opts), C.POINTER(Stats), C.POINTER(_D)]),
    "apply_heff": (_I, [_P, _I, _I, _I, _I, _I, _I, _I, _I, _P, _P, _P, _P, _P, _P]),
    "apply_heff_batched": (_I, [_P, _I, _I, C.POINTER(HeffDesc)]),
    "apply_heff_noalloc": (_I, [_P, _I, _I, _I, _I, _I, _I, _I, _I, _P, _P, _P, _P, _P, _P]),
    "apply_heff_noalloc_max_bytes": (C.c_size_t, []),
    "env_update": (_I, [_P, _I, _I, _I, _I, _I, _I, _I, _P, _P, _P, _P]),
    "env_update_adjoint": (_I, [_P, _I, _I, _I, _I, _I, _I, _I] + [_P] * 7),
    "apply_heff_u1": (_I, [_P, _I, _I, _I, _I, _I, _I, _I, _I, _PI, _PI, _PI, _PI, _PI] + [_P] * 6),
    "env_update_u1": (_I, [_P, _I, _I, _I, _I, _I, _I, _I, _PI, _PI, _PI, _PI, _PI] + [_P] * 4),
    "apply_heff_adjoint": (_I, [_P, _I, _I, _I, _I, _I, _I, _I, _I] + [_P] * 11),
    "expect": (_I, [_P, _P, _I, _PI, _PD, _PD]),
    "transition_expect": (_I, [_P, _P, _P, _I, _PI, _PD, _PD]),
    "mps_apply_site": (_I, [_P, _P, _I, _PD]),
    "expect2": (_I, [_P, _P, _I, _PI, _PI, _PD, _PD, _PD]),
    "energy": (_I, [_P, _P, _P, _PD]),
    "norm2": (_I, [_P, _P, _PD]),
    "overlap": (_I, [_P, _P, _P, _PD]),
    "tdvp_seg_opts_default": (_I, [C.POINTER(SegOpts)]),
    "seg_init": (_I, [_P, _P, _I, _I, _PI, C.POINTER(_P), _I, _PI, _I, C.POINTER(_P)]),
    "seg_step": (_I, [_P, _P, _P, _D, C.POINTER(SegOpts), C.POINTER(Stats)]),
    "seg_get_info": (_I, [_P, _PI, _PI, _PI, _PD]),
    "seg_get_psi": (_I, [_P, _I, _PD]),
    "seg_get_bond": (_I, [_P, _I, _PD]),
    "seg_destroy": (_I, [_P]),
    "seg_norm2": (_I, [_P, _P, _PD]),
    "seg_reorthonormalize": (_I, [_P, _P, _P]),
    "seg_schedule": (_I, [_I, _PI, _D, _I, _I, _PI, _PI, _PI, _PD, _PI]),
    "seg_schedule1": (_I, [_I, _PI, _D, _I, _I, _PI, _PI, _PI, _PD, _PI]),
    "tdvp_profile_enable": (_I, [_P, _I]),
    "tdvp_ctx_set_gemm_form": (_I, [_P, _I]),
    "tdvp_profile_read": (_I, [_P, _I, C.c_char_p, _PD, _PD, _PD, C.POINTER(C.c_long), _PI]),
}


def lib_path() -> str:
    return _LIB_PATH


def load() -> C.CDLL:
    """Load libtdvp.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(
            f"{_LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_1912_06127_amd.build)")
    lib = C.CDLL(_LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
