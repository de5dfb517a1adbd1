"""Sums of exponentials for power-law couplings (Sec. II C): marshalling for
the library's fit (``tdvp_fit_exponentials`` / ``tdvp_fit_power_law`` in
``include/tdvp.h``, a matrix pencil with optional Levenberg-Marquardt
refinement, host code in ``csrc/fit.cpp``)."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib


def _out(K: int):
    return np.zeros(2 * K, dtype=np.float64), np.zeros(2 * K, dtype=np.float64), C.c_double(0.0)


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(rc: int, what: str):
    if rc != 0:
        from .api import TDVPError
        raise TDVPError(rc, what)


def fit_exponentials(samples, K: int, refine: bool = False):
    """Return (c, lam, max_abs_err) with f(r) ~ Re sum_k c_k lam_k^r, r = 1..len(samples)."""
    f = np.ascontiguousarray(samples, dtype=np.float64)
    c, lam, err = _out(K)
    _check(_lib.load().tdvp_fit_exponentials(_dp(f), f.size, int(K), int(refine), _dp(c), _dp(lam), C.byref(err)),
           "tdvp_fit_exponentials failed")
    return c.view(np.complex128), lam.view(np.complex128), err.value


def fit_power_law(alpha: float, K: int, rmax: int, refine: bool = False):
    """Fit r^-alpha on r = 1..rmax with K exponentials."""
    c, lam, err = _out(K)
    _check(_lib.load().tdvp_fit_power_law(float(alpha), int(K), int(rmax), int(refine), _dp(c), _dp(lam),
                                          C.byref(err)), "tdvp_fit_power_law failed")
    return c.view(np.complex128), lam.view(np.complex128), err.value
