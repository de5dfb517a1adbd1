"""Sums of exponentials for power-law couplings (Sec. II C).

Power laws have no compact MPO, so f(r) = r^-alpha is approximated by
sum_k c_k lambda_k^r, which the MPO encodes with one decaying channel per
exponential.  The paper cites the method of Pirvu et al. without its steps;
this is a matrix-pencil fit: the Hankel matrix of the samples f(1..R) is cut
to rank K by an SVD, the decay factors are the eigenvalues of the shift
operator on its dominant right singular vectors, and the weights follow by
linear least squares.  Host-side preprocessing of MPO parameters.
"""
from __future__ import annotations

import numpy as np


def fit_exponentials(samples, K: int):
    """Return (c, lam, max_abs_err) with f(r) ~ Re sum_k c_k lam_k^r, r = 1..len(samples)."""
    f = np.asarray(samples, dtype=np.float64)
    R = f.size
    if K < 1 or R < 2 * K:
        raise ValueError("need K >= 1 and at least 2K samples")
    P = R // 2
    hankel = np.lib.stride_tricks.sliding_window_view(f, P + 1)  # rows f(i+1 .. i+P+1)
    _, _, vh = np.linalg.svd(hankel, full_matrices=False)
    top = vh[:K]
    shift = top[:, 1:] @ np.linalg.pinv(top[:, :-1])
    lam = np.linalg.eigvals(shift)
    powers = lam[None, :] ** np.arange(1, R + 1)[:, None]
    c = np.linalg.lstsq(powers, f.astype(np.complex128), rcond=None)[0]
    err = float(np.max(np.abs((powers @ c).real - f)))
    return c, lam, err


def fit_power_law(alpha: float, K: int, rmax: int):
    """Fit r^-alpha on r = 1..rmax with K exponentials."""
    r = np.arange(1, rmax + 1, dtype=np.float64)
    return fit_exponentials(r ** (-alpha), K)


def coupling_values(c, lam, rmax: int) -> np.ndarray:
    """[f(1), ..., f(rmax)] of the fitted sum."""
    r = np.arange(1, rmax + 1)
    return (np.asarray(lam)[None, :] ** r[:, None] @ np.asarray(c)).real
