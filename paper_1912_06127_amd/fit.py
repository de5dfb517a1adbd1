"""Sums of exponentials for power-law couplings (Sec. II C).

Power laws have no compact MPO, so f(r) = r^-alpha is approximated by
sum_k c_k lambda_k^r, which the MPO encodes with one decaying channel per
exponential.  The paper cites the method of Pirvu et al. without its steps;
this is a matrix-pencil fit: the Hankel matrix of the samples f(1..R) is cut
to rank K by an SVD, the decay factors are the eigenvalues of the shift
operator on its dominant right singular vectors, and the weights follow by
linear least squares.  Optionally the pencil result is refined by
Levenberg-Marquardt iterations on all 4K real parameters (real and imaginary
parts of the weights and decay factors), minimising the squared residuals
of the real part and the imaginary part of the sum (the latter keeps
conjugate pairs conjugate), inside Lawson's reweighting towards the
minimax fit (weights multiplied by the absolute residual after each
solve); the refined fit is kept only when its maximum absolute error is
smaller.  Host-side preprocessing of MPO parameters.
"""
from __future__ import annotations

import numpy as np


def _refine(f, c, lam, iters: int = 200, weights=None):
    """Levenberg-Marquardt on (Re c, Im c, Re lam, Im lam) for the weighted
    residuals sqrt(w_r) (Re(sum c lam^r) - f(r)) and Im(sum c lam^r), r = 1..R."""
    R, K = f.size, c.size
    r = np.arange(1, R + 1)
    sw = np.sqrt(np.ones(R) if weights is None else weights)
    sw2 = np.concatenate([sw, sw])

    def residual(c, lam):
        z = (lam[None, :] ** r[:, None]) @ c
        return sw2 * np.concatenate([z.real - f, z.imag])

    def jacobian(c, lam):
        P = lam[None, :] ** r[:, None]                                   # d/dc
        dP = c[None, :] * r[:, None] * lam[None, :] ** (r[:, None] - 1)  # d/dlam
        cols = [P, 1j * P, dP, 1j * dP]                                  # d/d(Re c, Im c, Re lam, Im lam)
        J = np.concatenate(cols, axis=1)
        return sw2[:, None] * np.concatenate([J.real, J.imag], axis=0)

    mu = 1e-3
    res = residual(c, lam)
    cost = float(res @ res)
    for _ in range(iters):
        J = jacobian(c, lam)
        A = J.T @ J
        g = J.T @ res
        step = np.linalg.solve(A + mu * np.diag(np.diag(A) + 1e-300), -g)
        dc = step[:K] + 1j * step[K:2 * K]
        dl = step[2 * K:3 * K] + 1j * step[3 * K:]
        c2, lam2 = c + dc, lam + dl
        if np.any(np.abs(lam2) >= 1.0):  # keep every channel decaying
            mu *= 10.0
            continue
        res2 = residual(c2, lam2)
        cost2 = float(res2 @ res2)
        if cost2 < cost:
            c, lam, res = c2, lam2, res2
            converged = cost - cost2 <= 1e-15 * cost
            cost = cost2
            mu = max(mu / 3.0, 1e-12)
            if converged:
                break
        else:
            mu *= 10.0
            if mu > 1e12:
                break
    return c, lam


def fit_exponentials(samples, K: int, refine: bool = False):
    """Return (c, lam, max_abs_err) with f(r) ~ Re sum_k c_k lam_k^r, r = 1..len(samples).

    refine = True adds Levenberg-Marquardt iterations after the matrix pencil."""
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
    if refine:
        # Lawson reweighting towards the minimax fit: weights grow where the
        # residual is large; the best maximum error seen is kept
        rr = np.arange(1, R + 1)
        w = np.ones(R)
        c2, lam2 = c, lam
        for _ in range(30):
            c2, lam2 = _refine(f, c2, lam2, weights=w)
            z = (lam2[None, :] ** rr[:, None]) @ c2
            res = np.abs(z.real - f)
            err2 = float(np.max(res))
            if err2 < err and np.all(np.abs(lam2) < 1.0):
                c, lam, err = c2, lam2, err2
            w = w * (res + 1e-3 * err2)
            w /= w.sum() / R
    return c, lam, err


def fit_power_law(alpha: float, K: int, rmax: int, refine: bool = False):
    """Fit r^-alpha on r = 1..rmax with K exponentials."""
    r = np.arange(1, rmax + 1, dtype=np.float64)
    return fit_exponentials(r ** (-alpha), K, refine)


def coupling_values(c, lam, rmax: int) -> np.ndarray:
    """[f(1), ..., f(rmax)] of the fitted sum."""
    r = np.arange(1, rmax + 1)
    return (np.asarray(lam)[None, :] ** r[:, None] @ np.asarray(c)).real
