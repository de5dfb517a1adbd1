"""Lanczos evaluation of exp(-i tau H) theta (Sec. III A; Park and Light).

Only products H v are used.  The Krylov basis is kept in complex128 with
two classical Gram-Schmidt passes against all previous vectors, the k x k
tridiagonal matrix T_k is diagonalised exactly, and the iteration stops on
the a-posteriori estimate beta_k |e_k^T exp(-i tau T_k) e_1| <= tol, or on a
happy breakdown.  The paper used ARPACK with at most 8 vectors and tolerance
1e-6 (Supplemental Material, simulation details); its stopping rule is not
stated, so this estimate is the oracle's reading.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def expm_krylov(apply, theta: np.ndarray, tau: float, kmax: int = 40, tol: float = 1e-13,
                return_info: bool = False):
    """exp(-i tau H) theta with H Hermitian, given apply(v) = H v."""
    shape = theta.shape
    v0 = theta.reshape(-1).astype(np.complex128)
    beta0 = np.linalg.norm(v0)
    if beta0 == 0.0:
        out = theta.copy()
        return (out, 0) if return_info else out
    V = [v0 / beta0]
    alphas, betas = [], []
    y = None
    k_used = 0
    for k in range(kmax):
        w = apply(V[k].reshape(shape)).reshape(-1)
        a = float(np.vdot(V[k], w).real)
        w = w - a * V[k]
        if k > 0:
            w = w - betas[-1] * V[k - 1]
        for _ in range(2):  # classical Gram-Schmidt, twice
            Vm = np.array(V)
            w = w - Vm.T @ (Vm.conj() @ w)
        b = float(np.linalg.norm(w))
        alphas.append(a)
        if k == 0:
            evals, evecs = np.array([a]), np.ones((1, 1))
        else:
            evals, evecs = sla.eigh_tridiagonal(np.array(alphas), np.array(betas))
        y = evecs @ (np.exp(-1j * tau * evals) * evecs[0, :])
        k_used = k + 1
        scale = max(max(abs(x) for x in alphas), max(betas) if betas else 0.0)
        if b * abs(y[-1]) <= tol or b <= 1e-14 * scale or scale == 0.0:
            break
        betas.append(b)
        V.append(w / b)
    out = beta0 * (np.array(V[:k_used]).T @ y)
    out = out.reshape(shape)
    return (out, k_used) if return_info else out
