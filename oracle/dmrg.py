"""Two-site DMRG sweeps for the ground state (test infrastructure: only the
tests, the package smoke check and the benchmark's CPU baseline use the
oracle).

The quench experiments of Sec. IV start from ground states computed with
two-site DMRG; Sec. III A notes that the effective environments of TDVP are
those of DMRG and that a 2TDVP step costs as much as a two-site DMRG sweep.
The sweep here follows the two-site TDVP step of `oracle.tdvp` with every
forward evolution replaced by the lowest eigenvector of the two-site
effective Hamiltonian and no backward one-site steps: a left-to-right pass,
the right-most pair once at the turn, then a right-to-left pass; each
updated pair is split by the truncated SVD of Sec. III C / III D.  The local
eigenproblem is solved with scipy's Lanczos (ARPACK) at tolerance 1e-14, or
densely for local spaces of fewer than 32 states.  The state is renormalised
at the end of the sweep.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as sla

from .env import update_left, update_right
from .tdvp import MPSState, Truncation, svd_split


def lowest_eigenvector(apply, theta: np.ndarray):
    """(E0, v0) of the Hermitian map `apply` on the space of theta's shape."""
    shape, n = theta.shape, theta.size
    if n < 32:
        H = np.stack([apply(e.reshape(shape)).reshape(n) for e in np.eye(n, dtype=np.complex128)], axis=1)
        w, V = np.linalg.eigh((H + H.conj().T) / 2)
        return float(w[0]), V[:, 0].reshape(shape)
    op = sla.LinearOperator((n, n), matvec=lambda v: apply(v.reshape(shape)).reshape(n), dtype=np.complex128)
    w, V = sla.eigsh(op, k=1, which="SA", v0=theta.reshape(n), tol=1e-14)
    return float(w[0]), V[:, 0].reshape(shape)


def dmrg2_sweep(st: MPSState, tr: Truncation) -> float:
    """One sweep; returns the last local ground-state energy."""
    T, N = st.T, st.N
    e = 0.0
    for j in range(N - 2):
        theta = np.einsum("asb,btc->astc", T[j], T[j + 1])
        e, theta = lowest_eigenvector(st.h2(j), theta)
        U, S, Vh, w = svd_split(theta, tr)
        st.stats.w_total += w
        T[j] = U
        T[j + 1] = S[:, None, None] * Vh
        st.beta[j + 1] = update_left(st.beta[j], T[j], st.W[j])
    j = N - 2
    theta = np.einsum("asb,btc->astc", T[j], T[j + 1])
    e, theta = lowest_eigenvector(st.h2(j), theta)
    U, S, Vh, w = svd_split(theta, tr)
    st.stats.w_total += w
    T[j] = U * S[None, None, :]
    T[j + 1] = Vh
    st.gamma[j] = update_right(st.gamma[j + 1], T[j + 1], st.W[j + 1])
    for j in range(N - 3, -1, -1):
        theta = np.einsum("asb,btc->astc", T[j], T[j + 1])
        e, theta = lowest_eigenvector(st.h2(j), theta)
        U, S, Vh, w = svd_split(theta, tr)
        st.stats.w_total += w
        T[j] = U * S[None, None, :]
        T[j + 1] = Vh
        st.gamma[j] = update_right(st.gamma[j + 1], T[j + 1], st.W[j + 1])
    T[0] = T[0] / np.linalg.norm(T[0])
    return e
