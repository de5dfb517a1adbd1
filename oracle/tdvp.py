"""One-site and two-site TDVP time steps in the mixed canonical gauge.

1TDVP (Sec. II D, Eq. proj1site): a left-to-right sweep evolves each site
tensor forward by dt/2 and each bond matrix backward by dt/2, then the
mirrored right-to-left sweep; the two consecutive forward half steps on the
last site use the same effective Hamiltonian and are merged into one full
step.  The backward term of Eq. proj1site is read as the zero-site bond
evolution of the Lubich/Haegeman splitting, the paper gives only the
projector.

2TDVP (Sec. II D, Eq. proj2site; Sec. III A): pairs evolve forward by dt/2
and single sites backward by dt/2; the right-most pair is evolved once by
the full dt (Sec. III A, turning point).  After each two-site update the
state is split by a truncated SVD (Fig. postupdate) with the truncation
rules of Sec. III C (Eq. discweight) and Sec. III D (relative cut eps).

The state is serial and mixed canonical; the paper's inverse canonical gauge
is the equivalent form used by the segment-parallel schedule.  Norms are not
restored after truncation, so <psi|psi> = 1 - w_total.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .env import right_envs, trivial_env, update_left, update_right
from .heff import apply_heff0, apply_heff1, apply_heff2
from .krylov import expm_krylov
from .mps import lq


@dataclass
class Truncation:
    chi_max: int = 1 << 30
    w_max: float = 0.0
    eps: float = 0.0
    multiplet_guard: bool = True


@dataclass
class Stats:
    w_total: float = 0.0
    matvecs: int = 0
    chi_peak: int = 0
    krylov_max_used: int = 0


def truncation_rank(s: np.ndarray, tr: Truncation):
    """Rank kept from descending singular values s (Sec. III C, Sec. III D).

    chi_w = smallest chi >= 1 whose discarded weight sum_{j>chi} s_j^2 is at
    most w_max; chi_eps = number of s_j >= eps s_1; chi = max(1, min(chi_w,
    chi_max, chi_eps)).  The multiplet guard (the paper is silent on ties)
    lowers chi while s_{chi+1} is within 1e-10 of s_chi.  Returns (chi, w).
    """
    full = len(s)
    s2 = s.astype(np.float64) ** 2
    tail = np.concatenate([np.cumsum(s2[::-1])[::-1], [0.0]])  # tail[c] = sum_{j>=c} s_j^2
    chi_w = full
    for c in range(1, full + 1):
        if tail[c] <= tr.w_max:
            chi_w = c
            break
    chi_eps = int(np.sum(s >= tr.eps * s[0])) if full else 0
    chi = max(1, min(chi_w, tr.chi_max, chi_eps))
    if tr.multiplet_guard:
        while 1 < chi < full and s[chi] >= (1.0 - 1e-10) * s[chi - 1]:
            chi -= 1
    w = float(tail[chi])
    return chi, w


def svd_split(theta: np.ndarray, tr: Truncation):
    """Theta[a, s1, s2, b] -> U[a, s1, c], S[c], Vh[c, s2, b] truncated; returns (U, S, Vh, w)."""
    chil, d1, d2, chir = theta.shape
    U, S, Vh = np.linalg.svd(theta.reshape(chil * d1, d2 * chir), full_matrices=False)
    chi, w = truncation_rank(S, tr)
    return (U[:, :chi].reshape(chil, d1, chi), S[:chi],
            Vh[:chi, :].reshape(chi, d2, chir), w)


class MPSState:
    """MPS + MPO + cached environments, centre at site 1 between steps."""

    def __init__(self, tensors, Ws):
        self.T = [np.array(A, dtype=np.complex128) for A in tensors]
        self.W = Ws
        self.N = len(tensors)
        self.beta = [None] * self.N
        self.beta[0] = trivial_env()
        self.gamma = right_envs(self.T, self.W)  # Sec. III A: built right to left
        self.stats = Stats()

    def _expm(self, apply, x, tau, kmax, tol):
        count = [0]

        def op(v):
            count[0] += 1
            return apply(v)

        out, k = expm_krylov(op, x, tau, kmax=kmax, tol=tol, return_info=True)
        self.stats.matvecs += count[0]
        self.stats.krylov_max_used = max(self.stats.krylov_max_used, k)
        return out

    def h1(self, j):
        b, W, g = self.beta[j], self.W[j], self.gamma[j]
        return lambda x: apply_heff1(b, W, g, x)

    def h0(self, j):
        """Bond between 0-based sites j and j+1."""
        b, g = self.beta[j + 1], self.gamma[j]
        return lambda x: apply_heff0(b, g, x)

    def h2(self, j):
        b, W1, W2, g = self.beta[j], self.W[j], self.W[j + 1], self.gamma[j + 1]
        return lambda x: apply_heff2(b, W1, W2, g, x)


def tdvp1_step(st: MPSState, dt: float, kmax: int = 40, tol: float = 1e-13):
    """One symmetric 1TDVP step of size dt (Eq. proj1site, Lie-Trotter-Suzuki splitting)."""
    T, N, tau = st.T, st.N, dt / 2.0
    for j in range(N - 1):
        T[j] = st._expm(st.h1(j), T[j], tau, kmax, tol)
        chil, d, chir = T[j].shape
        Q, R = np.linalg.qr(T[j].reshape(chil * d, chir))
        T[j] = Q.reshape(chil, d, Q.shape[1])
        st.beta[j + 1] = update_left(st.beta[j], T[j], st.W[j])
        C = st._expm(st.h0(j), R, -tau, kmax, tol)
        T[j + 1] = np.einsum("ab,bsc->asc", C, T[j + 1])
    T[N - 1] = st._expm(st.h1(N - 1), T[N - 1], dt, kmax, tol)  # merged turning point
    for j in range(N - 1, 0, -1):
        chil, d, chir = T[j].shape
        L, Q = lq(T[j].reshape(chil, d * chir))
        T[j] = Q.reshape(Q.shape[0], d, chir)
        st.gamma[j - 1] = update_right(st.gamma[j], T[j], st.W[j])
        C = st._expm(st.h0(j - 1), L, -tau, kmax, tol)
        T[j - 1] = np.einsum("asb,bc->asc", T[j - 1], C)
        T[j - 1] = st._expm(st.h1(j - 1), T[j - 1], tau, kmax, tol)
    st.stats.chi_peak = max(st.stats.chi_peak, max(A.shape[2] for A in T))
    return st


def tdvp2_step(st: MPSState, dt: float, tr: Truncation, kmax: int = 40, tol: float = 1e-13):
    """One symmetric 2TDVP step of size dt (Eq. proj2site; Sec. III A)."""
    T, N, tau = st.T, st.N, dt / 2.0
    for j in range(N - 2):
        theta = np.einsum("asb,btc->astc", T[j], T[j + 1])
        theta = st._expm(st.h2(j), theta, tau, kmax, tol)
        U, S, Vh, w = svd_split(theta, tr)
        st.stats.w_total += w
        T[j] = U
        T[j + 1] = S[:, None, None] * Vh
        st.beta[j + 1] = update_left(st.beta[j], T[j], st.W[j])
        T[j + 1] = st._expm(st.h1(j + 1), T[j + 1], -tau, kmax, tol)
    j = N - 2
    theta = np.einsum("asb,btc->astc", T[j], T[j + 1])
    theta = st._expm(st.h2(j), theta, dt, kmax, tol)  # turning point, full step
    U, S, Vh, w = svd_split(theta, tr)
    st.stats.w_total += w
    T[j] = U * S[None, None, :]
    T[j + 1] = Vh
    st.gamma[j] = update_right(st.gamma[j + 1], T[j + 1], st.W[j + 1])
    for j in range(N - 3, -1, -1):
        T[j + 1] = st._expm(st.h1(j + 1), T[j + 1], -tau, kmax, tol)
        theta = np.einsum("asb,btc->astc", T[j], T[j + 1])
        theta = st._expm(st.h2(j), theta, tau, kmax, tol)
        U, S, Vh, w = svd_split(theta, tr)
        st.stats.w_total += w
        T[j] = U * S[None, None, :]
        T[j + 1] = Vh
        st.gamma[j] = update_right(st.gamma[j + 1], T[j + 1], st.W[j + 1])
    st.stats.chi_peak = max(st.stats.chi_peak, max(A.shape[2] for A in T))
    return st


def chi_saturated(tensors, chi_max: int) -> bool:
    """True when every bond j = 1..N-1 holds min(chi_max, d^min(j, N-j)):
    the bond dimensions can grow no further (Sec. Discussion, hybrid scheme)."""
    N, d = len(tensors), tensors[0].shape[1]
    return all(tensors[j - 1].shape[2] >= min(chi_max, d ** min(j, N - j)) for j in range(1, N))


def hybrid_step(st: MPSState, dt: float, tr: Truncation, kmax: int = 40, tol: float = 1e-13):
    """The hybrid scheme proposed in the paper's Discussion: a two-site step
    while chi_max is not saturated, a one-site step once it is.  Returns
    True when the one-site step ran."""
    if chi_saturated(st.T, tr.chi_max):
        tdvp1_step(st, dt, kmax, tol)
        return True
    tdvp2_step(st, dt, tr, kmax, tol)
    return False


def imaginary_time_step(st: MPSState, dtau: float, tr: Truncation | None = None, kmax: int = 40,
                        tol: float = 1e-13):
    """One imaginary-time step exp(-dtau H) (the paper's Discussion notes that
    p2TDVP applies to imaginary time): the TDVP step with dt = -i dtau, so that
    forward local steps apply exp(-tau H_eff) and backward ones exp(+tau H_eff),
    followed by renormalisation of the centre tensor (the evolution is not
    unitary).  tr = None: one-site step, else two-site with truncation tr."""
    if tr is None:
        tdvp1_step(st, -1j * dtau, kmax, tol)
    else:
        tdvp2_step(st, -1j * dtau, tr, kmax, tol)
    st.T[0] = st.T[0] / np.linalg.norm(st.T[0])
    return st
