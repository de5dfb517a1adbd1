"""Effective environments beta_j and gamma_j (Sec. III A, Fig. environments).

beta_j[a', k, a] contracts sites 1..j-1 of <psi|H|psi> with the MPO bond
left open; gamma_j[b', l, b] contracts sites j+1..N.  beta_1 and gamma_N are
the trivial 1x1x1 identity.  Environments are updated one site at a time
from the cached neighbour rather than rebuilt (Sec. III A).
"""
from __future__ import annotations

import numpy as np

from .heff import EINSUM_PATH


def trivial_env() -> np.ndarray:
    return np.ones((1, 1, 1), dtype=np.complex128)


def update_left(beta: np.ndarray, A: np.ndarray, W: np.ndarray) -> np.ndarray:
    """beta_{j+1}[b', l, b] = sum conj(A[a', s', b']) beta_j[a', k, a] W[k, l, s', s] A[a, s, b]."""
    return np.einsum("xky,xtb,klts,ysc->blc", beta, A.conj(), W, A, optimize=EINSUM_PATH)


def update_right(gamma: np.ndarray, B: np.ndarray, W: np.ndarray) -> np.ndarray:
    """gamma_{j-1}[a', k, a] = sum B[a, s, b] W[k, l, s', s] gamma_j[b', l, b] conj(B[a', s', b'])."""
    return np.einsum("ysc,klts,blc,xtb->xky", B, W, gamma, B.conj(), optimize=EINSUM_PATH)


def right_envs(tensors, Ws):
    """gamma_1 .. gamma_N built right to left at the start of a run (Sec. III A)."""
    N = len(tensors)
    gam = [None] * N
    gam[N - 1] = trivial_env()
    for j in range(N - 1, 0, -1):
        gam[j - 1] = update_right(gam[j], tensors[j], Ws[j])
    return gam


def left_envs(tensors, Ws):
    """beta_1 .. beta_N built left to right."""
    N = len(tensors)
    bet = [None] * N
    bet[0] = trivial_env()
    for j in range(0, N - 1):
        bet[j + 1] = update_left(bet[j], tensors[j], Ws[j])
    return bet
