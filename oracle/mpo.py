"""Hamiltonian MPOs for long-range spin chains (Sec. II C).

Two constructions:

* ``mpo_exact``: every coupling f(r), r = 1..N-1, gets its own chain of
  bond states (a "shift register").  Arbitrary long range is not compact in
  N (Sec. II C), so the bond dimension is n_H (N-1) + 2; for one term and
  N = 10 this is 11.
* ``mpo_exponentials``: f(r) ~ sum_k c_k lambda_k^r, which the MPO encodes
  with one decaying channel per exponential and term, giving the bond
  dimension m = n_H n_exps + 2 stated in Sec. II C.

Bond state 0 means "nothing placed yet" and m-1 means "term complete".  The
first site keeps row 0 of the bulk tensor and the last site keeps column
m-1.  W[k, l, s', s] with s' the output index.

``fit_exponentials`` approximates samples of f by a sum of exponentials.  The
paper names the method of Pirvu et al. without stating its steps; the
oracle uses the matrix-pencil reading (Hankel matrix of the samples, rank-K
truncated SVD, shift invariance of the right singular vectors, then linear
least squares for the weights).
"""
from __future__ import annotations

import numpy as np



def _boundaries(Wb: np.ndarray, N: int):
    m = Wb.shape[0]
    Ws = []
    for j in range(N):
        if N == 1:
            Ws.append(Wb[0:1, m - 1:m].copy())
        elif j == 0:
            Ws.append(Wb[0:1, :].copy())
        elif j == N - 1:
            Ws.append(Wb[:, m - 1:m].copy())
        else:
            Ws.append(Wb.copy())
    return Ws


def mpo_exact(N: int, f, pairs, onsite=None, h: float = 0.0):
    """Shift-register MPO of sum_{i<j} f(j-i) sum_a g_a A_a(i) B_a(j) + h sum X(i)."""
    nH = len(pairs)
    R = N - 1
    m = nH * R + 2
    d = np.asarray(pairs[0][1]).shape[0]
    I = np.eye(d, dtype=np.complex128)
    Wb = np.zeros((m, m, d, d), dtype=np.complex128)
    Wb[0, 0] = I
    Wb[m - 1, m - 1] = I
    if onsite is not None:
        Wb[0, m - 1] = h * onsite
    for a, (g, A, B) in enumerate(pairs):
        s = lambda r: 1 + a * R + (r - 1)  # state "A_a placed r-1 sites ago"
        Wb[0, s(1)] = A
        for r in range(1, R):
            Wb[s(r), s(r + 1)] = I
        for r in range(1, R + 1):
            fr = f(r) if callable(f) else f[r]
            Wb[s(r), m - 1] = g * fr * B
    return _boundaries(Wb, N)


def mpo_exponentials(N: int, c, lam, pairs, onsite=None, h: float = 0.0):
    """MPO of sum_{i<j} (sum_k c_k lam_k^(j-i)) sum_a g_a A_a(i) B_a(j) + h sum X(i).

    Channel (a, k): A_a opens it, each intermediate site multiplies by
    lam_k, and B_a closes it with weight g_a c_k lam_k, so a pair at
    distance r collects c_k lam_k^r (Sec. II C, sums of exponentials).
    """
    c = np.asarray(c, dtype=np.complex128)
    lam = np.asarray(lam, dtype=np.complex128)
    K = len(c)
    nH = len(pairs)
    m = nH * K + 2
    d = np.asarray(pairs[0][1]).shape[0]
    I = np.eye(d, dtype=np.complex128)
    Wb = np.zeros((m, m, d, d), dtype=np.complex128)
    Wb[0, 0] = I
    Wb[m - 1, m - 1] = I
    if onsite is not None:
        Wb[0, m - 1] = h * onsite
    for a, (g, A, B) in enumerate(pairs):
        for k in range(K):
            s = 1 + a * K + k
            Wb[0, s] = A
            Wb[s, s] = lam[k] * I
            Wb[s, m - 1] = g * c[k] * lam[k] * B
    return _boundaries(Wb, N)


def fit_exponentials(fvals: np.ndarray, K: int):
    """Matrix-pencil fit f(r) ~ sum_k c_k lam_k^r from samples f(1..R).

    Returns (c, lam, max_abs_err) with complex c, lam.  The shift matrix of
    K exponentials is determined only by at least 2K samples; fewer are
    rejected (the pencil would be rank deficient and the fit meaningless).
    """
    f = np.asarray(fvals, dtype=np.float64)
    R = len(f)
    if K < 1 or R < 2 * K:
        raise ValueError("need K >= 1 and at least 2K samples")
    P = R // 2
    Y = np.array([[f[i + j] for j in range(P + 1)] for i in range(R - P)])
    _, _, Vh = np.linalg.svd(Y)
    Vk = Vh[:K, :]
    M = Vk[:, 1:] @ np.linalg.pinv(Vk[:, :-1])
    lam = np.linalg.eigvals(M)
    r = np.arange(1, R + 1)
    Z = lam[None, :] ** r[:, None]
    c, *_ = np.linalg.lstsq(Z, f.astype(np.complex128), rcond=None)
    approx = (Z @ c).real
    return c, lam, float(np.max(np.abs(approx - f)))


def eval_exponentials(c, lam, rmax: int) -> np.ndarray:
    """Array g with g[r] = sum_k c_k lam_k^r (real part), g[0] unused."""
    r = np.arange(0, rmax + 1)
    return (np.asarray(lam)[None, :] ** r[:, None] @ np.asarray(c)).real


def mpo_to_dense(Ws) -> np.ndarray:
    """Contract the MPO into the dense 2^N x 2^N operator (definition, Sec. II C)."""
    O = Ws[0][0]  # [w, d', d]
    for W in Ws[1:]:
        # O[k, P', P] x W[k, l, s', s] -> [l, (P' s'), (P s)]
        Onew = np.einsum("kpq,klst->lpsqt", O, W)
        w = Onew.shape[0]
        D = Onew.shape[1] * Onew.shape[2]
        O = Onew.reshape(w, D, D)
    return O[0]
