"""Matrix product states: construction, canonical forms, dense conversion,
norms, overlaps and expectation values.

An MPS is a Python list of site tensors A[a, s, b] (Eq. mps-no-gauge).  The
mixed canonical form (Eqs. mixed-mps1/2) keeps A_p left-orthonormal
(sum_s A^dag A = 1) left of the centre and B_q right-orthonormal
(sum_s B B^dag = 1) right of it.
"""
from __future__ import annotations

import numpy as np


def to_dense(tensors) -> np.ndarray:
    """psi[s_1 ... s_N] = A_1^{s_1} ... A_N^{s_N} (Eq. mps-no-gauge)."""
    v = tensors[0]  # [1, d, chi]
    v = v.reshape(v.shape[1], v.shape[2])
    for A in tensors[1:]:
        v = np.einsum("pa,asb->psb", v, A).reshape(-1, A.shape[2])
    return v.reshape(-1)


def lq(M: np.ndarray):
    """M = L Q with Q having orthonormal rows (via QR of M^dagger)."""
    Q, R = np.linalg.qr(M.conj().T)
    return R.conj().T, Q.conj().T


def right_canonicalize(tensors):
    """Right-orthonormalise sites N..2 by successive LQ decompositions.

    Returns new tensors with sites 2..N right-orthonormal and the whole
    state (norm included) in site 1, the orthogonality centre.
    """
    T = [A.copy() for A in tensors]
    for j in range(len(T) - 1, 0, -1):
        chil, d, chir = T[j].shape
        L, Q = lq(T[j].reshape(chil, d * chir))
        T[j] = Q.reshape(Q.shape[0], d, chir)
        T[j - 1] = np.einsum("asb,bc->asc", T[j - 1], L)
    return T


def normalize_centre(tensors, centre: int = 0):
    """Scale the centre tensor to unit Frobenius norm."""
    T = list(tensors)
    T[centre] = T[centre] / np.linalg.norm(T[centre])
    return T


def padded_product_state(bits, chi):
    """Right-canonical MPS of |s_1 ... s_N> padded to bond dimensions chi.

    Row 0 of site j carries the product state (entry (s_j, 0)); the other
    rows are the remaining unit vectors e_(s, b) in lexicographic order, which
    keeps every site right-orthonormal.  Requires chi[j-1] <= d chi[j].
    """
    d = 2
    N = len(bits)
    T = []
    for j in range(N):
        chil, chir = chi[j], chi[j + 1]
        assert chil <= d * chir
        B = np.zeros((chil, d, chir), dtype=np.complex128)
        B[0, int(bits[j]), 0] = 1.0
        rows = [(s, b) for s in range(d) for b in range(chir) if (s, b) != (int(bits[j]), 0)]
        for r in range(1, chil):
            s, b = rows[r - 1]
            B[r, s, b] = 1.0
        T.append(B)
    return T


def is_right_orthonormal(B, tol=1e-12) -> bool:
    chil = B.shape[0]
    M = B.reshape(chil, -1)
    return np.allclose(M @ M.conj().T, np.eye(chil), atol=tol)


def is_left_orthonormal(A, tol=1e-12) -> bool:
    chir = A.shape[2]
    M = A.reshape(-1, chir)
    return np.allclose(M.conj().T @ M, np.eye(chir), atol=tol)


# ---------------------------------------------------------------------------
# Transfer-matrix contractions (definitions; used for observables, Sec. IV)
# ---------------------------------------------------------------------------

def _left_step(E, Abra, Aket, O=None):
    """E'[b', b] = sum conj(Abra[a', s', b']) E[a', a] O[s', s] Aket[a, s, b]."""
    if O is None:
        return np.einsum("xy,xsb,ysc->bc", E, Abra.conj(), Aket)
    return np.einsum("xy,xtb,ts,ysc->bc", E, Abra.conj(), O, Aket)


def _right_step(E, Abra, Aket, O=None):
    """E'[a', a] = sum Aket[a, s, b] O[s', s] E[b', b] conj(Abra[a', s', b'])."""
    if O is None:
        return np.einsum("bc,xsb,ysc->xy", E, Abra.conj(), Aket)
    return np.einsum("bc,xtb,ts,ysc->xy", E, Abra.conj(), O, Aket)


def left_transfers(tensors):
    """E_L[j] for j = 0..N: contraction of <psi|psi> over sites 1..j."""
    E = [np.ones((1, 1), dtype=np.complex128)]
    for A in tensors:
        E.append(_left_step(E[-1], A, A))
    return E


def right_transfers(tensors):
    """E_R[j] for j = 1..N+1 (index j-1 in the list): sites j..N."""
    N = len(tensors)
    E = [None] * (N + 1)
    E[N] = np.ones((1, 1), dtype=np.complex128)
    for j in range(N - 1, -1, -1):
        E[j] = _right_step(E[j + 1], tensors[j], tensors[j])
    return E


def norm2(tensors) -> float:
    return float(left_transfers(tensors)[-1][0, 0].real)


def overlap(bra, ket) -> complex:
    """<bra|ket> by a left-to-right transfer contraction."""
    E = np.ones((1, 1), dtype=np.complex128)
    for A, B in zip(bra, ket):
        E = _left_step(E, A, B)
    return complex(E[0, 0])


def infidelity(psi1, psi2) -> float:
    """I = 1 - |<psi1|psi2>| / sqrt(<psi1|psi1><psi2|psi2>) (Sec. IV, modulus not squared)."""
    num = abs(overlap(psi1, psi2))
    den = np.sqrt(overlap(psi1, psi1).real * overlap(psi2, psi2).real)
    return float(1.0 - num / den)


def expect_sites(tensors, O) -> np.ndarray:
    """<psi|O_i|psi>/<psi|psi> for every site i = 1..N."""
    EL = left_transfers(tensors)
    ER = right_transfers(tensors)
    n2 = EL[-1][0, 0].real
    out = np.empty(len(tensors), dtype=np.complex128)
    for i, A in enumerate(tensors):
        E = _left_step(EL[i], A, A, O)
        out[i] = np.sum(E * ER[i + 1]) / n2
    return out


def expect_two_point(tensors, i: int, j: int, Oi, Oj) -> complex:
    """<psi|Oi(i) Oj(j)|psi>/<psi|psi>, sites 1-based (equal-time correlator, Eq. IsingCorrelation)."""
    if i > j:
        i, j, Oi, Oj = j, i, Oj, Oi
    EL = left_transfers(tensors)
    ER = right_transfers(tensors)
    n2 = EL[-1][0, 0].real
    if i == j:
        E = _left_step(EL[i - 1], tensors[i - 1], tensors[i - 1], Oi @ Oj)
        return complex(np.sum(E * ER[i]) / n2)
    E = _left_step(EL[i - 1], tensors[i - 1], tensors[i - 1], Oi)
    for q in range(i, j - 1):
        E = _left_step(E, tensors[q], tensors[q])
    E = _left_step(E, tensors[j - 1], tensors[j - 1], Oj)
    return complex(np.sum(E * ER[j]) / n2)


def mpo_expectation(tensors, Ws) -> complex:
    """<psi|H|psi>/<psi|psi> with H given as an MPO."""
    E = np.ones((1, 1, 1), dtype=np.complex128)  # [a', k, a]
    for A, W in zip(tensors, Ws):
        E = np.einsum("xky,xtb,klts,ysc->blc", E, A.conj(), W, A)
    return complex(E[0, 0, 0] / norm2(tensors))


def move_centre_right(tensors, upto: int):
    """Left-orthonormalise sites 1..upto by QR, pushing the centre to site upto+1.

    Assumes the centre starts at site 1 (0-based index 0).
    """
    T = [A.copy() for A in tensors]
    for j in range(upto):
        chil, d, chir = T[j].shape
        Q, R = np.linalg.qr(T[j].reshape(chil * d, chir))
        T[j] = Q.reshape(chil, d, Q.shape[1])
        T[j + 1] = np.einsum("ab,bsc->asc", R, T[j + 1])
    return T


def left_block_states(tensors, j: int) -> np.ndarray:
    """Phi_L[(s_1..s_j), a] for the first j sites (dense, small N only)."""
    v = np.ones((1, 1), dtype=np.complex128)
    for A in tensors[:j]:
        v = np.einsum("pa,asb->psb", v, A).reshape(-1, A.shape[2])
    return v


def right_block_states(tensors, j: int) -> np.ndarray:
    """Phi_R[b, (s_{j+1}..s_N)] for sites j+1..N (dense, small N only)."""
    v = np.ones((1, 1), dtype=np.complex128)
    for A in reversed(tensors[j:]):
        v = np.einsum("asb,bq->asq", A, v).reshape(A.shape[0], -1)
    return v
