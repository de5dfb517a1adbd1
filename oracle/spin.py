"""Dense spin-chain operators and exact diagonalisation (small N only).

Basis order |s_1 s_2 ... s_N> with site 1 the most significant factor of
every Kronecker product; |up> is basis index 0, so sigma^z|up> = +|up>.
Hamiltonians follow Sec. IV: long-range Ising (Eq. IsingHamiltonian, written
here with the signs of the workload: + J r^-alpha zz + h x), XY
(Eq. xyHamiltonian) and XXX (Eq. HaldaneHamiltonian).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
ID2 = np.eye(2, dtype=np.complex128)


def site_op(op: np.ndarray, i: int, N: int) -> sp.csr_matrix:
    """op acting on site i (1-based) of an N-site chain, identity elsewhere."""
    d = op.shape[0]
    left = sp.identity(d ** (i - 1), dtype=np.complex128, format="csr")
    right = sp.identity(d ** (N - i), dtype=np.complex128, format="csr")
    return sp.kron(sp.kron(left, sp.csr_matrix(op)), right, format="csr")


def longrange_hamiltonian(N: int, f, pairs, onsite=None, h: float = 0.0) -> np.ndarray:
    """Dense H = sum_{i<j} f(j-i) sum_a g_a A_a(i) B_a(j) + h sum_i X(i).

    ``pairs`` is a list of (g_a, A_a, B_a); ``f`` maps r = 1..N-1 to the
    coupling (a callable or an array indexed by r).  Built by Kronecker
    products, independently of any MPO.
    """
    d = np.asarray(pairs[0][1]).shape[0] if pairs else np.asarray(onsite).shape[0]
    dim = d ** N
    H = sp.csr_matrix((dim, dim), dtype=np.complex128)
    ops_cache = {}

    def get(op_id, op, i):
        key = (op_id, i)
        if key not in ops_cache:
            ops_cache[key] = site_op(op, i, N)
        return ops_cache[key]

    for i in range(1, N + 1):
        for j in range(i + 1, N + 1):
            r = j - i
            fr = f(r) if callable(f) else f[r]
            for a, (g, A, B) in enumerate(pairs):
                H = H + (g * fr) * (get(("A", a), A, i) @ get(("B", a), B, j))
    if onsite is not None and h != 0.0:
        for i in range(1, N + 1):
            H = H + h * get(("X", 0), onsite, i)
    return H.toarray()


def ising_pairs():
    return [(1.0, SZ, SZ)]


def xy_pairs():
    """The 1/2 (xx + yy) of Eq. (xyHamiltonian)."""
    return [(0.5, SX, SX), (0.5, SY, SY)]


def xxx_pairs():
    """The 1/4 (xx + yy + zz) of Eq. (HaldaneHamiltonian)."""
    return [(0.25, SX, SX), (0.25, SY, SY), (0.25, SZ, SZ)]


def product_state(bits) -> np.ndarray:
    """Dense |s_1 ... s_N> with bit 0 = up, 1 = down."""
    N = len(bits)
    idx = 0
    for b in bits:
        idx = 2 * idx + int(b)
    psi = np.zeros(2 ** N, dtype=np.complex128)
    psi[idx] = 1.0
    return psi


class ExactEvolution:
    """e^{-iHt} psi0 by full eigendecomposition of the dense Hamiltonian."""

    def __init__(self, H: np.ndarray):
        self.evals, self.evecs = sla.eigh(H)

    def evolve(self, psi0: np.ndarray, t: float) -> np.ndarray:
        c = self.evecs.conj().T @ psi0
        return self.evecs @ (np.exp(-1j * self.evals * t) * c)


def expval(psi: np.ndarray, O) -> complex:
    """<psi|O|psi> / <psi|psi> for a dense or sparse operator."""
    return np.vdot(psi, O @ psi) / np.vdot(psi, psi)
