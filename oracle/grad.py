"""Forward-mode derivative (JVP) of one-site TDVP time steps with respect to
the MPO, and of a site expectation value of the evolved state.

Reference gradient for the differentiable one-site TDVP (Sec. II D,
Eq. proj1site; the paper itself differentiates nothing).  A direction dW of
the MPO tensors is carried through every operation of ``tdvp.tdvp1_step`` in
the same order, each tangent taken from the definition of the operation:

* environments (Sec. III A, Fig. environments) and the effective
  Hamiltonians (Fig. update) are multilinear in their factors, so their
  tangents are sums of the same contraction with one factor replaced by its
  tangent (the conjugated site tensor of the bra included);
* the Krylov exponential exp(-i tau H_eff) x is replaced by the exact
  exponential of the block operator [[X, E], [0, X]] with X = -i tau H_eff and
  E = -i tau dH_eff, whose action on [dx; x] is [d(e^X x); e^X x] (the
  Frechet derivative of the exponential as the off-diagonal block), evaluated
  by Arnoldi on the 2n-dimensional operator with the small Hessenberg
  exponential taken by scipy's expm;
* the QR gauge move M = QR (R with a real diagonal, as LAPACK returns it):
  with C = Q^H dM R^-1, U upper triangular with U_ij = C_ij + conj(C_ji) for
  i < j and U_ii = Re C_ii, the tangents are dR = U R and
  dQ = Q (C - U) + (I - Q Q^H) dM R^-1; the LQ move uses the QR of M^H.

Pins (tests/test_oracle_grad.py): at full bond dimension one-site TDVP is
exact, so the JVP of <sigma^z_i(t)> equals the exact-diagonalisation
derivative from the Daleckii-Krein formula in H's eigenbasis; under
truncated bond dimensions it equals central finite differences of the
forward oracle; the exponential tangent equals the Frechet derivative from
scipy's expm_frechet and the QR tangent equals differences of numpy's QR.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .env import right_envs, trivial_env, update_left, update_right
from .heff import EINSUM_PATH, apply_heff0, apply_heff1


# ------------------------------------------------------------- tangents of the pieces

def left_env_jvp(beta, dbeta, A, dA, W, dW):
    """beta' and its tangent; beta'[b',l,b] = sum conj(A[a',s',b']) beta[a',k,a] W[k,l,s',s] A[a,s,b]."""
    e = lambda b, Ab, w, Ak: np.einsum("xky,xtb,klts,ysc->blc", b, np.conj(Ab), w, Ak, optimize=EINSUM_PATH)
    out = update_left(beta, A, W)
    d = e(dbeta, A, W, A) + e(beta, dA, W, A) + e(beta, A, dW, A) + e(beta, A, W, dA)
    return out, d


def right_env_jvp(gamma, dgamma, B, dB, W, dW):
    """gamma' and its tangent; gamma'[a',k,a] = sum B[a,s,b] W[k,l,s',s] gamma[b',l,b] conj(B[a',s',b'])."""
    e = lambda g, Bk, w, Bb: np.einsum("ysc,klts,blc,xtb->xky", Bk, w, g, np.conj(Bb), optimize=EINSUM_PATH)
    out = update_right(gamma, B, W)
    d = e(dgamma, B, W, B) + e(gamma, dB, W, B) + e(gamma, B, dW, B) + e(gamma, B, W, dB)
    return out, d


def qr_jvp(M, dM):
    """Reduced QR M = Q R (m >= n, full column rank, real diagonal of R) and its tangent."""
    Q, R = np.linalg.qr(M)
    Rinv = np.linalg.inv(R)
    C = Q.conj().T @ dM @ Rinv
    n = R.shape[0]
    U = np.zeros_like(C)
    for i in range(n):
        U[i, i] = C[i, i].real
        for j in range(i + 1, n):
            U[i, j] = C[i, j] + np.conj(C[j, i])
    dR = U @ R
    dQ = Q @ (C - U) + (dM @ Rinv - Q @ (Q.conj().T @ dM @ Rinv))
    return Q, R, dQ, dR


def lq_jvp(M, dM):
    """M = L Q with orthonormal rows of Q (through the QR of M^H) and its tangent."""
    Qh, Rh, dQh, dRh = qr_jvp(M.conj().T, dM.conj().T)
    return Rh.conj().T, Qh.conj().T, dRh.conj().T, dQh.conj().T


def expm_jvp(apply, dapply, x, dx, tau, kmax: int = 80, tol: float = 1e-13):
    """(exp(-i tau H) x, its tangent) for H = apply (Hermitian) moving along dapply = dH.

    Arnoldi on B[u; v] = [X u + E v; X v], X = -i tau H, E = -i tau dH, from the
    start vector [dx; x]; the k x k Hessenberg exponential is scipy's expm and the
    iteration stops when h_{k+1,k} |e_k^T exp(H_k) e_1| <= tol (relative to the
    start vector) or on a happy breakdown.
    """
    shape = x.shape
    n = x.size

    def op(z):
        u = z[:n].reshape(shape)
        v = z[n:].reshape(shape)
        top = -1j * tau * (apply(u) + dapply(v))
        bot = -1j * tau * apply(v)
        return np.concatenate([top.reshape(-1), bot.reshape(-1)])

    z0 = np.concatenate([np.asarray(dx, dtype=np.complex128).reshape(-1),
                         np.asarray(x, dtype=np.complex128).reshape(-1)])
    b0 = np.linalg.norm(z0)
    if b0 == 0.0:
        return np.zeros(shape, dtype=np.complex128), np.zeros(shape, dtype=np.complex128)
    V = [z0 / b0]
    Hs = np.zeros((kmax + 1, kmax), dtype=np.complex128)
    y = None
    k_used = 0
    for k in range(kmax):
        w = op(V[k])
        for _ in range(2):  # classical Gram-Schmidt against the whole basis, twice
            Vm = np.array(V)
            c = Vm.conj() @ w
            Hs[: k + 1, k] += c
            w = w - Vm.T @ c
        h = np.linalg.norm(w)
        Hs[k + 1, k] = h
        E = sla.expm(Hs[: k + 1, : k + 1])
        y = E[:, 0]
        k_used = k + 1
        scale = np.max(np.abs(Hs[: k + 2, : k + 1]))
        if h * abs(y[-1]) <= tol or h <= 1e-14 * scale or scale == 0.0:
            break
        V.append(w / h)
    z = b0 * (np.array(V[:k_used]).T @ y)
    return z[n:].reshape(shape), z[:n].reshape(shape)


# ------------------------------------------------------------------ the TDVP step

class JVPState:
    """MPS tensors, MPO tensors, environments and the tangents of all of them
    along one MPO direction dWs (state tangents start at zero)."""

    def __init__(self, tensors, Ws, dWs):
        self.T = [np.array(A, dtype=np.complex128) for A in tensors]
        self.dT = [np.zeros_like(A) for A in self.T]
        self.W = [np.asarray(W, dtype=np.complex128) for W in Ws]
        self.dW = [np.asarray(W, dtype=np.complex128) for W in dWs]
        self.N = len(self.T)
        self.beta = [None] * self.N
        self.dbeta = [None] * self.N
        self.beta[0] = trivial_env()
        self.dbeta[0] = np.zeros_like(self.beta[0])
        self.gamma = [None] * self.N
        self.dgamma = [None] * self.N
        self.gamma[self.N - 1] = trivial_env()
        self.dgamma[self.N - 1] = np.zeros_like(self.gamma[self.N - 1])
        for j in range(self.N - 1, 0, -1):  # right environments, built right to left (Sec. III A)
            self.gamma[j - 1], self.dgamma[j - 1] = right_env_jvp(
                self.gamma[j], self.dgamma[j], self.T[j], self.dT[j], self.W[j], self.dW[j])
        assert all(np.allclose(g, r) for g, r in zip(self.gamma, right_envs(self.T, self.W)))

    def site(self, j):
        b, db, W, dW, g, dg = self.beta[j], self.dbeta[j], self.W[j], self.dW[j], self.gamma[j], self.dgamma[j]
        h = lambda v: apply_heff1(b, W, g, v)
        dh = lambda v: apply_heff1(db, W, g, v) + apply_heff1(b, dW, g, v) + apply_heff1(b, W, dg, v)
        return h, dh

    def bond(self, j):
        """Bond between 0-based sites j and j+1."""
        b, db, g, dg = self.beta[j + 1], self.dbeta[j + 1], self.gamma[j], self.dgamma[j]
        h = lambda v: apply_heff0(b, g, v)
        dh = lambda v: apply_heff0(db, g, v) + apply_heff0(b, dg, v)
        return h, dh


def tdvp1_step_jvp(st: JVPState, dt: float, kmax: int = 80, tol: float = 1e-13):
    """One symmetric 1TDVP step (the order of ``tdvp.tdvp1_step``) with tangents."""
    T, dT, N, tau = st.T, st.dT, st.N, dt / 2.0
    for j in range(N - 1):
        T[j], dT[j] = expm_jvp(*st.site(j), T[j], dT[j], tau, kmax, tol)
        chil, d, chir = T[j].shape
        Q, R, dQ, dR = qr_jvp(T[j].reshape(chil * d, chir), dT[j].reshape(chil * d, chir))
        T[j], dT[j] = Q.reshape(chil, d, chir), dQ.reshape(chil, d, chir)
        st.beta[j + 1], st.dbeta[j + 1] = left_env_jvp(st.beta[j], st.dbeta[j], T[j], dT[j], st.W[j], st.dW[j])
        C, dC = expm_jvp(*st.bond(j), R, dR, -tau, kmax, tol)
        T[j + 1], dT[j + 1] = (np.einsum("ab,bsc->asc", C, T[j + 1]),
                               np.einsum("ab,bsc->asc", dC, T[j + 1]) + np.einsum("ab,bsc->asc", C, dT[j + 1]))
    T[N - 1], dT[N - 1] = expm_jvp(*st.site(N - 1), T[N - 1], dT[N - 1], dt, kmax, tol)  # merged turning point
    for j in range(N - 1, 0, -1):
        chil, d, chir = T[j].shape
        L, Q, dL, dQ = lq_jvp(T[j].reshape(chil, d * chir), dT[j].reshape(chil, d * chir))
        T[j], dT[j] = Q.reshape(chil, d, chir), dQ.reshape(chil, d, chir)
        st.gamma[j - 1], st.dgamma[j - 1] = right_env_jvp(st.gamma[j], st.dgamma[j], T[j], dT[j], st.W[j], st.dW[j])
        C, dC = expm_jvp(*st.bond(j - 1), L, dL, -tau, kmax, tol)
        T[j - 1], dT[j - 1] = (np.einsum("asb,bc->asc", T[j - 1], C),
                               np.einsum("asb,bc->asc", dT[j - 1], C) + np.einsum("asb,bc->asc", T[j - 1], dC))
        T[j - 1], dT[j - 1] = expm_jvp(*st.site(j - 1), T[j - 1], dT[j - 1], tau, kmax, tol)
    return st


def _transfer(E, Abra, Aket, O=None):
    """E'[b', b] = sum conj(Abra[a', s', b']) E[a', a] O[s', s] Aket[a, s, b] (O = identity if None)."""
    if O is None:
        return np.einsum("xy,xsb,ysc->bc", E, np.conj(Abra), Aket, optimize=EINSUM_PATH)
    return np.einsum("xy,xtb,ts,ysc->bc", E, np.conj(Abra), O, Aket, optimize=EINSUM_PATH)


def expect_site_jvp(T, dT, site: int, O):
    """(<psi|O_site|psi>/<psi|psi>, its tangent) for 0-based ``site`` by transfer contractions."""
    E = np.ones((1, 1), dtype=np.complex128)
    dE = np.zeros_like(E)
    num = dnum = None
    for j, (A, dA) in enumerate(zip(T, dT)):
        Oj = O if j == site else None
        if num is not None or Oj is not None:
            src, dsrc = (E, dE) if Oj is not None else (num, dnum)
            num, dnum = (_transfer(src, A, A, Oj),
                         _transfer(dsrc, A, A, Oj) + _transfer(src, dA, A, Oj) + _transfer(src, A, dA, Oj))
        E, dE = (_transfer(E, A, A),
                 _transfer(dE, A, A) + _transfer(E, dA, A) + _transfer(E, A, dA))
    n, dn, e, de = num[0, 0], dnum[0, 0], E[0, 0], dE[0, 0]
    return float((n / e).real), float(((dn * e - n * de) / e ** 2).real)


def loss_jvp(T0, Ws, dWs, dt: float, steps: int, site: int, O, kmax: int = 80, tol: float = 1e-13,
             progress=None, every_step: bool = False):
    """<O_site> after ``steps`` one-site TDVP steps from T0 under Ws, and its
    derivative along the MPO direction dWs (0-based site).  With ``every_step``
    the list of (value, derivative) after each step is returned."""
    st = JVPState(T0, Ws, dWs)
    hist = []
    for s in range(steps):
        tdvp1_step_jvp(st, dt, kmax, tol)
        if every_step:
            hist.append(expect_site_jvp(st.T, st.dT, site, O))
        if progress is not None:
            progress(s + 1)
    return hist if every_step else expect_site_jvp(st.T, st.dT, site, O)


def exact_gradient(H, dH, psi0, t: float, Obs):
    """d/dx <psi0| e^{iHt} Obs e^{-iHt} |psi0> along dH (dense, small N).

    Daleckii-Krein: with H = V diag(l) V^H, the derivative of e^{-iHt} along dH
    is V (G o (V^H dH V)) V^H with G_ij = (e^{-i l_i t} - e^{-i l_j t})/(l_i - l_j)
    for l_i != l_j and -i t e^{-i l_i t} on (near) coincident eigenvalues.
    """
    lam, V = np.linalg.eigh(H)
    f = np.exp(-1j * t * lam)
    dl = lam[:, None] - lam[None, :]
    close = np.abs(dl) < 1e-9
    G = np.where(close, -1j * t * f[:, None], (f[:, None] - f[None, :]) / np.where(close, 1.0, dl))
    dU = V @ (G * (V.conj().T @ dH @ V)) @ V.conj().T
    psi = V @ (f * (V.conj().T @ psi0))
    dpsi = dU @ psi0
    val = np.vdot(psi, Obs @ psi).real
    return float(val), float(2.0 * np.vdot(psi, Obs @ dpsi).real)
