"""Pins of the oracle's forward-mode gradient (oracle/grad.py).

Comparison objects: scipy's Frechet derivative of the matrix exponential,
central differences of numpy's QR, the Daleckii-Krein derivative of exact
evolution (one-site TDVP is exact at full bond dimension, Sec. II D), and
central differences of the forward oracle under truncated bond dimensions.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import grad, mpo, mps, spin, tdvp


def _herm(rng, n):
    G = wl.cgauss(rng, (n, n))
    return (G + G.conj().T) / 2


def test_expm_tangent_equals_frechet_derivative():
    rng = np.random.default_rng(5)
    n = 24
    H, dH = _herm(rng, n), _herm(rng, n)
    x, dx = wl.cgauss(rng, (n,)), wl.cgauss(rng, (n,))
    for tau in (0.3, -0.05, 1.7):
        y, dy = grad.expm_jvp(lambda v: H @ v, lambda v: dH @ v, x, dx, tau)
        E, F = sla.expm_frechet(-1j * tau * H, -1j * tau * dH)
        assert np.linalg.norm(y - E @ x) < 1e-12 * np.linalg.norm(x)
        assert np.linalg.norm(dy - (E @ dx + F @ x)) < 1e-11 * (np.linalg.norm(x) + np.linalg.norm(dx))
    # zero state and zero tangent
    y, dy = grad.expm_jvp(lambda v: H @ v, lambda v: dH @ v, np.zeros(n, complex), np.zeros(n, complex), 0.1)
    assert not np.any(y) and not np.any(dy)


@pytest.mark.parametrize("shape", [(12, 5), (8, 8)])
def test_qr_and_lq_tangents_equal_differences(shape):
    rng = np.random.default_rng(7)
    M, dM = wl.cgauss(rng, shape), wl.cgauss(rng, shape)
    eps = 1e-6
    Q, R, dQ, dR = grad.qr_jvp(M, dM)
    Qp, Rp = np.linalg.qr(M + eps * dM)
    Qm, Rm = np.linalg.qr(M - eps * dM)
    assert np.allclose(Q @ R, M, atol=1e-13)
    assert np.max(np.abs(dQ - (Qp - Qm) / (2 * eps))) < 1e-8
    assert np.max(np.abs(dR - (Rp - Rm) / (2 * eps))) < 1e-8
    L, Qr, dL, dQr = grad.lq_jvp(M.T.copy(), dM.T.copy())
    Lp, Qrp = mps.lq(M.T + eps * dM.T)
    Lm, Qrm = mps.lq(M.T - eps * dM.T)
    assert np.max(np.abs(dL - (Lp - Lm) / (2 * eps))) < 1e-8
    assert np.max(np.abs(dQr - (Qrp - Qrm) / (2 * eps))) < 1e-8


def _ising(N, h):
    c, lam, _ = mpo.fit_exponentials(1.0 / np.arange(1, 17) ** 2.0, 3)
    bulk = mpo.mpo_exponentials(4, c, lam, spin.ising_pairs(), spin.SX, h)[1]
    return c, lam, bulk


def _directions(c, lam):
    """MPO bulk directions: the coupling J, the field h, an on-site sigma^y
    field and a sigma^x admixture to the operator that opens each channel."""
    K = len(c)
    m = K + 2
    z = lambda: np.zeros((m, m, 2, 2), dtype=np.complex128)
    dJ, dh, dy, dA = z(), z(), z(), z()
    for k in range(K):
        dJ[1 + k, m - 1] = c[k] * lam[k] * spin.SZ
        dA[0, 1 + k] = spin.SX
    dh[0, m - 1] = spin.SX
    dy[0, m - 1] = spin.SY
    return {"J": dJ, "h": dh, "onsite_y": dy, "open_x": dA}


def _dense_tangent(bulk, dbulk, N):
    """dH of the MPO contraction along dbulk at every site (product rule of the
    multilinear contraction, Sec. II C)."""
    Ws = mpo._boundaries(bulk, N)
    dWs = mpo._boundaries(dbulk, N)
    return sum(mpo.mpo_to_dense([dWs[i] if i == j else Ws[i] for i in range(N)]) for j in range(N))


def test_jvp_full_rank_equals_daleckii_krein():
    N, dt, steps, site, h = 6, 0.05, 4, 2, 0.7
    c, lam, bulk = _ising(N, h)
    T0 = mps.normalize_centre(mps.right_canonicalize(wl.random_site_tensors(6, wl.full_rank_bonds(N, 2), 2)))
    psi0 = mps.to_dense(T0)
    Ws = mpo._boundaries(bulk, N)
    H = mpo.mpo_to_dense(Ws)
    g = mpo.eval_exponentials(c, lam, N - 1)
    assert np.max(np.abs(H - spin.longrange_hamiltonian(N, g, spin.ising_pairs(), spin.SX, h))) < 1e-12
    Z = spin.site_op(spin.SZ, site + 1, N).toarray()
    dense_dirs = {"J": spin.longrange_hamiltonian(N, g, spin.ising_pairs()),
                  "h": spin.longrange_hamiltonian(N, g, [], spin.SX, 1.0)}
    for name, V in _directions(c, lam).items():
        dH = _dense_tangent(bulk, V, N)
        if name in dense_dirs:  # the product rule agrees with the Kronecker-built derivative
            assert np.max(np.abs(dH - dense_dirs[name])) < 1e-12
        assert np.max(np.abs(dH - dH.conj().T)) < 1e-12
        val_ed, d_ed = grad.exact_gradient(H, dH, psi0, dt * steps, Z)
        val, d = grad.loss_jvp(T0, Ws, mpo._boundaries(V, N), dt, steps, site, spin.SZ)
        assert abs(val - val_ed) < 1e-10
        assert abs(d - d_ed) < 1e-8 * max(1.0, abs(d_ed)), (name, d, d_ed)


def test_jvp_truncated_equals_central_differences():
    N, dt, steps, site = 8, 0.05, 3, 3
    c, lam, bulk = _ising(N, 1.0)
    T0 = mps.normalize_centre(mps.right_canonicalize(wl.random_site_tensors(32, wl.full_rank_bonds(N, 2, 4), 2)))

    def forward(b):
        st = tdvp.MPSState(T0, mpo._boundaries(b, N))
        for _ in range(steps):
            tdvp.tdvp1_step(st, dt)
        return float(mps.expect_sites(st.T, spin.SZ)[site].real)

    eps = 1e-4
    for name, V in _directions(c, lam).items():
        val, d = grad.loss_jvp(T0, mpo._boundaries(bulk, N), mpo._boundaries(V, N), dt, steps, site, spin.SZ)
        fd = (forward(bulk + eps * V) - forward(bulk - eps * V)) / (2 * eps)
        assert abs(val - forward(bulk)) < 1e-12
        assert abs(d - fd) < 1e-9 * max(1.0, abs(fd)), (name, d, fd)
