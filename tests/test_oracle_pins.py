"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the definition, closed form or invariant it checks.  None of
them re-types the oracle's own formula: the comparison object is a dense
Kronecker-product Hamiltonian, exact diagonalisation, scipy's expm, the
Eckart-Young theorem, or a closed-form value.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import env, heff, krylov, mpo, mps, spin, tdvp


def ising_n10():
    p = wl.ISING_N10
    N, J, h, alpha = p["N"], p["J"], p["h"], p["alpha"]
    f = lambda r: J / r ** alpha
    Ws = mpo.mpo_exact(N, f, spin.ising_pairs(), spin.SX, h)
    H = spin.longrange_hamiltonian(N, f, spin.ising_pairs(), spin.SX, h)
    return N, Ws, H


def random_canonical(N, seed, cap=None):
    chi = wl.full_rank_bonds(N, 2, cap)
    T = mps.right_canonicalize(wl.random_site_tensors(seed, chi, 2))
    return mps.normalize_centre(T)


def fitted_xxx(N, K):
    fvals = np.array([1.0 / r ** 2 for r in range(1, N)])
    c, lam, _ = mpo.fit_exponentials(fvals, K)
    return c, lam, mpo.eval_exponentials(c, lam, N - 1)


# --------------------------------------------------------------- MPO (Sec. II C)

def test_exact_mpo_equals_kronecker_hamiltonian():
    N, Ws, H = ising_n10()
    assert Ws[1].shape[0] == N + 1  # shift-register bond dimension
    assert np.max(np.abs(mpo.mpo_to_dense(Ws) - H)) < 1e-13


@pytest.mark.parametrize("pairs,K", [(spin.xy_pairs, 2), (spin.xxx_pairs, 3)])
def test_exponential_mpo_equals_kronecker_hamiltonian(pairs, K):
    N = 7
    c, lam, g = fitted_xxx(N, K)
    Ws = mpo.mpo_exponentials(N, c, lam, pairs(), spin.SX, 0.3)
    assert Ws[1].shape[0] == len(pairs()) * K + 2  # m = n_H n_exps + 2
    H = spin.longrange_hamiltonian(N, g, pairs(), spin.SX, 0.3)
    assert np.max(np.abs(mpo.mpo_to_dense(Ws) - H)) < 1e-13
    assert np.max(np.abs(H - H.conj().T)) < 1e-13


def test_fit_recovers_exact_exponentials():
    r = np.arange(1, 41)
    f = 0.7 * 0.8 ** r - 0.2 * (-0.5) ** r
    c, lam, err = mpo.fit_exponentials(f, 2)
    order = np.argsort(-lam.real)
    assert np.allclose(lam[order], [0.8, -0.5], atol=1e-12)
    assert np.allclose(c[order], [0.7, -0.2], atol=1e-12)
    assert err < 1e-12


def test_fit_rejects_underdetermined_pencil():
    # K exponentials have 2K unknowns: fewer samples leave the shift matrix
    # rank deficient, so the fit must refuse instead of returning garbage.
    with pytest.raises(ValueError):
        mpo.fit_exponentials(1.0 / np.arange(1, 6) ** 2.0, 3)
    c, lam, err = mpo.fit_exponentials(0.5 ** np.arange(1, 7), 3)
    assert err < 1e-12


def test_fit_power_law_error_scale():
    # 1/r^2 with 12 exponentials on r <= 200: the paper reports an absolute
    # error of 1.5e-7 with its fit (Supplemental Material, XXX model).  A
    # different fitting method need not match it; require the same order.
    f = 1.0 / np.arange(1, 201) ** 2.0
    _, _, err = mpo.fit_exponentials(f, 12)
    assert err < 1e-5


# ------------------------------------------------------ MPS and observables

def test_padded_product_state_is_the_product_state():
    N = 10
    chi = wl.full_rank_bonds(N, 2, 32)
    bits = [0, 1, 1, 0, 1, 0, 0, 0, 1, 1]
    T = mps.padded_product_state(bits, chi)
    assert all(mps.is_right_orthonormal(B) for B in T)
    assert np.array_equal(mps.to_dense(T), spin.product_state(bits))


def test_observables_match_dense():
    N = 8
    T = random_canonical(N, 11)
    psi = mps.to_dense(T)
    z = mps.expect_sites(T, spin.SZ)
    for i in range(1, N + 1):
        assert abs(z[i - 1] - spin.expval(psi, spin.site_op(spin.SZ, i, N))) < 1e-13
    zz = mps.expect_two_point(T, 2, 6, spin.SZ, spin.SX)
    ref = spin.expval(psi, spin.site_op(spin.SZ, 2, N) @ spin.site_op(spin.SX, 6, N))
    assert abs(zz - ref) < 1e-13
    # same site: Oi(i) Oj(i) is the operator product Oi Oj on site i (non-commuting
    # pair, so a swapped order fails), and both argument orders of i > j
    for i, j in ((4, 4), (7, 3)):
        got = mps.expect_two_point(T, i, j, spin.SX, spin.SY)
        ref = spin.expval(psi, spin.site_op(spin.SX, i, N) @ spin.site_op(spin.SY, j, N))
        assert abs(got - ref) < 1e-13, (i, j, got, ref)
    assert abs(mps.expect_two_point(T, 4, 4, spin.SX, spin.SY) - 1j * z[3]) < 1e-13  # sx sy = i sz
    T2 = random_canonical(N, 12)
    assert abs(mps.overlap(T, T2) - np.vdot(psi, mps.to_dense(T2))) < 1e-13
    c, lam, g = fitted_xxx(N, 3)
    Ws = mpo.mpo_exponentials(N, c, lam, spin.xxx_pairs())
    H = spin.longrange_hamiltonian(N, g, spin.xxx_pairs())
    assert abs(mps.mpo_expectation(T, Ws) - spin.expval(psi, H)) < 1e-12


def test_infidelity_matches_dense_and_closed_form():
    """Infidelity of Sec. IV: 1 - |<psi1|psi2>| / (||psi1|| ||psi2||) (modulus, not squared)."""
    N = 7
    T1 = random_canonical(N, 21)
    T2 = random_canonical(N, 22)
    # unnormalised inputs: scale one site of each state
    T1[3] = 1.7 * T1[3]
    T2[5] = (0.4 - 0.3j) * T2[5]
    a, b = mps.to_dense(T1), mps.to_dense(T2)
    ref = 1.0 - abs(np.vdot(a, b)) / (np.linalg.norm(a) * np.linalg.norm(b))
    assert abs(mps.infidelity(T1, T2) - ref) < 1e-13
    # a global phase and a scale leave it at zero
    T3 = [A.copy() for A in T1]
    T3[0] = np.exp(0.9j) * 2.5 * T3[0]
    assert abs(mps.infidelity(T1, T3)) < 1e-13
    # product states cos t|up> + sin t|down> on every site: 1 - |cos(t1 - t2)|^N
    def product(t):
        A = np.zeros((1, 2, 1), dtype=np.complex128)
        A[0, 0, 0], A[0, 1, 0] = np.cos(t), np.sin(t)
        return [A.copy() for _ in range(N)]
    t1, t2 = 0.3, 1.1
    assert abs(mps.infidelity(product(t1), product(t2)) - (1.0 - abs(np.cos(t1 - t2)) ** N)) < 1e-14
    # orthogonal product states (up vs down at one site): infidelity 1
    P, Q = product(0.0), product(0.0)
    Q[2] = product(np.pi / 2)[2]
    assert abs(mps.infidelity(P, Q) - 1.0) < 1e-15


# ------------------------------------------------ environments (Sec. III A)

def _partial_mpo_left(Ws, j):
    """Dense operators O_k on sites 1..j with the MPO bond k left open."""
    O = Ws[0][0]
    for W in Ws[1:j]:
        Onew = np.einsum("kpq,klst->lpsqt", O, W)
        O = Onew.reshape(Onew.shape[0], Onew.shape[1] * Onew.shape[2], -1)
    return O


def test_left_environment_equals_dense_block():
    N = 8
    T = random_canonical(N, 3)
    c, lam, _ = fitted_xxx(N, 3)
    Ws = mpo.mpo_exponentials(N, c, lam, spin.xxx_pairs(), spin.SX, 0.4)
    T = mps.move_centre_right(T, 5)
    bet = env.left_envs(T, Ws)
    for j in (1, 3, 5):
        Phi = mps.left_block_states(T, j)  # [(s_1..s_j), a]
        O = _partial_mpo_left(Ws, j)       # [k, P', P]
        ref = np.einsum("px,kpq,qy->xky", Phi.conj(), O, Phi)
        assert np.max(np.abs(bet[j] - ref)) < 1e-12


# ------------------------------- effective Hamiltonians = E^dag H E (Fig. update)

def _embedding(T, j0, nsite):
    """Isometry from the local state at sites j0+1..j0+nsite into the full space."""
    PhiL = mps.left_block_states(T, j0)
    PhiR = mps.right_block_states(T, j0 + nsite)
    dloc = 2 ** nsite
    E = np.einsum("pa,st,bq->psqatb", PhiL, np.eye(dloc), PhiR)
    D = PhiL.shape[0] * dloc * PhiR.shape[1]
    return E.reshape(D, -1)


def _heff_matrix(apply, shape):
    n = int(np.prod(shape))
    cols = [apply(np.eye(n, dtype=np.complex128)[:, i].reshape(shape)).reshape(-1) for i in range(n)]
    return np.array(cols).T


@pytest.mark.parametrize("nsite", [0, 1, 2])
def test_heff_equals_dense_projection(nsite):
    N, j = 8, 3  # local sites j+1 (and j+2), 1-based
    T = random_canonical(N, 21, cap=8)
    c, lam, g = fitted_xxx(N, 3)
    Ws = mpo.mpo_exponentials(N, c, lam, spin.xxx_pairs(), spin.SX, 0.2)
    H = spin.longrange_hamiltonian(N, g, spin.xxx_pairs(), spin.SX, 0.2)
    if nsite == 0:
        T = mps.move_centre_right(T, j)
        chil, d, chir = T[j].shape
        Q, _ = np.linalg.qr(T[j].reshape(chil * d, chir))
        T[j] = Q.reshape(chil, d, chir)  # sites 1..j+1 left-, j+2..N right-orthonormal
        bet = env.left_envs(T, Ws)
        gam = env.right_envs(T, Ws)
        chi = T[j].shape[2]
        Hm = _heff_matrix(lambda x: heff.apply_heff0(bet[j + 1], gam[j], x), (chi, chi))
        E = _embedding(T, j + 1, 0)
    else:
        T = mps.move_centre_right(T, j)
        bet = env.left_envs(T, Ws)
        gam = env.right_envs(T, Ws)
        if nsite == 1:
            shape = T[j].shape
            Hm = _heff_matrix(lambda x: heff.apply_heff1(bet[j], Ws[j], gam[j], x), shape)
        else:
            shape = (T[j].shape[0], 2, 2, T[j + 1].shape[2])
            Hm = _heff_matrix(lambda x: heff.apply_heff2(bet[j], Ws[j], Ws[j + 1], gam[j + 1], x), shape)
        E = _embedding(T, j, nsite)
    assert np.allclose(E.conj().T @ E, np.eye(E.shape[1]), atol=1e-12)
    ref = E.conj().T @ H @ E
    assert np.linalg.norm(Hm - ref) <= 1e-12 * np.linalg.norm(ref)


# ----------------------------------------------------- Lanczos (Sec. III A)

@pytest.mark.parametrize("n,tau", [(1, 0.3), (7, -0.05), (300, 0.05), (300, 1.0)])
def test_lanczos_equals_expm(n, tau):
    rng = np.random.default_rng(n)
    G = wl.cgauss(rng, (n, n))
    A = (G + G.conj().T) / (2 * np.sqrt(n))
    x = wl.cgauss(rng, (n,))
    ref = sla.expm(-1j * tau * A) @ x
    out = krylov.expm_krylov(lambda v: A @ v, x, tau, kmax=60, tol=1e-13)
    assert np.linalg.norm(out - ref) <= 1e-12 * np.linalg.norm(ref)


def test_lanczos_zero_vector_and_happy_breakdown():
    A = np.diag([1.0, 2.0, 3.0]).astype(np.complex128)
    z = np.zeros(3, dtype=np.complex128)
    assert np.array_equal(krylov.expm_krylov(lambda v: A @ v, z, 0.1), z)
    e = np.array([0, 1.0, 0], dtype=np.complex128)  # eigenvector: one iteration
    out, k = krylov.expm_krylov(lambda v: A @ v, e, 0.1, return_info=True)
    assert k == 1 and np.allclose(out, np.exp(-0.2j) * e, atol=1e-15)


# -------------------------------------------- truncation (Sec. III C, III D)

def test_truncation_eckart_young_and_rules():
    rng = np.random.default_rng(5)
    theta = wl.cgauss(rng, (6, 2, 2, 5))
    s = np.linalg.svd(theta.reshape(12, 10), compute_uv=False)
    tr = tdvp.Truncation(chi_max=4, w_max=0.0, eps=0.0, multiplet_guard=False)
    U, S, Vh, w = tdvp.svd_split(theta, tr)
    approx = np.einsum("asc,c,ctb->astb", U, S, Vh)
    assert abs(np.linalg.norm(theta - approx) ** 2 - w) < 1e-12
    assert abs(w - np.sum(s[4:] ** 2)) < 1e-12
    # discarded-weight rule: smallest chi with tail <= w_max
    sv = np.array([1.0, 0.5, 0.1, 0.01, 1e-3])
    assert tdvp.truncation_rank(sv, tdvp.Truncation(w_max=1.5e-4, multiplet_guard=False))[0] == 3
    assert tdvp.truncation_rank(sv, tdvp.Truncation(w_max=0.0, eps=0.05, multiplet_guard=False))[0] == 3
    assert tdvp.truncation_rank(sv, tdvp.Truncation(chi_max=2, multiplet_guard=False))[0] == 2
    assert tdvp.truncation_rank(sv, tdvp.Truncation(w_max=10.0))[0] == 1
    deg = np.array([1.0, 0.5, 0.5, 0.1])
    assert tdvp.truncation_rank(deg, tdvp.Truncation(chi_max=2, multiplet_guard=True))[0] == 1


# ------------------------------- 1TDVP at full bond dimension equals ED (Sec. II D)

def test_tdvp1_full_rank_equals_exact_evolution_and_conserves():
    N, Ws, H = ising_n10()
    p = wl.ISING_N10
    chi = wl.full_rank_bonds(N, 2, p["chi_cap"])
    T = mps.padded_product_state([0] * N, chi)
    psi0 = spin.product_state([0] * N)
    E0 = sum((N - r) / r ** 3 for r in range(1, N))
    assert abs(E0 - 10.425552125575392) < 1e-14
    assert abs(mps.mpo_expectation(T, Ws) - E0) < 1e-13
    ex = spin.ExactEvolution(H)
    st = tdvp.MPSState(T, Ws)
    steps = 30
    for _ in range(steps):
        tdvp.tdvp1_step(st, p["dt"])
    psi = ex.evolve(psi0, steps * p["dt"])
    z = mps.expect_sites(st.T, spin.SZ).real
    zref = [spin.expval(psi, spin.site_op(spin.SZ, i, N)).real for i in range(1, N + 1)]
    assert np.max(np.abs(z - zref)) < 1e-10
    assert abs(z[4] - z[5]) < 1e-10                   # reflection symmetry
    assert np.max(np.abs(z - z[::-1])) < 1e-10
    assert abs(mps.mpo_expectation(st.T, Ws).real - E0) < 1e-10  # energy (Sec. II D)
    assert abs(mps.norm2(st.T) - 1.0) < 1e-12                   # norm


def test_tdvp1_short_time_expansion():
    # <sigma^z_i(t)> = 1 - 2 h^2 t^2 + O(t^4) from |up...up> under zz + h x.
    N, Ws, _ = ising_n10()
    T = mps.padded_product_state([0] * N, wl.full_rank_bonds(N, 2, 32))
    st = tdvp.MPSState(T, Ws)
    t = 0.01
    tdvp.tdvp1_step(st, t)
    z = mps.expect_sites(st.T, spin.SZ).real
    assert np.max(np.abs(z - (1 - 2 * t ** 2))) < 10 * t ** 4


def test_tdvp1_time_reversal():
    N = 8
    T = random_canonical(N, 8)
    c, lam, _ = fitted_xxx(N, 3)
    Ws = mpo.mpo_exponentials(N, c, lam, spin.xxx_pairs(), spin.SX, 0.5)
    psi0 = mps.to_dense(T)
    st = tdvp.MPSState(T, Ws)
    tdvp.tdvp1_step(st, 0.1)
    assert np.linalg.norm(mps.to_dense(st.T) - psi0) > 1e-2
    tdvp.tdvp1_step(st, -0.1)
    assert np.linalg.norm(mps.to_dense(st.T) - psi0) < 1e-11


def test_tdvp1_reduced_rank_conserves_energy_and_norm():
    N = 10
    T = random_canonical(N, 9, cap=4)
    c, lam, _ = fitted_xxx(N, 3)
    Ws = mpo.mpo_exponentials(N, c, lam, spin.xxx_pairs(), spin.SX, 0.5)
    E0 = mps.mpo_expectation(T, Ws).real
    st = tdvp.MPSState(T, Ws)
    for _ in range(5):
        tdvp.tdvp1_step(st, 0.05)
    assert abs(mps.mpo_expectation(st.T, Ws).real - E0) < 1e-10
    assert abs(mps.norm2(st.T) - 1.0) < 1e-12


# ------------------------------- 2TDVP at full bond dimension equals ED (Sec. II D)

def test_tdvp2_full_rank_equals_exact_evolution():
    N = 8
    T = random_canonical(N, 5)
    c, lam, g = fitted_xxx(N, 3)
    Ws = mpo.mpo_exponentials(N, c, lam, spin.xxx_pairs())
    H = spin.longrange_hamiltonian(N, g, spin.xxx_pairs())
    psi0 = mps.to_dense(T)
    st = tdvp.MPSState(T, Ws)
    for _ in range(5):
        tdvp.tdvp2_step(st, 0.05, tdvp.Truncation())
    psi = spin.ExactEvolution(H).evolve(psi0, 0.25)
    assert np.linalg.norm(mps.to_dense(st.T) - psi) < 1e-9


def test_tdvp2_truncated_norm_is_one_minus_wtotal():
    N = 8
    c, lam, _ = fitted_xxx(N, 3)
    Ws = mpo.mpo_exponentials(N, c, lam, spin.xxx_pairs())
    bits = [i % 2 for i in range(N)]
    bits[N // 2 - 1] ^= 1
    T = mps.padded_product_state(bits, [1] * (N + 1))
    st = tdvp.MPSState(T, Ws)
    tr = tdvp.Truncation(chi_max=6, w_max=1e-8, eps=1e-12)
    for _ in range(6):
        tdvp.tdvp2_step(st, 0.05, tr)
    assert st.stats.w_total > 0
    assert abs(mps.norm2(st.T) - (1.0 - st.stats.w_total)) < 1e-12
    assert max(A.shape[2] for A in st.T) <= 6


def test_spin_one_mpo_equals_kronecker_hamiltonian():
    # local dimension d = 3: the MPO builders and the Kronecker Hamiltonian agree
    Sz = np.diag([1.0, 0.0, -1.0]).astype(np.complex128)
    Sx = (np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]]) / np.sqrt(2)).astype(np.complex128)
    Sy = (np.array([[0, -1j, 0], [1j, 0, -1j], [0, 1j, 0]]) / np.sqrt(2)).astype(np.complex128)
    pairs = [(1.0, Sx, Sx), (1.0, Sy, Sy), (1.0, Sz, Sz)]
    N = 5
    f = lambda r: 1.0 / r ** 2
    Ws = mpo.mpo_exact(N, f, pairs, Sz, 0.3)
    H = spin.longrange_hamiltonian(N, f, pairs, Sz, 0.3)
    assert H.shape == (3 ** N, 3 ** N)
    assert np.max(np.abs(mpo.mpo_to_dense(Ws) - H)) < 1e-13
    c, lam, _ = mpo.fit_exponentials(1.0 / np.arange(1, 17) ** 2.0, 3)
    g = mpo.eval_exponentials(c, lam, N - 1)
    Ws2 = mpo.mpo_exponentials(N, c, lam, pairs, Sz, 0.3)
    H2 = spin.longrange_hamiltonian(N, g, pairs, Sz, 0.3)
    assert np.max(np.abs(mpo.mpo_to_dense(Ws2) - H2)) < 1e-12


def test_chi_saturation_rule():
    """Saturated means every bond at min(chi_max, d^min(j, N-j)) (hybrid scheme)."""
    full = [np.zeros((a, 2, b)) for a, b in zip(wl.full_rank_bonds(6, 2)[:-1], wl.full_rank_bonds(6, 2)[1:])]
    assert tdvp.chi_saturated(full, 1 << 30)            # 1 2 4 8 4 2 1
    capped = [np.zeros((a, 2, b)) for a, b in zip(wl.full_rank_bonds(6, 2, 3)[:-1], wl.full_rank_bonds(6, 2, 3)[1:])]
    assert tdvp.chi_saturated(capped, 3) and not tdvp.chi_saturated(capped, 4)
    product = [np.zeros((1, 2, 1)) for _ in range(6)]
    assert not tdvp.chi_saturated(product, 2)
    assert tdvp.chi_saturated(product, 1)


def test_hybrid_saturated_start_is_one_site_and_exact():
    """A product state padded to full bond dimension is saturated from the
    start: every hybrid step is one-site, and one-site TDVP at full rank is
    exact, so the run equals exact evolution."""
    N = 8
    c, lam, g = fitted_xxx(N, 3)
    Ws = mpo.mpo_exponentials(N, c, lam, spin.xxx_pairs())
    H = spin.longrange_hamiltonian(N, g, spin.xxx_pairs())
    bits = [i % 2 for i in range(N)]
    T = mps.padded_product_state(bits, wl.full_rank_bonds(N, 2))
    psi0 = mps.to_dense(T)
    st = tdvp.MPSState(T, Ws)
    kinds = [tdvp.hybrid_step(st, 0.05, tdvp.Truncation()) for _ in range(6)]
    assert all(kinds)
    psi = spin.ExactEvolution(H).evolve(psi0, 0.3)
    assert np.linalg.norm(mps.to_dense(st.T) - psi) < 1e-9


def test_hybrid_truncated_keeps_chi_max_and_conserves_energy_after_switch():
    """Under truncation the switch happens when every bond reaches chi_max;
    after it the bond dimensions stay fixed and, as 1TDVP is a projected
    Hamiltonian flow, the energy and norm are conserved (up to Lanczos error)."""
    N = 10
    c, lam, _ = fitted_xxx(N, 3)
    Ws = mpo.mpo_exponentials(N, c, lam, spin.xxx_pairs())
    bits = [i % 2 for i in range(N)]
    bits[N // 2 - 1] ^= 1
    st = tdvp.MPSState(mps.padded_product_state(bits, [1] * (N + 1)), Ws)
    tr = tdvp.Truncation(chi_max=4, w_max=0.0, eps=1e-14)
    kinds, energies, norms = [], [], []
    for _ in range(16):
        kinds.append(tdvp.hybrid_step(st, 0.05, tr))
        energies.append(mps.mpo_expectation(st.T, Ws).real / mps.norm2(st.T))
        norms.append(mps.norm2(st.T))
    first = kinds.index(True)
    assert first > 0 and all(kinds[first:])
    chi = [A.shape[2] for A in st.T[:-1]]
    assert chi == [min(4, 2 ** min(j, N - j)) for j in range(1, N)]
    assert max(abs(e - energies[first]) for e in energies[first:]) < 1e-10
    assert max(abs(n - norms[first]) for n in norms[first:]) < 1e-12


def _ground(H):
    w, V = np.linalg.eigh(H)
    return w[0], V[:, 0], w[1] - w[0]


@pytest.mark.parametrize("model", ["xxx", "ising"])
def test_dmrg_reaches_the_exact_ground_state(model):
    """Two-site DMRG at full bond dimension converges to the lowest eigenpair
    of the Kronecker-built Hamiltonian (non-degenerate here)."""
    from oracle import dmrg
    N = 8
    if model == "xxx":
        c, lam, g = fitted_xxx(N, 3)
        Ws = mpo.mpo_exponentials(N, c, lam, spin.xxx_pairs(), spin.SZ, 0.1)
        H = spin.longrange_hamiltonian(N, g, spin.xxx_pairs(), spin.SZ, 0.1)
    else:
        f = lambda r: 1.0 / r ** 3
        Ws = mpo.mpo_exact(N, f, spin.ising_pairs(), spin.SX, 1.0)
        H = spin.longrange_hamiltonian(N, f, spin.ising_pairs(), spin.SX, 1.0)
    E0, psi0, gap = _ground(H)
    assert gap > 1e-3
    st = tdvp.MPSState(random_canonical(N, 3, 4), Ws)
    energies = [dmrg.dmrg2_sweep(st, tdvp.Truncation(eps=1e-14)) for _ in range(4)]
    assert abs(energies[-1] - E0) < 1e-10
    assert abs(abs(np.vdot(psi0, mps.to_dense(st.T))) - 1.0) < 1e-10
    assert abs(mps.norm2(st.T) - 1.0) < 1e-12


def test_dmrg_truncated_is_variational_and_monotone():
    """Under truncation (chi_max = 3) every sweep's energy is an upper bound
    of the exact ground energy and does not increase from sweep to sweep."""
    from oracle import dmrg
    N = 10
    c, lam, g = fitted_xxx(N, 3)
    Ws = mpo.mpo_exponentials(N, c, lam, spin.xxx_pairs())
    H = spin.longrange_hamiltonian(N, g, spin.xxx_pairs())
    E0 = np.linalg.eigvalsh(H)[0]
    st = tdvp.MPSState(random_canonical(N, 4, 3), Ws)
    es = []
    for _ in range(4):
        dmrg.dmrg2_sweep(st, tdvp.Truncation(chi_max=3))
        es.append(mps.mpo_expectation(st.T, Ws).real / mps.norm2(st.T))
    assert all(e >= E0 - 1e-12 for e in es)
    assert all(b <= a + 1e-10 for a, b in zip(es, es[1:]))
    assert es[-1] - E0 < 0.05 * abs(E0)


@pytest.mark.parametrize("two_site", [False, True])
def test_imaginary_time_full_rank_equals_normalised_exp(two_site):
    """At full bond dimension the TDVP splitting is exact, so imaginary-time
    steps give exp(-tau H) psi_0 / ||.|| of the Kronecker-built Hamiltonian,
    and a long run approaches its ground energy."""
    N = 8
    c, lam, g = fitted_xxx(N, 3)
    Ws = mpo.mpo_exponentials(N, c, lam, spin.xxx_pairs(), spin.SZ, 0.1)
    H = spin.longrange_hamiltonian(N, g, spin.xxx_pairs(), spin.SZ, 0.1)
    T = random_canonical(N, 6)
    psi0 = mps.to_dense(T)
    st = tdvp.MPSState(T, Ws)
    tr = tdvp.Truncation() if two_site else None
    for _ in range(5):
        tdvp.imaginary_time_step(st, 0.1, tr)
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    ref = sla.expm(-0.5 * Hd) @ psi0
    ref /= np.linalg.norm(ref)
    assert np.linalg.norm(mps.to_dense(st.T) - ref) < 1e-9
    for _ in range(60):
        tdvp.imaginary_time_step(st, 0.25, tr)
    # tau = 15.5: the energy of the exact normalised exp(-tau H) psi_0, below
    # the start and approaching the ground energy
    far = sla.expm(-15.5 * Hd) @ psi0
    far /= np.linalg.norm(far)
    E = mps.mpo_expectation(st.T, Ws).real
    assert abs(E - np.vdot(far, Hd @ far).real) < 1e-9
    E0 = np.linalg.eigvalsh(Hd)[0]
    assert E0 <= E < E0 + 1e-3 < np.vdot(psi0, Hd @ psi0).real
