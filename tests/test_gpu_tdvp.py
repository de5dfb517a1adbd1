"""Parity of the device TDVP time steps and observables with the FP64 oracle
and with exact diagonalisation (Sec. II D, Sec. III A, Sec. IV).

Bars: the complex128 path matches observables to 1e-10, the complex64 path
(FP32 MFMA contractions, FP64 Lanczos/QR/SVD) to 1e-4 absolute.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import mpo as ompo
from oracle import mps as omps
from oracle import spin
from oracle import tdvp as otdvp

pytestmark = pytest.mark.gpu

OBS_TOL = {"c128": 1e-10, "c64": 1e-4}


@pytest.fixture(scope="module")
def ctx():
    import paper_1912_06127_amd as pkg
    c = pkg.Context(0)
    yield c
    c.sync()
    c.close()


def ising_n10():
    p = wl.ISING_N10
    f = lambda r: p["J"] / r ** p["alpha"]
    Ws = ompo.mpo_exact(p["N"], f, spin.ising_pairs(), spin.SX, p["h"])
    H = spin.longrange_hamiltonian(p["N"], f, spin.ising_pairs(), spin.SX, p["h"])
    return p, f, Ws, H


def xxx_fit(N, K):
    c, lam, _ = ompo.fit_exponentials(1.0 / np.arange(1, N) ** 2.0, K)
    return c, lam


def test_mps_init_product_state_matches_padding(ctx):
    import paper_1912_06127_amd as pkg
    N = 10
    chi = wl.full_rank_bonds(N, 2, 32)
    bits = [0, 1, 1, 0, 1, 0, 0, 0, 1, 1]
    m = pkg.MPS.init(ctx, N, 2, chi, basis_state=bits)
    ref = omps.padded_product_state(bits, chi)
    for j in range(N):
        assert np.array_equal(m.tensor(j), ref[j])


def test_random_mps_is_right_canonical(ctx):
    import paper_1912_06127_amd as pkg
    N = 8
    chi = wl.full_rank_bonds(N, 2, 8)
    m = pkg.MPS.init(ctx, N, 2, chi, seed=3)
    T = m.tensors()
    assert all(omps.is_right_orthonormal(B, 1e-12) for B in T[1:])
    assert abs(omps.norm2(T) - 1.0) < 1e-12
    assert abs(pkg.norm2(ctx, m) - 1.0) < 1e-12


def test_observables_match_oracle(ctx):
    import paper_1912_06127_amd as pkg
    N = 8
    T = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(4, wl.full_rank_bonds(N, 2, 6), 2)))
    T[3] = T[3] * 1.3  # unnormalised state: observables divide by <psi|psi>
    m = pkg.MPS.from_tensors(ctx, T)
    z = pkg.expect(ctx, m, list(range(N)), spin.SZ)
    assert np.max(np.abs(z - omps.expect_sites(T, spin.SZ))) < 1e-12
    x = pkg.expect2(ctx, m, [1, 5, 3], [5, 1, 3], spin.SZ, spin.SX)
    ref = [omps.expect_two_point(T, 2, 6, spin.SZ, spin.SX), omps.expect_two_point(T, 6, 2, spin.SZ, spin.SX),
           omps.expect_two_point(T, 4, 4, spin.SZ, spin.SX)]
    assert np.max(np.abs(x - np.array(ref))) < 1e-12
    assert abs(pkg.norm2(ctx, m) - omps.norm2(T)) < 1e-12
    c, lam = xxx_fit(N, 3)
    Ws = ompo.mpo_exponentials(N, c, lam, spin.xxx_pairs(), spin.SX, 0.3)
    W = pkg.MPO.from_tensors(ctx, Ws)
    assert abs(pkg.energy(ctx, m, W) - omps.mpo_expectation(T, Ws)) < 1e-12
    T2 = omps.right_canonicalize(wl.random_site_tensors(5, wl.full_rank_bonds(N, 2, 4), 2))
    m2 = pkg.MPS.from_tensors(ctx, T2)
    assert abs(pkg.overlap(ctx, m, m2) - omps.overlap(T, T2)) < 1e-12


def test_mpo_longrange_matches_oracle_builders(ctx):
    import paper_1912_06127_amd as pkg
    N = 7
    c, lam = xxx_fit(N, 3)
    W = pkg.MPO.longrange(ctx, N, spin.xxx_pairs(), c=c, lam=lam, onsite=spin.SX, h=0.3)
    ref = ompo.mpo_exponentials(N, c, lam, spin.xxx_pairs(), spin.SX, 0.3)
    for j in range(N):
        assert np.max(np.abs(W.tensor(j) - ref[j])) < 1e-15
    p, f, Ws, _ = ising_n10()
    W2 = pkg.MPO.longrange(ctx, p["N"], spin.ising_pairs(), coupling=[f(r) for r in range(1, p["N"])],
                           onsite=spin.SX, h=p["h"])
    for j in range(p["N"]):
        assert np.max(np.abs(W2.tensor(j) - Ws[j])) < 1e-15


def test_mpo_longrange_fits_the_power_law_itself(ctx):
    """mpo_longrange with alpha and K (no c, lambda): the library fits r^-alpha
    (Sec. II C) and builds the MPO; its dense operator equals the oracle's MPO
    from the oracle's independent fit, and the reported fit error matches."""
    import paper_1912_06127_amd as pkg
    for N, alpha, K, pairs in ((8, 2.0, 3, spin.xxx_pairs()), (7, 1.5, 2, spin.xy_pairs())):
        W = pkg.MPO.longrange(ctx, N, pairs, alpha=alpha, K=K, onsite=spin.SX, h=0.3)
        c, lam, err = ompo.fit_exponentials(1.0 / np.arange(1, N) ** alpha, K)
        ref = ompo.mpo_exponentials(N, c, lam, pairs, spin.SX, 0.3)
        assert W.w == [1] + [len(pairs) * K + 2] * (N - 1) + [1]
        dense = ompo.mpo_to_dense([W.tensor(j) for j in range(N)])
        assert np.max(np.abs(dense - ompo.mpo_to_dense(ref))) < 1e-9
        assert np.max(np.abs(dense - dense.conj().T)) < 1e-12
        assert abs(W.fit_max_abs_err - err) < 1e-10
    # the N = 201 XY workload's fit (alpha = 1.5, K = 6 on r <= 200) and the refined variant
    p = wl.XY_N201
    W = pkg.MPO.longrange(ctx, 201, spin.xy_pairs(), alpha=p["alpha"], K=p["K"])
    _, _, err = ompo.fit_exponentials(1.0 / np.arange(1, 201) ** p["alpha"], p["K"])
    assert abs(W.fit_max_abs_err - err) < 1e-3 * err
    Wr = pkg.MPO.longrange(ctx, 201, spin.xy_pairs(), alpha=p["alpha"], K=p["K"], fit_refine=True)
    assert Wr.fit_max_abs_err < W.fit_max_abs_err


@pytest.mark.parametrize("dt_", ["c128", "c64"])
def test_tdvp1_ising_n10_matches_exact_evolution(ctx, dt_):
    """Long-range Ising quench, N = 10, exact MPO, 1TDVP at D <= 32 vs ED (2^10 states)."""
    import paper_1912_06127_amd as pkg
    p, f, Ws, H = ising_n10()
    N = p["N"]
    print(f"tdvp1 Ising N=10 {dt_}", flush=True)
    W = pkg.MPO.longrange(ctx, N, spin.ising_pairs(), coupling=[f(r) for r in range(1, N)],
                          onsite=spin.SX, h=p["h"])
    m = pkg.MPS.init(ctx, N, 2, wl.full_rank_bonds(N, 2, p["chi_cap"]), basis_state=[0] * N)
    ex = spin.ExactEvolution(H)
    psi0 = spin.product_state([0] * N)
    Z = [spin.site_op(spin.SZ, i, N) for i in (5, 6)]
    E0 = sum((N - r) / r ** 3 for r in range(1, N))
    opts = pkg.TDVPOptions(compute=dt_)
    worst = 0.0
    for s in range(1, p["steps"] + 1):
        st = pkg.tdvp1_step(ctx, m, W, p["dt"], opts)
        assert st["flags"] == 0
        if s % 10 == 0:
            psi = ex.evolve(psi0, s * p["dt"])
            z = pkg.expect(ctx, m, [4, 5], spin.SZ).real
            zref = [spin.expval(psi, Zi).real for Zi in Z]
            e = pkg.energy(ctx, m, W).real
            worst = max(worst, np.max(np.abs(z - zref)), abs(e - E0))
    assert worst <= OBS_TOL[dt_], worst
    assert abs(pkg.norm2(ctx, m) - 1.0) <= OBS_TOL[dt_]


@pytest.mark.parametrize("dt_,svd_mode", [("c128", 0), ("c64", 0), ("c128", 1), ("c64", 1)])
def test_tdvp2_truncated_matches_oracle(ctx, dt_, svd_mode):
    """2TDVP with truncation (w_max, chi_max, eps) on a fitted 1/r^2 XXX chain.

    svd_mode 0 picks the reduced-density-matrix split (w_max = 1e-8), 1 the SVD."""
    import paper_1912_06127_amd as pkg
    N = 10
    print(f"tdvp2 XXX N={N} {dt_}", flush=True)
    c, lam = xxx_fit(N, 3)
    Ws = ompo.mpo_exponentials(N, c, lam, spin.xxx_pairs())
    bits = [i % 2 for i in range(N)]
    bits[N // 2 - 1] ^= 1
    T0 = omps.padded_product_state(bits, [1] * (N + 1))
    st_o = otdvp.MPSState(T0, Ws)
    tr = otdvp.Truncation(chi_max=12, w_max=1e-8, eps=1e-12)
    W = pkg.MPO.longrange(ctx, N, spin.xxx_pairs(), c=c, lam=lam)
    m = pkg.MPS.init(ctx, N, 2, [1] * (N + 1), basis_state=bits)
    opts = pkg.TDVPOptions(compute=dt_, chi_max=12, w_max=1e-8, eps_rel=1e-12, svd_mode=svd_mode)
    for s in range(8):
        otdvp.tdvp2_step(st_o, 0.05, tr)
        st = pkg.tdvp2_step(ctx, m, W, 0.05, opts)
        z = pkg.expect(ctx, m, list(range(N)), spin.SZ).real
        zref = omps.expect_sites(st_o.T, spin.SZ).real
        assert np.max(np.abs(z - zref)) <= OBS_TOL[dt_], (s, np.max(np.abs(z - zref)))
    if dt_ == "c128":
        assert m.chi == [1] + [A.shape[2] for A in st_o.T]
        assert abs(st["w_total"] - st_o.stats.w_total) <= 1e-12
        assert abs(pkg.norm2(ctx, m) - (1.0 - st["w_total"])) <= 1e-11


@pytest.mark.parametrize("dt_", ["c128", "c64"])
def test_tdvp2_neel_quench_tracks_oracle_over_many_steps(ctx, dt_):
    """Long truncated 2TDVP quench from a Neel state with one flipped spin
    (the XXX workload of Sec. IV at N = 24).  Its density-matrix splits are
    rank deficient at every step (exact null spaces), the case in which
    non-unitary eigen-solver rotations would shrink a kept vector without
    changing any truncation decision: state, norm, discarded weight and
    right-orthonormality are compared with the oracle after the last step."""
    import paper_1912_06127_amd as pkg
    N, steps = 24, 30
    print(f"tdvp2 Neel quench N={N} {dt_}", flush=True)
    c, lam = xxx_fit(N, 6)
    Ws = ompo.mpo_exponentials(N, c, lam, spin.xxx_pairs())
    bits = [i % 2 for i in range(N)]
    bits[N // 2 - 1] ^= 1
    st_o = otdvp.MPSState(omps.padded_product_state(bits, [1] * (N + 1)), Ws)
    tr = otdvp.Truncation(chi_max=512, w_max=1e-8, eps=1e-12)
    W = pkg.MPO.longrange(ctx, N, spin.xxx_pairs(), c=c, lam=lam)
    m = pkg.MPS.init(ctx, N, 2, [1] * (N + 1), basis_state=bits)
    opts = pkg.TDVPOptions(compute=dt_, chi_max=512, w_max=1e-8, eps_rel=1e-12, krylov_tol=1e-10)
    for _ in range(steps):
        otdvp.tdvp2_step(st_o, 0.05, tr, tol=1e-10)
        st = pkg.tdvp2_step(ctx, m, W, 0.05, opts)
    T = m.tensors()
    z = pkg.expect(ctx, m, list(range(N)), spin.SZ).real
    zref = omps.expect_sites(st_o.T, spin.SZ).real
    assert np.max(np.abs(z - zref)) <= OBS_TOL[dt_], np.max(np.abs(z - zref))
    n_o, n_g = omps.norm2(st_o.T), omps.norm2(T)
    assert abs(n_g - n_o) <= OBS_TOL[dt_], (n_g, n_o)
    assert all(omps.is_right_orthonormal(B, 1e-10 if dt_ == "c128" else 1e-6) for B in T[1:])
    if dt_ == "c128":
        assert 1.0 - abs(omps.overlap(st_o.T, T)) ** 2 / (n_o * n_g) <= 1e-10
        assert abs(st["w_total"] - st_o.stats.w_total) <= 1e-9 * st_o.stats.w_total
        assert st_o.stats.w_total > 1e-7  # truncation is active


@pytest.mark.parametrize("dt_", ["c128", "c64"])
def test_hybrid_step_matches_oracle(ctx, dt_):
    """Hybrid scheme (two-site until chi_max is saturated, then one-site):
    same switch step as the oracle and observables to the bar every step."""
    import paper_1912_06127_amd as pkg
    N = 10
    print(f"hybrid XXX N={N} {dt_}", flush=True)
    c, lam = xxx_fit(N, 3)
    Ws = ompo.mpo_exponentials(N, c, lam, spin.xxx_pairs())
    bits = [i % 2 for i in range(N)]
    bits[N // 2 - 1] ^= 1
    st_o = otdvp.MPSState(omps.padded_product_state(bits, [1] * (N + 1)), Ws)
    tr = otdvp.Truncation(chi_max=4, w_max=0.0, eps=1e-14)
    W = pkg.MPO.longrange(ctx, N, spin.xxx_pairs(), c=c, lam=lam)
    m = pkg.MPS.init(ctx, N, 2, [1] * (N + 1), basis_state=bits)
    opts = pkg.TDVPOptions(compute=dt_, chi_max=4, w_max=0.0, eps_rel=1e-14)
    kinds_o, kinds_g = [], []
    for s in range(16):
        kinds_o.append(otdvp.hybrid_step(st_o, 0.05, tr))
        kinds_g.append(pkg.tdvp_hybrid_step(ctx, m, W, 0.05, opts)["one_site"])
        z = pkg.expect(ctx, m, list(range(N)), spin.SZ).real
        zref = omps.expect_sites(st_o.T, spin.SZ).real
        assert np.max(np.abs(z - zref)) <= OBS_TOL[dt_], (s, np.max(np.abs(z - zref)))
    assert kinds_g == kinds_o and any(kinds_o) and not kinds_o[0]
    assert m.chi == [1] + [A.shape[2] for A in st_o.T]


@pytest.mark.parametrize("two_site", [False, True])
def test_imaginary_time_full_rank_matches_normalised_exp(ctx, two_site):
    """Imaginary-time steps at full bond dimension equal exp(-tau H) psi_0 / ||.||."""
    import scipy.linalg as sla
    import paper_1912_06127_amd as pkg
    N = 8
    print(f"imaginary time N={N} two_site={two_site}", flush=True)
    c, lam = xxx_fit(N, 3)
    g = ompo.eval_exponentials(c, lam, N - 1)
    H = spin.longrange_hamiltonian(N, g, spin.xxx_pairs(), spin.SZ, 0.1)
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    T = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(61, wl.full_rank_bonds(N, 2), 2)))
    W = pkg.MPO.longrange(ctx, N, spin.xxx_pairs(), c=c, lam=lam, onsite=spin.SZ, h=0.1)
    m = pkg.MPS.from_tensors(ctx, T)
    opts = pkg.TDVPOptions(compute="c128", imaginary=True)
    step = pkg.tdvp2_step if two_site else pkg.tdvp1_step
    for _ in range(5):
        step(ctx, m, W, 0.1, opts)
    ref = sla.expm(-0.5 * Hd) @ omps.to_dense(T)
    ref /= np.linalg.norm(ref)
    assert np.linalg.norm(omps.to_dense(m.tensors()) - ref) < 1e-9
    assert abs(pkg.norm2(ctx, m) - 1.0) < 1e-12


@pytest.mark.parametrize("dt_", ["c128", "c64"])
def test_imaginary_time_truncated_matches_oracle(ctx, dt_):
    import paper_1912_06127_amd as pkg
    N = 10
    print(f"imaginary time truncated N={N} {dt_}", flush=True)
    c, lam = xxx_fit(N, 3)
    Ws = ompo.mpo_exponentials(N, c, lam, spin.xxx_pairs())
    bits = [i % 2 for i in range(N)]
    st_o = otdvp.MPSState(omps.padded_product_state(bits, [1] * (N + 1)), Ws)
    tr = otdvp.Truncation(chi_max=6, w_max=1e-10, eps=1e-12)
    W = pkg.MPO.longrange(ctx, N, spin.xxx_pairs(), c=c, lam=lam)
    m = pkg.MPS.init(ctx, N, 2, [1] * (N + 1), basis_state=bits)
    opts = pkg.TDVPOptions(compute=dt_, chi_max=6, w_max=1e-10, eps_rel=1e-12, imaginary=True)
    for s in range(8):
        otdvp.imaginary_time_step(st_o, 0.1, tr)
        pkg.tdvp2_step(ctx, m, W, 0.1, opts)
        z = pkg.expect(ctx, m, list(range(N)), spin.SZ).real
        zref = omps.expect_sites(st_o.T, spin.SZ).real
        assert np.max(np.abs(z - zref)) <= OBS_TOL[dt_], (s, np.max(np.abs(z - zref)))
    e = pkg.energy(ctx, m, W).real
    e_ref = omps.mpo_expectation(st_o.T, Ws).real / omps.norm2(st_o.T)
    assert abs(e - e_ref) <= OBS_TOL[dt_]


def test_tdvp2_full_rank_matches_exact_evolution(ctx):
    import paper_1912_06127_amd as pkg
    N = 8
    c, lam = xxx_fit(N, 3)
    Ws = ompo.mpo_exponentials(N, c, lam, spin.xxx_pairs())
    g = ompo.eval_exponentials(c, lam, N - 1)
    H = spin.longrange_hamiltonian(N, g, spin.xxx_pairs())
    T = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(5, wl.full_rank_bonds(N, 2), 2)))
    psi0 = omps.to_dense(T)
    m = pkg.MPS.from_tensors(ctx, T)
    W = pkg.MPO.from_tensors(ctx, Ws)
    for _ in range(5):
        pkg.tdvp2_step(ctx, m, W, 0.05, pkg.TDVPOptions())
    psi = spin.ExactEvolution(H).evolve(psi0, 0.25)
    assert np.linalg.norm(omps.to_dense(m.tensors()) - psi) < 1e-9


def test_tdvp1_random_state_matches_oracle_and_reverses(ctx):
    import paper_1912_06127_amd as pkg
    N = 12
    c, lam = xxx_fit(N, 3)
    Ws = ompo.mpo_exponentials(N, c, lam, spin.xxx_pairs(), spin.SX, 0.5)
    T = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(9, wl.full_rank_bonds(N, 2, 16), 2)))
    st_o = otdvp.MPSState(T, Ws)
    m = pkg.MPS.from_tensors(ctx, T)
    W = pkg.MPO.from_tensors(ctx, Ws)
    for _ in range(3):
        otdvp.tdvp1_step(st_o, 0.05)
        pkg.tdvp1_step(ctx, m, W, 0.05)
    assert abs(abs(omps.overlap(m.tensors(), st_o.T)) - 1.0) < 1e-11
    for _ in range(3):
        pkg.tdvp1_step(ctx, m, W, -0.05)
    assert abs(abs(omps.overlap(m.tensors(), T)) - 1.0) < 1e-11


def test_strict_krylov_nonconvergence_is_reported(ctx):
    import paper_1912_06127_amd as pkg
    p, f, Ws, _ = ising_n10()
    W = pkg.MPO.from_tensors(ctx, Ws)
    m = pkg.MPS.init(ctx, p["N"], 2, wl.full_rank_bonds(p["N"], 2, 32), basis_state=[0] * p["N"])
    st = pkg.tdvp1_step(ctx, m, W, 0.01, pkg.TDVPOptions(krylov_max=1, krylov_tol=1e-15))
    assert st["flags"] & 1
    with pytest.raises(pkg.TDVPError) as e:
        pkg.tdvp1_step(ctx, m, W, 0.01, pkg.TDVPOptions(krylov_max=1, krylov_tol=1e-15, strict=True))
    assert e.value.status == 6
