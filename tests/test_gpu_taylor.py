"""The truncated-Taylor exponential action (Al-Mohy and Higham 2011; the
alternative to Lanczos named in Sec. III A) inside the device TDVP steps,
against exact evolution and the FP64 oracle.

Bars: complex128 1e-9 on the state at full bond dimension (as the Lanczos
path), 1e-10 on observables against the oracle; complex64 1e-4.
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


def xxx(N, K=3, h=0.0):
    c, lam, _ = ompo.fit_exponentials(1.0 / np.arange(1, max(N, 2 * K + 1)) ** 2.0, K)
    g = ompo.eval_exponentials(c, lam, N - 1)
    H = spin.longrange_hamiltonian(N, g, spin.xxx_pairs(), spin.SX, h)
    return c, lam, H


@pytest.mark.parametrize("N,two_site,dt,steps", [
    (8, False, 0.05, 5),
    (8, True, 0.05, 5),
    (8, False, 4.0, 1),   # |tau| rho above theta_55: several scaling steps
    (3, True, 0.3, 2),    # the shortest chain: the turning-point pair is the whole sweep
])
def test_taylor_full_rank_matches_exact_evolution(ctx, N, two_site, dt, steps):
    import paper_1912_06127_amd as pkg
    print(f"taylor full rank N={N} two_site={two_site} dt={dt}", flush=True)
    c, lam, H = xxx(N, h=0.3)
    T = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(70 + N, wl.full_rank_bonds(N, 2), 2)))
    m = pkg.MPS.from_tensors(ctx, T)
    W = pkg.MPO.longrange(ctx, N, spin.xxx_pairs(), c=c, lam=lam, onsite=spin.SX, h=0.3)
    step = pkg.tdvp2_step if two_site else pkg.tdvp1_step
    opts = pkg.TDVPOptions(exp_method="taylor")
    for _ in range(steps):
        st = step(ctx, m, W, dt, opts)
        assert st["matvecs"] > 0 and st["flags"] == 0
    psi = spin.ExactEvolution(H).evolve(omps.to_dense(T), dt * steps)
    assert np.linalg.norm(omps.to_dense(m.tensors()) - psi) < 1e-9


@pytest.mark.parametrize("dt_", ["c128", "c64"])
def test_taylor_truncated_tdvp2_matches_oracle(ctx, dt_):
    """Neel quench with truncation against the oracle's Lanczos-based run:
    both evaluate the same exp(-i tau H_eff) Theta to ~1e-13."""
    import paper_1912_06127_amd as pkg
    N = 10
    print(f"taylor truncated tdvp2 N={N} {dt_}", flush=True)
    c, lam, _ = xxx(N)
    Ws = ompo.mpo_exponentials(N, c, lam, spin.xxx_pairs())
    bits = [i % 2 for i in range(N)]
    bits[N // 2 - 1] ^= 1
    st_o = otdvp.MPSState(omps.padded_product_state(bits, [1] * (N + 1)), Ws)
    tr = otdvp.Truncation(chi_max=12, w_max=1e-8, eps=1e-12)
    W = pkg.MPO.longrange(ctx, N, spin.xxx_pairs(), c=c, lam=lam)
    m = pkg.MPS.init(ctx, N, 2, [1] * (N + 1), basis_state=bits)
    opts = pkg.TDVPOptions(compute=dt_, chi_max=12, w_max=1e-8, eps_rel=1e-12, exp_method="taylor")
    for s in range(8):
        otdvp.tdvp2_step(st_o, 0.05, tr)
        st = pkg.tdvp2_step(ctx, m, W, 0.05, opts)
        z = pkg.expect(ctx, m, list(range(N)), spin.SZ).real
        zref = omps.expect_sites(st_o.T, spin.SZ).real
        assert np.max(np.abs(z - zref)) <= OBS_TOL[dt_], (s, np.max(np.abs(z - zref)))
    if dt_ == "c128":
        assert m.chi == [1] + [A.shape[2] for A in st_o.T]
        assert abs(st["w_total"] - st_o.stats.w_total) <= 1e-12


def test_taylor_and_lanczos_steps_agree(ctx):
    """The two exponential methods on the same truncated run (c128)."""
    import paper_1912_06127_amd as pkg
    N = 12
    c, lam, _ = xxx(N)
    W = pkg.MPO.longrange(ctx, N, spin.xxx_pairs(), c=c, lam=lam)
    T = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(81, wl.full_rank_bonds(N, 2, 10), 2)))
    a = pkg.MPS.from_tensors(ctx, T)
    b = pkg.MPS.from_tensors(ctx, T)
    mv = {"lanczos": 0, "taylor": 0}
    for _ in range(4):
        for m, meth in ((a, "lanczos"), (b, "taylor")):
            st = pkg.tdvp2_step(ctx, m, W, 0.05, pkg.TDVPOptions(chi_max=10, w_max=1e-9, exp_method=meth))
            mv[meth] += st["matvecs"]
    Ta, Tb = a.tensors(), b.tensors()
    ov = abs(omps.overlap(Ta, Tb)) / np.sqrt(omps.norm2(Ta) * omps.norm2(Tb))
    print(f"matvecs over 4 steps: {mv}", flush=True)
    assert abs(ov - 1.0) <= 1e-10
    assert a.chi == b.chi


def test_taylor_imaginary_time_full_rank_matches_normalised_exp(ctx):
    import scipy.linalg as sla
    import paper_1912_06127_amd as pkg
    N = 8
    c, lam = ompo.fit_exponentials(1.0 / np.arange(1, N) ** 2.0, 3)[:2]
    g = ompo.eval_exponentials(c, lam, N - 1)
    H = spin.longrange_hamiltonian(N, g, spin.xxx_pairs(), spin.SZ, 0.1)
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    T = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(61, wl.full_rank_bonds(N, 2), 2)))
    W = pkg.MPO.longrange(ctx, N, spin.xxx_pairs(), c=c, lam=lam, onsite=spin.SZ, h=0.1)
    m = pkg.MPS.from_tensors(ctx, T)
    opts = pkg.TDVPOptions(imaginary=True, exp_method="taylor")
    for _ in range(5):
        pkg.tdvp2_step(ctx, m, W, 0.1, opts)
    ref = sla.expm(-0.5 * Hd) @ omps.to_dense(T)
    ref /= np.linalg.norm(ref)
    assert np.linalg.norm(omps.to_dense(m.tensors()) - ref) < 1e-9
    assert abs(pkg.norm2(ctx, m) - 1.0) < 1e-12
