"""Two-site DMRG sweeps of the library against exact diagonalisation and the
oracle's DMRG (the ground states the quench experiments of Sec. IV start
from; same environments, H_eff and splits as 2TDVP, Sec. III A).

Bars: complex128 energy within 1e-10 of the exact ground energy and state
fidelity within 1e-9; complex64 (FP32 MFMA matvecs, FP64 Lanczos) energy
within 1e-5 relative; truncated runs match the oracle sweep by sweep to 1e-8.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import dmrg as odmrg
from oracle import mpo as ompo
from oracle import mps as omps
from oracle import spin
from oracle import tdvp as otdvp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1912_06127_amd as pkg
    c = pkg.Context(0)
    yield c
    c.sync()
    c.close()


def _canonical(seed, N, cap):
    T = wl.random_site_tensors(seed, wl.full_rank_bonds(N, 2, cap), 2)
    return omps.normalize_centre(omps.right_canonicalize(T))


@pytest.mark.parametrize("dt_", ["c128", "c64"])
def test_dmrg_ising_n10_reaches_exact_ground_state(ctx, dt_):
    import paper_1912_06127_amd as pkg
    p = wl.ISING_N10
    N = p["N"]
    f = lambda r: p["J"] / r ** p["alpha"]
    print(f"dmrg Ising N={N} {dt_}", flush=True)
    H = spin.longrange_hamiltonian(N, f, spin.ising_pairs(), spin.SX, p["h"])
    w, V = np.linalg.eigh(H)
    E0, psi0 = w[0], V[:, 0]
    W = pkg.MPO.longrange(ctx, N, spin.ising_pairs(), coupling=[f(r) for r in range(1, N)], onsite=spin.SX, h=p["h"])
    m = pkg.MPS.from_tensors(ctx, _canonical(5, N, 6))
    opts = pkg.TDVPOptions(compute=dt_, chi_max=32, eps_rel=1e-14, krylov_max=40,
                           krylov_tol=1e-12 if dt_ == "c128" else 1e-6)
    for _ in range(5):
        st = pkg.dmrg2_sweep(ctx, m, W, opts)
    E = st["energy"]
    if dt_ == "c128":
        assert abs(E - E0) < 1e-10
        psi = omps.to_dense(m.tensors())
        assert 1.0 - abs(np.vdot(psi0, psi)) < 1e-9
        assert abs(pkg.norm2(ctx, m) - 1.0) < 1e-12
        assert abs(pkg.energy(ctx, m, W).real - E0) < 1e-10
    else:
        assert abs(E - E0) < 1e-5 * abs(E0)


def test_dmrg_truncated_matches_oracle_sweep_by_sweep(ctx):
    import paper_1912_06127_amd as pkg
    N = 10
    print(f"dmrg truncated XXX N={N}", flush=True)
    c, lam, _ = ompo.fit_exponentials(1.0 / np.arange(1, N) ** 2.0, 3)
    Ws = ompo.mpo_exponentials(N, c, lam, spin.xxx_pairs(), spin.SZ, 0.1)
    T0 = _canonical(9, N, 3)
    st_o = otdvp.MPSState(T0, Ws)
    tr = otdvp.Truncation(chi_max=4, eps=1e-14)
    W = pkg.MPO.longrange(ctx, N, spin.xxx_pairs(), c=c, lam=lam, onsite=spin.SZ, h=0.1)
    m = pkg.MPS.from_tensors(ctx, T0)
    opts = pkg.TDVPOptions(compute="c128", chi_max=4, eps_rel=1e-14, krylov_max=40, krylov_tol=1e-12)
    for s in range(3):
        e_o = odmrg.dmrg2_sweep(st_o, tr)
        e_g = pkg.dmrg2_sweep(ctx, m, W, opts)["energy"]
        assert abs(e_g - e_o) < 1e-8, (s, e_g, e_o)
    assert m.chi == [1] + [A.shape[2] for A in st_o.T]
    e_ref = omps.mpo_expectation(st_o.T, Ws).real
    assert abs(pkg.energy(ctx, m, W).real - e_ref) < 1e-8
