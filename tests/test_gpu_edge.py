"""Degenerate and boundary cases of the device path against exact
diagonalisation and the oracle: the shortest chains (the turning-point pair is
the whole sweep), a spin-1 chain (local dimension 3), the zero local state,
empty and single-problem batches, and the smallest segment partition."""
import numpy as np
import pytest

import workloads as wl
from oracle import heff as oheff
from oracle import mpo as ompo
from oracle import mps as omps
from oracle import spin
from tests.adapters import L_from_beta, R_from_gamma, rel_err

pytestmark = pytest.mark.gpu

SZ1 = np.diag([1.0, 0.0, -1.0]).astype(np.complex128)
SX1 = (np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]]) / np.sqrt(2)).astype(np.complex128)
SY1 = (np.array([[0, -1j, 0], [1j, 0, -1j], [0, 1j, 0]]) / np.sqrt(2)).astype(np.complex128)


@pytest.fixture(scope="module")
def ctx():
    import paper_1912_06127_amd as pkg
    c = pkg.Context(0)
    yield c
    c.sync()
    c.close()


def _t(x, dt="c128"):
    import torch
    tdt = torch.complex64 if dt == "c64" else torch.complex128
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=tdt)


@pytest.mark.parametrize("N", [2, 3, 4])
def test_tdvp2_shortest_chains_match_exact_evolution(ctx, N):
    import paper_1912_06127_amd as pkg
    f = lambda r: 1.0 / r ** 2
    pairs = spin.xxx_pairs()
    coupling = [f(r) for r in range(1, N)]
    W = pkg.MPO.longrange(ctx, N, pairs, coupling=coupling, onsite=spin.SX, h=0.3)
    H = spin.longrange_hamiltonian(N, f, pairs, spin.SX, 0.3)
    T = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(40 + N, wl.full_rank_bonds(N, 2), 2)))
    m = pkg.MPS.from_tensors(ctx, T)
    print(f"tdvp2 N={N}", flush=True)
    for _ in range(4):
        pkg.tdvp2_step(ctx, m, W, 0.05, pkg.TDVPOptions())
    ref = spin.ExactEvolution(H).evolve(omps.to_dense(T), 0.2)
    assert np.linalg.norm(omps.to_dense(m.tensors()) - ref) < 1e-10


@pytest.mark.parametrize("dt_", ["c128", "c64"])
def test_spin_one_chain_matches_exact_evolution(ctx, dt_):
    """Local dimension 3: long-range spin-1 XXZ-type chain, full-rank 1TDVP is exact."""
    import paper_1912_06127_amd as pkg
    N = 5
    pairs = [(1.0, SX1, SX1), (1.0, SY1, SY1), (0.7, SZ1, SZ1)]
    c, lam, _ = ompo.fit_exponentials(1.0 / np.arange(1, 17) ** 1.5, 3)
    g = ompo.eval_exponentials(c, lam, N - 1)
    W = pkg.MPO.longrange(ctx, N, pairs, c=c, lam=lam, onsite=SZ1, h=0.2)
    Ws = ompo.mpo_exponentials(N, c, lam, pairs, SZ1, 0.2)
    for j in range(N):
        assert np.max(np.abs(W.tensor(j) - Ws[j])) < 1e-14
    H = spin.longrange_hamiltonian(N, g, pairs, SZ1, 0.2)
    T = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(77, wl.full_rank_bonds(N, 3), 3)))
    m = pkg.MPS.from_tensors(ctx, T)
    print(f"spin-1 N={N} {dt_}", flush=True)
    for _ in range(5):
        pkg.tdvp1_step(ctx, m, W, 0.04, pkg.TDVPOptions(compute=dt_))
    psi = spin.ExactEvolution(H).evolve(omps.to_dense(T), 0.2)
    Z = [spin.site_op(SZ1, i, N) for i in range(1, N + 1)]
    z = pkg.expect(ctx, m, list(range(N)), SZ1).real
    zref = np.array([spin.expval(psi, Zi).real for Zi in Z])
    assert np.max(np.abs(z - zref)) <= (1e-10 if dt_ == "c128" else 1e-4)
    if dt_ == "c128":
        assert np.linalg.norm(omps.to_dense(m.tensors()) - psi) < 1e-10


def test_apply_heff_zero_state_and_trivial_batches(ctx):
    import torch
    import paper_1912_06127_amd as pkg
    rng = np.random.default_rng(5)
    chil, chir, w = 9, 7, 4
    beta = wl.cgauss(rng, (chil, w, chil))
    gamma = wl.cgauss(rng, (chir, w, chir))
    W1 = wl.cgauss(rng, (w, w, 2, 2))
    theta = np.zeros((chil, 2, 2, chir), dtype=np.complex128)
    L, R = _t(L_from_beta(beta)), _t(R_from_gamma(gamma))
    y = pkg.apply_heff(ctx, L, R, _t(theta), _t(W1), _t(W1))
    ctx.sync()
    assert torch.count_nonzero(y).item() == 0
    assert pkg.apply_heff_batched(ctx, []) == []
    theta = wl.cgauss(rng, (chil, 2, 2, chir))
    (yb,) = pkg.apply_heff_batched(ctx, [(L, R, _t(theta), _t(W1), _t(W1))])
    ref = oheff.apply_heff2(beta, W1, W1, gamma, theta)
    assert rel_err(yb.cpu().numpy(), ref) <= 1e-12


def test_smallest_segment_partition_is_exact_at_full_rank(ctx):
    """Two segments of two sites: every boundary rule at once; full rank is exact."""
    import paper_1912_06127_amd as pkg
    N = 4
    pairs = [(0.5, spin.SX, spin.SX), (0.5, spin.SY, spin.SY)]
    f = lambda r: 1.0 / r ** 1.5
    coupling = [f(r) for r in range(1, N)]
    W = pkg.MPO.longrange(ctx, N, pairs, coupling=coupling, onsite=spin.SZ, h=0.4)
    H = spin.longrange_hamiltonian(N, f, pairs, spin.SZ, 0.4)
    T = wl.random_site_tensors(13, wl.full_rank_bonds(N, 2), 2)
    psi0 = omps.to_dense(T)
    psi0 = psi0 / np.linalg.norm(psi0)
    sg = pkg.Segments.init(ctx, W, T, [2, 2], compute="c128")
    for _ in range(3):
        sg.step(W, 0.05, pkg.SegmentOptions(compute="c128", krylov_k=16))
    ref = spin.ExactEvolution(H).evolve(psi0, 0.15)
    got = omps.to_dense(sg.tensors())
    assert abs(abs(np.vdot(ref, got)) - 1.0) < 1e-10
