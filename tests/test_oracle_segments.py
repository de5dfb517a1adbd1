"""Pins of the segment-parallel 2TDVP oracle (Sec. II A, Sec. III B, Sec. III D).

The schedule's reading is pinned by: the sweep pattern of Fig. partitioning;
the time bookkeeping of Eq. proj2site (every pair forward by dt, every inner
site backward by dt, per step); the Schmidt decomposition (inverse canonical
gauge); reduction to the serial step at p = 1; exactness at full bond
dimension (every local update is then an exact exp(-i tau H) of the whole
state); and first-order convergence of the parallel result to the serial one
as dt -> 0 under truncation (Sec. III D).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import mpo as ompo
from oracle import mps as omps
from oracle import segments as seg
from oracle import spin
from oracle import tdvp as otdvp


def xxx(N, h=0.4):
    c, lam, _ = ompo.fit_exponentials(1.0 / np.arange(1, 17) ** 2.0, 3)
    Ws = ompo.mpo_exponentials(N, c, lam, spin.xxx_pairs(), spin.SX, h)
    g = ompo.eval_exponentials(c, lam, N - 1)
    return Ws, g


def test_directions_follow_partition_figure():
    # two central segments sweep away from the centre, neighbours alternate
    assert seg.directions(1, True) == [1] and seg.directions(1, False) == [-1]
    assert seg.directions(2, True) == [-1, 1]
    assert seg.directions(4, True) == [1, -1, 1, -1]
    assert seg.directions(6, True) == [-1, 1, -1, 1, -1, 1]
    d32 = seg.directions(32, True)
    assert d32[15] == -1 and d32[16] == 1
    assert all(d32[s] == -d32[s + 1] for s in range(31))
    assert seg.directions(4, False) == [-1, 1, -1, 1]
    with pytest.raises(ValueError):
        seg.directions(3, True)


@pytest.mark.parametrize("sizes", [[10], [5, 5], [3, 2, 2, 3], [2, 2, 2, 2, 2, 2], [11] + [6] * 30 + [10]])
def test_schedule_time_bookkeeping(sizes):
    """Per step every pair moves forward by dt and every site 1..N-2 backward
    by dt (Eq. proj2site); ops inside one phase touch disjoint sites."""
    N, dt = sum(sizes), 0.1
    fwd = np.zeros(N - 1)
    bwd = np.zeros(N)
    for first in (True, False):
        for ph in seg.schedule(sizes, dt, first):
            touched = []
            for op in ph.ops:
                if op.kind == "pair":
                    fwd[op.j] += op.tau
                    touched += [op.j, op.j + 1]
                else:
                    bwd[op.j] += op.tau
                    touched.append(op.j)
            assert len(touched) == len(set(touched)), ph.name
    assert np.allclose(fwd, dt, atol=1e-15)
    assert np.allclose(bwd[1:N - 1], -dt, atol=1e-15)
    assert bwd[0] == 0.0 and bwd[N - 1] == 0.0


def test_inverse_canonical_gauge_is_the_schmidt_form():
    N = 9
    T = wl.random_site_tensors(3, wl.full_rank_bonds(N, 2, 6), 2)
    Psi, V = seg.to_inverse_canonical(T)
    psi = omps.to_dense(T)
    psi = psi / np.linalg.norm(psi)  # the gauge holds the normalised state
    assert np.linalg.norm(omps.to_dense(seg.from_inverse_canonical(Psi, V)) - psi) < 1e-12
    for j in range(N - 1):
        A = Psi[j] * V[j][None, None, :]
        assert omps.is_left_orthonormal(A, 1e-12)
        B = V[j][:, None, None] * Psi[j + 1]
        if j < N - 2:
            assert omps.is_right_orthonormal(B, 1e-12)
        # 1/V_j are the Schmidt coefficients of the bipartition after site j
        s = np.linalg.svd(psi.reshape(2 ** (j + 1), -1), compute_uv=False)
        k = len(V[j])
        assert np.allclose(np.sort(1.0 / V[j])[::-1], s[:k], atol=1e-12 * s[0])
        assert np.all(s[k:] < 1e-12 * s[0])


def test_single_segment_is_the_serial_step():
    N = 10
    Ws, _ = xxx(N)
    T0 = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(11, wl.full_rank_bonds(N, 2), 2)))
    tr = otdvp.Truncation(chi_max=12, w_max=1e-8, eps=1e-12)
    st = seg.SegmentState(T0, Ws, tr)
    so = otdvp.MPSState(T0, Ws)
    for _ in range(3):
        seg.step(st, [N], 0.05)
        otdvp.tdvp2_step(so, 0.05, tr)
    assert so.stats.w_total > 1e-4  # truncation is active
    assert abs(st.stats.w_total - so.stats.w_total) < 1e-12
    assert np.linalg.norm(omps.to_dense(st.tensors()) - omps.to_dense(so.T)) < 1e-10


@pytest.mark.parametrize("sizes", [[5, 5], [3, 2, 2, 3]])
def test_full_rank_parallel_step_is_exact(sizes):
    N = 10
    Ws, g = xxx(N)
    H = spin.longrange_hamiltonian(N, g, spin.xxx_pairs(), spin.SX, 0.4)
    T0 = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(12, wl.full_rank_bonds(N, 2), 2)))
    st = seg.SegmentState(T0, Ws)
    for _ in range(4):
        seg.step(st, sizes, 0.05)
    ref = spin.ExactEvolution(H).evolve(omps.to_dense(T0), 0.2)
    assert np.linalg.norm(omps.to_dense(st.tensors()) - ref) < 1e-10


def test_parallel_error_is_first_order_in_dt():
    """With truncated bonds the out-of-date environments make the segmented
    result differ from the serial one by O(dt) at fixed final time."""
    N, Tt = 12, 0.2
    Ws, _ = xxx(N)
    T0 = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(11, wl.full_rank_bonds(N, 2, 8), 2)))
    chi = [A.shape[2] for A in T0]
    diffs = []
    for dt in (0.05, 0.025, 0.0125):
        a = seg.SegmentState(T0, Ws, chi_static=chi)
        b = seg.SegmentState(T0, Ws, chi_static=chi)
        for _ in range(round(Tt / dt)):
            seg.step(a, [N], dt)
            seg.step(b, [2] * 6, dt)
        diffs.append(np.linalg.norm(omps.to_dense(a.tensors()) - omps.to_dense(b.tensors())))
    assert diffs[0] > 1e-5  # the segments do see out-of-date environments
    assert diffs[0] / diffs[1] > 1.8 and diffs[1] / diffs[2] > 1.8
    assert all(x == y for x, y in zip([a.shape for a in b.Psi], [tuple(t.shape) for t in T0]))


def test_segment_order_does_not_change_the_result():
    N = 12
    Ws, _ = xxx(N)
    T0 = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(13, wl.full_rank_bonds(N, 2, 8), 2)))
    chi = [A.shape[2] for A in T0]
    sizes = [3, 3, 2, 4]
    a = seg.SegmentState(T0, Ws, chi_static=chi)
    b = seg.SegmentState(T0, Ws, chi_static=chi)
    for _ in range(2):
        seg.step(a, sizes, 0.05)
        seg.step(b, sizes, 0.05, order=[2, 0, 3, 1])
    for x, y in zip(a.Psi, b.Psi):
        assert np.array_equal(x, y)


def _bond_energy(st, j):
    """<psi|H|psi> contracted at bond j from beta_{j+1}, the Schmidt values and
    gamma_j; equal to the exact energy only if the gauge and the stored
    environments are both right."""
    S = 1.0 / st.V[j]
    return np.einsum("blc,b,c,blc->", st.beta[j + 1], S, S, st.gamma[j]).real


def test_reorthonormalize_restores_gauge_norm_and_environments():
    """Sec. III D, Fig. reorth: truncated parallel steps break the gauge at
    the partition boundaries and the norm drifts; reorthonormalisation
    restores both without changing the direction of the state, keeps every
    bond dimension, and the recomputed environments give the exact energy at
    every bond."""
    N = 12
    Ws, g = xxx(N)
    H = spin.longrange_hamiltonian(N, g, spin.xxx_pairs(), spin.SX, 0.4)
    H = H.toarray() if hasattr(H, "toarray") else H
    T0 = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(14, wl.full_rank_bonds(N, 2, 8), 2)))
    chi = [A.shape[2] for A in T0]
    st = seg.SegmentState(T0, Ws, chi_static=chi)
    for _ in range(3):
        seg.step(st, [3, 3, 3, 3], 0.1)
    psi = omps.to_dense(st.tensors())
    n2 = seg.norm2(st)
    assert abs(n2 - np.vdot(psi, psi).real) < 1e-12
    assert abs(n2 - 1.0) > 1e-6
    assert seg.gauge_defect(st) > 1e-6
    e_exact = np.vdot(psi, H @ psi).real / n2
    assert max(abs(_bond_energy(st, j) - e_exact) for j in range(N - 1)) > 1e-6
    shapes = [P.shape for P in st.Psi]
    seg.reorthonormalize(st)
    assert [P.shape for P in st.Psi] == shapes
    assert seg.gauge_defect(st) < 1e-12
    assert abs(seg.norm2(st) - 1.0) < 1e-13
    assert np.linalg.norm(omps.to_dense(st.tensors()) - psi / np.sqrt(n2)) < 1e-12
    for j in range(N - 1):
        assert abs(_bond_energy(st, j) - e_exact) < 1e-11
        assert abs(np.sum(st.V[j] ** -2.0) - 1.0) < 1e-13


def test_reorthonormalize_is_identity_on_a_fresh_state():
    N = 8
    Ws, _ = xxx(N)
    T0 = wl.random_site_tensors(15, wl.full_rank_bonds(N, 2, 6), 2)
    st = seg.SegmentState(T0, Ws)
    assert seg.gauge_defect(st) < 1e-12 and abs(seg.norm2(st) - 1.0) < 1e-13
    V0 = [v.copy() for v in st.V]
    psi = omps.to_dense(st.tensors())
    seg.reorthonormalize(st)
    for a, b in zip(V0, st.V):
        assert np.allclose(np.sort(a), np.sort(b), rtol=1e-11)
    assert np.linalg.norm(omps.to_dense(st.tensors()) - psi) < 1e-12


# ------------------------------------------------- one-site segment schedule

@pytest.mark.parametrize("sizes", [[10], [5, 5], [2, 3, 3, 2], [3, 4, 4, 3, 3, 3], [11] + [6] * 30 + [10]])
def test_one_site_schedule_time_bookkeeping(sizes):
    """Per step: boundary pairs forward by dt, every other site forward by dt,
    every other bond backward by dt (Eq. proj1site with the boundary terms
    merged into two-site terms); ops inside a phase touch disjoint sites."""
    N, dt = sum(sizes), 0.1
    bounds = np.cumsum(sizes)[:-1] - 1  # boundary bonds b (pairs (b, b+1))
    pair = np.zeros(N - 1)
    site = np.zeros(N)
    bond = np.zeros(N - 1)
    for first in (True, False):
        for ph in seg.schedule1(sizes, dt, first):
            touched = []
            for op in ph.ops:
                if op.kind == "pair":
                    pair[op.j] += op.tau
                    touched += [op.j, op.j + 1]
                elif op.kind == "site":
                    site[op.j] += op.tau
                    touched.append(op.j)
                else:
                    bond[op.j] += op.tau
                    touched += [op.j, op.j + 1]
            assert len(touched) == len(set(touched)), ph.name
    in_pair = set(bounds) | set(bounds + 1)
    for j in range(N):
        assert abs(site[j] - (0.0 if j in in_pair else dt)) < 1e-15, j
    for j in range(N - 1):
        if j in set(bounds):
            assert abs(pair[j] - dt) < 1e-15 and bond[j] == 0.0
        else:
            assert pair[j] == 0.0 and abs(bond[j] + dt) < 1e-15, j
    with pytest.raises(ValueError):
        seg.schedule1([3, 2, 2, 3], dt, True)  # inner segments need three sites


def test_one_site_single_segment_is_the_serial_step():
    N = 10
    Ws, _ = xxx(N)
    T0 = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(11, wl.full_rank_bonds(N, 2, 6), 2)))
    st = seg.SegmentState(T0, Ws, chi_static=[A.shape[2] for A in T0])
    so = otdvp.MPSState(T0, Ws)
    for _ in range(3):
        seg.step1(st, [N], 0.05)
        otdvp.tdvp1_step(so, 0.05)
    assert np.linalg.norm(omps.to_dense(st.tensors()) - omps.to_dense(so.T)) < 1e-12
    assert st.stats.pair_updates == 0 and st.stats.bond_updates == 6 * (N - 1)


@pytest.mark.parametrize("sizes", [[5, 5], [2, 3, 3, 2]])
def test_one_site_full_rank_parallel_step_is_exact(sizes):
    N = 10
    Ws, g = xxx(N)
    H = spin.longrange_hamiltonian(N, g, spin.xxx_pairs(), spin.SX, 0.4)
    T0 = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(12, wl.full_rank_bonds(N, 2), 2)))
    chi = [A.shape[2] for A in T0]
    st = seg.SegmentState(T0, Ws, chi_static=chi)
    for _ in range(4):
        seg.step1(st, sizes, 0.05)
    ref = spin.ExactEvolution(H).evolve(omps.to_dense(T0), 0.2)
    assert np.linalg.norm(omps.to_dense(st.tensors()) - ref) < 1e-10
    assert [P.shape[2] for P in st.Psi] == chi


def test_one_site_parallel_error_is_first_order_and_norm_tracks_boundary_weight():
    N, Tt = 12, 0.2
    Ws, _ = xxx(N)
    T0 = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(11, wl.full_rank_bonds(N, 2, 8), 2)))
    chi = [A.shape[2] for A in T0]
    diffs = []
    for dt in (0.05, 0.025, 0.0125):
        a = seg.SegmentState(T0, Ws, chi_static=chi)
        b = seg.SegmentState(T0, Ws, chi_static=chi)
        for _ in range(round(Tt / dt)):
            seg.step1(a, [N], dt)
            seg.step1(b, [3, 3, 3, 3], dt)
        diffs.append(np.linalg.norm(omps.to_dense(a.tensors()) - omps.to_dense(b.tensors())))
    assert diffs[0] > 1e-5
    assert diffs[0] / diffs[1] > 1.8 and diffs[1] / diffs[2] > 1.8
    # one-site steps conserve the norm; only the boundary splits truncate
    assert b.stats.w_total > 1e-7
    assert abs(seg.norm2(b) - (1.0 - b.stats.w_total)) < 1e-10
    assert [P.shape[2] for P in b.Psi] == chi


def test_segment_hybrid_switches_once_saturated():
    """Discussion: two-site steps while the bond dimensions can grow, the
    one-site schedule once every bond holds min(chi_max, d^min(j, N-j));
    from then on the bond dimensions stay fixed."""
    N, sizes = 12, [3, 3, 3, 3]
    Ws, _ = xxx(N)
    T0 = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(21, wl.full_rank_bonds(N, 2, 3), 2)))
    st = seg.SegmentState(T0, Ws, otdvp.Truncation(chi_max=8))
    assert not seg.saturated(st)
    ran = []
    for _ in range(4):
        ran.append(seg.hybrid_step(st, sizes, 0.05))
        if ran[-1]:
            chi = [len(v) for v in st.V]
    assert ran[0] is False and ran[-1] is True
    assert ran.index(True) >= 1 and all(ran[ran.index(True):])
    assert seg.saturated(st) and [len(v) for v in st.V] == chi
    assert max(len(v) for v in st.V) == 8


def test_one_site_segment_order_does_not_change_the_result():
    N = 13
    Ws, _ = xxx(N)
    T0 = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(17, wl.full_rank_bonds(N, 2, 8), 2)))
    chi = [A.shape[2] for A in T0]
    sizes = [3, 4, 3, 3]
    a = seg.SegmentState(T0, Ws, chi_static=chi)
    b = seg.SegmentState(T0, Ws, chi_static=chi)
    for _ in range(2):
        seg.step1(a, sizes, 0.05)
        seg.step1(b, sizes, 0.05, order=[3, 1, 0, 2])
    for x, y in zip(a.Psi, b.Psi):
        assert np.array_equal(x, y)
