"""Segment-parallel two-site TDVP on the GPU against the FP64 oracle
(Sec. II A inverse canonical gauge, Sec. III B schedule).

Bars: complex128 path 1e-10 on observables and on the state overlap,
complex64 path (FP32 MFMA matvecs) 1e-4 on observables.  Graph replay is
bitwise equal to eager execution (same kernels, deterministic reductions).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import mpo as ompo
from oracle import mps as omps
from oracle import segments as oseg
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


def xy_mpo(N, alpha=1.5, K=6):
    """Long-range XY chain (1/2 sum r^-alpha (xx + yy)), sum of K exponentials."""
    c, lam, _ = ompo.fit_exponentials(1.0 / np.arange(1, max(N - 1, 2 * K) + 1) ** alpha, K)
    pairs = [(0.5, spin.SX, spin.SX), (0.5, spin.SY, spin.SY)]
    return c, lam, pairs, ompo.mpo_exponentials(N, c, lam, pairs)


def case(N, sizes, chi_lo, chi_hi, seed):
    chi = wl.segment_bond_profile(sizes, 2, chi_lo, chi_hi, seed)
    T = wl.random_site_tensors(seed + 1, chi, 2)
    return chi, T


def sz_profile(T):
    return omps.expect_sites(T, spin.SZ).real


def test_inverse_canonical_state_matches_oracle(ctx):
    import paper_1912_06127_amd as pkg
    N, sizes = 12, [3, 3, 3, 3]
    chi, T = case(N, sizes, 4, 16, 31)
    c, lam, pairs, Ws = xy_mpo(N)
    W = pkg.MPO.from_tensors(ctx, Ws)
    sg = pkg.Segments.init(ctx, W, T, sizes, compute="c128")
    Psi, V = oseg.to_inverse_canonical(T)
    assert sg.chi == chi
    # the density-matrix split resolves s_i to ~1e-16 (s_1/s_i)^2 relative
    # (here s_1/s_min ~ 400): 1e-9
    for j in range(N - 1):
        assert np.allclose(np.sort(1.0 / sg.bond(j)), np.sort(1.0 / V[j]), rtol=1e-9, atol=0)
    Tg = sg.tensors()
    ref = omps.to_dense(T)
    ref = ref / np.linalg.norm(ref)  # the gauge holds the normalised state
    assert np.linalg.norm(omps.to_dense(Tg) - ref) <= 1e-12
    for j in range(N - 1):  # Psi_j V_j is left orthonormal (same accuracy bound)
        A = sg.psi(j) * sg.bond(j)[None, None, :]
        assert omps.is_left_orthonormal(A, 1e-9)


SEG_CASES = [
    # N, sizes, chi_lo, chi_hi, seed
    (20, [4, 3, 3, 3, 3, 4], 6, 24, 41),
    (16, [16], 4, 20, 43),
    (24, [5, 2, 3, 4, 4, 6], 8, 40, 45),
]


@pytest.mark.parametrize("batched", [True, False])
@pytest.mark.parametrize("dt_", ["c128", "c64"])
@pytest.mark.parametrize("cs", SEG_CASES, ids=lambda c: f"N{c[0]}_p{len(c[1])}")
def test_segment_steps_match_oracle(ctx, cs, dt_, batched):
    import paper_1912_06127_amd as pkg
    N, sizes, lo, hi, seed = cs
    print(f"segments N={N} sizes={sizes} {dt_} batched={batched}", flush=True)
    chi, T = case(N, sizes, lo, hi, seed)
    c, lam, pairs, Ws = xy_mpo(N)
    W = pkg.MPO.from_tensors(ctx, Ws)
    sg = pkg.Segments.init(ctx, W, T, sizes, compute=dt_)
    st_o = oseg.SegmentState(T, Ws, chi_static=chi[1:], kmax=8, tol=0.0)
    opts = pkg.SegmentOptions(compute=dt_, batched=batched)
    for s in range(2):
        oseg.step(st_o, sizes, 0.02)
        info = sg.step(W, 0.02, opts)
        assert info["matvecs"] > 0
        Tg, To = sg.tensors(), st_o.tensors()
        err = np.max(np.abs(sz_profile(Tg) - sz_profile(To)))
        assert err <= OBS_TOL[dt_], (s, err)
    assert sg.chi == chi
    if dt_ == "c128":
        ov = abs(omps.overlap(Tg, To)) / np.sqrt(omps.norm2(Tg) * omps.norm2(To))
        assert abs(ov - 1.0) <= 1e-10
        assert abs(sg.w_total - st_o.stats.w_total) <= 1e-10 * max(1.0, st_o.stats.w_total)
        for j in range(N - 1):
            assert np.allclose(np.sort(1.0 / sg.bond(j)), np.sort(1.0 / st_o.V[j]), rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("dt_", ["c128", "c64"])
def test_reorthonormalize_matches_oracle(ctx, dt_):
    """Sec. III D, Fig. reorth: after truncated parallel steps the norm has
    drifted; the repair normalises the state without changing its direction,
    restores the gauge, and the recomputed environments drive the next step
    exactly as the oracle's do."""
    import paper_1912_06127_amd as pkg
    N, sizes, lo, hi, seed = SEG_CASES[0]
    print(f"reorthonormalise N={N} {dt_}", flush=True)
    chi, T = case(N, sizes, lo, hi, seed)
    *_, Ws = xy_mpo(N)
    W = pkg.MPO.from_tensors(ctx, Ws)
    sg = pkg.Segments.init(ctx, W, T, sizes, compute=dt_)
    st_o = oseg.SegmentState(T, Ws, chi_static=chi[1:], kmax=8, tol=0.0)
    opts = pkg.SegmentOptions(compute=dt_)
    for _ in range(3):
        oseg.step(st_o, sizes, 0.05)
        sg.step(W, 0.05, opts)
    Tb = sg.tensors()
    n_gpu, n_o = sg.norm2(), oseg.norm2(st_o)
    assert abs(n_gpu - omps.norm2(Tb)) <= 1e-12  # the device transfer sum of its own state
    assert abs(n_o - 1.0) > 1e-6  # the drift is there to repair
    assert abs(n_gpu - n_o) <= OBS_TOL[dt_]
    sg.reorthonormalize(W)
    oseg.reorthonormalize(st_o)
    assert sg.chi == chi
    Ta = sg.tensors()
    assert abs(sg.norm2() - 1.0) <= 1e-12
    assert abs(omps.norm2(Ta) - 1.0) <= 1e-12
    ov = abs(omps.overlap(Tb, Ta)) / np.sqrt(omps.norm2(Tb))
    assert abs(ov - 1.0) <= 1e-12
    for j in range(N - 1):
        A = sg.psi(j) * sg.bond(j)[None, None, :]
        assert omps.is_left_orthonormal(A, 1e-9), j
        if dt_ == "c128":
            assert np.allclose(np.sort(1.0 / sg.bond(j)), np.sort(1.0 / st_o.V[j]), rtol=1e-8, atol=1e-12), j
    # the next step runs on the recomputed environments
    oseg.step(st_o, sizes, 0.05)
    sg.step(W, 0.05, opts)
    Tg, To = sg.tensors(), st_o.tensors()
    assert np.max(np.abs(sz_profile(Tg) - sz_profile(To))) <= OBS_TOL[dt_]
    if dt_ == "c128":
        ov = abs(omps.overlap(Tg, To)) / np.sqrt(omps.norm2(Tg) * omps.norm2(To))
        assert abs(ov - 1.0) <= 1e-10


ONE_SITE_CASES = [
    # N, sizes, chi_lo, chi_hi, seed
    (20, [4, 3, 3, 3, 3, 4], 6, 24, 41),
    (16, [16], 4, 20, 43),
]


@pytest.mark.parametrize("batched", [True, False])
@pytest.mark.parametrize("dt_", ["c128", "c64"])
@pytest.mark.parametrize("cs", ONE_SITE_CASES, ids=lambda c: f"N{c[0]}_p{len(c[1])}")
def test_one_site_segment_steps_match_oracle(ctx, cs, dt_, batched):
    """The one-site schedule (site steps forward, zero-site bond steps
    backward, two-site boundary pairs) against the oracle's step1."""
    import paper_1912_06127_amd as pkg
    N, sizes, lo, hi, seed = cs
    print(f"one-site segments N={N} sizes={sizes} {dt_} batched={batched}", flush=True)
    chi, T = case(N, sizes, lo, hi, seed)
    *_, Ws = xy_mpo(N)
    W = pkg.MPO.from_tensors(ctx, Ws)
    sg = pkg.Segments.init(ctx, W, T, sizes, compute=dt_)
    st_o = oseg.SegmentState(T, Ws, chi_static=chi[1:], kmax=8, tol=0.0)
    opts = pkg.SegmentOptions(compute=dt_, batched=batched, one_site=True)
    for s in range(2):
        oseg.step1(st_o, sizes, 0.02)
        info = sg.step(W, 0.02, opts)
        assert info["matvecs"] > 0
        Tg, To = sg.tensors(), st_o.tensors()
        err = np.max(np.abs(sz_profile(Tg) - sz_profile(To)))
        assert err <= OBS_TOL[dt_], (s, err)
    assert sg.chi == chi
    if dt_ == "c128":
        ov = abs(omps.overlap(Tg, To)) / np.sqrt(omps.norm2(Tg) * omps.norm2(To))
        assert abs(ov - 1.0) <= 1e-10
        assert abs(sg.w_total - st_o.stats.w_total) <= 1e-10 * max(1.0, st_o.stats.w_total)
        assert abs(sg.norm2() - oseg.norm2(st_o)) <= 1e-10


def test_one_site_then_two_site_goes_through_the_repair(ctx):
    """One-site steps leave unit V on inner bonds; a two-site step is refused
    until seg_reorthonormalize restores the Schmidt form, and the sequence
    one-site step, repair, two-site step equals the oracle's."""
    import paper_1912_06127_amd as pkg
    N, sizes, lo, hi, seed = ONE_SITE_CASES[0]
    chi, T = case(N, sizes, lo, hi, seed)
    *_, Ws = xy_mpo(N)
    W = pkg.MPO.from_tensors(ctx, Ws)
    sg = pkg.Segments.init(ctx, W, T, sizes, compute="c128")
    st_o = oseg.SegmentState(T, Ws, chi_static=chi[1:], kmax=8, tol=0.0)
    sg.step(W, 0.02, pkg.SegmentOptions(compute="c128", one_site=True))
    oseg.step1(st_o, sizes, 0.02)
    with pytest.raises(pkg.TDVPError):
        sg.step(W, 0.02, pkg.SegmentOptions(compute="c128"))
    sg.reorthonormalize(W)
    oseg.reorthonormalize(st_o)
    sg.step(W, 0.02, pkg.SegmentOptions(compute="c128"))
    oseg.step(st_o, sizes, 0.02)
    Tg, To = sg.tensors(), st_o.tensors()
    assert np.max(np.abs(sz_profile(Tg) - sz_profile(To))) <= 1e-10
    ov = abs(omps.overlap(Tg, To)) / np.sqrt(omps.norm2(Tg) * omps.norm2(To))
    assert abs(ov - 1.0) <= 1e-10
    for j in range(N - 1):
        assert np.allclose(np.sort(1.0 / sg.bond(j)), np.sort(1.0 / st_o.V[j]), rtol=1e-8, atol=1e-12), j


@pytest.mark.parametrize("sizes", [[5, 5], [3, 4]])
def test_one_site_segments_full_rank_match_exact_evolution(ctx, sizes):
    import paper_1912_06127_amd as pkg
    N = sum(sizes)
    print(f"one-site segments full rank {sizes}", flush=True)
    c, lam, pairs, Ws = xy_mpo(N)
    g = ompo.eval_exponentials(c, lam, N - 1)
    H = spin.longrange_hamiltonian(N, g, pairs)
    T = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(90, wl.full_rank_bonds(N, 2), 2)))
    psi0 = omps.to_dense(T)
    W = pkg.MPO.from_tensors(ctx, Ws)
    sg = pkg.Segments.init(ctx, W, T, sizes, compute="c128")
    for _ in range(4):
        sg.step(W, 0.05, pkg.SegmentOptions(compute="c128", krylov_k=16, one_site=True))
    ref = spin.ExactEvolution(H).evolve(psi0, 0.2)
    got = omps.to_dense(sg.tensors())
    assert abs(abs(np.vdot(ref, got)) - 1.0) < 1e-10
    assert np.linalg.norm(got - ref) < 1e-9


def test_batched_equals_instance_by_instance(ctx):
    import paper_1912_06127_amd as pkg
    N, sizes, lo, hi, seed = SEG_CASES[2]
    chi, T = case(N, sizes, lo, hi, seed)
    *_, Ws = xy_mpo(N)
    W = pkg.MPO.from_tensors(ctx, Ws)
    a = pkg.Segments.init(ctx, W, T, sizes, compute="c128")
    b = pkg.Segments.init(ctx, W, T, sizes, compute="c128")
    for _ in range(2):
        a.step(W, 0.02, pkg.SegmentOptions(compute="c128", batched=True))
        b.step(W, 0.02, pkg.SegmentOptions(compute="c128", batched=False))
    # the site tensors themselves are gauge dependent (eigenvectors inside nearly
    # degenerate groups may rotate); compare the state, its Schmidt values and
    # the spin profile
    Ta, Tb = a.tensors(), b.tensors()
    ov = abs(omps.overlap(Ta, Tb)) / np.sqrt(omps.norm2(Ta) * omps.norm2(Tb))
    assert abs(ov - 1.0) <= 1e-10
    for j in range(N - 1):
        assert np.allclose(np.sort(a.bond(j)), np.sort(b.bond(j)), rtol=1e-8, atol=0), j
    assert np.max(np.abs(sz_profile(Ta) - sz_profile(Tb))) <= 1e-10


@pytest.mark.parametrize("dt_", ["c64", "c128"])
def test_graph_replay_equals_eager(ctx, dt_):
    """Every phase's batched exponentiation captured on first use and replayed
    in later steps, with the eager splits in between; bitwise equal to eager."""
    import paper_1912_06127_amd as pkg
    N, sizes, lo, hi, seed = SEG_CASES[0]
    chi, T = case(N, sizes, lo, hi, seed)
    *_, Ws = xy_mpo(N)
    W = pkg.MPO.from_tensors(ctx, Ws)
    a = pkg.Segments.init(ctx, W, T, sizes, compute=dt_)
    b = pkg.Segments.init(ctx, W, T, sizes, compute=dt_)
    for s in range(3):
        print(f"graph step {s} {dt_}", flush=True)
        a.step(W, 0.02, pkg.SegmentOptions(compute=dt_))
        b.step(W, 0.02, pkg.SegmentOptions(compute=dt_, use_graph=True))
        for j in range(N):
            assert np.array_equal(a.psi(j), b.psi(j)), (s, j)


@pytest.mark.parametrize("batched", [True, False])
def test_segment_hybrid_switch_matches_oracle(ctx, batched):
    """one_site = "auto": two-site steps while the bonds can grow (dynamic
    shapes up to chi_max), the one-site schedule once they are saturated;
    the switch step, the bond profile and the state equal the oracle's."""
    import paper_1912_06127_amd as pkg
    N, sizes = 12, [3, 3, 3, 3]
    print(f"segment hybrid N={N} batched={batched}", flush=True)
    *_, Ws = xy_mpo(N)
    T = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(21, wl.full_rank_bonds(N, 2, 3), 2)))
    W = pkg.MPO.from_tensors(ctx, Ws)
    sg = pkg.Segments.init(ctx, W, T, sizes, compute="c128")
    st_o = oseg.SegmentState(T, Ws, otdvp.Truncation(chi_max=8), kmax=8, tol=0.0)
    # SVD splits: the new bond directions carry Schmidt values ~3e-4
    opts = pkg.SegmentOptions(compute="c128", chi_max=8, static_shapes=False, batched=batched, one_site="auto",
                              svd_mode=1)
    ran = []
    for s in range(4):
        one = oseg.hybrid_step(st_o, sizes, 0.05)
        info = sg.step(W, 0.05, opts)
        assert bool(info["flags"] & 2) == one == info["one_site"], s
        ran.append(one)
        assert sg.chi == [1] + [len(v) for v in st_o.V] + [1], s
        Tg, To = sg.tensors(), st_o.tensors()
        assert np.max(np.abs(sz_profile(Tg) - sz_profile(To))) <= 1e-10, s
    assert ran[0] is False and ran[-1] is True
    ov = abs(omps.overlap(Tg, To)) / np.sqrt(omps.norm2(Tg) * omps.norm2(To))
    assert abs(ov - 1.0) <= 1e-10


def test_one_site_graph_replay_equals_eager(ctx):
    """One-site schedule: the site exponentials of every phase replayed from
    captured graphs, the bond steps and boundary splits eager in between;
    bitwise equal to eager execution."""
    import paper_1912_06127_amd as pkg
    N, sizes, lo, hi, seed = ONE_SITE_CASES[0]
    chi, T = case(N, sizes, lo, hi, seed)
    *_, Ws = xy_mpo(N)
    W = pkg.MPO.from_tensors(ctx, Ws)
    a = pkg.Segments.init(ctx, W, T, sizes, compute="c64")
    b = pkg.Segments.init(ctx, W, T, sizes, compute="c64")
    for s in range(3):
        print(f"one-site graph step {s}", flush=True)
        a.step(W, 0.02, pkg.SegmentOptions(compute="c64", one_site=True))
        b.step(W, 0.02, pkg.SegmentOptions(compute="c64", one_site=True, use_graph=True))
        for j in range(N):
            assert np.array_equal(a.psi(j), b.psi(j)), (s, j)


def test_segment_arguments_are_checked(ctx):
    import paper_1912_06127_amd as pkg
    N = 8
    chi, T = case(N, [4, 4], 2, 8, 3)
    *_, Ws = xy_mpo(N)
    W = pkg.MPO.from_tensors(ctx, Ws)
    with pytest.raises(pkg.TDVPError):  # odd number of segments
        pkg.Segments.init(ctx, W, T, [3, 3, 2])
    with pytest.raises(pkg.TDVPError):  # sizes do not add up
        pkg.Segments.init(ctx, W, T, [4, 3])
    sg = pkg.Segments.init(ctx, W, T, [4, 4], compute="c64")
    with pytest.raises(pkg.TDVPError):  # compute dtype differs from the state's
        sg.step(W, 0.01, pkg.SegmentOptions(compute="c128"))
    with pytest.raises(pkg.TDVPError):  # graphs need static shapes
        sg.step(W, 0.01, pkg.SegmentOptions(compute="c64", static_shapes=False, use_graph=True))
    N = 10
    chi, T = case(N, [3, 2, 2, 3], 2, 8, 5)
    *_, Ws = xy_mpo(N)
    W = pkg.MPO.from_tensors(ctx, Ws)
    sg = pkg.Segments.init(ctx, W, T, [3, 2, 2, 3], compute="c64")
    with pytest.raises(pkg.TDVPError):  # one-site schedule: inner segments need three sites
        sg.step(W, 0.01, pkg.SegmentOptions(compute="c64", one_site=True))
