"""Run-to-run determinism of the library (no oracle involved): the same call
on the same inputs gives bitwise the same output.  Every reduction in the
kernels has a fixed order (split-K partial sums reduced in a fixed order,
per-instance Lanczos reductions in fixed chunks), so repeated H_eff
applications, batched applications and whole time steps must agree to the
last bit; the concurrent split lanes of a segment step touch disjoint
tensors, so 8 lanes must equal 1 lane bitwise (a data race between lanes
would show up here)."""
import numpy as np
import pytest

import workloads as wl
from oracle import spin
from tests.adapters import L_from_beta, R_from_gamma

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1912_06127_amd as pkg
    c = pkg.Context(0)
    yield c
    c.sync()
    c.close()


def _t(x, dt):
    import torch
    tdt = torch.complex64 if dt == "c64" else torch.complex128
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=tdt)


def _inputs(seed, nsite, chil, chir, d, w):
    rng = np.random.default_rng(seed)
    beta = wl.cgauss(rng, (chil, w, chil))
    gamma = wl.cgauss(rng, (chir, w, chir))
    W1 = wl.cgauss(rng, (w, w, d, d))
    W2 = wl.cgauss(rng, (w, w, d, d)) if nsite == 2 else None
    theta = wl.cgauss(rng, (chil,) + (d,) * nsite + (chir,))
    return L_from_beta(beta), W1, W2, R_from_gamma(gamma), theta


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("cfg,ks", [(None, None), (12, 3), (13, 1), (16, 2)])
def test_apply_heff_repeats_bitwise(ctx, dt, cfg, ks, monkeypatch):
    import paper_1912_06127_amd as pkg
    if cfg is not None:
        if dt == "c128" and cfg == 13:
            cfg = 2
        monkeypatch.setenv("TDVP_GEMM_CFG", str(cfg))
        monkeypatch.setenv("TDVP_GEMM_KSPLIT", str(ks))
    for nsite, chil, chir in ((2, 150, 131), (1, 97, 64)):
        print(f"repeat apply_heff {dt} cfg {cfg} ks {ks} nsite {nsite}", flush=True)
        L, W1, W2, R, th = _inputs(chil + nsite, nsite, chil, chir, 2, 7)
        args = (_t(L, dt), _t(R, dt), _t(th, dt), _t(W1, dt), None if W2 is None else _t(W2, dt))
        y0 = pkg.apply_heff(ctx, *args)
        y1 = pkg.apply_heff(ctx, *args)
        ctx.sync()
        assert bool((y0 == y1).all())


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_apply_heff_batched_repeats_bitwise(ctx, dt):
    import paper_1912_06127_amd as pkg
    probs = []
    for i, (nsite, chil, chir, w) in enumerate([(2, 150, 130, 7), (1, 200, 170, 9), (2, 37, 45, 5), (0, 96, 96, 8)]):
        L, W1, W2, R, th = _inputs(40 + i, max(nsite, 1), chil, chir, 2, w)
        if nsite == 0:
            probs.append((_t(L, dt), _t(R, dt), _t(np.ascontiguousarray(th[:, 0, :]), dt), None, None))
        else:
            probs.append((_t(L, dt), _t(R, dt), _t(th, dt), _t(W1, dt), None if W2 is None else _t(W2, dt)))
    print(f"repeat apply_heff_batched {dt}", flush=True)
    a = pkg.apply_heff_batched(ctx, probs)
    b = pkg.apply_heff_batched(ctx, probs)
    ctx.sync()
    for x, y in zip(a, b):
        assert bool((x == y).all())


@pytest.mark.parametrize("dt_", ["c64", "c128"])
def test_tdvp2_steps_repeat_bitwise(ctx, dt_):
    """Two copies of the same state through the same truncated 2TDVP steps
    (adaptive Lanczos, density-matrix splits, environment updates)."""
    import paper_1912_06127_amd as pkg
    from oracle import mpo as ompo
    N = 12
    c, lam, _ = ompo.fit_exponentials(1.0 / np.arange(1, N) ** 2.0, 3)
    W = pkg.MPO.longrange(ctx, N, spin.xxx_pairs(), c=c, lam=lam)
    bits = [i % 2 for i in range(N)]
    bits[N // 2] ^= 1
    opts = pkg.TDVPOptions(compute=dt_, chi_max=16, w_max=1e-8, eps_rel=1e-12)
    a = pkg.MPS.init(ctx, N, 2, [1] * (N + 1), basis_state=bits)
    b = pkg.MPS.init(ctx, N, 2, [1] * (N + 1), basis_state=bits)
    for s in range(6):
        print(f"repeat tdvp2 step {s} {dt_}", flush=True)
        sa = pkg.tdvp2_step(ctx, a, W, 0.05, opts)
        sb = pkg.tdvp2_step(ctx, b, W, 0.05, opts)
        assert sa["w_total"] == sb["w_total"] and sa["matvecs"] == sb["matvecs"]
    assert a.chi == b.chi
    for j in range(N):
        assert np.array_equal(a.tensor(j), b.tensor(j)), j


@pytest.mark.parametrize("dt_", ["c64", "c128"])
def test_segment_step_eight_lanes_equal_one_lane(ctx, dt_, monkeypatch):
    import paper_1912_06127_amd as pkg
    from oracle import mpo as ompo
    from oracle import mps as omps
    N, sizes = 24, [5, 6, 7, 6]
    c, lam, _ = ompo.fit_exponentials(1.0 / np.arange(1, N) ** 1.5, 3)
    Ws = ompo.mpo_exponentials(N, c, lam, spin.xy_pairs())
    chi = wl.full_rank_bonds(N, 2, 24)
    T = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(77, chi, 2)))
    W = pkg.MPO.from_tensors(ctx, Ws)
    runs = []
    for lanes in ("1", "8"):
        monkeypatch.setenv("TDVP_SEG_LANES", lanes)
        sg = pkg.Segments.init(ctx, W, T, sizes, compute=dt_)
        for s in range(2):
            print(f"segment step {s} lanes {lanes} {dt_}", flush=True)
            sg.step(W, 0.02, pkg.SegmentOptions(compute=dt_))
        runs.append([sg.psi(j) for j in range(N)])
    for j in range(N):
        assert np.array_equal(runs[0][j], runs[1][j]), j

