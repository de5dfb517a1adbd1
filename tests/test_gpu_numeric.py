"""Failure detection for non-finite values (Sec. III D: the paper tracks the
norm and the discarded weight to detect a run going wrong; here a NaN or Inf
anywhere in a step must stop it with TDVP_E_NUMERIC instead of propagating).
The non-finite value is planted from the host in an input tensor; every
kernel runs to completion (NaN arithmetic does not trap)."""
import numpy as np
import pytest

import workloads as wl
from oracle import mpo as ompo
from oracle import spin

pytestmark = pytest.mark.gpu

E_NUMERIC = 7


@pytest.fixture(scope="module")
def ctx():
    import paper_1912_06127_amd as pkg
    c = pkg.Context(0)
    yield c
    c.sync()
    c.close()


def _mpo(N, poison=None):
    c, lam, _ = ompo.fit_exponentials(1.0 / np.arange(1, 17) ** 2.0, 3)
    Ws = [W.copy() for W in ompo.mpo_exponentials(N, c, lam, spin.xxx_pairs(), spin.SX, 0.4)]
    if poison is not None:
        Ws[N // 2][1, 1, 0, 0] = poison
    return Ws


@pytest.mark.parametrize("compute", ["c128", "c64"])
@pytest.mark.parametrize("poison", [np.nan, np.inf])
@pytest.mark.parametrize("two_site", [False, True])
def test_nonfinite_mpo_entry_is_reported(ctx, compute, poison, two_site):
    import paper_1912_06127_amd as pkg
    N = 8
    print(f"non-finite MPO entry {poison} {compute} two_site={two_site}", flush=True)
    mps = pkg.MPS.init(ctx, N, 2, wl.full_rank_bonds(N, 2, 8), seed=3)
    W = pkg.MPO.from_tensors(ctx, _mpo(N, poison))
    opts = pkg.TDVPOptions(compute=compute, chi_max=8)
    step = pkg.tdvp2_step if two_site else pkg.tdvp1_step
    with pytest.raises(pkg.TDVPError) as e:
        step(ctx, mps, W, 0.05, opts)
    assert e.value.status == E_NUMERIC, str(e.value)
    # the context stays usable: a finite MPO steps normally afterwards
    mps2 = pkg.MPS.init(ctx, N, 2, wl.full_rank_bonds(N, 2, 8), seed=3)
    st = step(ctx, mps2, pkg.MPO.from_tensors(ctx, _mpo(N)), 0.05, opts)
    assert st["matvecs"] > 0


@pytest.mark.parametrize("compute", ["c128", "c64"])
def test_nonfinite_state_is_reported(ctx, compute):
    import paper_1912_06127_amd as pkg
    N = 8
    mps = pkg.MPS.init(ctx, N, 2, wl.full_rank_bonds(N, 2, 8), seed=4)
    A = mps.tensor(0)
    A[0, 1, 0] = np.nan
    mps.set_tensor(0, A)
    with pytest.raises(pkg.TDVPError) as e:
        pkg.tdvp1_step(ctx, mps, pkg.MPO.from_tensors(ctx, _mpo(N)), 0.05, pkg.TDVPOptions(compute=compute))
    assert e.value.status == E_NUMERIC, str(e.value)


@pytest.mark.parametrize("compute", ["c128", "c64"])
def test_nonfinite_mpo_entry_is_reported_by_the_segment_step(ctx, compute):
    """Segment runs check a device flag set by the batched Krylov kernels."""
    import paper_1912_06127_amd as pkg
    N, sizes = 12, [3, 3, 3, 3]
    chi = wl.segment_bond_profile(sizes, 2, 4, 16, 31)
    T = wl.random_site_tensors(32, chi, 2)
    W = pkg.MPO.from_tensors(ctx, _mpo(N, np.nan))
    sg = pkg.Segments.init(ctx, W, T, sizes, compute=compute)
    with pytest.raises(pkg.TDVPError) as e:
        sg.step(W, 0.02, pkg.SegmentOptions(compute=compute))
    assert e.value.status == E_NUMERIC, str(e.value)
    sg.close()


def test_nonfinite_state_is_reported_by_the_segment_init(ctx):
    import paper_1912_06127_amd as pkg
    N, sizes = 12, [3, 3, 3, 3]
    chi = wl.segment_bond_profile(sizes, 2, 4, 16, 31)
    T = wl.random_site_tensors(33, chi, 2)
    T[5][0, 0, 0] = np.nan
    W = pkg.MPO.from_tensors(ctx, _mpo(N))
    with pytest.raises(pkg.TDVPError) as e:
        pkg.Segments.init(ctx, W, T, sizes, compute="c128")
    assert e.value.status == E_NUMERIC, str(e.value)
