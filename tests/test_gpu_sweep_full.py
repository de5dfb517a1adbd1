"""The N=64 two-site TDVP quench at full size (the workload bench.py times:
1/r^2 XXX fitted with K = 6 exponentials, w = 20, Neel state with site 32
flipped, dt = 0.05, 40 steps, w_max = 1e-8, eps = 1e-12, chi_max = 512)
against the oracle's run of the same steps (Sec. IV, Eq. HaldaneHamiltonian).

Bars: complex128 spin profile within 1e-10 and discarded weight within 1e-9
relative of the oracle, same bond dimensions; complex64 contractions (FP64
Lanczos and splits) spin profile within 1e-4.
"""
import numpy as np
import pytest

from oracle import mpo as ompo
from oracle import mps as omps
from oracle import spin
from oracle import tdvp as otdvp

pytestmark = pytest.mark.gpu

N, STEPS, DT = 64, 40, 0.05


@pytest.fixture(scope="module")
def oracle_run():
    print("oracle N=64 quench, 40 steps", flush=True)
    c, lam, _ = ompo.fit_exponentials(np.arange(1, N, dtype=float) ** -2.0, 6)
    Ws = ompo.mpo_exponentials(N, c, lam, spin.xxx_pairs())
    bits = [j % 2 for j in range(N)]
    bits[31] ^= 1
    st = otdvp.MPSState(omps.padded_product_state(bits, [1] * (N + 1)), Ws)
    tr = otdvp.Truncation(chi_max=512, w_max=1e-8, eps=1e-12)
    for s in range(STEPS):
        otdvp.tdvp2_step(st, DT, tr, tol=1e-10)
        if s % 10 == 9:
            print(f"oracle step {s + 1}", flush=True)
    z = omps.expect_sites(st.T, spin.SZ).real
    return c, lam, bits, z, st.stats.w_total, [1] + [A.shape[2] for A in st.T]


@pytest.fixture(scope="module")
def ctx():
    import paper_1912_06127_amd as pkg
    cx = pkg.Context(0)
    yield cx
    cx.sync()
    cx.close()


@pytest.mark.parametrize("dt_", ["c128", "c64"])
def test_n64_quench_matches_oracle(ctx, oracle_run, dt_):
    import paper_1912_06127_amd as pkg
    c, lam, bits, zref, wref, chiref = oracle_run
    print(f"library N=64 quench {dt_}", flush=True)
    W = pkg.MPO.longrange(ctx, N, spin.xxx_pairs(), c=c, lam=lam)
    m = pkg.MPS.init(ctx, N, 2, [1] * (N + 1), basis_state=bits)
    opts = pkg.TDVPOptions(compute=dt_, chi_max=512, w_max=1e-8, eps_rel=1e-12, krylov_max=40, krylov_tol=1e-10)
    for _ in range(STEPS):
        st = pkg.tdvp2_step(ctx, m, W, DT, opts)
    z = pkg.expect(ctx, m, list(range(N)), spin.SZ).real
    if dt_ == "c128":
        assert np.max(np.abs(z - zref)) < 1e-10
        assert abs(st["w_total"] - wref) < 1e-9 * wref
        assert m.chi == chiref
    else:
        assert np.max(np.abs(z - zref)) < 1e-4
    W.close()
    m.close()
