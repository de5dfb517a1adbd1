"""The one-site segment schedule and the serial repair at the full N = 201
segment workload (32 segments 11 | 6 x 30 | 10, chi up to ~1000, w = 14,
complex64 matvecs), checked through properties that hold at any size: the
one-site step keeps every bond dimension, a two-site step is refused until
the repair, and the repair brings the norm back to one without changing a
bond dimension (Sec. III D, Fig. reorth)."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def test_one_site_step_and_repair_at_full_size():
    import paper_1912_06127_amd as pkg
    p = wl.XY_N201
    N, sizes = p["N"], p["segments"]
    chi = wl.segment_bond_profile(sizes, 2, p["chi_lo"], p["chi_hi"], p["seed_chi"])
    T = wl.random_site_tensors(p["seed_state"], chi, 2)
    ctx = pkg.Context(0)
    try:
        c, lam, _ = pkg.fit.fit_power_law(p["alpha"], p["K"], N - 1)
        sx, sy = (np.array(q, dtype=np.complex128) for q in (pkg.PAULI_X, pkg.PAULI_Y))
        mpo = pkg.MPO.longrange(ctx, N, [(0.5, sx, sx), (0.5, sy, sy)], c=c, lam=lam)
        print(f"full-size segments N={N}: init", flush=True)
        sg = pkg.Segments.init(ctx, mpo, T, sizes, compute="c64")
        del T
        n0 = sg.norm2()
        assert abs(n0 - 1.0) <= 1e-12
        print("one-site step", flush=True)
        st = sg.step(mpo, p["dt"], pkg.SegmentOptions(one_site=True))
        assert st["flags"] & 2 and st["matvecs"] > 0
        assert sg.chi == chi
        n1 = sg.norm2()
        assert np.isfinite(n1) and 0.0 < n1 <= 1.0 + 1e-6
        with pytest.raises(pkg.TDVPError):
            sg.step(mpo, p["dt"], pkg.SegmentOptions())
        print("repair", flush=True)
        sg.reorthonormalize(mpo)
        assert sg.chi == chi
        assert abs(sg.norm2() - 1.0) <= 1e-12
        sg.close()
        mpo.close()
    finally:
        ctx.sync()
        ctx.close()
