"""The allocation-free H_eff entry point (apply_heff_noalloc) against the
allocating one (apply_heff), through the C ABI: two calls in a row, the second
on a smaller problem (the shared scratch keeps the first call's contents), and
the same bar as the apply_heff parity tests (1e-12 relative in complex128,
1e-5 in complex64).  A problem beyond the scratch limit is refused before any
work is queued.  Every call also leaves torch's allocator untouched."""
import numpy as np
import pytest

import workloads as wl
from tests.adapters import rel_err

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}


def _case(seed, nsite, chil, chir, d, w, dt):
    import torch
    tdt = torch.complex64 if dt == "c64" else torch.complex128
    rng = np.random.default_rng(seed)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=tdt)
    L = t(wl.cgauss(rng, (w, chil, chil)))
    R = t(wl.cgauss(rng, (w, chir, chir)))
    shape = {0: (chil, chir), 1: (chil, d, chir), 2: (chil, d, d, chir)}[nsite]
    theta = t(wl.cgauss(rng, shape))
    W1 = t(wl.cgauss(rng, (w, w, d, d))) if nsite >= 1 else None
    W2 = t(wl.cgauss(rng, (w, w, d, d))) if nsite == 2 else None
    return L, R, theta, W1, W2


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("nsite", [2, 1, 0])
def test_noalloc_equals_apply_heff_twice(dt, nsite):
    import torch
    import paper_1912_06127_amd as pkg
    ctx = pkg.Context(0)
    try:
        # first call spans several GEMM tiles and a ragged tail; the second is
        # smaller (and the fused small-bond path for two sites)
        for seed, chil, chir in ((1, 150, 131), (2, 29, 23)):
            print(f"noalloc nsite={nsite} {dt} chil={chil} chir={chir}", flush=True)
            if nsite == 0:
                chir = chil
            L, R, theta, W1, W2 = _case(seed + 10 * nsite, nsite, chil, chir, 2, 6, dt)
            ref = pkg.apply_heff(ctx, L, R, theta, W1, W2)
            out = torch.full_like(theta, float("nan"))
            torch.cuda.synchronize()
            before = torch.cuda.memory_stats()["allocation.all.allocated"]
            pkg.apply_heff(ctx, L, R, theta, W1, W2, out=out, noalloc=True)
            ctx.sync()
            assert torch.cuda.memory_stats()["allocation.all.allocated"] == before
            a = out.cpu().to(torch.complex128).numpy()
            b = ref.cpu().to(torch.complex128).numpy()
            assert np.all(np.isfinite(a))
            assert rel_err(a, b) <= TOL[dt], (chil, chir, rel_err(a, b))
    finally:
        ctx.close()


def test_noalloc_rejects_problems_beyond_the_scratch():
    import torch
    import paper_1912_06127_amd as pkg
    from paper_1912_06127_amd.api import TDVPError
    assert pkg.api.apply_heff_noalloc_max_bytes() == 64 << 20
    ctx = pkg.Context(0)
    try:
        # two-site, w = 10, chi = 400 in complex128 needs ~400 MB of intermediates
        L, R, theta, W1, W2 = _case(5, 2, 400, 400, 2, 10, "c128")
        out = torch.zeros_like(theta)
        with pytest.raises(TDVPError) as e:
            pkg.apply_heff(ctx, L, R, theta, W1, W2, out=out, noalloc=True)
        assert "scratch" in str(e.value)
        ctx.sync()
        assert not torch.any(out != 0)
    finally:
        ctx.close()
