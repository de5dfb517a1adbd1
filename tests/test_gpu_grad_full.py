"""Gradients of the differentiable one-site TDVP at the full size of the
differentiation workload: long-range Ising, N = 32, alpha = 2 (K = 8 fitted,
w = 10), random right-canonical state with bonds up to 128 (seed 32), 20 steps
of dt = 0.05 with environments checkpointed every 5 steps (so three blocks
are recomputed in the backward pass), loss <sigma^z_16>.  Autograd through
the library's kernels is compared with the oracle's forward-mode derivative
along J and h (tests/golden/grad_ising_n32.json, written by
tests/golden/make_grad_ising_n32.py from the oracle only)."""
import json
import os

import numpy as np
import pytest

import workloads as wl
from oracle import mps as omps
from oracle import spin

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "grad_ising_n32.json")


def _golden():
    if not os.path.exists(GOLDEN):  # the oracle run that writes it takes hours
        pytest.skip("oracle reference not written yet: python tests/golden/make_grad_ising_n32.py")
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def ctx():
    import paper_1912_06127_amd as pkg
    c = pkg.Context(0)
    yield c
    c.sync()
    c.close()


@pytest.mark.parametrize("compute", ["c128", "c64"])
def test_gradient_at_full_size_matches_oracle_jvp(ctx, compute):
    import torch
    import paper_1912_06127_amd.autodiff as ad
    g = _golden()
    N, steps = g["N"], g["steps"]
    c = np.array([complex(*z) for z in g["fit_c"]])
    lam = np.array([complex(*z) for z in g["fit_lam"]])
    T0 = omps.normalize_centre(omps.right_canonicalize(
        wl.random_site_tensors(g["seed"], wl.full_rank_bonds(N, 2, g["chi_cap"]), 2)))
    J = torch.tensor(g["J"], dtype=torch.float64, device="cuda", requires_grad=True)
    h = torch.tensor(g["h"], dtype=torch.float64, device="cuda", requires_grad=True)
    Ws, _ = ad.mpo_sum_of_exponentials(N, c, lam, spin.ising_pairs(), spin.SX, J, h)
    cdt = torch.complex64 if compute == "c64" else torch.complex128
    print(f"gradient N={N} chi<=128 {steps} steps {compute}", flush=True)
    T = ad.evolve(ctx, [torch.from_numpy(A).to("cuda") for A in T0], Ws, g["dt"], steps, compute=cdt,
                  checkpoint_every=5)
    loss = ad.expect_site(ctx, T, g["site0"], torch.from_numpy(spin.SZ).to("cuda"))
    loss.backward()
    got = {"loss": float(loss.detach()), "J": float(J.grad), "h": float(h.grad)}
    ref = {"loss": g["loss"][steps - 1], "J": g["dloss_dJ"][steps - 1], "h": g["dloss_dh"][steps - 1]}
    print(f"  got {got}\n  oracle {ref}", flush=True)
    tol_obs, tol_grad = (1e-10, 1e-8) if compute == "c128" else (1e-4, 1e-4)
    assert abs(got["loss"] - ref["loss"]) <= tol_obs
    for k in ("J", "h"):
        assert abs(got[k] - ref[k]) <= tol_grad * max(abs(ref[k]), 1e-2), (k, got[k], ref[k])
