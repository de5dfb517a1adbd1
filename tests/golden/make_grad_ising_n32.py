"""Write grad_ising_n32.json: the oracle's loss and forward-mode derivatives
for the differentiable one-site TDVP workload at full size.

Workload: long-range Ising chain, N = 32, couplings J/r^2 (alpha = 2) fitted by
K = 8 exponentials on r = 1..31 (MPO bond dimension 10), field h = 1; random
right-canonical initial state with bond dimensions min(2^j, 2^(32-j), 128)
from seed 32; one-site TDVP steps of dt = 0.05 (Sec. II D, Eq. proj1site);
loss <sigma^z_16> (1-based site 16) after every step, and its derivatives with
respect to J and h from the oracle's forward-mode JVP (oracle/grad.py).

Only ``oracle/`` and the seeded input generators of ``workloads/`` are used.
Run from the repository root: ``python tests/golden/make_grad_ising_n32.py``
(about three hours on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import grad, mpo, mps, spin  # noqa: E402

N, ALPHA, K, SEED, CAP, DT, STEPS, SITE = 32, 2.0, 8, 32, 128, 0.05, 20, 15


def main(out=os.path.join(os.path.dirname(os.path.abspath(__file__)), "grad_ising_n32.json")):
    c, lam, fit_err = mpo.fit_exponentials(1.0 / np.arange(1, N) ** ALPHA, K)
    bulk = mpo.mpo_exponentials(4, c, lam, spin.ising_pairs(), spin.SX, 1.0)[1]
    m = K + 2
    dJ = np.zeros_like(bulk)
    for k in range(K):
        dJ[1 + k, m - 1] = c[k] * lam[k] * spin.SZ
    dh = np.zeros_like(bulk)
    dh[0, m - 1] = spin.SX
    T0 = mps.normalize_centre(mps.right_canonicalize(
        wl.random_site_tensors(SEED, wl.full_rank_bonds(N, 2, CAP), 2)))
    Ws = mpo._boundaries(bulk, N)
    res = {}
    t0 = time.perf_counter()
    for name, V in (("J", dJ), ("h", dh)):
        hist = grad.loss_jvp(T0, Ws, mpo._boundaries(V, N), DT, STEPS, SITE, spin.SZ, every_step=True,
                             progress=lambda s: print(f"{name}: step {s} {time.perf_counter() - t0:.0f} s",
                                                      flush=True))
        res[name] = hist
    doc = {
        "workload": "1TDVP, N=32 long-range Ising alpha=2 (K=8 fitted on r<=31, w=10), J=h=1, "
                    "random right-canonical state chi<=128 seed 32, dt=0.05, loss <sigma^z_16>",
        "N": N, "alpha": ALPHA, "K": K, "seed": SEED, "chi_cap": CAP, "dt": DT, "steps": STEPS,
        "site0": SITE, "J": 1.0, "h": 1.0,
        "fit_c": [[float(z.real), float(z.imag)] for z in c],
        "fit_lam": [[float(z.real), float(z.imag)] for z in lam],
        "fit_max_abs_err": fit_err,
        "loss": [v for v, _ in res["J"]],
        "dloss_dJ": [d for _, d in res["J"]],
        "dloss_dh": [d for _, d in res["h"]],
        "generator": "tests/golden/make_grad_ising_n32.py (oracle forward-mode JVP)",
    }
    assert max(abs(a - b) for (a, _), (b, _) in zip(res["J"], res["h"])) < 1e-12
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
