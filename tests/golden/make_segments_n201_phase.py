"""Write segments_n201_phase0.json: the oracle's results for the first phase
of a segment-parallel time step at the full N = 201 workload.

Workload: long-range XY chain, N = 201, 1/2 sum r^-1.5 (xx + yy) with K = 6
exponentials fitted on r = 1..200 (MPO bond dimension 14); 32 segments
11 | 6 x 30 | 10 (Supplemental Material); bond dimensions per segment drawn
from 64..1024 (seed 201, isometry-feasible); random site tensors (seed 202)
brought to the inverse canonical gauge (Sec. II A).  The first phase of the
step (Sec. III B) evolves the 17 departing boundary pairs by dt/2 = 0.005
with 8 Lanczos vectors and splits them at their static bond dimension
(Fig. postupdate).  For every pair the script records the largest and the
smallest kept Schmidt values, their sum of squares and the discarded
weight.  Environments are streamed (only those the phase reads are kept).

Only ``oracle/`` and the seeded input generators of ``workloads/`` are used.
Run from the repository root (about ten minutes on 8 cores, ~20 GB).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import env as oenv  # noqa: E402
from oracle import mpo as ompo  # noqa: E402
from oracle import segments as oseg  # noqa: E402
from oracle import spin  # noqa: E402
from oracle.heff import apply_heff2  # noqa: E402
from oracle.tdvp import Truncation  # noqa: E402

TOP, BOTTOM = 32, 8


def main(out=os.path.join(os.path.dirname(os.path.abspath(__file__)), "segments_n201_phase0.json")):
    p = wl.XY_N201
    N, sizes, dt = p["N"], p["segments"], p["dt"]
    t0 = time.perf_counter()
    log = lambda m: print(f"[{time.perf_counter() - t0:7.0f} s] {m}", flush=True)
    c, lam, fit_err = ompo.fit_exponentials(1.0 / np.arange(1, N) ** p["alpha"], p["K"])
    Ws = ompo.mpo_exponentials(N, c, lam, spin.xy_pairs())
    chi = wl.segment_bond_profile(sizes, 2, p["chi_lo"], p["chi_hi"], p["seed_chi"])
    T = wl.random_site_tensors(p["seed_state"], chi, 2)
    log("inverse canonical gauge")
    Psi, V = oseg.to_inverse_canonical(T)
    del T
    ops = oseg.schedule(sizes, dt, True)[0].ops
    need_beta = {op.j for op in ops}
    need_gamma = {op.j + 1 for op in ops}
    beta, gamma = {}, {}
    b = oenv.trivial_env()
    for j in range(max(need_beta) + 1):
        if j in need_beta:
            beta[j] = b
        if j < max(need_beta):
            b = oenv.update_left(b, Psi[j] * V[j][None, None, :], Ws[j])
        if j % 20 == 0:
            log(f"left environments: site {j}")
    g = oenv.trivial_env()
    for j in range(N - 1, min(need_gamma) - 1, -1):
        if j in need_gamma:
            gamma[j] = g
        if j > min(need_gamma):
            g = oenv.update_right(g, V[j - 1][:, None, None] * Psi[j], Ws[j])
        if j % 20 == 0:
            log(f"right environments: site {j}")
    res = []
    for op in ops:
        j = op.j
        tr = Truncation(chi_max=chi[j + 1])
        hop = lambda x, j=j: apply_heff2(beta[j], Ws[j], Ws[j + 1], gamma[j + 1], x)
        _, S, _, w = oseg.local_pair_update(Psi[j], V[j], Psi[j + 1], hop, op.tau, tr, kmax=8, tol=0.0)
        res.append({"j": j, "tau": op.tau, "chi": [chi[j], chi[j + 1], chi[j + 2]], "kept": int(len(S)),
                    "s_top": [float(x) for x in S[:TOP]], "s_bottom": [float(x) for x in S[-BOTTOM:]],
                    "sum_s2": float(np.sum(S ** 2)), "w": float(w)})
        log(f"pair ({j}, {j + 1}) chi {chi[j]}x{chi[j + 1]}x{chi[j + 2]}: w = {w:.3e}")
    doc = {
        "workload": "segment-parallel 2TDVP, N=201 XY alpha=1.5 (K=6 fitted on r<=200, w=14), segments "
                    "11|6x30|10, chi per segment U{64..1024} seed 201, random state seed 202, first phase "
                    "of the first half (departing boundary pairs, dt/2 = 0.005), 8 Lanczos vectors, static shapes",
        "fit_c": [[float(z.real), float(z.imag)] for z in c],
        "fit_lam": [[float(z.real), float(z.imag)] for z in lam],
        "fit_max_abs_err": fit_err,
        "pairs": res,
        "w_phase": float(sum(r["w"] for r in res)),
        "generator": "tests/golden/make_segments_n201_phase.py (oracle only)",
    }
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    log(f"wrote {out}")


if __name__ == "__main__":
    main()
