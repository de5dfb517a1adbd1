#!/usr/bin/env python3
"""Benchmark of the TDVP hot path on one MI355X.

Workload: the two-site effective-Hamiltonian application H_eff Theta
(L.W.W.R.Theta, Sec. III A, Eq. eqnscaling) at bond dimension D = 1024,
d = 2, MPO bond w = 10 (long-range XY, alpha = 0.75, K = 4 exponentials per
channel), environments Hermitian per MPO index with complex Gaussian entries,
Theta a unit-norm complex Gaussian.  One step = one application.  The
headline runs complex64 on FP32 MFMA (3M form, FP32 accumulation); the same
line reports the complex128 (FP64 MFMA) path, the D = 128..1024 sweep, a
2TDVP sweep timing, the roofline of the dominant kernel and the FP64 CPU
oracle timed on the host cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
PMC_SUMMARY = os.path.join(ROOT, "profiles", "heff_cgemm_f32_D1024_pmc.txt")
GEMM_SOURCE = os.path.join(ROOT, "paper_1912_06127_amd", "csrc", "gemm.hip")


def heff2_flops(D: int, w: int, d: int = 2) -> float:
    """Algorithmic flops of one two-site application, 8 per complex MAC (Eq. eqnscaling)."""
    return 16.0 * w * d * d * D ** 3 + 16.0 * w * w * d ** 3 * D ** 2


def xy_bulk_tensor(pkg, ctx, alpha=0.75, K=4, rmax=100):
    import numpy as np
    c, lam, _ = pkg.fit.fit_power_law(alpha, K, rmax)
    half = 0.5
    sx = np.array(pkg.PAULI_X, dtype=np.complex128)
    sy = np.array(pkg.PAULI_Y, dtype=np.complex128)
    mpo = pkg.MPO.longrange(ctx, 6, [(half, sx, sx), (half, sy, sy)], c=c, lam=lam)
    W = mpo.tensor(2)
    mpo.close()
    return W


def gemm_source_hash() -> str:
    return hashlib.sha256(open(GEMM_SOURCE, "rb").read()).hexdigest()[:16]


def traffic_from_profiles(D: int):
    """HBM bytes per launch of the dominant kernel from the committed PMC summary,
    or None when the summary is missing or was taken on a different kernel source."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    text = open(PMC_SUMMARY).read()
    m_hash = re.search(r"gemm_source_sha256_16:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (m_hash and m_bytes) or m_hash.group(1) != gemm_source_hash():
        return None
    return float(m_bytes.group(1))


def time_heff(pkg, ctx, torch, tensors, steps, warmup, profile=False):
    L, R, th, W = tensors
    out = torch.empty_like(th)
    for _ in range(warmup):
        pkg.apply_heff(ctx, L, R, th, W, W, out=out)
    torch.cuda.synchronize()
    if profile:
        ctx.profile(True)
        ctx.profile_read()
    stream = ctx.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        pkg.apply_heff(ctx, L, R, th, W, W, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    prof = ctx.profile_read() if profile else {}
    if profile:
        ctx.profile(False)
    return ev0.elapsed_time(ev1) / steps, prof, out


def device_inputs(torch, wl, W, D, w, dtype):
    import numpy as np
    Lk, Rk, theta = wl.heff_micro_inputs(D, w)
    to = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype).contiguous()
    return to(Lk), to(Rk), to(theta), to(W)


def cpu_baseline(wl, W, D=1024, budget_s=15.0, max_reps=10):
    """FP64 oracle einsum on the host cores: the headline workload itself (two-site
    H_eff at D=1024), repeated until about budget_s seconds of work."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import heff as oheff
    Lk, Rk, theta = wl.heff_micro_inputs(D, 10)
    beta = np.transpose(Lk, (1, 0, 2))
    gamma = np.transpose(Rk, (2, 0, 1))
    t0 = time.perf_counter()
    reps = 0
    while reps < max_reps and (reps == 0 or time.perf_counter() - t0 < budget_s):
        oheff.apply_heff2(beta, W, W, gamma, theta)
        reps += 1
    dt = (time.perf_counter() - t0) / reps
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    return {
        "value": round(heff2_flops(D, 10) / dt * 1e-9, 3),
        "unit": "GFLOP/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"{reps} two-site H_eff applications at D={D}, w=10 (numpy einsum, complex128), "
                  f"{dt:.2f} s each; host {cpu_model()}, {os.cpu_count()} logical CPUs",
    }


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def gpu_state() -> dict | None:
    """Clocks, power and temperature of GPU 0 as rocm-smi reports them (the
    fields whose names mention a clock, power or temperature), or None."""
    import subprocess
    try:
        r = subprocess.run(["rocm-smi", "-d", "0", "--showclocks", "--showpower", "--showtemp", "--json"],
                           capture_output=True, text=True, timeout=30)
        data = json.loads(r.stdout)
    except (OSError, ValueError, subprocess.SubprocessError):
        return None
    card = next(iter(data.values()), {}) if isinstance(data, dict) else {}
    keep = ("clk", "power", "temperature")
    return {k: v for k, v in card.items() if any(t in k.lower() for t in keep)} or None


def oracle_timings(wl, W, budget_s=20.0):
    """The FP64 oracle (numpy/scipy, complex128) timed on the host cores beside
    each GPU workload, on bounded samples of the same inputs.  Test
    infrastructure: only this leg of the benchmark calls the oracle."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import env as oenv
    from oracle import heff as oheff
    from oracle import mpo as ompo
    from oracle import mps as omps
    from oracle import segments as oseg
    from oracle import spin
    from oracle import tdvp as otdvp
    out = {"cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
           "blas_threads": int(max([q.get("num_threads", 1) for q in threadpool_info()] or [1]))}
    # two-site H_eff at D = 1024, one BLAS thread
    Lk, Rk, theta = wl.heff_micro_inputs(1024, 10)
    beta, gamma = np.transpose(Lk, (1, 0, 2)), np.transpose(Rk, (2, 0, 1))
    with threadpool_limits(1):
        t0 = time.perf_counter()
        oheff.apply_heff2(beta, W, W, gamma, theta)
        t1 = time.perf_counter() - t0
    out["heff_D1024_1thread"] = {"s": round(t1, 2), "gflops": round(heff2_flops(1024, 10) / t1 * 1e-9, 2)}
    del Lk, Rk, theta, beta, gamma
    # N = 10 Ising quench, one-site TDVP (exact MPO), 10 steps
    p = wl.ISING_N10
    N = p["N"]
    Ws = ompo.mpo_exact(N, lambda r: p["J"] / r ** p["alpha"], spin.ising_pairs(), spin.SX, p["h"])
    st = otdvp.MPSState(omps.padded_product_state([0] * N, wl.full_rank_bonds(N, 2, p["chi_cap"])), Ws)
    t0 = time.perf_counter()
    for _ in range(10):
        otdvp.tdvp1_step(st, p["dt"])
    out["ising_n10_1tdvp"] = {"s_per_step": round((time.perf_counter() - t0) / 10, 4), "steps_timed": 10}
    # N = 64 XXX quench, two-site TDVP: the first steps within the budget
    N = 64
    c, lam, _ = ompo.fit_exponentials(np.arange(1, N, dtype=float) ** -2.0, 6)
    Ws = ompo.mpo_exponentials(N, c, lam, spin.xxx_pairs())
    bits = [j % 2 for j in range(N)]
    bits[31] ^= 1
    st = otdvp.MPSState(omps.padded_product_state(bits, [1] * (N + 1)), Ws)
    tr = otdvp.Truncation(chi_max=512, w_max=1e-8, eps=1e-12)
    t0, n = time.perf_counter(), 0
    while n < 10 and (n == 0 or time.perf_counter() - t0 < budget_s):
        otdvp.tdvp2_step(st, 0.05, tr, tol=1e-10)
        n += 1
    out["xxx_n64_2tdvp"] = {"s_per_step": round((time.perf_counter() - t0) / n, 3), "steps_timed": n,
                            "note": "the first steps of the 40-step quench (chi grows with time)"}
    # N = 201 segments: one two-site update of the first phase at a real shape
    # (bonds 384 | 192 | 192, w = 14, 8 Lanczos vectors and the split) and one
    # two-site matvec at the largest shape of that phase (601 | 601 | 1009)
    q = wl.XY_N201
    c, lam, _ = ompo.fit_exponentials(1.0 / np.arange(1, q["N"]) ** q["alpha"], q["K"])
    Wb = ompo.mpo_exponentials(6, c, lam, spin.xy_pairs())[2]
    w = Wb.shape[0]
    rng = np.random.default_rng(5)
    res = {}
    for tag, (cl, cm, cr), full in (("update_384x192x192", (384, 192, 192), True),
                                    ("matvec_601x601x1009", (601, 601, 1009), False)):
        b = wl.cgauss(rng, (cl, w, cl)) / np.sqrt(cl)
        g = wl.cgauss(rng, (cr, w, cr)) / np.sqrt(cr)
        Pl, Pr = wl.cgauss(rng, (cl, 2, cm)), wl.cgauss(rng, (cm, 2, cr))
        V = np.ones(cm)
        hop = lambda x: oheff.apply_heff2(b, Wb, Wb, g, x)
        t0 = time.perf_counter()
        if full:
            oseg.local_pair_update(Pl, V, Pr, hop, 0.005, otdvp.Truncation(chi_max=cm), kmax=8, tol=0.0)
        else:
            hop(np.einsum("asb,btc->astc", Pl, Pr))
        res[tag] = round(time.perf_counter() - t0, 3)
    out["xy_n201_segments"] = {**res, "note": "synthetic environments at the real shapes of the first phase"}
    # N = 32 Ising (the differentiation workload), one one-site TDVP step forward
    p = wl.ISING_N32_GRAD
    N = p["N"]
    c, lam, _ = ompo.fit_exponentials(1.0 / np.arange(1, N) ** p["alpha"], p["K"])
    Ws = ompo.mpo_exponentials(N, c, lam, spin.ising_pairs(), spin.SX, p["h"])
    T0 = omps.normalize_centre(omps.right_canonicalize(
        wl.random_site_tensors(p["seed_state"], wl.full_rank_bonds(N, 2, p["chi_cap"]), 2)))
    st = otdvp.MPSState(T0, Ws)
    t0 = time.perf_counter()
    otdvp.tdvp1_step(st, p["dt"])
    out["ising_n32_1tdvp"] = {"s_per_step": round(time.perf_counter() - t0, 2), "steps_timed": 1}
    return out


def ising_timing(pkg, ctx, wl):
    """1TDVP quench of the N=10 long-range Ising chain (exact MPO, w = 11).

    H = sum_{i<j} |i-j|^-3 sigma^z_i sigma^z_j + sum_i sigma^x_i from all spins
    up, padded to chi = (1, 2, 4, 8, 16, 32, 16, 8, 4, 2, 1); dt = 0.01, 100
    steps, complex128 and complex64.  Per step median time; <sigma^z_5>,
    <sigma^z_6> and the energy at the end, compared between the precisions.
    """
    import numpy as np
    p = wl.ISING_N10
    N = p["N"]
    sx, sz = (np.array(q, dtype=np.complex128) for q in (pkg.PAULI_X, pkg.PAULI_Z))
    mpo = pkg.MPO.longrange(ctx, N, [(p["J"], sz, sz)], coupling=[r ** -p["alpha"] for r in range(1, N)],
                            onsite=sx, h=p["h"])
    res, obs = {}, {}
    for comp in ("c128", "c64"):
        mps = pkg.MPS.init(ctx, N, 2, wl.full_rank_bonds(N, 2, p["chi_cap"]), basis_state=[0] * N)
        opts = pkg.TDVPOptions(compute=comp)
        times = []
        for _ in range(p["steps"]):
            times.append(pkg.tdvp1_step(ctx, mps, mpo, p["dt"], opts)["seconds"])
        z = pkg.expect(ctx, mps, [4, 5], sz).real
        obs[comp] = np.array([z[0], z[1], pkg.energy(ctx, mps, mpo).real])
        res[comp] = {"s_per_step_median": round(float(np.median(times)), 5),
                     "sz5": float(z[0]), "sz6": float(z[1]), "energy": float(obs[comp][2])}
        mps.close()
    mpo.close()
    res["max_abs_obs_diff_c64_vs_c128"] = float(np.max(np.abs(obs["c64"] - obs["c128"])))
    res["workload"] = "1TDVP, N=10 long-range Ising (alpha=3, J=h=1, exact MPO w=11), chi<=32, dt=0.01, 100 steps"
    return res


def sweep_timing(pkg, ctx, steps=40, taylor=True):
    """2TDVP quench of the N=64 1/r^2 XXX chain (K = 6 exponentials, w = 20).

    Neel state (odd sites up, 1-based) with site 32 flipped; dt = 0.05,
    w_max = 1e-8, eps = 1e-12, chi_max = 512.  Each precision runs the
    evolution twice: an untimed pass that lets the GEMM autotuner see every
    shape, then the timed pass.  Observables are excluded from the step time.
    The spin profile C_i = <sigma^z_i>/4 at the end is compared between the
    FP32-MFMA and the FP64 path.  The FP64 evolution is then repeated with the
    truncated-Taylor exponential in place of Lanczos (timed pass only).
    """
    import numpy as np
    N, cap = 64, 512
    c, lam, _ = pkg.fit.fit_power_law(2.0, 6, N - 1)
    sx, sy, sz = (np.array(p, dtype=np.complex128) for p in (pkg.PAULI_X, pkg.PAULI_Y, pkg.PAULI_Z))
    mpo = pkg.MPO.longrange(ctx, N, [(0.25, sx, sx), (0.25, sy, sy), (0.25, sz, sz)], c=c, lam=lam)
    bits = [j % 2 for j in range(N)]
    bits[31] ^= 1
    res, prof = {}, {}
    for comp in ("c64", "c128"):
        opts = pkg.TDVPOptions(compute=comp, chi_max=cap, w_max=1e-8, eps_rel=1e-12, krylov_max=40,
                               krylov_tol=1e-10)
        for timed in (False, True):
            mps = pkg.MPS.init(ctx, N, 2, [1] * (N + 1), basis_state=bits)
            times, flops, mv, wt = [], 0.0, 0, 0.0
            for _ in range(steps):
                st = pkg.tdvp2_step(ctx, mps, mpo, 0.05, opts)
                times.append(st["seconds"])
                flops += st["flops"]
                mv += st["matvecs"]
                wt = st["w_total"]
            if timed:
                prof[comp] = 0.25 * pkg.expect(ctx, mps, list(range(N)), sz).real
                res[comp] = {"s_per_step": round(float(np.mean(times)), 4),
                             "s_per_step_first10": round(float(np.mean(times[:10])), 4),
                             "s_per_step_last10": round(float(np.mean(times[-10:])), 4),
                             "matvecs_per_step": mv / steps,
                             "heff_env_gflops": round(flops / sum(times) * 1e-9, 1),
                             "chi_peak": max(mps.chi), "w_total": wt}
            mps.close()
    # the FP64 evolution again with the truncated-Taylor exponential (shapes already tuned)
    if taylor:
        opts = pkg.TDVPOptions(compute="c128", chi_max=cap, w_max=1e-8, eps_rel=1e-12, krylov_tol=1e-10,
                               exp_method="taylor")
        mps = pkg.MPS.init(ctx, N, 2, [1] * (N + 1), basis_state=bits)
        times, mv = [], 0
        for _ in range(steps):
            st = pkg.tdvp2_step(ctx, mps, mpo, 0.05, opts)
            times.append(st["seconds"])
            mv += st["matvecs"]
        pt = 0.25 * pkg.expect(ctx, mps, list(range(N)), sz).real
        res["c128_taylor"] = {"s_per_step": round(float(np.mean(times)), 4), "matvecs_per_step": mv / steps,
                              "chi_peak": max(mps.chi),
                              "max_abs_obs_diff_vs_lanczos": float(np.max(np.abs(pt - prof["c128"])))}
        mps.close()
    mpo.close()
    res["speedup_fp32_vs_fp64"] = round(res["c128"]["s_per_step"] / res["c64"]["s_per_step"], 2)
    res["max_abs_obs_diff_c64_vs_c128"] = float(np.max(np.abs(prof["c64"] - prof["c128"])))
    res["workload"] = ("2TDVP quench, N=64 XXX 1/r^2 (K=6, w=20), Neel + flip at site 32, dt=0.05, "
                       f"{steps} steps, w_max=1e-8, eps=1e-12, chi_max=512")
    return res


def sweep_u1_timing(pkg, ctx, steps=40):
    """The N = 64 XXX quench of the sweep workload in the U(1) form: the MPO
    written with sigma+ sigma- + sigma- sigma+ (+ sigma^z sigma^z) channels, each
    of definite charge, run once dense and once with charge labels on the state
    and the MPO (splits sector by sector; matvecs and environments on the
    block kernels from chi_l * chi_r >= 256^2 on, "u1", or always,
    "u1_blocks"), complex64 contractions.  Each mode runs an untimed pass (GEMM
    autotuning) and a timed pass; the spin profiles at the end are compared."""
    import numpy as np
    N, cap, K = 64, 512, 6
    c, lam, _ = pkg.fit.fit_power_law(2.0, K, N - 1)
    sp = np.array([[0, 1], [0, 0]], dtype=np.complex128)
    sm = sp.T.copy()
    sz = np.array(pkg.PAULI_Z, dtype=np.complex128)
    mpo = pkg.MPO.longrange(ctx, N, [(0.5, sp, sm), (0.5, sm, sp), (0.25, sz, sz)], c=c, lam=lam)
    inner = [0] + [1] * K + [-1] * K + [0] * K + [0]
    bits = [j % 2 for j in range(N)]
    bits[31] ^= 1
    up = np.cumsum([0] + [1 - b for b in bits])
    labels = [[int(u)] for u in up]
    opts = pkg.TDVPOptions(compute="c64", chi_max=cap, w_max=1e-8, eps_rel=1e-12, krylov_max=40, krylov_tol=1e-10)
    res, prof = {}, {}
    for mode in ("dense", "u1", "u1_blocks"):
        mpo.set_charges([[0]] + [inner] * (N - 1) + [[0]] if mode != "dense" else None)
        opts.u1_block_min = 1 if mode == "u1_blocks" else 0
        for timed in (False, True):
            mps = pkg.MPS.init(ctx, N, 2, [1] * (N + 1), basis_state=bits)
            if mode != "dense":
                mps.set_charges([1, 0], labels)
            times, mv, wt = [], 0, 0.0
            for k in range(steps):
                st = pkg.tdvp2_step(ctx, mps, mpo, 0.05, opts)
                times.append(st["seconds"])
                mv += st["matvecs"]
                wt = st["w_total"]
                if (k + 1) % 10 == 0:
                    progress(f"sweep {mode} {'timed' if timed else 'tuning'} pass: step {k + 1}, "
                             f"{times[-1]:.3f} s, chi_max {max(mps.chi)}")
            if timed:
                prof[mode] = 0.25 * pkg.expect(ctx, mps, list(range(N)), sz).real
                res[mode] = {"s_per_step": round(float(np.mean(times)), 4),
                             "s_per_step_last10": round(float(np.mean(times[-10:])), 4),
                             "matvecs_per_step": mv / steps, "chi_peak": max(mps.chi), "w_total": wt}
                if mode != "dense":
                    res[mode]["sectors_at_centre"] = len(set(mps.charges()[1][N // 2]))
            mps.close()
    mpo.close()
    for mode in ("u1", "u1_blocks"):
        res[f"speedup_{mode}_vs_dense"] = round(res["dense"]["s_per_step"] / res[mode]["s_per_step"], 2)
        res[f"max_abs_obs_diff_{mode}_vs_dense"] = float(np.max(np.abs(prof[mode] - prof["dense"])))
    res["workload"] = ("2TDVP quench, N=64 XXX 1/r^2 in sigma+- form (K=6, w=20), Neel + flip at site 32, "
                       f"dt=0.05, {steps} steps, w_max=1e-8, eps=1e-12, chi_max=512, complex64; dense vs U(1)")
    return res


def sweep_u1_large_timing(pkg, ctx, chi=256, steps=3):
    """The N = 64 XXX quench (sigma+- MPO, K = 6, w = 20) carried on in U(1)
    mode with dt = 0.1 until every central bond reaches chi (chi_max = chi,
    w_max = 1e-10); from that state, `steps` 2TDVP steps (dt = 0.05, complex64)
    dense and in U(1) mode, each after one untimed step from the same state
    (GEMM autotuning).  The spin profiles after the timed steps are compared."""
    import numpy as np
    N, K = 64, 6
    c, lam, _ = pkg.fit.fit_power_law(2.0, K, N - 1)
    sp = np.array([[0, 1], [0, 0]], dtype=np.complex128)
    sm = sp.T.copy()
    sz = np.array(pkg.PAULI_Z, dtype=np.complex128)
    mpo = pkg.MPO.longrange(ctx, N, [(0.5, sp, sm), (0.5, sm, sp), (0.25, sz, sz)], c=c, lam=lam)
    charges = [[0]] + [[0] + [1] * K + [-1] * K + [0] * K + [0]] * (N - 1) + [[0]]
    mpo.set_charges(charges)
    bits = [j % 2 for j in range(N)]
    bits[31] ^= 1
    up = np.cumsum([0] + [1 - b for b in bits])
    grow = pkg.TDVPOptions(compute="c64", chi_max=chi, w_max=1e-10, eps_rel=1e-12, krylov_max=40, krylov_tol=1e-10)
    m = pkg.MPS.init(ctx, N, 2, [1] * (N + 1), basis_state=bits)
    m.set_charges([1, 0], [[int(u)] for u in up])
    t_grow = 0.0
    for k in range(200):
        st = pkg.tdvp2_step(ctx, m, mpo, 0.1, grow)
        t_grow += st["seconds"]
        if (k + 1) % 5 == 0:
            progress(f"U(1) quench growth: step {k + 1}, chi {max(m.chi)}, {st['seconds']:.3f} s")
        if min(m.chi[24:41]) >= chi:
            break
    T, (qp, labels), chi_reached = m.tensors(), m.charges(), max(m.chi)
    m.close()
    opts = pkg.TDVPOptions(compute="c64", chi_max=chi, w_max=1e-10, eps_rel=1e-12, krylov_max=40, krylov_tol=1e-10)
    res, prof = {"growth_steps": k + 1, "growth_seconds": round(t_grow, 1), "chi": chi_reached,
                 "sectors_at_centre": len(set(labels[N // 2]))}, {}
    for mode in ("dense", "u1"):
        mpo.set_charges(charges if mode == "u1" else None)
        times = []
        for timed in (False, True):
            x = pkg.MPS.from_tensors(ctx, T)
            if mode == "u1":
                x.set_charges(qp, labels)
            for _ in range(steps if timed else 1):
                st = pkg.tdvp2_step(ctx, x, mpo, 0.05, opts)
                if timed:
                    times.append(st["seconds"])
            progress(f"chi={chi} sweep {mode} {'timed' if timed else 'tuning'} pass done")
            if timed:
                prof[mode] = 0.25 * pkg.expect(ctx, x, list(range(N)), sz).real
                res[mode] = {"s_per_step": round(float(np.mean(times)), 3), "matvecs_last_step": st["matvecs"]}
            x.close()
    mpo.close()
    res["speedup_u1_vs_dense"] = round(res["dense"]["s_per_step"] / res["u1"]["s_per_step"], 2)
    res["max_abs_obs_diff_u1_vs_dense"] = float(np.max(np.abs(prof["u1"] - prof["dense"])))
    res["workload"] = (f"2TDVP, N=64 XXX 1/r^2 sigma+- (K=6, w=20), state from the Neel + flip quench grown in "
                       f"U(1) mode to chi={chi}; {steps} steps dt=0.05, complex64, dense vs U(1) "
                       f"(block kernels from chi_l*chi_r >= 256^2)")
    return res


def segments_timing(pkg, ctx, np, graph=True, extras=True):
    """Segment-parallel 2TDVP, N=201 long-range XY (alpha 1.5, K = 6, w = 14),
    32 segments (11 | 6 x 30 | 10), uneven bond profile (one seeded draw in
    [64, 1024] per segment), seeded random state, dt = 0.01, static shapes,
    FP32-MFMA matvecs with FP64 Lanczos and splits, 8 Lanczos steps.

    One untimed step (tile tuning), one timed eager step, one step that
    captures every phase's batched exponentiation in a HIP graph and one step
    that replays them; then the norm of the state and one serial
    reorthonormalisation with environment recompute (Sec. III D), timed; then
    the one-site schedule (two-site boundary pairs) on the same state: one
    untimed step (tile tuning for the one-site shapes) and one timed step.
    """
    import workloads as wl
    p = wl.XY_N201
    N, sizes = p["N"], p["segments"]
    chi = wl.segment_bond_profile(sizes, 2, p["chi_lo"], p["chi_hi"], p["seed_chi"])
    T = wl.random_site_tensors(p["seed_state"], chi, 2)
    c, lam, err = pkg.fit.fit_power_law(p["alpha"], p["K"], N - 1)
    sx, sy = (np.array(q, dtype=np.complex128) for q in (pkg.PAULI_X, pkg.PAULI_Y))
    mpo = pkg.MPO.longrange(ctx, N, [(0.5, sx, sx), (0.5, sy, sy)], c=c, lam=lam)
    progress("segments: building the inverse canonical state")
    t0 = time.perf_counter()
    sg = pkg.Segments.init(ctx, mpo, T, sizes, compute="c64")
    ctx.sync()
    init_s = time.perf_counter() - t0
    del T
    res = {"init_s": round(init_s, 2)}
    eager = pkg.SegmentOptions()
    graph_opts = pkg.SegmentOptions(use_graph=True)
    progress("segments: warm-up step (tile tuning)")
    sg.step(mpo, p["dt"], eager)
    progress("segments: timed eager step")
    ctx.profile(True)
    st = sg.step(mpo, p["dt"], eager)
    prof = ctx.profile_read()
    ctx.profile(False)
    g = {k: v for k, v in prof.items() if k.startswith("cgemm2g")}
    gms = sum(v["ms"] for v in g.values())
    gfl = sum(v["flops"] for v in g.values())
    res["s_per_step_eager"] = round(st["seconds"], 3)
    res["flops_per_step"] = st["flops"]
    res["step_tflops"] = round(st["flops"] / st["seconds"] * 1e-12, 2)
    res["grouped_gemm_tflops"] = round(gfl / (gms * 1e-3) * 1e-12, 2)
    res["grouped_gemm_frac_of_fp32_peak"] = round(gfl / (gms * 1e-3) * 1e-12 / PEAK_FP32_MFMA_TFLOPS, 4)
    res["batched_expm_s"] = round(prof.get("seg_batched_expm", {}).get("ms", 0.0) * 1e-3, 3)
    res["splits_s"] = round(prof.get("seg_splits", {}).get("ms", 0.0) * 1e-3, 3)
    res["mpo_stage_s"] = round(sum(v["ms"] for k, v in prof.items() if k.startswith("wstage_grouped")) * 1e-3, 3)
    if graph:
        progress("segments: graph capture step")
        sg.step(mpo, p["dt"], graph_opts)
        progress("segments: graph replay step")
        st = sg.step(mpo, p["dt"], graph_opts)
        res["s_per_step_graph"] = round(st["seconds"], 3)
    res["matvecs_per_step"] = st["matvecs"]
    res["chi_max"] = max(chi)
    res["w_total"] = sg.w_total
    if extras:
        one_site_and_repair(pkg, ctx, sg, mpo, p, chi, res)
    sg.close()
    mpo.close()
    res["workload"] = ("segment-parallel 2TDVP, N=201 XY alpha=1.5 (K=6, w=14), 32 segments 11|6x30|10, "
                       "chi per segment U{64..1024} (seeded), dt=0.01, static shapes, k=8")
    return res


def segments_fp64_timing(pkg, ctx, np):
    """The segment-parallel step of segments_timing with every contraction in
    FP64 (complex128 environments and matvecs on the FP64 MFMA path): one
    untimed step (tile tuning), then one timed eager step, for the FP32 / FP64
    comparison at equal schedule and state."""
    import workloads as wl
    p = wl.XY_N201
    N, sizes = p["N"], p["segments"]
    chi = wl.segment_bond_profile(sizes, 2, p["chi_lo"], p["chi_hi"], p["seed_chi"])
    T = wl.random_site_tensors(p["seed_state"], chi, 2)
    c, lam, err = pkg.fit.fit_power_law(p["alpha"], p["K"], N - 1)
    sx, sy = (np.array(q, dtype=np.complex128) for q in (pkg.PAULI_X, pkg.PAULI_Y))
    mpo = pkg.MPO.longrange(ctx, N, [(0.5, sx, sx), (0.5, sy, sy)], c=c, lam=lam)
    progress("segments FP64: building the inverse canonical state")
    sg = pkg.Segments.init(ctx, mpo, T, sizes, compute="c128")
    del T
    eager = pkg.SegmentOptions(compute="c128")
    progress("segments FP64: warm-up step (tile tuning)")
    sg.step(mpo, p["dt"], eager)
    progress("segments FP64: timed eager step")
    ctx.profile(True)
    st = sg.step(mpo, p["dt"], eager)
    prof = ctx.profile_read()
    ctx.profile(False)
    g = {k: v for k, v in prof.items() if k.startswith("cgemm2g")}
    gms = sum(v["ms"] for v in g.values())
    gfl = sum(v["flops"] for v in g.values())
    res = {"s_per_step_eager": round(st["seconds"], 3), "step_tflops": round(st["flops"] / st["seconds"] * 1e-12, 2),
           "grouped_gemm_tflops": round(gfl / (gms * 1e-3) * 1e-12, 2),
           "grouped_gemm_frac_of_fp64_peak": round(gfl / (gms * 1e-3) * 1e-12 / PEAK_FP64_MFMA_TFLOPS, 4),
           "batched_expm_s": round(prof.get("seg_batched_expm", {}).get("ms", 0.0) * 1e-3, 3),
           "splits_s": round(prof.get("seg_splits", {}).get("ms", 0.0) * 1e-3, 3),
           "w_total": sg.w_total,
           "workload": "the segment-parallel N=201 step above with complex128 environments and matvecs (FP64 MFMA)"}
    sg.close()
    mpo.close()
    return res


def one_site_and_repair(pkg, ctx, sg, mpo, p, chi, res):
    """Norm drift, the serial repair and the one-site schedule on the state
    the two-site steps left."""
    progress("segments: norm and reorthonormalisation (serial repair)")
    t0 = time.perf_counter()
    n2 = sg.norm2()
    res["norm2_s"] = round(time.perf_counter() - t0, 3)
    res["norm_drift"] = n2 - 1.0
    t0 = time.perf_counter()
    sg.reorthonormalize(mpo)
    ctx.sync()
    res["reorth_s"] = round(time.perf_counter() - t0, 2)
    res["norm_drift_after_reorth"] = sg.norm2() - 1.0
    progress("segments: one-site schedule, warm-up step (tile tuning)")
    o1 = pkg.SegmentOptions(one_site=True)
    sg.step(mpo, p["dt"], o1)
    progress("segments: one-site schedule, timed step")
    ctx.profile(True)
    st1 = sg.step(mpo, p["dt"], o1)
    prof1 = ctx.profile_read()
    ctx.profile(False)
    res["one_site"] = {"s_per_step": round(st1["seconds"], 3), "flops_per_step": st1["flops"],
                       "matvecs_per_step": st1["matvecs"],
                       "batched_expm_s": round(prof1.get("seg_batched_expm", {}).get("ms", 0.0) * 1e-3, 3),
                       "bond_steps_s": round(prof1.get("seg_bonds", {}).get("ms", 0.0) * 1e-3, 3),
                       "boundary_splits_s": round(prof1.get("seg_splits", {}).get("ms", 0.0) * 1e-3, 3),
                       "chi_unchanged": sg.chi == chi, "w_total": sg.w_total}


def gradient_timing(pkg, ctx, torch, np, steps=2):
    """Differentiable 1TDVP: N=32 long-range Ising (alpha 2, J = h = 1, K = 8,
    w = 10), random right-canonical state chi_j = min(2^j, 2^(32-j), 128),
    dt = 0.05, loss <sigma^z_16>, checkpoint every 5 steps; gradients with
    respect to J and h through the hand-written apply_heff and environment
    adjoints.  One untimed forward step per precision first."""
    import workloads as wl
    import paper_1912_06127_amd.autodiff as ad
    p = wl.ISING_N32_GRAD
    N = p["N"]
    chi = wl.full_rank_bonds(N, 2, p["chi_cap"])
    m = pkg.MPS.from_tensors(ctx, wl.random_site_tensors(p["seed_state"], chi, 2))
    m.right_canonicalize()
    T0 = [torch.from_numpy(A).to("cuda") for A in m.tensors()]
    m.close()
    c, lam, _ = pkg.fit.fit_power_law(p["alpha"], p["K"], N - 1)
    sz = torch.tensor(pkg.PAULI_Z, dtype=torch.complex128, device="cuda")
    sx = np.array(pkg.PAULI_X, dtype=np.complex128)
    res = {}
    for comp, cdt in (("c64", torch.complex64), ("c128", torch.complex128)):
        J = torch.tensor(p["J"], dtype=torch.float64, device="cuda", requires_grad=True)
        h = torch.tensor(p["h"], dtype=torch.float64, device="cuda", requires_grad=True)
        Ws, _ = ad.mpo_sum_of_exponentials(N, c, lam, [(1.0, np.diag([1.0, -1.0]).astype(np.complex128),
                                                         np.diag([1.0, -1.0]).astype(np.complex128))], sx, J, h)
        with torch.no_grad():  # untimed step: the GEMM autotuner sees this precision's shapes
            ad.evolve(ctx, T0, [W.detach() for W in Ws], p["dt"], 1, compute=cdt, checkpoint_every=0)
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()  # buffers of earlier workloads still held
        t0 = time.perf_counter()
        with torch.no_grad():
            ad.evolve(ctx, T0, [W.detach() for W in Ws], p["dt"], steps, compute=cdt, checkpoint_every=0)
        torch.cuda.synchronize()
        fwd = (time.perf_counter() - t0) / steps
        progress(f"gradient {comp}: forward {fwd:.3f} s/step; forward + backward over {steps} steps")
        t0 = time.perf_counter()
        T = ad.evolve(ctx, T0, Ws, p["dt"], steps, compute=cdt, checkpoint_every=p["checkpoint_every"])
        loss = ad.expect_site(ctx, T, p["site"] - 1, sz)
        loss.backward()
        torch.cuda.synchronize()
        both = (time.perf_counter() - t0) / steps
        res[comp] = {"s_per_step_forward": round(fwd, 3), "s_per_step_forward_backward": round(both, 3),
                     "peak_mem_gib": round((torch.cuda.max_memory_allocated() - base) / 2 ** 30, 2),
                     "dloss_dJ": float(J.grad), "dloss_dh": float(h.grad)}
    res["workload"] = (f"differentiable 1TDVP, N=32 Ising alpha=2 (K=8, w=10), chi<=128, dt=0.05, "
                       f"{steps} steps, loss <sigma^z_16>, checkpoint every 5")
    return res


def u1_timing(pkg, ctx, torch, np, chi=512, K=6, reps=10):
    """Two-site H_eff at the N = 64 quench's bond cap (chi = 512 on both bonds,
    XXX with K = 6 exponentials, w = 20) on charge-symmetric inputs: the dense
    path against the U(1) block-sparse path (half-chain S^z sector profiles),
    complex64.  Dense: HIP-event time per call; blocked: kernel time per call
    from the library's profiler and wall time per call (the block tables are
    built on the host each call)."""
    import workloads as wl
    sp = np.array([[0, 1], [0, 0]], dtype=np.complex128)
    sm = sp.T.copy()
    sz = np.diag([1.0, -1.0]).astype(np.complex128)
    pairs = [(0.5, sp, sm), (0.5, sm, sp), (0.25, sz, sz)]
    c, lam, _ = pkg.fit.fit_power_law(2.0, K, 63)
    mpo = pkg.MPO.longrange(ctx, 6, pairs, c=c, lam=lam)
    W = mpo.tensor(2)
    mpo.close()
    cw = [0] + [1] * K + [-1] * K + [0] * K + [0]
    ql, qr, qs = wl.u1_labels(chi, 16, 2.5, 31), wl.u1_labels(chi, 17, 2.5, 32), [1, 0]
    pat = wl.u1_patterns(ql, qr, qs, cw)
    to = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda", torch.complex64)
    L, R = to(wl.u1_symmetric(41, pat["L"])), to(wl.u1_symmetric(42, pat["R"]))
    th, Wd = to(wl.u1_symmetric(43, pat["two_site"])), to(W)
    out = torch.empty_like(th)
    kw = dict(q_left=ql, q_right=qr, q_phys=qs, c_left=cw, c_right=cw, out=out)
    for _ in range(2):
        pkg.apply_heff(ctx, L, R, th, Wd, Wd, out=out)
        pkg.apply_heff_u1(ctx, L, R, th, Wd, Wd, **kw)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(ctx.stream)
    for _ in range(reps):
        pkg.apply_heff(ctx, L, R, th, Wd, Wd, out=out)
    e1.record(ctx.stream)
    torch.cuda.synchronize()
    dense_ms = e0.elapsed_time(e1) / reps
    ctx.profile(True)
    ctx.profile_read()
    t0 = time.perf_counter()
    for _ in range(reps):
        pkg.apply_heff_u1(ctx, L, R, th, Wd, Wd, **kw)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / reps
    prof = ctx.profile_read()
    ctx.profile(False)
    kern_ms = sum(v["ms"] for v in prof.values()) / reps
    block_flops = sum(v["flops"] for k, v in prof.items() if k.startswith("cgemm2_blocks")) / reps
    nsec = len(set(int(q) for q in ql))
    return {"dense_ms": round(dense_ms, 3), "u1_kernel_ms": round(kern_ms, 3), "u1_wall_ms": round(wall_ms, 3),
            "speedup_kernel": round(dense_ms / kern_ms, 2), "speedup_wall": round(dense_ms / wall_ms, 2),
            "dense_flops": heff2_flops(chi, 20), "block_gemm_flops": block_flops, "sectors_left": nsec,
            "u1_kernel_ms_by_kernel": {k: round(v["ms"] / reps, 4) for k, v in prof.items()},
            "u1_launches_per_call": sum(v["count"] for v in prof.values()) / reps,
            "workload": f"two-site H_eff, chi={chi} both bonds, XXX K={K} (w=20), complex64, S^z sectors "
                        f"(Gaussian profile, spread 2.5), dense path vs U(1) blocks"}


def copy_calibration(torch, gib=1):
    """Plain device copy of known size, used to scale HBM byte counters."""
    n = gib * (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": n * 4, "launches": 5}))


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline kernel only (for profiling)")
    ap.add_argument("--no-gpu-state", action="store_true",
                    help="do not run rocm-smi for the clocks around the timed region (for runs under a profiler)")
    ap.add_argument("--sweep-steps", type=int, default=40)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-segments", action="store_true", help="skip the segment-parallel N=201 step")
    ap.add_argument("--only-segments", action="store_true",
                    help="run only the segment-parallel N=201 workload and print its timings (for profiling)")
    ap.add_argument("--segments-no-graph", action="store_true", help="segment workload: eager steps only")
    ap.add_argument("--only-segments-fp64", action="store_true",
                    help="run only the segment-parallel N=201 step with FP64 contractions and print its timings")
    ap.add_argument("--segments-no-extras", action="store_true",
                    help="segment workload: skip the repair and the one-site schedule")
    ap.add_argument("--sweep-no-taylor", action="store_true", help="sweep workload: skip the Taylor-exponential pass")
    ap.add_argument("--only-sweep", action="store_true",
                    help="run only the N=64 2TDVP quench sweep and print its timings (for profiling)")
    ap.add_argument("--grad-steps", type=int, default=2)
    ap.add_argument("--only-u1", action="store_true", help="run only the U(1) block-sparse H_eff timing")
    ap.add_argument("--only-sweep-u1", action="store_true",
                    help="run only the N=64 quench sweep dense against U(1) blocks and print its timings")
    ap.add_argument("--only-sweep-u1-large", type=int, default=0,
                    help="run only the N=64 quench grown to this bond dimension in U(1) mode, then dense against "
                         "U(1) steps from that state")
    ap.add_argument("--only-D", type=int, default=0,
                    help="run only the two-site H_eff timing at this bond dimension (both precisions; for profiling)")
    ap.add_argument("--only-grad", action="store_true",
                    help="run only the differentiable 1TDVP workload (--grad-steps steps) and print its timings")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1912_06127_amd as pkg
    import workloads as wl

    if args.copy_calibration:
        copy_calibration(torch)
        return

    if args.only_sweep:
        ctx = pkg.Context(0)
        print(json.dumps({"sweep": sweep_timing(pkg, ctx, args.sweep_steps, taylor=not args.sweep_no_taylor)}))
        ctx.close()
        return

    if args.only_u1:
        ctx = pkg.Context(0)
        print(json.dumps({"u1": {str(chi): u1_timing(pkg, ctx, torch, np, chi=chi) for chi in (64, 128, 256, 512)}}))
        ctx.close()
        return

    if args.only_sweep_u1_large:
        ctx = pkg.Context(0)
        print(json.dumps({"sweep_u1_large": sweep_u1_large_timing(pkg, ctx, args.only_sweep_u1_large)}))
        ctx.close()
        return

    if args.only_sweep_u1:
        ctx = pkg.Context(0)
        print(json.dumps({"sweep_u1": sweep_u1_timing(pkg, ctx, args.sweep_steps)}))
        ctx.close()
        return

    if args.only_grad:
        ctx = pkg.Context(0)
        print(json.dumps({"gradient": gradient_timing(pkg, ctx, torch, np, args.grad_steps)}))
        ctx.close()
        return

    if args.only_D:
        ctx = pkg.Context(0)
        W = xy_bulk_tensor(pkg, ctx)
        r = {}
        for name, dt in (("c64", torch.complex64), ("c128", torch.complex128)):
            xs = device_inputs(torch, wl, W, args.only_D, 10, dt)
            msx, _, _ = time_heff(pkg, ctx, torch, xs, args.steps, args.warmup)
            r[name] = {"gflops": round(heff2_flops(args.only_D, 10) / (msx * 1e-3) * 1e-9, 1), "ms": round(msx, 5)}
            del xs
        print(json.dumps({"heff_D": args.only_D, **r}))
        ctx.close()
        return

    if args.only_segments_fp64:
        ctx = pkg.Context(0)
        print(json.dumps({"segments_fp64": segments_fp64_timing(pkg, ctx, np)}))
        ctx.close()
        return

    if args.only_segments:
        ctx = pkg.Context(0)
        print(json.dumps({"segments": segments_timing(pkg, ctx, np, graph=not args.segments_no_graph,
                                                      extras=not args.segments_no_extras)}))
        ctx.close()
        return

    ctx = pkg.Context(0)
    D, w = 1024, 10
    W = xy_bulk_tensor(pkg, ctx)
    assert W.shape == (w, w, 2, 2)
    F = heff2_flops(D, w)

    progress("inputs ready; timing complex64 D=1024")
    x64 = device_inputs(torch, wl, W, D, w, torch.complex64)
    state_before = None if args.no_gpu_state else gpu_state()
    ms64, prof64, _ = time_heff(pkg, ctx, torch, x64, args.steps, args.warmup, profile=True)
    state_after = None if args.no_gpu_state else gpu_state()
    value = F / (ms64 * 1e-3) * 1e-9
    del x64

    # dominant kernel: the FP32 3M GEMM of both H_eff stages
    kname = max(prof64, key=lambda k: prof64[k]["ms"])
    kp = prof64[kname]
    achieved = kp["flops"] / (kp["ms"] * 1e-3) * 1e-12
    per_launch_flops = kp["flops"] / kp["count"]
    per_launch_ms = kp["ms"] / kp["count"]
    traffic = traffic_from_profiles(D)
    roofline = {
        "bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP32_MFMA_TFLOPS, 4), "traffic": traffic,
        "kernel": kname, "launches": kp["count"], "avg_launch_us": round(per_launch_ms * 1e3, 1),
        "algorithmic_flops_per_launch": per_launch_flops,
        "mfma_executed_frac": round(0.75 * achieved / PEAK_FP32_MFMA_TFLOPS, 4),
        "note": "3M form: three real products per complex product, so the matrix cores execute 3/4 of the "
                "algorithmic flops and frac can exceed 1; mfma_executed_frac is the fraction of the "
                "instruction peak actually issued",
        "kernel_share_of_step": round(kp["ms"] / (ms64 * args.steps), 3),
        "other_kernels_ms_per_step": {k: round(v["ms"] / args.steps, 4) for k, v in prof64.items() if k != kname},
    }

    line = {
        "metric": "apply_heff GFLOP/s + TDVP sweep s/step, FP32-MFMA vs FP64, at <=1e-4 obs err",
        "value": round(value, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms64, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "apply_heff two-site, D=1024, d=2, w=10 (long-range XY alpha=0.75, K=4), "
                               "complex64 on FP32 MFMA (3M)",
                   "D": D, "d": 2, "w": w, "parallelism": "single GPU"},
        "roofline": roofline,
        "gpu_state": {"before_timed_region": state_before, "after_timed_region": state_after},
    }

    if not args.no_extras:
        progress(f"complex64 {value:.0f} GFLOP/s; timing complex128")
        x128 = device_inputs(torch, wl, W, D, w, torch.complex128)
        ms128, prof128, _ = time_heff(pkg, ctx, torch, x128, max(3, args.steps // 2), 1, profile=True)
        del x128
        k128 = max(prof128, key=lambda k: prof128[k]["ms"])
        a128 = prof128[k128]["flops"] / (prof128[k128]["ms"] * 1e-3) * 1e-12
        line["fp64"] = {"gflops": round(F / (ms128 * 1e-3) * 1e-9, 1), "ms_per_step": round(ms128, 4),
                        "kernel": k128, "kernel_tflops": round(a128, 2),
                        "kernel_frac_of_fp64_peak": round(a128 / PEAK_FP64_MFMA_TFLOPS, 4)}
        line["speedup_fp32_vs_fp64"] = round(ms128 / ms64, 2)
        progress("complex64 in the 4M form")
        x4 = device_inputs(torch, wl, W, D, w, torch.complex64)
        ctx.set_gemm_form(4)
        ms4m, _, _ = time_heff(pkg, ctx, torch, x4, max(3, args.steps // 2), 1)
        ctx.set_gemm_form(0)
        del x4
        line["c64_4m"] = {"gflops": round(F / (ms4m * 1e-3) * 1e-9, 1), "ms_per_step": round(ms4m, 4),
                          "speedup_3m_vs_4m": round(ms4m / ms64, 2)}
        progress("D sweep")
        byD = {}
        for Dx in (128, 256, 512):
            r = {}
            for name, dt in (("c64", torch.complex64), ("c128", torch.complex128)):
                xs = device_inputs(torch, wl, W, Dx, w, dt)
                msx, _, _ = time_heff(pkg, ctx, torch, xs, 10, 2)
                r[name] = round(heff2_flops(Dx, w) / (msx * 1e-3) * 1e-9, 1)
                del xs
            byD[str(Dx)] = r
        byD["1024"] = {"c64": line["value"], "c128": line["fp64"]["gflops"]}
        line["gflops_by_D"] = byD
        progress("1TDVP N=10 Ising timing")
        line["ising_n10"] = ising_timing(pkg, ctx, wl)
        if args.sweep_steps > 0:
            progress("2TDVP sweep timing")
            line["sweep"] = sweep_timing(pkg, ctx, args.sweep_steps)
        if not args.no_segments:
            progress("segment-parallel step (N=201, 32 segments)")
            line["segments"] = segments_timing(pkg, ctx, np)
        progress("U(1) block-sparse H_eff at chi = 512")
        line["u1"] = u1_timing(pkg, ctx, torch, np)
        if args.sweep_steps > 0:
            progress("2TDVP sweep, dense against U(1) blocks")
            line["sweep_u1"] = sweep_u1_timing(pkg, ctx, args.sweep_steps)
        if args.grad_steps > 0:
            progress("differentiable 1TDVP timing")
            line["gradient"] = gradient_timing(pkg, ctx, torch, np, args.grad_steps)

    if not args.no_cpu_baseline:
        progress("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(wl, W)
        if not args.no_extras:
            progress("CPU oracle beside the other workloads")
            line["oracle_timings"] = oracle_timings(wl, W)

    ctx.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
