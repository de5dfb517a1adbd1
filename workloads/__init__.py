"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only draws random numbers and fixes workload parameters.  It
holds none of the method's arithmetic (no contraction, no canonicalisation,
no fit): each side turns these raw inputs into MPS/MPO objects with its own
code.  Complex Gaussian entries are (N(0,1) + i N(0,1)) / sqrt(2).
"""
from __future__ import annotations

import numpy as np


def cgauss(rng: np.random.Generator, shape) -> np.ndarray:
    """Complex Gaussian array, unit variance per entry."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def hermitian_stack(seed: int, w: int, D: int) -> np.ndarray:
    """w Hermitian D x D blocks (G + G^H) / (2 sqrt(D)), complex Gaussian G."""
    rng = np.random.default_rng(seed)
    g = cgauss(rng, (w, D, D))
    return np.ascontiguousarray((g + np.conj(np.transpose(g, (0, 2, 1)))) / (2.0 * np.sqrt(D)))


def unit_vector(seed: int, shape) -> np.ndarray:
    """Complex Gaussian tensor scaled to unit Frobenius norm."""
    rng = np.random.default_rng(seed)
    x = cgauss(rng, shape)
    return x / np.linalg.norm(x)


def random_site_tensors(seed: int, chi, d: int):
    """Raw complex Gaussian site tensors [chi[j-1], d, chi[j]] for j = 1..N.

    Not canonical; the consumer orthonormalises them with its own code.
    """
    rng = np.random.default_rng(seed)
    return [cgauss(rng, (chi[j], d, chi[j + 1])) for j in range(len(chi) - 1)]


def full_rank_bonds(N: int, d: int, cap: int | None = None):
    """Bond dimensions chi_0..chi_N = min(d^j, d^(N-j)[, cap])."""
    chi = [min(d ** j, d ** (N - j)) for j in range(N + 1)]
    if cap is not None:
        chi = [min(c, cap) for c in chi]
    return chi


def segment_bounds(sizes):
    """[(lo, hi)] inclusive 0-based site ranges of contiguous segments."""
    out, lo = [], 0
    for n in sizes:
        out.append((lo, lo + n - 1))
        lo += n
    return out


def segment_bond_profile(sizes, d: int, chi_lo: int, chi_hi: int, seed: int):
    """Bond dimensions chi_0..chi_N for a segmented chain with uneven bonds.

    One value D_s per segment drawn uniformly from [chi_lo, chi_hi]; bonds
    inside segment s take D_s, a bond between two segments the smaller of the
    two; then chi_j <= min(d^j, d^(N-j)) and chi_j <= d min(chi_{j-1},
    chi_{j+1}) are imposed until nothing changes, so that every site tensor
    can be an isometry in either direction.
    """
    N = sum(sizes)
    Ds = np.random.default_rng(seed).integers(chi_lo, chi_hi + 1, len(sizes))
    seg_of = np.repeat(np.arange(len(sizes)), sizes)
    chi = [1] * (N + 1)
    for j in range(1, N):
        chi[j] = int(min(Ds[seg_of[j - 1]], Ds[seg_of[j]]))
        chi[j] = min(chi[j], d ** min(j, N - j))
    changed = True
    while changed:
        changed = False
        for j in range(1, N):
            cap = d * min(chi[j - 1], chi[j + 1])
            if chi[j] > cap:
                chi[j] = cap
                changed = True
    return chi


# ---------------------------------------------------------------------------
# Workload parameters (spin-1/2 chains, d = 2).
# ---------------------------------------------------------------------------

ISING_N10 = dict(  # long-range transverse Ising quench, exact MPO, 1TDVP
    N=10, d=2, J=1.0, h=1.0, alpha=3.0, dt=0.01, steps=100, chi_cap=32)

HEFF_MICRO = dict(  # two-site effective-Hamiltonian microbenchmark
    D=(128, 256, 512, 1024), d=2, w=10, alpha=0.75, K=4, fit_rmax=100,
    seed_L=6127, seed_R=7127, seed_theta=8127)

XXX_N64 = dict(  # 2TDVP sweep, 1/r^2 Heisenberg, fitted with K=6 exponentials
    N=64, d=2, alpha=2.0, K=6, dt=0.05, steps=40, w_max=1e-8, eps=1e-12,
    chi_max=512, centre=32)

XY_N201 = dict(  # batched uneven segments, long-range XY
    N=201, d=2, alpha=1.5, K=6, dt=0.01, segments=[11] + [6] * 30 + [10],
    chi_lo=64, chi_hi=1024, seed_chi=201, seed_state=202)

ISING_N32_GRAD = dict(  # differentiation workload
    N=32, d=2, J=1.0, h=1.0, alpha=2.0, K=8, chi_cap=128, dt=0.05, steps=20,
    seed_state=32, site=16, checkpoint_every=5, fd_step=1e-6)


def heff_micro_inputs(D: int, w: int = 10, d: int = 2):
    """Environments and state for the two-site microbenchmark at bond D.

    Returns (Lk, Rk, theta) with Lk[k] and Rk[k] Hermitian D x D blocks,
    theta[D, d, d, D] of unit norm.  Lk[k] is indexed [bra, ket] and Rk[k]
    [ket, bra]; both are Hermitian so the distinction only matters for the
    layout adapters of each side.
    """
    Lk = hermitian_stack(HEFF_MICRO["seed_L"] + D, w, D)
    Rk = hermitian_stack(HEFF_MICRO["seed_R"] + D, w, D)
    theta = unit_vector(HEFF_MICRO["seed_theta"] + D, (D, d, d, D))
    return Lk, Rk, theta


def u1_labels(chi: int, centre: int, spread: float, seed: int):
    """Sorted integer charge labels of a bond of dimension chi: sector sizes
    drawn around `centre` with a Gaussian profile of width `spread` (the shape
    of the S^z sector distribution of a half chain), every label at least
    once in [centre - 3 spread, centre + 3 spread] when chi allows."""
    import numpy as np
    rng = np.random.default_rng(seed)
    qs = np.arange(int(np.floor(centre - 3 * spread)), int(np.ceil(centre + 3 * spread)) + 1)
    wgt = np.exp(-0.5 * ((qs - centre) / max(spread, 1e-9)) ** 2)
    wgt = wgt / wgt.sum()
    labels = rng.choice(qs, size=chi, p=wgt)
    return np.sort(labels)


def u1_symmetric(seed: int, mask):
    """Complex Gaussian entries where the boolean `mask` (a charge-selection
    pattern) is set, zeros elsewhere."""
    import numpy as np
    rng = np.random.default_rng(seed)
    return np.where(mask, cgauss(rng, mask.shape), 0.0)


def u1_patterns(ql, qr, qs, cw):
    """Charge-selection patterns (integer labels; see u1_labels): site / local
    state T[a][s][b] with q(a) + q(s) = q(b), two-site T[a][s1][s2][b], and the
    environments L[k][a'][a] (q(a') - q(a) = c(k)) and R[l][b][b'] (q(b') - q(b) = c(l))."""
    import numpy as np
    ql, qr, qs, cw = (np.asarray(x) for x in (ql, qr, qs, cw))
    site = (ql[:, None, None] + qs[None, :, None]) == qr[None, None, :]
    two = (ql[:, None, None, None] + qs[None, :, None, None] + qs[None, None, :, None]) == qr[None, None, None, :]
    envL = (ql[None, :, None] - ql[None, None, :]) == cw[:, None, None]
    envR = (qr[None, None, :] - qr[None, :, None]) == cw[:, None, None]
    return {"site": site, "two_site": two, "L": envL, "R": envR}
