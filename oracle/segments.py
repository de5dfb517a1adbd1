"""Segment-parallel two-site TDVP in the inverse canonical gauge (oracle).

Test infrastructure only: nothing in the product path imports this module.

Inverse canonical gauge (Sec. II A): the state is Psi_1 V_1 Psi_2 ... V_{N-1}
Psi_N with Psi_j = Lambda_{j-1} Gamma_j Lambda_j and V_j = Lambda_j^{-1}, so
that Psi_j V_j is left orthonormal and V_{j-1} Psi_j right orthonormal.  The
two-site local state is Theta = Psi_j V_j Psi_{j+1}; after its update the
truncated SVD Theta = U S Vh gives Psi_j = U S, V_j = 1/S, Psi_{j+1} = S Vh
(Fig. postupdate).  A left environment beta_{j+1} is built from beta_j and
A_j = Psi_j V_j, a right environment gamma_j from gamma_{j+1} and B_{j+1} =
V_j Psi_{j+1} (Fig. environments).

Segment schedule (Sec. III B, Fig. partitioning).  The chain is cut into p
contiguous segments (p = 1 or even, each of at least two sites).  In the
first half of a time step the two central segments sweep away from the centre
and neighbours alternate direction; the second half reverses every direction.
The paper's step-by-step diagrams of the parallel step are not part of the
text, so the following reading is ours; at p = 1 it is exactly the serial
step (Sec. III A):

* Every boundary -- a bond between two segments, and each chain end -- owns
  one boundary pair: (b, b+1) for the bond after site b, (0, 1) for the left
  end and (N-2, N-1) for the right end.  A boundary is *meeting* in a half
  when the segment(s) next to it sweep toward it, else *departing*.
* A segment's own sweep covers sites ls..rs, where ls = lo (or 1 at the
  left chain end) and rs = hi (or N-2 at the right chain end).  Sweeping
  right it does: backward step on ls, then for j = ls..rs-1 the pair (j, j+1)
  forward by dt/2 and a backward step on j+1 (mirror image sweeping left).
  Every site in ls..rs thus gets one backward half step per half.
* First half: before the sweeps, every departing boundary pair is evolved by
  dt/2; after the sweeps every meeting boundary pair is evolved by dt (the
  merged turning point of Sec. III A).  Second half: departing boundary pairs
  (which met in the first half) get nothing, meeting pairs get dt/2 after the
  sweeps -- the other dt/2 is the first operation of the next step.
* The left segment performs a boundary-pair update (Sec. III B); afterwards
  both environments across that bond, beta_{b+1} and gamma_b, are rebuilt.
  Environments of a departing boundary are the ones left by the last update
  there, i.e. out of date (Sec. III D, item i).

One-site variant (``schedule1``, ``step1``; proposed in the Discussion
without a boundary rule): one-site sweeps inside the segments and the same
two-site boundary pairs; see ``schedule1`` for the reading.  ``hybrid_step``
runs two-site steps until the bond dimensions are saturated (``saturated``)
and the one-site schedule from then on.

Repair (Sec. III D, Fig. reorth): the parallel updates break the gauge at
the partition boundaries and the norm drifts; ``reorthonormalize`` brings the
state back to the inverse canonical gauge of the normalised state and
recomputes every environment, a serial step taken now and then.

Within one phase the segments touch disjoint tensors and environments, so
they may run in any order with identical results.  Per step every pair is
evolved forward by dt and every site 1..N-2 backward by dt, as in Eq. proj2site.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .env import trivial_env, update_left, update_right
from .heff import apply_heff0, apply_heff1, apply_heff2
from .krylov import expm_krylov
from .mps import lq
from .tdvp import Truncation, truncation_rank


# --------------------------------------------------------------------- gauge

def to_inverse_canonical(tensors):
    """Any MPS -> (Psi, V) of the normalised state in the inverse canonical
    gauge (Sec. II A).

    Right-orthonormalise, then sweep left to right with SVDs: the singular
    values at bond j are the Schmidt coefficients Lambda_j (unit 2-norm for
    the normalised state), A_j = U is left orthonormal and Psi_j = A_j
    Lambda_j, V_j = 1/Lambda_j.  The global factor is dropped on the way (it
    would overflow for long chains of unnormalised tensors).
    """
    T = [np.array(A, dtype=np.complex128) for A in tensors]
    N = len(T)
    for j in range(N - 1, 0, -1):  # right-orthonormalise by LQ (via QR of the adjoint)
        chil, d, chir = T[j].shape
        Q, R = np.linalg.qr(T[j].reshape(chil, d * chir).conj().T)
        T[j] = Q.conj().T.reshape(Q.shape[1], d, chir)
        T[j - 1] = np.einsum("asb,bc->asc", T[j - 1], R.conj().T, optimize=True)
        T[j - 1] /= np.linalg.norm(T[j - 1])
    Psi, V = [], []
    M = T[0]
    for j in range(N - 1):
        chil, d, chir = M.shape
        U, S, Vh = np.linalg.svd(M.reshape(chil * d, chir), full_matrices=False)
        S = S / np.linalg.norm(S)
        Psi.append((U * S[None, :]).reshape(chil, d, len(S)))
        V.append(1.0 / S)
        M = np.einsum("ab,bsc->asc", S[:, None] * Vh, T[j + 1], optimize=True)
    Psi.append(M)
    return Psi, V


def from_inverse_canonical(Psi, V):
    """Site tensors of the same state in an ordinary MPS (V folded to the right)."""
    T = [Psi[0]]
    for j in range(1, len(Psi)):
        T.append(V[j - 1][:, None, None] * Psi[j])
    return T


# ------------------------------------------------------------------ schedule

def directions(p: int, first_half: bool):
    """+1 (right) or -1 (left) per segment (Fig. partitioning)."""
    if p == 1:
        return [1 if first_half else -1]
    if p % 2:
        raise ValueError("the number of segments must be 1 or even")
    h = p // 2
    dirs = []
    for s in range(p):
        dist = (h - 1 - s) if s < h else (s - h)
        away = -1 if s < h else 1  # away from the centre
        dirs.append(away if dist % 2 == 0 else -away)
    return dirs if first_half else [-x for x in dirs]


@dataclass
class Op:
    kind: str        # "pair", "site" or "bond" (zero-site, one-site schedule)
    j: int           # first site of the pair, or the site
    tau: float       # forward time (negative for backward steps)
    segment: int
    refresh: str     # "left", "right", "both" or "" (pairs only)


@dataclass
class Phase:
    name: str
    ops: list = field(default_factory=list)


def schedule(sizes, dt: float, first_half: bool):
    """Phases of one half step; the ops inside a phase are independent.

    Returns a list of phases: boundary pairs before the sweeps, the sweep
    micro-steps (op i of every still active segment), boundary pairs after.
    """
    p = len(sizes)
    if any(n < 2 for n in sizes):
        raise ValueError("every segment needs at least two sites")
    N = sum(sizes)
    if N < 4:
        raise ValueError("need at least four sites")
    bounds, lo = [], 0
    for n in sizes:
        bounds.append((lo, lo + n - 1))
        lo += n
    dirs = directions(p, first_half)
    half = dt / 2.0

    # boundaries: ("left-end", seg), ("bond", left seg), ("right-end", seg)
    def meets(kind, s):
        if kind == "left-end":
            return dirs[s] == -1
        if kind == "right-end":
            return dirs[s] == 1
        return dirs[s] == 1 and dirs[s + 1] == -1

    boundaries = [("left-end", 0, 0)]
    boundaries += [("bond", s, bounds[s][1]) for s in range(p - 1)]
    boundaries += [("right-end", p - 1, N - 2)]

    before, after = Phase("boundary pairs (departing)"), Phase("boundary pairs (meeting)")
    for kind, s, j in boundaries:
        if meets(kind, s):
            after.ops.append(Op("pair", j, dt if first_half else half, s, "both"))
        elif first_half:
            before.ops.append(Op("pair", j, half, s, "both"))

    sweeps = []
    for s, (lo_s, hi_s) in enumerate(bounds):
        ls, rs = max(lo_s, 1), min(hi_s, N - 2)
        ops = []
        if dirs[s] == 1:
            ops.append(Op("site", ls, -half, s, ""))
            for j in range(ls, rs):
                ops.append(Op("pair", j, half, s, "left"))
                ops.append(Op("site", j + 1, -half, s, ""))
        else:
            ops.append(Op("site", rs, -half, s, ""))
            for j in range(rs - 1, ls - 1, -1):
                ops.append(Op("pair", j, half, s, "right"))
                ops.append(Op("site", j, -half, s, ""))
        sweeps.append(ops)
    phases = [before] if before.ops else []
    for i in range(max(len(o) for o in sweeps)):
        ph = Phase(f"sweep micro-step {i}")
        ph.ops = [o[i] for o in sweeps if i < len(o)]
        phases.append(ph)
    if after.ops:
        phases.append(after)
    return phases


# --------------------------------------------------------------------- state

@dataclass
class SegStats:
    w_total: float = 0.0
    matvecs: int = 0
    pair_updates: int = 0
    site_updates: int = 0
    bond_updates: int = 0


def local_pair_update(Psi_l, V, Psi_r, heff2, tau: float, tr: Truncation, kmax: int, tol: float):
    """One two-site update of the segment schedule on its local data (Sec. III A
    in the inverse canonical gauge, Fig. postupdate): Theta = Psi_l V Psi_r,
    Theta <- exp(-i tau H_eff) Theta by Lanczos (heff2 applies H_eff), then the
    truncated SVD Theta = U S Vh.  Returns (U [chil, d, chi], S, Vh [chi, d, chir],
    discarded weight); the new tensors are Psi_l = U S, V = 1/S, Psi_r = S Vh."""
    theta = np.einsum("asb,b,btc->astc", Psi_l, V, Psi_r, optimize=True)
    theta = expm_krylov(heff2, theta, tau, kmax=kmax, tol=tol)
    chil, d1, d2, chir = theta.shape
    U, S, Vh = np.linalg.svd(theta.reshape(chil * d1, d2 * chir), full_matrices=False)
    chi, w = truncation_rank(S, tr)
    U, S, Vh = U[:, :chi], S[:chi], Vh[:chi, :]
    return U.reshape(chil, d1, chi), S, Vh.reshape(chi, d2, chir), w


class SegmentState:
    """Inverse canonical MPS, MPO and one stored beta/gamma per site.

    ``chi_static``: optional per-bond caps (bond j after site j) for static
    shapes; combined with ``tr`` by taking the smaller chi_max.
    """

    def __init__(self, tensors, Ws, tr: Truncation | None = None, chi_static=None,
                 kmax: int = 40, tol: float = 1e-13):
        self.Psi, self.V = to_inverse_canonical(tensors)
        self.W = [np.asarray(W, dtype=np.complex128) for W in Ws]
        self.N = len(self.Psi)
        self.tr = tr if tr is not None else Truncation()
        self.chi_static = chi_static
        self.kmax, self.tol = kmax, tol
        self.stats = SegStats()
        self.build_environments()

    def build_environments(self):
        """Every beta/gamma from the current gauge (Fig. environments); at
        the start they come from the exactly canonical state (Sec. III B)."""
        N = self.N
        self.beta = [None] * N
        self.gamma = [None] * N
        self.beta[0] = trivial_env()
        self.gamma[N - 1] = trivial_env()
        for j in range(N - 1):
            A = self.Psi[j] * self.V[j][None, None, :]
            self.beta[j + 1] = update_left(self.beta[j], A, self.W[j])
        for j in range(N - 1, 0, -1):
            B = self.V[j - 1][:, None, None] * self.Psi[j]
            self.gamma[j - 1] = update_right(self.gamma[j], B, self.W[j])

    def tensors(self):
        return from_inverse_canonical(self.Psi, self.V)

    def _expm(self, apply, x, tau):
        count = [0]

        def op(v):
            count[0] += 1
            return apply(v)

        out = expm_krylov(op, x, tau, kmax=self.kmax, tol=self.tol)
        self.stats.matvecs += count[0]
        return out

    def site_update(self, j: int, tau: float):
        b, W, g = self.beta[j], self.W[j], self.gamma[j]
        self.Psi[j] = self._expm(lambda x: apply_heff1(b, W, g, x), self.Psi[j], tau)
        self.stats.site_updates += 1

    def pair_update(self, j: int, tau: float, refresh: str):
        tr = self.tr
        if self.chi_static is not None:
            tr = Truncation(min(tr.chi_max, self.chi_static[j]), tr.w_max, tr.eps, tr.multiplet_guard)
        count = [0]

        def op(x):
            count[0] += 1
            return apply_heff2(self.beta[j], self.W[j], self.W[j + 1], self.gamma[j + 1], x)

        U, S, Vh, w = local_pair_update(self.Psi[j], self.V[j], self.Psi[j + 1], op, tau, tr, self.kmax, self.tol)
        self.stats.matvecs += count[0]
        chil, d1, chi = U.shape
        d2, chir = Vh.shape[1], Vh.shape[2]
        U, Vh = U.reshape(chil * d1, chi), Vh.reshape(chi, d2 * chir)
        self.stats.w_total += w
        self.stats.pair_updates += 1
        self.Psi[j] = (U * S[None, :]).reshape(chil, d1, chi)
        self.V[j] = 1.0 / S
        self.Psi[j + 1] = (S[:, None] * Vh).reshape(chi, d2, chir)
        if refresh in ("left", "both"):
            self.beta[j + 1] = update_left(self.beta[j], U.reshape(chil, d1, chi), self.W[j])
        if refresh in ("right", "both"):
            self.gamma[j] = update_right(self.gamma[j + 1], Vh.reshape(chi, d2, chir), self.W[j + 1])

    def bond_update(self, j: int, tau: float, refresh: str):
        """Zero-site step on the bond between sites j and j+1 (one-site
        schedule, Eq. proj1site).  "left" (sweeping right): Psi_j = Q R,
        the bond matrix is R (V_j Psi_{j+1} is right orthonormal) and
        beta_{j+1} comes from Q; "right" (sweeping left): Psi_{j+1} = L Q',
        the bond matrix is L (Psi_j V_j is left orthonormal) and gamma_j comes
        from Q'.  C <- exp(-i tau H_0) C, then C = u s vh restores the inverse
        canonical form across the bond: Psi_j = (Q or Psi_j V_j) u s, V_j =
        1/s, Psi_{j+1} = s vh (V_j Psi_{j+1} or Q'), and the environment on
        the sweep's side is rebuilt from the new isometry."""
        chil, d, chim = self.Psi[j].shape
        chir = self.Psi[j + 1].shape[2]
        if refresh == "left":
            Q, C = np.linalg.qr(self.Psi[j].reshape(chil * d, chim))
            Q = Q.reshape(chil, d, chim)
            Qr = self.V[j][:, None, None] * self.Psi[j + 1]
            beta = update_left(self.beta[j], Q, self.W[j])
            gamma = self.gamma[j]
        else:
            C, Qh = lq(self.Psi[j + 1].reshape(chim, d * chir))
            Qr = Qh.reshape(chim, d, chir)
            Q = self.Psi[j] * self.V[j][None, None, :]
            beta = self.beta[j + 1]
            gamma = update_right(self.gamma[j + 1], Qr, self.W[j + 1])
        C = self._expm(lambda x: apply_heff0(beta, gamma, x), C, tau)
        u, S, vh = np.linalg.svd(C)
        self.Psi[j] = np.einsum("asb,bc->asc", Q, u * S[None, :])
        self.V[j] = 1.0 / S
        self.Psi[j + 1] = np.einsum("ab,bsc->asc", S[:, None] * vh, Qr)
        if refresh == "left":
            self.beta[j + 1] = update_left(self.beta[j], np.einsum("asb,bc->asc", Q, u), self.W[j])
        else:
            self.gamma[j] = update_right(self.gamma[j + 1], np.einsum("ab,bsc->asc", vh, Qr), self.W[j + 1])
        self.stats.bond_updates += 1

    def run(self, op: Op):
        if op.kind == "site":
            self.site_update(op.j, op.tau)
        elif op.kind == "bond":
            self.bond_update(op.j, op.tau, op.refresh)
        else:
            self.pair_update(op.j, op.tau, op.refresh)


def schedule1(sizes, dt: float, first_half: bool):
    """Phases of one half step of the segment-parallel one-site scheme.

    The Discussion proposes a parallel one-site TDVP without giving its
    boundary rule; the reading here keeps the two-site boundary pairs of the
    two-site schedule and runs one-site sweeps inside the segments.  It
    integrates the tangent-space splitting of Eq. proj1site with, at every
    boundary bond b, the terms of sites b, b+1 and bond b replaced by the one
    two-site term of (b, b+1) (which contains them): the pair goes forward,
    every other site forward, every other bond backward.

    Directions and boundary timing are those of ``schedule``: a boundary
    pair departing in the first half goes forward by dt/2 before the sweeps,
    a meeting one by dt after them in the first half and by dt/2 in the
    second.  A segment sweeping right over its own sites a..z (its sites
    minus the ones in boundary pairs) does: the bond from its left boundary
    site backward by dt/2, site a forward by dt/2, then bond j backward and
    site j+1 forward for j = a..z-1, then the bond into its right boundary
    pair backward (mirror image sweeping left); the chain ends have no
    bonds.  At p = 1 this is the serial one-site step.  Inner segments need
    at least three sites, the end segments two.  Bond dimensions are fixed:
    the boundary splits truncate back to the current dimension.
    """
    p = len(sizes)
    if any(n < 2 for n in sizes) or any(n < 3 for n in sizes[1:-1]):
        raise ValueError("end segments need two sites and inner segments three")
    N = sum(sizes)
    if N < 4:
        raise ValueError("need at least four sites")
    bounds, lo = [], 0
    for n in sizes:
        bounds.append((lo, lo + n - 1))
        lo += n
    dirs = directions(p, first_half)
    half = dt / 2.0
    before, after = Phase("boundary pairs (departing)"), Phase("boundary pairs (meeting)")
    for s in range(p - 1):
        b = bounds[s][1]
        if dirs[s] == 1 and dirs[s + 1] == -1:
            after.ops.append(Op("pair", b, dt if first_half else half, s, "both"))
        elif first_half:
            before.ops.append(Op("pair", b, half, s, "both"))
    sweeps = []
    for s, (lo_s, hi_s) in enumerate(bounds):
        a = lo_s + (1 if s > 0 else 0)
        z = hi_s - (1 if s < p - 1 else 0)
        ops = []
        if dirs[s] == 1:
            if s > 0:
                ops.append(Op("bond", lo_s, -half, s, "left"))
            ops.append(Op("site", a, half, s, ""))
            for j in range(a, z):
                ops.append(Op("bond", j, -half, s, "left"))
                ops.append(Op("site", j + 1, half, s, ""))
            if s < p - 1:
                ops.append(Op("bond", z, -half, s, "left"))
        else:
            if s < p - 1:
                ops.append(Op("bond", z, -half, s, "right"))
            ops.append(Op("site", z, half, s, ""))
            for j in range(z - 1, a - 1, -1):
                ops.append(Op("bond", j, -half, s, "right"))
                ops.append(Op("site", j, half, s, ""))
            if s > 0:
                ops.append(Op("bond", lo_s, -half, s, "right"))
        sweeps.append(ops)
    phases = [before] if before.ops else []
    for i in range(max(len(o) for o in sweeps)):
        ph = Phase(f"sweep micro-step {i}")
        ph.ops = [o[i] for o in sweeps if i < len(o)]
        phases.append(ph)
    if after.ops:
        phases.append(after)
    return phases


def step1(st: SegmentState, sizes, dt: float, order=None):
    """One time step of the segment-parallel one-site scheme.  The state
    should be built with ``chi_static`` equal to its bond profile so that the
    boundary pairs keep the bond dimensions fixed.  ``order`` as in ``step``."""
    for first in (True, False):
        for ph in schedule1(sizes, dt, first):
            ops = ph.ops
            if order is not None:
                rank = {s: i for i, s in enumerate(order)}
                ops = sorted(ops, key=lambda o: rank[o.segment])
            for op in ops:
                st.run(op)
    return st


def saturated(st: SegmentState) -> bool:
    """Every bond holds min(chi_max, d^min(j, N-j)) and, with per-bond caps,
    its cap: the bond dimensions can grow no further."""
    N, d = st.N, st.Psi[0].shape[1]
    for j in range(1, N):
        cap = st.tr.chi_max if st.chi_static is None else min(st.tr.chi_max, st.chi_static[j - 1])
        if len(st.V[j - 1]) < min(cap, d ** min(j, N - j)):
            return False
    return True


def hybrid_step(st: SegmentState, sizes, dt: float) -> bool:
    """The hybrid scheme of the Discussion on segments: two-site steps until
    the bond dimensions are saturated, one-site steps from then on.  Returns
    True when the one-site schedule ran."""
    one = getattr(st, "one_site_started", False) or saturated(st)
    if one:
        st.one_site_started = True
        step1(st, sizes, dt)
    else:
        step(st, sizes, dt)
    return one


def norm2(st: SegmentState) -> float:
    """<psi|psi> of the state Psi_1 V_1 Psi_2 ... Psi_N as it stands.  The
    parallel updates break the gauge conditions at the partition boundaries,
    so this drifts from 1 (Sec. III D, item ii, Fig. reorth)."""
    E = np.ones((1, 1), dtype=np.complex128)
    for A in st.tensors():
        E = np.einsum("ab,asc,bsd->cd", E, A.conj(), A)
    return float(E[0, 0].real)


def gauge_defect(st: SegmentState) -> float:
    """Largest deviation from the inverse canonical conditions: Psi_j V_j
    left orthonormal and V_{j-1} Psi_j right orthonormal (Sec. II A)."""
    dev = 0.0
    for j in range(st.N - 1):
        A = st.Psi[j] * st.V[j][None, None, :]
        chil, d, chir = A.shape
        M = A.reshape(chil * d, chir)
        dev = max(dev, np.max(np.abs(M.conj().T @ M - np.eye(chir))))
        B = st.V[j][:, None, None] * st.Psi[j + 1]
        chil, d, chir = B.shape
        M = B.reshape(chil, d * chir)
        if j + 1 < st.N - 1:  # the last tensor carries the norm
            dev = max(dev, np.max(np.abs(M @ M.conj().T - np.eye(chil))))
    return float(dev)


def reorthonormalize(st: SegmentState) -> SegmentState:
    """Serial repair of a segment run (Sec. III D, Fig. reorth): bring the
    state as it stands back to the inverse canonical gauge of the normalised
    state and recompute every environment.  The bond dimensions are kept;
    nothing is truncated, so the state changes only by its normalisation."""
    st.Psi, st.V = to_inverse_canonical(st.tensors())
    st.build_environments()
    return st


def step(st: SegmentState, sizes, dt: float, order=None):
    """One time step of the segment schedule.  ``order`` (a permutation of the
    segment indices) changes the execution order inside each phase; results
    do not depend on it."""
    for first in (True, False):
        for ph in schedule(sizes, dt, first):
            ops = ph.ops
            if order is not None:
                rank = {s: i for i, s in enumerate(order)}
                ops = sorted(ops, key=lambda o: rank[o.segment])
            for op in ops:
                st.run(op)
    return st
