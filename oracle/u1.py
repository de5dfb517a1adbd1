"""U(1) charge labels and block-sparse contractions (quantum-number blocks).

Test infrastructure only: nothing in the product path imports this module.

The long-range XY and XXX chains of Sec. IV conserve the total S^z, and the
paper's largest runs exploit it by storing every tensor in blocks labelled by
that charge (Supplemental Material, Implementation: U(1) symmetric tensors of
the TNT library).  Conventions (charges are integers):

* physical index: q(up) = 1, q(down) = 0 (the number of up spins);
* a bond index of the MPS carries the charge of the block to its left, so a
  site tensor A[a, s, b] may be non-zero only where q(a) + q(s) = q(b);
* an MPO bond index k carries c(k), the charge that the operator string to
  its left adds, so W[k, l, s', s] may be non-zero only where
  c(l) = c(k) + q(s') - q(s) (boundary bonds have c = 0);
* left environment beta[a', k, a] (library L[k][a'][a]): non-zero only where
  q(a') - q(a) = c(k); right environment gamma[b', l, b] (library
  R[l][b][b']): only where q(b') - q(b) = c(l).

``heff2_blocks`` / ``heff1_blocks`` / ``env_left_blocks`` /
``env_right_blocks`` evaluate the contractions of oracle/heff.py and
oracle/env.py block by block, visiting only charge-allowed combinations of
sectors and MPO indices.  Pinned (tests/test_oracle_u1.py) against the dense
contractions on symmetric inputs, and the symmetric XXX MPO against the
Kronecker-built Hamiltonian.
"""
from __future__ import annotations

import numpy as np


SP = np.array([[0, 1], [0, 0]], dtype=np.complex128)  # sigma^+ = |up><down| (up is index 0)
SM = SP.T.copy()                                        # sigma^-
Q_SPIN = np.array([1, 0])                               # q(up), q(down)


def xxx_pairs_u1():
    """1/4 (xx + yy + zz) = 1/2 (s+ s- + s- s+) + 1/4 zz: each operator has a
    definite charge (+1, -1, 0), so the MPO is block sparse."""
    SZ = np.diag([1.0, -1.0]).astype(np.complex128)
    return [(0.5, SP, SM), (0.5, SM, SP), (0.25, SZ, SZ)]


def xy_pairs_u1():
    """1/2 (xx + yy) = s+ s- + s- s+."""
    return [(1.0, SP, SM), (1.0, SM, SP)]


def operator_charge(O, qs=Q_SPIN) -> int:
    """The charge q(s') - q(s) shared by every non-zero entry O[s', s]."""
    nz = np.argwhere(np.abs(O) > 0)
    ch = {int(qs[i] - qs[j]) for i, j in nz}
    if len(ch) != 1:
        raise ValueError("operator has no definite charge")
    return ch.pop()


def mpo_charges(pairs, K: int, qs=Q_SPIN):
    """Bond charges of the sum-of-exponentials MPO (oracle/mpo.py layout: 0 =
    nothing placed, (a, k) = A_a placed, m-1 = done)."""
    c = [0]
    for _, A, _ in pairs:
        c += [operator_charge(A, qs)] * K
    return np.array(c + [0])


def sectors(q):
    """[(charge, start, stop)] of a non-decreasing label array."""
    q = np.asarray(q)
    assert np.all(np.diff(q) >= 0), "charge labels must be sorted"
    out, i = [], 0
    while i < len(q):
        j = i
        while j < len(q) and q[j] == q[i]:
            j += 1
        out.append((int(q[i]), i, j))
        i = j
    return out


def mask_site(ql, qs, qr):
    """Allowed entries of a tensor T[a, s, b]: q(a) + q(s) = q(b)."""
    return (np.asarray(ql)[:, None, None] + np.asarray(qs)[None, :, None]) == np.asarray(qr)[None, None, :]


def mask_two_site(ql, qs, qr):
    q = np.asarray(qs)
    return (np.asarray(ql)[:, None, None, None] + q[None, :, None, None] + q[None, None, :, None]
            == np.asarray(qr)[None, None, None, :])


def mask_mpo(cl, qs, cr):
    """Allowed entries of W[k, l, s', s]: c(l) = c(k) + q(s') - q(s)."""
    q = np.asarray(qs)
    return (np.asarray(cl)[:, None, None, None] + q[None, None, :, None] - q[None, None, None, :]
            == np.asarray(cr)[None, :, None, None])


def mask_env_left(q, c):
    """beta[a', k, a]: q(a') - q(a) = c(k)."""
    q = np.asarray(q)
    return (q[:, None, None] - q[None, None, :]) == np.asarray(c)[None, :, None]


def mask_env_right(q, c):
    """gamma[b', l, b]: q(b') - q(b) = c(l)."""
    return mask_env_left(q, c)


def _idx(c, value):
    return np.nonzero(np.asarray(c) == value)[0]


def heff2_blocks(beta, W1, W2, gamma, theta, ql, qr, qs, cl, cm, cr):
    """Two-site H_eff theta (oracle/heff.apply_heff2) block by block: for every
    allowed output block (Qa', s1', s2', Qb') and allowed input block
    (Qa, s1, s2, Qb), only the MPO indices k, l, n whose charges the rules fix
    (c(k) = Qa' - Qa, c(n) = Qb' - Qb, c(l) = c(k) + q(s1') - q(s1))."""
    d = theta.shape[1]
    y = np.zeros_like(theta)
    SL, SR = sectors(ql), sectors(qr)
    for Qo, a0, a1 in SL:
        for s1p in range(d):
            for s2p in range(d):
                Qbo = Qo + qs[s1p] + qs[s2p]
                outs = [s for s in SR if s[0] == Qbo]
                if not outs:
                    continue
                _, b0, b1 = outs[0]
                acc = np.zeros((a1 - a0, b1 - b0), dtype=np.complex128)
                for Qi, c0, c1 in SL:
                    ks = _idx(cl, Qo - Qi)
                    if len(ks) == 0:
                        continue
                    for s1 in range(d):
                        for s2 in range(d):
                            Qbi = Qi + qs[s1] + qs[s2]
                            ins = [s for s in SR if s[0] == Qbi]
                            if not ins:
                                continue
                            _, e0, e1 = ins[0]
                            ns = _idx(cr, Qbo - Qbi)
                            if len(ns) == 0:
                                continue
                            blk = theta[c0:c1, s1, s2, e0:e1]
                            for k in ks:
                                lset = _idx(cm, cl[k] + qs[s1p] - qs[s1])
                                if len(lset) == 0:
                                    continue
                                # sum_l W1[k, l, s1', s1] W2[l, n, s2', s2] for the allowed n
                                wkn = np.einsum("l,ln->n", W1[k, lset, s1p, s1], W2[np.ix_(lset, ns)][:, :, s2p, s2])
                                g = np.einsum("n,bnc->bc", wkn, gamma[b0:b1][:, ns][:, :, e0:e1])  # [b', b]
                                acc += beta[a0:a1, k, c0:c1] @ blk @ g.T
                y[a0:a1, s1p, s2p, b0:b1] = acc
    return y


def heff1_blocks(beta, W, gamma, theta, ql, qr, qs, cl, cr):
    """One-site H_eff theta (oracle/heff.apply_heff1) block by block."""
    d = theta.shape[1]
    y = np.zeros_like(theta)
    SL, SR = sectors(ql), sectors(qr)
    for Qo, a0, a1 in SL:
        for sp in range(d):
            outs = [s for s in SR if s[0] == Qo + qs[sp]]
            if not outs:
                continue
            _, b0, b1 = outs[0]
            acc = np.zeros((a1 - a0, b1 - b0), dtype=np.complex128)
            for Qi, c0, c1 in SL:
                ks = _idx(cl, Qo - Qi)
                for s in range(d):
                    ins = [x for x in SR if x[0] == Qi + qs[s]]
                    if not ins or len(ks) == 0:
                        continue
                    _, e0, e1 = ins[0]
                    for k in ks:
                        ls = _idx(cr, cl[k] + qs[sp] - qs[s])
                        if len(ls) == 0:
                            continue
                        g = np.einsum("l,blc->bc", W[k, ls, sp, s], gamma[b0:b1][:, ls][:, :, e0:e1])
                        acc += beta[a0:a1, k, c0:c1] @ theta[c0:c1, s, e0:e1] @ g.T
            y[a0:a1, sp, b0:b1] = acc
    return y


def env_left_blocks(beta, A, W, ql, qr, qs, cl, cr):
    """beta_{j+1} (oracle/env.update_left) block by block:
    out[b', l, b] = sum conj(A[a', s', b']) beta[a', k, a] W[k, l, s', s] A[a, s, b]."""
    chir = A.shape[2]
    wr = W.shape[1]
    d = A.shape[1]
    out = np.zeros((chir, wr, chir), dtype=np.complex128)
    SL, SR = sectors(ql), sectors(qr)
    for l in range(wr):
        for Qbp, p0, p1 in SR:
            for Qb, b0, b1 in SR:
                if Qbp - Qb != cr[l]:
                    continue
                acc = np.zeros((p1 - p0, b1 - b0), dtype=np.complex128)
                for sp in range(d):
                    bra = [x for x in SL if x[0] == Qbp - qs[sp]]
                    if not bra:
                        continue
                    _, x0, x1 = bra[0]
                    for s in range(d):
                        ket = [x for x in SL if x[0] == Qb - qs[s]]
                        if not ket:
                            continue
                        _, y0, y1 = ket[0]
                        ks = _idx(cl, (Qbp - qs[sp]) - (Qb - qs[s]))
                        for k in ks:
                            if W[k, l, sp, s] == 0:
                                continue
                            acc += W[k, l, sp, s] * (A[x0:x1, sp, p0:p1].conj().T @ beta[x0:x1, k, y0:y1]
                                                     @ A[y0:y1, s, b0:b1])
                out[p0:p1, l, b0:b1] = acc
    return out


def env_right_blocks(gamma, B, W, ql, qr, qs, cl, cr):
    """gamma_{j-1} (oracle/env.update_right) block by block:
    out[a', k, a] = sum B[a, s, b] W[k, l, s', s] gamma[b', l, b] conj(B[a', s', b'])."""
    chil = B.shape[0]
    wl = W.shape[0]
    d = B.shape[1]
    out = np.zeros((chil, wl, chil), dtype=np.complex128)
    SL, SR = sectors(ql), sectors(qr)
    for k in range(wl):
        for Qap, p0, p1 in SL:
            for Qa, a0, a1 in SL:
                if Qap - Qa != cl[k]:
                    continue
                acc = np.zeros((p1 - p0, a1 - a0), dtype=np.complex128)
                for sp in range(d):
                    bra = [x for x in SR if x[0] == Qap + qs[sp]]
                    if not bra:
                        continue
                    _, x0, x1 = bra[0]
                    for s in range(d):
                        ket = [x for x in SR if x[0] == Qa + qs[s]]
                        if not ket:
                            continue
                        _, y0, y1 = ket[0]
                        ls = _idx(cr, (Qap + qs[sp]) - (Qa + qs[s]))
                        for l in ls:
                            if W[k, l, sp, s] == 0:
                                continue
                            acc += W[k, l, sp, s] * (B[p0:p1, sp, x0:x1].conj() @ gamma[x0:x1, l, y0:y1]
                                                     @ B[a0:a1, s, y0:y1].T)
                out[p0:p1, k, a0:a1] = acc
    return out
