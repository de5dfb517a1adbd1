"""U(1) block-sparse H_eff application and environment updates against the
FP64 oracle (oracle/u1.py conventions; the dense contractions of
oracle/heff.py and oracle/env.py on charge-symmetric inputs, which the block
oracle reproduces).  Ragged sectors spanning several GEMM tiles, one-, two-
and zero-site, both precisions, and the shape of the N = 64 XXX quench at its
bond cap (chi = 512, w = 20) with a half-chain S^z sector profile.

Bars as for the dense path: 1e-12 (complex128) and 1e-5 (complex64)
relative, plus exact zeros outside the allowed blocks."""
import numpy as np
import pytest

import workloads as wl
from oracle import env as oenv
from oracle import heff as oheff
from oracle import mpo as ompo
from oracle import spin
from oracle import u1
from tests.adapters import L_from_beta, R_from_gamma, rel_err

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}


@pytest.fixture(scope="module")
def ctx():
    import paper_1912_06127_amd as pkg
    c = pkg.Context(0)
    yield c
    c.sync()
    c.close()


def _t(x, dt):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", torch.complex64 if dt == "c64" else torch.complex128)


def _h(t):
    import torch
    return t.detach().to("cpu", torch.complex128).numpy()


def _sym(rng, mask):
    return np.where(mask, wl.cgauss(rng, mask.shape), 0.0)


def _xxx_bulk(K):
    c, lam, _ = ompo.fit_exponentials(1.0 / np.arange(1, 64) ** 2.0, K)
    return ompo.mpo_exponentials(4, c, lam, u1.xxx_pairs_u1())[1], u1.mpo_charges(u1.xxx_pairs_u1(), K)


CASES = [  # nsite, chil, chir, spread, K
    (2, 150, 170, 2.0, 3),
    (2, 37, 29, 1.0, 2),
    (1, 140, 133, 2.5, 3),
    (0, 96, 96, 2.0, 3),
]


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "n%d_%dx%d" % c[:3])
def test_apply_heff_u1_matches_oracle(ctx, dt, case):
    import paper_1912_06127_amd as pkg
    nsite, chil, chir, spread, K = case
    rng = np.random.default_rng(chil * 7 + chir)
    W, cw = _xxx_bulk(K)
    qs = u1.Q_SPIN
    ql = wl.u1_labels(chil, 10, spread, chil)
    qr = ql if nsite == 0 else wl.u1_labels(chir, 10 + nsite / 2.0, spread, chir)
    beta = _sym(rng, u1.mask_env_left(ql, cw))
    gamma = _sym(rng, u1.mask_env_right(qr, cw))
    if nsite == 2:
        mask = u1.mask_two_site(ql, qs, qr)
    elif nsite == 1:
        mask = u1.mask_site(ql, qs, qr)
    else:
        mask = ql[:, None] == qr[None, :]
    theta = _sym(rng, mask)
    if nsite == 2:
        ref = oheff.apply_heff2(beta, W, W, gamma, theta)
        W1, W2 = _t(W, dt), _t(W, dt)
    elif nsite == 1:
        ref = oheff.apply_heff1(beta, W, gamma, theta)
        W1, W2 = _t(W, dt), None
    else:
        ref = oheff.apply_heff0(beta, gamma, theta)
        W1 = W2 = None
    print(f"apply_heff_u1 nsite={nsite} {chil}x{chir} sectors {len(u1.sectors(ql))}/{len(u1.sectors(qr))} {dt}",
          flush=True)
    y = pkg.apply_heff_u1(ctx, _t(L_from_beta(beta), dt), _t(R_from_gamma(gamma), dt), _t(theta, dt), W1, W2,
                          q_left=ql, q_right=qr, q_phys=qs, c_left=cw, c_right=cw)
    ctx.sync()
    yh = _h(y)
    assert rel_err(yh, ref) <= TOL[dt]
    assert not np.any(yh[~mask])
    if nsite == 2 and chil < 50:  # the block-by-block oracle as well
        yb = u1.heff2_blocks(beta, W, W, gamma, theta, ql, qr, qs, cw, cw, cw)
        assert rel_err(yh, yb) <= TOL[dt]


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("direction", [1, -1])
def test_env_update_u1_matches_oracle(ctx, dt, direction):
    import paper_1912_06127_amd as pkg
    chil, chir, K = 120, 137, 3
    rng = np.random.default_rng(500 + direction)
    W, cw = _xxx_bulk(K)
    qs = u1.Q_SPIN
    ql = wl.u1_labels(chil, 10, 2.0, 11)
    qr = wl.u1_labels(chir, 10.5, 2.0, 12)
    A = _sym(rng, u1.mask_site(ql, qs, qr))
    print(f"env_update_u1 dir={direction} {dt}", flush=True)
    if direction == 1:
        beta = _sym(rng, u1.mask_env_left(ql, cw))
        ref = L_from_beta(oenv.update_left(beta, A, W))
        out = pkg.env_update_u1(ctx, 1, _t(L_from_beta(beta), dt), _t(A, dt), _t(W, dt), q_left=ql, q_right=qr,
                                q_phys=qs, c_left=cw, c_right=cw)
        mask = L_from_beta(u1.mask_env_left(qr, cw))
    else:
        gamma = _sym(rng, u1.mask_env_right(qr, cw))
        ref = R_from_gamma(oenv.update_right(gamma, A, W))
        out = pkg.env_update_u1(ctx, -1, _t(R_from_gamma(gamma), dt), _t(A, dt), _t(W, dt), q_left=ql, q_right=qr,
                                q_phys=qs, c_left=cw, c_right=cw)
        mask = R_from_gamma(u1.mask_env_right(ql, cw))
    ctx.sync()
    oh = _h(out)
    assert rel_err(oh, ref) <= TOL[dt]
    assert not np.any(oh[~mask])


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_apply_heff_u1_at_the_quench_bond_cap(ctx, dt):
    """Two-site, chi = 512 on both bonds, w = 20 (XXX, K = 6): the whole output
    against the oracle, and equal to the dense library path."""
    import paper_1912_06127_amd as pkg
    chi = 512
    rng = np.random.default_rng(512)
    W, cw = _xxx_bulk(6)
    assert W.shape[0] == 20
    qs = u1.Q_SPIN
    ql = wl.u1_labels(chi, 16, 2.5, 31)
    qr = wl.u1_labels(chi, 17, 2.5, 32)
    beta = _sym(rng, u1.mask_env_left(ql, cw))
    gamma = _sym(rng, u1.mask_env_right(qr, cw))
    theta = _sym(rng, u1.mask_two_site(ql, qs, qr))
    ref = oheff.apply_heff2(beta, W, W, gamma, theta)
    L, R, th, Wd = _t(L_from_beta(beta), dt), _t(R_from_gamma(gamma), dt), _t(theta, dt), _t(W, dt)
    print(f"apply_heff_u1 chi=512 w=20 sectors {len(u1.sectors(ql))} {dt}", flush=True)
    y = pkg.apply_heff_u1(ctx, L, R, th, Wd, Wd, q_left=ql, q_right=qr, q_phys=qs, c_left=cw, c_right=cw)
    yd = pkg.apply_heff(ctx, L, R, th, Wd, Wd)
    ctx.sync()
    assert rel_err(_h(y), ref) <= TOL[dt]
    assert rel_err(_h(y), _h(yd)) <= 2 * TOL[dt]


def test_apply_heff_u1_rejects_unsorted_labels(ctx):
    import paper_1912_06127_amd as pkg
    W, cw = _xxx_bulk(2)
    chi = 8
    q = np.array([0, 1, 1, 0, 2, 2, 3, 3])
    L = _t(np.zeros((W.shape[0], chi, chi)), "c128")
    th = _t(np.zeros((chi, 2, 2, chi)), "c128")
    Wd = _t(W, "c128")
    with pytest.raises(pkg.TDVPError) as e:
        pkg.apply_heff_u1(ctx, L, L, th, Wd, Wd, q_left=q, q_right=np.sort(q), q_phys=u1.Q_SPIN, c_left=cw,
                          c_right=cw)
    assert e.value.status == 1
