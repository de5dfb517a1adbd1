"""Pins of the U(1) block-sparse oracle (oracle/u1.py): the charge-conserving
MPO equals the Kronecker-built Hamiltonian, the dense contractions map
symmetric inputs to symmetric outputs (the Hamiltonian conserves S^z), and
the block-by-block contractions equal the dense ones on symmetric inputs."""
import numpy as np
import pytest

import workloads as wl
from oracle import env, heff, mpo, spin, u1


def _sym(rng, mask):
    return np.where(mask, wl.cgauss(rng, mask.shape), 0.0)


@pytest.mark.parametrize("pairs_fn,ref_pairs", [(u1.xxx_pairs_u1, spin.xxx_pairs), (u1.xy_pairs_u1, spin.xy_pairs)])
def test_symmetric_mpo_equals_kronecker_and_obeys_charges(pairs_fn, ref_pairs):
    N, K = 7, 2
    c, lam, _ = mpo.fit_exponentials(1.0 / np.arange(1, N) ** 2.0, K)
    g = mpo.eval_exponentials(c, lam, N - 1)
    Ws = mpo.mpo_exponentials(N, c, lam, pairs_fn(), spin.SZ, 0.3)
    H = spin.longrange_hamiltonian(N, g, ref_pairs(), spin.SZ, 0.3)
    assert np.max(np.abs(mpo.mpo_to_dense(Ws) - H)) < 1e-13
    cw = u1.mpo_charges(pairs_fn(), K)
    for j, W in enumerate(Ws):
        cl = cw[:1] if j == 0 else cw
        cr = cw[-1:] if j == N - 1 else cw
        assert not np.any(W[~u1.mask_mpo(cl, u1.Q_SPIN, cr)]), j


def _case(seed, chil, chir, K=2):
    rng = np.random.default_rng(seed)
    ql = wl.u1_labels(chil, 5, 1.5, seed)
    qr = wl.u1_labels(chir, 6, 1.5, seed + 1)
    c, lam, _ = mpo.fit_exponentials(1.0 / np.arange(1, 12) ** 2.0, K)
    W = mpo.mpo_exponentials(4, c, lam, u1.xxx_pairs_u1(), spin.SZ, 0.4)[1]
    cw = u1.mpo_charges(u1.xxx_pairs_u1(), K)
    return rng, ql, qr, W, cw


def test_two_site_heff_blocks_equal_dense_and_conserve_charge():
    rng, ql, qr, W, cw = _case(3, 23, 19)
    qs = u1.Q_SPIN
    # two-site: the right bond sits two sites further, its charges are higher by up to 2
    qr = qr + 1
    beta = _sym(rng, u1.mask_env_left(ql, cw))
    gamma = _sym(rng, u1.mask_env_right(qr, cw))
    mask = u1.mask_two_site(ql, qs, qr)
    theta = _sym(rng, mask)
    y = heff.apply_heff2(beta, W, W, gamma, theta)
    assert np.max(np.abs(y[~mask])) < 1e-13 * np.max(np.abs(y))  # charge conserved
    yb = u1.heff2_blocks(beta, W, W, gamma, theta, ql, qr, qs, cw, cw, cw)
    assert np.linalg.norm(yb - y) <= 1e-12 * np.linalg.norm(y)
    # entries outside the blocks are never read
    noisy = theta + np.where(mask, 0.0, wl.cgauss(rng, theta.shape))
    assert np.linalg.norm(u1.heff2_blocks(beta, W, W, gamma, noisy, ql, qr, qs, cw, cw, cw) - yb) == 0.0


def test_one_site_heff_blocks_equal_dense():
    rng, ql, qr, W, cw = _case(5, 17, 21)
    qs = u1.Q_SPIN
    beta = _sym(rng, u1.mask_env_left(ql, cw))
    gamma = _sym(rng, u1.mask_env_right(qr, cw))
    mask = u1.mask_site(ql, qs, qr)
    theta = _sym(rng, mask)
    y = heff.apply_heff1(beta, W, gamma, theta)
    assert np.max(np.abs(y[~mask])) < 1e-13 * np.max(np.abs(y))
    yb = u1.heff1_blocks(beta, W, gamma, theta, ql, qr, qs, cw, cw)
    assert np.linalg.norm(yb - y) <= 1e-12 * np.linalg.norm(y)


def test_environment_blocks_equal_dense_and_keep_the_charge_rules():
    rng, ql, qr, W, cw = _case(7, 15, 18)
    qs = u1.Q_SPIN
    A = _sym(rng, u1.mask_site(ql, qs, qr))
    beta = _sym(rng, u1.mask_env_left(ql, cw))
    out = env.update_left(beta, A, W)
    assert np.max(np.abs(out[~u1.mask_env_left(qr, cw)])) < 1e-13 * np.max(np.abs(out))
    ob = u1.env_left_blocks(beta, A, W, ql, qr, qs, cw, cw)
    assert np.linalg.norm(ob - out) <= 1e-12 * np.linalg.norm(out)
    gamma = _sym(rng, u1.mask_env_right(qr, cw))
    out = env.update_right(gamma, A, W)
    assert np.max(np.abs(out[~u1.mask_env_right(ql, cw)])) < 1e-13 * np.max(np.abs(out))
    ob = u1.env_right_blocks(gamma, A, W, ql, qr, qs, cw, cw)
    assert np.linalg.norm(ob - out) <= 1e-12 * np.linalg.norm(out)
