"""Pins of the oracle's H_eff adjoint: the adjoint identity
Re<ybar, H(x + dx) - H(x)> = Re<xbar, dx> for each input x (H is linear in
every factor), checked with the forward oracle only."""
import numpy as np
import pytest

import workloads as wl
from oracle import adjoint as oadj
from oracle import heff as oheff


def inner(a, b):
    return float(np.real(np.vdot(a, b)))


@pytest.mark.parametrize("nsite", [0, 1, 2])
def test_adjoint_identity(nsite):
    rng = np.random.default_rng(40 + nsite)
    chil, chir, d, w = 5, 4, 2, 3
    beta = wl.cgauss(rng, (chil, w, chil))
    gamma = wl.cgauss(rng, (chir, w, chir))
    W1 = wl.cgauss(rng, (w, w, d, d))
    W2 = wl.cgauss(rng, (w, w, d, d))
    if nsite == 2:
        theta = wl.cgauss(rng, (chil, d, d, chir))
        f = lambda t, b, g: oheff.apply_heff2(b, W1, W2, g, t)
    elif nsite == 1:
        theta = wl.cgauss(rng, (chil, d, chir))
        f = lambda t, b, g, W=W1: oheff.apply_heff1(b, W, g, t)
    else:
        chir = chil
        gamma = wl.cgauss(rng, (chir, w, chir))
        theta = wl.cgauss(rng, (chil, chir))
        f = lambda t, b, g: oheff.apply_heff0(b, g, t)
    y = f(theta, beta, gamma)
    ybar = wl.cgauss(rng, y.shape)
    if nsite == 2:
        tb, bb, gb = oadj.heff2_adjoint(beta, W1, W2, gamma, theta, ybar)
    elif nsite == 1:
        tb, bb, wb, gb = oadj.heff1_adjoint(beta, W1, gamma, theta, ybar)
    else:
        tb, bb, gb = oadj.heff0_adjoint(beta, gamma, theta, ybar)
    for x, xbar, g in [(theta, tb, lambda dx: f(theta + dx, beta, gamma)),
                       (beta, bb, lambda dx: f(theta, beta + dx, gamma)),
                       (gamma, gb, lambda dx: f(theta, beta, gamma + dx))]:
        dx = wl.cgauss(rng, x.shape)
        assert abs(inner(ybar, g(dx) - y) - inner(xbar, dx)) < 1e-10 * (1 + abs(inner(xbar, dx)))
    if nsite == 1:
        dW = wl.cgauss(rng, W1.shape)
        lhs = inner(ybar, f(theta, beta, gamma, W=W1 + dW) - y)
        assert abs(lhs - inner(wb, dW)) < 1e-10 * (1 + abs(lhs))
