"""Adjoint of the effective-Hamiltonian application (reverse mode).

For a real loss l and the gradient convention g = dl/dRe z + i dl/dIm z (so
that dl = Re sum conj(g) dz), the gradient of the linear map y = H_eff theta
(Sec. III A, Fig. update) with respect to each factor is the contraction of
ybar with the complex conjugate of all other factors.  Written directly from
that definition in the paper's index order beta[a', k, a], gamma[b', l, b].
Pinned by the adjoint identity Re<ybar, dy> = Re<xbar, dx> for every input x.
"""
from __future__ import annotations

import numpy as np

from .heff import EINSUM_PATH


def heff1_adjoint(beta, W, gamma, theta, ybar):
    """Gradients (theta_bar, beta_bar, W_bar, gamma_bar) of Re<ybar, H1 theta>."""
    c = np.conj
    tb = np.einsum("xky,klps,blc,xpb->ysc", c(beta), c(W), c(gamma), ybar, optimize=EINSUM_PATH)
    bb = np.einsum("xpb,klps,blc,ysc->xky", ybar, c(W), c(gamma), c(theta), optimize=EINSUM_PATH)
    wb = np.einsum("xpb,xky,blc,ysc->klps", ybar, c(beta), c(gamma), c(theta), optimize=EINSUM_PATH)
    gb = np.einsum("xpb,xky,klps,ysc->blc", ybar, c(beta), c(W), c(theta), optimize=EINSUM_PATH)
    return tb, bb, wb, gb


def heff2_adjoint(beta, W1, W2, gamma, theta, ybar):
    """Gradients (theta_bar, beta_bar, gamma_bar) of Re<ybar, H2 theta>."""
    c = np.conj
    tb = np.einsum("xky,klps,lnqt,bnc,xpqb->ystc", c(beta), c(W1), c(W2), c(gamma), ybar, optimize=EINSUM_PATH)
    bb = np.einsum("xpqb,klps,lnqt,bnc,ystc->xky", ybar, c(W1), c(W2), c(gamma), c(theta), optimize=EINSUM_PATH)
    gb = np.einsum("xpqb,xky,klps,lnqt,ystc->bnc", ybar, c(beta), c(W1), c(W2), c(theta), optimize=EINSUM_PATH)
    return tb, bb, gb


def heff0_adjoint(beta_next, gamma, C, ybar):
    """Gradients (C_bar, beta_bar, gamma_bar) of Re<ybar, H0 C>."""
    c = np.conj
    cb = np.einsum("xky,bkc,xb->yc", c(beta_next), c(gamma), ybar, optimize=EINSUM_PATH)
    bb = np.einsum("xb,bkc,yc->xky", ybar, c(gamma), c(C), optimize=EINSUM_PATH)
    gb = np.einsum("xb,xky,yc->bkc", ybar, c(beta_next), c(C), optimize=EINSUM_PATH)
    return cb, bb, gb
