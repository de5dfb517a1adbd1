"""Effective Hamiltonians applied to local states (Sec. III A, Fig. update).

H_eff is never formed: Lanczos only needs H_eff Theta (Sec. III A).  Each
function is the single tensor-network expression of the figure, evaluated
by numpy.einsum in the paper's index order beta[a', k, a], gamma[b', l, b].
"""
from __future__ import annotations

import numpy as np

# Pairwise contraction order chosen by numpy's greedy path search; the memory
# limit is lifted so that intermediates larger than the inputs are allowed.
EINSUM_PATH = ("greedy", 2 ** 40)


def apply_heff2(beta, W1, W2, gamma, theta):
    """y[a', s1', s2', b'] = beta[a',k,a] W1[k,l,s1',s1] W2[l,n,s2',s2] gamma[b',n,b] theta[a,s1,s2,b]."""
    return np.einsum("xky,klps,lnqt,bnc,ystc->xpqb", beta, W1, W2, gamma, theta, optimize=EINSUM_PATH)


def apply_heff1(beta, W, gamma, theta):
    """y[a', s', b'] = beta[a',k,a] W[k,l,s',s] gamma[b',l,b] theta[a,s,b]."""
    return np.einsum("xky,klps,blc,ysc->xpb", beta, W, gamma, theta, optimize=EINSUM_PATH)


def apply_heff0(beta_next, gamma, C):
    """Zero-site (bond) H_eff of the second sum of Eq. proj1site.

    y[a', b'] = beta_{j+1}[a', k, a] gamma_j[b', k, b] C[a, b], the bond
    between sites j and j+1.
    """
    return np.einsum("xky,bkc,yc->xb", beta_next, gamma, C, optimize=EINSUM_PATH)
