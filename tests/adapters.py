"""Layout adapters between the oracle's index order and the library's.

The oracle keeps environments as beta[a', k, a] and gamma[b', l, b]; the
library stores L[k][a'][a] and R[l][b][b'] so that both GEMMs of H_eff are
plain row-major products.
"""
import numpy as np


def L_from_beta(beta):
    return np.ascontiguousarray(np.transpose(beta, (1, 0, 2)))


def beta_from_L(L):
    return np.ascontiguousarray(np.transpose(L, (1, 0, 2)))


def R_from_gamma(gamma):
    return np.ascontiguousarray(np.transpose(gamma, (1, 2, 0)))


def gamma_from_R(R):
    return np.ascontiguousarray(np.transpose(R, (2, 0, 1)))


def rel_err(x, ref):
    return float(np.linalg.norm(np.asarray(x) - ref) / max(np.linalg.norm(ref), 1e-300))
