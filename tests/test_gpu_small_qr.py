"""The one-workgroup QR / LQ of small gauge moves (m n <= 4096, at most 64
columns; larger matrices go to rocSOLVER) through the library's right
canonicalisation (Sec. III A: sites N..2 by successive LQ decompositions,
the state in site 1): every site after the first has orthonormal rows, the
state is unchanged (equal to the oracle's canonicalisation and to the input,
as dense vectors), also for a zero-padded product state, whose LQ factors
are rank deficient, and across the size limit of the small path."""
import numpy as np
import pytest

import workloads as wl
from oracle import mps as omps

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1912_06127_amd as pkg
    c = pkg.Context(0)
    yield c
    c.sync()
    c.close()


def _check_right_canonical(T, tol):
    for j in range(1, len(T)):
        chil, d, chir = T[j].shape
        B = T[j].reshape(chil, d * chir)
        assert np.max(np.abs(B @ B.conj().T - np.eye(chil))) <= tol, j


# chi cap 16: every LQ is small (<= 16 x 32); cap 64: 64 x 128 = 8192 elements
# exceed the small path at the centre, so both paths meet in one chain
@pytest.mark.parametrize("cap", [16, 64])
def test_right_canonicalize_random_state(ctx, cap):
    import paper_1912_06127_amd as pkg
    N = 14
    chi = wl.full_rank_bonds(N, 2, cap)
    print(f"right canonicalisation, random state N={N} cap={cap}", flush=True)
    T0 = wl.random_site_tensors(5, chi, 2)
    m = pkg.MPS.from_tensors(ctx, T0)
    m.right_canonicalize()
    T = m.tensors()
    m.close()
    _check_right_canonical(T, 1e-12)
    To = omps.right_canonicalize(T0)
    psi, ref, orig = omps.to_dense(T), omps.to_dense(To), omps.to_dense(T0)
    assert np.linalg.norm(psi - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.linalg.norm(psi - orig) <= 1e-12 * np.linalg.norm(orig)


def test_right_canonicalize_padded_product_state(ctx):
    import paper_1912_06127_amd as pkg
    N = 10
    bits = [j % 2 for j in range(N)]
    chi = wl.full_rank_bonds(N, 2, 32)
    print("right canonicalisation, zero-padded product state", flush=True)
    m = pkg.MPS.init(ctx, N, 2, chi, basis_state=bits)
    T0 = m.tensors()
    m.right_canonicalize()
    T = m.tensors()
    m.close()
    _check_right_canonical(T, 1e-12)
    psi, orig = omps.to_dense(T), omps.to_dense(T0)
    assert abs(np.vdot(orig, psi)) == pytest.approx(1.0, abs=1e-12)
    assert np.linalg.norm(psi - orig) <= 1e-12
