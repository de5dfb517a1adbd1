"""Host-side checks of the C ABI: the library loads, exports what the header
declares, and rejects bad arguments without touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1912_06127_amd as pkg
from paper_1912_06127_amd import _lib
from oracle import mpo as omp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "tdvp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^(?:int|size_t|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_header_function():
    lib = _lib.load()
    names = header_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES)


def test_version_and_default_options():
    lib = _lib.load()
    assert lib.tdvp_version().startswith(b"tdvp-gfx950")
    o = _lib.Opts()
    assert lib.tdvp_opts_default(C.byref(o)) == 0
    assert o.compute == _lib.TDVP_C128 and o.krylov_max == 40 and o.multiplet_guard == 1
    assert o.imaginary == 0 and o.exp_method == 0
    assert lib.tdvp_opts_default(None) == 1
    with pytest.raises(ValueError):
        pkg.TDVPOptions(exp_method="pade").to_c()


def test_taylor_degree_bounds_match_published_table():
    """theta_m of the truncated-Taylor exponential, generated here from the
    backward-error definition, against the table published with the method
    (Al-Mohy and Higham 2011, three significant digits) as shipped by scipy's
    implementation of it."""
    em = pytest.importorskip("scipy.sparse.linalg._expm_multiply")
    ref = getattr(em, "_theta", None)
    if not ref:
        pytest.skip("scipy does not expose the published table")
    text = open(os.path.join(ROOT, "paper_1912_06127_amd", "csrc", "taylor_theta.inc")).read()
    vals = {int(m): float(v) for v, m in re.findall(r"^\s+([0-9.eE+-]+),\s+// m = (\d+)$", text, flags=re.M)}
    assert sorted(vals) == list(range(1, 56))
    assert all(vals[m] < vals[m + 1] for m in range(1, 55))
    for m, t in ref.items():
        # m = 1: the published 2.29e-16 against 2u = 2.22e-16 from the leading term
        assert abs(vals[m] / t - 1.0) < (0.04 if m == 1 else 0.01), (m, vals[m], t)


def test_null_arguments_are_rejected():
    lib = _lib.load()
    assert lib.tdvp_ctx_destroy(None) == 1
    assert lib.tdvp_ctx_sync(None) == 1
    assert lib.apply_heff(None, 2, 0, 4, 4, 2, 3, 3, 3, None, None, None, None, None, None) == 1
    assert lib.env_update(None, 1, 0, 4, 4, 2, 3, 3, None, None, None, None) == 1
    assert lib.mps_destroy(None) == 1 and lib.mpo_destroy(None) == 1
    assert lib.tdvp1_step(None, None, None, 0.1, None, None) == 1
    assert lib.tdvp_last_error(None) == b"null context"
    h = C.c_void_p()
    assert lib.tdvp_ctx_create(0, None, _lib.ALLOC_FN(), _lib.FREE_FN(), None, None) == 1


def _sum_exp(c, lam, R):
    """Re sum_k c_k lam_k^r for r = 1..R."""
    return ((np.asarray(lam)[None, :] ** np.arange(1, R + 1)[:, None]) @ np.asarray(c)).real


def test_library_fit_matches_oracle_fit():
    # the library (host C++) and the oracle (numpy) implement the fit independently
    for alpha, K, R in [(0.75, 4, 100), (2.0, 6, 63), (1.5, 6, 200), (2.0, 8, 31), (2.0, 12, 200)]:
        c1, l1, e1 = pkg.fit.fit_power_law(alpha, K, R)
        c2, l2, e2 = omp.fit_exponentials(1.0 / np.arange(1, R + 1) ** alpha, K)
        g1 = _sum_exp(c1, l1, R)
        g2 = omp.eval_exponentials(c2, l2, R)[1:]
        assert np.max(np.abs(g1 - g2)) < max(1e-10, 1e-3 * e2), (alpha, K, R)
        assert abs(e1 - e2) < max(1e-10, 1e-3 * e2), (alpha, K, R, e1, e2)
        assert abs(e1 - np.max(np.abs(g1 - np.arange(1, R + 1) ** -alpha))) < 1e-15
        assert all(np.min(np.abs(l1 - w)) < 1e-8 for w in l2), (l1, l2)


def test_library_fit_recovers_exponential_sums_and_rejects_bad_sizes():
    r = np.arange(1, 41)
    # a real pair and a complex-conjugate pair: 2 Re(c lam^r) = c lam^r + conj(c lam^r)
    lam_c = 0.85 * np.exp(0.4j)
    f = 0.7 * 0.9 ** r - 0.2 * (-0.5) ** r + 2 * ((0.3 - 0.1j) * lam_c ** r).real
    c, lam, err = pkg.fit.fit_exponentials(f, 4)
    assert err < 1e-12
    want = np.array([0.9, -0.5, lam_c, np.conj(lam_c)])
    assert all(np.min(np.abs(lam - w)) < 1e-10 for w in want), lam
    assert np.max(np.abs(_sum_exp(c, lam, 40) - f)) < 1e-12
    with pytest.raises(pkg.TDVPError):
        pkg.fit.fit_exponentials(1.0 / np.arange(1, 6) ** 2.0, 3)  # fewer than 2K samples
    with pytest.raises(pkg.TDVPError):
        pkg.fit.fit_exponentials(np.ones(10), 0)
    bad = np.ones(10)
    bad[3] = np.nan
    with pytest.raises(pkg.TDVPError):
        pkg.fit.fit_exponentials(bad, 2)


@pytest.mark.parametrize("sizes", [[10], [5, 5], [3, 2, 2, 3], [2, 2, 2, 2, 2, 2], [11] + [6] * 30 + [10]])
def test_library_segment_schedule_equals_oracle(sizes):
    """The library's segment schedule (host logic, no device) lists the same
    operations, phase by phase, as the oracle's reading of Sec. III B."""
    import paper_1912_06127_amd as pkg
    from oracle import segments as oseg
    for first in (True, False):
        got = pkg.segment_schedule(sizes, 0.1, first)
        ref = []
        for p, ph in enumerate(oseg.schedule(sizes, 0.1, first)):
            for op in ph.ops:
                ref.append((p, 2 if op.kind == "pair" else 1, op.j, op.tau))
        assert sorted(got) == sorted(ref)
    with pytest.raises(pkg.TDVPError):
        pkg.segment_schedule([3, 3, 3], 0.1, True)


@pytest.mark.parametrize("sizes", [[10], [5, 5], [2, 3, 3, 2], [3, 4, 4, 3, 3, 3], [11] + [6] * 30 + [10]])
def test_library_one_site_schedule_equals_oracle(sizes):
    """The one-site schedule (host logic) lists the oracle's operations phase by phase."""
    import paper_1912_06127_amd as pkg
    from oracle import segments as oseg
    code = {"pair": 2, "site": 1}
    for first in (True, False):
        got = pkg.segment_schedule(sizes, 0.1, first, one_site=True)
        ref = []
        for p, ph in enumerate(oseg.schedule1(sizes, 0.1, first)):
            for op in ph.ops:
                k = code.get(op.kind) or (3 if op.refresh == "left" else 4)
                ref.append((p, k, op.j, op.tau))
        assert sorted(got) == sorted(ref)
    with pytest.raises(pkg.TDVPError):
        pkg.segment_schedule([3, 2, 2, 3], 0.1, True, one_site=True)


def test_refined_fit_lowers_the_maximum_error():
    """Levenberg-Marquardt with Lawson reweighting after the matrix pencil:
    never worse, clearly better on power laws, every channel still decaying,
    and an exact sum of exponentials stays exact."""
    from paper_1912_06127_amd import fit
    for alpha, K, R in [(2.0, 6, 63), (1.5, 6, 200), (0.75, 4, 100)]:
        _, _, e0 = fit.fit_power_law(alpha, K, R)
        c, lam, e1 = fit.fit_power_law(alpha, K, R, refine=True)
        assert e1 <= e0 / 1.5
        assert np.all(np.abs(lam) < 1.0)
        vals = _sum_exp(c, lam, R)
        assert np.max(np.abs(vals - np.arange(1, R + 1) ** -alpha)) <= e1 * (1 + 1e-9)
    r = np.arange(1, 41)
    f = 0.7 * 0.9 ** r + 0.3 * (-0.5) ** r
    c, lam, err = fit.fit_exponentials(f, 2, refine=True)
    assert err < 1e-13


def test_taylor_degree_bounds_are_reproduced_by_their_generator():
    """The shipped table is what its generator computes from the definition
    (a few degrees, recomputed here in 80-digit arithmetic)."""
    import importlib.util
    pytest.importorskip("mpmath")
    path = os.path.join(ROOT, "paper_1912_06127_amd", "csrc", "taylor_theta.py")
    spec = importlib.util.spec_from_file_location("taylor_theta_gen", path)
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    text = open(os.path.join(ROOT, "paper_1912_06127_amd", "csrc", "taylor_theta.inc")).read()
    vals = {int(m): float(v) for v, m in re.findall(r"^\s+([0-9.eE+-]+),\s+// m = (\d+)$", text, flags=re.M)}
    fact = [gen.mp.mpf(1)]
    for n in range(1, gen.K + 1):
        fact.append(fact[-1] * n)
    for m in (2, 12, 55):
        assert abs(float(gen.theta(m, fact)) / vals[m] - 1.0) < 1e-14, m
