"""Reverse-mode gradients: the hand-written apply_heff adjoint kernels against
the oracle's adjoint, and autograd through one-site TDVP against central
finite differences of the FP64 oracle and, at full bond dimension, of exact
diagonalisation."""
import numpy as np
import pytest

import workloads as wl
from oracle import adjoint as oadj
from oracle import mpo as ompo
from oracle import mps as omps
from oracle import spin
from oracle import tdvp as otdvp
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


def _t(x, dt="c128"):
    import torch
    tdt = torch.complex64 if dt == "c64" else torch.complex128
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=tdt)


def _h(t):
    import torch
    return t.detach().to("cpu", dtype=torch.complex128).numpy()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("nsite", [0, 1, 2])
def test_apply_heff_adjoint_matches_oracle(ctx, dt, nsite):
    import paper_1912_06127_amd as pkg
    rng = np.random.default_rng(100 + nsite)
    chil, chir, d, w = 70, 53, 2, 6
    if nsite == 0:
        chir = chil
    beta = wl.cgauss(rng, (chil, w, chil))
    gamma = wl.cgauss(rng, (chir, w, chir))
    W1 = wl.cgauss(rng, (w, w, d, d))
    W2 = wl.cgauss(rng, (w, w, d, d))
    shape = {0: (chil, chir), 1: (chil, d, chir), 2: (chil, d, d, chir)}[nsite]
    theta = wl.cgauss(rng, shape)
    ybar = wl.cgauss(rng, shape)
    print(f"adjoint nsite={nsite} {dt}", flush=True)
    if nsite == 2:
        tb, bb, gb = oadj.heff2_adjoint(beta, W1, W2, gamma, theta, ybar)
        wb = None
        g = pkg.apply_heff_adjoint(ctx, _t(L_from_beta(beta), dt), _t(R_from_gamma(gamma), dt), _t(theta, dt),
                                   _t(ybar, dt), _t(W1, dt), _t(W2, dt), need=("theta", "L", "R"))
    elif nsite == 1:
        tb, bb, wb, gb = oadj.heff1_adjoint(beta, W1, gamma, theta, ybar)
        g = pkg.apply_heff_adjoint(ctx, _t(L_from_beta(beta), dt), _t(R_from_gamma(gamma), dt), _t(theta, dt),
                                   _t(ybar, dt), _t(W1, dt))
    else:
        tb, bb, gb = oadj.heff0_adjoint(beta, gamma, theta, ybar)
        wb = None
        g = pkg.apply_heff_adjoint(ctx, _t(L_from_beta(beta), dt), _t(R_from_gamma(gamma), dt), _t(theta, dt),
                                   _t(ybar, dt))
    ctx.sync()
    assert rel_err(_h(g["theta"]), tb) <= TOL[dt]
    assert rel_err(_h(g["L"]), L_from_beta(bb)) <= TOL[dt]
    assert rel_err(_h(g["R"]), R_from_gamma(gb)) <= TOL[dt]
    if wb is not None:
        assert rel_err(_h(g["W"]), wb) <= TOL[dt]


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("direction", [1, -1])
def test_env_update_adjoint_matches_oracle(ctx, dt, direction):
    """Adjoint identity Re<gbar, dF> = Re<g_x, dx> for each input x of the
    environment update, with dF from the oracle's forward update: central
    differences with step 1 are exact (the update is linear in the environment
    and the MPO tensor, quadratic in the site tensor)."""
    import paper_1912_06127_amd as pkg
    from oracle import env as oenv
    rng = np.random.default_rng(300 + direction)
    chil, chir, d, wl_, wr = 37, 29, 2, 5, 6
    A = wl.cgauss(rng, (chil, d, chir))
    W = wl.cgauss(rng, (wl_, wr, d, d))
    if direction == 1:
        env = wl.cgauss(rng, (chil, wl_, chil))                      # beta [a', k, a]
        fwd = lambda e, a, w: L_from_beta(oenv.update_left(e, a, w))  # L' [l][b'][b]
        env_lib = L_from_beta(env)
        to_lib = L_from_beta
        gbar = wl.cgauss(rng, (wr, chir, chir))
    else:
        env = wl.cgauss(rng, (chir, wr, chir))                        # gamma [b', l, b]
        fwd = lambda e, a, w: R_from_gamma(oenv.update_right(e, a, w))
        env_lib = R_from_gamma(env)
        to_lib = R_from_gamma
        gbar = wl.cgauss(rng, (wl_, chil, chil))
    print(f"env adjoint dir={direction} {dt}", flush=True)
    g = pkg.env_update_adjoint(ctx, direction, _t(env_lib, dt), _t(A, dt), _t(W, dt), _t(gbar, dt))
    ctx.sync()
    tol = TOL[dt] * 10
    for name in ("env", "A", "W"):
        for rep in range(3):
            dx = wl.cgauss(rng, {"env": env.shape, "A": A.shape, "W": W.shape}[name])
            args_p = [env, A, W]
            args_m = [env, A, W]
            i = ("env", "A", "W").index(name)
            args_p[i] = args_p[i] + dx
            args_m[i] = args_m[i] - dx
            dF = (fwd(*args_p) - fwd(*args_m)) / 2.0
            lhs = float(np.real(np.vdot(gbar, dF)))
            dx_lib = to_lib(dx) if name == "env" else dx
            rhs = float(np.real(np.vdot(_h(g[name]), dx_lib)))
            scale = np.linalg.norm(gbar) * np.linalg.norm(dF)
            assert abs(lhs - rhs) <= tol * scale, (name, rep, lhs, rhs)


def ising_fit(N, K=3, alpha=2.0, rmax=16):
    """1/r^alpha fitted on r = 1..max(rmax, N-1): a well-posed pencil for any N."""
    c, lam, _ = ompo.fit_exponentials(1.0 / np.arange(1, max(rmax, N - 1) + 1) ** alpha, K)
    return c, lam


def oracle_loss(bulk, T0, N, dt, steps, site):
    Ws = ompo._boundaries(np.asarray(bulk, dtype=np.complex128), N)
    st = otdvp.MPSState(T0, Ws)
    for _ in range(steps):
        otdvp.tdvp1_step(st, dt)
    return float(omps.expect_sites(st.T, spin.SZ)[site].real)


def gpu_grad(ctx, bulk_np, T0, N, dt, steps, site, compute, checkpoint_every=2):
    import torch
    import paper_1912_06127_amd.autodiff as ad
    cdt = torch.complex64 if compute == "c64" else torch.complex128
    bulk = torch.from_numpy(bulk_np).to("cuda").requires_grad_()
    Ws = ad.sites_from_bulk(bulk, N)
    T = [torch.from_numpy(A).to("cuda") for A in T0]
    T = ad.evolve(ctx, T, Ws, dt, steps, compute=cdt, checkpoint_every=checkpoint_every)
    loss = ad.expect_site(ctx, T, site, torch.from_numpy(spin.SZ).to("cuda"))
    loss.backward()
    return float(loss.detach()), bulk.grad.detach().cpu().numpy()


def directions(c, lam, N):
    """Hermitian MPO directions: the coupling J, the field h and two on-site
    operators (raw entries of the bulk tensor)."""
    K = len(c)
    m = K + 2
    dJ = np.zeros((m, m, 2, 2), dtype=np.complex128)
    for k in range(K):
        dJ[1 + k, m - 1] = c[k] * lam[k] * spin.SZ
    dh = np.zeros_like(dJ)
    dh[0, m - 1] = spin.SX
    dy = np.zeros_like(dJ)
    dy[0, m - 1] = spin.SY
    dz = np.zeros_like(dJ)
    dz[0, m - 1] = spin.SZ
    dirs = {"J": dJ, "h": dh, "onsite_y": dy, "onsite_z": dz}
    # random directions with every block W[k][l] Hermitian: each virtual path is
    # then a Kronecker product of Hermitian matrices, so H stays Hermitian
    rng = np.random.default_rng(2024)
    for i in range(2):
        G = wl.cgauss(rng, (m, m, 2, 2))
        dirs[f"random_hermitian_{i}"] = 0.02 * (G + np.conj(np.transpose(G, (0, 1, 3, 2))))
    return dirs


@pytest.mark.parametrize("compute", ["c128", "c64"])
def test_tdvp1_gradient_matches_oracle_finite_differences(ctx, compute):
    N, dt, steps, site = 8, 0.05, 4, 3
    c, lam = ising_fit(N)
    bulk = ompo.mpo_exponentials(4, c, lam, spin.ising_pairs(), spin.SX, 1.0)[1]
    T0 = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(32, wl.full_rank_bonds(N, 2, 8), 2)))
    print(f"tdvp1 gradient {compute}", flush=True)
    loss, gbar = gpu_grad(ctx, bulk, T0, N, dt, steps, site, compute)
    l0 = oracle_loss(bulk, T0, N, dt, steps, site)
    assert abs(loss - l0) <= (1e-10 if compute == "c128" else 1e-4)
    eps = 1e-4  # central differences: truncation ~1e-12 here, rounding ~1e-12
    for name, V in directions(c, lam, N).items():
        fd = (oracle_loss(bulk + eps * V, T0, N, dt, steps, site) -
              oracle_loss(bulk - eps * V, T0, N, dt, steps, site)) / (2 * eps)
        ad = float(np.real(np.vdot(gbar, V)))
        tol = 1e-9 * max(1.0, abs(fd)) if compute == "c128" else 1e-5 * max(1.0, abs(fd))
        print(f"  {name}: autograd {ad:.12e} oracle FD {fd:.12e} diff {abs(ad - fd):.2e}", flush=True)
        assert abs(ad - fd) <= tol, (name, ad, fd)


def test_tdvp1_gradient_full_rank_matches_exact_diagonalisation(ctx):
    """At full bond dimension 1TDVP is exact, so d<sigma^z>/dh equals the ED value."""
    N, dt, steps, site = 6, 0.05, 4, 2
    c, lam = ising_fit(N)
    g = ompo.eval_exponentials(c, lam, N - 1)
    bulk = ompo.mpo_exponentials(4, c, lam, spin.ising_pairs(), spin.SX, 0.7)[1]
    T0 = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(6, wl.full_rank_bonds(N, 2), 2)))
    psi0 = omps.to_dense(T0)
    Z = spin.site_op(spin.SZ, site + 1, N)

    def ed_loss(h):
        H = spin.longrange_hamiltonian(N, g, spin.ising_pairs(), spin.SX, h)
        psi = spin.ExactEvolution(H).evolve(psi0, dt * steps)
        return float(spin.expval(psi, Z).real)

    fd = (ed_loss(0.7 + 1e-4) - ed_loss(0.7 - 1e-4)) / 2e-4
    _, gbar = gpu_grad(ctx, bulk, T0, N, dt, steps, site, "c128")
    ad = float(np.real(np.vdot(gbar, directions(c, lam, N)["h"])))
    print(f"  full rank: autograd {ad:.12e} ED FD {fd:.12e} diff {abs(ad - fd):.2e}", flush=True)
    assert abs(ad - fd) <= 1e-9, (ad, fd)


def test_checkpointing_does_not_change_gradients(ctx):
    N, dt, steps, site = 6, 0.05, 4, 2
    c, lam = ising_fit(N)
    bulk = ompo.mpo_exponentials(4, c, lam, spin.ising_pairs(), spin.SX, 1.0)[1]
    T0 = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(7, wl.full_rank_bonds(N, 2, 4), 2)))
    _, g1 = gpu_grad(ctx, bulk, T0, N, dt, steps, site, "c128", checkpoint_every=0)
    _, g2 = gpu_grad(ctx, bulk, T0, N, dt, steps, site, "c128", checkpoint_every=2)
    assert np.max(np.abs(g1 - g2)) <= 1e-12 * max(1.0, np.max(np.abs(g1)))


def test_gradient_flows_to_couplings(ctx):
    """J and h as leaves through the differentiable MPO builder."""
    import torch
    import paper_1912_06127_amd.autodiff as ad
    N, dt, steps, site = 6, 0.05, 3, 2
    c, lam = ising_fit(N)
    J = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    h = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    Ws, _ = ad.mpo_sum_of_exponentials(N, c, lam, spin.ising_pairs(), spin.SX, J, h)
    T0 = omps.normalize_centre(omps.right_canonicalize(wl.random_site_tensors(8, wl.full_rank_bonds(N, 2, 4), 2)))
    T = ad.evolve(ctx, [torch.from_numpy(A).to("cuda") for A in T0], Ws, dt, steps)
    loss = ad.expect_site(ctx, T, site, torch.from_numpy(spin.SZ).to("cuda"))
    loss.backward()
    bulk = ompo.mpo_exponentials(4, c, lam, spin.ising_pairs(), spin.SX, 1.0)[1]
    dirs = directions(c, lam, N)
    for name, grad in (("J", J.grad), ("h", h.grad)):
        fd = (oracle_loss(bulk + 1e-4 * dirs[name], T0, N, dt, steps, site) -
              oracle_loss(bulk - 1e-4 * dirs[name], T0, N, dt, steps, site)) / 2e-4
        print(f"  {name}: autograd {float(grad):.12e} oracle FD {fd:.12e}", flush=True)
        assert abs(float(grad) - fd) <= 1e-9 * max(1.0, abs(fd)), (name, float(grad), fd)
