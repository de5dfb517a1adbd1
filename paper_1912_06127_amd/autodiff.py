"""Reverse-mode differentiation of one-site TDVP (Sec. II D, Eq. proj1site).

Every effective-Hamiltonian application runs through ``ApplyHeff`` and every
environment update through ``EnvUpdate``: ``torch.autograd.Function``s whose
forwards are the library's ``apply_heff`` / ``env_update`` kernels and whose
backwards are the hand-written ``apply_heff_adjoint`` / ``env_update_adjoint``
kernels (gradients with respect to the state, both environments and the MPO
tensor).  The expectation value of the loss is a chain of environment updates
with a one-channel MPO.  What remains torch operations, chained by autograd,
is the Lanczos recursion on vectors, the small Krylov exponential, the QR/LQ
gauge moves and the product of a bond matrix with the next site tensor.
Environments are held in the compute precision (complex64 runs the
contractions on FP32 MFMA), site tensors and Lanczos vectors in complex128.
Environments are not stored across time steps: ``checkpoint_every`` steps form
one ``torch.utils.checkpoint`` block that is recomputed during the backward
pass.

Layouts follow the library: site tensors A[a][s][b], MPO W[k][l][s'][s],
environments L[k][a'][a] and R[l][b][b'].
"""
from __future__ import annotations

import numpy as np
import torch
from torch.utils.checkpoint import checkpoint

from . import api


def _dense(t, dtype):
    """t in `dtype`, contiguous, with any lazy conjugation or negation applied
    to its memory (the library reads raw device memory)."""
    return t.to(dtype).resolve_conj().resolve_neg().contiguous()


class ApplyHeff(torch.autograd.Function):
    """y = H_eff x for a zero-site (W None) or one-site local state.

    ``compute`` is the dtype the kernel runs in (complex64: FP32 MFMA).  The
    environments are expected in that dtype already (``EnvUpdate`` produces
    them so); the state may be complex128 and is cast on the way in and out.
    """

    @staticmethod
    def forward(ctx_, lib_ctx, compute, x, L, W, R):
        cx = _dense(x, compute)
        cL = _dense(L, compute)
        cR = _dense(R, compute)
        cW = None if W is None else _dense(W, compute)
        y = api.apply_heff(lib_ctx, cL, cR, cx, cW)
        ctx_.save_for_backward(x, cL, cW if cW is not None else torch.empty(0, device=x.device), cR)
        ctx_.lib_ctx = lib_ctx
        ctx_.compute = compute
        ctx_.has_w = W is not None
        ctx_.dtypes = (x.dtype, L.dtype, None if W is None else W.dtype, R.dtype)
        return y.to(x.dtype)

    @staticmethod
    def backward(ctx_, ybar):
        x, cL, cW, cR = ctx_.saved_tensors
        cdt = ctx_.compute
        cx = _dense(x, cdt)
        W = cW if ctx_.has_w else None
        need = []
        if ctx_.needs_input_grad[2]:
            need.append("theta")
        if ctx_.needs_input_grad[3]:
            need.append("L")
        if ctx_.has_w and ctx_.needs_input_grad[4]:
            need.append("W")
        if ctx_.needs_input_grad[5]:
            need.append("R")
        g = api.apply_heff_adjoint(ctx_.lib_ctx, cL, cR, cx, _dense(ybar, cdt), W, need=need)
        xd, Ld, Wd, Rd = ctx_.dtypes
        conv = lambda k, dt: g[k].to(dt) if k in g else None
        return (None, None, conv("theta", xd), conv("L", Ld), conv("W", Wd) if Wd is not None else None,
                conv("R", Rd))


class EnvUpdate(torch.autograd.Function):
    """Environment update (direction +1: left, -1: right) in the compute dtype;
    backward by the library's env_update_adjoint."""

    @staticmethod
    def forward(ctx_, lib_ctx, compute, direction, env, A, W):
        cenv = _dense(env, compute)
        cA = _dense(A, compute)
        cW = _dense(W, compute)
        out = api.env_update(lib_ctx, direction, cenv, cA, cW)
        ctx_.save_for_backward(cenv, cA, cW)
        ctx_.lib_ctx = lib_ctx
        ctx_.direction = direction
        ctx_.dtypes = (env.dtype, A.dtype, W.dtype)
        return out

    @staticmethod
    def backward(ctx_, gout):
        cenv, cA, cW = ctx_.saved_tensors
        need = [k for k, i in (("env", 3), ("A", 4), ("W", 5)) if ctx_.needs_input_grad[i]]
        if not need:
            return None, None, None, None, None, None
        g = api.env_update_adjoint(ctx_.lib_ctx, ctx_.direction, cenv, cA, cW, _dense(gout, cA.dtype), need=need)
        ed, ad, wd = ctx_.dtypes
        conv = lambda k, dt: g[k].to(dt) if k in g else None
        return None, None, None, conv("env", ed), conv("A", ad), conv("W", wd)


def env_left(lib_ctx, compute, L, A, W):
    """L'[l][b'][b] = sum conj(A[a' s' b']) L[k][a'][a] W[k][l][s'][s] A[a s b] (library kernel)."""
    return EnvUpdate.apply(lib_ctx, compute, 1, L, A, W)


def env_right(lib_ctx, compute, R, A, W):
    """R'[k][a][a'] = sum A[a s b] W[k][l][s'][s] R[l][b][b'] conj(A[a' s' b']) (library kernel)."""
    return EnvUpdate.apply(lib_ctx, compute, -1, R, A, W)


class Project(torch.autograd.Function):
    """w - sum_i V_i (V_i^H w) for 1-D vectors V_i (one Gram-Schmidt pass).

    Saves references to its inputs only, so a Krylov run keeps O(k) vectors
    for the backward pass instead of a stacked copy of the basis per step.
    Backward (gradients in the convention g = dl/dRe + i dl/dIm):
    g_w = G - sum_i V_i (V_i^H G), g_{V_i} = -G conj(V_i^H w) - w conj(V_i^H G).
    """

    @staticmethod
    def forward(ctx_, w, *V):
        Vm = torch.stack(V)
        out = w - Vm.T @ (Vm.conj() @ w)
        ctx_.save_for_backward(w, *V)
        return out

    @staticmethod
    def backward(ctx_, G):
        w, *V = ctx_.saved_tensors
        Vm = torch.stack(V)
        c = Vm.conj() @ w
        a = Vm.conj() @ G
        gw = G - Vm.T @ a
        gV = -(c.conj()[:, None] * G[None, :]) - (a.conj()[:, None] * w[None, :])
        return (gw, *gV.unbind(0))


def _tail_weight(alphas, betas, tau):
    """|e_k^T exp(-i tau T) e_1| for the host tridiagonal T (convergence test)."""
    k = len(alphas)
    T = np.diag(np.asarray(alphas, dtype=np.float64))
    if k > 1:
        off = np.asarray(betas, dtype=np.float64)
        T = T + np.diag(off, 1) + np.diag(off, -1)
    lam, Z = np.linalg.eigh(T)
    return abs(np.sum(Z[k - 1] * np.exp(-1j * tau * lam) * Z[0]))


def expm_lanczos(op, x, tau, kmax=40, tol=1e-13, extra=5):
    """exp(-i tau H) x by Lanczos with two Gram-Schmidt passes (differentiable).

    The derivative of a Krylov approximation converges one order later than
    its value, so ``extra`` iterations run past the convergence point (unless
    the space is exhausted) to keep gradients as accurate as the forward.
    The stopping test reads alpha_k and beta_k once per iteration and works on
    the host copy of the tridiagonal matrix; the exponential that enters the
    result is the differentiable one of the final tridiagonal matrix."""
    shape = x.shape
    v = x.reshape(-1)
    beta0 = torch.linalg.vector_norm(v)
    V = [v / beta0]
    alphas, betas = [], []
    ha, hb = [], []  # host copies of alphas, betas
    stop_at = kmax
    for k in range(kmax):
        w = op(V[k].reshape(shape)).reshape(-1)
        a = torch.vdot(V[k], w).real
        w = w - a * V[k]
        if k > 0:
            w = w - betas[-1] * V[k - 1]
        for _ in range(2):
            w = Project.apply(w, *V)
        b = torch.linalg.vector_norm(w)
        alphas.append(a)
        with torch.no_grad():
            a_h, b_h = torch.stack([a.detach(), b.detach()]).tolist()
        ha.append(a_h)
        scale = max(max(abs(t) for t in ha), max(hb, default=0.0))
        exhausted = b_h <= 1e-14 * scale or scale == 0.0 or len(alphas) >= v.numel()
        if stop_at == kmax and b_h * _tail_weight(ha, hb, tau) <= tol:
            stop_at = min(kmax, k + 1 + extra)
        if exhausted or k + 1 >= stop_at:
            break
        betas.append(b)
        hb.append(b_h)
        V.append(w / b)
    T = torch.diag(torch.stack(alphas))
    if len(alphas) > 1:
        off = torch.stack(betas)
        T = T + torch.diag(off, 1) + torch.diag(off, -1)
    y = torch.linalg.matrix_exp((-1j * tau) * T.to(x.dtype))[:, 0]
    out = beta0 * (torch.stack(V[: len(alphas)]).T @ y)
    return out.reshape(shape)


def _lq(M):
    """M = L Q with orthonormal rows of Q (through the QR of M^dagger)."""
    Q, R = torch.linalg.qr(M.conj().T)
    return R.conj().T, Q.conj().T


def right_envs(lib_ctx, T, Ws, compute):
    N = len(T)
    one = torch.ones((1, 1, 1), dtype=compute, device=T[0].device)
    R = [None] * N
    R[N - 1] = one
    for j in range(N - 1, 0, -1):
        R[j - 1] = env_right(lib_ctx, compute, R[j], T[j], Ws[j])
    return R


def _absorb_left(C, A):
    """C[a][b] A[b][s][c] (bond matrix into the next site)."""
    return (C @ A.reshape(A.shape[0], -1)).reshape(C.shape[0], A.shape[1], A.shape[2])


def _absorb_right(A, C):
    """A[a][s][b] C[b][c] (bond matrix into the previous site)."""
    return (A.reshape(-1, A.shape[2]) @ C).reshape(A.shape[0], A.shape[1], C.shape[1])


def tdvp1_step(lib_ctx, T, Ws, dt, compute=torch.complex128, kmax=40, tol=1e-13):
    """One symmetric one-site TDVP step on torch tensors (returns new tensors).

    T: right-canonical site tensors with the centre on site 1; Ws: MPO site
    tensors.  Differentiable with respect to T and Ws.
    """
    T = list(T)
    N = len(T)
    tau = dt / 2.0
    one = torch.ones((1, 1, 1), dtype=compute, device=T[0].device)
    L = [None] * N
    L[0] = one
    R = right_envs(lib_ctx, T, Ws, compute)
    h1 = lambda j: (lambda x: ApplyHeff.apply(lib_ctx, compute, x, L[j], Ws[j], R[j]))
    h0 = lambda j: (lambda x: ApplyHeff.apply(lib_ctx, compute, x, L[j + 1], None, R[j]))
    for j in range(N - 1):
        T[j] = expm_lanczos(h1(j), T[j], tau, kmax, tol)
        chil, d, chir = T[j].shape
        Q, C = torch.linalg.qr(T[j].reshape(chil * d, chir))
        T[j] = Q.reshape(chil, d, chir)
        L[j + 1] = env_left(lib_ctx, compute, L[j], T[j], Ws[j])
        C = expm_lanczos(h0(j), C, -tau, kmax, tol)
        T[j + 1] = _absorb_left(C, T[j + 1])
    T[N - 1] = expm_lanczos(h1(N - 1), T[N - 1], dt, kmax, tol)
    for j in range(N - 1, 0, -1):
        chil, d, chir = T[j].shape
        Lf, Q = _lq(T[j].reshape(chil, d * chir))
        T[j] = Q.reshape(chil, d, chir)
        R[j - 1] = env_right(lib_ctx, compute, R[j], T[j], Ws[j])
        Lf = expm_lanczos(h0(j - 1), Lf, -tau, kmax, tol)
        T[j - 1] = _absorb_right(T[j - 1], Lf)
        T[j - 1] = expm_lanczos(h1(j - 1), T[j - 1], tau, kmax, tol)
    return T


def expect_site(lib_ctx, T, site, O):
    """<psi|O_site|psi>/<psi|psi> (0-based site) as two chains of left
    environment updates with one-channel MPOs (identity, and O on ``site``),
    run by the library's kernels in complex128."""
    dev, cdt = T[0].device, torch.complex128
    d = T[0].shape[1]
    eye = torch.eye(d, dtype=cdt, device=dev).reshape(1, 1, d, d)
    Oj = torch.as_tensor(O, dtype=cdt, device=dev).reshape(1, 1, d, d)
    E = torch.ones((1, 1, 1), dtype=cdt, device=dev)
    num = None
    for j, A in enumerate(T):
        if j == site:
            num = env_left(lib_ctx, cdt, E, A, Oj)
        elif num is not None:
            num = env_left(lib_ctx, cdt, num, A, eye)
        E = env_left(lib_ctx, cdt, E, A, eye)
    return (num[0, 0, 0] / E[0, 0, 0]).real


def evolve(lib_ctx, T, Ws, dt, steps, compute=torch.complex128, checkpoint_every=5, kmax=40, tol=1e-13):
    """`steps` 1TDVP steps; each block of `checkpoint_every` steps is recomputed in backward."""
    T = list(T)
    done = 0
    while done < steps:
        nblk = min(checkpoint_every, steps - done) if checkpoint_every > 0 else steps - done

        def block(*args, nblk=nblk):
            ts = list(args[: len(T)])
            ws = list(args[len(T):])
            for _ in range(nblk):
                ts = tdvp1_step(lib_ctx, ts, ws, dt, compute, kmax, tol)
            return tuple(ts)

        if checkpoint_every and torch.is_grad_enabled():
            T = list(checkpoint(block, *T, *Ws, use_reentrant=False))
        else:
            T = list(block(*T, *Ws))
        done += nblk
    return T


def mpo_sum_of_exponentials(N, c, lam, pairs, onsite, J, h, dtype=torch.complex128, device="cuda"):
    """MPO site tensors of J sum_{i<j} f(j-i) sum_a g_a A_a B_a + h sum X as torch
    functions of the real parameters J and h (Sec. II C, sums of exponentials).

    Returns (Ws, bulk): ``bulk`` is the bulk tensor W[k][l][s'][s]; site j uses
    row 0 (first site), column m-1 (last site) or all of it.
    """
    c = torch.as_tensor(c, dtype=torch.complex128, device=device)
    lam = torch.as_tensor(lam, dtype=torch.complex128, device=device)
    K = len(c)
    m = len(pairs) * K + 2
    d = onsite.shape[0]
    eye = torch.eye(d, dtype=torch.complex128, device=device)
    base = torch.zeros((m, m, d, d), dtype=torch.complex128, device=device)
    WJ = torch.zeros_like(base)
    Wh = torch.zeros_like(base)
    base[0, 0] = eye
    base[m - 1, m - 1] = eye
    Wh[0, m - 1] = torch.as_tensor(onsite, dtype=torch.complex128, device=device)
    for a, (g, A, B) in enumerate(pairs):
        A = torch.as_tensor(A, dtype=torch.complex128, device=device)
        B = torch.as_tensor(B, dtype=torch.complex128, device=device)
        for k in range(K):
            s = 1 + a * K + k
            base[0, s] = A
            base[s, s] = lam[k] * eye
            WJ[s, m - 1] = g * c[k] * lam[k] * B
    bulk = (base + J.to(torch.complex128) * WJ + h.to(torch.complex128) * Wh).to(dtype)
    return sites_from_bulk(bulk, N), bulk


def sites_from_bulk(bulk, N):
    m = bulk.shape[0]
    Ws = []
    for j in range(N):
        if j == 0:
            Ws.append(bulk[0:1])
        elif j == N - 1:
            Ws.append(bulk[:, m - 1:m])
        else:
            Ws.append(bulk)
    return Ws
