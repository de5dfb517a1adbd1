"""Python binding of the gfx950 TDVP library (argument marshalling only).

Every computation happens in libtdvp.so on the GPU; this module converts
torch tensors and numpy arrays into pointers and sizes, checks status codes
and turns them into exceptions.  torch supplies device memory (through the
caching allocator, handed to the library as allocation callbacks) and the
stream.
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import TDVP_C64, TDVP_C128, MpoSpec, Opts, SegOpts, Stats


class TDVPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_lib.STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(ctx_handle, rc: int):
    if rc != 0:
        lib = _lib.load()
        msg = lib.tdvp_last_error(ctx_handle).decode() if ctx_handle else ""
        raise TDVPError(rc, msg)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _c128(x) -> np.ndarray:
    """Host complex128 array as contiguous interleaved doubles."""
    return np.ascontiguousarray(np.asarray(x, dtype=np.complex128)).view(np.float64)


_LIVE_CONTEXTS = weakref.WeakSet()


@atexit.register
def _close_all_contexts():
    # Library objects must be destroyed before their context, and before
    # torch (whose allocator backs them) is torn down at interpreter exit.
    for c in list(_LIVE_CONTEXTS):
        c.close()


class Context:
    """Device, stream and allocator for library calls.

    With ``torch_allocator=True`` the library's device memory comes from
    torch's caching allocator on the context stream.  Closing the context
    first closes every MPS and MPO created on it.
    """

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None,
                 torch_allocator: bool = True):
        lib = _lib.load()
        self._children = weakref.WeakSet()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._sizes = {}
        if torch_allocator:
            dev = device

            def _alloc(nbytes, stream_ptr, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream_ptr or 0))
                except Exception:
                    return None

            def _free(ptr, nbytes, stream_ptr, user):
                if ptr:
                    torch.cuda.caching_allocator_delete(int(ptr))

            self._alloc = _lib.ALLOC_FN(_alloc)
            self._free = _lib.FREE_FN(_free)
        else:
            self._alloc = _lib.ALLOC_FN()
            self._free = _lib.FREE_FN()
        h = C.c_void_p()
        rc = lib.tdvp_ctx_create(device, C.c_void_p(self.stream.cuda_stream), self._alloc, self._free,
                                 None, C.byref(h))
        if rc != 0:
            raise TDVPError(rc, "tdvp_ctx_create failed")
        self.handle = h
        _LIVE_CONTEXTS.add(self)

    def _adopt(self, obj):
        if not self.handle:
            raise RuntimeError("context is closed")
        self._children.add(obj)

    def sync(self):
        _check(self.handle, _lib.load().tdvp_ctx_sync(self.handle))

    def profile(self, on: bool = True):
        """Bracket every library kernel launch with HIP events."""
        _check(self.handle, _lib.load().tdvp_profile_enable(self.handle, int(on)))

    def set_gemm_form(self, form: int):
        """Complex-GEMM form of apply_heff / env_update / apply_heff_batched on
        this context: 0 default (3M for complex64), 3 or 4."""
        _check(self.handle, _lib.load().tdvp_ctx_set_gemm_form(self.handle, int(form)))

    def profile_read(self) -> dict:
        """{kernel: {ms, flops, bytes, count}} since the last read (synchronises)."""
        n = 256
        names = C.create_string_buffer(64 * n)
        ms, fl, by = np.zeros(n), np.zeros(n), np.zeros(n)
        cnt = np.zeros(n, dtype=np.int64)
        nout = C.c_int()
        rc = _lib.load().tdvp_profile_read(self.handle, n, names, _dptr(ms), _dptr(fl), _dptr(by),
                                           cnt.ctypes.data_as(C.POINTER(C.c_long)), C.byref(nout))
        _check(self.handle, rc)
        out = {}
        raw = names.raw
        for i in range(nout.value):
            name = raw[64 * i:64 * (i + 1)].split(b"\0", 1)[0].decode()
            out[name] = {"ms": float(ms[i]), "flops": float(fl[i]), "bytes": float(by[i]), "count": int(cnt[i])}
        return out

    def close(self):
        if getattr(self, "handle", None):
            for child in list(self._children):
                child.close()
            _lib.load().tdvp_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.complex64:
        return TDVP_C64
    if t.dtype == torch.complex128:
        return TDVP_C128
    raise TypeError(f"expected complex64 or complex128, got {t.dtype}")


def _dev(t: torch.Tensor, dtype) -> C.c_void_p:
    if not t.is_cuda or not t.is_contiguous() or t.dtype != dtype:
        raise ValueError("tensor must be a contiguous device tensor of the common dtype")
    if t.is_conj() or t.is_neg():
        # a lazily conjugated (or negated) view: its memory does not hold its values
        raise ValueError("tensor has a pending conjugation or negation; call resolve_conj()/resolve_neg() first")
    return C.c_void_p(t.data_ptr())


def apply_heff(ctx: Context, L, R, theta, W1=None, W2=None, out=None, noalloc: bool = False) -> torch.Tensor:
    """H_eff theta for a zero-, one- or two-site local state.

    L [wl][chil][chil], R [wr][chir][chir]; theta [chil][chir] (zero-site),
    [chil][d][chir] (one-site, W1 [wl][wr][d][d]) or [chil][d][d][chir]
    (two-site, W1 [wl][wm][d][d], W2 [wm][wr][d][d]).  ``noalloc`` calls the
    library's allocation-free entry point (intermediates in its fixed
    per-device scratch array; pass ``out`` to keep the call itself free of
    allocations).
    """
    nsite = theta.dim() - 2
    dt = theta.dtype
    wl, chil = L.shape[0], L.shape[1]
    wr, chir = R.shape[0], R.shape[1]
    d = theta.shape[1] if nsite >= 1 else 1
    wm = W1.shape[1] if nsite == 2 else wl
    if out is None:
        out = torch.empty_like(theta)
    ptr = lambda t: _dev(t, dt) if t is not None else C.c_void_p()
    lib = _lib.load()
    fn = lib.apply_heff_noalloc if noalloc else lib.apply_heff
    rc = fn(ctx.handle, nsite, _dtype_code(theta), chil, chir, d, wl, wm, wr,
            ptr(L), ptr(W1), ptr(W2), ptr(R), ptr(theta), ptr(out))
    _check(ctx.handle, rc)
    return out


def apply_heff_noalloc_max_bytes() -> int:
    """Size of the fixed per-device scratch array of the allocation-free H_eff call."""
    return int(_lib.load().apply_heff_noalloc_max_bytes())


def apply_heff_batched(ctx: Context, problems):
    """H_eff theta for many local states at once.

    problems: sequence of (L, R, theta, W1, W2) tuples as for apply_heff (W1,
    W2 may be None); all tensors of one dtype.  Returns the list of outputs.
    """
    if not problems:
        return []
    dt = problems[0][2].dtype
    descs = (_lib.HeffDesc * len(problems))()
    outs, keep = [], []
    ptr = lambda t: _dev(t, dt).value if t is not None else None
    for i, (L, R, theta, W1, W2) in enumerate(problems):
        nsite = theta.dim() - 2
        out = torch.empty_like(theta)
        outs.append(out)
        keep += [L, R, theta, W1, W2]
        q = descs[i]
        q.nsite = nsite
        q.chil, q.chir = L.shape[1], R.shape[1]
        q.d = theta.shape[1] if nsite >= 1 else 1
        q.wl, q.wr = L.shape[0], R.shape[0]
        q.wm = W1.shape[1] if nsite == 2 else L.shape[0]
        q.L, q.R, q.theta, q.out = ptr(L), ptr(R), ptr(theta), ptr(out)
        q.W1, q.W2 = ptr(W1), ptr(W2)
    rc = _lib.load().apply_heff_batched(ctx.handle, _dtype_code(problems[0][2]), len(problems), descs)
    _check(ctx.handle, rc)
    return outs


def apply_heff_adjoint(ctx: Context, L, R, theta, ybar, W1=None, W2=None, need=("theta", "L", "R", "W")):
    """Gradients of Re<ybar, H_eff theta> w.r.t. theta, L, R and (one-site) W.

    Returns a dict with the requested entries ("theta", "L", "R", "W").
    """
    nsite = theta.dim() - 2
    dt = theta.dtype
    wl, chil = L.shape[0], L.shape[1]
    wr, chir = R.shape[0], R.shape[1]
    d = theta.shape[1] if nsite >= 1 else 1
    wm = W1.shape[1] if nsite == 2 else wl
    out = {}
    if "theta" in need:
        out["theta"] = torch.empty_like(theta)
    if "L" in need:
        out["L"] = torch.empty_like(L)
    if "R" in need:
        out["R"] = torch.empty_like(R)
    if "W" in need and nsite == 1:
        out["W"] = torch.empty_like(W1)
    ptr = lambda t: _dev(t, dt) if t is not None else C.c_void_p()
    rc = _lib.load().apply_heff_adjoint(
        ctx.handle, nsite, _dtype_code(theta), chil, chir, d, wl, wm, wr, ptr(L), ptr(W1), ptr(W2), ptr(R),
        ptr(theta), ptr(ybar), ptr(out.get("theta")), ptr(out.get("L")), ptr(out.get("W")), C.c_void_p(),
        ptr(out.get("R")))
    _check(ctx.handle, rc)
    return out


def env_update(ctx: Context, direction: int, env, A, W, out=None) -> torch.Tensor:
    """Left (direction=+1) or right (-1) environment update with site tensor A [chil][d][chir]."""
    dt = A.dtype
    chil, d, chir = A.shape
    wl, wr = W.shape[0], W.shape[1]
    if out is None:
        shape = (wr, chir, chir) if direction == 1 else (wl, chil, chil)
        out = torch.empty(shape, dtype=dt, device=A.device)
    rc = _lib.load().env_update(ctx.handle, direction, _dtype_code(A), chil, chir, d, wl, wr,
                                _dev(env, dt), _dev(A, dt), _dev(W, dt), _dev(out, dt))
    _check(ctx.handle, rc)
    return out


def _labels(q, n, what):
    a = np.ascontiguousarray(q, dtype=np.int32)
    if a.shape != (n,):
        raise ValueError(f"{what}: expected {n} charge labels")
    return a


def apply_heff_u1(ctx: Context, L, R, theta, W1=None, W2=None, *, q_left, q_right, q_phys, c_left, c_right,
                  out=None) -> torch.Tensor:
    """U(1) block-sparse H_eff theta (tensors as for apply_heff; integer charge
    labels of the bond, physical and outer MPO indices, bond labels sorted)."""
    nsite = theta.dim() - 2
    dt = theta.dtype
    wl, chil = L.shape[0], L.shape[1]
    wr, chir = R.shape[0], R.shape[1]
    d = theta.shape[1] if nsite >= 1 else 1
    wm = W1.shape[1] if nsite == 2 else wl
    if out is None:
        out = torch.empty_like(theta)
    keep = [_labels(q_left, chil, "q_left"), _labels(q_right, chir, "q_right"),
            _labels(q_phys if nsite else [0], d, "q_phys"), _labels(c_left, wl, "c_left"),
            _labels(c_right, wr, "c_right")]
    ptr = lambda t: _dev(t, dt) if t is not None else C.c_void_p()
    rc = _lib.load().apply_heff_u1(ctx.handle, nsite, _dtype_code(theta), chil, chir, d, wl, wm, wr,
                                   *[_iptr(k) for k in keep], ptr(L), ptr(W1), ptr(W2), ptr(R), ptr(theta), ptr(out))
    _check(ctx.handle, rc)
    return out


def env_update_u1(ctx: Context, direction: int, env, A, W, *, q_left, q_right, q_phys, c_left, c_right,
                  out=None) -> torch.Tensor:
    """U(1) block-sparse environment update (as env_update, with charge labels)."""
    dt = A.dtype
    chil, d, chir = A.shape
    wl, wr = W.shape[0], W.shape[1]
    if out is None:
        shape = (wr, chir, chir) if direction == 1 else (wl, chil, chil)
        out = torch.empty(shape, dtype=dt, device=A.device)
    keep = [_labels(q_left, chil, "q_left"), _labels(q_right, chir, "q_right"), _labels(q_phys, d, "q_phys"),
            _labels(c_left, wl, "c_left"), _labels(c_right, wr, "c_right")]
    rc = _lib.load().env_update_u1(ctx.handle, direction, _dtype_code(A), chil, chir, d, wl, wr,
                                   *[_iptr(k) for k in keep], _dev(env, dt), _dev(A, dt), _dev(W, dt), _dev(out, dt))
    _check(ctx.handle, rc)
    return out


def env_update_adjoint(ctx: Context, direction: int, env, A, W, out_bar, need=("env", "A", "W")) -> dict:
    """Gradients of Re<out_bar, env_update(direction, env, A, W)> with respect to
    env, A and W (the requested entries of "env", "A", "W")."""
    dt = A.dtype
    out = {}
    if "env" in need:
        out["env"] = torch.empty_like(env)
    if "A" in need:
        out["A"] = torch.empty_like(A)
    if "W" in need:
        out["W"] = torch.empty_like(W)
    chil, d, chir = A.shape
    wl, wr = W.shape[0], W.shape[1]
    ptr = lambda t: _dev(t, dt) if t is not None else C.c_void_p()
    rc = _lib.load().env_update_adjoint(ctx.handle, direction, _dtype_code(A), chil, chir, d, wl, wr, ptr(env),
                                        ptr(A), ptr(W), ptr(out_bar), ptr(out.get("env")), ptr(out.get("A")),
                                        ptr(out.get("W")))
    _check(ctx.handle, rc)
    return out


class MPO:
    """Long-range Hamiltonian MPO held by the library (Sec. II C)."""

    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle
        ctx._adopt(self)
        lib = _lib.load()
        N, d = C.c_int(), C.c_int()
        _check(ctx.handle, lib.mpo_get_info(handle, C.byref(N), C.byref(d), None))
        self.N, self.d = N.value, d.value
        w = np.zeros(self.N + 1, dtype=np.int32)
        _check(ctx.handle, lib.mpo_get_info(handle, None, None, _iptr(w)))
        self.w = [int(x) for x in w]

    @classmethod
    def longrange(cls, ctx: Context, N: int, pairs, *, c=None, lam=None, coupling=None,
                  onsite=None, h: float = 0.0, alpha=None, K: int = 0, fit_rmax: int = 0,
                  fit_refine: bool = False):
        """sum_{i<j} f(j-i) sum_a g_a A_a(i) B_a(j) + h sum X(i).

        pairs: list of (g_a, A_a, B_a).  Either (c, lam) for f(r) = Re sum
        c_k lam_k^r, or (alpha, K) for f(r) = r^-alpha fitted by the library
        with K exponentials on r = 1..fit_rmax (0: N-1; the maximum fit error
        is kept as ``fit_max_abs_err``), or coupling = [f(1), ..., f(N-1)] for
        the exact MPO.
        """
        d = np.asarray(pairs[0][1]).shape[0] if pairs else np.asarray(onsite).shape[0]
        g = np.array([p[0] for p in pairs], dtype=np.float64)
        Aops = _c128(np.array([p[1] for p in pairs]).reshape(-1, d, d)) if pairs else np.zeros(2)
        Bops = _c128(np.array([p[2] for p in pairs]).reshape(-1, d, d)) if pairs else np.zeros(2)
        spec = MpoSpec()
        spec.N, spec.d, spec.n_terms = N, d, len(pairs)
        spec.g, spec.A_ops, spec.B_ops = _dptr(g), _dptr(Aops), _dptr(Bops)
        keep = [g, Aops, Bops]
        if c is not None:
            cc, ll = _c128(c), _c128(lam)
            keep += [cc, ll]
            spec.K, spec.c, spec.lam = len(np.atleast_1d(c)), _dptr(cc), _dptr(ll)
        elif alpha is not None:
            spec.K, spec.alpha, spec.fit_rmax, spec.fit_refine = int(K), float(alpha), int(fit_rmax), int(fit_refine)
        else:
            cp = np.ascontiguousarray(coupling, dtype=np.float64)
            keep.append(cp)
            spec.K, spec.coupling = 0, _dptr(cp)
        if onsite is not None:
            on = _c128(onsite)
            keep.append(on)
            spec.onsite, spec.h = _dptr(on), float(h)
        h_ = C.c_void_p()
        err = C.c_double(0.0)
        _check(ctx.handle, _lib.load().mpo_longrange(ctx.handle, C.byref(spec), C.byref(h_), C.byref(err)))
        mpo = cls(ctx, h_)
        mpo.fit_max_abs_err = err.value
        return mpo

    @classmethod
    def from_tensors(cls, ctx: Context, Ws):
        N = len(Ws)
        d = Ws[0].shape[2]
        w = np.array([1] + [W.shape[1] for W in Ws], dtype=np.int32)
        flat = np.concatenate([_c128(W).reshape(-1) for W in Ws])
        h_ = C.c_void_p()
        _check(ctx.handle, _lib.load().mpo_from_tensors(ctx.handle, N, d, _iptr(w), _dptr(flat), C.byref(h_)))
        return cls(ctx, h_)

    def set_charges(self, charges):
        """U(1) charges of the bond indices: a list of N+1 integer lists
        (len w_j each, 0 on both boundary bonds); None clears them."""
        if charges is None:
            _check(self.ctx.handle, _lib.load().mpo_set_charges(self.handle, None))
            return
        assert [len(c) for c in charges] == self.w, "one charge per bond index"
        flat = np.ascontiguousarray(np.concatenate([np.asarray(c, dtype=np.int32) for c in charges]))
        _check(self.ctx.handle, _lib.load().mpo_set_charges(self.handle, _iptr(flat)))

    def tensor(self, site: int) -> np.ndarray:
        shape = (self.w[site], self.w[site + 1], self.d, self.d)
        out = np.zeros(shape, dtype=np.complex128)
        _check(self.ctx.handle, _lib.load().mpo_get_tensor(self.handle, site, _dptr(out.view(np.float64))))
        return out

    def close(self):
        if getattr(self, "handle", None):
            if self.ctx.handle:  # otherwise the context already released it
                _lib.load().mpo_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MPS:
    """MPS held by the library in right-canonical form, centre on site 1."""

    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle
        ctx._adopt(self)
        N, d = C.c_int(), C.c_int()
        _check(ctx.handle, _lib.load().mps_get_info(handle, C.byref(N), C.byref(d), None))
        self.N, self.d = N.value, d.value

    @classmethod
    def init(cls, ctx: Context, N: int, d: int, chi, basis_state=None, seed: int = 0):
        chi = np.ascontiguousarray(chi, dtype=np.int32)
        bs = None if basis_state is None else np.ascontiguousarray(basis_state, dtype=np.int32)
        h_ = C.c_void_p()
        rc = _lib.load().mps_init(ctx.handle, N, d, _iptr(chi), None if bs is None else _iptr(bs),
                                  C.c_uint64(seed), C.byref(h_))
        _check(ctx.handle, rc)
        return cls(ctx, h_)

    @classmethod
    def from_tensors(cls, ctx: Context, tensors):
        """MPS with the given host tensors [chi_l][d][chi_r] (taken as they are)."""
        N = len(tensors)
        d = tensors[0].shape[1]
        chi = [1] + [T.shape[2] for T in tensors]
        m = cls.init(ctx, N, d, [1] * (N + 1), basis_state=[0] * N)
        for j, T in enumerate(tensors):
            m.set_tensor(j, T)
        assert m.chi == chi
        return m

    @property
    def chi(self):
        c = np.zeros(self.N + 1, dtype=np.int32)
        _check(self.ctx.handle, _lib.load().mps_get_info(self.handle, None, None, _iptr(c)))
        return [int(x) for x in c]

    def set_charges(self, q_phys, labels):
        """U(1) labels: q_phys [d] and one non-decreasing integer list per
        bond (len chi_j each); (None, None) clears them."""
        if q_phys is None and labels is None:
            _check(self.ctx.handle, _lib.load().mps_set_charges(self.handle, None, None))
            return
        assert [len(q) for q in labels] == self.chi, "one label per bond index"
        qp = np.ascontiguousarray(q_phys, dtype=np.int32)
        flat = np.ascontiguousarray(np.concatenate([np.asarray(q, dtype=np.int32) for q in labels]))
        _check(self.ctx.handle, _lib.load().mps_set_charges(self.handle, _iptr(qp), _iptr(flat)))

    def charges(self):
        """(q_phys, [labels of bond j for j = 0..N]) as held by the library."""
        chi = self.chi
        qp = np.zeros(self.d, dtype=np.int32)
        flat = np.zeros(sum(chi), dtype=np.int32)
        _check(self.ctx.handle, _lib.load().mps_get_charges(self.handle, _iptr(qp), _iptr(flat)))
        out, o = [], 0
        for c in chi:
            out.append([int(x) for x in flat[o:o + c]])
            o += c
        return [int(x) for x in qp], out

    def tensor(self, site: int) -> np.ndarray:
        chi = self.chi
        out = np.zeros((chi[site], self.d, chi[site + 1]), dtype=np.complex128)
        _check(self.ctx.handle, _lib.load().mps_get_tensor(self.handle, site, _dptr(out.view(np.float64))))
        return out

    def tensors(self):
        return [self.tensor(j) for j in range(self.N)]

    def set_tensor(self, site: int, T):
        T = _c128(T)
        chil, _, chir = np.asarray(T).view(np.complex128).shape
        _check(self.ctx.handle, _lib.load().mps_set_tensor(self.handle, site, _dptr(T), chil, chir))

    def apply_site(self, site: int, op):
        """Site tensor <- op acting on its physical index (op [d][d]); a unitary op
        keeps the canonical form."""
        o = _c128(np.asarray(op, dtype=np.complex128))
        _check(self.ctx.handle, _lib.load().mps_apply_site(self.ctx.handle, self.handle, int(site), _dptr(o)))

    def copy(self) -> "MPS":
        """An independent MPS with the same tensors (through host memory)."""
        return MPS.from_tensors(self.ctx, self.tensors())

    def right_canonicalize(self):
        _check(self.ctx.handle, _lib.load().mps_right_canonicalize(self.ctx.handle, self.handle))

    def close(self):
        if getattr(self, "handle", None):
            if self.ctx.handle:
                _lib.load().mps_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class TDVPOptions:
    compute: str = "c128"       # "c64": FP32 MFMA contractions, FP64 Lanczos/QR/SVD
    krylov_max: int = 40
    krylov_tol: float = 1e-13
    chi_max: int = 1 << 30
    w_max: float = 0.0
    eps_rel: float = 0.0
    multiplet_guard: bool = True
    strict: bool = False
    gemm_form: int = 0
    svd_mode: int = 0           # 1 SVD, 2 density-matrix eigen-decomposition, 0 automatic
    imaginary: bool = False     # imaginary time: exp(-dt H), state renormalised after each step
    exp_method: str = "lanczos"  # local exponentials: "lanczos" or "taylor" (Al-Mohy-Higham)
    u1_block_min: int = 0       # U(1) mode: block kernels when chi_l * chi_r >= this (0: 256^2, 1: always)

    def to_c(self) -> Opts:
        o = Opts()
        o.compute = TDVP_C64 if self.compute == "c64" else TDVP_C128
        o.krylov_max = self.krylov_max
        o.krylov_tol = self.krylov_tol
        o.chi_max = self.chi_max
        o.w_max = self.w_max
        o.eps_rel = self.eps_rel
        o.multiplet_guard = int(self.multiplet_guard)
        o.strict = int(self.strict)
        o.gemm_form = self.gemm_form
        o.svd_mode = self.svd_mode
        o.imaginary = int(self.imaginary)
        if self.exp_method not in ("lanczos", "taylor"):
            raise ValueError(f"exp_method must be 'lanczos' or 'taylor', not {self.exp_method!r}")
        o.exp_method = 1 if self.exp_method == "taylor" else 0
        o.u1_block_min = self.u1_block_min
        return o


def tdvp1_step(ctx: Context, mps: MPS, mpo: MPO, dt: float, opts: TDVPOptions | None = None) -> dict:
    o = (opts or TDVPOptions()).to_c()
    st = Stats()
    _check(ctx.handle, _lib.load().tdvp1_step(ctx.handle, mps.handle, mpo.handle, float(dt), C.byref(o), C.byref(st)))
    return st.as_dict()


def tdvp2_step(ctx: Context, mps: MPS, mpo: MPO, dt: float, opts: TDVPOptions | None = None) -> dict:
    o = (opts or TDVPOptions()).to_c()
    st = Stats()
    _check(ctx.handle, _lib.load().tdvp2_step(ctx.handle, mps.handle, mpo.handle, float(dt), C.byref(o), C.byref(st)))
    return st.as_dict()


def dmrg2_sweep(ctx: Context, mps: MPS, mpo: MPO, opts: TDVPOptions | None = None) -> dict:
    """One two-site DMRG sweep towards the ground state; the statistics carry
    "energy", the variational energy after the sweep (the state is
    renormalised)."""
    o = (opts or TDVPOptions()).to_c()
    st = Stats()
    e = C.c_double(0.0)
    _check(ctx.handle, _lib.load().dmrg2_sweep(ctx.handle, mps.handle, mpo.handle, C.byref(o), C.byref(st),
                                               C.byref(e)))
    d = st.as_dict()
    d["energy"] = e.value
    return d


def tdvp_hybrid_step(ctx: Context, mps: MPS, mpo: MPO, dt: float, opts: TDVPOptions | None = None) -> dict:
    """Two-site step until chi_max is saturated on every bond, one-site step
    after that (the hybrid scheme of the paper's Discussion).  The returned
    statistics carry "one_site": True when the one-site step ran."""
    o = (opts or TDVPOptions()).to_c()
    st = Stats()
    one = C.c_int(0)
    _check(ctx.handle, _lib.load().tdvp_hybrid_step(ctx.handle, mps.handle, mpo.handle, float(dt), C.byref(o),
                                                    C.byref(st), C.byref(one)))
    d = st.as_dict()
    d["one_site"] = bool(one.value)
    return d


@dataclass
class SegmentOptions:
    compute: str = "c64"         # matvec / environment precision (fixed at construction)
    krylov_k: int = 8            # Lanczos steps per exponentiation
    chi_max: int = 1 << 30
    w_max: float = 0.0
    eps_rel: float = 0.0
    multiplet_guard: bool = True
    static_shapes: bool = True
    batched: bool = True
    use_graph: bool = False
    svd_mode: int = 0
    one_site: bool | str = False  # one-site sweeps with two-site boundary pairs; "auto": hybrid switch
    max_phases: int = 0          # > 0: stop after this many phases (inspection; leaves the state mid-step)

    def to_c(self) -> SegOpts:
        o = SegOpts()
        o.compute = TDVP_C64 if self.compute == "c64" else TDVP_C128
        o.krylov_k = self.krylov_k
        o.chi_max = self.chi_max
        o.w_max = self.w_max
        o.eps_rel = self.eps_rel
        o.multiplet_guard = int(self.multiplet_guard)
        o.static_shapes = int(self.static_shapes)
        o.batched = int(self.batched)
        o.use_graph = int(self.use_graph)
        o.svd_mode = self.svd_mode
        if self.one_site == "auto":
            o.one_site = 2
        elif isinstance(self.one_site, (bool, int)) and int(self.one_site) in (0, 1):
            o.one_site = int(self.one_site)
        else:
            raise ValueError(f"one_site must be a bool or 'auto', not {self.one_site!r}")
        o.max_phases = int(self.max_phases)
        return o


def segment_schedule(sizes, dt: float, first_half: bool, one_site: bool = False):
    """[(phase, kind, site, tau)] of one half step as the library runs it (kind 2 pair, 1 site;
    one-site schedule: 3 / 4 bond sweeping right / left)."""
    sz = np.ascontiguousarray(sizes, dtype=np.int32)
    n = C.c_int()
    lib = _lib.load()
    fn = lib.seg_schedule1 if one_site else lib.seg_schedule
    rc = fn(len(sz), _iptr(sz), float(dt), int(first_half), 0, None, None, None, None, C.byref(n))
    if rc != 0 and not (rc == 2 and n.value > 0):  # 2: the count exceeds max_ops = 0
        raise TDVPError(rc, "seg_schedule rejected the segment sizes")
    m = n.value
    ph, kd, st = (np.zeros(m, dtype=np.int32) for _ in range(3))
    tau = np.zeros(m)
    rc = fn(len(sz), _iptr(sz), float(dt), int(first_half), m, _iptr(ph), _iptr(kd), _iptr(st), _dptr(tau),
            C.byref(n))
    if rc != 0:
        raise TDVPError(rc, "seg_schedule failed")
    return [(int(a), int(b), int(c), float(t)) for a, b, c, t in zip(ph, kd, st, tau)]


class Segments:
    """Segment-parallel two-site TDVP state (inverse canonical gauge) held by the library."""

    def __init__(self, ctx: Context, handle, compute: str):
        self.ctx = ctx
        self.handle = handle
        self.compute = compute
        ctx._adopt(self)
        N, d = C.c_int(), C.c_int()
        _check(ctx.handle, _lib.load().seg_get_info(handle, C.byref(N), C.byref(d), None, None))
        self.N, self.d = N.value, d.value

    @classmethod
    def init(cls, ctx: Context, mpo: "MPO", tensors, sizes, compute: str = "c64"):
        """From host site tensors [chi_l][d][chi_r] (any gauge) and segment sizes."""
        N = len(tensors)
        d = tensors[0].shape[1]
        arrs = [np.ascontiguousarray(T, dtype=np.complex128) for T in tensors]
        chi = np.ascontiguousarray([1] + [A.shape[2] for A in arrs], dtype=np.int32)
        ptrs = (C.c_void_p * N)(*[A.ctypes.data for A in arrs])
        sz = np.ascontiguousarray(sizes, dtype=np.int32)
        h_ = C.c_void_p()
        rc = _lib.load().seg_init(ctx.handle, mpo.handle, N, d, _iptr(chi), ptrs, len(sz), _iptr(sz),
                                  TDVP_C64 if compute == "c64" else TDVP_C128, C.byref(h_))
        _check(ctx.handle, rc)
        return cls(ctx, h_, compute)

    def step(self, mpo: "MPO", dt: float, opts: SegmentOptions | None = None) -> dict:
        o = (opts or SegmentOptions(compute=self.compute)).to_c()
        st = Stats()
        _check(self.ctx.handle, _lib.load().seg_step(self.ctx.handle, self.handle, mpo.handle, float(dt),
                                                     C.byref(o), C.byref(st)))
        out = st.as_dict()
        out["one_site"] = bool(st.flags & 2)  # which schedule ran (the "auto" mode decides per step)
        return out

    @property
    def chi(self):
        c = np.zeros(self.N + 1, dtype=np.int32)
        _check(self.ctx.handle, _lib.load().seg_get_info(self.handle, None, None, _iptr(c), None))
        return [int(x) for x in c]

    @property
    def w_total(self) -> float:
        w = C.c_double()
        _check(self.ctx.handle, _lib.load().seg_get_info(self.handle, None, None, None, C.byref(w)))
        return w.value

    def psi(self, j: int) -> np.ndarray:
        chi = self.chi
        out = np.zeros((chi[j], self.d, chi[j + 1]), dtype=np.complex128)
        _check(self.ctx.handle, _lib.load().seg_get_psi(self.handle, j, _dptr(out.view(np.float64))))
        return out

    def bond(self, j: int) -> np.ndarray:
        """V_j = 1/Lambda_j of the bond after site j."""
        out = np.zeros(self.chi[j + 1], dtype=np.float64)
        _check(self.ctx.handle, _lib.load().seg_get_bond(self.handle, j, _dptr(out)))
        return out

    def norm2(self) -> float:
        """<psi|psi> of the state as it stands (drifts from 1 under the
        parallel updates)."""
        out = C.c_double()
        _check(self.ctx.handle, _lib.load().seg_norm2(self.ctx.handle, self.handle, C.byref(out)))
        return out.value

    def reorthonormalize(self, mpo: "MPO") -> None:
        """Back to the inverse canonical gauge of the normalised state, with
        every environment recomputed (a serial step)."""
        _check(self.ctx.handle, _lib.load().seg_reorthonormalize(self.ctx.handle, self.handle, mpo.handle))

    def tensors(self):
        """Ordinary MPS tensors of the state: Psi_0, V_0 Psi_1, V_1 Psi_2, ..."""
        out = [self.psi(0)]
        for j in range(1, self.N):
            out.append(self.bond(j - 1)[:, None, None] * self.psi(j))
        return out

    def close(self):
        if getattr(self, "handle", None):
            if self.ctx.handle:
                _lib.load().seg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def expect(ctx: Context, mps: MPS, sites, ops) -> np.ndarray:
    sites = np.ascontiguousarray(sites, dtype=np.int32)
    n = len(sites)
    ops = np.asarray(ops, dtype=np.complex128)
    if ops.ndim == 2:
        ops = np.broadcast_to(ops, (n,) + ops.shape)
    ops = _c128(ops)
    out = np.zeros(n, dtype=np.complex128)
    _check(ctx.handle, _lib.load().expect(ctx.handle, mps.handle, n, _iptr(sites), _dptr(ops),
                                          _dptr(out.view(np.float64))))
    return out


def transition_expect(ctx: Context, bra: MPS, ket: MPS, sites, ops) -> np.ndarray:
    """<bra|O_i|ket> for each site (not normalised)."""
    sites = np.ascontiguousarray(sites, dtype=np.int32)
    n = len(sites)
    ops = np.asarray(ops, dtype=np.complex128)
    if ops.ndim == 2:
        ops = np.broadcast_to(ops, (n,) + ops.shape)
    ops = _c128(ops)
    out = np.zeros(n, dtype=np.complex128)
    _check(ctx.handle, _lib.load().transition_expect(ctx.handle, bra.handle, ket.handle, n, _iptr(sites), _dptr(ops),
                                                     _dptr(out.view(np.float64))))
    return out


def expect2(ctx: Context, mps: MPS, i, j, Oi, Oj) -> np.ndarray:
    i = np.ascontiguousarray(np.atleast_1d(i), dtype=np.int32)
    j = np.ascontiguousarray(np.atleast_1d(j), dtype=np.int32)
    n = len(i)
    Oi = np.asarray(Oi, dtype=np.complex128)
    Oj = np.asarray(Oj, dtype=np.complex128)
    if Oi.ndim == 2:
        Oi = np.broadcast_to(Oi, (n,) + Oi.shape)
    if Oj.ndim == 2:
        Oj = np.broadcast_to(Oj, (n,) + Oj.shape)
    Oi, Oj = _c128(Oi), _c128(Oj)
    out = np.zeros(n, dtype=np.complex128)
    _check(ctx.handle, _lib.load().expect2(ctx.handle, mps.handle, n, _iptr(i), _iptr(j), _dptr(Oi),
                                           _dptr(Oj), _dptr(out.view(np.float64))))
    return out


def energy(ctx: Context, mps: MPS, mpo: MPO) -> complex:
    out = np.zeros(2)
    _check(ctx.handle, _lib.load().energy(ctx.handle, mps.handle, mpo.handle, _dptr(out)))
    return complex(out[0], out[1])


def norm2(ctx: Context, mps: MPS) -> float:
    out = np.zeros(1)
    _check(ctx.handle, _lib.load().norm2(ctx.handle, mps.handle, _dptr(out)))
    return float(out[0])


def overlap(ctx: Context, bra: MPS, ket: MPS) -> complex:
    out = np.zeros(2)
    _check(ctx.handle, _lib.load().overlap(ctx.handle, bra.handle, ket.handle, _dptr(out)))
    return complex(out[0], out[1])


def infidelity(ctx: Context, a: MPS, b: MPS) -> float:
    """1 - |<a|b>| / sqrt(<a|a><b|b>) (Sec. IV)."""
    return 1.0 - abs(overlap(ctx, a, b)) / np.sqrt(norm2(ctx, a) * norm2(ctx, b))
