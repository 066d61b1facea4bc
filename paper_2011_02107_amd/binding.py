"""Thin ctypes binding over libdacp.so (the C ABI declared in include/dacp.h).

Argument marshalling only: every step of the path runs in the HIP library.
Device buffers are torch tensors on a ROCm device (their data pointers are
passed through); host outputs come back as numpy arrays.  The binding raises
if the compiled library is missing -- there is no fallback path.
"""
import ctypes
import os

import numpy as np

from .inputs import TERM_DTYPE

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdacp.so")

DACP_F64, DACP_F32 = 0, 1
STATUS = {
    0: "DACP_OK",
    -1: "DACP_E_INVALID",
    -2: "DACP_E_NOMEM",
    -3: "DACP_E_HIP",
    -4: "DACP_E_BOUNDS",
    -5: "DACP_E_WINDOW",
    -6: "DACP_E_NUMERIC",
    -7: "DACP_E_CONVERGENCE",
}


class DacpError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class FilterParams(ctypes.Structure):
    _fields_ = [
        ("e_bound", ctypes.c_double),
        ("a", ctypes.c_double),
        ("K", ctypes.c_int),
        ("b", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("fp64_tail", ctypes.c_int),
        ("seed", ctypes.c_uint64),
    ]


class BasisParams(ctypes.Structure):
    _fields_ = [
        ("e_bound", ctypes.c_double),
        ("a", ctypes.c_double),
        ("n", ctypes.c_int),
        ("b", ctypes.c_int),
        ("group", ctypes.c_int),
    ]


class Opts(ctypes.Structure):
    _fields_ = [
        ("b", ctypes.c_int),
        ("group", ctypes.c_int),
        ("kfac", ctypes.c_double),
        ("window_ratio", ctypes.c_double),
        ("basis_ratio", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("tol_rel", ctypes.c_double),
        ("lanczos_steps", ctypes.c_int),
        ("kpm_moments", ctypes.c_int),
        ("kpm_vectors", ctypes.c_int),
        ("e_bound", ctypes.c_double),
        ("a", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("fp64_tail_frac", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("max_retries", ctypes.c_int),
        ("moment_mode", ctypes.c_int),
        ("sectors", ctypes.c_int),
    ]


class Report(ctypes.Structure):
    _fields_ = [
        ("e_bound", ctypes.c_double),
        ("a", ctypes.c_double),
        ("a_r", ctypes.c_double),
        ("K", ctypes.c_int),
        ("n", ctypes.c_int),
        ("b", ctypes.c_int),
        ("m", ctypes.c_int),
        ("rank", ctypes.c_int),
        ("n_candidates", ctypes.c_int),
        ("n_accepted", ctypes.c_int),
        ("retries", ctypes.c_int),
        ("evol_steps", ctypes.c_int64),
        ("evol_launches", ctypes.c_int64),
        ("t_bound_ms", ctypes.c_double),
        ("t_filter_ms", ctypes.c_double),
        ("t_evol_ms", ctypes.c_double),
        ("t_project_ms", ctypes.c_double),
        ("t_gep_ms", ctypes.c_double),
        ("t_accept_ms", ctypes.c_double),
        ("t_total_ms", ctypes.c_double),
        ("evol_kernel_ms", ctypes.c_double),
        ("max_err_est", ctypes.c_double),
        ("evol_group", ctypes.c_int),
        ("n_ghost", ctypes.c_int),
        ("model_used", ctypes.c_int),
        ("model_fallback", ctypes.c_int),
        ("n_clusters_at_b", ctypes.c_int),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)

# name -> (restype, argtypes); mirrors include/dacp.h
SIGNATURES = {
    "dacp_create": (ctypes.c_int, [ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "dacp_destroy": (None, [_vp]),
    "dacp_last_error": (ctypes.c_char_p, [_vp]),
    "dacp_set_stream": (ctypes.c_int, [_vp, _vp]),
    "dacp_set_tile": (ctypes.c_int, [_vp, ctypes.c_int]),
    "dacp_tune": (ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_int]),
    "dacp_tune_get": (ctypes.c_int, [_vp, ctypes.c_char_p, _ip]),
    "dacp_version": (ctypes.c_char_p, []),
    "dacp_build_hamiltonian": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "dacp_free_hamiltonian": (None, [_vp]),
    "dacp_ham_info": (ctypes.c_int, [_vp, _ip, _dp, _dp, _ip]),
    "dacp_ham_flip_symmetry": (ctypes.c_int, [_vp, _ip]),
    "dacp_apply": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _i64, _vp, _i64]),
    "dacp_spectral_bound": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, ctypes.c_uint64, ctypes.c_double, _dp, _dp, _dp]),
    "dacp_dos_moments": (ctypes.c_int, [_vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_uint64, _dp]),
    "dacp_random_block": (ctypes.c_int, [_vp, _i64, ctypes.c_int, ctypes.c_uint64, _vp]),
    "dacp_filter": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(FilterParams), _vp, _vp]),
    "dacp_basis": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(BasisParams), _vp, _vp, _i64, _ip]),
    "dacp_project": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _i64, _vp, _vp, _i64]),
    "dacp_rayleigh_ritz": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _i64, ctypes.c_double, _dp, _vp, _ip]),
    "dacp_syev": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _i64, _dp, _vp]),
    "dacp_basis_moments": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(BasisParams), _vp, _vp, _vp, _i64, _ip]),
    "dacp_basis_stored_moments": (
        ctypes.c_int,
        [_vp, _vp, ctypes.POINTER(BasisParams), _vp, _vp, _i64, _vp, _vp, _i64, _ip],
    ),
    "dacp_syev_batched": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "dacp_syev_batched_noalloc": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "dacp_gemm": (
        ctypes.c_int,
        [_vp, ctypes.c_int, ctypes.c_int, _i64, _i64, _i64, ctypes.c_double, _vp, _i64, _vp, _i64, ctypes.c_double, _vp, _i64],
    ),
    "dacp_default_opts": (None, [ctypes.POINTER(Opts)]),
    "dacp_central_eigs": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.POINTER(Opts), _dp, _dp, _ip, ctypes.POINTER(Report)]),
    "dacp_central_eigpairs": (
        ctypes.c_int,
        [_vp, _vp, ctypes.c_int, ctypes.POINTER(Opts), _dp, _dp, _vp, _i64, _ip, ctypes.POINTER(Report)],
    ),
    "dacp_spacing_ratios": (ctypes.c_int, [_dp, ctypes.c_int, _dp, _dp]),
    "dacp_accept_rule": (
        ctypes.c_int,
        [ctypes.c_int, _dp, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, _ip, _ip, _dp, _ip],
    ),
    "dacp_plan": (
        ctypes.c_int,
        [_i64, ctypes.c_int, ctypes.c_double, _dp, ctypes.c_int, ctypes.POINTER(Opts), ctypes.c_int, _dp, _ip,
         ctypes.POINTER(_i64), ctypes.c_int],
    ),
    "dacp_autotune": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, _ip, _dp]),
    "dacp_mlp_create": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(_vp)]),
    "dacp_mlp_free": (None, [_vp]),
    "dacp_mlp_params": (ctypes.c_int, [_vp, _vp, _vp, _vp, _ip]),
    "dacp_mlp_loss_grad": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _dp, _dp, _dp, _dp]),
    "dacp_mlp_train": (
        ctypes.c_int,
        [_vp, _vp, ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_uint64, _dp],
    ),
    "dacp_mlp_predict": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _dp, _dp]),
    "dacp_window_features": (ctypes.c_int, [_vp, _dp]),
    "dacp_window_labels": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(Opts), _dp]),
    "dacp_central_eigs_learned": (
        ctypes.c_int,
        [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(Opts), _dp, _dp, _ip, ctypes.POINTER(Report)],
    ),
    "dacp_central_eigs_batched": (
        ctypes.c_int,
        [_vp, ctypes.c_int, ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(Opts), _dp, _dp, _ip, ctypes.POINTER(Report)],
    ),
    "dacp_autotune_batched": (
        ctypes.c_int,
        [_vp, ctypes.c_int, ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(Opts), ctypes.c_int, ctypes.POINTER(Opts),
         _dp],
    ),
    "dacp_central_eigs_batched_learned": (
        ctypes.c_int,
        [_vp, ctypes.c_int, ctypes.POINTER(_vp), _vp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(Opts), _dp, _dp, _ip,
         ctypes.POINTER(Report)],
    ),
}

_lib = None


def load_library():
    """Load libdacp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() (there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _f64(x):
    return x.ctypes.data_as(_dp)


class Context:
    """A library context bound to a device and a HIP stream (torch's current one by default)."""

    def __init__(self, device=0, stream=None):
        import torch

        self.lib = load_library()
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        h = _vp()
        st = self.lib.dacp_create(int(device), _vp(stream), ctypes.byref(h))
        if st != 0:
            raise DacpError(st, "dacp_create failed")
        self.handle = h
        self.device = device

    def check(self, st):
        if st != 0:
            raise DacpError(st, self.lib.dacp_last_error(self.handle).decode())

    def set_tile(self, tile_elems):
        self.check(self.lib.dacp_set_tile(self.handle, int(tile_elems)))

    def tune(self, key, value):
        self.check(self.lib.dacp_tune(self.handle, key.encode(), int(value)))

    def tune_get(self, key):
        v = ctypes.c_int()
        self.check(self.lib.dacp_tune_get(self.handle, key.encode(), ctypes.byref(v)))
        return v.value

    def close(self):
        if self.handle:
            self.lib.dacp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hamiltonian:
    def __init__(self, ctx, handle, L):
        self.ctx = ctx
        self.handle = handle
        self.L = L
        self.D = 1 << L

    def info(self):
        L = ctypes.c_int()
        sa = ctypes.c_double()
        sq = ctypes.c_double()
        nf = ctypes.c_int()
        self.ctx.check(self.ctx.lib.dacp_ham_info(self.handle, ctypes.byref(L), ctypes.byref(sa), ctypes.byref(sq), ctypes.byref(nf)))
        return {"L": L.value, "sum_abs": sa.value, "sum_sq": sq.value, "n_flip_groups": nf.value}

    def flip_symmetry(self):
        """True when H commutes with the global spin flip prod_i sigma^x_i."""
        f = ctypes.c_int()
        self.ctx.check(self.ctx.lib.dacp_ham_flip_symmetry(self.handle, ctypes.byref(f)))
        return bool(f.value)

    def close(self):
        if self.handle:
            self.ctx.lib.dacp_free_hamiltonian(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dacp_build_hamiltonian(ctx, L, terms):
    terms = np.ascontiguousarray(np.asarray(terms, dtype=TERM_DTYPE))
    h = _vp()
    ctx.check(ctx.lib.dacp_build_hamiltonian(ctx.handle, int(L), len(terms), terms.ctypes.data_as(_vp), ctypes.byref(h)))
    return Hamiltonian(ctx, h, L)


def dacp_apply(ctx, ham, x, y):
    import torch

    dtype = {torch.float64: DACP_F64, torch.float32: DACP_F32}[x.dtype]
    assert y.dtype == x.dtype and x.shape == y.shape and x.shape[0] == ham.D
    b = 1 if x.dim() == 1 else x.shape[1]
    ctx.check(ctx.lib.dacp_apply(ctx.handle, ham.handle, dtype, b, _ptr(x), b, _ptr(y), b))


def dacp_random_block(ctx, D, b, seed, out):
    ctx.check(ctx.lib.dacp_random_block(ctx.handle, int(D), int(b), int(seed), _ptr(out)))


def dacp_spectral_bound(ctx, ham, steps=80, v0=None, seed=0, safety=1.01):
    eb, lo, hi = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    ctx.check(
        ctx.lib.dacp_spectral_bound(
            ctx.handle, ham.handle, int(steps), _ptr(v0), int(seed), float(safety), ctypes.byref(eb), ctypes.byref(lo), ctypes.byref(hi)
        )
    )
    return eb.value, lo.value, hi.value


def dacp_dos_moments(ctx, ham, e_bound, n_moments, nvec=8, R=None, seed=0):
    mu = np.zeros(n_moments)
    ctx.check(ctx.lib.dacp_dos_moments(ctx.handle, ham.handle, float(e_bound), int(n_moments), int(nvec), _ptr(R), int(seed), _f64(mu)))
    return mu


def dacp_filter(ctx, ham, psi_out, e_bound, a, K, start=None, precision=DACP_F64, fp64_tail=0, seed=0):
    p = FilterParams(float(e_bound), float(a), int(K), int(psi_out.shape[1]), int(precision), int(fp64_tail), int(seed))
    ctx.check(ctx.lib.dacp_filter(ctx.handle, ham.handle, ctypes.byref(p), _ptr(start), _ptr(psi_out)))


def dacp_basis(ctx, ham, psi_e, V, e_bound, a, n, group=0):
    b = int(psi_e.shape[1])
    p = BasisParams(float(e_bound), float(a), int(n), b, int(group))
    m = ctypes.c_int()
    ctx.check(ctx.lib.dacp_basis(ctx.handle, ham.handle, ctypes.byref(p), _ptr(psi_e), _ptr(V), int(V.shape[1]), ctypes.byref(m)))
    return m.value


def dacp_basis_moments(ctx, ham, psi_e, S, P, e_bound, a, n, group=0):
    """Moment mode: S and P (device m x m tensors) of the uniform-grid Chebyshev basis from moments,
    without storing it; returns m = b (2n + 1)."""
    b = int(psi_e.shape[1])
    p = BasisParams(float(e_bound), float(a), int(n), b, int(group))
    m = ctypes.c_int()
    ctx.check(ctx.lib.dacp_basis_moments(ctx.handle, ham.handle, ctypes.byref(p), _ptr(psi_e), _ptr(S), _ptr(P),
                                         int(S.shape[1]), ctypes.byref(m)))
    return m.value


def dacp_basis_stored_moments(ctx, ham, psi_e, V, S, P, e_bound, a, n, group=0):
    """Uniform-grid basis stored in V (device D x ldv tensor) and S, P (device m x m tensors) from the
    moments of its anchor panels; returns m = b (2n + 1)."""
    b = int(psi_e.shape[1])
    p = BasisParams(float(e_bound), float(a), int(n), b, int(group))
    m = ctypes.c_int()
    ctx.check(ctx.lib.dacp_basis_stored_moments(ctx.handle, ham.handle, ctypes.byref(p), _ptr(psi_e), _ptr(V),
                                                int(V.shape[1]), _ptr(S), _ptr(P), int(S.shape[1]), ctypes.byref(m)))
    return m.value


def dacp_project(ctx, ham, V, S, P, m=None):
    m = int(V.shape[1]) if m is None else int(m)
    ctx.check(ctx.lib.dacp_project(ctx.handle, ham.handle, m, _ptr(V), int(V.shape[1]), _ptr(S), _ptr(P), int(S.shape[1])))


def dacp_rayleigh_ritz(ctx, S, P, eps=1e-12, B_out=None):
    m = int(S.shape[0])
    theta = np.zeros(m)
    r = ctypes.c_int()
    ctx.check(ctx.lib.dacp_rayleigh_ritz(ctx.handle, m, _ptr(S), _ptr(P), int(S.shape[1]), float(eps), _f64(theta), _ptr(B_out), ctypes.byref(r)))
    return theta[: r.value], r.value


def dacp_syev(ctx, A, Z=None):
    n = int(A.shape[0])
    w = np.zeros(n)
    ctx.check(ctx.lib.dacp_syev(ctx.handle, n, _ptr(A), int(A.shape[1]), _f64(w), _ptr(Z)))
    return w


def dacp_syev_batched(ctx, As, Zs=None, noalloc=False):
    """Eigen-decompositions of square device matrices `As` (destroyed) in one launch; returns the
    list of ascending eigenvalue arrays.  Zs: matching device matrices for the eigenvectors (rows).
    noalloc: call dacp_syev_batched_noalloc (fixed per-device workspace, no device allocation)."""
    count = len(As)
    ns = (ctypes.c_int * count)(*[int(a.shape[0]) for a in As])
    ws = [np.zeros(int(a.shape[0])) for a in As]
    a_ptrs = (_vp * count)(*[_ptr(a) for a in As])
    w_ptrs = (_vp * count)(*[w.ctypes.data_as(_vp) for w in ws])
    z_ptrs = (_vp * count)(*[(_ptr(z) if z is not None else None) for z in (Zs or [None] * count)])
    fn = ctx.lib.dacp_syev_batched_noalloc if noalloc else ctx.lib.dacp_syev_batched
    ctx.check(fn(ctx.handle, count, ns, a_ptrs, w_ptrs, z_ptrs))
    return ws


def dacp_gemm(ctx, transA, transB, A, B, C, alpha=1.0, beta=0.0):
    M, N = C.shape
    K = A.shape[0] if transA else A.shape[1]
    ctx.check(
        ctx.lib.dacp_gemm(
            ctx.handle, int(transA), int(transB), M, N, K, float(alpha), _ptr(A), A.shape[1], _ptr(B), B.shape[1], float(beta), _ptr(C), C.shape[1]
        )
    )


def default_opts(**overrides):
    o = Opts()
    load_library().dacp_default_opts(ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def dacp_central_eigs(ctx, ham, N, opts=None, raise_on_window=True):
    """Returns (eigs ascending, error estimates, report dict, status)."""
    if opts is None:
        opts = default_opts()
    eigs = np.zeros(N)
    errs = np.zeros(N)
    n_out = ctypes.c_int()
    rep = Report()
    st = ctx.lib.dacp_central_eigs(ctx.handle, ham.handle, int(N), ctypes.byref(opts), _f64(eigs), _f64(errs), ctypes.byref(n_out), ctypes.byref(rep))
    if st != 0 and (raise_on_window or st != -5):
        ctx.check(st)
    n = n_out.value if st == 0 else 0
    d = rep.as_dict()
    d["n_out"] = n_out.value  # on DACP_E_WINDOW: the number accepted
    return eigs[:n], errs[:n], d, st


def dacp_central_eigpairs(ctx, ham, N, vecs, opts=None, raise_on_window=True):
    """dacp_central_eigs that also writes the unit eigenvectors into the device tensor vecs
    (2^L x ldvec FP64, ldvec >= N; column i belongs to eigs[i]).  Returns as dacp_central_eigs."""
    if opts is None:
        opts = default_opts()
    if vecs.dim() != 2 or vecs.shape[0] != 1 << ham.L or vecs.shape[1] < N or str(vecs.dtype) != "torch.float64":
        raise ValueError("vecs must be a float64 2^L x ldvec tensor with ldvec >= N")
    eigs = np.zeros(N)
    errs = np.zeros(N)
    n_out = ctypes.c_int()
    rep = Report()
    st = ctx.lib.dacp_central_eigpairs(ctx.handle, ham.handle, int(N), ctypes.byref(opts), _f64(eigs), _f64(errs),
                                       _ptr(vecs), int(vecs.shape[1]), ctypes.byref(n_out), ctypes.byref(rep))
    if st != 0 and (raise_on_window or st != -5):
        ctx.check(st)
    n = n_out.value if st == 0 else 0
    return eigs[:n], errs[:n], rep.as_dict(), st


def dacp_plan(D, N, e_bound, mu=None, opts=None, attempt=0, max_samples=1 << 16):
    """Parameters of one attempt (host code): dict with n_w, a_r, a, K, b, n, m and the sampled
    orders k_samples (the first max_samples of them)."""
    if opts is None:
        opts = default_opts()
    m = np.ascontiguousarray(mu if mu is not None else np.zeros(0), dtype=np.float64)
    fout = np.zeros(3)
    iout = np.zeros(4, dtype=np.int32)
    ks = np.zeros(max_samples, dtype=np.int64)
    st = load_library().dacp_plan(int(D), int(N), float(e_bound), _f64(m) if len(m) else None, int(len(m)),
                                  ctypes.byref(opts), int(attempt), _f64(fout),
                                  iout.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                  ks.ctypes.data_as(ctypes.POINTER(_i64)), int(max_samples))
    if st != 0:
        raise ValueError(f"dacp_plan: invalid arguments (status {st})")
    n = int(iout[2])
    return {"n_w": fout[0], "a_r": fout[1], "a": fout[2], "K": int(iout[0]), "b": int(iout[1]), "n": n,
            "m": int(iout[3]), "k_samples": ks[:min(n, max_samples)].copy()}


def dacp_accept_rule(theta, rnorm, a, tol):
    """(core positions in the (|theta|, theta) order, estimates, ghost count); host code."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    rn = np.ascontiguousarray(rnorm, dtype=np.float64)
    core = ctypes.c_int()
    pos = np.zeros(max(len(rn), 1), dtype=np.int32)
    est = np.zeros(max(len(rn), 1))
    ng = ctypes.c_int()
    st = load_library().dacp_accept_rule(int(len(th)), _f64(th), int(len(rn)), _f64(rn), float(a), float(tol),
                                         ctypes.byref(core), pos.ctypes.data_as(_ip), _f64(est), ctypes.byref(ng))
    if st != 0:
        raise ValueError(f"dacp_accept_rule: invalid arguments (status {st})")
    return pos[:core.value].copy(), est[:len(rn)].copy(), ng.value


def dacp_spacing_ratios(eigs):
    """(gap ratios [n-2], their mean) of ascending levels; host code, no device needed."""
    e = np.ascontiguousarray(eigs, dtype=np.float64)
    r = np.zeros(max(len(e) - 2, 0))
    mean = ctypes.c_double()
    st = load_library().dacp_spacing_ratios(_f64(e), int(len(e)), _f64(r), ctypes.byref(mean))
    if st != 0:
        raise ValueError("dacp_spacing_ratios: need n >= 3 ascending levels")
    return r, mean.value


def dacp_central_eigs_batched(ctx, hams, N, opts=None, raise_on_window=True, model=None, bound_margin=0.05):
    """Returns (eigs [count, N], errs [count, N], n_out [count], list of report dicts, status).
    model: a trained Mlp -> dacp_central_eigs_batched_learned with that bound margin."""
    if opts is None:
        opts = default_opts()
    count = len(hams)
    eigs = np.zeros((count, N))
    errs = np.zeros((count, N))
    n_out = np.zeros(count, dtype=np.int32)
    reps = (Report * count)()
    handles = (_vp * count)(*[h.handle for h in hams])
    if model is not None:
        st = ctx.lib.dacp_central_eigs_batched_learned(
            ctx.handle, count, handles, model.handle, float(bound_margin), int(N), ctypes.byref(opts), _f64(eigs),
            _f64(errs), n_out.ctypes.data_as(_ip), reps)
    else:
        st = ctx.lib.dacp_central_eigs_batched(
            ctx.handle, count, handles, int(N), ctypes.byref(opts), _f64(eigs), _f64(errs),
            n_out.ctypes.data_as(_ip), reps)
    if st != 0 and (raise_on_window or st != -5):
        ctx.check(st)
    return eigs, errs, n_out, [r.as_dict() for r in reps], st


def dacp_autotune_batched(ctx, hams, N, opts=None, sample_every=8):
    """Fastest (window ratio, basis ratio, kfac) on a sample of the realisations (sample_every = 1:
    all of them), window retries as in opts included; returns (tuned Opts, sample time in s)."""
    if opts is None:
        opts = default_opts()
    count = len(hams)
    handles = (_vp * count)(*[h.handle for h in hams])
    best = Opts()
    t = ctypes.c_double()
    ctx.check(ctx.lib.dacp_autotune_batched(ctx.handle, count, handles, int(N), ctypes.byref(opts), int(sample_every),
                                            ctypes.byref(best), ctypes.byref(t)))
    return best, t.value


WINDOW_FEATURES = 8


class Mlp:
    """Owns a dacp_mlp handle (the learned window's network)."""

    def __init__(self, ctx, n_in=WINDOW_FEATURES, hidden=64, layers=3, n_out=2, seed=0):
        self.ctx = ctx
        h = _vp()
        ctx.check(ctx.lib.dacp_mlp_create(ctx.handle, int(n_in), int(hidden), int(layers), int(n_out), int(seed), ctypes.byref(h)))
        self.handle = h
        self.n_in, self.n_out = int(n_in), int(n_out)

    def close(self):
        if self.handle:
            self.ctx.lib.dacp_mlp_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dacp_mlp_params(ctx, mlp, set_to=None):
    """Returns the current parameters (float32); with set_to, loads those first."""
    n = ctypes.c_int()
    ctx.check(ctx.lib.dacp_mlp_params(ctx.handle, mlp.handle, None, None, ctypes.byref(n)))
    if set_to is not None:
        src = np.ascontiguousarray(set_to, dtype=np.float32)
        assert src.size == n.value
        ctx.check(ctx.lib.dacp_mlp_params(ctx.handle, mlp.handle, None, src.ctypes.data_as(_vp), None))
    out = np.zeros(n.value, dtype=np.float32)
    ctx.check(ctx.lib.dacp_mlp_params(ctx.handle, mlp.handle, out.ctypes.data_as(_vp), None, None))
    return out


def dacp_mlp_loss_grad(ctx, mlp, X, T):
    X = np.ascontiguousarray(X, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    n = ctypes.c_int()
    ctx.check(ctx.lib.dacp_mlp_params(ctx.handle, mlp.handle, None, None, ctypes.byref(n)))
    grad = np.zeros(n.value)
    loss = ctypes.c_double()
    ctx.check(ctx.lib.dacp_mlp_loss_grad(ctx.handle, mlp.handle, X.shape[0], _f64(X), _f64(T), ctypes.byref(loss), _f64(grad)))
    return loss.value, grad


def dacp_mlp_train(ctx, mlp, X, Y, epochs=200, batch=64, lr=1e-3, seed=0):
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    loss = ctypes.c_double()
    ctx.check(ctx.lib.dacp_mlp_train(ctx.handle, mlp.handle, X.shape[0], _f64(X), _f64(Y), int(epochs), int(batch),
                                     float(lr), int(seed), ctypes.byref(loss)))
    return loss.value


def dacp_mlp_predict(ctx, mlp, X):
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.zeros((X.shape[0], mlp.n_out))
    ctx.check(ctx.lib.dacp_mlp_predict(ctx.handle, mlp.handle, X.shape[0], _f64(X), _f64(Y)))
    return Y


def dacp_window_features(ctx, ham):
    f = np.zeros(WINDOW_FEATURES)
    ctx.check(ctx.lib.dacp_window_features(ham.handle, _f64(f)))
    return f


def dacp_window_labels(ctx, hams, opts=None):
    count = len(hams)
    out = np.zeros((count, 2))
    handles = (_vp * count)(*[h.handle for h in hams])
    ctx.check(ctx.lib.dacp_window_labels(ctx.handle, count, handles, ctypes.byref(opts) if opts is not None else None, _f64(out)))
    return out


def dacp_central_eigs_learned(ctx, ham, mlp, N, bound_margin=0.05, opts=None, raise_on_window=True):
    """Returns (eigs ascending, error estimates, report dict, status)."""
    if opts is None:
        opts = default_opts()
    eigs = np.zeros(N)
    errs = np.zeros(N)
    n_out = ctypes.c_int()
    rep = Report()
    st = ctx.lib.dacp_central_eigs_learned(ctx.handle, ham.handle, mlp.handle, float(bound_margin), int(N), ctypes.byref(opts),
                                           _f64(eigs), _f64(errs), ctypes.byref(n_out), ctypes.byref(rep))
    if st != 0 and (raise_on_window or st != -5):
        ctx.check(st)
    n = n_out.value if st == 0 else 0
    return eigs[:n], errs[:n], rep.as_dict(), st


def dacp_autotune(ctx, ham, b=64, steps=64):
    """Returns (best group width, microseconds per column and step); the context keeps the winner."""
    g = ctypes.c_int()
    us = ctypes.c_double()
    ctx.check(ctx.lib.dacp_autotune(ctx.handle, ham.handle, int(b), int(steps), ctypes.byref(g), ctypes.byref(us)))
    return g.value, us.value
