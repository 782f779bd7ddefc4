"""Python binding of the MI355X loop library (include/floop.h).

Disconnected fermion loops L(x) = Tr[Gamma G(x;x)] of arXiv:1108.2473
(Eq. (loop)), exact and stochastic, computed by hand-written HIP kernels
for gfx950.  This module only marshals arguments: every step of the
computation runs inside libfloop.so.  Arrays are numpy (host memory) or
torch CUDA tensors (device memory, used in place on torch's current stream).

Layouts (complex128):  U[4][V][3][3], spinors [nrhs][V][4][3],
loops [ngamma][nt][Vs].  Gamma insertions are 4-bit masks
(Gamma = g1^b0 g2^b1 g3^b2 g4^b3; 1 -> 0, g5 -> 15).
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FLOOP_LIB selects another build of the same library (e.g. a debug build)
LIB_PATH = os.environ.get("FLOOP_LIB") or os.path.join(_HERE, "_lib", "libfloop.so")

FL_HOST, FL_DEVICE = 0, 1
PREC_F64, PREC_F32, PREC_BF16, PREC_H16 = 0, 1, 2, 3
SOLVER_BICGSTAB, SOLVER_CGNR = 0, 1
NOISE_Z4, NOISE_CZ2, NOISE_Z2 = 0, 1, 2
DIL_TIME, DIL_SPIN, DIL_COLOUR, DIL_EVENODD, DIL_CUBIC = 1, 2, 4, 8, 16
# profiling slots: the first hop of an iteration; the hop with the fused
# epilogue ending it; the iteration's vector update (x and p)
PROF_DSLASH, PROF_DSLASH_END, PROF_BLAS_UPDATE = 0, 1, 2
GAMMA_1, GAMMA_5 = 0, 15
GAMMAS_PAPER = [0, 15, 1, 2, 4, 8]  # 1, g5, g1, g2, g3, g4

_STATUS = {0: "FL_OK", -1: "FL_ERR_ARG", -2: "FL_ERR_STATE", -3: "FL_ERR_DEVICE", -4: "FL_ERR_NOMEM",
           -5: "FL_ERR_NOCONV", -6: "FL_ERR_BREAKDOWN"}


class FloopError(RuntimeError):
    """A non-zero fl_status.  For FL_ERR_NOCONV and FL_ERR_BREAKDOWN of a call
    that returns arrays, `result` holds what the call returned (built from the
    best iterates); fl_last_stats names the solves (Lattice.last_stats)."""

    def __init__(self, status, msg, result=None):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status
        self.result = result


NOCONV, BREAKDOWN = -5, -6


class _SolverParams(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("inner_prec", ctypes.c_int), ("gauge_reals", ctypes.c_int), ("delta", ctypes.c_double),
                ("truncated", ctypes.c_int), ("batch", ctypes.c_int), ("max_outer", ctypes.c_int)]


class _SolverStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("updates", ctypes.c_int), ("converged", ctypes.c_int),
                ("true_resid", ctypes.c_double), ("seconds", ctypes.c_double)]


class _NoiseParams(ctypes.Structure):
    _fields_ = [("noise", ctypes.c_int), ("seed", ctypes.c_ulonglong), ("r0", ctypes.c_longlong),
                ("n_lp", ctypes.c_int), ("n_hp", ctypes.c_int), ("dilution", ctypes.c_int),
                ("t_begin", ctypes.c_int), ("t_end", ctypes.c_int)]


@dataclass
class SolverParams:
    """Solver parameters (see fl_solver_params in include/floop.h)."""
    solver: int = SOLVER_BICGSTAB
    tol: float = 1e-12
    max_iter: int = 20000
    inner_prec: int = PREC_F32
    gauge_reals: int = 12
    delta: float = 0.0  # 0: the library default (0.1; 0.3 for 16-bit storage)
    truncated: bool = False
    batch: int = 0
    max_outer: int = 0  # FP64 residual replacements per right-hand side (0: no limit)

    def c(self):
        return _SolverParams(self.solver, self.tol, self.max_iter, self.inner_prec, self.gauge_reals,
                             self.delta, int(self.truncated), self.batch, self.max_outer)


@dataclass
class NoiseParams:
    """Stochastic / truncated-solver estimator (see fl_noise_params)."""
    noise: int = NOISE_Z4
    seed: int = 0
    r0: int = 0
    n_lp: int = 1
    n_hp: int = 0
    dilution: int = DIL_TIME | DIL_SPIN | DIL_COLOUR
    t_begin: int = 0
    t_end: int = 1

    def c(self):
        return _NoiseParams(self.noise, self.seed & (2**64 - 1), self.r0, self.n_lp, self.n_hp,
                            self.dilution, self.t_begin, self.t_end)


_lib = None


def lib():
    """The loaded libfloop.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FloopError(-3, f"HIP library not built: {LIB_PATH} missing (run __graft_entry__.build())")
    # torch ships its own HIP runtime under the same soname; loading it first
    # makes libfloop bind to that copy, so torch tensors and the library share
    # one runtime (a second runtime in the process hides the GPU from torch)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_double)
    ll = ctypes.c_longlong
    L.fl_version.restype = ctypes.c_char_p
    L.fl_last_error.restype = ctypes.c_char_p
    L.fl_last_error.argtypes = [vp]
    L.fl_create.argtypes = [ctypes.POINTER(vp), i, ctypes.POINTER(i), i]
    L.fl_destroy.argtypes = [vp]
    L.fl_set_stream.argtypes = [vp, vp]
    L.fl_set_gauge.argtypes = [vp, vp, i]
    L.fl_set_kappa.argtypes = [vp, d]
    L.fl_apply_D.argtypes = [vp, vp, vp, i, i, i]
    L.fl_apply_D_noalloc.argtypes = [vp, vp, vp, i, i]
    L.fl_apply_schur.argtypes = [vp, vp, vp, i, i, ctypes.POINTER(_SolverParams), i]
    L.fl_solve.argtypes = [vp, vp, vp, i, ctypes.POINTER(_SolverParams), ctypes.POINTER(_SolverStats), i]
    L.fl_loops_exact.argtypes = [vp, ctypes.POINTER(i), i, ctypes.POINTER(i), i,
                                 ctypes.POINTER(_SolverParams), vp, vp, i]
    L.fl_loops_exact_sites.argtypes = [vp, ctypes.POINTER(ll), ll, ctypes.POINTER(i), i,
                                       ctypes.POINTER(_SolverParams), vp, vp, i]
    L.fl_loops_stochastic.argtypes = [vp, ctypes.POINTER(_NoiseParams), ctypes.POINTER(i), i,
                                      ctypes.POINTER(_SolverParams), ctypes.POINTER(_SolverParams), vp, i]
    L.fl_loops_stochastic_multi.argtypes = [ctypes.POINTER(vp), i, ctypes.POINTER(_NoiseParams),
                                            ctypes.POINTER(i), i, ctypes.POINTER(_SolverParams),
                                            ctypes.POINTER(_SolverParams), ctypes.POINTER(vp), i]
    L.fl_loops_grad.argtypes = [vp, ctypes.POINTER(i), i, ctypes.POINTER(i), i, vp,
                                ctypes.POINTER(_SolverParams), vp, dp, i]
    L.fl_profile_enable.argtypes = [vp, i, i]
    L.fl_profile_read.argtypes = [vp, i, dp, ctypes.POINTER(ll), dp]
    L.fl_bench_dslash.argtypes = [vp, i, i, i, i, i, i, i, i, dp, dp]
    L.fl_set_tile.argtypes = [vp, i, i, i, i, i]
    L.fl_autotune.argtypes = [vp, i, i, i, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i), dp]
    L.fl_momentum_project.argtypes = [vp, vp, i, i, ctypes.POINTER(i), i, vp, i]
    L.fl_smear.argtypes = [vp, vp, i, d, i, d, i]
    L.fl_ape_smear.argtypes = [vp, d, i, vp, i]
    L.fl_pion_corr.argtypes = [vp, ctypes.c_longlong, ctypes.POINTER(_SolverParams), d, i, d, i, i,
                               ctypes.POINTER(i), i, vp, i]
    L.fl_disconnected_corr.argtypes = [vp, vp, vp, i, i, ctypes.POINTER(i), i, vp, i]
    L.fl_solver_params_default.argtypes = [ctypes.POINTER(_SolverParams)]
    L.fl_last_stats.argtypes = [vp, ctypes.POINTER(_SolverStats), ll, ctypes.POINTER(ll)]
    for name in ("fl_create", "fl_destroy", "fl_set_stream", "fl_set_gauge", "fl_set_kappa", "fl_apply_D",
                 "fl_apply_schur", "fl_solve", "fl_loops_exact", "fl_loops_exact_sites", "fl_loops_stochastic",
                 "fl_loops_stochastic_multi", "fl_loops_grad", "fl_profile_enable", "fl_profile_read",
                 "fl_bench_dslash", "fl_set_tile", "fl_autotune", "fl_momentum_project", "fl_disconnected_corr", "fl_smear",
                 "fl_pion_corr", "fl_last_stats", "fl_apply_D_noalloc", "fl_ape_smear"):
        getattr(L, name).restype = i
    _lib = L
    return L


def version() -> str:
    return lib().fl_version().decode()


def _ints(seq):
    seq = [int(v) for v in seq]
    return (ctypes.c_int * max(1, len(seq)))(*seq), len(seq)


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _torch():
    import torch
    return torch


class _Arr:
    """Pointer and location of an input array (numpy host or torch device)."""

    def __init__(self, a, shape_tail=None):
        if _is_torch(a):
            torch = _torch()
            if not a.is_cuda:
                a = a.detach().numpy()
            else:
                if a.dtype != torch.complex128:
                    raise TypeError("device arrays must be torch.complex128")
                a = a.contiguous()
                self.obj, self.ptr, self.where, self.torch = a, a.data_ptr(), FL_DEVICE, True
                self.shape = tuple(a.shape)
                return
        a = np.ascontiguousarray(a, dtype=np.complex128)
        self.obj, self.ptr, self.where, self.torch = a, a.ctypes.data, FL_HOST, False
        self.shape = a.shape


def _empty_like_where(ref: _Arr, shape):
    if ref.torch:
        torch = _torch()
        t = torch.empty(shape, dtype=torch.complex128, device=ref.obj.device)
        return t, t.data_ptr()
    a = np.empty(shape, dtype=np.complex128)
    return a, a.ctypes.data


class Lattice:
    """One lattice on one GPU: context of the C library (fl_ctx)."""

    def __init__(self, dims, bc_t=-1, device=0):
        self.dims = tuple(int(v) for v in dims)
        self.V = int(np.prod(self.dims))
        self.Vs = self.dims[0] * self.dims[1] * self.dims[2]
        self.bc_t = bc_t
        h = ctypes.c_void_p()
        d = (ctypes.c_int * 4)(*self.dims)
        st = lib().fl_create(ctypes.byref(h), device, d, bc_t)
        if st != 0:
            raise FloopError(st, lib().fl_last_error(None).decode())
        self._h = h
        self.device = device
        self.kappa = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().fl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, result=None):
        if st != 0:
            raise FloopError(st, lib().fl_last_error(self._h).decode(),
                             result if st in (NOCONV, BREAKDOWN) else None)

    def _stream_for(self, arr: _Arr):
        if arr.torch:
            torch = _torch()
            s = torch.cuda.current_stream(arr.obj.device).cuda_stream
        else:
            s = None
        self._check(lib().fl_set_stream(self._h, s))

    def set_stream(self, stream_ptr):
        self._check(lib().fl_set_stream(self._h, stream_ptr))

    def set_gauge(self, U):
        a = _Arr(U)
        if a.shape != (4, self.V, 3, 3):
            raise ValueError(f"gauge field must have shape (4, {self.V}, 3, 3)")
        self._stream_for(a)
        self._check(lib().fl_set_gauge(self._h, ctypes.c_void_p(a.ptr), a.where))

    def set_kappa(self, kappa):
        self._check(lib().fl_set_kappa(self._h, float(kappa)))
        self.kappa = float(kappa)

    def _spinors(self, psi):
        a = _Arr(psi)
        if a.shape[-3:] != (self.V, 4, 3):
            raise ValueError(f"spinors must have shape (..., {self.V}, 4, 3)")
        nrhs = int(np.prod(a.shape[:-3])) if len(a.shape) > 3 else 1
        return a, nrhs

    def apply_D(self, psi, dagger=False):
        a, nrhs = self._spinors(psi)
        out, optr = _empty_like_where(a, a.shape)
        self._stream_for(a)
        self._check(lib().fl_apply_D(self._h, ctypes.c_void_p(a.ptr), ctypes.c_void_p(optr), nrhs,
                                     int(dagger), a.where))
        return out

    def apply_D_noalloc(self, psi, out, dagger=False):
        """out = D psi (fl_apply_D_noalloc) for torch complex128 CUDA tensors
        psi and out of shape (..., V, 4, 3): no device allocation inside the
        library; enqueued on torch's current stream, not synchronised."""
        a, nrhs = self._spinors(psi)
        o, n2 = self._spinors(out)
        if not (a.torch and o.torch) or a.shape != o.shape:
            raise ValueError("apply_D_noalloc takes two CUDA tensors of the same shape")
        if o.obj is not out:
            raise ValueError("out must be a contiguous complex128 tensor")
        self._stream_for(a)
        self._check(lib().fl_apply_D_noalloc(self._h, ctypes.c_void_p(a.ptr), ctypes.c_void_p(o.ptr), nrhs,
                                             int(dagger)))
        return out

    def apply_schur(self, psi, params: SolverParams = None, dagger=False):
        """Dhat = 1 - kappa^2 H_eo H_oe on the even sites of psi, computed in the
        iteration precision and link storage of params (odd sites of the result 0)."""
        params = params or SolverParams()
        a, nrhs = self._spinors(psi)
        out, optr = _empty_like_where(a, a.shape)
        self._stream_for(a)
        self._check(lib().fl_apply_schur(self._h, ctypes.c_void_p(a.ptr), ctypes.c_void_p(optr), nrhs,
                                         int(dagger), ctypes.byref(params.c()), a.where))
        return out

    def solve(self, b, params: SolverParams = None, check=True):
        """Solve D x = b; returns (x, stats) with stats a list of dicts."""
        params = params or SolverParams()
        a, nrhs = self._spinors(b)
        out, optr = _empty_like_where(a, a.shape)
        stats = (_SolverStats * max(1, nrhs))()
        self._stream_for(a)
        st = lib().fl_solve(self._h, ctypes.c_void_p(a.ptr), ctypes.c_void_p(optr), nrhs,
                            ctypes.byref(params.c()), stats, a.where)
        if check and st not in (0,):
            self._check(st)
        info = [dict(iters=s.iters, updates=s.updates, converged=bool(s.converged),
                     true_resid=s.true_resid, seconds=s.seconds) for s in stats[:nrhs]]
        return out, info

    def last_stats(self):
        """Per-solve statistics of the last solving call on this lattice
        (fl_last_stats): numpy arrays iters, updates, converged (bool),
        true_resid and seconds, one entry per right-hand side in the order of
        that call."""
        n = ctypes.c_longlong()
        self._check(lib().fl_last_stats(self._h, None, 0, ctypes.byref(n)))
        buf = (_SolverStats * max(1, n.value))()
        self._check(lib().fl_last_stats(self._h, buf, n.value, ctypes.byref(n)))
        rows = buf[:n.value]
        return dict(iters=np.array([r.iters for r in rows], dtype=np.int64),
                    updates=np.array([r.updates for r in rows], dtype=np.int64),
                    converged=np.array([bool(r.converged) for r in rows], dtype=bool),
                    true_resid=np.array([r.true_resid for r in rows], dtype=np.float64),
                    seconds=np.array([r.seconds for r in rows], dtype=np.float64))

    def _out(self, shape, device):
        if device:
            torch = _torch()
            t = torch.zeros(shape, dtype=torch.complex128, device=f"cuda:{self.device}")
            self.set_stream(torch.cuda.current_stream(t.device).cuda_stream)
            return t, t.data_ptr(), FL_DEVICE
        a = np.zeros(shape, dtype=np.complex128)
        return a, a.ctypes.data, FL_HOST

    def loops_exact(self, t0, gammas, params: SolverParams = None, want_S=False, device=False):
        """Exact loops, Eq. (loop), on whole timeslices: L [ngamma][nt][Vs] (and S)."""
        params = params or SolverParams()
        t_arr, nt = _ints(t0)
        g_arr, ng = _ints(gammas)
        L, lp, where = self._out((ng, nt, self.Vs), device)
        S, sp = (None, None)
        if want_S:
            S, sp, _ = self._out((nt, self.Vs, 4, 4), device)
        self._check(lib().fl_loops_exact(self._h, t_arr, nt, g_arr, ng, ctypes.byref(params.c()),
                                         ctypes.c_void_p(lp), ctypes.c_void_p(sp) if want_S else None, where),
                    (L, S) if want_S else L)
        return (L, S) if want_S else L

    def loops_exact_sites(self, sites, gammas, params: SolverParams = None, want_S=False, device=False):
        """Exact loops at explicit lexicographic sites: L [ngamma][nsites] (and S)."""
        params = params or SolverParams()
        sites = np.ascontiguousarray(sites, dtype=np.int64)
        g_arr, ng = _ints(gammas)
        L, lp, where = self._out((ng, sites.size), device)
        S, sp = (None, None)
        if want_S:
            S, sp, _ = self._out((sites.size, 4, 4), device)
        self._check(lib().fl_loops_exact_sites(
            self._h, sites.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), sites.size, g_arr, ng,
            ctypes.byref(params.c()), ctypes.c_void_p(lp), ctypes.c_void_p(sp) if want_S else None, where),
            (L, S) if want_S else L)
        return (L, S) if want_S else L

    def momentum_project(self, L, mom):
        """Lp[g][k][t] = sum_x exp(+i p_k.x) L[g][t][x] for integer momentum vectors
        mom[k] = (n_x, n_y, n_z), p = 2 pi n / L (Eq. all_dis_corr).  L: [ngamma][nt][Vs]
        (numpy or a torch complex128 cuda tensor; the result follows it)."""
        a = _Arr(L)
        ng, nt = a.shape[0], a.shape[1]
        if a.shape[2] != self.Vs:
            raise ValueError(f"loops must have {self.Vs} spatial sites")
        m = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
        out, optr = _empty_like_where(a, (ng, m.shape[0], nt))
        self._check(lib().fl_momentum_project(self._h, ctypes.c_void_p(a.ptr), ng, nt,
                                              m.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), m.shape[0],
                                              ctypes.c_void_p(optr), a.where))
        return out

    def ape_smear(self, alpha=0.5, n=20, want_links=True):
        """APE-smear the spatial links used by the Gaussian smearing kernel
        (fl_ape_smear; kept for smear and pion_corr, the Dirac operator keeps
        the unsmeared links; n = 0 returns to the unsmeared links).  Returns
        the smeared field U'[4][V][3][3] (numpy) when want_links."""
        out = np.empty((4, self.V, 3, 3), dtype=np.complex128) if want_links else None
        self._check(lib().fl_ape_smear(self._h, float(alpha), int(n),
                                       ctypes.c_void_p(out.ctypes.data) if want_links else None, FL_HOST))
        return out

    def smear(self, psi, alpha=4.0, n=50, norm=1.0):
        """F psi with F = ((1 + alpha H)/norm)^n (Gaussian smearing, Sec. III); psi [nrhs][V][4][3]
        (numpy: a smeared copy is returned; torch cuda: smeared in place and returned)."""
        a = _Arr(psi)
        if a.torch:
            self._check(lib().fl_smear(self._h, ctypes.c_void_p(a.ptr), a.shape[0], float(alpha), int(n),
                                       float(norm), a.where))
            return a.obj
        out = np.array(a.obj, copy=True)
        self._check(lib().fl_smear(self._h, ctypes.c_void_p(out.ctypes.data), out.shape[0], float(alpha), int(n),
                                   float(norm), FL_HOST))
        return out

    def pion_corr(self, y0, params: SolverParams = None, alpha=4.0, n=50, norm=1.0, smear_source=True,
                  smear_sink=True, mom=((0, 0, 0),)):
        """Connected pseudoscalar two-point function C[k][t] from a point source at site y0
        (Eq. all_corr, g5-hermiticity), smeared at source and/or sink, t from the source time."""
        params = params or SolverParams()
        m = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
        out = np.empty((m.shape[0], self.dims[3]), dtype=np.complex128)
        self._check(lib().fl_pion_corr(self._h, int(y0), ctypes.byref(params.c()), float(alpha), int(n),
                                       float(norm), int(bool(smear_source)), int(bool(smear_sink)),
                                       m.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), m.shape[0],
                                       ctypes.c_void_p(out.ctypes.data), FL_HOST))
        return out

    def disconnected_corr(self, Lp1, Lp2, pairs):
        """D[j][k][t] = (1/Vs)(1/T) sum_ti Lp1[A_j][k][ti+t] Lp2[B_j][k][ti] (Eq. all_dis_corr):
        Lp1 projected with +p, Lp2 with -p, both over all T timeslices."""
        a1, a2 = _Arr(Lp1), _Arr(Lp2)
        if a1.shape != a2.shape or a1.where != a2.where:
            raise ValueError("Lp1 and Lp2 must have the same shape and location")
        ng, nm, T = a1.shape
        pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        out, optr = _empty_like_where(a1, (pr.shape[0], nm, T))
        self._check(lib().fl_disconnected_corr(self._h, ctypes.c_void_p(a1.ptr), ctypes.c_void_p(a2.ptr), ng, nm,
                                               pr.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), pr.shape[0],
                                               ctypes.c_void_p(optr), a1.where))
        return out

    def loops_stochastic(self, noise: NoiseParams, gammas, lp: SolverParams = None,
                         hp: SolverParams = None, device=False):
        """Diluted stochastic / truncated-solver loops: L [ngamma][t_end-t_begin][Vs]."""
        return loops_stochastic_multi([self], [noise], gammas, lp, hp, device)[0]

    def loops_grad(self, t0, gammas, w, params: SolverParams = None):
        """Gradient of F = Re sum conj(w) L_exact w.r.t. the links and kappa.

        Returns (dU [4][V][3][3], dkappa) with dU = dF/dRe U + i dF/dIm U."""
        params = params or SolverParams()
        t_arr, nt = _ints(t0)
        g_arr, ng = _ints(gammas)
        a = _Arr(w)
        if a.shape != (ng, nt, self.Vs):
            raise ValueError(f"weights must have shape ({ng}, {nt}, {self.Vs})")
        dU, dptr = _empty_like_where(a, (4, self.V, 3, 3))
        dk = ctypes.c_double(0.0)
        self._stream_for(a)
        self._check(lib().fl_loops_grad(self._h, t_arr, nt, g_arr, ng, ctypes.c_void_p(a.ptr),
                                        ctypes.byref(params.c()), ctypes.c_void_p(dptr), ctypes.byref(dk),
                                        a.where), (dU, dk.value))
        return dU, dk.value

    def profile_enable(self, kernel=PROF_DSLASH, on=True):
        self._check(lib().fl_profile_enable(self._h, kernel, int(on)))

    def profile_read(self, kernel=PROF_DSLASH):
        ms, n, b = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
        self._check(lib().fl_profile_read(self._h, kernel, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)))
        return dict(ms=ms.value, launches=n.value, bytes=b.value)

    def bench_dslash(self, prec=PREC_F32, gauge_reals=12, nrhs=1, nrep=100, nsets=8, rt=0, group=0, lds=-1):
        ms, b = ctypes.c_double(), ctypes.c_double()
        self._check(lib().fl_bench_dslash(self._h, prec, gauge_reals, nrhs, nrep, nsets, rt, group, lds,
                                          ctypes.byref(ms), ctypes.byref(b)))
        return dict(ms=ms.value, bytes=b.value, gbs=b.value / ms.value / 1e6 if ms.value > 0 else 0.0)

    def set_tile(self, prec=PREC_F32, gauge_reals=12, rt=0, group=0, lds=-1):
        self._check(lib().fl_set_tile(self._h, prec, gauge_reals, rt, group, lds))

    def autotune(self, prec=PREC_F32, gauge_reals=12, nrhs=1, cache=None):
        """Time the hopping kernel over workgroup shapes and LDS modes and keep
        the fastest for this lattice (fl_autotune).  cache: path of a JSON file
        of earlier results keyed by device name, lattice extents, precision,
        link reals and right-hand sides; a hit applies the stored shape
        (fl_set_tile) without timing, a miss times and adds its result."""
        key = None
        if cache is not None:
            key = tune_key(_device_name(self.device), self.dims, prec, gauge_reals, nrhs, version())
            hit = tune_cache_load(cache).get(key)
            if hit is not None:
                self.set_tile(prec, gauge_reals, hit["rt"], hit["group"], hit["lds"])
                return dict(hit, cached=True)
        rt, g, ld, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        self._check(lib().fl_autotune(self._h, prec, gauge_reals, nrhs, ctypes.byref(rt), ctypes.byref(g),
                                      ctypes.byref(ld), ctypes.byref(ms)))
        res = dict(rt=rt.value, group=g.value, lds=ld.value, ms=ms.value)
        if cache is not None:
            tune_cache_store(cache, key, res)
        return dict(res, cached=False)


def _device_name(device):
    """Marketing name and architecture of a HIP device (torch's view of it)."""
    import torch
    p = torch.cuda.get_device_properties(device)
    return f"{p.name} {getattr(p, 'gcnArchName', '')}".strip()


def tune_key(device_name, dims, prec, gauge_reals, nrhs, lib_version):
    """Key of one autotuner result: the device, the lattice, the storage, the
    right-hand sides and the library version (which names the hash of the
    kernel sources, so a result timed on other kernels is not reused)."""
    return (f"{device_name}|{'x'.join(str(int(d)) for d in dims)}|prec{int(prec)}|r{int(gauge_reals)}"
            f"|nrhs{int(nrhs)}|{lib_version}")


def tune_cache_load(path):
    """Autotuner results stored at path ({} if the file does not exist)."""
    import json
    try:
        with open(path) as f:
            d = json.load(f)
    except FileNotFoundError:
        return {}
    if not isinstance(d, dict):
        raise ValueError(f"{path}: not an autotuner cache")
    return d


def tune_cache_store(path, key, result):
    """Add one result to the cache file (written to a temporary file and
    renamed, so a reader never sees a partial file)."""
    import json
    d = tune_cache_load(path)
    d[key] = {k: result[k] for k in ("rt", "group", "lds", "ms")}
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def loops_stochastic_multi(lattices, noises, gammas, lp: SolverParams = None, hp: SolverParams = None,
                           device=False):
    """Stochastic / truncated-solver loops for up to 4 lattices solved in one batch."""
    lp = lp or SolverParams()
    hp = hp or SolverParams()
    n = len(lattices)
    g_arr, ng = _ints(gammas)
    hs = (ctypes.c_void_p * n)(*[l._h.value for l in lattices])
    nps = (_NoiseParams * n)(*[q.c() for q in noises])
    outs, ptrs, where = [], [], FL_HOST
    for lat, q in zip(lattices, noises):
        o, p, where = lat._out((ng, q.t_end - q.t_begin, lat.Vs), device)
        outs.append(o)
        ptrs.append(p)
    parr = (ctypes.c_void_p * n)(*ptrs)
    st = lib().fl_loops_stochastic_multi(hs, n, nps, g_arr, ng, ctypes.byref(lp.c()), ctypes.byref(hp.c()),
                                         parr, where)
    if st != 0:
        # the thread's last error: also set by checks made before any context is used
        raise FloopError(st, lib().fl_last_error(None).decode(), outs if st in (NOCONV, BREAKDOWN) else None)
    return outs


def _loop_fn_class():
    import torch

    class LoopFn(torch.autograd.Function):
        """Exact loops L[ngamma][nt][Vs] = fl_loops_exact(kappa, U) as a differentiable
        function of kappa (0-dim float64 tensor) and the links U (complex128
        [4][V][3][3]); the backward pass is the adjoint gradient fl_loops_grad
        (gamma_5-hermiticity gives the adjoint solutions from the forward ones).
        PyTorch's complex convention is used throughout: the incoming gradient w
        of L defines dLoss = Re sum conj(w) dL, and U.grad = dLoss/dRe U + i dLoss/dIm U.
        """

        @staticmethod
        def forward(ctx, kappa, U, lattice, t0, gammas, params):
            lattice.set_gauge(U.detach())
            lattice.set_kappa(float(kappa.detach()))
            L = lattice.loops_exact(t0, gammas, params, device=U.is_cuda)
            if not U.is_cuda:
                L = torch.from_numpy(L)
            ctx.lattice, ctx.t0, ctx.gammas, ctx.params = lattice, list(t0), list(gammas), params
            ctx.save_for_backward(kappa, U)
            return L

        @staticmethod
        def backward(ctx, gL):
            kappa, U = ctx.saved_tensors
            lat = ctx.lattice
            lat.set_gauge(U.detach())
            lat.set_kappa(float(kappa))
            w = gL.detach().to(torch.complex128).contiguous()
            if not U.is_cuda:
                w = w.cpu().numpy()
            dU, dk = lat.loops_grad(ctx.t0, ctx.gammas, w, ctx.params)
            if not U.is_cuda:
                dU = torch.from_numpy(dU)
            gk = torch.tensor(dk, dtype=kappa.dtype, device=kappa.device)
            return gk, dU, None, None, None, None

    return LoopFn


def loops_exact_autograd(kappa, U, lattice, t0, gammas, params: SolverParams = None):
    """Differentiable exact loops (see LoopFn)."""
    return _loop_fn_class().apply(kappa, U, lattice, t0, gammas, params or SolverParams())


def stats_records(stats, **fields):
    """One dict per solve of a per-solve statistics result (Lattice.last_stats()):
    index, iterations, FP64 replacements, converged, |Dx-b|/|b| on the full
    operator and the batch's seconds, each with the given extra fields."""
    n = len(stats["iters"])
    return [dict(fields, solve=k, iters=int(stats["iters"][k]), updates=int(stats["updates"][k]),
                 converged=bool(stats["converged"][k]), true_resid=float(stats["true_resid"][k]),
                 seconds=float(stats["seconds"][k])) for k in range(n)]


def append_jsonl(path, records):
    """Append records (dicts) to path as JSON lines, one write per call."""
    import json
    txt = "".join(json.dumps(r, sort_keys=True) + "\n" for r in records)
    with open(path, "a") as f:
        f.write(txt)


def loop_key(U, kappa, gammas, params: SolverParams):
    """Identity of an exact-loop computation: SHA-256 (first 16 hex digits) of
    the links, kappa, the insertions and the solver parameters."""
    import hashlib
    h = hashlib.sha256()
    a = U.detach().cpu().numpy() if _is_torch(U) else np.asarray(U)
    h.update(np.ascontiguousarray(a, dtype=np.complex128).tobytes())
    h.update(repr((float(kappa), [int(g) for g in gammas],
                   (params.solver, params.tol, params.max_iter, params.inner_prec, params.gauge_reals,
                    params.delta, bool(params.truncated), params.max_outer))).encode())
    return h.hexdigest()[:16]


def loops_exact_checkpointed(lattice, t0s, gammas, params: SolverParams, directory, key, log=None):
    """Exact loops L[ngamma][nt][Vs] of several timeslices, one solving call
    per timeslice, each timeslice's result kept as <directory>/<key>_t<t>.npy
    (written to a temporary file and renamed).  A timeslice whose file exists
    is loaded instead of solved again, so an interrupted run resumes where it
    stopped; key names the computation (loop_key of the links, kappa, the
    insertions and the solver parameters)."""
    os.makedirs(directory, exist_ok=True)
    out = []
    for t in t0s:
        path = os.path.join(directory, f"{key}_t{int(t)}.npy")
        if os.path.exists(path):
            L = np.load(path)
            if log:
                log(f"timeslice {t}: loaded {path}")
        else:
            L = lattice.loops_exact([int(t)], gammas, params)
            if _is_torch(L):
                L = L.cpu().numpy()
            tmp = f"{path}.{os.getpid()}.tmp.npy"
            np.save(tmp, L)
            os.replace(tmp, path)
            if log:
                log(f"timeslice {t}: solved, saved {path}")
        out.append(L[:, 0])
    return np.stack(out, axis=1)
