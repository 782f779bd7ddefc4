"""FP64 CPU oracle for disconnected fermion loops (arXiv:1108.2473).

TEST INFRASTRUCTURE ONLY.  This package is the checker for the GPU library:
only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it.  It shares no code with the GPU path; both follow
the paper's definitions independently.

Canonical layouts (numpy complex128, C order):
  gauge field   U[4][V][3][3]      (direction mu = x,y,z,t; row, column)
  spinors       psi[nrhs][V][4][3] (spin, colour); a single spinor may be
                passed as [V][4][3]
with the lexicographic site index s = x + Lx*(y + Ly*(z + Lz*t)).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None
_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_long_p = ctypes.POINTER(ctypes.c_long)
_c_double_p = ctypes.POINTER(ctypes.c_double)


def _load():
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(_build.LIB):
        _build.build()
    lib = ctypes.CDLL(_build.LIB)
    i, d, l, u64 = ctypes.c_int, ctypes.c_double, ctypes.c_long, ctypes.c_uint64
    ip, dp, lp = _c_int_p, _c_double_p, _c_long_p
    lib.or_num_threads.restype = i
    lib.or_set_num_threads.argtypes = [i]
    lib.or_gamma.argtypes = [i, i, dp]
    lib.or_hop.argtypes = [ip, i, i, dp, dp, dp, i, i]
    lib.or_apply_D.argtypes = [ip, i, i, d, dp, dp, dp, i, i]
    lib.or_apply_Dhat.argtypes = [ip, i, i, d, dp, dp, dp, i]
    lib.or_solve.argtypes = [ip, i, i, d, dp, dp, dp, i, d, i, i, ip, dp]
    lib.or_solve.restype = i
    lib.or_loops_exact.argtypes = [ip, i, i, d, dp, ip, i, ip, i, d, i, dp, dp]
    lib.or_loops_exact.restype = i
    lib.or_loops_exact_sites.argtypes = [ip, i, i, d, dp, lp, l, ip, i, d, i, dp, dp]
    lib.or_loops_exact_sites.restype = i
    lib.or_splitmix64.argtypes = [u64, u64]
    lib.or_splitmix64.restype = u64
    lib.or_noise.argtypes = [i, u64, l, ip, dp]
    lib.or_loops_tsm.argtypes = [ip, i, i, d, dp, i, u64, l, i, i, d, d, i, i, i, ip, i, i, dp]
    lib.or_loops_tsm.restype = i
    lib.or_loops_stochastic.argtypes = [ip, i, i, d, dp, i, u64, l, i, i, i, i, ip, i, d, i, dp]
    lib.or_loops_stochastic.restype = i
    lib.or_loops_grad.argtypes = [ip, i, i, d, dp, ip, i, ip, i, dp, d, i, dp, dp]
    lib.or_loops_grad.restype = i
    _LIB = lib
    return lib


def _dims(dims):
    return (ctypes.c_int * 4)(*[int(v) for v in dims])


def _ptr(a):
    return a.ctypes.data_as(_c_double_p)


def _cplx(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _gauge(U, dims):
    """U as complex128 after checking that it holds 4 x V links (the C side
    trusts the sizes it is given)."""
    U = _cplx(U)
    if U.size != 4 * int(np.prod(dims)) * 9:
        raise ValueError(f"gauge field of {U.size} elements, expected 4*V*9 for dims {tuple(dims)}")
    return U


def _spinors(psi, dims, single=False):
    """psi as complex128 after checking that it holds whole spinor fields
    (exactly one with single=True)."""
    psi = _cplx(psi)
    n = int(np.prod(dims)) * 12
    if psi.size == 0 or psi.size % n or (single and psi.size != n):
        raise ValueError(f"spinor array of {psi.size} elements, expected {'' if single else 'a multiple of '}"
                         f"V*12 = {n} for dims {tuple(dims)}")
    return psi


def _ints(seq):
    seq = [int(v) for v in seq]
    return (ctypes.c_int * max(1, len(seq)))(*seq), len(seq)


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's later parallel regions in this thread (n >= 1)."""
    _load().or_set_num_threads(int(n))


def gamma(mask: int, basis: int = 0) -> np.ndarray:
    """Gamma = g1^b0 g2^b1 g3^b2 g4^b3 for a 4-bit mask (g5 = mask 15)."""
    out = np.zeros((4, 4), dtype=np.complex128)
    _load().or_gamma(basis, mask, _ptr(out))
    return out


def hop(U, psi, dims, bc_t, out_parity=-1, dagger=False, basis=0):
    """Hopping term sum_mu [(1-g_mu)U_mu(x)psi(x+mu) + (1+g_mu)U_mu(x-mu)^+psi(x-mu)]."""
    U = _gauge(U, dims)
    psi = _spinors(psi, dims, single=True)
    out = np.zeros_like(psi)
    _load().or_hop(_dims(dims), bc_t, basis, _ptr(U), _ptr(psi), _ptr(out), out_parity,
                   int(dagger))
    return out


def apply_D(U, psi, dims, bc_t, kappa, dagger=False, basis=0):
    """Wilson-Dirac operator D = 1 - kappa*Hop (or D^+) applied to psi."""
    U = _gauge(U, dims)
    psi = _spinors(psi, dims)
    V = int(np.prod(dims))
    nrhs = psi.size // (V * 12)
    out = np.zeros_like(psi)
    _load().or_apply_D(_dims(dims), bc_t, basis, kappa, _ptr(U), _ptr(psi), _ptr(out), nrhs,
                       int(dagger))
    return out


def apply_Dhat(U, psi_even, dims, bc_t, kappa, dagger=False, basis=0):
    """Schur operator 1 - kappa^2 H_eo H_oe on a full-lattice vector (odd part ignored)."""
    U = _gauge(U, dims)
    psi = _spinors(psi_even, dims, single=True)
    out = np.zeros_like(psi)
    _load().or_apply_Dhat(_dims(dims), bc_t, basis, kappa, _ptr(U), _ptr(psi), _ptr(out),
                          int(dagger))
    return out


def solve(U, b, dims, bc_t, kappa, tol=1e-13, max_iter=20000, method=0, basis=0):
    """Solve D x = b to relative full-operator residual tol.

    method 0: even-odd BiCGStab with CGNR fallback; 1: full BiCGStab;
    2: even-odd CGNR.  Returns (x, iters, resid, n_failed).
    """
    U = _gauge(U, dims)
    b = _spinors(b, dims)
    V = int(np.prod(dims))
    nrhs = b.size // (V * 12)
    x = np.zeros_like(b)
    iters = np.zeros(nrhs, dtype=np.int32)
    resid = np.zeros(nrhs, dtype=np.float64)
    fails = _load().or_solve(_dims(dims), bc_t, basis, kappa, _ptr(U), _ptr(b), _ptr(x), nrhs,
                             tol, max_iter, method, iters.ctypes.data_as(_c_int_p),
                             _ptr(resid))
    return x, iters, resid, fails


def loops_exact(U, dims, bc_t, kappa, t0, gammas, tol=1e-13, max_iter=20000, basis=0,
                want_S=False):
    """Exact loops L_Gamma(y) = Tr[Gamma G(y;y)] on whole timeslices.

    Returns L [ngamma][nt][Vs] (and S [nt][Vs][4][4] when want_S).
    """
    U = _gauge(U, dims)
    t_arr, nt = _ints(t0)
    g_arr, ng = _ints(gammas)
    Vs = int(dims[0] * dims[1] * dims[2])
    L = np.zeros((ng, nt, Vs), dtype=np.complex128)
    S = np.zeros((nt, Vs, 4, 4), dtype=np.complex128) if want_S else None
    fails = _load().or_loops_exact(_dims(dims), bc_t, basis, kappa, _ptr(U), t_arr, nt, g_arr,
                                   ng, tol, max_iter, _ptr(L),
                                   _ptr(S) if want_S else None)
    if fails:
        raise RuntimeError(f"oracle: {fails} exact-loop solves missed tol={tol}")
    return (L, S) if want_S else L


def loops_exact_sites(U, dims, bc_t, kappa, sites, gammas, tol=1e-13, max_iter=20000,
                      basis=0, want_S=False):
    """Exact loops at an explicit list of lexicographic sites: L [ngamma][nsites]."""
    U = _gauge(U, dims)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    g_arr, ng = _ints(gammas)
    L = np.zeros((ng, sites.size), dtype=np.complex128)
    S = np.zeros((sites.size, 4, 4), dtype=np.complex128) if want_S else None
    fails = _load().or_loops_exact_sites(_dims(dims), bc_t, basis, kappa, _ptr(U),
                                         sites.ctypes.data_as(_c_long_p), sites.size, g_arr,
                                         ng, tol, max_iter, _ptr(L),
                                         _ptr(S) if want_S else None)
    if fails:
        raise RuntimeError(f"oracle: {fails} exact-loop solves missed tol={tol}")
    return (L, S) if want_S else L


NOISE_Z4, NOISE_CZ2, NOISE_Z2 = 0, 1, 2
DIL_TIME, DIL_SPIN, DIL_COLOUR, DIL_EVENODD, DIL_CUBIC = 1, 2, 4, 8, 16


def splitmix64(seed: int, k: int) -> int:
    """k-th output (0-based) of SplitMix64 started from state `seed`."""
    return int(_load().or_splitmix64(seed & (2**64 - 1), k & (2**64 - 1)))


def noise(noise_type, seed, r, dims):
    """Noise vector xi_r [V][4][3] of the counter-based generator."""
    V = int(np.prod(dims))
    out = np.zeros((V, 4, 3), dtype=np.complex128)
    _load().or_noise(noise_type, seed & (2**64 - 1), r, _dims(dims), _ptr(out))
    return out


def loops_tsm(U, dims, bc_t, kappa, noise_type, seed, r0, n_lp, n_hp, tol_lp, tol_hp,
              dilution, t_begin, t_end, gammas, max_iter=20000, basis=0):
    """Truncated-solver-method estimate L [ngamma][t_end-t_begin][Vs]."""
    U = _gauge(U, dims)
    g_arr, ng = _ints(gammas)
    Vs = int(dims[0] * dims[1] * dims[2])
    L = np.zeros((ng, t_end - t_begin, Vs), dtype=np.complex128)
    fails = _load().or_loops_tsm(_dims(dims), bc_t, basis, kappa, _ptr(U), noise_type,
                                 seed & (2**64 - 1), r0, n_lp, n_hp, tol_lp, tol_hp, dilution,
                                 t_begin, t_end, g_arr, ng, max_iter, _ptr(L))
    if fails:
        raise RuntimeError(f"oracle: {fails} high-precision solves missed tol={tol_hp}")
    return L


def loops_stochastic(U, dims, bc_t, kappa, noise_type, seed, r0, n_noise, dilution, t_begin,
                     t_end, gammas, tol=1e-13, max_iter=20000, basis=0):
    """Plain diluted stochastic estimate, Eq. (loop stochastic): [ngamma][nt][Vs]."""
    return loops_tsm(U, dims, bc_t, kappa, noise_type, seed, r0, n_noise, 0, tol, tol,
                     dilution, t_begin, t_end, gammas, max_iter=max_iter, basis=basis)


def loops_grad(U, dims, bc_t, kappa, t0, gammas, w, tol=1e-13, max_iter=20000, basis=0):
    """Adjoint gradient of F = Re sum conj(w) L for exact timeslice loops.

    w: complex [ngamma][nt][Vs].  Returns (dU [4][V][3][3], dkappa) with
    dU = dF/dRe U + i dF/dIm U.
    """
    U = _gauge(U, dims)
    t_arr, nt = _ints(t0)
    g_arr, ng = _ints(gammas)
    w = _cplx(w)
    V = int(np.prod(dims))
    dU = np.zeros((4, V, 3, 3), dtype=np.complex128)
    dk = ctypes.c_double(0.0)
    fails = _load().or_loops_grad(_dims(dims), bc_t, basis, kappa, _ptr(U), t_arr, nt, g_arr,
                                  ng, _ptr(w), tol, max_iter, _ptr(dU), ctypes.byref(dk))
    if fails:
        raise RuntimeError(f"oracle: {fails} gradient solves missed tol={tol}")
    return dU, dk.value


# ---------------------------------------------------------------------------
# momentum-projected loops and the disconnected two-point function
# (Sec. III, Eq. all_dis_corr), written out from their definitions
# ---------------------------------------------------------------------------
def momentum_project(L, dims, mom):
    """Lp[g][k][t] = sum_x exp(+i p_k . x) L[g][t][x] over the spatial sites x
    of each timeslice, p_k = 2 pi (n_x/Lx, n_y/Ly, n_z/Lz) for the integer
    vectors n_k = mom[k]; x = (x, y, z) with x fastest in the spatial index
    xs = x + Lx*(y + Ly*z).  L: complex [ngamma][nt][Vs]."""
    L = np.asarray(L, dtype=np.complex128)
    Lx, Ly, Lz = dims[0], dims[1], dims[2]
    xs = np.arange(Lx * Ly * Lz)
    x, y, z = xs % Lx, (xs // Lx) % Ly, xs // (Lx * Ly)
    out = np.zeros((L.shape[0], len(mom), L.shape[1]), dtype=np.complex128)
    for k, (nx, ny, nz) in enumerate(mom):
        phase = np.exp(2j * np.pi * (nx * x / Lx + ny * y / Ly + nz * z / Lz))
        for g in range(L.shape[0]):
            for t in range(L.shape[1]):
                out[g, k, t] = np.sum(phase * L[g, t])
    return out


def disconnected_correlator(Lp1, Lp2, Vs, pairs):
    """D[j][k][t] = (1/Vs) (1/T) sum_{ti} Lp1[A_j][k][(ti + t) mod T] Lp2[B_j][k][ti]
    for pairs j = (A_j, B_j): Lp1 projected with +p_k, Lp2 with -p_k, both over
    all T timeslices (time translation average of Eq. all_dis_corr; with
    independent stochastic estimates in Lp1 and Lp2 the product is unbiased)."""
    Lp1 = np.asarray(Lp1, dtype=np.complex128)
    Lp2 = np.asarray(Lp2, dtype=np.complex128)
    T = Lp1.shape[2]
    D = np.zeros((len(pairs), Lp1.shape[1], T), dtype=np.complex128)
    for j, (A, B) in enumerate(pairs):
        for k in range(Lp1.shape[1]):
            for t in range(T):
                acc = 0j
                for ti in range(T):
                    acc += Lp1[A, k, (ti + t) % T] * Lp2[B, k, ti]
                D[j, k, t] = acc / (Vs * T)
    return D


# ---------------------------------------------------------------------------
# Gaussian smearing and the connected pseudoscalar two-point function
# (Sec. III: smeared quark fields, Eq. all_corr with Gamma_A = Gamma_B = g5)
# ---------------------------------------------------------------------------
def _site_coords(dims):
    V = int(np.prod(dims))
    s = np.arange(V)
    return s % dims[0], (s // dims[0]) % dims[1], (s // (dims[0] * dims[1])) % dims[2], s // (dims[0] * dims[1] * dims[2])


def _shift_index(dims, mu, step):
    """index of x + step * mu-hat (periodic) for every site x"""
    c = list(_site_coords(dims))
    c[mu] = (c[mu] + step) % dims[mu]
    return c[0] + dims[0] * (c[1] + dims[1] * (c[2] + dims[2] * c[3]))


def smear_step(U, psi, dims, alpha, norm=1.0):
    """One step psi <- (1 + alpha H) psi / norm with the spatial hopping
    H(x, y) = sum_{i=1..3} [U_i(x) delta_{x, y-i} + U_i(x-i)^+ delta_{x, y+i}],
    acting on colour (spin is a spectator) within each timeslice.
    psi: [nrhs][V][4][3]."""
    U = np.asarray(U, dtype=np.complex128)
    psi = np.asarray(psi, dtype=np.complex128)
    out = psi.copy()
    for i in range(3):
        fw = _shift_index(dims, i, +1)
        bw = _shift_index(dims, i, -1)
        # U_i(x) psi(x + i)
        out = out + alpha * np.einsum("vab,rvsb->rvsa", U[i], psi[:, fw])
        # U_i(x - i)^+ psi(x - i)
        out = out + alpha * np.einsum("vba,rvsb->rvsa", U[i][bw].conj(), psi[:, bw])
    return out / norm


def smear(U, psi, dims, alpha, n, norm=1.0):
    """F psi with F = ((1 + alpha H) / norm)^n (Gaussian smearing, Sec. III)."""
    for _ in range(n):
        psi = smear_step(U, psi, dims, alpha, norm)
    return psi


def su3_project(V):
    """The SU(3) matrix assigned to a nonsingular 3x3 complex V (last two axes):
    the unitary factor W of the polar decomposition V = W P (W = A B^+ from the
    singular value decomposition V = A S B^+), divided by a cube root of its
    determinant, det(W)^(1/3) = exp(i arg(det W) / 3) with arg in (-pi, pi]."""
    A, _, Bh = np.linalg.svd(V)
    W = A @ Bh
    ph = np.angle(np.linalg.det(W))
    return W * np.exp(-1j * ph / 3)[..., None, None]


def ape_smear(U, dims, alpha, n):
    """APE smearing of the spatial links (Sec. III: the links entering the
    smearing kernel H are APE smeared; the paper does not give its form or
    parameters), n steps of
        U'_i(x) = P_SU3[ U_i(x) + alpha sum_{j=1..3, j != i} ( U_j(x) U_i(x+j) U_j(x+i)^+
                                                          + U_j(x-j)^+ U_i(x-j) U_j(x-j+i) ) ]
    with P_SU3 of su3_project; the time links are returned unchanged."""
    U = np.array(U, dtype=np.complex128, copy=True)
    for _ in range(n):
        new = U.copy()
        for i in range(3):
            fi = _shift_index(dims, i, +1)
            acc = U[i].copy()
            for j in range(3):
                if j == i:
                    continue
                fj = _shift_index(dims, j, +1)
                bj = _shift_index(dims, j, -1)
                dag = lambda M: M.conj().transpose(0, 2, 1)
                up = U[j] @ U[i][fj] @ dag(U[j][fi])
                dn = dag(U[j][bj]) @ U[i][bj] @ U[j][fi[bj]]
                acc = acc + alpha * (up + dn)
            new[i] = su3_project(acc)
        U = new
    return U


def point_sources(dims, y0):
    """The 12 spin-colour point sources at lexicographic site y0: [12][V][4][3]."""
    V = int(np.prod(dims))
    b = np.zeros((12, V, 4, 3), dtype=np.complex128)
    for k in range(12):
        b[k, y0, k // 3, k % 3] = 1.0
    return b


def pion_correlator(U, dims, bc_t, kappa, y0, mom, alpha=0.0, n=0, norm=1.0, smear_source=False,
                    smear_sink=False, tol=1e-13, U_smear=None):
    """Connected pseudoscalar two-point function of Eq. (all_corr) with
    Gamma_A = Gamma_B = g5 and a point source at y0 (optionally smeared):
    by g5-hermiticity Tr[g5 G(x;y0) g5 G(y0;x)] = sum |G(x;y0)|^2, so
    C[k][t] = sum_x exp(+i p_k.(x - y0)) sum_{sources, components} |phi(x, t0 + t)|^2
    with phi = F_sink D^-1 F_source e_{y0} (F = identity when not smeared).
    The smearing kernel uses the links U_smear (e.g. APE smeared) when given,
    the Dirac operator always U."""
    Us = U if U_smear is None else U_smear
    b = point_sources(dims, y0)
    if smear_source:
        b = smear(Us, b, dims, alpha, n, norm)
    x, it, res, fails = solve(U, b, dims, bc_t, kappa, tol=tol)
    if fails:
        raise RuntimeError("oracle solve did not converge")
    if smear_sink:
        x = smear(Us, x, dims, alpha, n, norm)
    Vs = dims[0] * dims[1] * dims[2]
    T = dims[3]
    rho = np.sum(np.abs(x) ** 2, axis=(0, 2, 3)).reshape(T, Vs)  # [t][xs]
    t0 = y0 // Vs
    xs0 = y0 % Vs
    P = momentum_project(rho[None], dims, mom)[0]  # [k][t]
    x0 = (xs0 % dims[0], (xs0 // dims[0]) % dims[1], xs0 // (dims[0] * dims[1]))
    C = np.zeros((len(mom), T), dtype=np.complex128)
    for k, nv in enumerate(mom):
        ph = np.exp(-2j * np.pi * sum(nv[d] * x0[d] / dims[d] for d in range(3)))
        for t in range(T):
            C[k, t] = ph * P[k, (t0 + t) % T]
    return C


# ---------------------------------------------------------------------------
# the paper's comparison of stochastic methods with the exact loops (Sec. III,
# figures "compare dilution" and "truncated"), composed from the oracle's own
# loops, projection and correlator
# ---------------------------------------------------------------------------
def dilution_study(configs, dims, bc_t, kappa, n_noise, schemes, tsm, seed, tol_hp, tol_lp, tol_exact=1e-13,
                   tsm_dilution=0, with_exact=True):
    """D(t) at p = 0 for Gamma = g5 per configuration: exact (point sources on
    every site), plain stochastic with complex Z2 noise for each dilution mask
    in `schemes` (name -> mask) and N noise vectors (unbiased mean over pairs
    r != s of per-vector loops), and the truncated solver method for each
    (n_lp, n_hp) in `tsm` (two independent halves correlated with each other;
    half h starts at noise index h (n_lp + n_hp) / 2 of seed + 1), its noise
    diluted with the mask `tsm_dilution` (Sec. II: the TSM combines with
    dilution; 0 = undiluted).  with_exact=False skips the exact evaluation
    (out["exact"] is then None).
    Configuration c uses seed + 1000 c.  Returns dicts of [nconf][T] arrays."""
    T = dims[3]
    Vs = dims[0] * dims[1] * dims[2]
    zero = [(0, 0, 0)]
    out = {"exact": [], "stochastic": {}, "tsm": {}}
    for ci, U in enumerate(configs):
        cseed = seed + 1000 * ci
        if with_exact:
            Lx = loops_exact(U, dims, bc_t, kappa, list(range(T)), [15], tol=tol_exact)
            P = momentum_project(Lx, dims, zero)
            out["exact"].append(disconnected_correlator(P, P, Vs, [(0, 0)])[0, 0])
        for name, mask in schemes.items():
            per = [momentum_project(loops_stochastic(U, dims, bc_t, kappa, NOISE_CZ2, cseed, r, 1, mask, 0, T,
                                                     [15], tol=tol_hp), dims, zero)[0]
                   for r in range(max(n_noise))]
            for N in n_noise:
                acc = np.zeros(T, dtype=np.complex128)
                for r in range(N):
                    for s in range(N):
                        if r != s:
                            acc += disconnected_correlator(per[r][None], per[s][None], Vs, [(0, 0)])[0, 0]
                out["stochastic"].setdefault((name, N), []).append(acc / (N * (N - 1)))
        for (n_lp, n_hp) in tsm:
            halves = [momentum_project(loops_tsm(U, dims, bc_t, kappa, NOISE_CZ2, cseed + 1, h * (n_lp + n_hp) // 2,
                                                 n_lp // 2, n_hp // 2, tol_lp, tol_hp, tsm_dilution, 0, T, [15]), dims,
                                                 zero)
                      for h in range(2)]
            out["tsm"].setdefault((n_lp, n_hp), []).append(
                disconnected_correlator(halves[0], halves[1], Vs, [(0, 0)])[0, 0])
    out["exact"] = np.array(out["exact"]) if with_exact else None
    out["stochastic"] = {k: np.array(v) for k, v in out["stochastic"].items()}
    out["tsm"] = {k: np.array(v) for k, v in out["tsm"].items()}
    return out


# ---------------------------------------------------------------------------
# the paper's comparison per insertion (Sec. IV, figures "spin gammas" and
# "truncated gammas"; Sec. V, figure "compare_unity"): momentum-projected
# loops of each (Gamma, p) estimated stochastically against the exact ones
# ---------------------------------------------------------------------------
GAMMA_MOMENTA = ((1, (1, 0, 0)), (2, (0, 1, 0)), (4, (0, 0, 1)), (8, (1, 0, 0)), (0, (0, 0, 0)))


def loop_error_study(configs, dims, bc_t, kappa, n_noise, schemes, tsm, seed, tol_hp, tol_lp, tol_exact=1e-13,
                     pairs=GAMMA_MOMENTA, tsm_dilution=0, with_exact=True):
    """Lp_Gamma(p, t) = sum_x exp(i p.x) L_Gamma(x, t) on all timeslices for
    each (Gamma, p) in `pairs` (default: g1 at p = (1,0,0), g2 at (0,1,0), g3 at
    (0,0,1), g4 at (1,0,0), as in the paper's nucleon three-point ratios, and
    the scalar at p = 0), per configuration:
      exact              loops from point sources on every site,
      stochastic         for each dilution mask of `schemes` (name -> mask) and
                         each N of n_noise, the mean of the loops of the first N
                         complex Z2 noise vectors (Eq. loop stochastic),
      tsm                for each (n_lp, n_hp), the truncated-solver estimate
                         (LP solves truncated at tol_lp, HP at tol_hp) with
                         noise seed + 1, diluted with `tsm_dilution`.
    Configuration c uses noise seed + 1000 c.  Returns dicts of arrays
    [nconf][npairs][T] (exact None when with_exact is False)."""
    T = dims[3]
    gam = sorted({g for g, _ in pairs})
    moms = sorted({tuple(m) for _, m in pairs})
    gi = {g: k for k, g in enumerate(gam)}
    mi = {m: k for k, m in enumerate(moms)}

    def project(L):  # [ngam][T][Vs] -> [npairs][T]
        P = momentum_project(L, dims, moms)
        return np.array([P[gi[g], mi[tuple(m)]] for g, m in pairs])

    out = {"exact": [], "stochastic": {}, "tsm": {}}
    for ci, U in enumerate(configs):
        cseed = seed + 1000 * ci
        if with_exact:
            out["exact"].append(project(loops_exact(U, dims, bc_t, kappa, list(range(T)), gam, tol=tol_exact)))
        for name, mask in schemes.items():
            per = [project(loops_stochastic(U, dims, bc_t, kappa, NOISE_CZ2, cseed, r, 1, mask, 0, T, gam,
                                            tol=tol_hp)) for r in range(max(n_noise))]
            for N in n_noise:
                out["stochastic"].setdefault((name, N), []).append(np.mean(per[:N], axis=0))
        for (n_lp, n_hp) in tsm:
            out["tsm"].setdefault((n_lp, n_hp), []).append(
                project(loops_tsm(U, dims, bc_t, kappa, NOISE_CZ2, cseed + 1, 0, n_lp, n_hp, tol_lp, tol_hp,
                                  tsm_dilution, 0, T, gam)))
    out["exact"] = np.array(out["exact"]) if with_exact else None
    out["stochastic"] = {k: np.array(v) for k, v in out["stochastic"].items()}
    out["tsm"] = {k: np.array(v) for k, v in out["tsm"].items()}
    return out
