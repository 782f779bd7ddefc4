"""Pins of the FP64 CPU oracle against facts fixed by the paper and by the
mathematics of the Wilson-Dirac operator (no GPU involved).

Each test states the fact it checks.  Together they are chosen so that a
plausible slip in the oracle (a dropped hop, a wrong projector sign, U in
place of U^+, a misplaced boundary sign, a transposed trace, a wrong noise
key) fails at least one of them.
"""
import numpy as np
import pytest

import oracle as O
import synth_inputs as S

GAMMAS = [0, 1, 2, 4, 8, 15]  # 1, g1, g2, g3, g4, g5


# ---------------------------------------------------------------------------
# independent helpers written from the mathematics, not from the oracle
# ---------------------------------------------------------------------------
def momenta(dims, bc_t):
    """Allowed momenta: p_k = 2 pi n / L_k; p_4 = (2n + (1-bc_t)/2) pi / L_t."""
    ps = [2 * np.pi * np.arange(L) / L for L in dims[:3]]
    Lt = dims[3]
    ps.append((2 * np.arange(Lt) + (1 - bc_t) / 2) * np.pi / Lt)
    return np.meshgrid(*ps, indexing="ij")


def free_AB(dims, kappa, bc_t, theta=(0.0, 0.0, 0.0, 0.0)):
    """Momentum-space Wilson operator A + i g.B for U = 1 (shifted by theta)."""
    P = momenta(dims, bc_t)
    P = [P[mu] + theta[mu] for mu in range(4)]
    A = 1 - 2 * kappa * sum(np.cos(p) for p in P)
    B = [2 * kappa * np.sin(p) for p in P]
    return A, B


def gamma_np(basis=0):
    """Dirac matrices written out independently (chiral or Dirac-Pauli)."""
    s = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]),
         np.array([[1, 0], [0, -1]], complex)]
    Z = np.zeros((2, 2))
    g = [np.block([[Z, -1j * sk], [1j * sk, Z]]) for sk in s]
    if basis == 0:
        g.append(np.block([[Z, np.eye(2)], [np.eye(2), Z]]).astype(complex))
    else:
        g.append(np.block([[np.eye(2), Z], [Z, -np.eye(2)]]).astype(complex))
    return g


def shift_index(dims, mu, step):
    """Lexicographic index of x + step*mu for every x, and the boundary hop flag."""
    V = S.volume(dims)
    s = np.arange(V)
    c = [(s // int(np.prod(dims[:m]))) % dims[m] for m in range(4)]
    cm = c[mu] + step
    crossed = (cm < 0) | (cm >= dims[mu])
    cm = cm % dims[mu]
    c2 = list(c)
    c2[mu] = cm
    idx = c2[0] + dims[0] * (c2[1] + dims[1] * (c2[2] + dims[2] * c2[3]))
    return idx, crossed


def dense_D(U, dims, kappa, bc_t):
    """Dense D (12V x 12V) assembled from oracle columns."""
    V = S.volume(dims)
    N = 12 * V
    E = np.eye(N, dtype=np.complex128).reshape(N, V, 4, 3)
    cols = O.apply_D(U, E, dims, bc_t, kappa)
    return cols.reshape(N, N).T


def loops_from_G(G, dims, sites, gammas, basis=0):
    """L_Gamma(y) = sum_{ab} Gamma_{b a} S_{a b}, S_{ab} = sum_c G[(y,a,c),(y,b,c)]."""
    out = np.zeros((len(gammas), len(sites)), complex)
    for j, y in enumerate(sites):
        blk = G[12 * y:12 * y + 12, 12 * y:12 * y + 12].reshape(4, 3, 4, 3)
        Sy = np.einsum("acbc->ab", blk)
        for k, gm in enumerate(gammas):
            out[k, j] = np.sum(O.gamma(gm, basis).T * Sy)
    return out


def timeslice_sites(dims, t):
    Vs = dims[0] * dims[1] * dims[2]
    return [ys + Vs * t for ys in range(Vs)]


def gauge_transform(U, Om, dims):
    """U'_mu(x) = Om(x) U_mu(x) Om(x+mu)^+."""
    Up = np.empty_like(U)
    for mu in range(4):
        fwd, _ = shift_index(dims, mu, +1)
        Up[mu] = Om @ U[mu] @ Om[fwd].conj().transpose(0, 2, 1)
    return Up


def plaquette_sum(U, dims, site):
    """sum over the 24 plaquettes containing `site` of Re Tr U_P."""
    fw = [shift_index(dims, mu, +1)[0] for mu in range(4)]
    bw = [shift_index(dims, mu, -1)[0] for mu in range(4)]
    tot = 0.0
    V = S.volume(dims)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            # the four plaquettes in plane (mu,nu) with a corner at `site`
            for x in (site, bw[mu][site], bw[nu][site], bw[nu][bw[mu][site]]):
                P = U[mu][x] @ U[nu][fw[mu][x]] @ U[mu][fw[nu][x]].conj().T @ U[nu][x].conj().T
                tot += np.trace(P).real
    assert V > 0
    return tot


# ---------------------------------------------------------------------------
# Dirac matrices and noise generator
# ---------------------------------------------------------------------------
def test_gamma_algebra_and_mask_encoding():
    """Hermitian, Clifford algebra, g5 = g1 g2 g3 g4 = diag(1,1,-1,-1) in the chiral basis."""
    for basis in (0, 1):
        g = [O.gamma(1 << m, basis) for m in range(4)]
        ref = gamma_np(basis)
        for m in range(4):
            assert np.allclose(g[m], ref[m])
            assert np.allclose(g[m], g[m].conj().T)
            for n in range(4):
                assert np.allclose(g[m] @ g[n] + g[n] @ g[m], 2 * (m == n) * np.eye(4))
        assert np.allclose(O.gamma(15, basis), g[0] @ g[1] @ g[2] @ g[3])
        assert np.allclose(O.gamma(0, basis), np.eye(4))
        assert np.allclose(O.gamma(5, basis), g[0] @ g[2])
    assert np.allclose(O.gamma(15, 0), np.diag([1, 1, -1, -1]))


def test_splitmix64_published_vectors():
    """SplitMix64 with state 1234567: the published first five outputs."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed1234567.txt")
    want = [int(l) for l in open(path) if l.strip() and not l.startswith("#")]
    got = [O.splitmix64(1234567, k) for k in range(5)]
    assert got == want


def test_noise_values_and_moments():
    """Noise: unit modulus, values in the stated sets, <xi> ~ 0, <xi xi*> = delta
    (Eq. delta functions)."""
    dims = (4, 4, 4, 8)
    sets = {O.NOISE_Z4: [1, 1j, -1, -1j],
            O.NOISE_CZ2: [(a + 1j * b) / np.sqrt(2) for a in (1, -1) for b in (1, -1)],
            O.NOISE_Z2: [1, -1]}
    for typ, allowed in sets.items():
        xi = np.stack([O.noise(typ, 77, r, dims).ravel() for r in range(16)])
        assert np.allclose(np.abs(xi), 1.0)
        d = np.min(np.abs(xi[..., None] - np.array(allowed)[None, None, :]), axis=-1)
        assert d.max() < 1e-15
        n = xi.size
        assert abs(xi.mean()) < 5 / np.sqrt(n)
        # off-diagonal correlation between distinct components, averaged over r
        c = np.mean(xi[:, :-1] * xi[:, 1:].conj())
        assert abs(c) < 5 / np.sqrt(n)
        # every value of the set occurs with its share
        counts = [np.sum(np.abs(xi - a) < 1e-12) / n for a in allowed]
        assert np.allclose(counts, 1 / len(allowed), atol=0.02)
    # the key depends on every field: different r, seed give different vectors
    a = O.noise(0, 1, 0, dims)
    assert not np.allclose(a, O.noise(0, 1, 1, dims))
    assert not np.allclose(a, O.noise(0, 2, 0, dims))


def test_noise_key_layout():
    """xi_r(site, spin, colour) takes the top two bits of splitmix64(seed, k) with
    k = ((r V + site) 4 + spin) 3 + colour."""
    dims = (2, 2, 2, 4)
    V = S.volume(dims)
    seed, r = 12345, 3
    xi = O.noise(O.NOISE_Z4, seed, r, dims)
    for site, al, a in [(0, 0, 0), (5, 2, 1), (31, 3, 2)]:
        h = O.splitmix64(seed, ((r * V + site) * 4 + al) * 3 + a)
        want = [1, 1j, -1, -1j][2 * (h >> 63) + ((h >> 62) & 1)]
        assert xi[site, al, a] == want


# ---------------------------------------------------------------------------
# operator
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("bc_t", [-1, 1])
def test_gamma5_hermiticity_and_adjoint(bc_t):
    """D^+ = g5 D g5 and <phi, D psi> = <D^+ phi, psi> for random links."""
    dims = (4, 2, 4, 6)
    U = S.random_links(dims, 0.7, 11)
    psi = S.random_spinors(dims, 2, 12)
    kappa = 0.13
    g5 = np.diag([1, 1, -1, -1]).astype(complex)
    Dpsi = O.apply_D(U, psi, dims, bc_t, kappa)
    Ddag = O.apply_D(U, psi, dims, bc_t, kappa, dagger=True)
    g5Dg5 = np.einsum("ab,nsbc->nsac", g5,
                      O.apply_D(U, np.einsum("ab,nsbc->nsac", g5, psi), dims, bc_t, kappa))
    assert np.abs(Ddag - g5Dg5).max() < 1e-13
    lhs = np.vdot(psi[1], Dpsi[0])
    rhs = np.vdot(Ddag[1], psi[0])
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_hop_unit_links_is_shift_operator():
    """With U = 1, (Hop psi)(x) = sum_mu (1-g_mu) psi(x+mu) + (1+g_mu) psi(x-mu),
    with the t-boundary hop multiplied by bc_t, checked against index shifts."""
    dims = (2, 4, 4, 6)
    V = S.volume(dims)
    U = S.unit_links(dims)
    psi = S.random_spinors(dims, 1, 3)[0]
    g = gamma_np(0)
    for bc in (-1, 1):
        want = np.zeros_like(psi)
        for mu in range(4):
            fw, cf = shift_index(dims, mu, +1)
            bw, cb = shift_index(dims, mu, -1)
            sf = np.where(cf & (mu == 3), bc, 1.0)[:, None, None]
            sb = np.where(cb & (mu == 3), bc, 1.0)[:, None, None]
            want += np.einsum("ab,sbc->sac", np.eye(4) - g[mu], sf * psi[fw])
            want += np.einsum("ab,sbc->sac", np.eye(4) + g[mu], sb * psi[bw])
        got = O.hop(U, psi, dims, bc)
        assert np.abs(got - want).max() < 1e-13
    assert V == 192


def test_gauge_covariance_of_D():
    """D[U^Om] (Om psi) = Om (D[U] psi) for a random SU(3) gauge transformation."""
    dims = (4, 4, 2, 4)
    V = S.volume(dims)
    U = S.random_links(dims, 0.6, 21)
    Om = S.random_su3_field(V, 2.0, 22)
    psi = S.random_spinors(dims, 1, 23)[0]
    Up = gauge_transform(U, Om, dims)
    lhs = O.apply_D(Up, np.einsum("sab,sxb->sxa", Om, psi), dims, -1, 0.12)
    rhs = np.einsum("sab,sxb->sxa", Om, O.apply_D(U, psi, dims, -1, 0.12))
    assert np.abs(lhs - rhs).max() < 1e-13


# ---------------------------------------------------------------------------
# solver and exact loops against dense inverses (brute force)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dims,eps,kappa,bc_t", [((2, 2, 2, 2), 0.5, 0.11, -1),
                                                  ((4, 4, 4, 4), 0.3, 0.10, -1),
                                                  ((4, 4, 4, 4), 0.3, 0.10, 1)])
def test_exact_loops_vs_dense_inverse(dims, eps, kappa, bc_t):
    """Exact loops on timeslice t0 equal those of the dense LU inverse G = D^{-1}.
    Extent 2 makes x+mu and x-mu the same site: both hops must be added."""
    U = S.random_links(dims, eps, 1000)
    G = np.linalg.inv(dense_D(U, dims, kappa, bc_t))
    t0 = 1
    L = O.loops_exact(U, dims, bc_t, kappa, [t0], GAMMAS, tol=1e-14)
    Ld = loops_from_G(G, dims, timeslice_sites(dims, t0), GAMMAS)
    scale = np.abs(Ld[0]).max()
    assert np.abs(L[:, 0, :] - Ld).max() < 1e-12 * scale


def test_solver_methods_agree_with_dense():
    """Even-odd BiCGStab, full BiCGStab and even-odd CGNR all reproduce D^{-1} b
    (Schur identity: x_e = Dhat^{-1}(b_e + k H_eo b_o), x_o = b_o + k H_oe x_e)."""
    dims = (2, 4, 2, 4)
    U = S.random_links(dims, 0.5, 31)
    kappa, bc = 0.13, -1
    b = S.random_spinors(dims, 2, 32)
    D = dense_D(U, dims, kappa, bc)
    xd = np.linalg.solve(D, b.reshape(2, -1).T).T.reshape(b.shape)
    for method in (0, 1, 2):
        x, it, res, fails = O.solve(U, b, dims, bc, kappa, tol=1e-13, method=method)
        assert fails == 0
        assert np.all(res <= 1e-13)
        assert np.abs(x - xd).max() < 1e-11 * np.abs(xd).max()


def test_schur_operator_vs_dense_blocks():
    """Dhat = 1 - D_eo D_oe (D_oo = 1) on even sites, built from dense D blocks,
    and Dhat^+ as the conjugate transpose of that block."""
    dims = (4, 2, 2, 4)
    V = S.volume(dims)
    U = S.random_links(dims, 0.5, 41)
    kappa, bc = 0.12, 1
    D = dense_D(U, dims, kappa, bc)
    par = np.array([sum(S.site_coords(dims, s)) % 2 for s in range(V)])
    ev = np.repeat(par == 0, 12)
    od = ~ev
    Dhat = np.eye(ev.sum()) - D[np.ix_(ev, od)] @ D[np.ix_(od, ev)]
    x = S.random_spinors(dims, 1, 42)[0]
    x[par == 1] = 0
    got = O.apply_Dhat(U, x, dims, bc, kappa).reshape(-1)
    assert np.abs(got[od]).max() == 0.0
    assert np.abs(got[ev] - Dhat @ x.reshape(-1)[ev]).max() < 1e-13
    # dagger = 1 is the conjugate transpose of the same dense block
    got = O.apply_Dhat(U, x, dims, bc, kappa, dagger=True).reshape(-1)
    assert np.abs(got[od]).max() == 0.0
    assert np.abs(got[ev] - Dhat.conj().T @ x.reshape(-1)[ev]).max() < 1e-13


def test_neumann_series():
    """For kappa < 1/8, G = sum_n kappa^n Hop^n, with tail <= (8k)^{N+1}/(1-8k)."""
    dims = (4, 4, 2, 2)
    U = S.random_links(dims, 0.8, 51)
    kappa = 0.06
    b = S.random_spinors(dims, 1, 52)[0]
    x, _, _, _ = O.solve(U, b, dims, -1, kappa, tol=1e-14)
    term = b.copy()
    acc = b.copy()
    for n in range(1, 40):
        term = kappa * O.hop(U, term, dims, -1)
        acc += term
    bound = (8 * kappa) ** 40 / (1 - 8 * kappa) * np.linalg.norm(b)
    assert np.linalg.norm(acc - x) < bound + 1e-12 * np.linalg.norm(b)


# ---------------------------------------------------------------------------
# loops: closed forms, symmetries, hopping expansion
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dims,kappa,bc_t", [((2, 2, 2, 2), 0.10, -1), ((2, 2, 2, 2), 0.10, 1),
                                             ((4, 4, 4, 4), 0.10, -1), ((4, 4, 4, 4), 0.10, 1),
                                             ((4, 2, 6, 8), 0.12, -1)])
def test_free_field_closed_form(dims, kappa, bc_t):
    """U = 1: L_1 = (12/V) sum_p A/(A^2+B^2), L_g5 = L_gmu = 0 at every site."""
    A, B = free_AB(dims, kappa, bc_t)
    V = S.volume(dims)
    L1 = 12.0 / V * np.sum(A / (A ** 2 + sum(b ** 2 for b in B)))
    U = S.unit_links(dims)
    L = O.loops_exact(U, dims, bc_t, kappa, [0, dims[3] - 1], GAMMAS, tol=1e-14)
    assert np.abs(L[0] - L1).max() < 1e-12 * L1
    assert np.abs(L[1:]).max() < 1e-12


def test_free_field_reference_values():
    """Closed-form free-field L_1 at the lattices of the workloads (4^4 and 2^4 at
    kappa=0.1) evaluated independently of the oracle's position-space code."""
    for dims, kappa, bc, want in [((2, 2, 2, 2), 0.10, -1, 12.865843218784393),
                                  ((2, 2, 2, 2), 0.10, 1, 15.809523809523812),
                                  ((4, 4, 4, 4), 0.10, -1, 11.865547549638279),
                                  ((4, 4, 4, 4), 0.10, 1, 11.973384355150129)]:
        A, B = free_AB(dims, kappa, bc)
        L1 = 12.0 / S.volume(dims) * np.sum(A / (A ** 2 + sum(b ** 2 for b in B)))
        assert abs(L1 - want) < 1e-13
        L = O.loops_exact_sites(S.unit_links(dims), dims, bc, kappa, [0], [0], tol=1e-14)
        assert abs(L[0, 0] - want) < 1e-12


def test_constant_diagonal_background():
    """U_mu = diag(e^{i th1}, e^{i th2}, e^{-i(th1+th2)}): colour c sees p + theta^c;
    L_1 = (4/V) sum_c sum_p A_c/(A_c^2+B_c^2), L_gmu = (-4i/V) sum_c sum_p B_cmu/(...),
    L_g5 = 0.  The sign of L_gmu fixes the (1 - g_mu) forward-hop convention."""
    dims = (2, 4, 4, 6)
    V = S.volume(dims)
    kappa, bc = 0.11, -1
    th = [(0.3, -0.5), (0.7, 0.2), (-0.4, 0.9), (0.25, 0.6)]
    U = S.diagonal_links(dims, th)
    cols = [[th[mu][0] for mu in range(4)], [th[mu][1] for mu in range(4)],
            [-(th[mu][0] + th[mu][1]) for mu in range(4)]]
    L1 = 0.0
    Lg = np.zeros(4, complex)
    for c in range(3):
        A, B = free_AB(dims, kappa, bc, cols[c])
        den = A ** 2 + sum(b ** 2 for b in B)
        L1 += 4.0 / V * np.sum(A / den)
        for mu in range(4):
            Lg[mu] += -4j / V * np.sum(B[mu] / den)
    L = O.loops_exact_sites(U, dims, bc, kappa, [0, 37, V - 1], GAMMAS, tol=1e-14)
    assert np.abs(L[0] - L1).max() < 1e-12 * abs(L1)
    for mu in range(4):
        assert np.abs(L[1 + mu] - Lg[mu]).max() < 1e-12 * abs(L1)
        assert abs(Lg[mu]) > 1e-3  # the check is not vacuous
    assert np.abs(L[5]).max() < 1e-12


def test_gamma5_hermiticity_of_loops():
    """From D^+ = g5 D g5: L_1 and L_g5 are real and L_gmu purely imaginary per site."""
    dims = (4, 4, 4, 4)
    U = S.random_links(dims, 0.5, 61)
    L = O.loops_exact(U, dims, -1, 0.12, [2], GAMMAS, tol=1e-14)
    assert np.abs(L[0].imag).max() < 1e-13
    assert np.abs(L[5].imag).max() < 1e-13
    assert np.abs(L[1:5].real).max() < 1e-13
    assert np.abs(L[1:5].imag).max() > 1e-5


def test_gauge_invariance_of_loops():
    """Each L_Gamma(x) is unchanged under U_mu(x) -> Om(x) U_mu(x) Om(x+mu)^+."""
    dims = (4, 4, 4, 4)
    V = S.volume(dims)
    U = S.random_links(dims, 0.5, 71)
    Om = S.random_su3_field(V, 3.0, 72)
    Up = gauge_transform(U, Om, dims)
    sites = [0, 5, 77, 200]
    L = O.loops_exact_sites(U, dims, -1, 0.12, sites, GAMMAS, tol=1e-14)
    Lp = O.loops_exact_sites(Up, dims, -1, 0.12, sites, GAMMAS, tol=1e-14)
    assert np.abs(L - Lp).max() < 1e-12


def test_basis_independence():
    """Chiral and Dirac-Pauli bases give the same loops (unitarily equivalent)."""
    dims = (4, 2, 2, 4)
    U = S.random_links(dims, 0.5, 81)
    L0 = O.loops_exact(U, dims, -1, 0.12, [1], GAMMAS, tol=1e-14, basis=0)
    L1 = O.loops_exact(U, dims, -1, 0.12, [1], GAMMAS, tol=1e-14, basis=1)
    assert np.abs(L0 - L1).max() < 1e-12


def test_hopping_expansion_plaquettes():
    """Extents >= 5: L_1(x) = 12 - 16 k^4 sum_{24 plaquettes at x} Re Tr U_P + O(k^6)
    (no k^2 term since (1-g)(1+g) = 0; spin trace around a plaquette = -8)."""
    dims = (6, 6, 6, 6)
    U = S.random_links(dims, 0.7, 91)
    sites = [0, 433]
    res = {}
    for k in (0.02, 0.04):
        L = O.loops_exact_sites(U, dims, -1, k, sites, [0], tol=1e-15)
        res[k] = np.array([L[0, j].real - 12 + 16 * k ** 4 * plaquette_sum(U, dims, s)
                           for j, s in enumerate(sites)])
    ratio = res[0.04] / res[0.02]
    # residual is O(k^6): doubling k multiplies it by ~2^6 (up to O(k^8) terms)
    assert np.all(np.abs(ratio - 64) < 4), ratio


def test_hopping_expansion_polyakov_boundary_sign():
    """Extent 4: each direction adds +64 k^4 bc_mu Re Tr P_mu(x) (straight Polyakov
    loop), which fixes the sign of the time-boundary hop."""
    dims = (4, 4, 4, 4)
    U = S.random_links(dims, 0.6, 95)
    site = 0
    fw = [shift_index(dims, mu, +1)[0] for mu in range(4)]

    def poly(mu):
        P = np.eye(3, dtype=complex)
        x = site
        for _ in range(dims[mu]):
            P = P @ U[mu][x]
            x = fw[mu][x]
        return np.trace(P).real

    for bc in (-1, 1):
        r = {}
        for k in (0.02, 0.04):
            L = O.loops_exact_sites(U, dims, bc, k, [site], [0], tol=1e-15)
            pred = 12 - 16 * k ** 4 * plaquette_sum(U, dims, site) + 64 * k ** 4 * (
                poly(0) + poly(1) + poly(2) + bc * poly(3))
            r[k] = L[0, 0].real - pred
        assert abs(r[0.04] / r[0.02] - 64) < 4, (bc, r)


# ---------------------------------------------------------------------------
# stochastic estimators and the truncated solver method
# ---------------------------------------------------------------------------
def dilution_components(dims, mask, t_lo, t_hi):
    """List of boolean masks [V][4][3] for each dilution component (test's own)."""
    V = S.volume(dims)
    c = np.array([S.site_coords(dims, s) for s in range(V)])
    ts = range(t_lo, t_hi) if mask & 1 else [None]
    spins = range(4) if mask & 2 else [None]
    cols = range(3) if mask & 4 else [None]
    if mask & 16:
        classes, cls = range(8), (c[:, 0] % 2) + 2 * (c[:, 1] % 2) + 4 * (c[:, 2] % 2)
    elif mask & 8:
        classes, cls = range(2), (c[:, 0] + c[:, 1] + c[:, 2]) % 2
    else:
        classes, cls = [None], np.zeros(V, int)
    comps = []
    for t in ts:
        for be in spins:
            for b in cols:
                for sc in classes:
                    m = np.ones((V, 4, 3), bool)
                    if t is not None:
                        m &= (c[:, 3] == t)[:, None, None]
                    if be is not None:
                        m[:, [a for a in range(4) if a != be], :] = False
                    if b is not None:
                        m[:, :, [a for a in range(3) if a != b]] = False
                    if sc is not None:
                        m &= (cls == sc)[:, None, None]
                    comps.append(m)
    return comps


@pytest.mark.parametrize("mask", [1 | 2 | 4, 1 | 8, 1 | 2 | 16, 0])
def test_stochastic_estimator_vs_dense(mask):
    """Lhat(x) = (1/N) sum_r sum_d eta_{r,d}^+ Gamma (G eta_{r,d}) evaluated with the
    dense inverse G and the oracle's noise equals the oracle's estimator."""
    dims = (2, 2, 4, 4)
    U = S.random_links(dims, 0.5, 101)
    kappa, bc = 0.12, -1
    G = np.linalg.inv(dense_D(U, dims, kappa, bc))
    nr, seed, t_lo, t_hi = 2, 555, 1, 3
    Vs = dims[0] * dims[1] * dims[2]
    want = np.zeros((len(GAMMAS), t_hi - t_lo, Vs), complex)
    for r in range(nr):
        xi = O.noise(O.NOISE_Z4, seed, r, dims)
        for m in dilution_components(dims, mask, t_lo, t_hi):
            eta = np.where(m, xi, 0)
            phi = (G @ eta.reshape(-1)).reshape(eta.shape)
            for k, gm in enumerate(GAMMAS):
                loc = np.einsum("sac,ab,sbc->s", eta.conj(), O.gamma(gm), phi)
                for tt in range(t_hi - t_lo):
                    want[k, tt] += loc[Vs * (t_lo + tt):Vs * (t_lo + tt + 1)] / nr
    got = O.loops_stochastic(U, dims, bc, kappa, O.NOISE_Z4, seed, 0, nr, mask, t_lo, t_hi,
                             GAMMAS, tol=1e-14)
    assert np.abs(got - want).max() < 1e-12


def _per_noise_estimates(U, dims, bc, kappa, fn, nr):
    return np.stack([fn(r) for r in range(nr)])


def test_stochastic_estimator_is_unbiased():
    """<phi xi*> = G (Eq. propagator noise*result): the mean over many noise vectors of
    the spin-colour-time diluted estimator agrees with the exact loop (z-test)."""
    dims = (2, 2, 2, 4)
    U = S.random_links(dims, 0.5, 111)
    kappa, bc = 0.12, -1
    exact = O.loops_exact(U, dims, bc, kappa, [0, 1], GAMMAS, tol=1e-14)
    nr = 300
    est = np.stack([O.loops_stochastic(U, dims, bc, kappa, O.NOISE_CZ2, 9, r, 1, 7, 0, 2,
                                       GAMMAS, tol=1e-13) for r in range(nr)])
    mean = est.mean(0)
    err = est.std(0) / np.sqrt(nr)
    z = np.abs(mean - exact) / np.maximum(err, 1e-12)
    # values whose estimator has no variance must be exact
    assert np.all((z < 5) | (np.abs(mean - exact) < 1e-10))
    # and the estimator is not trivially exact
    assert err.max() > 1e-4


def test_tsm_collapses_when_lp_equals_hp():
    """TSM with tol_LP = tol_HP: phi^LP = phi^HP, the correction vanishes and the
    estimate equals the plain estimator over the LP ensemble."""
    dims = (2, 2, 2, 4)
    U = S.random_links(dims, 0.5, 121)
    kappa, bc = 0.12, -1
    tsm = O.loops_tsm(U, dims, bc, kappa, O.NOISE_CZ2, 5, 0, 3, 2, 1e-13, 1e-13, 1 | 2 | 4, 0,
                      4, GAMMAS)
    plain = O.loops_stochastic(U, dims, bc, kappa, O.NOISE_CZ2, 5, 0, 3, 1 | 2 | 4, 0, 4,
                               GAMMAS, tol=1e-13)
    assert np.abs(tsm - plain).max() < 1e-13


def test_tsm_lp_error_is_bounded_by_truncation():
    """|Lhat_LP - Lhat_(exact solves, same noise)| is of the order of tol_LP."""
    dims = (2, 2, 4, 4)
    U = S.random_links(dims, 0.5, 131)
    kappa, bc = 0.12, -1
    args = (U, dims, bc, kappa, O.NOISE_CZ2, 8, 0)
    lp = O.loops_tsm(*args, 2, 0, 1e-3, 1e-3, 0, 0, 4, GAMMAS)
    ex = O.loops_tsm(*args, 2, 0, 1e-13, 1e-13, 0, 0, 4, GAMMAS)
    diff = np.abs(lp - ex).max()
    assert 0 < diff < 30 * 1e-3 * np.abs(ex[0]).max()


def test_tsm_is_unbiased():
    """TSM mean over independent noise draws agrees with the exact loop (z-test)."""
    dims = (2, 2, 2, 4)
    U = S.random_links(dims, 0.5, 141)
    kappa, bc = 0.12, -1
    exact = O.loops_exact(U, dims, bc, kappa, [0, 1, 2, 3], GAMMAS, tol=1e-14)
    reps = 80
    est = np.stack([O.loops_tsm(U, dims, bc, kappa, O.NOISE_CZ2, 1000 + i, 0, 4, 2, 5e-2,
                                1e-13, 0, 0, 4, GAMMAS) for i in range(reps)])
    mean, err = est.mean(0), est.std(0) / np.sqrt(reps)
    z = np.abs(mean - exact) / np.maximum(err, 1e-12)
    assert np.all((z < 5) | (np.abs(mean - exact) < 1e-10))


# ---------------------------------------------------------------------------
# gradients
# ---------------------------------------------------------------------------
def _F(U, dims, bc, kappa, t0, gammas, w):
    L = O.loops_exact(U, dims, bc, kappa, t0, gammas, tol=1e-15)
    return float(np.sum((w.conj() * L).real))


@pytest.mark.parametrize("bc", [-1, 1])
def test_gradient_vs_finite_differences(bc):
    """Adjoint gradient (D^{-+} = g5 D^{-1} g5) against central differences along
    Lie directions U -> exp(i h X) U and along kappa."""
    dims = (2, 2, 2, 4)
    V = S.volume(dims)
    U = S.random_links(dims, 0.5, 151)
    kappa = 0.14
    t0 = [3]
    gammas = [0, 15, 4]
    rng = np.random.Generator(np.random.PCG64(152))
    w = (rng.standard_normal((3, 1, 8)) + 1j * rng.standard_normal((3, 1, 8)))
    w[:, :, 5:] = 0  # sites with no weight are skipped by the adjoint
    dU, dk = O.loops_grad(U, dims, bc, kappa, t0, gammas, w, tol=1e-15)
    h = 1e-5
    X = S.random_su3_directions(4 * V, 153).reshape(4, V, 3, 3)
    for trial in range(3):
        mask = rng.random((4, V)) < 0.3 if trial else np.ones((4, V), bool)
        Xm = X * mask[..., None, None]
        w_, Q = np.linalg.eigh(Xm)
        expo = lambda t: np.einsum("...ij,...j,...kj->...ik", Q, np.exp(1j * t * w_), Q.conj())
        Fp = _F(expo(h) @ U, dims, bc, kappa, t0, gammas, w)
        Fm = _F(expo(-h) @ U, dims, bc, kappa, t0, gammas, w)
        fd = (Fp - Fm) / (2 * h)
        pred = float(np.sum((dU.conj() * (1j * Xm @ U)).real))
        assert abs(fd - pred) < 1e-6 * max(1.0, abs(pred)), (trial, fd, pred)
    hk = 1e-5
    fd = (_F(U, dims, bc, kappa + hk, t0, gammas, w) - _F(U, dims, bc, kappa - hk, t0, gammas, w)) / (2 * hk)
    assert abs(fd - dk) < 1e-6 * max(1.0, abs(dk)), (fd, dk)


def test_tsm_decomposes_into_lp_and_hp_ensembles():
    """TSM = plain LP estimate over r in [0, n_lp) + (HP - LP) estimate over the
    independent indices [n_lp, n_lp + n_hp), each evaluated separately."""
    dims = (2, 2, 2, 4)
    U = S.random_links(dims, 0.5, 161)
    kappa, bc = 0.12, -1
    base = (U, dims, bc, kappa, O.NOISE_CZ2, 17)
    n_lp, n_hp, tlp, thp = 3, 2, 1e-2, 1e-13
    tsm = O.loops_tsm(*base, 0, n_lp, n_hp, tlp, thp, 1 | 2, 0, 4, GAMMAS)
    lp = O.loops_tsm(*base, 0, n_lp, 0, tlp, tlp, 1 | 2, 0, 4, GAMMAS)
    hp_hp = O.loops_tsm(*base, n_lp, n_hp, 0, thp, thp, 1 | 2, 0, 4, GAMMAS)
    hp_lp = O.loops_tsm(*base, n_lp, n_hp, 0, tlp, tlp, 1 | 2, 0, 4, GAMMAS)
    assert np.abs(tsm - (lp + hp_hp - hp_lp)).max() < 1e-13
    assert np.abs(hp_hp - hp_lp).max() > 1e-6  # the correction is not vacuous


def test_wrappers_reject_mis_sized_arrays():
    """The C oracle trusts the sizes it is given: the Python wrappers refuse a
    gauge field or spinor array that does not hold whole fields of the lattice
    (a half-lattice vector handed to the Schur operator, which takes a
    full-lattice vector, would otherwise be read and written past its end)."""
    dims = (2, 2, 2, 4)
    V = 32
    U = S.random_links(dims, 0.3, 5)
    psi = S.random_spinors(dims, 1, 6)[0]
    O.apply_Dhat(U, psi, dims, -1, 0.1)  # well-formed call
    with pytest.raises(ValueError):
        O.apply_Dhat(U, psi[:V // 2], dims, -1, 0.1)
    with pytest.raises(ValueError):
        O.apply_D(U[:, :V // 2], psi, dims, -1, 0.1)
    with pytest.raises(ValueError):
        O.hop(U, S.random_spinors(dims, 2, 7), dims, -1)
    with pytest.raises(ValueError):
        O.solve(U, psi.reshape(-1)[:-12], dims, -1, 0.1)
