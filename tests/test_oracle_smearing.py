"""Pins of the oracle's Gaussian smearing and connected pseudoscalar
two-point function (Sec. III) against closed forms, symmetries and a dense
brute-force inverse."""
import numpy as np

import oracle as O
import synth_inputs as S


def test_smearing_free_field_plane_wave():
    """U = 1: a plane wave exp(i p.x) is an eigenvector of 1 + alpha H with
    eigenvalue 1 + 2 alpha sum_i cos(p_i) (spin and colour spectators)."""
    dims = (4, 6, 2, 3)
    U = S.unit_links(dims)
    x, y, z, t = O._site_coords(dims)
    n = (1, 2, 1)
    p = [2 * np.pi * n[d] / dims[d] for d in range(3)]
    wave = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z))
    psi = np.zeros((1, S.volume(dims), 4, 3), complex)
    psi[0, :, 2, 1] = wave
    alpha = 0.7
    out = O.smear(U, psi, dims, alpha, 3, norm=1.3)
    lam = (1 + 2 * alpha * sum(np.cos(q) for q in p)) / 1.3
    assert np.allclose(out, lam ** 3 * psi, rtol=1e-13, atol=1e-13)


def test_smearing_is_hermitian_and_gauge_covariant():
    dims = (4, 4, 2, 4)
    V = S.volume(dims)
    U = S.random_links(dims, 0.6, 5)
    a, b = S.random_spinors(dims, 1, 6), S.random_spinors(dims, 1, 7)
    Fa, Fb = O.smear(U, a, dims, 0.5, 2), O.smear(U, b, dims, 0.5, 2)
    assert abs(np.vdot(a, Fb) - np.vdot(Fa, b)) <= 1e-12 * abs(np.vdot(a, Fb))
    # gauge covariance: U_i(x) -> W(x) U_i(x) W(x+i)^+, psi -> W psi
    W = S.random_su3_field(V, 0.8, 8)
    Ug = np.empty_like(U)
    for mu in range(4):
        fw = O._shift_index(dims, mu, 1)
        Ug[mu] = np.einsum("vab,vbc,vdc->vad", W, U[mu], W[fw].conj())
    ag = np.einsum("vab,rvsb->rvsa", W, a)
    assert np.allclose(O.smear(Ug, ag, dims, 0.5, 2), np.einsum("vab,rvsb->rvsa", W, Fa), rtol=1e-12, atol=1e-12)
    # smearing never mixes timeslices
    c = np.zeros_like(a)
    Vs = 32
    c[0, Vs * 2:Vs * 3] = a[0, Vs * 2:Vs * 3]
    Fc = O.smear(U, c, dims, 0.5, 3)
    assert np.abs(Fc[0, :Vs * 2]).max() == 0 and np.abs(Fc[0, Vs * 3:]).max() == 0


def test_pion_correlator_against_dense_inverse():
    """C(p, t) from the oracle's solver equals the same sum over the columns of
    a dense LU inverse of D (2^3 x 4, random links), local and smeared."""
    dims = (2, 2, 2, 4)
    V = S.volume(dims)
    kappa, bc = 0.11, -1
    U = S.random_links(dims, 0.5, 9)
    # dense D from applying the oracle's operator to unit vectors
    n = V * 12
    E = np.eye(n, dtype=complex).reshape(n, V, 4, 3)
    Dm = O.apply_D(U, E, dims, bc, kappa).reshape(n, n).T
    Ginv = np.linalg.inv(Dm)
    y0 = 5
    mom = [(0, 0, 0), (1, 0, 1)]
    for sm in (False, True):
        b = O.point_sources(dims, y0)
        if sm:
            b = O.smear(U, b, dims, 0.4, 2)
        phi = (Ginv @ b.reshape(12, n).T).T.reshape(12, V, 4, 3)
        if sm:
            phi = O.smear(U, phi, dims, 0.4, 2)
        rho = np.sum(np.abs(phi) ** 2, axis=(0, 2, 3))
        got = O.pion_correlator(U, dims, bc, kappa, y0, mom, 0.4, 2, 1.0, sm, sm, tol=1e-14)
        x, y, z, t = O._site_coords(dims)
        for k, nv in enumerate(mom):
            for dt in range(4):
                tt = (t[y0] + dt) % 4
                sel = t == tt
                ph = np.exp(2j * np.pi * (nv[0] * (x - x[y0]) / 2 + nv[1] * (y - y[y0]) / 2 + nv[2] * (z - z[y0]) / 2))
                want = np.sum(ph[sel] * rho[sel])
                assert abs(got[k, dt] - want) <= 1e-10 * abs(want) + 1e-14


def test_pion_correlator_zero_momentum_positive():
    dims = (2, 2, 2, 6)
    U = S.random_links(dims, 0.5, 10)
    C = O.pion_correlator(U, dims, -1, 0.12, 3, [(0, 0, 0)])
    assert np.all(C.real > 0) and np.abs(C.imag).max() <= 1e-12 * C.real.max()


# ---------------------------------------------------------------------------
# APE smearing of the links of H (Sec. III) and its SU(3) projection
# ---------------------------------------------------------------------------
def _shift(dims, mu, step):
    """lexicographic index of x + step mu-hat for every x (periodic)"""
    V = S.volume(dims)
    s = np.arange(V)
    c = [(s // int(np.prod(dims[:m]))) % dims[m] for m in range(4)]
    c[mu] = (c[mu] + step) % dims[mu]
    return c[0] + dims[0] * (c[1] + dims[1] * (c[2] + dims[2] * c[3]))


def _mean_spatial_plaquette(U, dims):
    tot, n = 0.0, 0
    for i in range(3):
        for j in range(i + 1, 3):
            fi, fj = _shift(dims, i, 1), _shift(dims, j, 1)
            P = U[i] @ U[j][fi] @ U[i][fj].conj().transpose(0, 2, 1) @ U[j].conj().transpose(0, 2, 1)
            tot += np.trace(P, axis1=1, axis2=2).real.sum() / 3
            n += P.shape[0]
    return tot / n


def test_su3_projection():
    """P(c W H) = W for W in SU(3), c > 0 and H Hermitian positive definite (the
    unitary polar factor, det 1 already); a phase e^{i phi} W with |phi| < pi/3
    returns W; every result is special unitary."""
    rng = np.random.Generator(np.random.PCG64(77))
    W = S.random_su3_field(20, 0.9, 78)
    A = rng.standard_normal((20, 3, 3)) + 1j * rng.standard_normal((20, 3, 3))
    H = A @ A.conj().transpose(0, 2, 1) + 0.5 * np.eye(3)
    assert np.abs(O.su3_project(2.5 * W @ H) - W).max() < 1e-12
    ph = np.exp(1j * rng.uniform(-1.0, 1.0, 20))[:, None, None]
    assert np.abs(O.su3_project(ph * W) - W).max() < 1e-12
    P = O.su3_project(A)
    assert np.abs(P @ P.conj().transpose(0, 2, 1) - np.eye(3)).max() < 1e-12
    assert np.abs(np.linalg.det(P) - 1).max() < 1e-12


def test_ape_fixed_points():
    """Unit links and a constant diagonal SU(3) background are unchanged: every
    staple equals the link itself, V = (1 + 4 alpha) U projects back to U."""
    dims = (4, 2, 4, 2)
    for U in (S.unit_links(dims), S.diagonal_links(dims, [(0.3, -0.2), (0.1, 0.7), (-0.5, 0.2), (0.4, 0.4)])):
        assert np.abs(O.ape_smear(U, dims, 0.5, 3) - U).max() < 1e-13


def test_ape_abelian_closed_form():
    """Diagonal (U(1)^2) links that vary from site to site: APE acts on each
    colour as complex numbers, v_c = e^{i th_i} + alpha sum_j (e^{i up_j} + e^{i down_j})
    with the staple phases th_j(x) + th_i(x+j) - th_j(x+i) and
    -th_j(x-j) + th_i(x-j) + th_j(x-j+i); the polar factor is v_c/|v_c| and the
    determinant phase is removed by a third of its principal argument."""
    dims = (4, 4, 2, 2)
    V = S.volume(dims)
    rng = np.random.Generator(np.random.PCG64(91))
    th = rng.uniform(-0.8, 0.8, (4, V, 2))
    th = np.concatenate([th, -th.sum(axis=2, keepdims=True)], axis=2)  # [mu][x][colour]
    U = np.zeros((4, V, 3, 3), complex)
    for c in range(3):
        U[:, :, c, c] = np.exp(1j * th[:, :, c])
    alpha = 0.4
    got = O.ape_smear(U, dims, alpha, 1)
    for i in range(3):
        fi = _shift(dims, i, 1)
        v = np.exp(1j * th[i])
        for j in range(3):
            if j == i:
                continue
            fj, bj = _shift(dims, j, 1), _shift(dims, j, -1)
            up = th[j] + th[i][fj] - th[j][fi]
            dn = -th[j][bj] + th[i][bj] + th[j][fi[bj]]
            v = v + alpha * (np.exp(1j * up) + np.exp(1j * dn))
        u = v / np.abs(v)
        phi = np.angle(np.prod(u, axis=1))
        want = u * np.exp(-1j * phi / 3)[:, None]
        assert np.abs(np.diagonal(got[i], axis1=1, axis2=2) - want).max() < 1e-13
        assert np.abs(got[i] - np.einsum("vc,cd->vcd", np.diagonal(got[i], axis1=1, axis2=2), np.eye(3))).max() == 0
    assert np.array_equal(got[3], U[3])


def test_ape_gauge_covariance_su3_and_smoothing():
    """U_mu(x) -> Om(x) U_mu(x) Om(x+mu)^+ commutes with APE (staples transform
    like the link, the projection commutes with unitary factors); the result
    is SU(3); the time links are untouched; each step raises the mean spatial
    plaquette of a rough field."""
    dims = (4, 4, 4, 2)
    V = S.volume(dims)
    U = S.random_links(dims, 0.8, 92)
    Om = S.random_su3_field(V, 1.0, 93)

    def transform(W):
        out = np.empty_like(W)
        for mu in range(4):
            out[mu] = Om @ W[mu] @ Om[_shift(dims, mu, 1)].conj().transpose(0, 2, 1)
        return out

    sm = O.ape_smear(U, dims, 0.5, 2)
    assert np.abs(O.ape_smear(transform(U), dims, 0.5, 2) - transform(sm)).max() < 1e-12
    assert np.abs(sm @ sm.conj().transpose(0, 1, 3, 2) - np.eye(3)).max() < 1e-12
    assert np.abs(np.linalg.det(sm) - 1).max() < 1e-12
    assert np.array_equal(sm[3], U[3])
    p = [_mean_spatial_plaquette(O.ape_smear(U, dims, 0.5, n), dims) for n in range(4)]
    assert all(b > a for a, b in zip(p, p[1:])), p
