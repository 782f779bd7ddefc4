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
