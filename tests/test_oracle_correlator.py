"""Pins of the oracle's momentum projection and disconnected correlator
(Sec. III, Eq. all_dis_corr) against facts other than their own formulas."""
import numpy as np

import oracle as O


def _rand(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_zero_momentum_is_the_spatial_sum():
    dims = (4, 2, 6, 8)
    L = _rand((3, 8, 48), 1)
    Lp = O.momentum_project(L, dims, [(0, 0, 0)])
    assert np.allclose(Lp[:, 0, :], L.sum(axis=2), rtol=1e-14, atol=1e-13)


def test_all_momenta_equal_the_inverse_fft():
    """Over all Vs momenta the projection is Vs times numpy's inverse FFT
    (which uses exp(+2 pi i k.x / N)) over the (z, y, x) axes of the slice."""
    dims = (4, 6, 2, 3)
    Vs = 48
    L = _rand((2, 3, Vs), 2)
    mom = [(nx, ny, nz) for nz in range(2) for ny in range(6) for nx in range(4)]
    Lp = O.momentum_project(L, dims, mom)
    for g in range(2):
        for t in range(3):
            ref = Vs * np.fft.ifftn(L[g, t].reshape(2, 6, 4))  # [z][y][x] -> frequencies [kz][ky][kx]
            got = np.array([Lp[g, k, t] for k in range(len(mom))]).reshape(2, 6, 4)
            assert np.allclose(got, ref, rtol=1e-12, atol=1e-11)


def test_translation_multiplies_by_a_phase():
    """L'(x) = L(x - a) gives Lp'(p) = exp(i p.a) Lp(p)."""
    dims = (4, 4, 4, 2)
    L = _rand((1, 2, 64), 3).reshape(1, 2, 4, 4, 4)  # [g][t][z][y][x]
    a = (1, 3, 2)
    Ls = np.roll(L, shift=(a[2], a[1], a[0]), axis=(2, 3, 4))
    mom = [(1, 0, 0), (0, 2, 1), (3, 1, 2), (1, 1, 1)]
    Lp = O.momentum_project(L.reshape(1, 2, 64), dims, mom)
    Lps = O.momentum_project(Ls.reshape(1, 2, 64), dims, mom)
    for k, n in enumerate(mom):
        ph = np.exp(2j * np.pi * sum(n[d] * a[d] / dims[d] for d in range(3)))
        assert np.allclose(Lps[0, k], ph * Lp[0, k], rtol=1e-12, atol=1e-12)


def test_correlator_of_point_loops_closed_form():
    """Loops supported on x = 0 only, L(0, t) = f(t): D(p, t) = (1/Vs)(1/T) sum_ti f(ti+t) g(ti)
    for every momentum (the phase at the origin is 1)."""
    dims = (2, 2, 2, 5)
    Vs, T = 8, 5
    f, g = _rand((T,), 4), _rand((T,), 5)
    L1 = np.zeros((1, T, Vs), complex)
    L2 = np.zeros((1, T, Vs), complex)
    L1[0, :, 0], L2[0, :, 0] = f, g
    mom = [(0, 0, 0), (1, 0, 1)]
    D = O.disconnected_correlator(O.momentum_project(L1, dims, mom),
                                  O.momentum_project(L2, dims, [(-a, -b, -c) for a, b, c in mom]), Vs, [(0, 0)])
    for t in range(T):
        want = sum(f[(ti + t) % T] * g[ti] for ti in range(T)) / (Vs * T)
        assert np.allclose(D[0, :, t], want, rtol=1e-13)


def test_correlator_time_translation_invariance_and_pair_symmetry():
    """Shifting both loop sets in time leaves D unchanged; swapping the two
    sets and the pair order maps D(t) to D(T - t)."""
    dims = (2, 2, 2, 6)
    L1, L2 = _rand((2, 6, 8), 6), _rand((2, 6, 8), 7)
    mom = [(0, 0, 0), (1, 1, 0)]
    neg = [(-a, -b, -c) for a, b, c in mom]
    P1, P2 = O.momentum_project(L1, dims, mom), O.momentum_project(L2, dims, neg)
    D = O.disconnected_correlator(P1, P2, 8, [(0, 1), (1, 0)])
    Ds = O.disconnected_correlator(np.roll(P1, 2, axis=2), np.roll(P2, 2, axis=2), 8, [(0, 1), (1, 0)])
    assert np.allclose(D, Ds, rtol=1e-13, atol=1e-15)
    # swapped roles: D'(t) = sum_ti P2[B](ti+t) P1[A](ti) = D(-t)
    Dsw = O.disconnected_correlator(P2, P1, 8, [(1, 0)])
    for t in range(6):
        assert np.allclose(Dsw[0, :, t], D[0, :, (-t) % 6], rtol=1e-13)
