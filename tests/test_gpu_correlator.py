"""GPU parity of the momentum projection and the disconnected two-point
function (Sec. III, Eq. all_dis_corr) against the oracle, on random loops and
on loops the library computes, at 4^3x8, 8^3x16 and 16^3x32."""
import numpy as np
import pytest

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu

GAMMAS = [0, 15, 1, 2, 4, 8]
MOM = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (-1, 0, 0), (1, 1, 0), (1, -1, 1), (2, 0, -1)]


@pytest.fixture(scope="module")
def F():
    import paper_1108_2473_amd as fl
    fl.lib()
    return fl


def _rand(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("dims", [(4, 4, 4, 8), (8, 8, 8, 16), (16, 16, 16, 32), (6, 4, 2, 4)])
def test_projection_and_correlator_random(F, dims):
    Vs, T = dims[0] * dims[1] * dims[2], dims[3]
    lat = F.Lattice(dims, -1)
    L1, L2 = _rand((6, T, Vs), 11), _rand((6, T, Vs), 12)
    neg = [(-a, -b, -c) for a, b, c in MOM]
    P1, P2 = lat.momentum_project(L1, MOM), lat.momentum_project(L2, neg)
    W1, W2 = O.momentum_project(L1, dims, MOM), O.momentum_project(L2, dims, neg)
    scale = np.sqrt(Vs)  # size of a sum of Vs unit-variance terms
    assert np.abs(P1 - W1).max() <= 1e-12 * scale
    assert np.abs(P2 - W2).max() <= 1e-12 * scale
    pairs = [(0, 0), (1, 1), (0, 1), (2, 5)]
    D = lat.disconnected_corr(P1, P2, pairs)
    Dw = O.disconnected_correlator(W1, W2, Vs, pairs)
    assert np.abs(D - Dw).max() <= 1e-12 * np.abs(Dw).max()
    lat.close()


@pytest.mark.parametrize("ng", [1, 3, 4, 5, 16])
def test_projection_gamma_counts(F, ng):
    """The projection handles the Gamma matrices in groups of four per
    workgroup: one, a partial group, exactly one group, a group and one more,
    and the maximum of sixteen, on a lattice with unequal spatial extents."""
    dims = (6, 4, 8, 4)
    Vs, T = 6 * 4 * 8, 4
    lat = F.Lattice(dims, -1)
    L = _rand((ng, T, Vs), 20 + ng)
    P = lat.momentum_project(L, MOM)
    assert P.shape == (ng, len(MOM), T)
    assert np.abs(P - O.momentum_project(L, dims, MOM)).max() <= 1e-12 * np.sqrt(Vs)
    lat.close()


def test_device_arrays_and_argument_checks(F):
    import torch
    dims = (4, 4, 4, 8)
    lat = F.Lattice(dims, -1)
    L = _rand((2, 8, 64), 13)
    Pd = lat.momentum_project(torch.from_numpy(L).cuda(), MOM)
    assert Pd.is_cuda
    assert np.abs(Pd.cpu().numpy() - O.momentum_project(L, dims, MOM)).max() <= 1e-12 * 8
    with pytest.raises(F.FloopError):
        lat.disconnected_corr(Pd, Pd, [(0, 2)])  # Gamma index out of range
    lat.close()
    # spatial extents beyond the projection's phase tables (Lx + Ly + Lz <= 1024)
    wide = F.Lattice((1022, 2, 2, 2), -1)
    with pytest.raises(F.FloopError):
        wide.momentum_project(_rand((1, 2, 1022 * 4), 14), MOM)
    wide.close()


def test_exact_loop_correlator_4x4x4x8(F):
    """Exact loops computed by the library on every timeslice of a 4^3x8
    lattice (eps 0.3, kappa 0.10), projected at zero and unit momenta and
    correlated, against the oracle's own exact loops put through the oracle's
    projection and correlator."""
    W = S.WORKLOADS["exact_4x4x4x4"]
    dims = (4, 4, 4, 8)
    U = S.random_links(dims, W["eps"], W["link_seed"])
    lat = F.Lattice(dims, -1)
    lat.set_gauge(U)
    lat.set_kappa(W["kappa"])
    L = lat.loops_exact(list(range(8)), GAMMAS, F.SolverParams(tol=1e-12))
    Lo = O.loops_exact(U, dims, -1, W["kappa"], list(range(8)), GAMMAS, tol=1e-14)
    mom = [(0, 0, 0), (1, 0, 0), (0, 0, 1)]
    neg = [(-a, -b, -c) for a, b, c in mom]
    D = lat.disconnected_corr(lat.momentum_project(L, mom), lat.momentum_project(L, neg), [(1, 1), (0, 0)])
    Dw = O.disconnected_correlator(O.momentum_project(Lo, dims, mom), O.momentum_project(Lo, dims, neg), 64,
                                   [(1, 1), (0, 0)])
    assert np.abs(D - Dw).max() <= 1e-9 * np.abs(Dw).max()
    # gamma_5 loops are real for exact loops, so the g5-g5 zero-momentum correlator is real
    assert np.abs(D[0, 0].imag).max() <= 1e-9 * np.abs(D[0, 0]).max()
    lat.close()
