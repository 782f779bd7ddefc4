"""GPU parity of Gaussian smearing and the connected pseudoscalar two-point
function (Sec. III, Eq. all_corr) against the oracle."""
import numpy as np
import pytest

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_1108_2473_amd as fl
    fl.lib()
    return fl


@pytest.mark.parametrize("dims,alpha,n,norm", [((4, 4, 4, 8), 0.5, 5, 1.0), ((8, 8, 8, 16), 4.0, 50, 25.0),
                                               ((6, 4, 2, 4), 1.5, 3, 2.0)])
def test_smearing_random_fields(F, dims, alpha, n, norm):
    U = S.random_links(dims, 0.5, 31)
    psi = S.random_spinors(dims, 13, 32)  # 13 fields: a ragged second batch of 12
    lat = F.Lattice(dims, -1)
    lat.set_gauge(U)
    got = lat.smear(psi, alpha, n, norm)
    want = O.smear(U, psi, dims, alpha, n, norm)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    lat.close()


def test_smearing_device_in_place(F):
    import torch
    dims = (4, 4, 4, 8)
    U = S.random_links(dims, 0.5, 33)
    psi = S.random_spinors(dims, 2, 34)
    lat = F.Lattice(dims, -1)
    lat.set_gauge(U)
    d = torch.from_numpy(psi).cuda()
    out = lat.smear(d, 4.0, 10, 25.0)
    assert out.data_ptr() == d.data_ptr()
    want = O.smear(U, psi, dims, 4.0, 10, 25.0)
    assert np.abs(d.cpu().numpy() - want).max() <= 1e-12 * np.abs(want).max()
    lat.close()


@pytest.mark.parametrize("smeared", [False, True])
def test_pion_correlator_4x4x4x8(F, smeared):
    dims = (4, 4, 4, 8)
    kappa = 0.12
    U = S.random_links(dims, 0.4, 35)
    lat = F.Lattice(dims, -1)
    lat.set_gauge(U)
    lat.set_kappa(kappa)
    mom = [(0, 0, 0), (1, 0, 0), (0, 1, 1)]
    y0 = 3 + 4 * (1 + 4 * (2 + 4 * 5))  # (3, 1, 2, 5)
    prm = F.SolverParams(tol=1e-12, inner_prec=F.PREC_F64, gauge_reals=18)
    got = lat.pion_corr(y0, prm, 2.0, 8, 13.0, smeared, smeared, mom)
    want = O.pion_correlator(U, dims, -1, kappa, y0, mom, 2.0, 8, 13.0, smeared, smeared, tol=1e-14)
    assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()
    assert np.all(got[0].real > 0) and np.abs(got[0].imag).max() <= 1e-10 * got[0].real.max()
    lat.close()


def test_pion_correlator_8x8x8x16_paper_smearing(F):
    """alpha = 4, n = 50 (the paper's values, norm 1 + 6 alpha), mixed-precision
    solves to 1e-12 against the oracle's FP64 solves."""
    W = S.WORKLOADS["exact_8x8x8x16"]
    dims = W["dims"]
    U = S.random_links(dims, W["eps"], W["link_seed"])
    lat = F.Lattice(dims, W["bc_t"])
    lat.set_gauge(U)
    lat.set_kappa(W["kappa"])
    mom = [(0, 0, 0), (1, 0, 0)]
    got = lat.pion_corr(0, F.SolverParams(tol=1e-12, inner_prec=F.PREC_H16, solver=F.SOLVER_CGNR), 4.0, 50, 25.0,
                        True, True, mom)
    want = O.pion_correlator(U, dims, W["bc_t"], W["kappa"], 0, mom, 4.0, 50, 25.0, True, True, tol=1e-13)
    assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()
    lat.close()
