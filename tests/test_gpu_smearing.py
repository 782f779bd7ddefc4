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


@pytest.mark.parametrize("dims,eps,alpha,n", [((4, 4, 4, 4), 0.6, 0.5, 3), ((6, 4, 2, 4), 0.4, 0.3, 5),
                                              ((8, 8, 8, 16), 0.5, 0.5, 20)])
def test_ape_smearing_matches_oracle(F, dims, eps, alpha, n):
    """APE-smeared links (Newton polar iteration on the GPU, SVD in the oracle)
    against the oracle's to 1e-12, special unitary; n = 0 returns the
    unsmeared field."""
    U = S.random_links(dims, eps, 36)
    lat = F.Lattice(dims, -1)
    lat.set_gauge(U)
    got = lat.ape_smear(alpha, n)
    want = O.ape_smear(U, dims, alpha, n)
    assert np.abs(got - want).max() <= 1e-12
    assert np.abs(np.linalg.det(got) - 1).max() <= 1e-12
    assert np.array_equal(lat.ape_smear(alpha, 0), U)
    lat.close()


def test_pion_correlator_with_ape_links(F):
    """The paper's setup: Gaussian smearing (alpha 4, n 20, norm 1 + 6 alpha)
    with APE-smeared links in H (alpha_APE 0.5, 10 steps), the Dirac operator
    on the unsmeared links; against the oracle; a new gauge field discards
    the smeared links."""
    dims = (4, 4, 4, 8)
    kappa = 0.12
    U = S.random_links(dims, 0.5, 37)
    lat = F.Lattice(dims, -1)
    lat.set_gauge(U)
    lat.set_kappa(kappa)
    Ua = lat.ape_smear(0.5, 10)
    mom = [(0, 0, 0), (1, 0, 0)]
    y0 = 77
    prm = F.SolverParams(tol=1e-12, inner_prec=F.PREC_F64, gauge_reals=18)
    got = lat.pion_corr(y0, prm, 4.0, 20, 25.0, True, True, mom)
    want = O.pion_correlator(U, dims, -1, kappa, y0, mom, 4.0, 20, 25.0, True, True, tol=1e-14,
                             U_smear=O.ape_smear(U, dims, 0.5, 10))
    assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()
    plain = O.pion_correlator(U, dims, -1, kappa, y0, mom, 4.0, 20, 25.0, True, True, tol=1e-14)
    assert np.abs(plain - want).max() > 1e-3 * np.abs(want).max()  # the links of H matter
    psi = S.random_spinors(dims, 2, 38)
    assert np.abs(lat.smear(psi, 4.0, 3, 25.0) - O.smear(Ua, psi, dims, 4.0, 3, 25.0)).max() <= 1e-12
    lat.set_gauge(U)
    assert np.abs(lat.smear(psi, 4.0, 3, 25.0) - O.smear(U, psi, dims, 4.0, 3, 25.0)).max() <= 1e-12
    lat.close()
