"""The comparison of stochastic methods with the exact loops (Sec. III,
figures "compare dilution" and "truncated") run by the GPU library and by
the oracle on the same tiny ensemble with the same noise: every
per-configuration D(t) agrees; and on a larger ensemble the stochastic
estimates approach the exact value as the number of inversions grows."""
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


def test_study_matches_oracle_2x2x2x4(F):
    from paper_1108_2473_amd import study
    dims, bc, kappa = (2, 2, 2, 4), -1, 0.12
    configs = [S.random_links(dims, 0.5, 5000 + c) for c in range(2)]
    hp = F.SolverParams(tol=1e-12, inner_prec=F.PREC_F64, gauge_reals=18)
    lp = F.SolverParams(tol=1e-12, truncated=True, inner_prec=F.PREC_F64, gauge_reals=18)
    res = study.run(configs, dims, bc, kappa, n_noise=(2, 4), tsm=((4, 2),), seed=11, hp=hp, lp_tsm=lp,
                    exact_params=hp)
    masks = {k: v[0] for k, v in study.SCHEMES.items()}
    ref = O.dilution_study(configs, dims, bc, kappa, (2, 4), masks, ((4, 2),), 11, 1e-13, 1e-13)
    # each estimator against its own size (the exact D(3) is ~1e-6 here, the
    # few-vector stochastic estimates ~0.1)
    assert np.abs(res.exact - ref["exact"]).max() <= 1e-9 * np.abs(ref["exact"]).max()
    for key, v in ref["stochastic"].items():
        assert np.abs(res.stochastic[key] - v).max() <= 1e-9 * np.abs(v).max(), key
    for key, v in ref["tsm"].items():
        assert np.abs(res.tsm[key] - v).max() <= 1e-8 * np.abs(v).max(), key


def test_stochastic_error_shrinks_with_inversions(F):
    """4^3x8, 3 configurations: the deviation of the even-odd-diluted estimate
    of D(3) from the exact value, summed over configurations, falls as the
    number of noise vectors grows from 2 to 32 (expected ~ 1/N for a product
    of two independent estimates)."""
    from paper_1108_2473_amd import study
    dims, bc, kappa = (4, 4, 4, 8), -1, 0.12
    configs = [S.random_links(dims, 0.4, 6000 + c) for c in range(3)]
    res = study.run(configs, dims, bc, kappa, n_noise=(2, 32), schemes=("even-odd",), tsm=(), seed=21)
    dev = {N: np.abs(res.stochastic[("even-odd", N)][:, 3] - res.exact[:, 3]).sum() for N in (2, 32)}
    assert dev[32] < 0.5 * dev[2], dev


def test_loop_study_matches_oracle_2x2x2x4(F):
    """The per-insertion comparison (g1..g4 at the lowest momenta, the scalar at
    p = 0): every projected estimate per configuration, GPU against the
    oracle's composition on the same noise (FP64 solves; the TSM's LP map as a
    truncated FP64 solve at 1e-12 so both sides solve to the same accuracy)."""
    from paper_1108_2473_amd import study
    dims, bc, kappa = (2, 2, 2, 4), -1, 0.12
    configs = [S.random_links(dims, 0.5, 5100 + c) for c in range(2)]
    hp = F.SolverParams(tol=1e-12, inner_prec=F.PREC_F64, gauge_reals=18)
    lp = F.SolverParams(tol=1e-12, truncated=True, inner_prec=F.PREC_F64, gauge_reals=18)
    res = study.run_loops(configs, dims, bc, kappa, n_noise=(1, 3), tsm=((3, 2),), seed=13, hp=hp, lp_tsm=lp,
                          exact_params=hp)
    masks = {k: v[0] for k, v in study.SCHEMES.items()}
    ref = O.loop_error_study(configs, dims, bc, kappa, (1, 3), masks, ((3, 2),), 13, 1e-13, 1e-13)
    assert res.pairs == O.GAMMA_MOMENTA
    scale = np.abs(ref["exact"]).max(axis=(0, 2))[None, :, None]
    assert (np.abs(res.exact - ref["exact"]) / scale).max() <= 1e-9
    for key, v in list(ref["stochastic"].items()):
        assert (np.abs(res.stochastic[key] - v) / scale).max() <= 1e-9, key
    for key, v in ref["tsm"].items():
        assert (np.abs(res.tsm[key] - v) / scale).max() <= 1e-9, key
    # the table's deviations are finite and shrink to 0 for no estimator here
    for _, _, d in study.table_loops(res):
        assert all(np.isfinite(x) and x > 0 for x in d.values())
