"""Failure reporting of the solves (the stopping rule of Sec. III) through the
C ABI: bounded iteration and outer-cycle budgets, a singular operator, and
the per-solve statistics of every loop entry point (fl_last_stats).

Every case is bounded (max_iter, max_outer), so every kernel exits normally.
Each failing case was first checked on the oracle: the free Wilson operator
at kappa = 1/8 with periodic time has the zero mode p = 0 (A = 1 - 8 kappa =
0, B = 0), and 3 BiCGStab iterations leave a 4^4 residual near 1e-3.
"""
import numpy as np
import pytest

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu

GAMMAS = [0, 15, 1, 2, 4, 8]
FAIL = (-5, -6)  # FL_ERR_NOCONV, FL_ERR_BREAKDOWN


@pytest.fixture(scope="module")
def F():
    import paper_1108_2473_amd as fl
    fl.lib()
    return fl


def make(F, dims, eps, kappa, bc, seed):
    U = S.random_links(dims, eps, seed)
    lat = F.Lattice(dims, bc)
    lat.set_gauge(U)
    lat.set_kappa(kappa)
    return lat, U


def unit_links(dims):
    U = np.zeros((4, S.volume(dims), 3, 3), complex)
    U[:] = np.eye(3)
    return U


PRECS = [("f64", dict(inner_prec=0, gauge_reals=18)), ("f32", dict(inner_prec=1, gauge_reals=12)),
         ("h16 cgnr", dict(inner_prec=3, gauge_reals=12, solver=1))]


@pytest.mark.parametrize("name,kw", PRECS, ids=[p[0] for p in PRECS])
def test_bounded_iterations_report_noconv(F, name, kw):
    """max_iter = 3 on 4^4 at kappa 0.1: fl_solve returns FL_ERR_NOCONV with the
    best iterate (finite) and statistics that say so."""
    dims = (4, 4, 4, 4)
    lat, U = make(F, dims, 0.3, 0.10, -1, 1000)
    b = S.random_spinors(dims, 3, 7)
    x, it, res, fails = O.solve(U, b, dims, -1, 0.10, tol=1e-12, max_iter=3)
    assert fails == 3  # the oracle fails the same way
    x, info = lat.solve(b, F.SolverParams(tol=1e-12, max_iter=3, **kw), check=False)
    assert np.isfinite(x).all()
    assert all(not i["converged"] and i["iters"] <= 3 and i["true_resid"] > 1e-12 for i in info), info
    with pytest.raises(F.FloopError) as e:
        lat.solve(b, F.SolverParams(tol=1e-12, max_iter=3, **kw))
    assert e.value.status == -5
    st = lat.last_stats()
    assert len(st["iters"]) == 3 and not st["converged"].any()
    # the reported residual is the full operator's, recomputed from x
    r = O.apply_D(U, x, dims, -1, 0.10) - b
    want = np.linalg.norm(r.reshape(3, -1), axis=1) / np.linalg.norm(b.reshape(3, -1), axis=1)
    assert np.allclose([i["true_resid"] for i in info], want, rtol=1e-6)


def test_outer_cycle_budget(F):
    """max_outer = 1 with FP32 iterations cannot reach 1e-12 (one FP64 residual
    replacement per decade of reduction at delta 0.1): FL_ERR_NOCONV after
    exactly one replacement."""
    dims = (4, 4, 4, 4)
    lat, U = make(F, dims, 0.3, 0.10, -1, 1000)
    b = S.random_spinors(dims, 2, 8)
    x, info = lat.solve(b, F.SolverParams(tol=1e-12, inner_prec=1, max_outer=1), check=False)
    assert all(not i["converged"] and i["updates"] == 1 for i in info), info
    assert np.isfinite(x).all()
    x, info = lat.solve(b, F.SolverParams(tol=1e-12, inner_prec=1))
    assert all(i["converged"] and i["updates"] > 1 for i in info), info


@pytest.mark.parametrize("solver", [0, 1])
def test_singular_free_field(F, solver):
    """Unit links, kappa = 1/8, periodic time: D has a zero mode; 50 iterations
    end in FL_ERR_NOCONV or FL_ERR_BREAKDOWN with finite outputs, for fl_solve
    and for the exact loops."""
    dims = (4, 4, 4, 4)
    U = unit_links(dims)
    b = S.random_spinors(dims, 2, 5)
    x, it, res, fails = O.solve(U, b, dims, 1, 0.125, tol=1e-12, max_iter=50)
    assert fails == 2
    lat = F.Lattice(dims, 1)
    lat.set_gauge(U)
    lat.set_kappa(0.125)
    prm = F.SolverParams(tol=1e-12, max_iter=50, solver=solver, inner_prec=1)
    with pytest.raises(F.FloopError) as e:
        lat.solve(b, prm)
    assert e.value.status in FAIL
    st = lat.last_stats()
    assert len(st["iters"]) == 2 and not st["converged"].any() and (st["iters"] <= 50).all()
    with pytest.raises(F.FloopError) as e:
        lat.loops_exact_sites([0, 37], GAMMAS, prm)
    assert e.value.status in FAIL and np.isfinite(e.value.result).all()
    st = lat.last_stats()
    assert len(st["iters"]) == 24 and not st["converged"].all()


def test_stochastic_loops_report_lp_failures(F):
    """The plain estimator (n_hp = 0, not truncated) is the benchmark's step: a
    solve of it that misses tol makes fl_loops_stochastic return
    FL_ERR_NOCONV, with the estimate of the best iterates attached; truncated
    LP solves that do not reach their own tolerance are reported too."""
    dims = (4, 4, 2, 6)
    lat, U = make(F, dims, 0.5, 0.12, -1, 61)
    q = F.NoiseParams(noise=0, seed=3, r0=0, n_lp=2, n_hp=0, dilution=1 | 2 | 4, t_begin=0, t_end=6)
    ncomp = 6 * 4 * 3
    for prm in (F.SolverParams(tol=1e-12, max_iter=3, inner_prec=3, gauge_reals=12, solver=1),
                F.SolverParams(tol=1e-8, max_iter=2, truncated=True)):
        with pytest.raises(F.FloopError) as e:
            lat.loops_stochastic(q, GAMMAS, lp=prm)
        assert e.value.status == -5
        assert np.isfinite(e.value.result[0]).all()
        st = lat.last_stats()
        assert len(st["iters"]) == 2 * ncomp and not st["converged"].any()


def test_statistics_of_converged_loops(F):
    """Converged calls return FL_OK and one entry per solve in the documented
    order: TSM (truncated LP at 1e-3, HP at 1e-12) gives n_lp + 2 n_hp vectors
    of components, the HP ones (the last n_hp blocks) accepted on the full
    operator; exact loops give 12 entries per site."""
    dims = (4, 4, 2, 6)
    lat, U = make(F, dims, 0.5, 0.12, -1, 81)
    q = F.NoiseParams(noise=1, seed=9, r0=0, n_lp=3, n_hp=2, dilution=2 | 4, t_begin=0, t_end=6)
    lat.loops_stochastic(q, GAMMAS, lp=F.SolverParams(tol=1e-3, truncated=True), hp=F.SolverParams(tol=1e-12))
    st = lat.last_stats()
    nc = 12
    assert len(st["iters"]) == (3 + 2 * 2) * nc and st["converged"].all()
    kinds = ["lp"] * 3 * nc + (["lp"] * nc + ["hp"] * nc) * 2
    hp = np.array([k == "hp" for k in kinds])
    assert (st["true_resid"][hp] <= 1e-12).all() and (st["true_resid"][~hp] <= 1e-3).all()
    assert (st["updates"][~hp] == 0).all() and (st["seconds"] > 0).all()
    sites = [0, 5, 77]
    lat.loops_exact_sites(sites, GAMMAS, F.SolverParams(tol=1e-12, inner_prec=3, gauge_reals=12, solver=1))
    st = lat.last_stats()
    assert len(st["iters"]) == 12 * len(sites) and st["converged"].all() and (st["true_resid"] <= 1e-12).all()


def test_empty_inputs_do_nothing(F):
    """Zero right-hand sides, an empty site list and an empty timeslice list
    are valid calls that launch nothing and return empty results."""
    dims = (4, 4, 2, 6)
    lat, _ = make(F, dims, 0.4, 0.12, -1, 61)
    try:
        V = S.volume(dims)
        empty = np.zeros((0, V, 4, 3), complex)
        print("empty inputs", flush=True)
        assert lat.apply_D(empty).shape == (0, V, 4, 3)
        x, info = lat.solve(empty, F.SolverParams(tol=1e-10))
        assert x.shape == (0, V, 4, 3) and len(info) == 0
        assert len(lat.last_stats()["iters"]) == 0
        L = lat.loops_exact_sites([], GAMMAS, F.SolverParams(tol=1e-10))
        assert L.shape == (len(GAMMAS), 0)
        L = lat.loops_exact([], GAMMAS, F.SolverParams(tol=1e-10))
        assert L.shape == (len(GAMMAS), 0, dims[0] * dims[1] * dims[2])
        # the context still works afterwards
        b = S.random_spinors(dims, 1, 3)
        x, info = lat.solve(b, F.SolverParams(tol=1e-10))
        assert info[0]["converged"]
    finally:
        lat.close()
