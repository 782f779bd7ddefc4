"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Every comparison uses the same seeded inputs on both sides.  Floating-point
results are compared with tolerances derived from the solver tolerance:
loops use the scale-aware error e_Gamma = max_x |L_gpu - L_oracle| / max_x |L_1|
(required <= 1e-10 for solves to 1e-12).
"""
import numpy as np
import pytest

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu

GAMMAS = [0, 15, 1, 2, 4, 8]


@pytest.fixture(scope="module")
def F():
    import paper_1108_2473_amd as fl
    fl.lib()  # raises if the HIP library is missing: no fallback
    return fl


def make(F, dims, eps, kappa, bc, seed):
    U = S.random_links(dims, eps, seed)
    lat = F.Lattice(dims, bc)
    lat.set_gauge(U)
    lat.set_kappa(kappa)
    return lat, U


def loop_err(got, want):
    scale = np.abs(want[0]).max()
    return np.abs(got - want).max() / scale


# ---------------------------------------------------------------------------
# operator
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (6, 2, 4, 10), (8, 4, 2, 6)])
@pytest.mark.parametrize("bc", [-1, 1])
@pytest.mark.parametrize("dagger", [False, True])
def test_apply_D(F, dims, bc, dagger):
    """D psi and D^+ psi (FP64 kernels) equal the oracle's to rounding; (6,2,4,10)
    has 240 sites per parity: three full 64-site blocks and a ragged tail."""
    lat, U = make(F, dims, 0.7, 0.13, bc, 7)
    psi = S.random_spinors(dims, 3, 8)
    got = lat.apply_D(psi, dagger)
    want = O.apply_D(U, psi, dims, bc, 0.13, dagger=dagger)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_apply_D_single_rhs_and_device_arrays(F):
    import torch
    dims = (4, 4, 2, 6)
    lat, U = make(F, dims, 0.5, 0.12, -1, 17)
    psi = S.random_spinors(dims, 1, 18)[0]
    want = O.apply_D(U, psi, dims, -1, 0.12)
    got = lat.apply_D(psi)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    lat.set_gauge(torch.from_numpy(U).cuda())
    got_d = lat.apply_D(torch.from_numpy(psi).cuda())
    assert got_d.is_cuda
    assert np.abs(got_d.cpu().numpy() - want).max() <= 1e-13 * np.abs(want).max()


# ---------------------------------------------------------------------------
# solver
# ---------------------------------------------------------------------------
SOLVERS = [("f64", 0, 18, 0), ("f32r12", 1, 12, 0), ("f32r18", 1, 18, 0), ("bf16r12", 2, 12, 0),
           ("h16", 3, 12, 0), ("cgnr-f64", 0, 18, 1), ("cgnr-f32", 1, 12, 1), ("cgnr-h16", 3, 12, 1)]


@pytest.mark.parametrize("name,prec,reals,solver", SOLVERS)
def test_solve_meets_stopping_rule(F, name, prec, reals, solver):
    """|D x - b| / |b| <= tol on the full operator, recomputed by the oracle, and x
    agrees with the oracle's solution; 5 right-hand sides give a ragged rhs block."""
    dims = (4, 4, 4, 8)
    lat, U = make(F, dims, 0.5, 0.13, -1, 21)
    b = S.random_spinors(dims, 5, 22)
    tol = 1e-12
    x, info = lat.solve(b, F.SolverParams(tol=tol, inner_prec=prec, gauge_reals=reals, solver=solver))
    r = b - O.apply_D(U, x, dims, -1, 0.13)
    rel = np.linalg.norm(r.reshape(5, -1), axis=1) / np.linalg.norm(b.reshape(5, -1), axis=1)
    assert np.all(rel <= 1.05 * tol), rel
    assert all(s["converged"] for s in info)
    for k in range(5):
        assert abs(info[k]["true_resid"] - rel[k]) <= 0.05 * rel[k] + 1e-15
    xo, _, _, fails = O.solve(U, b, dims, -1, 0.13, tol=1e-14)
    assert fails == 0
    assert np.abs(x - xo).max() <= 1e-10 * np.abs(xo).max()


@pytest.mark.parametrize("prec,solver", [(1, 0), (2, 0), (3, 0), (1, 1), (2, 1), (3, 1)])
@pytest.mark.parametrize("src", ["point-even", "point-odd", "random"])
def test_solve_fast_convergence_matrix(F, prec, solver, src):
    """Every mixed-precision iteration (FP32, bf16 links, 16-bit storage;
    BiCGStab and CGNR) on a lattice where one iteration gains ~3x (4^4,
    kappa = 0.1), so that the iteration runs far ahead of the host's
    replacement checks: sparse and dense sources meet the stopping rule on
    the full operator, recomputed by the oracle."""
    dims = (4, 4, 4, 4)
    lat, U = make(F, dims, 0.3, 0.10, -1, 1000)
    V = S.volume(dims)
    if src == "random":
        b = S.random_spinors(dims, 3, 51)
    else:
        site = 0 if src == "point-even" else 1
        b = np.zeros((3, V, 4, 3), complex)
        for k in range(3):
            b[k, site, k, (2 * k) % 3] = 1.0
    x, info = lat.solve(b, F.SolverParams(tol=1e-12, inner_prec=prec, gauge_reals=12, solver=solver))
    assert all(i["converged"] for i in info), info
    r = b - O.apply_D(U, x, dims, -1, 0.10)
    rel = np.linalg.norm(r.reshape(3, -1), axis=1) / np.linalg.norm(b.reshape(3, -1), axis=1)
    assert np.all(rel <= 1.05e-12), rel
    assert max(i["iters"] for i in info) <= 80, info


def test_solve_zero_and_point_sources(F):
    """A zero right-hand side gives x = 0 with no iterations; point sources on even
    and odd sites are solved through the Schur complement."""
    dims = (4, 2, 2, 4)
    lat, U = make(F, dims, 0.4, 0.12, 1, 31)
    b = np.zeros((3,) + (S.volume(dims), 4, 3), complex)
    b[1, 0, 2, 1] = 1.0
    b[2, 5, 0, 0] = 1.0  # site 5 is odd
    x, info = lat.solve(b, F.SolverParams(tol=1e-12, inner_prec=F.PREC_F32))
    assert np.abs(x[0]).max() == 0.0 and info[0]["iters"] == 0
    xo, _, _, _ = O.solve(U, b[1:], dims, 1, 0.12, tol=1e-14)
    assert np.abs(x[1:] - xo).max() <= 1e-10 * np.abs(xo).max()


@pytest.mark.parametrize("prec", [1, 3])
@pytest.mark.parametrize("solver", [0, 1])
def test_truncated_solve_stops_at_its_tolerance(F, prec, solver):
    """LP solve (truncated): FP32 (or 16-bit storage) iteration stopped at
    |r| <= tol |b|, no FP64 step; the true residual of the full operator then
    confirms that the low-precision operator is D to well below tol."""
    dims = (4, 4, 4, 8)
    lat, U = make(F, dims, 0.5, 0.13, -1, 41)
    b = S.random_spinors(dims, 4, 42)
    x, info = lat.solve(b, F.SolverParams(tol=1e-3, truncated=True, inner_prec=prec, solver=solver))
    r = b - O.apply_D(U, x, dims, -1, 0.13)
    rel = np.linalg.norm(r.reshape(4, -1), axis=1) / np.linalg.norm(b.reshape(4, -1), axis=1)
    assert np.all(rel <= 1.2e-3), rel
    assert np.all(rel > 1e-6)  # it did stop early


# ---------------------------------------------------------------------------
# exact loops
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec,reals", [(0, 18), (1, 12), (2, 12), (3, 12)])
def test_exact_loops_4x4x4x4(F, prec, reals):
    """The 4^4 workload (eps 0.3, kappa 0.10, antiperiodic time): all 768 point-source
    solves of timeslice 0, every Gamma, against the oracle (e <= 1e-10)."""
    dims = (4, 4, 4, 4)
    lat, U = make(F, dims, 0.3, 0.10, -1, 1000)
    got = lat.loops_exact([0], GAMMAS, F.SolverParams(tol=1e-12, inner_prec=prec, gauge_reals=reals))
    want = O.loops_exact(U, dims, -1, 0.10, [0], GAMMAS, tol=1e-14)
    assert loop_err(got, want) <= 1e-10
    # gamma_5-hermiticity of the GPU loops: L_1, L_g5 real, L_gmu imaginary
    assert np.abs(got[0].imag).max() < 1e-10 * np.abs(got[0]).max()


def test_exact_loops_S_blocks_and_sites(F):
    """S(y) blocks and an explicit site list (even and odd sites, several timeslices)."""
    dims = (4, 2, 4, 6)
    lat, U = make(F, dims, 0.5, 0.12, 1, 51)
    sites = [0, 1, 7, 13, 40, 95]
    L, Sg = lat.loops_exact_sites(sites, GAMMAS, F.SolverParams(tol=1e-12), want_S=True)
    Lw, Sw = O.loops_exact_sites(U, dims, 1, 0.12, sites, GAMMAS, tol=1e-14, want_S=True)
    assert loop_err(L, Lw) <= 1e-10
    assert np.abs(Sg - Sw).max() <= 1e-10 * np.abs(Sw).max()


def test_exact_loops_8x8x8x16_sampled(F):
    """The 8^3x16 workload (eps 0.5, kappa 0.14): the whole timeslice t0 = 0 (6144
    point sources, FP32 inner + FP64 reliable updates to 1e-12), checked at sampled
    sites of both parities against the oracle."""
    dims = (8, 8, 8, 16)
    lat, U = make(F, dims, 0.5, 0.14, -1, 1010)
    got = lat.loops_exact([0], GAMMAS, F.SolverParams(tol=1e-12, inner_prec=F.PREC_F32, batch=768))
    sample = [0, 1, 137, 511]
    want = O.loops_exact_sites(U, dims, -1, 0.14, sample, GAMMAS, tol=1e-14)
    scale = np.abs(want[0]).max()
    assert np.abs(got[:, 0, sample] - want).max() / scale <= 1e-10
    # every site, gamma_5-hermiticity: L_1 and L_g5 real, L_gmu imaginary
    assert np.abs(got[0:2, 0].imag).max() < 1e-10 * scale
    assert np.abs(got[2:6, 0].real).max() < 1e-10 * scale


# ---------------------------------------------------------------------------
# stochastic loops and the truncated solver method
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dil", [1 | 2 | 4, 1 | 8, 1 | 2 | 16, 0, 2 | 4])
@pytest.mark.parametrize("noise", [0, 1, 2])
def test_stochastic_loops(F, dil, noise):
    """Diluted stochastic estimator (Eq. loop stochastic) against the oracle with the
    same counter-based noise: agreement to 1e-10 needs bit-identical noise."""
    dims = (4, 4, 2, 6)
    lat, U = make(F, dims, 0.5, 0.12, -1, 61)
    q = F.NoiseParams(noise=noise, seed=2000 + noise, r0=3, n_lp=2, n_hp=0, dilution=dil, t_begin=1, t_end=4)
    got = lat.loops_stochastic(q, GAMMAS, lp=F.SolverParams(tol=1e-12))
    want = O.loops_stochastic(U, dims, -1, 0.12, noise, 2000 + noise, 3, 2, dil, 1, 4, GAMMAS, tol=1e-14)
    assert loop_err(got, want) <= 1e-10


def test_tsm_collapses_when_lp_is_hp(F):
    """With the LP solver equal to the HP solver the correction vanishes exactly and
    the TSM estimate equals the plain estimator over the LP ensemble."""
    dims = (4, 4, 2, 6)
    lat, U = make(F, dims, 0.5, 0.12, -1, 71)
    prm = F.SolverParams(tol=1e-12)
    q = F.NoiseParams(noise=1, seed=5, r0=0, n_lp=3, n_hp=2, dilution=1 | 2 | 4, t_begin=0, t_end=6)
    tsm = lat.loops_stochastic(q, GAMMAS, lp=prm, hp=prm)
    q0 = F.NoiseParams(noise=1, seed=5, r0=0, n_lp=3, n_hp=0, dilution=1 | 2 | 4, t_begin=0, t_end=6)
    plain = lat.loops_stochastic(q0, GAMMAS, lp=prm)
    assert np.array_equal(tsm, plain)
    want = O.loops_stochastic(U, dims, -1, 0.12, 1, 5, 0, 3, 1 | 2 | 4, 0, 6, GAMMAS, tol=1e-14)
    assert loop_err(plain, want) <= 1e-10


def test_tsm_against_oracle_parts(F):
    """TSM with truncated FP32 LP solves (tol 1e-3) and FP64-corrected HP solves:
    the HP ensemble's (phi^HP) part equals the oracle's to 1e-10 and the LP-solve
    parts differ from the oracle's only at the truncation level."""
    dims = (4, 4, 2, 6)
    lat, U = make(F, dims, 0.5, 0.12, -1, 81)
    lp = F.SolverParams(tol=1e-3, truncated=True)
    hp = F.SolverParams(tol=1e-12)
    base = dict(noise=1, seed=9, dilution=0, t_begin=0, t_end=6)
    tsm = lat.loops_stochastic(F.NoiseParams(r0=0, n_lp=3, n_hp=2, **base), GAMMAS, lp=lp, hp=hp)
    lp_only = lat.loops_stochastic(F.NoiseParams(r0=0, n_lp=3, n_hp=0, **base), GAMMAS, lp=lp)
    hp_lp = lat.loops_stochastic(F.NoiseParams(r0=3, n_lp=2, n_hp=0, **base), GAMMAS, lp=lp)
    hp_hp = lat.loops_stochastic(F.NoiseParams(r0=3, n_lp=2, n_hp=0, **base), GAMMAS, lp=hp)
    # the TSM combination of its parts (same deterministic LP map in both sums)
    assert np.abs(tsm - (lp_only + hp_hp - hp_lp)).max() <= 1e-12 * np.abs(tsm[0]).max()
    want_hp = O.loops_stochastic(U, dims, -1, 0.12, 1, 9, 3, 2, 0, 0, 6, GAMMAS, tol=1e-14)
    assert loop_err(hp_hp, want_hp) <= 1e-10
    want_lp = O.loops_stochastic(U, dims, -1, 0.12, 1, 9, 0, 3, 0, 0, 6, GAMMAS, tol=1e-14)
    assert loop_err(lp_only, want_lp) <= 50 * 1e-3


def test_multi_lattice_batch_equals_single(F):
    """Three lattices of uneven size solved in one batch give bit-identical results
    to the same lattices solved alone (per-system recurrences, fixed reductions)."""
    cfg = [((4, 4, 4, 4), 0.4, 1030), ((2, 4, 4, 6), 0.5, 1031), ((4, 2, 2, 8), 0.6, 1032)]
    lats = [make(F, d, e, 0.13, -1, s)[0] for d, e, s in cfg]
    lp = F.SolverParams(tol=1e-3, truncated=True)
    hp = F.SolverParams(tol=1e-12)
    qs = [F.NoiseParams(noise=1, seed=2030 + k, r0=0, n_lp=6, n_hp=2, dilution=0, t_begin=0, t_end=d[3])
          for k, (d, _, _) in enumerate(cfg)]
    multi = F.loops_stochastic_multi(lats, qs, GAMMAS, lp, hp)
    for lat, q, m in zip(lats, qs, multi):
        single = lat.loops_stochastic(q, GAMMAS, lp=lp, hp=hp)
        assert np.array_equal(single, m)


def test_deterministic_repeat(F):
    dims = (4, 4, 2, 6)
    lat, U = make(F, dims, 0.5, 0.12, -1, 91)
    q = F.NoiseParams(noise=0, seed=1, r0=0, n_lp=2, n_hp=1, dilution=1 | 2 | 4, t_begin=0, t_end=6)
    lp = F.SolverParams(tol=1e-3, truncated=True)
    a = lat.loops_stochastic(q, GAMMAS, lp=lp, hp=F.SolverParams())
    b = lat.loops_stochastic(q, GAMMAS, lp=lp, hp=F.SolverParams())
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# gradient
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("bc", [-1, 1])
def test_gradient_vs_oracle(F, bc):
    """Adjoint link and kappa gradients of F = Re sum conj(w) L against the oracle."""
    dims = (4, 2, 2, 4)
    lat, U = make(F, dims, 0.5, 0.14, bc, 101)
    rng = np.random.Generator(np.random.PCG64(102))
    w = rng.standard_normal((2, 1, 16)) + 1j * rng.standard_normal((2, 1, 16))
    w[:, :, 10:] = 0
    dU, dk = lat.loops_grad([2], [0, 15], w, F.SolverParams(tol=1e-12))
    dUo, dko = O.loops_grad(U, dims, bc, 0.14, [2], [0, 15], w, tol=1e-14)
    assert np.abs(dU - dUo).max() <= 1e-9 * np.abs(dUo).max()
    assert abs(dk - dko) <= 1e-9 * abs(dko)


@pytest.mark.parametrize("prec", ["h16", "f32", "bf16"])
@pytest.mark.parametrize("solver", [0, 1])
def test_reliable_updates_keep_the_residual(F, solver, prec):
    """With 16-bit or FP32 iteration vectors (and 16-bit or FP32 links) the
    FP64 residual is carried from one replacement to the next as
    rh -= Dhat xl (not recomputed from x): over several replacements (4-8 per
    solve here, one per host check at most) its rounding must stay at the
    FP64 level: a carried residual that drifted below the true one would stop
    the iteration early, and the solution would miss the stopping rule on the
    full operator, recomputed here by the oracle (the reported residual must
    agree with the oracle's too).  bf16 links recompute rh = bh - Dhat xh at
    every replacement, under the same checks."""
    ip, minupd = {"h16": (F.PREC_H16, 5), "f32": (F.PREC_F32, 4), "bf16": (F.PREC_BF16, 4)}[prec]
    dims = (8, 4, 4, 8)
    lat, U = make(F, dims, 0.5, 0.14, -1, 31)
    b = S.random_spinors(dims, 6, 32)
    tol = 1e-12
    x, info = lat.solve(b, F.SolverParams(tol=tol, inner_prec=ip, gauge_reals=12, solver=solver))
    assert all(i["converged"] for i in info), info
    assert min(i["updates"] for i in info) >= minupd, info
    r = b - O.apply_D(U, x, dims, -1, 0.14)
    rel = np.linalg.norm(r.reshape(6, -1), axis=1) / np.linalg.norm(b.reshape(6, -1), axis=1)
    assert np.all(rel <= 1.05 * tol), rel
    for k in range(6):
        assert abs(info[k]["true_resid"] - rel[k]) <= 0.05 * rel[k] + 1e-15


def test_cgnr_16bit_fast_convergence(F):
    """16-bit CGNR on a small, well-conditioned lattice (4^4, kappa = 0.1),
    where an iteration cuts the residual ~3x: point sources (sparse) and a
    random source reach the FP64 stopping rule in at most twice the FP32
    iteration count.  Between two host checks (8 iterations) the 16-bit
    recursive residual runs below what the 16-bit iterate resolves, so the
    replaced residual differs from it by ~10 %; CGNR keeps p across the
    replacement, and without restoring <z, p> = |z|^2 for the replaced z the
    recurrence diverged (true residual growing ~1.3x per iteration)."""
    dims = (4, 4, 4, 4)
    lat, U = make(F, dims, 0.3, 0.10, -1, 1000)
    b = np.zeros((13, 256, 4, 3), complex)
    for sc in range(12):
        b[sc, 1, sc // 3, sc % 3] = 1.0
    b[12] = S.random_spinors(dims, 1, 3)[0]
    it = {}
    for prec in (1, 3):
        x, info = lat.solve(b, F.SolverParams(tol=1e-12, inner_prec=prec, gauge_reals=12, solver=F.SOLVER_CGNR))
        assert all(i["converged"] and i["true_resid"] <= 1e-12 for i in info), (prec, info)
        it[prec] = max(i["iters"] for i in info)
        r = O.apply_D(U, x[12], dims, -1, 0.10) - b[12]
        assert np.linalg.norm(r) <= 1.01e-12 * np.linalg.norm(b[12])
    assert it[3] <= 2 * it[1], it
