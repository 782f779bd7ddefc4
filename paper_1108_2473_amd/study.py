"""The paper's comparison of stochastic methods with the exact loops (Sec.
III, figures "compare dilution" and "truncated"): the disconnected
pseudoscalar two-point function D(t) at p = 0 (Eq. all_dis_corr,
Gamma = g5) on an ensemble of gauge configurations, computed exactly
(all-to-all: point sources on every site of every timeslice) and
stochastically as a function of the number of inversions, for colour, spin,
even-odd and cubic dilution and for the truncated solver method.

Every step runs on the GPU library: loops (fl_loops_exact,
fl_loops_stochastic), momentum projection and correlator
(fl_momentum_project, fl_disconnected_corr).  Stochastic products are
unbiased: with per-noise-vector loops L^r the estimate over N vectors is
    D_N = [D(S, S) - sum_r D(L^r, L^r)] / (N (N - 1)),  S = sum_r L^r,
and a TSM estimate correlates two independent halves (each with its own LP
and HP vectors).  No time dilution: D(t) needs loops on all timeslices.
"""
from dataclasses import dataclass, field

import numpy as np

from . import (DIL_COLOUR, DIL_CUBIC, DIL_EVENODD, DIL_SPIN, NOISE_CZ2, Lattice, NoiseParams, SolverParams,
               SOLVER_BICGSTAB, PREC_F64)

G5 = 15
SCHEMES = {"colour": (DIL_COLOUR, 3), "spin": (DIL_SPIN, 4), "even-odd": (DIL_EVENODD, 2), "cubic": (DIL_CUBIC, 8)}


@dataclass
class StudyResult:
    """Per-configuration D(t) (rows: configurations) for every estimator."""
    T: int
    exact: np.ndarray = None                      # [nconf][T]
    stochastic: dict = field(default_factory=dict)  # (scheme, N) -> [nconf][T]
    tsm: dict = field(default_factory=dict)         # (n_lp, n_hp) -> [nconf][T]
    inversions: dict = field(default_factory=dict)  # key -> inversions per configuration

    @staticmethod
    def mean_err(rows, t):
        """Ensemble mean and its standard error at separation t."""
        v = np.asarray(rows)[:, t].real
        n = len(v)
        return float(v.mean()), float(v.std(ddof=1) / np.sqrt(n)) if n > 1 else 0.0


def _pair_estimate(lat, Lps):
    """Unbiased D from per-vector projected loops Lps [N][1][T] (p = 0)."""
    N = Lps.shape[0]
    S = Lps.sum(axis=0)[None]  # [1][1][T]
    d_ss = lat.disconnected_corr(S, S, [(0, 0)])[0, 0]
    d_diag = lat.disconnected_corr(Lps, Lps, [(r, r) for r in range(N)])[:, 0].sum(axis=0)
    return (d_ss - d_diag) / (N * (N - 1))


def run(configs, dims, bc_t, kappa, n_noise=(2, 4, 8), schemes=tuple(SCHEMES), tsm=((8, 2),), seed=777,
        hp=None, lp_tsm=None, exact_params=None):
    """configs: list of gauge fields U[4][V][3][3].  Returns a StudyResult."""
    T, Vs = dims[3], dims[0] * dims[1] * dims[2]
    hp = hp or SolverParams(tol=1e-8, solver=SOLVER_BICGSTAB)
    lp_tsm = lp_tsm or SolverParams(tol=1e-2, truncated=True, solver=SOLVER_BICGSTAB)
    exact_params = exact_params or SolverParams(tol=1e-12)
    nmax = max(n_noise) if n_noise else 0
    res = StudyResult(T=T)
    exact, stoch, tsm_rows = [], {}, {}
    lat = Lattice(dims, bc_t)
    zero = [(0, 0, 0)]
    try:
        for ci, U in enumerate(configs):
            lat.set_gauge(U)
            lat.set_kappa(kappa)
            cseed = seed + 1000 * ci
            Lx = lat.loops_exact(list(range(T)), [G5], exact_params)
            P = lat.momentum_project(Lx, zero)
            exact.append(lat.disconnected_corr(P, P, [(0, 0)])[0, 0])
            for name in schemes:
                dil, factor = SCHEMES[name]
                per = []
                for r in range(nmax):
                    q = NoiseParams(noise=NOISE_CZ2, seed=cseed, r0=r, n_lp=1, n_hp=0, dilution=dil,
                                    t_begin=0, t_end=T)
                    per.append(lat.momentum_project(lat.loops_stochastic(q, [G5], lp=hp), zero)[0])
                per = np.array(per)  # [nmax][1][T]
                for N in n_noise:
                    stoch.setdefault((name, N), []).append(_pair_estimate(lat, per[:N]))
                    res.inversions[(name, N)] = N * factor
            for (n_lp, n_hp) in tsm:
                halves = []
                for h in range(2):
                    q = NoiseParams(noise=NOISE_CZ2, seed=cseed + 1, r0=h * (n_lp + n_hp) // 2, n_lp=n_lp // 2,
                                    n_hp=n_hp // 2, dilution=0, t_begin=0, t_end=T)
                    halves.append(lat.momentum_project(lat.loops_stochastic(q, [G5], lp=lp_tsm, hp=hp), zero))
                tsm_rows.setdefault((n_lp, n_hp), []).append(
                    lat.disconnected_corr(halves[0], halves[1], [(0, 0)])[0, 0])
                res.inversions[(n_lp, n_hp)] = (n_lp, n_hp)
    finally:
        lat.close()
    res.exact = np.array(exact)
    res.stochastic = {k: np.array(v) for k, v in stoch.items()}
    res.tsm = {k: np.array(v) for k, v in tsm_rows.items()}
    return res


def table(res: StudyResult, t=3):
    """Rows (method, inversions, mean, error) of D(t) over the ensemble."""
    rows = [("exact", None) + res.mean_err(res.exact, t)]
    for (name, N), v in sorted(res.stochastic.items()):
        rows.append((f"{name} N={N}", res.inversions[(name, N)]) + res.mean_err(v, t))
    for (n_lp, n_hp), v in sorted(res.tsm.items()):
        rows.append((f"TSM LP={n_lp} HP={n_hp}", res.inversions[(n_lp, n_hp)]) + res.mean_err(v, t))
    return rows


# ---------------------------------------------------------------------------
# the comparison per insertion (Sec. IV, figures "spin gammas" and "truncated
# gammas"; Sec. V, figure "compare_unity"): momentum-projected loops
# Lp_Gamma(p, t) = sum_x exp(i p.x) L_Gamma(x, t) of g1..g4 at the lowest
# momenta of the paper's three-point ratios and of the scalar at p = 0,
# stochastic and truncated-solver estimates against the exact loops
# ---------------------------------------------------------------------------
GAMMA_MOMENTA = ((1, (1, 0, 0)), (2, (0, 1, 0)), (4, (0, 0, 1)), (8, (1, 0, 0)), (0, (0, 0, 0)))
PAIR_NAMES = {1: "g1", 2: "g2", 4: "g3", 8: "g4", 0: "1", 15: "g5"}


@dataclass
class LoopStudyResult:
    """Per-configuration projected loops [nconf][npairs][T] for every estimator."""
    T: int
    pairs: tuple
    exact: np.ndarray = None
    stochastic: dict = field(default_factory=dict)  # (scheme, N) -> [nconf][npairs][T]
    tsm: dict = field(default_factory=dict)         # (n_lp, n_hp) -> [nconf][npairs][T]
    inversions: dict = field(default_factory=dict)  # key -> inversions per configuration

    def rel_deviation(self, rows):
        """Per pair: RMS over configurations and t of |estimate - exact|, over
        the RMS of the exact value (the ensemble's own scale)."""
        d = np.asarray(rows) - self.exact
        return np.sqrt((np.abs(d) ** 2).mean(axis=(0, 2)) / (np.abs(self.exact) ** 2).mean(axis=(0, 2)))


def run_loops(configs, dims, bc_t, kappa, n_noise=(4, 16, 64), schemes=tuple(SCHEMES), tsm=((64, 8),), seed=777,
              hp=None, lp_tsm=None, exact_params=None, pairs=GAMMA_MOMENTA, tsm_dilution=0):
    """configs: gauge fields U[4][V][3][3].  Noise as in the D(t) comparison:
    complex Z2, configuration c seeded seed + 1000 c; stochastic estimates over
    N vectors are the mean of the first N per-vector loops (Eq. loop
    stochastic); TSM with seed + 1, noise indices from 0."""
    T = dims[3]
    hp = hp or SolverParams(tol=1e-8, solver=SOLVER_BICGSTAB)
    lp_tsm = lp_tsm or SolverParams(tol=1e-2, truncated=True, solver=SOLVER_BICGSTAB)
    exact_params = exact_params or SolverParams(tol=1e-12)
    gam = sorted({g for g, _ in pairs})
    moms = sorted({tuple(m) for _, m in pairs})
    gi = {g: k for k, g in enumerate(gam)}
    mi = {m: k for k, m in enumerate(moms)}
    res = LoopStudyResult(T=T, pairs=tuple(pairs))
    exact, stoch, tsm_rows = [], {}, {}
    nmax = max(n_noise) if n_noise else 0
    lat = Lattice(dims, bc_t)

    def project(L):  # [ngam][T][Vs] -> [npairs][T]
        P = lat.momentum_project(L, moms)
        return np.array([P[gi[g], mi[tuple(m)]] for g, m in pairs])

    try:
        for ci, U in enumerate(configs):
            lat.set_gauge(U)
            lat.set_kappa(kappa)
            cseed = seed + 1000 * ci
            exact.append(project(lat.loops_exact(list(range(T)), gam, exact_params)))
            for name in schemes:
                dil, factor = SCHEMES[name]
                per = [project(lat.loops_stochastic(NoiseParams(noise=NOISE_CZ2, seed=cseed, r0=r, n_lp=1, n_hp=0,
                                                                dilution=dil, t_begin=0, t_end=T), gam, lp=hp))
                       for r in range(nmax)]
                for N in n_noise:
                    stoch.setdefault((name, N), []).append(np.mean(per[:N], axis=0))
                    res.inversions[(name, N)] = N * factor
            for (n_lp, n_hp) in tsm:
                q = NoiseParams(noise=NOISE_CZ2, seed=cseed + 1, r0=0, n_lp=n_lp, n_hp=n_hp, dilution=tsm_dilution,
                                t_begin=0, t_end=T)
                tsm_rows.setdefault((n_lp, n_hp), []).append(project(lat.loops_stochastic(q, gam, lp=lp_tsm, hp=hp)))
                res.inversions[(n_lp, n_hp)] = (n_lp + n_hp, n_hp)  # (LP solves, HP solves)
    finally:
        lat.close()
    res.exact = np.array(exact)
    res.stochastic = {k: np.array(v) for k, v in stoch.items()}
    res.tsm = {k: np.array(v) for k, v in tsm_rows.items()}
    return res


def table_loops(res: LoopStudyResult):
    """Rows (method, inversions, {pair: relative deviation}) over the ensemble."""
    names = [f"{PAIR_NAMES.get(g, g)} p={tuple(m)}" for g, m in res.pairs]
    rows = []
    for (name, N), v in sorted(res.stochastic.items()):
        rows.append((f"{name} N={N}", res.inversions[(name, N)], dict(zip(names, res.rel_deviation(v)))))
    for (n_lp, n_hp), v in sorted(res.tsm.items()):
        rows.append((f"TSM LP={n_lp} HP={n_hp}", res.inversions[(n_lp, n_hp)],
                     dict(zip(names, res.rel_deviation(v)))))
    return rows


def main(argv=None):
    """Run the comparison on a synthetic ensemble and print one JSON line."""
    import argparse
    import json
    import time

    import synth_inputs as S

    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--dims", type=int, nargs=4, default=[6, 6, 6, 12])
    ap.add_argument("--configs", type=int, default=8)
    ap.add_argument("--eps", type=float, default=0.6)
    ap.add_argument("--kappa", type=float, default=0.155)
    ap.add_argument("--noise", type=int, nargs="+", default=[4, 16, 64])
    ap.add_argument("--tsm", type=int, nargs="+", default=[64, 8, 256, 16], help="pairs n_lp n_hp")
    ap.add_argument("--t", type=int, default=3)
    ap.add_argument("--loops", action="store_true",
                    help="the per-insertion comparison of momentum-projected loops instead of D(t)")
    a = ap.parse_args(argv)
    dims = tuple(a.dims)
    configs = [S.random_links(dims, a.eps, 7000 + c) for c in range(a.configs)]
    t0 = time.perf_counter()
    if a.loops:
        res = run_loops(configs, dims, -1, a.kappa, n_noise=tuple(a.noise), tsm=tuple(zip(a.tsm[::2], a.tsm[1::2])))
        dt = time.perf_counter() - t0
        rows = [{"method": m, "inversions_per_config": inv, "rel_deviation": {k: round(float(x), 5) for k, x in d.items()}}
                for m, inv, d in table_loops(res)]
        print(json.dumps({"lattice": list(dims), "configs": a.configs, "eps": a.eps, "kappa": a.kappa,
                          "seconds": round(dt, 1), "rows": rows}), flush=True)
        return
    res = run(configs, dims, -1, a.kappa, n_noise=tuple(a.noise), tsm=tuple(zip(a.tsm[::2], a.tsm[1::2])))
    dt = time.perf_counter() - t0
    rows = [{"method": m, "inversions_per_config": inv, "D_mean": mu, "D_err": er} for m, inv, mu, er in table(res, a.t)]
    print(json.dumps({"lattice": list(dims), "configs": a.configs, "eps": a.eps, "kappa": a.kappa, "t": a.t,
                      "seconds": round(dt, 1), "rows": rows}), flush=True)


if __name__ == "__main__":
    main()
