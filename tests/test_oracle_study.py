"""Pins of the oracle's composition of the paper's comparison of stochastic
methods with the exact loops (Sec. III, figures "compare dilution" and
"truncated"): oracle.dilution_study, which the GPU study is checked against.

Two facts fix what it must return, independently of how it is written:

* With time, spin, colour and cubic dilution on a lattice of 2^3 spatial
  sites every dilution component is supported on ONE site, spin and colour,
  so with unit-modulus noise each diluted estimate of Eq. (loop stochastic)
  is the exact loop Tr[Gamma G(x;x)] (|xi|^2 = 1), for every noise vector,
  and an estimator that is a correctly normalised mean over independent
  products must give exactly the exact D(t).  The truncated solver method
  collapses the same way: the low-precision map is homogeneous in the
  source (Krylov iterates scale with a unit phase of b), so its
  contributions cancel between the two sums and what is left is the
  high-precision (exact) loop.
* Without dilution the estimators of D(t) are unbiased (Sec. II; products of
  independent noise vectors only): over many seeds their mean agrees with
  the exact D(t) within its standard error, while the estimator that keeps
  the r = s products does not.
"""
import numpy as np
import pytest

import oracle as O
import synth_inputs as S

DIMS, BC, KAPPA = (2, 2, 2, 4), -1, 0.12
FULL = O.DIL_TIME | O.DIL_SPIN | O.DIL_COLOUR | O.DIL_CUBIC


@pytest.fixture(scope="module")
def links():
    return S.random_links(DIMS, 0.5, 9100)


@pytest.fixture(scope="module")
def exact_D(links):
    return O.dilution_study([links], DIMS, BC, KAPPA, (2,), {}, (), 7, 1e-13, 1e-2)["exact"][0]


def test_full_dilution_reproduces_the_exact_correlator(links, exact_D):
    """Pair estimator over N = 2, 3 vectors and the TSM (4 LP vectors truncated
    at 1e-2, 2 HP vectors) with single-site dilution equal the exact D(t).
    A divisor N^2 in place of N (N - 1) would be 1/N off, a wrong sign or
    weight of the TSM correction ~1e-2 off (the LP truncation)."""
    r = O.dilution_study([links], DIMS, BC, KAPPA, (2, 3), {"full": FULL}, ((4, 2),), 5, 1e-13, 1e-2,
                         tsm_dilution=FULL)
    scale = np.abs(exact_D).max()
    assert scale > 0
    for key, v in list(r["stochastic"].items()) + list(r["tsm"].items()):
        err = np.abs(v[0] - exact_D).max() / scale
        assert err < 1e-10, (key, err)


def test_estimators_are_unbiased_and_the_diagonal_is_excluded(links, exact_D):
    """300 seeds, undiluted complex Z2 noise: the N = 2 pair estimator and the
    TSM (halves of 1 LP + 1 HP vector) have means within 4.5 standard errors
    of the exact D(t) at every t; the biased estimator that also keeps the
    r = s products, built here from the oracle's per-vector loops of the
    same seeds, is rejected at more than 6 standard errors."""
    nseed, T, Vs = 300, DIMS[3], DIMS[0] * DIMS[1] * DIMS[2]
    r = O.dilution_study([links] * nseed, DIMS, BC, KAPPA, (2,), {"none": 0}, ((2, 2),), 7, 1e-12, 1e-2,
                         with_exact=False)
    assert r["exact"] is None
    for key, v in list(r["stochastic"].items()) + list(r["tsm"].items()):
        z = np.abs(v.mean(axis=0) - exact_D) / (v.std(axis=0, ddof=1) / np.sqrt(nseed))
        assert z.max() < 4.5, (key, z)
    zero = [(0, 0, 0)]
    rows = []
    for c in range(nseed):
        per = [O.momentum_project(O.loops_stochastic(links, DIMS, BC, KAPPA, O.NOISE_CZ2, 7 + 1000 * c, k, 1, 0,
                                                     0, T, [15], tol=1e-12), DIMS, zero) for k in range(2)]
        rows.append(sum(O.disconnected_correlator(per[a], per[b], Vs, [(0, 0)])[0, 0]
                        for a in range(2) for b in range(2)) / 4)
    rows = np.array(rows)
    z = np.abs(rows.mean(axis=0) - exact_D) / (rows.std(axis=0, ddof=1) / np.sqrt(nseed))
    assert z.max() > 6.0, z


# ---------------------------------------------------------------------------
# oracle.loop_error_study: per-insertion momentum-projected loops
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def exact_Lp(links):
    return O.loop_error_study([links], DIMS, BC, KAPPA, (1,), {}, (), 7, 1e-13, 1e-2)["exact"][0]


def test_loop_study_full_dilution_is_exact(links, exact_Lp):
    """Single-site dilution: every stochastic mean (N = 1, 3) and the TSM (3 LP
    vectors at 1e-2, 2 HP) reproduce the exact Lp_Gamma(p, t) of every pair,
    including the nonzero momenta.  A wrong mean normalisation, a missing phase
    or a wrong TSM weight would be off by O(1) or by the LP truncation."""
    r = O.loop_error_study([links], DIMS, BC, KAPPA, (1, 3), {"full": FULL}, ((3, 2),), 5, 1e-13, 1e-2,
                           tsm_dilution=FULL)
    scale = np.abs(exact_Lp).max(axis=1)
    assert (scale > 0).all()
    for key, v in list(r["stochastic"].items()) + list(r["tsm"].items()):
        err = (np.abs(v[0] - exact_Lp).max(axis=1) / scale).max()
        assert err < 1e-10, (key, err)


def test_loop_study_estimates_are_unbiased(links, exact_Lp):
    """300 seeds, undiluted noise: the N = 2 mean and the TSM (2 LP + 1 HP) of
    every (Gamma, p) and t agree with the exact value within 4.5 standard
    errors."""
    nseed = 300
    r = O.loop_error_study([links] * nseed, DIMS, BC, KAPPA, (2,), {"none": 0}, ((2, 1),), 9, 1e-12, 1e-2,
                           with_exact=False)
    for key, v in list(r["stochastic"].items()) + list(r["tsm"].items()):
        for part in (np.real, np.imag):
            se = part(v).std(axis=0, ddof=1) / np.sqrt(nseed)
            dev = np.abs(part(v).mean(axis=0) - part(exact_Lp))
            z = np.where(se > 0, dev / np.where(se > 0, se, 1), 0.0)
            assert z.max() < 4.5, (key, z.max())
