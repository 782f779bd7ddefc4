"""Live kernel timing of the two hops that the benchmark reports
(fl_profile_enable / fl_profile_read): for a CGNR solve both slots see one
launch per iteration chunk step, the end hop's algorithmic bytes count two
more fields per site and right-hand side than H_oe's, and both times are
positive.  BiCGStab fills the same slots."""
import numpy as np
import pytest

import synth_inputs as S

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("solver,fields_end", [(1, 4), (0, 3)])
def test_first_and_end_hop_slots(solver, fields_end):
    import paper_1108_2473_amd as fl
    dims = (8, 8, 8, 8)
    lat = fl.Lattice(dims, -1)
    try:
        lat.set_gauge(S.random_links(dims, 0.4, 41))
        lat.set_kappa(0.12)
        b = S.random_spinors(dims, 4, 5)
        prm = fl.SolverParams(tol=1e-10, solver=solver, inner_prec=fl.PREC_H16)
        print(f"profiling slots, solver {solver}", flush=True)
        for k in (fl.PROF_DSLASH, fl.PROF_DSLASH_END):
            lat.profile_enable(k, True)
        x, info = lat.solve(b, prm)
        first, end = lat.profile_read(fl.PROF_DSLASH), lat.profile_read(fl.PROF_DSLASH_END)
        for k in (fl.PROF_DSLASH, fl.PROF_DSLASH_END):
            lat.profile_enable(k, False)
        assert all(s["converged"] for s in info)
        iters = max(s["iters"] for s in info)
        # one launch of each per iteration of the batch (converged systems are masked, not skipped)
        assert first["launches"] == end["launches"] >= iters
        assert first["ms"] > 0 and end["ms"] > 0
        Vh = int(np.prod(dims)) // 2
        links = 8 * 24 * Vh * first["launches"]
        per_field_first = (first["bytes"] - links) / 2
        per_field_end = (end["bytes"] - links) / fields_end
        assert per_field_first > 0 and abs(per_field_end - per_field_first) <= 1e-9 * per_field_first
    finally:
        lat.close()
