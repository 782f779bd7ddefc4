"""Live kernel timing of the three iteration kernels that the benchmark
reports (fl_profile_enable / fl_profile_read): for a CGNR solve every slot
sees one launch per iteration, the end hop's algorithmic bytes count two
more fields per site and right-hand side than H_oe's, the vector update's
five fields and no links, and all times are positive.  BiCGStab fills the
same slots (its end hop three fields, its update seven)."""
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
        slots = (fl.PROF_DSLASH, fl.PROF_DSLASH_END, fl.PROF_BLAS_UPDATE)
        for k in slots:
            lat.profile_enable(k, True)
        x, info = lat.solve(b, prm)
        first, end, upd = (lat.profile_read(k) for k in slots)
        for k in slots:
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
        # the vector update: one launch per iteration, no links, 5 (CGNR) or 7 (BiCGStab) fields
        assert upd["launches"] == first["launches"] and upd["ms"] > 0
        per_field_upd = upd["bytes"] / (5 if solver == 1 else 7)
        assert abs(per_field_upd - per_field_first) <= 1e-9 * per_field_first
    finally:
        lat.close()
