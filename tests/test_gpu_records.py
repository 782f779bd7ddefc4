"""Run records on the GPU: the resumable timeslice-by-timeslice driver of
the exact loops returns what one call per timeslice returns, bit for bit,
also when it resumes from saved timeslices, and agrees with one call over
all of them to the solver tolerance (the batch decides when the host checks
the solves, so iterates differ by rounding); the per-solve JSON lines of a
solving call match its statistics."""
import json

import numpy as np
import pytest

import synth_inputs as S

pytestmark = pytest.mark.gpu


def test_checkpointed_exact_loops_match_one_call(tmp_path):
    import paper_1108_2473_amd as fl
    dims = (4, 4, 4, 4)
    U = S.random_links(dims, 0.4, 31)
    lat = fl.Lattice(dims, -1)
    try:
        lat.set_gauge(U)
        lat.set_kappa(0.12)
        prm = fl.SolverParams(tol=1e-12, solver=fl.SOLVER_CGNR, inner_prec=fl.PREC_H16)
        gam = [0, 15, 8]
        print("checkpointed exact loops 4^4, timeslices 0 2 3", flush=True)
        one = lat.loops_exact([0, 2, 3], gam, prm)
        ref = np.stack([lat.loops_exact([t], gam, prm)[:, 0] for t in (0, 2, 3)], axis=1)
        scale = np.abs(one).max()
        assert np.abs(ref - one).max() <= 1e-10 * scale
        key = fl.loop_key(U, 0.12, gam, prm)
        L1 = fl.loops_exact_checkpointed(lat, [0, 2, 3], gam, prm, tmp_path, key)
        assert np.array_equal(L1, ref)
        (tmp_path / f"{key}_t2.npy").unlink()
        L2 = fl.loops_exact_checkpointed(lat, [0, 2, 3], gam, prm, tmp_path, key)
        assert np.array_equal(L2, ref)
        st = lat.last_stats()  # the one timeslice solved again
        assert len(st["iters"]) == 12 * 64 and st["converged"].all()
        p = tmp_path / "solves.jsonl"
        fl.append_jsonl(p, fl.stats_records(st, timeslice=2))
        rows = [json.loads(l) for l in open(p)]
        assert len(rows) == 12 * 64
        assert all(r["converged"] and r["true_resid"] <= 1e-12 and r["timeslice"] == 2 for r in rows)
        assert [r["iters"] for r in rows] == [int(v) for v in st["iters"]]
    finally:
        lat.close()
