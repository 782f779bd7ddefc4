"""Host-side run records: per-solve JSON lines and the resumable exact-loop
driver (no GPU: a stand-in lattice returns deterministic arrays)."""
import json

import numpy as np

import paper_1108_2473_amd as fl


def _stats(n):
    return dict(iters=np.arange(n) + 10, updates=np.arange(n) % 3, converged=np.arange(n) % 2 == 0,
                true_resid=np.linspace(1e-13, 9e-13, n), seconds=np.full(n, 0.5))


def test_stats_jsonl_roundtrip(tmp_path):
    p = tmp_path / "m.jsonl"
    fl.append_jsonl(p, fl.stats_records(_stats(3), step=0, lattice="16x16x16x32"))
    fl.append_jsonl(p, fl.stats_records(_stats(2), step=1, lattice="16x16x16x32"))
    rows = [json.loads(l) for l in open(p)]
    assert len(rows) == 5
    assert rows[0] == {"step": 0, "lattice": "16x16x16x32", "solve": 0, "iters": 10, "updates": 0,
                       "converged": True, "true_resid": 1e-13, "seconds": 0.5}
    assert [r["step"] for r in rows] == [0, 0, 0, 1, 1]
    assert rows[4]["solve"] == 1 and rows[4]["converged"] is False


class _FakeLattice:
    def __init__(self, ng, Vs):
        self.ng, self.Vs, self.calls = ng, Vs, []

    def loops_exact(self, t0, gammas, params):
        (t,) = t0
        self.calls.append(t)
        L = np.zeros((len(gammas), 1, self.Vs), complex)
        for g in range(len(gammas)):
            L[g, 0] = t + 1j * g + np.arange(self.Vs)
        return L


def test_checkpointed_loops_resume(tmp_path):
    U = np.ones((4, 16, 3, 3), complex)
    prm = fl.SolverParams(tol=1e-12)
    key = fl.loop_key(U, 0.15, [0, 15], prm)
    lat = _FakeLattice(2, 5)
    L = fl.loops_exact_checkpointed(lat, [0, 3, 7], [0, 15], prm, tmp_path, key)
    assert lat.calls == [0, 3, 7]
    assert L.shape == (2, 3, 5)
    assert np.array_equal(L[1, 2], 7 + 1j + np.arange(5))
    # an interrupted run: one file gone, the others are reused
    (tmp_path / f"{key}_t3.npy").unlink()
    lat2 = _FakeLattice(2, 5)
    L2 = fl.loops_exact_checkpointed(lat2, [0, 3, 7], [0, 15], prm, tmp_path, key)
    assert lat2.calls == [3]
    assert np.array_equal(L, L2)
    assert not list(tmp_path.glob("*.tmp.npy"))


def test_loop_key_names_the_computation():
    U = np.random.default_rng(1).normal(size=(4, 16, 3, 3)) * (1 + 0j)
    prm = fl.SolverParams(tol=1e-12)
    k = fl.loop_key(U, 0.15, [0, 15], prm)
    assert k == fl.loop_key(U.copy(), 0.15, [0, 15], fl.SolverParams(tol=1e-12))
    U2 = U.copy()
    U2[0, 0, 0, 0] += 1e-15
    others = [fl.loop_key(U2, 0.15, [0, 15], prm), fl.loop_key(U, 0.151, [0, 15], prm),
              fl.loop_key(U, 0.15, [0], prm), fl.loop_key(U, 0.15, [0, 15], fl.SolverParams(tol=1e-10)),
              fl.loop_key(U, 0.15, [0, 15], fl.SolverParams(tol=1e-12, inner_prec=fl.PREC_H16))]
    assert len(set(others + [k])) == 6
