"""GPU parity of the low-precision Schur operator Dhat = 1 - kappa^2 H_eo H_oe
(the operator the mixed-precision solvers iterate with, Sec. III) against the
FP64 oracle, element by element, for every storage format and every LDS mode
of the hopping kernel, including the packed 16-bit integer hop (lds 3, and
4 without neighbour windows).

Tolerance, as a norm-wise relative error |out - ref| / |ref| per right-hand
side, from the storage rounding of each format:
  FP64   1e-13  (rounding order only)
  FP32   1e-5   (vectors and links rounded to 2^-24, a few hundred flops)
  BF16   5e-3   (links rounded to 2^-9 relative; the hop part is about a
                 third of Dhat psi at kappa = 0.2)
  16-bit 1e-3   (each stored vector rounded to 1/32766 of its site's largest
                 component, links to 1/65534 absolute, staged for the packed
                 hop at 1/32767: a few 1e-4 per hop on the hop part)
A dropped or sign-flipped hop direction changes at least 1/8 of the hop
part, about 4e-2 of Dhat psi, far above every tolerance.
"""
import numpy as np
import pytest

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu

KAPPA = 0.2
TOL = {0: 1e-13, 1: 1e-5, 2: 5e-3, 3: 1e-3}
# (precision, link reals, lds mode); -1 is the built-in choice
CASES = [(0, 18, -1), (0, 18, 0), (0, 18, 4), (1, 18, 2), (1, 18, 4), (1, 12, 0), (1, 12, 1), (1, 12, 2),
         (1, 12, 4), (2, 12, 2), (2, 12, 4), (3, 12, 0), (3, 12, 1), (3, 12, 2), (3, 12, 3), (3, 12, 4)]


@pytest.fixture(scope="module")
def F():
    import paper_1108_2473_amd as fl
    fl.lib()  # raises if the HIP library is missing: no fallback
    return fl


_LATS = {}


def lattice(F, dims):
    if dims not in _LATS:
        U = S.random_links(dims, 0.5, 1100 + sum(dims))
        lat = F.Lattice(dims, -1)
        lat.set_gauge(U)
        lat.set_kappa(KAPPA)
        _LATS[dims] = (lat, U)
    return _LATS[dims]


def even_mask(dims):
    x = np.indices(dims[::-1]).reshape(4, -1)[::-1]  # canonical order, x fastest
    return (x.sum(axis=0) % 2) == 0


# (6, 4, 4, 6): Vh = 288, a ragged last wave; 3 right-hand sides: a partial
# workgroup of right-hand sides; (2, 2, 2, 4): extents of 2, where the
# forward and backward neighbour of a direction are the same site (both
# hops add), and a single partial wave
@pytest.mark.parametrize("dims", [(4, 4, 4, 8), (6, 4, 4, 6), (2, 2, 2, 4)])
@pytest.mark.parametrize("prec,reals,lds", CASES)
@pytest.mark.parametrize("dagger", [False, True])
def test_schur_operator(F, dims, prec, reals, lds, dagger):
    lat, U = lattice(F, dims)
    psi = S.random_spinors(dims, 3, 77)
    lat.set_tile(prec=prec, gauge_reals=reals, rt=0, group=0, lds=lds)
    try:
        got = lat.apply_schur(psi, F.SolverParams(inner_prec=prec, gauge_reals=reals), dagger=dagger)
    finally:
        lat.set_tile(prec=prec, gauge_reals=reals, rt=0, group=0, lds=-1)
    ev = even_mask(dims)
    V = int(np.prod(dims))
    for k in range(psi.shape[0]):
        ref = O.apply_Dhat(U, psi[k], dims, -1, KAPPA, dagger=dagger).reshape(V, 12)
        g = got[k].reshape(V, 12)
        assert np.all(g[~ev] == 0)
        err = np.linalg.norm(g[ev] - ref[ev]) / np.linalg.norm(ref[ev])
        assert err <= TOL[prec], (k, err)


def test_packed_hop_matches_float_hop(F):
    """lds 3 (exact integer products with half-scale links) and lds 2 (FP32
    arithmetic on the same 16-bit storage) differ only by the link re-rounding
    and the rounding of FP32 products: their difference is well inside the
    16-bit tolerance."""
    dims = (4, 4, 4, 8)
    lat, U = lattice(F, dims)
    psi = S.random_spinors(dims, 2, 78)
    out = {}
    for lds in (2, 3):
        lat.set_tile(prec=3, gauge_reals=12, rt=0, group=0, lds=lds)
        try:
            out[lds] = lat.apply_schur(psi, F.SolverParams(inner_prec=3, gauge_reals=12))
        finally:
            lat.set_tile(prec=3, gauge_reals=12, rt=0, group=0, lds=-1)
    d = np.linalg.norm(out[3] - out[2]) / np.linalg.norm(out[2])
    assert 0 < d <= 1e-3


def test_schur_rejects_bad_lds(F):
    lat, _ = lattice(F, (4, 4, 4, 8))
    with pytest.raises(F.FloopError):
        lat.set_tile(prec=1, gauge_reals=12, rt=0, group=0, lds=3)
    with pytest.raises(F.FloopError):
        lat.set_tile(prec=3, gauge_reals=12, rt=0, group=0, lds=5)


@pytest.mark.parametrize("lds", [3, 4])
def test_solver_with_16_waves_per_workgroup(F, lds):
    """16 right-hand sides per workgroup in the 16-bit iteration: the FP64
    reliable-update launches of the same solve must keep their own shape
    (at most 8 waves, the FP64 kernels' limit); the solve meets the FP64
    stopping rule |D x - b| <= tol |b|."""
    dims = (4, 4, 4, 8)
    lat, U = lattice(F, dims)
    b = S.random_spinors(dims, 16, 79)
    lat.set_tile(prec=3, gauge_reals=12, rt=16, group=0, lds=lds)
    try:
        x, info = lat.solve(b, F.SolverParams(tol=1e-10, inner_prec=3, gauge_reals=12, solver=F.SOLVER_CGNR))
    finally:
        lat.set_tile(prec=3, gauge_reals=12, rt=0, group=0, lds=-1)
    assert all(i["converged"] and i["true_resid"] <= 1e-10 for i in info), info
    r = O.apply_D(U, x[3], dims, -1, KAPPA) - b[3]
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b[3]) * 1.01


def test_autotune_cache_hit(F, tmp_path):
    """A first autotune call times and stores its result; a second call with
    the same key applies the stored shape without timing."""
    lat, U = lattice(F, (4, 4, 4, 8))
    path = str(tmp_path / "tune.json")
    try:
        first = lat.autotune(prec=3, gauge_reals=12, nrhs=8, cache=path)
        second = lat.autotune(prec=3, gauge_reals=12, nrhs=8, cache=path)
    finally:
        lat.set_tile(prec=3, gauge_reals=12, rt=0, group=0, lds=-1)
    assert not first["cached"] and second["cached"]
    assert (first["rt"], first["group"], first["lds"]) == (second["rt"], second["group"], second["lds"])
    assert first["lds"] in range(0, 5) and first["ms"] > 0
    assert len(F.tune_cache_load(path)) == 1


@pytest.mark.parametrize("prec,solver", [(3, 1), (1, 0), (1, 1)], ids=["h16 cgnr", "f32 bicgstab", "f32 cgnr"])
def test_workgroup_shape_does_not_change_any_bit(F, prec, solver):
    """Regression for the store discipline of every kernel: a batch of point
    and random sources with two zero sources among them, so that some systems
    are masked out of the launches while the others iterate, solved with 4, 8 and 16
    right-hand sides per workgroup gives bit-identical solutions and
    statistics (per-system recurrences; reductions over fixed 64-site
    blocks; a store overwritten by later vector work would differ)."""
    dims = (4, 4, 4, 8)
    U = S.random_links(dims, 0.5, 1180)
    lat = F.Lattice(dims, -1)  # its own lattice at kappa 0.13, below the critical value
    lat.set_gauge(U)
    lat.set_kappa(0.13)
    V = S.volume(dims)
    b = S.random_spinors(dims, 24, 81)
    for k in range(0, 24, 3):  # every third source a point source
        b[k] = 0
        b[k, (37 * k) % V, k % 4, k % 3] = 1.0
    b[1] = 0  # two zero sources: masked out of every launch from the start
    b[13] = 0
    prm = F.SolverParams(tol=1e-11, inner_prec=prec, gauge_reals=12, solver=solver)
    out = {}
    try:
        for rt in (4, 8, 16):
            lat.set_tile(prec=prec, gauge_reals=12, rt=rt, group=0, lds=-1)
            x, info = lat.solve(b, prm)
            assert all(i["converged"] for i in info), (rt, info)
            out[rt] = (x, [(i["iters"], i["updates"], i["true_resid"]) for i in info])
    finally:
        lat.close()
    its = [s[0] for s in out[4][1]]
    assert its[1] == its[13] == 0 and min(its[k] for k in range(24) if k not in (1, 13)) > 0
    for rt in (8, 16):
        assert np.array_equal(out[rt][0], out[4][0]), rt
        assert out[rt][1] == out[4][1], rt
