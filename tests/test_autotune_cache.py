"""Autotuner result cache of the binding (host logic only; the GPU side is
in tests/test_gpu_schur.py::test_autotune_cache_hit)."""
import json

import paper_1108_2473_amd as fl


def test_key_names_every_field():
    v = "floop 0.2 (gfx950) src 0123456789abcdef"
    k = fl.tune_key("AMD Instinct MI355X gfx950", (16, 16, 16, 32), fl.PREC_H16, 12, 384, v)
    assert k == "AMD Instinct MI355X gfx950|16x16x16x32|prec3|r12|nrhs384|" + v
    assert k != fl.tune_key("AMD Instinct MI355X gfx950", (16, 16, 16, 32), fl.PREC_F32, 12, 384, v)
    assert k != fl.tune_key("other", (16, 16, 16, 32), fl.PREC_H16, 12, 384, v)
    # a library built from other kernel sources does not reuse the result
    assert k != fl.tune_key("AMD Instinct MI355X gfx950", (16, 16, 16, 32), fl.PREC_H16, 12, 384,
                            "floop 0.2 (gfx950) src fedcba9876543210")


def test_library_version_names_its_kernel_sources():
    from paper_1108_2473_amd import build
    assert fl.version().endswith("src " + build.source_hash()[:16])


def test_store_and_load_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    assert fl.tune_cache_load(path) == {}
    fl.tune_cache_store(path, "a", dict(rt=8, group=1, lds=4, ms=0.85, extra=1))
    fl.tune_cache_store(path, "b", dict(rt=4, group=0, lds=2, ms=1.5))
    d = fl.tune_cache_load(path)
    assert d == {"a": dict(rt=8, group=1, lds=4, ms=0.85), "b": dict(rt=4, group=0, lds=2, ms=1.5)}
    # overwrite one key, keep the other
    fl.tune_cache_store(path, "a", dict(rt=16, group=2, lds=3, ms=0.9))
    assert json.load(open(path))["a"]["rt"] == 16 and fl.tune_cache_load(path)["b"]["lds"] == 2
    assert not [p for p in tmp_path.iterdir() if p.name.endswith(".tmp")]
