"""The C-ABI library loads and exports every symbol include/ecmg.h declares, and
its host-only logic (problem validation, memory plan) works without a GPU."""
import os
import re

import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ecmg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ecmg_[a-z_]+)\s*\(", src)) - {"ecmg_host_fn", "ecmg_device_fn"})


@pytest.fixture(scope="module")
def ecmg():
    import paper_1506_02983_amd as E
    return E


def test_library_exports_every_declared_symbol(ecmg):
    L = ecmg.load_library()
    decl = _declared()
    assert decl, "no declarations parsed"
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(ecmg.EXPORTS) == decl


def test_plan_bytes_host_only(ecmg):
    p = workloads.variable_beta_robin_cube(levels=7)
    b = ecmg.plan_bytes(p)
    nodes = 513 ** 3
    assert 60 * nodes < b < 90 * nodes            # ~ 72 B per finest node incl. coarser levels
    assert ecmg.plan_bytes(p, ecmg.MIXED) > b


@pytest.mark.parametrize("mutate, msg", [
    (dict(lo=(1.0, 0, 0), hi=(0.0, 1, 1)), "box"),
    (dict(n0=(0, 4, 4)), "n0"),
    (dict(levels=1), "levels"),
    (dict(face_type=(0, 0, 0, 0, 0, 7)), "face_type"),
    (dict(face_type=(1,) * 6), "singular"),
])
def test_validation_errors(ecmg, mutate, msg):
    p = workloads.paper_problem1(levels=3).with_(**mutate)
    with pytest.raises(ecmg.EcmgError) as e:
        ecmg.plan_bytes(p)
    assert e.value.code == ecmg.EINVAL
    assert msg in str(e.value)


def test_missing_library_fails_loudly(ecmg, tmp_path):
    import importlib
    mod = importlib.import_module("paper_1506_02983_amd")
    saved = mod._lib
    try:
        mod._lib = None
        with pytest.raises(ImportError):
            mod.load_library(str(tmp_path / "nope.so"))
    finally:
        mod._lib = saved
