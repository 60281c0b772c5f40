"""Host side of the autotuner: the JSON tuning cache is read by the library
without a device (ecmg_tune_lookup), with the documented schema, and rejects
files that are not tuning caches."""
import json

import pytest


@pytest.fixture(scope="module")
def ecmg():
    import paper_1506_02983_amd as E
    E.load_library()
    return E


def _write(path, obj):
    with open(path, "w") as fh:
        if isinstance(obj, str):
            fh.write(obj)
        else:
            json.dump(obj, fh)


def test_lookup_entries(ecmg, tmp_path):
    path = str(tmp_path / "tune.json")
    _write(path, {"format": "ecmg-tune-1", "device": "gfx950 256 CUs", "levels": {
        "fp64 128x128x128": {"path": "tiled", "kz": 8, "seg": 0, "nwg": 0, "us_default": 61.5, "us_best": 53.25},
        "fp64 64x64x64": {"path": "persistent", "kz": 0, "seg": 4, "nwg": 128, "us_default": 41.0, "us_best": 39.5},
        "mixed 128x128x128": {"path": "tiled", "kz": 16, "seg": 0, "nwg": 0, "us_default": 40.0, "us_best": 35.0},
        "fp64 64x32x32": {"path": "gather", "kz": 0, "seg": 0, "nwg": 0, "us_default": 12.0, "us_best": 10.5},
        "fp64 32x32x32": {"path": "tiled", "kz": 0}}})           # no usable choice: ignored
    r = ecmg.tune_lookup(path, (128, 128, 128))
    assert r["path"] == "tiled" and r["kz"] == 8 and r["us_best"] == 53.25 and r["level"] == -1
    r = ecmg.tune_lookup(path, (64, 64, 64))
    assert r["path"] == "persistent" and (r["seg"], r["nwg"]) == (4, 128)
    assert ecmg.tune_lookup(path, (128, 128, 128), precision=ecmg.MIXED)["kz"] == 16
    assert ecmg.tune_lookup(path, (64, 32, 32))["path"] == "gather"
    assert ecmg.tune_lookup(path, (32, 32, 32)) is None
    assert ecmg.tune_lookup(path, (16, 16, 16)) is None
    assert ecmg.tune_lookup(str(tmp_path / "missing.json"), (128, 128, 128)) is None


@pytest.mark.parametrize("text", ["[1, 2]", "{\"format\": \"other\"}", "{\"format\": \"ecmg-tune-1\", ",
                                  "not json at all"])
def test_lookup_rejects_non_cache(ecmg, tmp_path, text):
    path = str(tmp_path / "bad.json")
    _write(path, text)
    with pytest.raises(ecmg.EcmgError) as e:
        ecmg.tune_lookup(path, (8, 8, 8))
    assert e.value.code == ecmg.EINVAL


def test_batch_entry_is_kept_apart_from_levels(ecmg, tmp_path):
    """A cache holding the batched solve's entry ("batch fp64", path "batch")
    still serves level lookups, and the batch entry is not taken for a level."""
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"format": "ecmg-tune-1", "device": "x", "levels": {
        "fp64 64x64x64": {"path": "tiled", "kz": 4, "seg": 0, "nwg": 0, "us_default": 2.0, "us_best": 1.0},
        "batch fp64": {"path": "batch", "kz": 0, "seg": 2, "nwg": 4096, "us_default": 9.0, "us_best": 8.0}}}))
    r = ecmg.tune_lookup(str(path), (64, 64, 64))
    assert r["path"] == "tiled" and r["kz"] == 4
    assert ecmg.tune_lookup(str(path), (8, 8, 8)) is None
