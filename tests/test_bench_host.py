"""bench.py's host-side bookkeeping (no GPU): the kernel each timing class runs
on a level of each path, the algorithmic bytes of the classes, and the
traffic lookup keyed by those kernel names."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import paper_1506_02983_amd as E  # noqa: E402


def test_kernel_symbol_per_path():
    ks = bench.kernel_symbol
    # JCG init: tiled, column or gather kernel by the level's path
    assert ks(2, E.PATH_TILED, 32, E) == "k_stencil<double, 1, 8, 1, 4>"
    assert ks(2, E.PATH_TILED_UNFOLDED, 32, E) == "k_stencil<double, 1, 8, 1, 4>"
    assert ks(2, E.PATH_COLUMN, 512, E) == "k_col<1, 2, 2, 1>"
    assert ks(2, E.PATH_GATHER, 64, E) == "k_gather_init"
    # pass A: iteration 0 and the later ones
    assert ks(10, E.PATH_COLUMN, 512, E) == "k_col<3, 4, 2, 1>"
    assert ks(10, E.PATH_GATHER, 64, E) == ks(11, E.PATH_GATHER, 64, E) == "k_p_update_fold + k_gather_a"
    assert ks(11, E.PATH_COLUMN, 256, E) == "k_p_update + k_col<3, 4, 2, 1>"
    assert ks(0, E.PATH_TILED, 32, E) == "k_stencil<double, 2, 8, 1, 4>"
    # pass B and its stop-test-only form
    assert ks(1, E.PATH_COLUMN, 512, E) == "k_passB<double, false>"
    assert ks(12, E.PATH_COLUMN, 512, E) == "k_passB<double, true>"
    # EXP_finite: the LDS-staged rows where a fine row holds whole waves of coarse elements
    assert ks(3, E.PATH_COLUMN, 512, E) == "k_exp_finite<true>"
    assert ks(3, E.PATH_GATHER, 64, E) == "k_exp_finite<false>"
    # every class bench.py times has a name
    for k in bench.KIND_NAMES:
        for p in range(8):
            assert ks(k, p, 512, E) != "?", (k, p)


def test_algorithmic_bytes():
    n, e, n1, n0 = 1000, 900, 150, 20
    ab = bench.algorithmic_bytes
    assert ab(0, n, e, n1, n0) == ab(11, n, e, n1, n0) == 8 * (6 * n + e)   # pass A, one launch or two
    assert ab(10, n, e, n1, n0) == 8 * (2 * n + e)
    assert ab(1, n, e, n1, n0) == 32 * n
    assert ab(12, n, e, n1, n0) == 16 * n                                     # stop test only: r, q
    assert ab(2, n, e, n1, n0) == 8 * (4 * n + e)
    assert ab(4, n, e, n1, n0) == 8 * (3 * n + n1)


def test_traffic_lookup(tmp_path, monkeypatch):
    # a summary taken on the current kernel source is used per kernel name and
    # working launch; one taken on another source is not
    prof = tmp_path / "profiles"
    prof.mkdir()
    t = {"kernel_source_hash": bench.kernel_source_hash(),
         "kernels": {"k_col<1, 2, 2, 1>": {"bytes_per_step": 9.0e9, "dispatches": 12}}}
    (prof / "traffic.json").write_text(json.dumps(t))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: t["kernel_source_hash"])
    assert bench.measured_traffic("k_col<1, 2, 2, 1>", 3) == pytest.approx(3.0e9)
    assert bench.measured_traffic("k_gather_init", 3) is None
    t["kernel_source_hash"] = "0" * 16
    (prof / "traffic.json").write_text(json.dumps(t))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "1" * 16)
    assert bench.measured_traffic("k_col<1, 2, 2, 1>", 3) is None
