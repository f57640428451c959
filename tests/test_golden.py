"""Stored values the paper prints for a worked example (tests/golden/), each
file citing its passage, checked against this project's own formulas."""
import os

import pytest

import bench

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    vals = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_bytes_per_cell_and_roofline_match_the_papers_example():
    g = _read("roofline_d3q19_fp64_single_node.txt")
    q, vb = int(g["stencil_q"]), int(g["value_bytes"])
    # one load and one store per population
    assert 2 * q == g["load_stores_per_cell"]
    assert bench.bytes_per_cell(q, vb) == g["bytes_per_cell"]
    pmax = bench.roofline_mlups(g["stream_bandwidth_GBps"] * 1e9, bench.bytes_per_cell(q, vb))
    assert pmax == pytest.approx(g["p_max_MLUPS"], rel=5e-3)
    # the paper's kernel reaches 89% of its bound
    assert g["kernel_measured_MLUPS"] / pmax == pytest.approx(0.892, abs=2e-3)


def test_bytes_per_cell_of_the_storage_forms():
    # FP32 and 16-bit storage of D3Q19, and D3Q27 with a solid flag
    assert bench.bytes_per_cell(19, bench.BYTES["f32"]) == 152
    assert bench.bytes_per_cell(19, bench.BYTES["f16"]) == 76
    assert bench.bytes_per_cell(19, bench.BYTES["bf16"]) == 76
    assert bench.bytes_per_cell(27, bench.BYTES["f32"], mask=True) == 217
    assert bench.roofline_mlups(8e12, 152) == pytest.approx(52631.6, rel=1e-6)
