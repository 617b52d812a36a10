"""Storage counts the paper prints (tests/golden/paper_storage_counts.json):
the fixture's own arithmetic here, and the library's allocation against it in
test_gpu_memory_matches_paper_counts (GPU)."""
import json
import os

import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_storage_counts.json")


def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def test_fixture_arithmetic():
    g = _golden()
    one = g["flip_flop_arrays"]["one_component"]
    two = g["flip_flop_arrays"]["two_component"]
    assert one["moment_arrays"] == 2 * sum(one["moment_fields"].values())
    assert one["population_arrays"] == 2 * one["q"]
    assert two["moment_arrays"] == one["moment_arrays"] + two["extra_density_arrays"]
    assert two["population_arrays"] == 2 * two["populations_per_component"] == 4 * one["q"]
    s = g["streaming_reads"]
    assert s["accesses"] == s["arrays"] * s["neighbours"] and s["bytes_single_precision"] == 4 * s["accesses"]
    m = g["gpu_memory"]
    assert 0.35 <= 1 - m["without_populations_gb"] / m["with_populations_gb"] <= 0.45


@pytest.mark.gpu
def test_gpu_memory_matches_paper_counts():
    """State memory of the library on a grid without layout padding, in units
    of one FP32 array of N values: moment scheme 2 x 10 (one component) and
    2 x 11 (two components: the mixture density, rho1, j and P, the paper's
    two density arrays counted as rho1 and the mixture); population scheme
    2 x 19 and 2 x 2 x 19 (+ one phase-field array)."""
    torch = pytest.importorskip("torch")
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2301_01622_amd.lbm import LBM
    g = _golden()["flip_flop_arrays"]
    nx, ny, nz = 64, 32, 8
    N = nx * ny * nz
    arrays = {}
    for species in (1, 2):
        for scheme in ("moment", "population"):
            sim = LBM((nx, ny, nz), 19, 0.8, species=species, storage="f32", scheme=scheme)
            state_bytes, _ = sim.memory_info()
            sim.close()
            arrays[(species, scheme)] = state_bytes / (4 * N)
    print(f"[gpu] arrays per node {arrays}", flush=True)
    assert arrays[(1, "moment")] == g["one_component"]["moment_arrays"]
    assert arrays[(1, "population")] == g["one_component"]["population_arrays"]
    assert arrays[(2, "moment")] == g["two_component"]["moment_arrays"]
    assert arrays[(2, "population")] == g["two_component"]["population_arrays"] + 1
    saving = 1 - arrays[(2, "moment")] / arrays[(2, "population")]
    assert 0.35 <= saving <= 0.75
