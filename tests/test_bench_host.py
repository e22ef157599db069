"""Host-side checks of bench.py's inputs (no GPU): the committed rocprofv3 traffic summaries
carry the bitmap kernel's counted bytes for the intersection source as it stands, so the
bench line's roofline has a non-null traffic figure."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("workload", ["rmat24", "rmat20"])
def test_traffic_summary_matches_the_intersection_source(workload):
    t = _bench().counted_traffic("k_isect_bitmap", workload)
    assert t is not None, f"profiles/traffic_{workload}.md is missing or was taken on another isect.hip"
    assert t > 1e9
