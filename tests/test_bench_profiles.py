"""bench.py's roofline `traffic` comes from the committed HBM-counter summary
only while that summary was taken on the same part-2 kernel instance and on
the current kernel sources (CPU only: reads files, runs nothing on a GPU)."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_matches_the_profiled_instance():
    b = _bench()
    t = b.traffic_from_profiles("k_stencil<0, 4, 32>")
    if t is None:
        pytest.skip("the counter summary predates the current kernel sources")
    assert t > 0
    # the algorithmic bytes of one 1920x1080 launch, and the measured bytes near them
    alg = b.FUSED_BYTES_PER_PX * 1920 * 1080
    assert 0.5 * alg < t < 2.0 * alg


def test_traffic_refused_for_another_instance():
    b = _bench()
    assert b.traffic_from_profiles("k_stencil<0, 4, 16>") is None
    assert b.traffic_from_profiles("k_stencil<0, 7, 32>") is None
