"""The seeded workload generators realise the shapes the benchmarks state:
segment counts, compact ids and the spread of segment sizes."""
import numpy as np
import pytest

from paper_1909_02294_amd import synth


@pytest.mark.parametrize("w,h,n", [(1280, 720, 8900), (320, 240, 1200)])
def test_weighted_jittered_voronoi_log_area_sigma(w, h, n):
    m, S = synth.voronoi(w, h, n, np.random.default_rng(n), 0.207, jittered=True)
    assert m.shape == (h, w) and m.dtype == np.int32
    assert S >= 0.995 * n
    assert np.array_equal(np.unique(m), np.arange(S))
    assert abs(synth.segment_area_sigma(m) - 0.5) < 0.04


def test_uniform_voronoi_is_the_unweighted_default():
    m, S = synth.voronoi(320, 240, 1200, np.random.default_rng(0))
    assert S <= 1200 and np.array_equal(np.unique(m), np.arange(S))
    assert synth.segment_area_sigma(m) > 0.5       # Poisson-Voronoi cells spread more


def test_segment_area_sigma_of_known_areas():
    seg = np.repeat(np.arange(3), [1, 10, 100])
    assert synth.segment_area_sigma(seg) == pytest.approx(np.log(10) * np.sqrt(2.0 / 3.0))
