"""Parity of the host depth optimisation (libivde: ivde_energy_value,
ivde_expansion, ivde_optimize) with the oracle of Eq. (1), Sec. III-B and
Sec. IV-A.  Energies are integers and each move takes the canonical minimum
cut, so labellings, energies and cycle counts must be identical.  Host code
only: these run without a GPU."""
import json
import os

import numpy as np
import pytest

from oracle import graphcut as G
from paper_1909_02294_amd import ivde
from tests import _problems as P


def _both(t):
    w = t.get("unary_weight", 1.0)
    o = G.Energy(t["rows"], t["num_labels"], unary=t["unary"], m=t["m"], hit=t["hit"], K=t["K"],
                 offsets=t["offsets"], index=t["index"], beta=t["beta"], quantum=t["quantum"], fixed=t["fixed"],
                 unary_weight=w)
    h = ivde.Energy(t["rows"], t["num_labels"], unary=t["unary"], m=t["m"], hit=t["hit"], K=t["K"],
                    offsets=t["offsets"], index=t["index"], beta=t["beta"], fixed=t["fixed"], quantum=t["quantum"],
                    unary_weight=w)
    return o, h


def test_hand_energy():
    g = json.load(open(os.path.join(P.GOLDEN, "hand_energy.json")))
    h = ivde.Energy(g["rows"], g["labels"], unary=g["unary"], m=g["m"], hit=g["hit"], K=g["K"],
                    offsets=g["offsets"], index=g["index"], beta=g["beta"], quantum=g["quantum"])
    for c in g["cases"]:
        assert h.value(c["d"]) == c["energy"], c["derivation"]


@pytest.mark.parametrize("seed", range(5))
def test_energy_values(seed):
    t = P.random_energy_terms(seed, rows=30, L=7)
    o, h = _both(t)
    rng = np.random.default_rng(seed)
    for _ in range(5):
        d = rng.integers(0, 7, 30)
        assert h.value(d) == o.energy(d)


@pytest.mark.parametrize("seed,rows,L,opts", [
    (1, 12, 4, {}), (2, 20, 6, {}), (3, 30, 5, {"unary": False}), (4, 24, 8, {"p_hit": 0.9}),
    (5, 16, 5, {"adj": False}), (6, 40, 6, {}), (7, 26, 4, {"quantum": 3.0}),
])
def test_expansion_identical(seed, rows, L, opts):
    t = P.random_energy_terms(seed, rows=rows, L=L, **opts)
    o, h = _both(t)
    rng = np.random.default_rng(seed + 9)
    d0 = rng.integers(0, L, rows)
    labels = list(range(L))
    d_o, e_o, c_o = o.expansion(d0, labels)
    d_h, e_h, c_h = h.expansion(d0, labels)
    np.testing.assert_array_equal(d_h, d_o)
    assert (e_h, c_h) == (e_o, c_o)
    assert e_h == h.value(d_h) <= h.value(d0)


def test_expansion_with_fixed_rows_and_a_label_subset():
    rows, L = 24, 7
    fixed = np.full(rows, -1)
    fixed[[1, 5, 14, 20]] = [3, 0, 6, 2]
    t = P.random_energy_terms(12, rows=rows, L=L, fixed=fixed)
    o, h = _both(t)
    d0 = np.where(fixed >= 0, fixed, 1)
    d_o, e_o, _ = o.expansion(d0, [1, 2, 4, 6])
    d_h, e_h, _ = h.expansion(d0, [6, 1, 4, 2, 4])          # order and repeats do not matter
    np.testing.assert_array_equal(d_h, d_o)
    assert e_h == e_o
    assert np.all(d_h[fixed >= 0] == fixed[fixed >= 0])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8])
@pytest.mark.parametrize("partition", [ivde.PARTITION_BLOCKS, ivde.PARTITION_INTERLEAVED])
def test_optimize_identical(n, partition):
    t = P.random_energy_terms(40 + n, rows=28, L=10)
    o, h = _both(t)
    d_o, e_o = o.optimize(n, partition)
    d_h, e_h = h.optimize(n, partition)
    np.testing.assert_array_equal(d_h, d_o)
    assert e_h == e_o == h.value(d_h)


def test_unary_weight():
    t = P.random_energy_terms(61, rows=30, L=6)
    t["unary_weight"] = 2.75
    o, h = _both(t)
    d_o, e_o = o.optimize(2, ivde.PARTITION_INTERLEAVED)
    d_h, e_h = h.optimize(2, ivde.PARTITION_INTERLEAVED)
    np.testing.assert_array_equal(d_h, d_o)
    assert e_h == e_o
    t1 = dict(t, unary_weight=1.0)
    assert h.value(d_h) != _both(t1)[1].value(d_h)


def test_optimize_larger_instance():
    """200 segments, 16 levels, 4 threads: the Python oracle's
    Edmonds-Karp and the library's search-tree max-flow cut alike."""
    t = P.random_energy_terms(99, rows=200, L=16)
    o, h = _both(t)
    for partition in (ivde.PARTITION_BLOCKS, ivde.PARTITION_INTERLEAVED):
        d_o, e_o = o.optimize(4, partition)
        d_h, e_h = h.optimize(4, partition)
        np.testing.assert_array_equal(d_h, d_o)
        assert e_h == e_o


def test_optimize_is_repeatable_and_thread_timing_free():
    t = P.random_energy_terms(5, rows=3000, L=24, p_hit=0.7)
    h = ivde.Energy(t["rows"], t["num_labels"], unary=t["unary"], m=t["m"], hit=t["hit"], K=t["K"],
                    offsets=t["offsets"], index=t["index"], beta=t["beta"], quantum=t["quantum"])
    runs = [h.optimize(8, ivde.PARTITION_INTERLEAVED) for _ in range(3)]
    for d, e in runs[1:]:
        np.testing.assert_array_equal(d, runs[0][0])
        assert e == runs[0][1]
    d1, e1 = h.optimize(1)
    d0 = np.argmin(t["unary"], axis=1)
    assert e1 <= h.value(d0)


@pytest.mark.parametrize("field,value,msg", [
    ("hit", "bad_hit", "window_hit"), ("beta", "negative", "beta"), ("fixed", "bad_fixed", "fixed"),
])
def test_argument_errors(field, value, msg):
    t = P.random_energy_terms(3, rows=10, L=4)
    if value == "bad_hit":
        t["hit"] = t["hit"].copy()
        t["hit"][2, 0, 1] = 10
    elif value == "negative":
        t["beta"] = t["beta"].copy()
        t["beta"][0] = -1.0
    else:
        t["fixed"] = np.full(10, -1)
        t["fixed"][3] = 4
    _, h = _both(t)
    with pytest.raises(ivde.IvdeError, match=msg):
        h.optimize(1)
