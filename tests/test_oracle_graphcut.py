"""Pins of the depth-optimisation oracle (Eq. (1) by alpha-expansion over
segment nodes, Sec. III-B; label-partitioned threads and merging,
Sec. IV-A): a hand-derived energy, Edmonds-Karp against enumerated cuts,
cut moves against enumerated moves, exact optima where alpha-expansion
reaches them (independent segments, two labels), local optimality,
and the merge and partition rules."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import graphcut as G
from tests import _problems as P


def _hand():
    g = json.load(open(os.path.join(P.GOLDEN, "hand_energy.json")))
    E = G.Energy(g["rows"], g["labels"], unary=g["unary"], m=g["m"], hit=g["hit"], K=g["K"],
                 offsets=g["offsets"], index=g["index"], beta=g["beta"], quantum=g["quantum"])
    return g, E


def test_hand_energy():
    g, E = _hand()
    for c in g["cases"]:
        assert E.energy(c["d"]) == c["energy"], c["derivation"]


def test_quantize_rounds_half_away_from_zero():
    np.testing.assert_array_equal(G.quantize([0.375, -0.375, 0.625, -0.625, 0.1], 4.0), [2, -2, 3, -3, 0])


def random_energy(seed, rows=9, L=4, p_hit=0.6, adj=True, unary=True, fixed=None):
    t = P.random_energy_terms(seed, rows, L, p_hit, adj, unary, fixed)
    return G.Energy(t["rows"], t["num_labels"], unary=t["unary"], m=t["m"], hit=t["hit"], K=t["K"],
                    offsets=t["offsets"], index=t["index"], beta=t["beta"], quantum=t["quantum"], fixed=t["fixed"])


@pytest.mark.parametrize("seed", range(6))
def test_edmonds_karp_against_enumerated_cuts(seed):
    rng = np.random.default_rng(seed)
    n = 8
    cap = {}
    for u in range(n):
        for v in range(n):
            if u != v and v != 0 and u != n - 1 and rng.random() < 0.35:
                cap[(u, v)] = int(rng.integers(0, 9))
    best, union = G.min_cut_brute(n, cap, 0, n - 1)
    res = {}
    adj = {}
    for (u, v), c in cap.items():
        res[(u, v)] = res.get((u, v), 0) + c
        res.setdefault((v, u), 0)
    for (u, v) in res:
        adj.setdefault(u, []).append(v)
    assert G.max_flow_edmonds_karp(res, adj, 0, n - 1) == best
    seen, stack = {0}, [0]
    while stack:
        u = stack.pop()
        for v in adj.get(u, []):
            if v not in seen and res[(u, v)] > 0:
                seen.add(v)
                stack.append(v)
    assert set(range(n)) - seen == union


@pytest.mark.parametrize("seed", range(8))
def test_cut_moves_equal_enumerated_moves(seed):
    E = random_energy(seed, rows=10, L=4)
    rng = np.random.default_rng(seed + 50)
    d = rng.integers(0, 4, 10)
    for alpha in range(4):
        sw = E.switchable(d, alpha)
        x_cut = E.best_move(d, alpha, sw)
        x_brute = E.best_move(d, alpha, sw, brute_limit=16)
        np.testing.assert_array_equal(x_cut, x_brute)
        # the move's binary energy is the energy of the labelling it gives
        const, unary, pair = E.move_tables(d, alpha, sw)
        y = np.where(x_cut == 1, alpha, d)
        assert G.Energy._binary_value(x_cut, const, unary, pair) == E.energy(y)


def _all_labellings(rows, L):
    return itertools.product(range(L), repeat=rows)


def test_independent_segments_reach_the_argmin():
    E = random_energy(3, rows=12, L=5, p_hit=0.0, adj=False)
    d, e = E.optimize(1)
    np.testing.assert_array_equal(d, np.argmin(E.U, axis=1))


@pytest.mark.parametrize("seed", range(4))
def test_two_labels_reach_the_global_minimum(seed):
    """With two labels and every segment starting at label 0, the first
    move chooses freely among all labellings: the global minimum."""
    E = random_energy(seed + 10, rows=9, L=2)
    d, e, _ = E.expansion(np.zeros(9, np.int64), [0, 1])
    best = min(E.energy(np.array(x)) for x in _all_labellings(9, 2))
    assert e == best == E.energy(d)


@pytest.mark.parametrize("seed", range(4))
def test_expansion_ends_in_a_local_minimum(seed):
    E = random_energy(seed + 20, rows=8, L=4)
    d, e, cycles = E.expansion(E.initial(range(4)), range(4), max_cycles=20)
    assert cycles < 20
    for alpha in range(4):
        sw = E.switchable(d, alpha)
        x = E.best_move(d, alpha, sw, brute_limit=16)
        assert E.energy(np.where(x == 1, alpha, d)) >= e
    # and never above the start
    assert e <= E.energy(E.initial(range(4)))


def test_fixed_segments_keep_their_labels():
    fixed = np.array([-1, 2, -1, -1, 0, -1, -1, 3, -1])
    E = random_energy(31, rows=9, L=4, fixed=fixed)
    for n in (1, 2, 3):
        d, _ = E.optimize(n)
        assert np.all(d[fixed >= 0] == fixed[fixed >= 0])


def test_partitions():
    assert G.partition_labels(10, 3, G.BLOCKS) == [[0, 1, 2], [3, 4, 5], [6, 7, 8, 9]]
    assert G.partition_labels(10, 3, G.INTERLEAVED) == [[0, 3, 6, 9], [1, 4, 7], [2, 5, 8]]
    assert G.partition_labels(3, 8, G.BLOCKS) == [[0], [1], [2]]
    assert G.partition_labels(5, 1, G.INTERLEAVED) == [[0, 1, 2, 3, 4]]


@pytest.mark.parametrize("seed", range(3))
def test_merge_picks_candidates_and_never_loses(seed):
    E = random_energy(seed + 40, rows=10, L=6)
    A = E.expansion(E.initial([0, 1, 2]), [0, 1, 2])
    B = E.expansion(E.initial([3, 4, 5]), [3, 4, 5])
    d, e, labels = E.merge((A[0], A[1], [0, 1, 2]), (B[0], B[1], [3, 4, 5]))
    assert labels == [0, 1, 2, 3, 4, 5]
    assert np.all((d == A[0]) | (d == B[0]))
    assert e == E.energy(d) <= min(A[1], B[1])


@pytest.mark.parametrize("partition", [G.BLOCKS, G.INTERLEAVED])
def test_threads_follow_the_merge_tree(partition):
    """Four threads: merges (0,1), (2,3), then (0,2); done by hand here."""
    E = random_energy(77, rows=10, L=8)
    subs = G.partition_labels(8, 4, partition)
    res = [E.expansion(E.initial(s), s) for s in subs]
    res = [(d, e, sorted(s)) for (d, e, _), s in zip(res, subs)]
    m01 = E.merge(res[0], res[1])
    m23 = E.merge(res[2], res[3])
    want = E.merge(m01, m23)
    d, e = E.optimize(4, partition)
    np.testing.assert_array_equal(d, want[0])
    assert e == want[1]
