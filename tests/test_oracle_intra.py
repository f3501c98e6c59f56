"""Pins of the oracle's intra-view term (Sec. III-D, Eqs. (2), (3), and the
intra-view double sum of Eq. (1)): a hand-derived case, the pure-Python
brute force, closed forms on stripe and block segmentations, and the
identities that tie the per-label costs to the energy."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from tests import _problems as P


def _hand():
    g = json.load(open(os.path.join(P.GOLDEN, "hand_intra.json")))
    w, h = g["width"], g["height"]
    K = [[5.0, 0, (w - 1) / 2], [0, 5.0, (h - 1) / 2], [0, 0, 1]]
    cams = [P.cam(K, np.eye(3), [-0.1 * i, 0, 0], w, h) for i in range(2)]
    planes = []
    for v in g["views"]:
        seg = np.array(v["seg"], np.int32)
        col = np.array(v["colours"], np.float64)
        planes.append([col[seg, k].astype(np.uint8) for k in range(3)])
    pb = oracle.Problem(cams, [p[0] for p in planes], [p[1] for p in planes], [p[2] for p in planes],
                        [np.array(v["seg"], np.int32) for v in g["views"]], [v["S"] for v in g["views"]],
                        8, 0, 1.0, 4.0, g["labels"], False)
    return g, pb


def _csr_lists(offsets, index):
    return [list(index[offsets[r]:offsets[r + 1]]) for r in range(len(offsets) - 1)]


def test_hand_derived_intra_term():
    g, pb = _hand()
    off, idx = oracle.adjacency(pb)
    assert _csr_lists(off, idx) == g["adjacency"]
    _, _, mean = oracle.all_segment_stats(pb)
    beta = oracle.smoothing_beta(mean, off, idx, g["beta0"], 8)
    rows = oracle.edge_rows(off)
    for s, t, b in zip(rows, idx, beta):
        key = f"{min(s, t)}-{max(s, t)}"
        assert b == pytest.approx(g["beta"][key], rel=1e-14), key
    lab = np.array(g["labelling"])
    U = oracle.intra_cost(off, idx, beta, lab, g["labels"])
    np.testing.assert_allclose(U[1], g["U_row1"], rtol=1e-14)
    np.testing.assert_allclose(U[8], g["U_row8"], rtol=1e-14)
    assert np.all(U[9] == 0)                        # the empty segment has no neighbours
    fixed = np.zeros(len(lab), bool)
    fixed[g["fixed_rows"]] = True
    Uf = oracle.intra_cost(off, idx, beta, lab, g["labels"], fixed=fixed)
    np.testing.assert_allclose(Uf[1], g["U_fixed_row1"], rtol=1e-14)
    np.testing.assert_allclose(Uf[8], g["U_fixed_row8"], rtol=1e-14)
    assert np.all(Uf[0] == 0)
    assert oracle.intra_energy(off, idx, beta, lab) == pytest.approx(g["energy"], rel=1e-14)


def _blocky_problem(seed, sizes, n_ids):
    ns = P.blocky_problem(seed, sizes, n_ids)
    return oracle.Problem(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, ns.chroma_shift, 1.0, 3.0, 6,
                          False)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_adjacency_and_terms_match_brute_force(seed):
    pb = _blocky_problem(seed, [(9, 7), (11, 5), (6, 8)], [12, 9, 20])
    off, idx = oracle.adjacency(pb)
    sets = brute.adjacency_sets(pb.seg, pb.S)
    row0 = pb.row_offsets()
    for v in range(pb.n_views):
        for s in range(pb.S[v]):
            want = sorted(row0[v] + t for (_, t) in sets[(v, s)])
            r = row0[v] + s
            assert list(idx[off[r]:off[r + 1]]) == want
    _, _, mean = oracle.all_segment_stats(pb)
    rng = np.random.default_rng(seed + 100)
    lab = rng.integers(0, 6, int(row0[-1]))
    beta = oracle.smoothing_beta(mean, off, idx, 25.0, 10)
    bb, Ub, Eb = brute.intra_terms(pb.seg, pb.S, mean.tolist(), 25.0, 10, lab.tolist(), 6)
    for s, t, b in zip(oracle.edge_rows(off), idx, beta):
        assert b == pytest.approx(bb[(s, t)], rel=1e-13)
    assert len(bb) == len(idx)
    np.testing.assert_allclose(oracle.intra_cost(off, idx, beta, lab, 6), np.array(Ub), rtol=1e-13, atol=1e-12)
    assert oracle.intra_energy(off, idx, beta, lab) == pytest.approx(Eb, rel=1e-13)


def _problem_from_maps(maps, n_labels=4):
    cams, Y = [], []
    for i, m in enumerate(maps):
        h, w = m.shape
        K = [[6.0, 0, (w - 1) / 2], [0, 6.0, (h - 1) / 2], [0, 0, 1]]
        cams.append(P.cam(K, np.eye(3), [-0.05 * i, 0, 0], w, h))
        Y.append(np.full((h, w), 100, np.uint8))
    return oracle.Problem(cams, Y, Y, Y, [m.astype(np.int32) for m in maps], [int(m.max()) + 1 for m in maps],
                          8, 0, 1.0, 3.0, n_labels, False)


def test_closed_forms_on_regular_segmentations():
    # vertical stripes of width 3: a path graph
    stripes = np.repeat(np.arange(5), 3)[None, :].repeat(4, axis=0)
    # horizontal stripes of height 2
    hstripes = np.repeat(np.arange(4), 2)[:, None].repeat(7, axis=1)
    # 3 x 4 grid of 2 x 2 blocks: the 4-neighbour grid graph, no diagonals
    blocks = np.kron(np.arange(12).reshape(3, 4), np.ones((2, 2), np.int64))
    # one segment per pixel: the pixel grid graph
    pixels = np.arange(20).reshape(4, 5)
    single = np.zeros((3, 5), np.int64)
    pb = _problem_from_maps([stripes, hstripes, blocks, pixels, single])
    off, idx = oracle.adjacency(pb)
    lists = _csr_lists(off, idx)
    row0 = pb.row_offsets()

    def local(v):
        return [[t - row0[v] for t in lists[row0[v] + s]] for s in range(pb.S[v])]

    def path(n):
        return [[j for j in (i - 1, i + 1) if 0 <= j < n] for i in range(n)]

    def grid(r, c):
        return [sorted(j * c + i for j, i in ((y - 1, x), (y + 1, x), (y, x - 1), (y, x + 1))
                       if 0 <= j < r and 0 <= i < c) for y in range(r) for x in range(c)]

    assert local(0) == path(5)
    assert local(1) == path(4)
    assert local(2) == grid(3, 4)
    assert local(3) == grid(4, 5)
    assert local(4) == [[]]
    # the number of adjacent ordered pairs in an r x c grid graph
    assert off[row0[3] + 20] - off[row0[3]] == 2 * (4 * 4 + 3 * 5)


def test_identities_between_costs_and_energy():
    ns = P.tiny_problem(71, n_views=3, width=23, height=15, n_seg=18, L=9, chroma_shift=1, bit_depth=10)
    pb = oracle.Problem(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, 10, 1, ns.z_near, ns.z_far, 9, False)
    off, idx = oracle.adjacency(pb)
    rows = oracle.edge_rows(off)
    # symmetric, no self loops, increasing lists
    pairs = set(zip(rows.tolist(), idx.tolist()))
    assert all((t, s) in pairs for s, t in pairs)
    assert not any(s == t for s, t in pairs)
    assert all(np.all(np.diff(idx[off[r]:off[r + 1]]) > 0) for r in range(len(off) - 1))
    _, _, mean = oracle.all_segment_stats(pb)
    beta = oracle.smoothing_beta(mean, off, idx, 30.0, 10)
    bmap = dict(zip(zip(rows.tolist(), idx.tolist()), beta.tolist()))
    assert all(bmap[(s, t)] == bmap[(t, s)] for s, t in pairs)
    assert np.all(beta > 0) and np.all(beta <= 30.0)
    rng = np.random.default_rng(5)
    lab = rng.integers(0, 9, len(off) - 1)
    U = oracle.intra_cost(off, idx, beta, lab, 9)
    E = oracle.intra_energy(off, idx, beta, lab)
    assert E == pytest.approx(U[np.arange(len(lab)), lab].sum(), rel=1e-12)
    assert oracle.intra_energy(off, idx, beta, np.full_like(lab, 4)) == 0.0
    # shifting every label by one keeps the energy and shifts the costs
    assert oracle.intra_energy(off, idx, beta, lab + 1) == pytest.approx(E, rel=1e-12)
    U1 = oracle.intra_cost(off, idx, beta, lab + 1, 10)
    np.testing.assert_allclose(U1[:, 1:], U, rtol=1e-12, atol=1e-12)
    # the mask: all fixed is the plain cost, none fixed is zero, and the
    # costs from two complementary masks add up
    allf = np.ones(len(lab), bool)
    np.testing.assert_array_equal(oracle.intra_cost(off, idx, beta, lab, 9, fixed=allf), U)
    assert np.all(oracle.intra_cost(off, idx, beta, lab, 9, fixed=~allf) == 0)
    m = rng.random(len(lab)) < 0.4
    np.testing.assert_allclose(oracle.intra_cost(off, idx, beta, lab, 9, fixed=m) +
                               oracle.intra_cost(off, idx, beta, lab, 9, fixed=~m), U, rtol=1e-12, atol=1e-12)
    # each U row is convex in the label (a sum of weighted absolute values)
    assert np.all(np.diff(U, 2, axis=1) >= -1e-9)


def test_islands_match_brute_force():
    """A segment with hundreds of pixels and hundreds of neighbours."""
    ns = P.islands_problem(3, width=40, height=30, n_islands=60)
    pb = oracle.Problem(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, 8, 0, 1.0, 3.0, 6, False)
    off, idx = oracle.adjacency(pb)
    sets = brute.adjacency_sets(pb.seg, pb.S)
    row0 = pb.row_offsets()
    for v in range(2):
        for s in range(pb.S[v]):
            r = row0[v] + s
            assert list(idx[off[r]:off[r + 1]]) == sorted(row0[v] + t for (_, t) in sets[(v, s)])
    assert off[1] - off[0] > 40


def test_beta_units_and_eps():
    """Identical means give beta0 / eps; a difference of 2^(b-8) code values
    in one component is one 8-bit code value."""
    mean = np.array([[400.0, 512, 512, 0], [400.0, 512, 512, 0], [404.0, 512, 512, 0], [400.0, 508, 516, 0]])
    off = np.array([0, 3, 4, 5, 6])
    idx = np.array([1, 2, 3, 0, 0, 0])
    b = oracle.smoothing_beta(mean, off, idx, 12.0, 10)
    np.testing.assert_allclose(b, [12.0, 12.0 / 2.0, 12.0 / 3.0, 12.0, 6.0, 4.0], rtol=1e-15)
    b8 = oracle.smoothing_beta(mean, off, idx, 12.0, 8)
    np.testing.assert_allclose(b8, [12.0, 12.0 / 5.0, 12.0 / 9.0, 12.0, 12.0 / 5.0, 12.0 / 9.0], rtol=1e-15)
