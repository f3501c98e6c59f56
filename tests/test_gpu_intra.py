"""GPU parity of the intra-view term (Sec. III-D, Eqs. (2), (3)): adjacency
lists bit-exact against the oracle, weights and per-label costs to FP32
rounding.

Weight tolerance: the GPU keeps segment means in FP32.  A b-bit mean is
below 2^b, so it is within half an FP32 ulp, 2^(b-25), of the exact mean:
2^-17 (7.6e-6) of an 8-bit code value once divided by 2^(b-8).  Six means
enter one L1 distance, which therefore moves by at most 4.6e-5 code values
(plus a few FP32 roundings of the sum); with eps = 1 that bounds the
relative change of beta, so beta and the costs (positive sums of
beta |l - d|) are compared at rtol = 1e-4."""
import json
import os

import numpy as np
import pytest

import oracle
from tests import _problems as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1909_02294_amd import ivde, synth  # noqa: E402

BETA_RTOL = 1e-4


def _case(name):
    print(f"[case] {name}", flush=True)


def _gpu(ns, beta0, capacity=None):
    dv = ivde.DeviceViews(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, ns.chroma_shift)
    off, idx, beta, ws = ivde.adjacency(dv, beta0, 1.0, capacity=capacity)
    torch.cuda.synchronize()
    assert ivde.workspace_status(ws) == ivde.IVDE_OK
    return off, idx, beta


def _oracle(ns, beta0):
    pb = oracle.Problem(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, ns.chroma_shift, 1.0, 3.0, 2, False)
    off, idx = oracle.adjacency(pb)
    _, _, mean = oracle.all_segment_stats(pb)
    return off, idx, oracle.smoothing_beta(mean, off, idx, beta0, ns.bit_depth)


def _compare(ns, beta0, L=7, seed=0):
    off_g, idx_g, beta_g = _gpu(ns, beta0)
    off_o, idx_o, beta_o = _oracle(ns, beta0)
    np.testing.assert_array_equal(off_g.cpu().numpy(), off_o)
    np.testing.assert_array_equal(idx_g.cpu().numpy(), idx_o)
    np.testing.assert_allclose(beta_g.cpu().numpy(), beta_o, rtol=BETA_RTOL)
    rng = np.random.default_rng(seed)
    rows = len(off_o) - 1
    lab = rng.integers(0, L, rows).astype(np.int32)
    fixed = rng.random(rows) < 0.5
    for mask in (None, fixed):
        U_g = ivde.intra_cost(off_g, idx_g, beta_g, torch.from_numpy(lab).cuda(), L,
                              None if mask is None else torch.from_numpy(mask.astype(np.uint8)).cuda())
        U_o = oracle.intra_cost(off_o, idx_o, beta_o, lab, L, fixed=mask)
        np.testing.assert_allclose(U_g.cpu().numpy(), U_o, rtol=BETA_RTOL, atol=1e-6 * max(1.0, np.abs(U_o).max()))
    return off_o, idx_o


def test_hand_case_on_gpu():
    _case("intra hand")
    g = json.load(open(os.path.join(P.GOLDEN, "hand_intra.json")))
    w, h = g["width"], g["height"]
    K = [[5.0, 0, (w - 1) / 2], [0, 5.0, (h - 1) / 2], [0, 0, 1]]
    from types import SimpleNamespace
    planes = []
    for v in g["views"]:
        seg = np.array(v["seg"], np.int32)
        col = np.array(v["colours"], np.float64)
        planes.append([col[seg, k].astype(np.uint8) for k in range(3)])
    ns = SimpleNamespace(cams=[P.cam(K, np.eye(3), [-0.1 * i, 0, 0], w, h) for i in range(2)],
                         Y=[p[0] for p in planes], U=[p[1] for p in planes], V=[p[2] for p in planes],
                         seg=[np.array(v["seg"], np.int32) for v in g["views"]], S=[v["S"] for v in g["views"]],
                         bit_depth=8, chroma_shift=0)
    off, idx, beta = _gpu(ns, g["beta0"])
    off, idx, beta = off.cpu().numpy(), idx.cpu().numpy(), beta.cpu().numpy()
    assert [list(idx[off[r]:off[r + 1]]) for r in range(len(off) - 1)] == g["adjacency"]
    rows = np.repeat(np.arange(len(off) - 1), np.diff(off))
    for s, t, b in zip(rows, idx, beta):
        assert b == pytest.approx(g["beta"][f"{min(s, t)}-{max(s, t)}"], rel=1e-6)
    lab = torch.tensor(g["labelling"], dtype=torch.int32, device="cuda")
    d = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    U = ivde.intra_cost(d(off), d(idx), d(beta), lab, g["labels"]).cpu().numpy()
    np.testing.assert_allclose(U[1], g["U_row1"], rtol=1e-6)
    np.testing.assert_allclose(U[8], g["U_row8"], rtol=1e-6)
    assert np.all(U[9] == 0)
    fixed = np.zeros(len(off) - 1, np.uint8)
    fixed[g["fixed_rows"]] = 1
    Uf = ivde.intra_cost(d(off), d(idx), d(beta), lab, g["labels"], d(fixed)).cpu().numpy()
    np.testing.assert_allclose(Uf[1], g["U_fixed_row1"], rtol=1e-6)
    np.testing.assert_allclose(Uf[8], g["U_fixed_row8"], rtol=1e-6)
    energy = float(U[np.arange(len(off) - 1), g["labelling"]].astype(np.float64).sum())
    assert energy == pytest.approx(g["energy"], rel=1e-6)


@pytest.mark.parametrize("seed,bits,chroma", [(1, 10, 1), (2, 8, 0), (3, 12, 1), (4, 16, 0)])
def test_blocky_maps(seed, bits, chroma):
    _case(f"intra blocky {seed}")
    ns = P.blocky_problem(seed, [(37, 23), (41, 19), (16, 30)], [60, 45, 80], bit_depth=bits, chroma_shift=chroma)
    _compare(ns, 25.0, L=70, seed=seed)


def test_islands_streamed_path():
    """A background segment of ~14000 pixels with a few hundred neighbours
    (islands may cover each other) takes the path that streams the pixel
    records on every extraction."""
    _case("intra islands")
    ns = P.islands_problem(5)
    off, _ = _compare(ns, 12.0, L=5, seed=5)
    assert off[1] - off[0] > 200


@pytest.mark.parametrize("L", [1, 64, 300])
def test_intra_cost_level_counts_and_long_rows(L):
    """Eq. (2) costs with 1, 64 and 300 levels (more label blocks than one
    pass of the kernel holds) on the islands map, whose background row has
    hundreds of entries (several 64-entry chunks)."""
    _case(f"intra cost L={L}")
    ns = P.islands_problem(6)
    _compare(ns, 9.0, L=L, seed=L)


def test_capacity_and_count_only():
    _case("intra capacity")
    ns = P.blocky_problem(9, [(30, 20), (25, 25)], [50, 40])
    off_full, idx_full, beta_full = _gpu(ns, 10.0)
    total = int(off_full[-1].item())
    off0, idx0, _ = _gpu(ns, 10.0, capacity=0)
    assert torch.equal(off0, off_full) and idx0.numel() == 0
    cap = total // 3
    dv = ivde.DeviceViews(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, ns.chroma_shift)
    off, idx, beta, _ = ivde.adjacency(dv, 10.0, 1.0, capacity=cap)
    torch.cuda.synchronize()
    assert torch.equal(off, off_full)
    assert torch.equal(idx, idx_full[:cap]) and torch.equal(beta, beta_full[:cap])


def test_arc_1080p_full_size():
    """8 views of 1920x1080, 20000 segments each: every list exact, every
    weight to FP32 rounding, the costs of 300 seeded rows at 256 labels."""
    _case("intra arc 1080p")
    wl = synth.make_arc_1080p()
    dv = ivde.DeviceViews.from_workload(wl)
    off_g, idx_g, beta_g, ws = ivde.adjacency(dv, 30.0, 1.0)
    torch.cuda.synchronize()
    assert ivde.workspace_status(ws) == ivde.IVDE_OK
    pb = oracle.Problem.from_workload(wl)
    off_o, idx_o = oracle.adjacency(pb)
    np.testing.assert_array_equal(off_g.cpu().numpy(), off_o)
    np.testing.assert_array_equal(idx_g.cpu().numpy(), idx_o)
    _, _, mean = oracle.all_segment_stats(pb)
    beta_o = oracle.smoothing_beta(mean, off_o, idx_o, 30.0, wl.bit_depth)
    rel = np.abs(beta_g.cpu().numpy() - beta_o) / beta_o
    print(f"[arc 1080p] entries {len(beta_o)}, beta max rel err {rel.max():.3g}, mean {rel.mean():.3g}", flush=True)
    np.testing.assert_allclose(beta_g.cpu().numpy(), beta_o, rtol=BETA_RTOL)
    rng = np.random.default_rng(21)
    rows = len(off_o) - 1
    L = wl.num_labels
    lab = rng.integers(0, L, rows).astype(np.int32)
    U_g = ivde.intra_cost(off_g, idx_g, beta_g, torch.from_numpy(lab).cuda(), L).cpu().numpy()
    pick = np.sort(rng.choice(rows, 300, replace=False))
    sub_off = np.concatenate([[0], np.cumsum(off_o[pick + 1] - off_o[pick])])
    sub_idx = np.concatenate([idx_o[off_o[r]:off_o[r + 1]] for r in pick])
    sub_beta = np.concatenate([beta_o[off_o[r]:off_o[r + 1]] for r in pick])
    U_o = oracle.intra_cost(sub_off, sub_idx, sub_beta, lab, L)
    np.testing.assert_allclose(U_g[pick], U_o, rtol=BETA_RTOL, atol=1e-6 * np.abs(U_o).max())
