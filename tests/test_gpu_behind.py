"""GPU parity where level points fall behind a camera, and bilinear sampling
on rectified rigs whose border rows project exactly onto the last row.

The paper's cameras are arbitrarily positioned (Sec. III-A).  On the facing
rig below, the rig-centre reference plane lies partly behind views 2 and 3
(tau <= 0 for a share of their (pixel, level) samples), so the host cannot
prove those views' points to be in front of the source camera and the sweep
runs its general validity test; and a fifth or more of all (pixel, level,
target) samples lie behind the target camera.  Both shares are computed from
FP64 geometry inside the tests.
"""
import numpy as np
import pytest

import oracle
from tests import _problems as P
from tests.gpu_common import compare, run_gpu, run_oracle
from tests.test_oracle_behind import hand_behind_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1909_02294_amd import ivde, synth  # noqa: E402


def _print_case(name):
    print(f"[case] {name}", flush=True)


@pytest.mark.parametrize("sampling", ["nearest", "bilinear"])
def test_hand_facing_cameras(sampling):
    _print_case(f"hand facing cameras {sampling}")
    ns, ref, expected = hand_behind_problem(sampling)
    G, _ = run_gpu(ns, depth_ref=ref)
    # sentinels exact; every other entry to FP32 rounding of the interpolation
    assert np.array_equal(G == 1.0, expected == 1.0)
    np.testing.assert_allclose(G, expected, rtol=0, atol=2e-7)


@pytest.mark.parametrize("ref", ["rig", "own", 0])
@pytest.mark.parametrize("bilinear,bit_depth,chroma_shift", [(True, 10, 1), (False, 8, 0)])
def test_facing_rig_parity(ref, bilinear, bit_depth, chroma_shift):
    _print_case(f"facing rig ref={ref} bilinear={bilinear}")
    ns = P.facing_problem(60, width=96, height=64, n_seg=60, L=48, bit_depth=bit_depth, chroma_shift=chroma_shift,
                          bilinear=bilinear)
    geo = P.behind_geometry(ns, ref)
    assert geo["behind_share"] >= 0.01 and geo["behind_flip_inside"] > 0
    if ref != "own":
        # some view has (pixel, level) samples with tau <= 0: no front-of-camera proof exists for it
        assert max(geo["tau_nonpos"]) >= 0.01
    gref = {"rig": ivde.REF_RIG_CENTER, "own": ivde.REF_OWN}.get(ref, ref)
    oref = {"rig": oracle.REF_RIG_CENTER, "own": oracle.REF_OWN}.get(ref, ref)
    G, _ = run_gpu(ns, depth_ref=gref)
    O = run_oracle(ns, depth_ref=oref)
    compare(G, O, label=f"facing {ref}")
    # entries without any valid target (sentinels) agree entry by entry,
    # except where one sample sits on a rounding or validity boundary
    assert ((G == 1.0) != (O == 1.0)).mean() <= 1e-3
    # both sentinel and matched entries occur
    assert 0.05 < (O == 1.0).mean() < 0.95


@pytest.mark.parametrize("seed", [1, 2])
def test_rectified_bilinear_border_rows(seed):
    """Rectified rig, bilinear: every pixel keeps its row in every target
    (v' = v exactly), so the bottom row samples exactly on row H - 1, the
    edge of the bilinear support.  Entries of segments on that row must
    match the oracle and count the row as valid."""
    _print_case(f"rectified bilinear seed {seed}")
    ns = P.tiny_problem(80 + seed, n_views=3, width=40, height=24, n_seg=24, L=33, bilinear=True, bit_depth=10,
                        chroma_shift=1)
    G, _ = run_gpu(ns)
    pb = oracle.Problem(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, ns.chroma_shift, ns.z_near, ns.z_far,
                        ns.num_labels, True)
    O, m, nv = oracle.cost_volume(pb, with_terms=True)
    compare(G, O, label="rectified bilinear")
    off = pb.row_offsets()
    for c in range(3):
        bottom = np.unique(ns.seg[c][-1])
        top = np.unique(ns.seg[c][0])
        for s in np.concatenate([bottom, top]):
            row = off[c] + s
            assert (nv[row] > 0).any()
            np.testing.assert_allclose(G[row], O[row], rtol=0, atol=1e-5)


def test_rectified_workload_bilinear():
    _print_case("rectified 320x240 bilinear")
    wl = synth.make_rectified_320x240()
    wl.bilinear = True
    G, _ = run_gpu(wl)
    O = run_oracle(wl)
    r = compare(G, O, label="rectified bilinear 320x240")
    assert r["max_err"] <= 1e-5, r
