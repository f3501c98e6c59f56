"""Depth maps end to end: painting (Sec. III-B) against the oracle, and the
whole chain -- GPU terms, host alpha-expansion (Sec. III-B, IV-A), GPU
painting -- on a rendered arc rig, checked against the scene's ground
truth (a sanity bar, not parity: the optimiser's inputs come from the GPU,
and its parity with the oracle is tested on the CPU)."""
import numpy as np
import pytest

import oracle
from tests import _problems as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1909_02294_amd import ivde, pipeline, synth  # noqa: E402


def _case(name):
    print(f"[case] {name}", flush=True)


@pytest.mark.parametrize("L", [1, 7, 256])
def test_depth_map_matches_oracle(L):
    _case(f"depth map L={L}")
    ns = P.tiny_problem(8, n_views=3, width=37, height=21, n_seg=30, L=L)
    dv = ivde.DeviceViews(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, ns.chroma_shift)
    lr = ivde.label_range(ns.z_near, ns.z_far, L)
    lab = np.random.default_rng(L).integers(0, L, dv.rows).astype(np.int32)
    got = ivde.depth_map(dv, lr, lab).cpu().numpy()
    pb = oracle.Problem(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, 8, 0, ns.z_near, ns.z_far, L, False)
    np.testing.assert_array_equal(got, oracle.depth_map(pb, lab).astype(np.float32))


def test_depth_map_marks_bad_levels():
    _case("depth map bad levels")
    ns = P.tiny_problem(9, n_views=2, width=20, height=12, n_seg=10, L=5)
    dv = ivde.DeviceViews(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, ns.chroma_shift)
    lab = np.zeros(dv.rows, np.int32)
    lab[3] = 5
    lab[4] = -1
    D = ivde.depth_map(dv, ivde.label_range(ns.z_near, ns.z_far, 5), lab).cpu().numpy()[:240].reshape(12, 20)
    bad = np.isin(ns.seg[0], [3, 4])
    assert np.all(np.isnan(D[bad])) and np.all(D[~bad] == np.float32(ns.z_far))


def _quality(labels, truth, tol=2):
    return float(np.mean(np.abs(labels.astype(np.int64) - truth) <= tol))


def test_pipeline_small_arc():
    """Cost volume as the unary term, window and intra-view terms: the cut
    never ends above the winner-take-all labelling it starts from (one
    thread), the depth map paints its labels, and most segments land within
    two levels of the ground truth."""
    _case("pipeline small arc")
    wl = synth.make_small_arc(seed=71, n_views=4, width=192, height=108, n_segments=200, num_labels=48)
    dv = ivde.DeviceViews.from_workload(wl)
    lr = ivde.label_range(wl.z_near, wl.z_far, wl.num_labels)
    res = pipeline.estimate_depth(dv, lr, n_threads=1, max_cycles=4)
    E = res["energy_obj"]
    wta = ivde.argmin(res["cost"]).cpu().numpy()
    assert res["energy"] == E.value(res["labels"]) <= E.value(wta)
    pb = oracle.Problem.from_workload(wl)
    np.testing.assert_array_equal(res["depth"].cpu().numpy(), oracle.depth_map(pb, res["labels"]).astype(np.float32))
    truth = synth.truth_labels(wl)
    q_cut, q_wta = _quality(res["labels"], truth), _quality(wta, truth)
    print(f"[pipeline] within 2 levels: cut {q_cut:.3f}, winner-take-all {q_wta:.3f}; times {res['times']}",
          flush=True)
    assert q_cut >= 0.75


def test_pipeline_paper_energy_threads():
    """The paper's own energy (window and intra-view terms, no unary), with
    4 threads on interleaved levels: repeatable, and below the energy of
    the start every thread uses when there is no unary term."""
    _case("pipeline paper energy")
    wl = synth.make_small_arc(seed=72, n_views=5, width=160, height=96, n_segments=150, num_labels=32)
    dv = ivde.DeviceViews.from_workload(wl)
    lr = ivde.label_range(wl.z_near, wl.z_far, wl.num_labels)
    a = pipeline.estimate_depth(dv, lr, unary_weight=0.0, n_threads=4)
    b = pipeline.estimate_depth(dv, lr, unary_weight=0.0, n_threads=4)
    np.testing.assert_array_equal(a["labels"], b["labels"])
    E = a["energy_obj"]
    assert a["energy"] < E.value(np.zeros(dv.rows, np.int32))
    truth = synth.truth_labels(wl)
    print(f"[pipeline] paper energy within 2 levels: {_quality(a['labels'], truth):.3f}", flush=True)
