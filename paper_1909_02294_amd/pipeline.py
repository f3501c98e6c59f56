"""Depth maps from a rig's images: the energy terms on the GPU, Eq. (1)
minimised on the host, segment depths painted on the GPU (Sec. III).

Every step is a library call: the whole-segment matching cost
(ivde_cost_volume, optional unary term), the window core of Eq. (4)
(ivde_window_cost), the adjacency with the Eq. (3) weights
(ivde_adjacency), the label-partitioned alpha-expansion of Sec. IV-A
(ivde_optimize) and the painting (ivde_depth_map).  This module only moves
buffers between them and times the stages.
"""
from __future__ import annotations

import time

from . import ivde


def estimate_depth(dv: ivde.DeviceViews, lr, *, sampling=ivde.BILINEAR, unary_weight=300.0, use_window=True,
                   radius=1, K=30.0, beta0=1.0, eps=1.0, n_threads=8, partition=ivde.PARTITION_INTERLEAVED,
                   max_cycles=4, quantum=64.0, fixed=None):
    """Returns a dict with labels (host int32 [rows]), energy, depth (device
    float32, views one after another), the host Energy, and stage times in
    seconds.  unary_weight = 0 leaves out the cost volume, use_window =
    False the window term, beta0 = 0 the intra-view term."""
    import torch

    times = {}
    t0 = time.perf_counter()
    cost = m = hit = adj = None
    if unary_weight:
        cost, _ = ivde.cost_volume(dv, lr, ivde.options(sampling, ivde.F32))
    if use_window:
        m, hit, _ = ivde.window_cost(dv, lr, radius)
    if beta0 > 0:
        off, idx, beta, _ = ivde.adjacency(dv, beta0, eps)
        adj = (off, idx, beta)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    times["gpu_terms"] = t1 - t0
    host = lambda a: a.cpu().numpy() if a is not None else None  # noqa: E731
    E = ivde.Energy(dv.rows, lr.num_labels, unary=host(cost), unary_weight=unary_weight, m=host(m), hit=host(hit),
                    K=K, offsets=host(adj[0]) if adj else None, index=host(adj[1]) if adj else None,
                    beta=host(adj[2]) if adj else None, fixed=fixed, quantum=quantum)
    t2 = time.perf_counter()
    times["to_host"] = t2 - t1
    labels, energy = E.optimize(n_threads, partition, max_cycles)
    t3 = time.perf_counter()
    times["optimize"] = t3 - t2
    depth = ivde.depth_map(dv, lr, labels)
    torch.cuda.synchronize()
    times["paint"] = time.perf_counter() - t3
    times["total"] = time.perf_counter() - t0
    return {"labels": labels, "energy": energy, "depth": depth, "energy_obj": E, "times": times,
            "cost": cost}
