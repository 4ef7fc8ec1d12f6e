"""Outer iterations replayed from captured HIP graphs match eager execution.

Two simulations of the same workload run side by side, one replaying each outer
iteration from its cached graph and one enqueuing the same work eagerly; the host
synchronizes after every replay (the convergence test), commits and sorts in between.
Both run in the deterministic mode (stable sort, fixed-point current sums across
workgroups), so every step's particle state and fields must agree bit for bit, and the
graph run must really have replayed graphs.
"""
import sys

import numpy as np
import pytest

from paper_2609_36383_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_36383_amd import gmhc as G
    return G


def _rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("fp32,timing,shape", [(False, 0, 2), (False, 1, 2), (True, 1, 2), (False, 0, 1)],
                         ids=["fp64", "fp64-timed", "fp32-timed", "fp64-linear"])
def test_graph_replays_match_eager(fp32, timing, shape):
    G = _gpu()
    w = W.spec("weibel2d", n=(16, 16), ppc=16)
    x, u, q = W.particles(w)
    base = W.config_dict(w, fp32_bulk=fp32)
    prec = G.FP32_BULK if fp32 else G.FP64
    sims = []
    for graphs in (1, 0):
        s = G.Simulation(G.config_from_dict(base, sort_every=4, timing=timing, graphs=graphs, precision=prec,
                                            shape_order=shape, deterministic=1), q.size)
        s.load_particles(x, u, q)
        s.initialize()
        sims.append(s)
    replays = 0
    for k in range(12):
        _, rg = sims[0].step()
        _, re = sims[1].step()
        replays += rg["graph_replays"]
        assert re["graph_replays"] == 0
        assert rg["outer_iters"] == re["outer_iters"]
        if timing:
            assert rg["orbit_ms"] > 0.0 and re["orbit_ms"] > 0.0
        xg, Pg, vg = sims[0].read_particles()
        xe, Pe, ve = sims[1].read_particles()
        assert np.array_equal(xg, xe) and np.array_equal(Pg, Pe) and np.array_equal(vg, ve), k
        for f in ("A", "phi", "J"):
            assert np.array_equal(sims[0].read_field(f), sims[1].read_field(f)), (k, f)
    print(f"graph replays over 12 steps: {replays}", flush=True)
    sys.stdout.flush()
    assert replays >= 12
