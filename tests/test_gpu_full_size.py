"""Parity at the measured sizes, in the launch configuration bench.py times.

* The large SBM (n = 2,000,000, K = 5, 48 M entries, FP32) on the column-sorted label pass:
  one GPU iteration from the oracle's iterate against one oracle iteration on the whole graph
  (every row of U_1, and E, g, q, alpha).
* The same graph solved with the captured iteration graph (replays of 16 iterations, as timed)
  and with per-launch tracing (no graph): bitwise the same iterates.
* The largest serving request (1024 x 1024 8-neighbour grid, K = 6): one iteration in lockstep.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_09738_amd import gfw
from synth import configs, graphs

from gpu_helpers import ctx, gpu_graph, lockstep, np_of, say, torch_u

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbm_large():
    say("[gpu] full size: generating the large SBM")
    prob = configs.sbm_large()
    G = gpu_graph(prob.graph, prob.K, prob.labelled_idx, prob.labels, gfw.F32)
    assert G.query(gfw.TUNE_LABEL_PATH) == 2  # the column-sorted pass, as in the benchmark
    return prob, G


def test_full_size_sbm_lockstep(sbm_large):
    prob, G = sbm_large
    say("[gpu] full size: large SBM lockstep")
    lockstep(prob, gfw.F32, [0, 2], label="sbm_large")


def test_full_size_graph_replay_equals_per_launch(sbm_large):
    prob, G = sbm_large
    say("[gpu] full size: graph replay vs per-launch")
    prm = gfw.params(eps=prob.eps, omega0=prob.omega0, max_iter=48, tol=-1.0)
    replay = gfw.solve(ctx(), G, prm, want_history=True)
    gfw.trace_enable(ctx(), True)
    try:
        traced = gfw.solve(ctx(), G, prm, want_history=True)
    finally:
        gfw.trace_enable(ctx(), False)
    np.testing.assert_array_equal(np_of(replay["U"]), np_of(traced["U"]))
    np.testing.assert_array_equal(replay["alpha"], traced["alpha"])
    np.testing.assert_array_equal(replay["E"], traced["E"])
    assert replay["iters"] == traced["iters"] == 48


def test_full_size_serving_grid_lockstep():
    say("[gpu] full size: 1024 x 1024 grid lockstep")
    prob = configs.serve_request(4, 0, side=1024, K=6)
    lockstep(prob, gfw.F32, [0, 3], label="grid1024")
