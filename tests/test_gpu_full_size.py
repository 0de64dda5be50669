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

from gpu_helpers import ctx, gpu_graph, lockstep, np_of, oracle_sensitivity, say, torch_u

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbm_large():
    say("[gpu] full size: generating the large SBM")
    prob = configs.sbm_large()
    G = gpu_graph(prob.graph, prob.K, prob.labelled_idx, prob.labels, gfw.F32)
    assert G.query(gfw.TUNE_LABEL_PATH) == 2  # the column-sorted pass, as in the benchmark
    return prob, G


def test_full_size_sbm_lockstep(sbm_large):
    """Lockstep on the whole large SBM at iterates 0, 2, 20 and 50.  On this input the
    unlabelled rows tie exactly at U_0 (89% of the nodes have no labelled neighbour), take
    class 0 by the lowest-index rule and drift towards it; the later iterates check the
    path on rows that are far from uniform."""
    prob, G = sbm_large
    say("[gpu] full size: large SBM lockstep")
    lockstep(prob, gfw.F32, [0, 2, 20, 50], label="sbm_large", traj_parallel=True)


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


def test_full_size_knn_mixture():
    """The k-NN workload at its full size (70,000 points in 784 dimensions, K = 10, about 1 M
    entries, 500 iterations): lockstep (FP32) at three iterates, then free-running solves
    against the oracle's.  In FP64 the GPU path follows the oracle: the same step sizes and
    the objective to 1e-12.  In FP32 the objective contract is 1e-6 relative, or 1.5 times the
    oracle's own sensitivity to rounding where that is larger: the oracle's objective on the
    same problem with its nodes renumbered, and with U stored in FP32 after every update,
    moves from its FP64 result by that much (an oracle-only measure)."""
    say("[gpu] full size: k-NN mixture (graph built with blocked products on the GPU)")
    prob = configs.knn_mixture(device="cuda")
    lockstep(prob, gfw.F32, [0, 100, 400], label="knn70000", traj_parallel=True)
    ro, sens = oracle_sensitivity(prob)
    acc = np.mean(ro["labels"] == prob.graph.truth)
    say(f"[gpu] knn70000: oracle sensitivity to rounding {sens:.3e}")
    bound = {gfw.F64: 1e-12, gfw.F32: max(1e-6, 1.5 * sens)}
    for dt in (gfw.F64, gfw.F32):
        G = gpu_graph(prob.graph, prob.K, prob.labelled_idx, prob.labels, dt)
        rg = gfw.solve(ctx(), G, gfw.params(eps=prob.eps, omega0=prob.omega0, max_iter=prob.max_iter, tol=prob.tol),
                       want_history=True)
        agree = np.mean(np_of(rg["labels"]) == ro["labels"])
        dE = abs(rg["objective"] - ro["objective"]) / abs(ro["objective"])
        same_steps = np.array_equal(rg["alpha"][:ro["iters"]], ro["alpha"][:ro["iters"]])
        say(f"[gpu] knn70000 dtype={dt}: iters {rg['iters']}/{ro['iters']}, label agreement {agree:.5f}, "
            f"rel dE {dE:.3e}, same step sizes {same_steps}, oracle accuracy {acc:.4f}")
        assert rg["iters"] == ro["iters"]
        assert agree >= 0.999
        assert dE <= bound[dt]
        if dt == gfw.F64:
            assert same_steps


def test_full_size_new_nodes_incremental():
    """The new-node workload at its benchmarked size: 1,000 nodes joining a segmented network
    of 1,000,000 (K = 5).  The old network is segmented by the oracle (its OpenMP build); from
    that warm start the incremental solve (moving rows only) and the full iteration agree: old
    rows untouched, the new nodes' labels identical, U within FP32 rounding, the same number of
    iterations and the objective to 1e-6."""
    say("[gpu] full size: 1,000,000 + 1,000 new nodes, incremental against the full iteration")
    old, full = configs.grown_sbm(seed=11, n_old=1_000_000, n_new=1000, K=5)
    r_old = O.solve_problem(old, max_iter=100, parallel=True)
    U0 = np.full((full.n, full.K), 1.0 / full.K, dtype=np.float32)
    U0[:old.n] = 0.0
    U0[np.arange(old.n), r_old["labels"]] = 1.0
    G = gpu_graph(full.graph, full.K, full.labelled_idx, full.labels, gfw.F32)
    Ut = torch_u(U0, gfw.F32)
    a = gfw.solve(ctx(), G, gfw.params(max_iter=300, tol=1e-6, U0=Ut))
    b = gfw.solve(ctx(), G, gfw.params(max_iter=300, tol=1e-6, U0=Ut, incremental=True))
    Ua, Ub = np_of(a["U"]), np_of(b["U"])
    np.testing.assert_array_equal(Ub[:old.n], U0[:old.n])
    assert np.abs(Ua - Ub).max() <= 1e-5
    la, lb = np_of(a["labels"]), np_of(b["labels"])
    assert np.array_equal(la[old.n:], lb[old.n:])
    assert abs(a["iters"] - b["iters"]) <= 1
    assert b["objective"] == pytest.approx(a["objective"], rel=1e-6)
    say(f"[gpu]   iterations {a['iters']} / {b['iters']}; new-node accuracy "
        f"{np.mean(lb[old.n:] == full.graph.truth[old.n:]):.4f}")


def test_full_size_many_classes_lockstep():
    """The many-classes workload at its benchmarked size (LFR-shaped, n = 100,000, K = 585, FP32,
    the 10-classes-per-lane row kernel) in lockstep with the oracle."""
    say("[gpu] full size: LFR-shaped n=100,000, K=585")
    prob = configs.lfr_many_classes()
    prob.max_iter = 12
    lockstep(prob, gfw.F32, [0, 1, 10], label="lfr100000", traj_parallel=True)
