"""Warm start for new nodes (Section 4, closing remarks): a network is segmented, grows by new
nodes, and GFW restarts from the old binary solution with the new rows uniform.  The GLMO
keeps binary rows, so only the new rows move.

The old solution comes from the oracle (no expected value or input is taken from the GPU).
The GPU's warm-started solve is compared with the oracle's solve from the same U_0.  The
server's warm start (host U_0, copied at submit) is compared with gfw_solve from the same U_0."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_09738_amd import gfw
from synth import configs

from gpu_helpers import ctx, gpu_graph, np_of, say, torch_u

pytestmark = pytest.mark.gpu


def _warm_start(old, full):
    r_old = O.solve_problem(old, max_iter=200)
    U0 = np.full((full.n, full.K), 1.0 / full.K)
    U0[:old.n] = 0.0
    U0[np.arange(old.n), r_old["labels"]] = 1.0
    return U0


def test_warm_start_new_nodes_f64():
    say("[gpu] warm start for new nodes f64")
    old, full = configs.grown_sbm(seed=6, n_old=3000, n_new=150)
    U0 = _warm_start(old, full)
    L = O.operator_for(full.graph)
    ro = O.solve(L, full.K, full.labelled_idx, full.labels, max_iter=100, tol=1e-6, U0=U0)
    G = gpu_graph(full.graph, full.K, full.labelled_idx, full.labels, gfw.F64)
    rg = gfw.solve(ctx(), G, gfw.params(max_iter=100, tol=1e-6, U0=torch_u(U0, gfw.F64)))
    Ug = np_of(rg["U"])
    # old rows are exactly the old binary solution; the new rows moved
    np.testing.assert_array_equal(Ug[:old.n], U0[:old.n])
    assert np.all(np.any(Ug[old.n:] != U0[old.n:], axis=1))
    # the same iterate as the oracle's
    assert rg["iters"] == ro["iters"]
    np.testing.assert_array_equal(np_of(rg["labels"]), ro["labels"])
    np.testing.assert_allclose(Ug, ro["U"], rtol=0, atol=1e-12)
    assert rg["objective"] == pytest.approx(ro["objective"], rel=1e-12)
    cold = gfw.solve(ctx(), G, gfw.params(max_iter=300, tol=1e-6))
    acc_new = np.mean(np_of(rg["labels"])[old.n:] == full.graph.truth[old.n:])
    say(f"[gpu] warm start: {rg['iters']} iterations (cold start from Uhat: {cold['iters']}), "
        f"new-node accuracy {acc_new:.3f}")


def test_server_warm_start_equals_solve():
    say("[gpu] server warm start")
    old, full = configs.grown_sbm(seed=8, n_old=2000, n_new=100, K=4)
    U0 = _warm_start(old, full).astype(np.float32)
    g = full.graph
    prm = gfw.params(max_iter=80, tol=1e-6)
    G = gpu_graph(g, full.K, full.labelled_idx, full.labels, gfw.F32)
    alone = gfw.solve(ctx(), G, gfw.params(max_iter=80, tol=1e-6, U0=torch_u(U0, gfw.F32)))
    sv = gfw.Server(ctx(), 1 << 30, 8)
    try:
        t_cold = sv.submit(g.n, full.K, g.indptr, g.indices, g.data, full.labelled_idx, full.labels, prm)
        t_warm = sv.submit(g.n, full.K, g.indptr, g.indices, g.data, full.labelled_idx, full.labels, prm, U0=U0)
        U0[:] = -1.0  # the server holds its own copy
        rw = sv.poll(t_warm)
        rc = sv.poll(t_cold)
    finally:
        sv.close()
    np.testing.assert_array_equal(rw["U"], np_of(alone["U"]))
    np.testing.assert_array_equal(rw["labels"], np_of(alone["labels"]))
    assert rw["iters"] == alone["iters"]
    say(f"[gpu] server: warm {rw['iters']} iterations, cold {rc['iters']}")
