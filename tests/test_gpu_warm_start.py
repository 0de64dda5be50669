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


def _oracle_warm(full, U0, **kw):
    L = O.operator_for(full.graph)
    return O.solve(L, full.K, full.labelled_idx, full.labels, U0=U0, **kw)


@pytest.mark.parametrize("one_shot,K", [(False, 3), (True, 3), (False, 7), (False, 13)])
def test_incremental_matches_the_oracle_f64(one_shot, K):
    """The incremental solve (moving rows only) against the oracle's full iteration from the
    same U_0: the same iterates up to the order of the sums (K in each class-count bucket of
    the moving-row kernels: 4, 8 and 16)."""
    say(f"[gpu] incremental solve f64 one_shot={one_shot} K={K}")
    old, full = configs.grown_sbm(seed=6, n_old=3000, n_new=150, K=K)
    U0 = _warm_start(old, full)
    kw = dict(max_iter=100, tol=1e-6)
    ro = _oracle_warm(full, U0, osfw=one_shot, **kw)
    G = gpu_graph(full.graph, full.K, full.labelled_idx, full.labels, gfw.F64)
    rg = gfw.solve(ctx(), G, gfw.params(one_shot=one_shot, U0=torch_u(U0, gfw.F64), incremental=True, **kw),
                   want_history=True)
    Ug = np_of(rg["U"])
    np.testing.assert_array_equal(Ug[:old.n], U0[:old.n])  # binary rows never touched
    assert rg["iters"] == ro["iters"] and rg["stop_reason"] == ro["stop_reason"]
    np.testing.assert_array_equal(np_of(rg["labels"]), ro["labels"])
    np.testing.assert_allclose(Ug, ro["U"], rtol=0, atol=1e-12)
    assert rg["objective"] == pytest.approx(ro["objective"], rel=1e-12)
    k = rg["iters"] + (1 if rg["stop_reason"] == gfw.STOP_TOL else 0)  # evaluated iterates
    # E carried by the quadratic update against the oracle's direct evaluation; g, q, alpha
    np.testing.assert_allclose(rg["E"][:k], ro["E"][:k], rtol=1e-10)
    np.testing.assert_allclose(rg["g"][:k], ro["g"][:k], rtol=1e-8, atol=1e-11)
    steps = rg["iters"]
    np.testing.assert_allclose(rg["q"][:steps], ro["q"][:steps], rtol=1e-8, atol=1e-11)
    np.testing.assert_array_equal(rg["alpha"][:steps], ro["alpha"][:steps])
    # the incremental history has the full iteration's non-binary counts
    np.testing.assert_array_equal(rg["nonbinary"][:k], ro["nonbinary"][:k])


def test_incremental_matches_the_full_iteration_f32():
    say("[gpu] incremental solve f32 vs full iteration")
    old, full = configs.grown_sbm(seed=9, n_old=20000, n_new=600, K=5)
    U0 = _warm_start(old, full).astype(np.float32)
    G = gpu_graph(full.graph, full.K, full.labelled_idx, full.labels, gfw.F32)
    Ut = torch_u(U0, gfw.F32)
    a = gfw.solve(ctx(), G, gfw.params(max_iter=150, tol=1e-6, U0=Ut))
    b = gfw.solve(ctx(), G, gfw.params(max_iter=150, tol=1e-6, U0=Ut, incremental=True))
    Ua, Ub = np_of(a["U"]), np_of(b["U"])
    np.testing.assert_array_equal(Ub[:old.n], U0[:old.n])
    assert np.abs(Ua - Ub).max() <= 1e-5
    assert np.mean(np_of(a["labels"]) == np_of(b["labels"])) >= 0.999
    assert abs(a["iters"] - b["iters"]) <= 1
    assert b["objective"] == pytest.approx(a["objective"], rel=1e-6)


def test_incremental_edge_cases():
    say("[gpu] incremental edge cases")
    old, full = configs.grown_sbm(seed=10, n_old=1000, n_new=40, K=3)
    g = full.graph
    G = gpu_graph(g, full.K, full.labelled_idx, full.labels, gfw.F64)
    # every row binary: nothing moves, g_0 = 0 stops the solve at once (as the full iteration)
    U0 = np.zeros((g.n, full.K))
    U0[np.arange(g.n), np.arange(g.n) % full.K] = 1.0
    Ut = torch_u(U0, gfw.F64)
    a = gfw.solve(ctx(), G, gfw.params(max_iter=20, tol=1e-6, U0=Ut))
    b = gfw.solve(ctx(), G, gfw.params(max_iter=20, tol=1e-6, U0=Ut, incremental=True))
    np.testing.assert_array_equal(np_of(b["U"]), U0)
    assert a["iters"] == b["iters"] == 0 and a["stop_reason"] == b["stop_reason"] == gfw.STOP_TOL
    assert b["objective"] == pytest.approx(a["objective"], rel=1e-12)
    # tol disabled: the zero steps run to max_iter, as the full iteration
    a = gfw.solve(ctx(), G, gfw.params(max_iter=5, tol=-1.0, U0=Ut))
    b = gfw.solve(ctx(), G, gfw.params(max_iter=5, tol=-1.0, U0=Ut, incremental=True))
    assert a["iters"] == b["iters"] == 5
    np.testing.assert_array_equal(np_of(b["U"]), U0)

    def status(fn):
        with pytest.raises(gfw.GfwError) as e:
            fn()
        return e.value.status

    assert status(lambda: gfw.solve(ctx(), G, gfw.params(incremental=True))) == -1  # no U0
    assert status(lambda: gfw.solve(ctx(), G, gfw.params(U0=Ut, incremental=True, lmo=gfw.LMO_FULL))) == -1
    assert status(lambda: gfw.solve(ctx(), G, gfw.params(U0=Ut, incremental=True, p_refresh=4))) == -1
    assert status(lambda: gfw.solve_batched(ctx(), [G], gfw.params(U0=Ut, incremental=True))) == -6
    x = np.random.default_rng(0).random((50, 3))
    gg = gfw.Graph.gaussian(ctx(), x, 3, 0.3, np.zeros(0, np.int32), np.zeros(0, np.int32), gfw.F64)
    U5 = torch_u(np.full((50, 3), 1.0 / 3), gfw.F64)
    assert status(lambda: gfw.solve(ctx(), gg, gfw.params(U0=U5, incremental=True))) == -6
