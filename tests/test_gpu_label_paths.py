"""The column-sorted label pass against the plain one (and, in lockstep, against the oracle).

Both passes sum every row's label histogram in CSR order, so Q = L_s S is the same; only the
order of the per-tile partial sums differs.  Graphs here are forced onto the sorted path with
gfw_graph_tune; they cover FP32/FP64, K = 2..16 (labels packed two per byte),
rows without entries, a ragged last tile, and runs of sorted entries whose columns span more
than 16 bits (read through the CSR columns instead of the anchor)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_09738_amd import gfw
from synth import configs, graphs

from gpu_helpers import ctx, gpu_graph, lockstep, say, torch_u

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("dtype,K,n", [(gfw.F32, 5, 40001), (gfw.F64, 3, 9000), (gfw.F32, 16, 12000),
                                       (gfw.F64, 16, 5000), (gfw.F32, 2, 70001)])
def test_sorted_label_pass_matches_plain(dtype, K, n):
    say(f"[gpu] sorted vs plain label pass dtype={dtype} K={K} n={n}")
    g = graphs.sbm_by_degree(n, K, 24.0, 8.0, 70 + K)
    # a few rows without entries: drop the edges of nodes 0..9
    import scipy.sparse as sp
    W = sp.csr_matrix((g.data, g.indices, g.indptr), shape=(g.n, g.n)).tolil()
    for i in range(10):
        W[i, :] = 0
        W[:, i] = 0
    W = W.tocsr()
    W.eliminate_zeros()
    W.sort_indices()
    g = graphs.Graph(g.n, K, W.indptr.astype(np.int64), W.indices.astype(np.int32), W.data, g.truth)
    idx, lab = graphs.stratified_labels(g.truth, K, 0.02, 70 + K)
    G = gpu_graph(g, K, idx, lab, dtype)
    prm = gfw.params(max_iter=25, tol=-1)
    G.tune(gfw.TUNE_LABEL_PATH, 1)
    assert G.query(gfw.TUNE_LABEL_PATH) == 1
    a = gfw.solve(ctx(), G, prm, want_history=True)
    G.tune(gfw.TUNE_LABEL_PATH, 2)
    assert G.query(gfw.TUNE_LABEL_PATH) == 2
    b = gfw.solve(ctx(), G, prm, want_history=True)
    np.testing.assert_array_equal(a["alpha"], b["alpha"])
    np.testing.assert_array_equal(_np(a["labels"]), _np(b["labels"]))
    np.testing.assert_allclose(_np(a["U"]), _np(b["U"]), atol=1e-12 if dtype == gfw.F64 else 1e-6)
    np.testing.assert_allclose(a["q"][:25], b["q"][:25], rtol=1e-9 if dtype == gfw.F64 else 1e-5)


def test_sorted_label_pass_lockstep_against_oracle():
    say("[gpu] sorted label pass lockstep")
    prob = configs.sbm_small(5, n_per=3000)
    L = O.operator_for(prob.graph)
    G = gpu_graph(prob.graph, prob.K, prob.labelled_idx, prob.labels, gfw.F64)
    G.tune(gfw.TUNE_LABEL_PATH, 2)
    for k in (0, 7, 40):
        Uk = O.fidelity(prob.n, prob.K, prob.labelled_idx, prob.labels, 1000.0)[0] if k == 0 else \
            O.solve(L, prob.K, prob.labelled_idx, prob.labels, max_iter=k, tol=-1)["U"]
        ro = O.solve(L, prob.K, prob.labelled_idx, prob.labels, max_iter=1, tol=-1, U0=Uk, record_s=True)
        rg = gfw.solve(ctx(), G, gfw.params(max_iter=1, tol=-1, U0=torch_u(Uk, gfw.F64)), want_s=True,
                       want_history=True)
        if np.array_equal(_np(rg["s"]), ro["s"][0]):
            assert rg["q"][0] == pytest.approx(ro["q"][0], rel=1e-9)
            assert rg["alpha"][0] == ro["alpha"][0]
            np.testing.assert_allclose(_np(rg["U"]), ro["U"], atol=1e-12)


def test_auto_choice():
    say("[gpu] automatic label path choice")
    grid = graphs.image_grid(20000, 4, 1, neighbours=4)
    G = gpu_graph(grid, 4, [0], [0], gfw.F32)
    assert G.query(gfw.TUNE_LABEL_PATH) == 1  # small and local: plain pass


def test_measured_choice():
    """Value 3 times both passes on the graph and keeps the faster; the solve is the same
    whichever is kept."""
    say("[gpu] measured label path choice")
    g = graphs.sbm_by_degree(200000, 5, 24.0, 8.0, 31)
    idx, lab = graphs.stratified_labels(g.truth, 5, 0.01, 31)
    G = gpu_graph(g, 5, idx, lab, gfw.F32)
    prm = gfw.params(max_iter=20, tol=-1)
    G.tune(gfw.TUNE_LABEL_PATH, gfw.LABEL_PATH_PLAIN)
    ref = _np(gfw.solve(ctx(), G, prm)["U"])
    G.tune(gfw.TUNE_LABEL_PATH, gfw.LABEL_PATH_MEASURED)
    plain_ns, sorted_ns = G.query(gfw.TUNE_LABEL_PLAIN_NS), G.query(gfw.TUNE_LABEL_SORTED_NS)
    chosen = G.query(gfw.TUNE_LABEL_PATH)
    say(f"[gpu] measured: plain {plain_ns / 1e3:.1f} us, sorted {sorted_ns / 1e3:.1f} us, chosen {chosen}")
    assert plain_ns > 0 and sorted_ns > 0
    assert chosen == (2 if sorted_ns < plain_ns else 1)
    np.testing.assert_array_equal(_np(gfw.solve(ctx(), G, prm)["U"]), ref)


def test_row_longer_than_a_sorted_tile():
    """A hub with 140,000 neighbours does not fit a column-sorted tile (131,072 entries): the
    sorted pass is refused, the measured choice falls back to the plain pass, and the solve
    still follows the oracle."""
    say("[gpu] hub row beyond the sorted tile size")
    import scipy.sparse as sp
    rng = np.random.default_rng(5)
    n, K, hub = 160000, 3, 0
    nb = rng.choice(np.arange(1, n), 140000, replace=False)
    a = np.concatenate([np.zeros(nb.size, np.int64), rng.integers(1, n, 300000)])
    b = np.concatenate([nb, rng.integers(1, n, 300000)])
    keep = a != b
    W = sp.coo_matrix((np.ones(keep.sum()), (a[keep], b[keep])), shape=(n, n)).tocsr()
    W = ((W + W.T) > 0).astype(np.float64).tocsr()
    W.sort_indices()
    truth = rng.integers(0, K, n).astype(np.int32)
    g = graphs.Graph(n, K, W.indptr.astype(np.int64), W.indices.astype(np.int32), W.data, truth)
    assert np.diff(g.indptr)[hub] > 131072
    idx, lab = graphs.stratified_labels(truth, K, 0.01, 5)
    G = gpu_graph(g, K, idx, lab, gfw.F64)
    with pytest.raises(gfw.GfwError) as e:
        G.tune(gfw.TUNE_LABEL_PATH, gfw.LABEL_PATH_SORTED)
    assert e.value.status == -6
    G.tune(gfw.TUNE_LABEL_PATH, gfw.LABEL_PATH_MEASURED)
    assert G.query(gfw.TUNE_LABEL_PATH) == 1
    prob = configs.Problem(g, idx, lab, K, "f64", 50.0, 1000.0, 20, 1e-6, "hub")
    lockstep(prob, gfw.F64, [0, 5, 15], label="hub")


def _wide_graph(seed=9, n_dense=60000, n_sparse=140000, K=4):
    """A random graph on the first n_dense nodes (mean degree about 12) plus a sparse region
    of mostly isolated nodes, where every 4000th node links to 20 random nodes of the whole
    graph.  The column-sorted tiles of the sparse region hold about a hundred entries spread
    over all columns, so their 64-entry runs span more than 32,767 columns."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    n = n_dense + n_sparse
    m = n_dense * 6
    a = rng.integers(0, n_dense, m)
    b = rng.integers(0, n_dense, m)
    hubs = np.arange(n_dense, n, 4000)
    a = np.concatenate([a, np.repeat(hubs, 20)])
    b = np.concatenate([b, rng.integers(0, n, hubs.size * 20)])
    keep = a != b
    w = rng.uniform(0.5, 2.0, keep.sum())
    W = sp.coo_matrix((w, (a[keep], b[keep])), shape=(n, n)).tocsr()
    W = (W + W.T).tocsr()
    W.sum_duplicates()
    W.sort_indices()
    truth = rng.integers(0, K, n).astype(np.int32)
    return graphs.Graph(n, K, W.indptr.astype(np.int64), W.indices.astype(np.int32), W.data, truth)


@pytest.mark.parametrize("dtype", [gfw.F32, gfw.F64])
def test_sorted_wide_chunks_match_plain(dtype):
    say(f"[gpu] sorted pass with wide chunks dtype={dtype}")
    g = _wide_graph()
    idx, lab = graphs.stratified_labels(g.truth, g.K, 0.02, 9)
    G = gpu_graph(g, g.K, idx, lab, dtype)
    prm = gfw.params(max_iter=25, tol=-1)
    G.tune(gfw.TUNE_LABEL_PATH, 1)
    assert G.query(gfw.TUNE_SORTED_WIDE_CHUNKS) == 0  # no sorted copy yet
    a = gfw.solve(ctx(), G, prm, want_history=True)
    G.tune(gfw.TUNE_LABEL_PATH, 2)
    wide = G.query(gfw.TUNE_SORTED_WIDE_CHUNKS)
    say(f"[gpu] wide chunks: {wide} of about {g.nnz // 64}")
    assert 0 < wide < g.nnz // 64 // 2  # both kinds of chunk are present
    b = gfw.solve(ctx(), G, prm, want_history=True)
    np.testing.assert_array_equal(a["alpha"], b["alpha"])
    np.testing.assert_array_equal(_np(a["labels"]), _np(b["labels"]))
    np.testing.assert_array_equal(_np(a["U"]), _np(b["U"]))
    np.testing.assert_allclose(a["q"][:25], b["q"][:25], rtol=1e-9 if dtype == gfw.F64 else 1e-5)


def test_sorted_wide_chunks_lockstep_against_oracle():
    say("[gpu] sorted pass with wide chunks: lockstep")
    g = _wide_graph(seed=10)
    idx, lab = graphs.stratified_labels(g.truth, g.K, 0.02, 10)
    prob = configs.Problem(g, idx, lab, g.K, "f64", 50.0, 1000.0, 20, 1e-6, "wide")
    lockstep(prob, gfw.F64, [0, 4], label="wide", label_path=gfw.LABEL_PATH_SORTED)


def test_sorted_tiles_built_after_a_solve_grow_the_partials():
    """A small graph gets about one sorted tile per CU, more tiles than 256-row blocks.  When
    the tiles are built after a solve on the plain pass, the label-pass partials buffer (sized
    at that solve) grows, the footprint counts it, and the sorted solves that follow match the
    plain one."""
    say("[gpu] sorted tiles built after a plain solve")
    n, K = 9000, 3
    g = graphs.sbm_by_degree(n, K, 24.0, 8.0, 44)
    idx, lab = graphs.stratified_labels(g.truth, K, 0.02, 44)
    G = gpu_graph(g, K, idx, lab, gfw.F64)
    prm = gfw.params(max_iter=20, tol=-1)
    assert G.query(gfw.TUNE_LABEL_PATH) == 1
    plain = gfw.solve(ctx(), G, prm, want_history=True)
    _, solve_before = G.footprint()
    G.tune(gfw.TUNE_LABEL_PATH, 2)
    _, solve_after = G.footprint()
    nb_row = -(-n // 256)
    assert solve_after - solve_before >= 8 * (200 - nb_row)  # about 255 tiles on 256 CUs
    for _ in range(2):  # the second solve replays the captured iterations
        b = gfw.solve(ctx(), G, prm, want_history=True)
        np.testing.assert_array_equal(plain["alpha"], b["alpha"])
        np.testing.assert_array_equal(_np(plain["labels"]), _np(b["labels"]))
        np.testing.assert_allclose(_np(plain["U"]), _np(b["U"]), atol=1e-12)


@pytest.mark.parametrize("K", list(range(2, 17)))
def test_every_class_count_sorted_equals_plain(K):
    """The single-graph row kernel and sorted label pass are instantiated per class count
    K = 2..16: each gives the same iterates as the plain pass (FP64, small SBM)."""
    say(f"[gpu] class count {K}: sorted vs plain")
    g = graphs.sbm_by_degree(3000, K, 20.0, 8.0, 500 + K)
    idx, lab = graphs.stratified_labels(g.truth, K, 0.05, 500 + K)
    G = gpu_graph(g, K, idx, lab, gfw.F64)
    prm = gfw.params(max_iter=10, tol=-1)
    G.tune(gfw.TUNE_LABEL_PATH, 1)
    a = gfw.solve(ctx(), G, prm, want_history=True)
    G.tune(gfw.TUNE_LABEL_PATH, 2)
    b = gfw.solve(ctx(), G, prm, want_history=True)
    np.testing.assert_array_equal(a["alpha"], b["alpha"])
    np.testing.assert_array_equal(_np(a["labels"]), _np(b["labels"]))
    np.testing.assert_allclose(_np(a["U"]), _np(b["U"]), rtol=0, atol=1e-12)
    assert np.all(np.isfinite(a["E"][:10]))
