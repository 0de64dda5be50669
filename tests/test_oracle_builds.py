"""The oracle's two builds and its FP32-storage switch (CPU only).

* The OpenMP timing build splits only loops over rows whose iterations are independent;
  every sum across rows stays serial, so its results are bit for bit those of the serial
  build (the parity reference).  Checked here on several workloads and solver variants.
* store_f32 rounds U to FP32 after each update (FP64 arithmetic, FP32 storage): every
  entry of the result is an FP32 number, labelled rows stay exactly one-hot, rows stay on
  the simplex to FP32 rounding, and the first step equals the FP64 one rounded.
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth import configs, graphs


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build(force=False)


def _same(a, b):
    for key in ("U", "labels", "E", "g", "q", "alpha", "nonbinary"):
        np.testing.assert_array_equal(a[key], b[key], err_msg=key)
    assert a["iters"] == b["iters"] and a["objective"] == b["objective"]


@pytest.mark.parametrize("case", ["sbm_small", "knn", "full_lmo", "exact", "short", "osfw", "grid"])
def test_openmp_build_is_bitwise_the_serial_build(case):
    if case == "knn":
        prob = configs.knn_mixture(seed=4, n=3000, d=32, K=6)
        prob.max_iter = 80
    elif case == "grid":
        g = graphs.image_grid(4096, 4, 3, neighbours=8)
        idx, lab = graphs.scribble_labels(g.truth, 64, 64, 4, 0.02, 3, stroke_len=4)
        prob = configs.Problem(g, idx, lab, 4, "f64", 50.0, 1000.0, 60, 1e-6, "grid")
    else:
        prob = configs.sbm_small(0)
    kw = {"full_lmo": dict(lmo_mode=O.LMO_FULL), "exact": dict(ls=O.LS_EXACT), "short": dict(ls=O.LS_SHORT),
          "osfw": dict(osfw=True)}.get(case, {})
    a = O.solve_problem(prob, **kw)
    b = O.solve_problem(prob, parallel=True, **kw)
    _same(a, b)


def test_store_f32_rounds_the_iterate_only():
    prob = configs.sbm_small(1, n_per=200)
    L = O.operator_for(prob.graph)
    r64 = O.solve(L, prob.K, prob.labelled_idx, prob.labels, max_iter=1, tol=-1)
    r32 = O.solve(L, prob.K, prob.labelled_idx, prob.labels, max_iter=1, tol=-1, store_f32=True)
    # the first step is taken from the same U_0 (exact in FP32), so it equals the FP64 step rounded
    assert r32["alpha"][0] == r64["alpha"][0]
    np.testing.assert_array_equal(r32["U"], r64["U"].astype(np.float32).astype(np.float64))
    r = O.solve(L, prob.K, prob.labelled_idx, prob.labels, max_iter=60, tol=-1, store_f32=True)
    U = r["U"]
    np.testing.assert_array_equal(U, U.astype(np.float32).astype(np.float64))
    assert np.all(U[prob.labelled_idx, prob.labels] == 1.0)
    assert np.abs(U.sum(axis=1) - 1.0).max() <= 4 * prob.K * 2.0 ** -24
