"""Batched solves (gfw_solve_batched): every graph's result equals its solve alone, bitwise,
whatever else shares the launches (sizes, K buckets, label paths, per-graph settings)."""
import numpy as np
import pytest

from paper_2508_09738_amd import gfw
from synth import configs, graphs

from gpu_helpers import ctx, gpu_graph, say

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _members(count=10, seed=7):
    probs = [configs.batch_member(seed, i, n_lo=500, n_hi=30000) for i in range(count)]
    # one K = 16 member, one K = 2 member
    g = graphs.sbm_by_degree(4000, 16, 20.0, 8.0, 99)
    idx, lab = graphs.stratified_labels(g.truth, 16, 0.03, 99)
    probs.append(configs.Problem(g, idx, lab, 16, "f32", 50.0, 1000.0, 300, 1e-6, "K16"))
    g = graphs.image_grid(3000, 2, 98, neighbours=8)
    idx, lab = graphs.stratified_labels(g.truth, 2, 0.03, 98)
    probs.append(configs.Problem(g, idx, lab, 2, "f32", 50.0, 1000.0, 300, 1e-6, "K2"))
    return probs


def test_batch_equals_alone_bitwise():
    say("[gpu] batch vs alone")
    probs = _members()
    Gs = [gpu_graph(p.graph, p.K, p.labelled_idx, p.labels, gfw.F32) for p in probs]
    Gs[3].tune(gfw.TUNE_LABEL_PATH, 2)  # one member on the column-sorted label pass
    prms = [gfw.params(max_iter=40 + 7 * i, tol=(1e-6 if i % 3 else -1.0)) for i in range(len(Gs))]
    alone = [gfw.solve(ctx(), G, pr) for G, pr in zip(Gs, prms)]
    batch = gfw.solve_batched(ctx(), Gs, prms)
    for i, (a, b) in enumerate(zip(alone, batch)):
        say(f"  member {i}: n={Gs[i].n} K={Gs[i].K} iters={a['iters']}")
        np.testing.assert_array_equal(_np(a["U"]), _np(b["U"]))
        np.testing.assert_array_equal(_np(a["labels"]), _np(b["labels"]))
        assert a["iters"] == b["iters"] and a["stop_reason"] == b["stop_reason"]
        assert a["objective"] == b["objective"] and a["gap"] == b["gap"]


def test_batch_shared_params_and_order_independence():
    say("[gpu] batch order independence")
    probs = _members(6, seed=8)
    Gs = [gpu_graph(p.graph, p.K, p.labelled_idx, p.labels, gfw.F32) for p in probs]
    pr = gfw.params(max_iter=30, tol=-1)
    a = gfw.solve_batched(ctx(), Gs, pr)
    order = list(reversed(range(len(Gs))))
    b = gfw.solve_batched(ctx(), [Gs[i] for i in order], pr)
    for j, i in enumerate(order):
        np.testing.assert_array_equal(_np(a[i]["U"]), _np(b[j]["U"]))


def test_batch_rejects_duplicates_and_mixed_dtypes():
    say("[gpu] batch argument checks")
    probs = _members(2, seed=9)
    G0 = gpu_graph(probs[0].graph, probs[0].K, probs[0].labelled_idx, probs[0].labels, gfw.F32)
    G1 = gpu_graph(probs[1].graph, probs[1].K, probs[1].labelled_idx, probs[1].labels, gfw.F64)
    with pytest.raises(gfw.GfwError) as e:
        gfw.solve_batched(ctx(), [G0, G0], gfw.params())
    assert e.value.status == -1
    with pytest.raises(gfw.GfwError) as e:
        gfw.solve_batched(ctx(), [G0, G1], gfw.params())
    assert e.value.status == -6


def test_batch_with_many_classes_equals_alone_bitwise():
    """Graphs with K > 16 (LFR-shaped, one of every classes-per-lane bucket) in one batch with
    small-K graphs: each result is bitwise the result alone."""
    say("[gpu] batch with many classes vs alone")
    probs = _members(3, seed=12)
    for j, K in enumerate((17, 100, 200, 300, 700)):
        probs.append(configs.lfr_many_classes(seed=40 + j, n=max(2000, 4 * K), K=K, frac=0.05))
    Gs = [gpu_graph(p.graph, p.K, p.labelled_idx, p.labels, gfw.F32) for p in probs]
    prms = [gfw.params(max_iter=25 + 5 * i, tol=(1e-6 if i % 2 else -1.0)) for i in range(len(Gs))]
    alone = [gfw.solve(ctx(), G, pr) for G, pr in zip(Gs, prms)]
    batch = gfw.solve_batched(ctx(), Gs, prms)
    for i, (a, b) in enumerate(zip(alone, batch)):
        say(f"  member {i}: n={Gs[i].n} K={Gs[i].K} iters={a['iters']}")
        np.testing.assert_array_equal(_np(a["U"]), _np(b["U"]))
        np.testing.assert_array_equal(_np(a["labels"]), _np(b["labels"]))
        assert a["iters"] == b["iters"] and a["objective"] == b["objective"] and a["gap"] == b["gap"]
