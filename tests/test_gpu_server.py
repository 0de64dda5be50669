"""The request server (gfw_server_*): admission by HBM budget, continuous batching, and
results identical to the solve of each request alone."""
import time

import numpy as np
import pytest

from paper_2508_09738_amd import gfw
from synth import configs, graphs

from gpu_helpers import ctx, gpu_graph, say

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _requests(count, seed):
    return [configs.serve_request(seed, i, sides=(32, 48, 64, 96), Ks=(3, 4, 6)) for i in range(count)]


def _submit(sv, p, prm):
    g = p.graph
    return sv.submit(g.n, p.K, g.indptr, g.indices, g.data, p.labelled_idx, p.labels, prm)


def test_server_results_equal_alone_with_staggered_arrivals():
    say("[gpu] server: staggered arrivals vs alone")
    reqs = _requests(9, 21)
    prms = [gfw.params(max_iter=20 + 9 * i, tol=1e-6 if i % 2 else -1.0) for i in range(len(reqs))]
    sv = gfw.Server(ctx(), 1 << 30, 4)
    tickets = {}
    for i in range(4):
        tickets[i] = _submit(sv, reqs[i], prms[i])
    first = sv.poll(tickets[0], blocking=True)  # while others still run
    for i in range(4, len(reqs)):
        tickets[i] = _submit(sv, reqs[i], prms[i])
        time.sleep(0.002)
    res = {0: first}
    for i in range(1, len(reqs)):
        res[i] = sv.poll(tickets[i], blocking=True)
    sv.close()
    for i, p in enumerate(reqs):
        G = gpu_graph(p.graph, p.K, p.labelled_idx, p.labels, gfw.F32)
        a = gfw.solve(ctx(), G, prms[i])
        np.testing.assert_array_equal(_np(a["U"]), res[i]["U"])
        np.testing.assert_array_equal(_np(a["labels"]), res[i]["labels"])
        assert a["iters"] == res[i]["iters"] and a["objective"] == res[i]["objective"]


def test_server_rejects_poisoned_request_alone_and_enforces_budget():
    say("[gpu] server: poisoned request, budget")
    reqs = _requests(3, 22)
    sv = gfw.Server(ctx(), 64 << 20, 8)
    prm = gfw.params(max_iter=15, tol=-1)
    good = [_submit(sv, p, prm) for p in reqs]
    bad = reqs[0].graph
    w = bad.data.copy()
    w[5] = np.nan
    # a NaN weight is found on the device at admission: that request alone fails, at poll
    t_bad = sv.submit(bad.n, reqs[0].K, bad.indptr, bad.indices, w, reqs[0].labelled_idx, reqs[0].labels, prm)
    with pytest.raises(gfw.GfwError) as e:
        sv.poll(t_bad)
    assert e.value.status == -2
    # a decreasing row pointer is caught at submit
    ip = bad.indptr.copy()
    ip[3] = ip[2] - 1
    with pytest.raises(gfw.GfwError) as e:
        sv.submit(bad.n, reqs[0].K, ip, bad.indices, bad.data, reqs[0].labelled_idx, reqs[0].labels, prm)
    assert e.value.status == -2
    big = graphs.image_grid(1024 * 1024, 3, 5, neighbours=8, side=1024)
    with pytest.raises(gfw.GfwError) as e:
        sv.submit(big.n, 3, big.indptr, big.indices, big.data, [0], [0], prm)
    assert e.value.status == -7  # over the 64 MiB budget
    for t, p in zip(good, reqs):
        r = sv.poll(t)
        G = gpu_graph(p.graph, p.K, p.labelled_idx, p.labels, gfw.F32)
        np.testing.assert_array_equal(_np(gfw.solve(ctx(), G, prm)["U"]), r["U"])
    sv.close()


def test_server_small_budget_serialises_but_completes():
    say("[gpu] server: one request at a time by budget")
    reqs = _requests(4, 23)
    prm = gfw.params(max_iter=12, tol=-1)
    sv = gfw.Server(ctx(), 2 << 20, 16)  # room for about one request at a time
    ts = [_submit(sv, p, prm) for p in reqs]
    nr = sv.poll(ts[-1], blocking=False)
    assert nr is None or nr["iters"] == 12
    out = [sv.poll(t) for t in ts[:-1]]
    if nr is None:
        out.append(sv.poll(ts[-1]))
    assert all(r["iters"] == 12 for r in out)
    sv.close()


def test_server_many_classes_request_equals_alone():
    say("[gpu] server: many-classes request")
    prob = configs.lfr_many_classes(seed=21, n=3000, K=120, frac=0.05)
    small = _requests(2, 24)
    prm = gfw.params(max_iter=30, tol=-1)
    sv = gfw.Server(ctx(), 1 << 30, 8)
    try:
        g = prob.graph
        t_big = sv.submit(g.n, prob.K, g.indptr, g.indices, g.data, prob.labelled_idx, prob.labels, prm)
        ts = [_submit(sv, p, prm) for p in small]
        r = sv.poll(t_big)
        rs = [sv.poll(t) for t in ts]
    finally:
        sv.close()
    G = gpu_graph(g, prob.K, prob.labelled_idx, prob.labels, gfw.F32)
    alone = gfw.solve(ctx(), G, prm)
    np.testing.assert_array_equal(r["U"], _np(alone["U"]))
    np.testing.assert_array_equal(r["labels"], _np(alone["labels"]))
    for p, rr in zip(small, rs):
        Gp = gpu_graph(p.graph, p.K, p.labelled_idx, p.labels, gfw.F32)
        np.testing.assert_array_equal(rr["U"], _np(gfw.solve(ctx(), Gp, prm)["U"]))


def test_served_results_against_oracle():
    """A sample of the serving mix (8-neighbour grids with scribbles, smaller sides) served
    together in FP64 and compared with the oracle's free-running solves: labels, iterations
    and the objective (1e-6 relative, or the oracle's own sensitivity to rounding)."""
    from oracle import oracle as O

    from gpu_helpers import oracle_sensitivity

    reqs = [configs.serve_request(31, i, sides=(64, 96, 128), Ks=(3, 4, 6)) for i in range(4)]
    prm = gfw.params(eps=50.0, omega0=1000.0, max_iter=300, tol=1e-6)
    sv = gfw.Server(ctx(), 1 << 30, 8)
    try:
        ts = [sv.submit(p.n, p.K, p.graph.indptr, p.graph.indices, p.graph.data, p.labelled_idx, p.labels, prm,
                        dtype=gfw.F64) for p in reqs]
        res = [sv.poll(t) for t in ts]
    finally:
        sv.close()
    for p, r in zip(reqs, res):
        ro, sens = oracle_sensitivity(p)
        agree = np.mean(r["labels"] == ro["labels"])
        dE = abs(r["objective"] - ro["objective"]) / abs(ro["objective"])
        say(f"[gpu] served n={p.n} K={p.K}: iters {r['iters']}/{ro['iters']}, agreement {agree:.5f}, "
            f"rel dE {dE:.3e} (oracle sensitivity {sens:.3e})")
        assert agree >= 0.999
        assert dE <= max(1e-6, 1.5 * sens)
