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


def _inferred_vertices(U_prev, U_next):
    """The GLMO vertex of every row from one update U_next = (1 - a) U_prev + a e_s: the one
    column that grows (a binary row kept by the GLMO does not change: its 1)."""
    d = U_next - U_prev
    s = np.argmax(d, axis=1)
    still = ~np.any(d != 0, axis=1)
    s[still] = np.argmax(U_prev[still], axis=1)
    return s.astype(np.int32)


@pytest.mark.parametrize("dtype", [gfw.F64, gfw.F32])
def test_batch_members_against_oracle(dtype):
    """Eight random members of the batch mix (SBMs and 4-neighbour grids, n log-uniform in
    [2e3, 2e5], K in 3..10) in lockstep with the oracle through one batched call per iterate:
    every member starts from the oracle's U_k and makes one batched iteration, compared with
    one oracle iteration (step size, U_{k+1}, objective); rows where the batch took another
    GLMO vertex must be near-ties, and the oracle is then re-run with the batch's vertices."""
    from oracle import oracle as O

    from gpu_helpers import MAX_DIFF_FRAC, MAX_DIFF_SLACK, NEAR_TIE_REL, armijo_ratio_near_power, glmo_margin, oracle_trajectory, torch_u

    rng = np.random.default_rng(11)
    picks = sorted(rng.choice(256, size=8, replace=False).tolist())
    probs = [configs.batch_member(3, int(i)) for i in picks]
    say(f"[gpu] batch vs oracle dtype={dtype}: members {picks}, n={[p.n for p in probs]}")
    Gs = [gpu_graph(p.graph, p.K, p.labelled_idx, p.labels, dtype) for p in probs]
    Ls = [O.operator_for(p.graph) for p in probs]
    ks = [0, 5, 40]
    trajs = [oracle_trajectory(p, ks, parallel=True) for p in probs]
    band = NEAR_TIE_REL[dtype]
    u_tol = 1e-12 if dtype == gfw.F64 else 1e-5
    for k in ks:
        say(f"[gpu] batch vs oracle k={k}")
        U0s = [torch_u(t[k], dtype) for t in trajs]
        prms = [gfw.params(eps=p.eps, omega0=p.omega0, max_iter=1, tol=-1.0, U0=u) for p, u in zip(probs, U0s)]
        out = gfw.solve_batched(ctx(), Gs, prms)
        for p, L, u0, r in zip(probs, Ls, U0s, out):
            Uk = _np(u0).astype(np.float64)
            Ug = _np(r["U"]).astype(np.float64)
            ro = O.solve(L, p.K, p.labelled_idx, p.labels, eps=p.eps, omega0=p.omega0, max_iter=1, tol=-1.0,
                         U0=Uk, record_s=True)
            s_g = _inferred_vertices(Uk, Ug)
            diff = np.flatnonzero(s_g != ro["s"][0])
            if diff.size:
                Uhat, omega = O.fidelity(p.n, p.K, p.labelled_idx, p.labels, p.omega0)
                Gk = O.gradient(L, Uk, Uhat, omega, p.eps)
                scale = np.maximum(np.abs(Gk).max(axis=1), 1e-300)
                assert np.all(glmo_margin(Uk, Gk)[diff] <= band * scale[diff]), "non-tie vertex differs"
                say(f"[gpu]   member n={p.n}: {diff.size} rows took another minimiser")
                assert diff.size <= MAX_DIFF_SLACK[dtype] + MAX_DIFF_FRAC[dtype] * p.n
                ro = O.solve(L, p.K, p.labelled_idx, p.labels, eps=p.eps, omega0=p.omega0, max_iter=1, tol=-1.0,
                             U0=Uk, record_s=True, s_first=s_g)
            if armijo_ratio_near_power(ro["g"][0], ro["q"][0]):
                continue
            assert r["alpha_last"] == ro["alpha"][0]
            assert np.abs(Ug - ro["U"]).max() <= u_tol
            e_rel = 1e-6 if dtype == gfw.F32 else max(1e-12, p.n * p.K * 2.0 ** -53)
            assert r["objective"] == pytest.approx(ro["objective"], rel=e_rel)


def test_batch_free_running_member_against_oracle_f64():
    """One member of the batch mix solved to its stop (300 iterations or gap 1e-6) inside a
    batch, in FP64, against the oracle's free-running solve: iterations, labels, objective."""
    from oracle import oracle as O

    from gpu_helpers import oracle_sensitivity

    probs = [configs.batch_member(3, i) for i in (17, 40, 41)]
    say(f"[gpu] batch free-running f64: n={[p.n for p in probs]}")
    Gs = [gpu_graph(p.graph, p.K, p.labelled_idx, p.labels, gfw.F64) for p in probs]
    out = gfw.solve_batched(ctx(), Gs, gfw.params(eps=50.0, omega0=1000.0, max_iter=300, tol=1e-6))
    p, r = probs[0], out[0]
    ro, sens = oracle_sensitivity(p)
    dE = abs(r["objective"] - ro["objective"]) / abs(ro["objective"])
    agree = np.mean(_np(r["labels"]) == ro["labels"])
    say(f"[gpu] batch member 17 (n={p.n}, K={p.K}): iters {r['iters']}/{ro['iters']}, agreement {agree:.5f}, "
        f"rel dE {dE:.3e} (oracle sensitivity {sens:.3e})")
    assert agree >= 0.999
    assert dE <= max(1e-6, 1.5 * sens)
