"""Helpers shared by the GPU tests: one synthetic instance handed to both the oracle and
the HIP library, and comparisons with near-tie accounting."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_09738_amd import gfw


def say(*a):
    """Print and flush, so that the case under test is named before any GPU step."""
    print(*a, flush=True)
    sys.stdout.flush()


_ctx = None


def ctx():
    global _ctx
    if _ctx is None:
        _ctx = gfw.Context(0)
    return _ctx


def gpu_graph(graph, K, idx, lab, dtype=gfw.F32, kind=gfw.GRAPH_W, data="graph"):
    data = graph.data if data == "graph" else data
    return gfw.Graph.from_host(ctx(), graph.n, K, graph.indptr, graph.indices, data, idx, lab, dtype, kind)


def torch_u(U, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(U), dtype=torch.float32 if dtype == gfw.F32 else torch.float64,
                        device="cuda")


def glmo_margin(U, G, mode=O.LMO_GREEDY):
    """Per row: gap between the smallest and second smallest G over the GLMO's candidate set
    (inf where there is a single candidate or the row is kept as binary)."""
    binary = np.all((U == 0) | (U == 1), axis=1)
    cand = (U != 0) if mode == O.LMO_GREEDY else np.ones(U.shape, dtype=bool)
    Gm = np.where(cand, G, np.inf)
    if U.shape[1] >= 2:
        two = np.partition(Gm, 1, axis=1)[:, :2]
        with np.errstate(invalid="ignore"):
            m = two[:, 1] - two[:, 0]
    else:
        m = np.full(U.shape[0], np.inf)
    m[cand.sum(axis=1) < 2] = np.inf
    if mode == O.LMO_GREEDY:
        m[binary] = np.inf
    return m


def armijo_ratio_near_power(g, q, gamma=1e-6, delta=0.5, rel=1e-6):
    """True if the Armijo bound 2 (1 - gamma) g / q lies within `rel` of a power of delta."""
    if not (q > 0):
        return False
    r = 2 * (1 - gamma) * g / q
    if r >= 1:
        return abs(r - 1) <= rel
    j = math.log(r) / math.log(delta)
    for jj in (math.floor(j), math.ceil(j)):
        if abs(delta ** jj - r) <= rel * r:
            return True
    return False


def relabelled(prob, seed):
    """The same problem with its nodes renumbered by a random permutation (an equivalent
    problem whose FP64 evaluation order differs).  Returns (problem, perm) with perm[i] the
    new index of node i."""
    import scipy.sparse as sp

    from synth import configs, graphs

    g = prob.graph
    n = g.n
    perm = np.random.default_rng(seed).permutation(n)
    inv = np.argsort(perm)
    W = sp.csr_matrix((g.data, g.indices, g.indptr), shape=(n, n))
    Pm = sp.csr_matrix((np.ones(n), (perm, np.arange(n))), shape=(n, n))
    W2 = (Pm @ W @ Pm.T).tocsr()
    W2.sort_indices()
    g2 = graphs.Graph(n, g.K, W2.indptr.astype(np.int64), W2.indices.astype(np.int32), W2.data, g.truth[inv])
    idx2 = perm[prob.labelled_idx].astype(np.int32)
    o = np.argsort(idx2)
    p2 = configs.Problem(g2, idx2[o], prob.labels[o], prob.K, prob.dtype, prob.eps, prob.omega0, prob.max_iter,
                         prob.tol)
    return p2, perm


def oracle_order_spread(prob, seeds=(0, 1, 2)):
    """Largest |E - E'| / |E| between the oracle's free-running result and its results on
    relabelled copies of the problem: the spread that rounding-level tie breaks alone give."""
    r0 = O.solve_problem(prob)
    worst = 0.0
    for s in seeds:
        p2, _ = relabelled(prob, s)
        r = O.solve_problem(p2)
        worst = max(worst, abs(r["objective"] - r0["objective"]) / abs(r0["objective"]))
    return r0, worst


def np_of(t):
    return t.detach().cpu().numpy()


def lockstep(prob, dtype, ks, lmo=O.LMO_GREEDY, ls=O.LS_ARMIJO, u_tol=None, label="", label_path=None):
    L = O.operator_for(prob.graph)
    G = gpu_graph(prob.graph, prob.K, prob.labelled_idx, prob.labels, dtype)
    if label_path is not None:
        G.tune(gfw.TUNE_LABEL_PATH, label_path)
    Uhat, omega = O.fidelity(prob.n, prob.K, prob.labelled_idx, prob.labels, prob.omega0)
    u_tol = u_tol if u_tol is not None else (1e-12 if dtype == gfw.F64 else 1e-5)
    # FP64 objectives: a sequential sum of the n*K per-entry terms (the oracle's) may be off by
    # up to (n*K) * 2^-53 relative to the exact sum, so the tolerance is at least that bound
    e_rel = 1e-6 if dtype == gfw.F32 else max(1e-12, prob.n * prob.K * 2.0 ** -53)
    excluded_rows = 0
    excluded_iters = 0
    for k in ks:
        say(f"[gpu] lockstep {label} dtype={dtype} k={k}")
        if k == 0:
            Uk = Uhat.copy()
        else:
            Uk = O.solve(L, prob.K, prob.labelled_idx, prob.labels, eps=prob.eps, omega0=prob.omega0, max_iter=k,
                         tol=-1.0, lmo_mode=lmo, ls=ls)["U"]
        Ut = torch_u(Uk, dtype)
        Uk_in = np_of(Ut).astype(np.float64)  # what the GPU starts from
        ro = O.solve(L, prob.K, prob.labelled_idx, prob.labels, eps=prob.eps, omega0=prob.omega0, max_iter=1,
                     tol=-1.0, lmo_mode=lmo, ls=ls, U0=Uk_in, record_s=True)
        rg = gfw.solve(ctx(), G, gfw.params(eps=prob.eps, omega0=prob.omega0, max_iter=1, tol=-1.0, lmo=lmo, ls=ls,
                                            U0=Ut), want_s=True, want_history=True)
        # objective and gap of U_k
        assert rg["E"][0] == pytest.approx(ro["E"][0], rel=e_rel)
        assert rg["g"][0] == pytest.approx(ro["g"][0], rel=1e-5 if dtype == gfw.F32 else 1e-10, abs=1e-9)
        # GLMO vertices: exact outside near-ties; inside, the GPU's choice must be near-optimal
        Gk = O.gradient(L, Uk_in, Uhat, omega, prob.eps)
        margin = glmo_margin(Uk_in, Gk, lmo)
        scale = np.abs(Gk).max(axis=1)
        near = margin <= 1e-5 * np.maximum(scale, 1e-300)
        s_g, s_o = np_of(rg["s"]), ro["s"][0]
        assert np.all(s_g[~near] == s_o[~near]), f"GLMO mismatch outside near-ties at k={k}"
        diff = np.flatnonzero(s_g != s_o)
        for i in diff:
            assert Gk[i, s_g[i]] - Gk[i, s_o[i]] <= 1e-5 * max(scale[i], 1e-300)
        excluded_rows += int(diff.size)
        if diff.size:
            # the GPU chose other minimisers on near-tie rows: the oracle's iteration with the
            # GPU's vertices is the reference for the rest of the step
            ro = O.solve(L, prob.K, prob.labelled_idx, prob.labels, eps=prob.eps, omega0=prob.omega0, max_iter=1,
                         tol=-1.0, lmo_mode=lmo, ls=ls, U0=Uk_in, record_s=True, s_first=s_g)
            assert rg["g"][0] == pytest.approx(ro["g"][0], rel=1e-5 if dtype == gfw.F32 else 1e-10, abs=1e-9)
        # step size (exclude Armijo bounds sitting on a power of two)
        if not armijo_ratio_near_power(ro["g"][0], ro["q"][0]):
            assert rg["q"][0] == pytest.approx(ro["q"][0], rel=1e-5 if dtype == gfw.F32 else 1e-9)
            if ls == O.LS_ARMIJO:
                assert rg["alpha"][0] == ro["alpha"][0]  # a power of delta: exact
            else:
                assert rg["alpha"][0] == pytest.approx(ro["alpha"][0], rel=1e-5 if dtype == gfw.F32 else 1e-9)
            Ug = np_of(rg["U"]).astype(np.float64)
            assert np.abs(Ug - ro["U"]).max() <= u_tol
            Eg = rg["objective"]
            assert Eg == pytest.approx(ro["objective"], rel=e_rel)
        else:
            excluded_iters += 1
    say(f"[gpu] lockstep {label}: near-tie rows differing {excluded_rows}, iterations excluded {excluded_iters}")
    assert excluded_iters <= len(ks) // 2
