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


def oracle_trajectory(prob, ks, lmo=O.LMO_GREEDY, ls=O.LS_ARMIJO, parallel=False):
    """The oracle's iterates U_k for every k in ks (tol disabled), each run continued from the
    previous one: the oracle's state between iterations is U alone (it forms L U afresh each
    iteration), so chaining gives the same iterates as runs from U_0.  parallel uses the
    OpenMP timing build, which returns the serial build's iterates bit for bit."""
    L = O.operator_for(prob.graph)
    Uhat, _ = O.fidelity(prob.n, prob.K, prob.labelled_idx, prob.labels, prob.omega0)
    out, U, at = {}, Uhat.copy(), 0
    for k in sorted(set(ks)):
        if k > at:
            U = O.solve(L, prob.K, prob.labelled_idx, prob.labels, eps=prob.eps, omega0=prob.omega0, max_iter=k - at,
                        tol=-1.0, lmo_mode=lmo, ls=ls, U0=U, parallel=parallel)["U"]
            at = k
        out[k] = U.copy()
    return out


# Near-tie band of the lockstep GLMO check, relative to max_c |G_ic| of the row: rows whose
# oracle margin (second-smallest minus smallest G over the candidates) lies inside it may
# take another minimiser; elsewhere the vertices must be identical.  FP32 carries about 7
# significant digits.  In FP64 the GPU forms L U with the oracle's operations in the
# oracle's order (the same rounding, no contraction), and the gradient likewise, so its
# vertices must equal the oracle's on every row, ties included: no band.
NEAR_TIE_REL = {gfw.F32: 1e-5, gfw.F64: 0.0}


# Bound on the rows per lockstep iteration whose GLMO vertex differs from the oracle's (each
# of them a near-tie), as a fraction of the rows: FP32 near-ties within 1e-5 are common on
# image grids, whose weights take few distinct values.
MAX_DIFF_FRAC = {gfw.F32: 1e-2, gfw.F64: 0.0}
MAX_DIFF_SLACK = {gfw.F32: 4, gfw.F64: 0}


def lockstep(prob, dtype, ks, lmo=O.LMO_GREEDY, ls=O.LS_ARMIJO, u_tol=None, label="", label_path=None,
             osfw=False, traj_parallel=False, max_diff_frac=None, G=None, band=None, op_rel=0.0):
    """One GPU iteration from each oracle iterate U_k (k in ks) against one oracle iteration
    from the same point.  Rows where the GPU chose another GLMO vertex must be near-ties
    (inside NEAR_TIE_REL[dtype], or `band`) with a GPU vertex that is a minimiser up to that
    band, and their number per iteration is bounded by max_diff_frac of the rows (plus 4).
    G: a GPU graph of the same operator built otherwise (default: from prob's CSR); op_rel:
    the relative error of its products with L_s against the oracle's, which widens the FP64
    tolerances of the gap, curvature, step and objective to it."""
    L = O.operator_for(prob.graph)
    if G is None:
        G = gpu_graph(prob.graph, prob.K, prob.labelled_idx, prob.labels, dtype)
    if label_path is not None:
        G.tune(gfw.TUNE_LABEL_PATH, label_path)
    Uhat, omega = O.fidelity(prob.n, prob.K, prob.labelled_idx, prob.labels, prob.omega0)
    u_tol = u_tol if u_tol is not None else (1e-12 if dtype == gfw.F64 else 1e-5)
    # FP64 objectives: a sequential sum of the n*K per-entry terms (the oracle's) may be off by
    # up to (n*K) * 2^-53 relative to the exact sum, so the tolerance is at least that bound
    e_rel = 1e-6 if dtype == gfw.F32 else max(1e-12, prob.n * prob.K * 2.0 ** -53, op_rel)
    g_rel = 1e-5 if dtype == gfw.F32 else max(1e-10, op_rel)
    q_rel = 1e-5 if dtype == gfw.F32 else max(1e-9, op_rel)
    band = NEAR_TIE_REL[dtype] if band is None else band
    max_diff_frac = MAX_DIFF_FRAC[dtype] if max_diff_frac is None else max_diff_frac
    excluded_rows = 0
    excluded_iters = 0
    traj = oracle_trajectory(prob, ks, lmo=lmo, ls=ls, parallel=traj_parallel)
    for k in ks:
        say(f"[gpu] lockstep {label} dtype={dtype} k={k}")
        Uk = traj[k]
        Ut = torch_u(Uk, dtype)
        Uk_in = np_of(Ut).astype(np.float64)  # what the GPU starts from
        ro = O.solve(L, prob.K, prob.labelled_idx, prob.labels, eps=prob.eps, omega0=prob.omega0, max_iter=1,
                     tol=-1.0, lmo_mode=lmo, ls=ls, U0=Uk_in, record_s=True, osfw=osfw)
        rg = gfw.solve(ctx(), G, gfw.params(eps=prob.eps, omega0=prob.omega0, max_iter=1, tol=-1.0, lmo=lmo, ls=ls,
                                            one_shot=osfw, U0=Ut), want_s=True, want_history=True)
        # objective and gap of U_k
        assert rg["E"][0] == pytest.approx(ro["E"][0], rel=e_rel)
        assert rg["g"][0] == pytest.approx(ro["g"][0], rel=g_rel, abs=1e-9)
        # GLMO vertices: exact outside near-ties; inside, the GPU's choice must be near-optimal
        Gk = O.gradient(L, Uk_in, Uhat, omega, prob.eps)
        margin = glmo_margin(Uk_in, Gk, lmo)
        scale = np.maximum(np.abs(Gk).max(axis=1), 1e-300)
        near = margin <= band * scale
        s_g, s_o = np_of(rg["s"]), ro["s"][0]
        assert np.all(s_g[~near] == s_o[~near]), f"GLMO mismatch outside near-ties at k={k}"
        diff = np.flatnonzero(s_g != s_o)
        if diff.size:
            cand = (Uk_in[diff] != 0) if lmo == O.LMO_GREEDY else np.ones((diff.size, prob.K), bool)
            assert np.all(cand[np.arange(diff.size), s_g[diff]]), "GPU vertex outside the support"
            assert np.all(Gk[diff, s_g[diff]] - Gk[diff, s_o[diff]] <= band * scale[diff])
        if diff.size:
            say(f"[gpu]   k={k}: {diff.size} rows took another minimiser ({int(near.sum())} oracle near-ties)")
        assert diff.size <= MAX_DIFF_SLACK[dtype] + max_diff_frac * prob.n, f"{diff.size} rows differ at k={k}"
        excluded_rows += int(diff.size)
        if diff.size:
            # the GPU chose other minimisers on near-tie rows: the oracle's iteration with the
            # GPU's vertices is the reference for the rest of the step
            ro = O.solve(L, prob.K, prob.labelled_idx, prob.labels, eps=prob.eps, omega0=prob.omega0, max_iter=1,
                         tol=-1.0, lmo_mode=lmo, ls=ls, U0=Uk_in, record_s=True, s_first=s_g, osfw=osfw)
            assert rg["g"][0] == pytest.approx(ro["g"][0], rel=g_rel, abs=1e-9)
        # step size (exclude Armijo bounds sitting on a power of two)
        if osfw or ls != O.LS_ARMIJO or not armijo_ratio_near_power(ro["g"][0], ro["q"][0]):
            assert rg["q"][0] == pytest.approx(ro["q"][0], rel=q_rel)
            if ls == O.LS_ARMIJO or osfw:
                assert rg["alpha"][0] == ro["alpha"][0]  # a power of delta (1 for the one-shot method): exact
            else:
                assert rg["alpha"][0] == pytest.approx(ro["alpha"][0], rel=q_rel)
            Ug = np_of(rg["U"]).astype(np.float64)
            assert np.abs(Ug - ro["U"]).max() <= u_tol
            Eg = rg["objective"]
            assert Eg == pytest.approx(ro["objective"], rel=e_rel)
        else:
            excluded_iters += 1
        if osfw:
            assert rg["iters"] == ro["iters"] == 1
    say(f"[gpu] lockstep {label}: near-tie rows differing {excluded_rows}, iterations excluded {excluded_iters}")
    assert excluded_iters <= len(ks) // 2
    return excluded_rows


def oracle_sensitivity(prob, seeds=(0, 1), parallel=True):
    """How far the oracle's own free-running objective moves under perturbations of rounding
    alone: the same problem with its nodes renumbered (a different FP64 evaluation order) and
    the same problem with U stored in FP32 after every update.  Returns (oracle result,
    largest relative |E - E'| / |E|).  Oracle only: no GPU result enters it."""
    r0 = O.solve_problem(prob, parallel=parallel)
    ren = 0.0
    for s in seeds:
        p2, _ = relabelled(prob, s)
        r = O.solve_problem(p2, parallel=parallel)
        ren = max(ren, abs(r["objective"] - r0["objective"]) / abs(r0["objective"]))
    r = O.solve_problem(prob, parallel=parallel, store_f32=True)
    f32 = abs(r["objective"] - r0["objective"]) / abs(r0["objective"])
    say(f"[oracle] sensitivity of the objective: renumbered nodes {ren:.3e}, U stored in FP32 {f32:.3e}")
    return r0, max(ren, f32)
