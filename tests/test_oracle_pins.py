"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Every test here checks the oracle against something other than itself: closed forms
derived by hand from the paper's definitions, textbook/library special cases (SciPy),
brute force on tiny inputs, and the invariants the paper proves (Prop. 1-2, Thm. 1-2,
Lemma 1, Cor. 1).  No GPU is needed.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph
import scipy.sparse.linalg as spla

from oracle import oracle as O
from synth import configs, graphs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _csr(g):
    return sp.csr_matrix((g.data, g.indices, g.indptr), shape=(g.n, g.n))


def _ev(expr, eps):
    return eval(expr, {"sqrt": math.sqrt, "eps": eps, "min": min})


@pytest.fixture(scope="module", autouse=True)
def _build_oracle():
    O.build(force=False)


# ---------------------------------------------------------------------------
# Worked example (closed forms derived from eqs. gl_vv2, gradgl_vv2g, Armijo)
# ---------------------------------------------------------------------------

def _path4():
    gold = json.load(open(os.path.join(GOLDEN, "path4_worked_example.json")))
    g = graphs.path_graph(4, 2)
    return gold, O.operator_for(g)


def test_golden_closed_forms_are_consistent():
    gold, _ = _path4()
    for case in gold["cases"].values():
        for v in case.values():
            if isinstance(v, dict) and "expr" in v:
                assert _ev(v["expr"], case["eps"]) == pytest.approx(v["value"], abs=1e-15)


def test_worked_example_armijo_two_iterations():
    gold, L = _path4()
    c = gold["cases"]["armijo_eps50"]
    r = O.solve(L, 2, [0, 3], [0, 1], eps=c["eps"], omega0=1000.0, max_iter=2, tol=1e-6, record_s=True)
    assert r["E"][0] == pytest.approx(c["E0"]["value"], abs=1e-14)
    assert r["g"][0] == pytest.approx(c["g0"]["value"], abs=1e-14)
    assert r["q"][0] == pytest.approx(c["q0"]["value"], abs=1e-14)
    assert r["alpha"][0] == c["alpha0"]
    assert list(r["s"][0]) == c["s0"]
    assert r["E"][1] == pytest.approx(c["E1"]["value"], abs=1e-14)
    assert list(r["s"][1]) == c["s1"]  # the Frank-Wolfe zig-zag
    assert r["g"][1] == pytest.approx(c["g1"]["value"], abs=1e-14)
    assert r["q"][1] == pytest.approx(c["q1"]["value"], abs=1e-13)
    assert r["alpha"][1] == c["alpha1"]
    r1 = O.solve(L, 2, [0, 3], [0, 1], eps=c["eps"], omega0=1000.0, max_iter=1, tol=1e-6)
    np.testing.assert_array_equal(r1["U"], np.array(c["U1"]))
    assert r1["objective"] == pytest.approx(c["E1"]["value"], abs=1e-14)


@pytest.mark.parametrize("delta", [0.5, 0.3, 0.9])
@pytest.mark.parametrize("gamma", [1e-6, 0.25, 0.45])
def test_worked_example_armijo_parameters(delta, gamma):
    """alpha_0 = delta^j for the smallest j with a g_0 - a^2 q_0 / 2 >= gamma a g_0, i.e. the
    largest power a = delta^j with a <= 2 (1 - gamma) g_0 / q_0 (g_0, q_0 closed forms)."""
    gold, L = _path4()
    c = gold["cases"]["armijo_eps50"]
    g0, q0 = c["g0"]["value"], c["q0"]["value"]
    a = 1.0
    while a > 2 * (1 - gamma) * g0 / q0:
        a *= delta
    r = O.solve(L, 2, [0, 3], [0, 1], eps=c["eps"], omega0=1000.0, max_iter=1, tol=1e-6,
                delta=delta, gamma=gamma)
    assert r["alpha"][0] == a
    if delta == 0.5:
        # second step of the eps = 50 example: the bound 2 (1 - gamma) g_1 / q_1 decides
        r2 = O.solve(L, 2, [0, 3], [0, 1], eps=c["eps"], omega0=1000.0, max_iter=2, tol=1e-6,
                     gamma=gamma)
        b = 1.0
        while b > 2 * (1 - gamma) * c["g1"]["value"] / c["q1"]["value"]:
            b *= 0.5
        assert r2["alpha"][1] == b


def test_worked_example_exact_step_stops_after_one():
    gold, L = _path4()
    c = gold["cases"]["exact_eps50"]
    r = O.solve(L, 2, [0, 3], [0, 1], eps=c["eps"], omega0=1000.0, max_iter=5, tol=1e-6, ls=O.LS_EXACT)
    assert r["alpha"][0] == pytest.approx(c["alpha0"]["value"], rel=1e-14)
    # at the exact minimiser along D_0 the gradient is orthogonal to D_0 and S_1 = S_0,
    # so g_1 = -(1 - a) <grad E(U_1), D_0> = 0
    assert abs(r["g"][1]) < 1e-14
    assert r["iters"] == 1 and r["stop_reason"] == O.STOP_TOL


def test_worked_example_short_step():
    """Short step (eq. alphabound): alpha_0 = min(1, g_0 / (Lbar ||D_0||^2)) with ||D_0||^2 = 1 on
    the path; U_1 = (1 - a) U_0 + a S_0 and E_1 = E_0 - a g_0 + a^2 q_0 / 2 (E is quadratic), all
    closed forms.  Lbar is given (3) or left to the default, whose closed form is
    rho_max + 2/eps + omega0 with rho_max = 1 + 1/sqrt(2) + 1/2 (largest absolute row sum of L_s)."""
    gold, L = _path4()
    c = gold["cases"]["short_eps50"]
    eps = c["eps"]
    r = O.solve(L, 2, [0, 3], [0, 1], eps=eps, omega0=1000.0, max_iter=1, tol=1e-6, ls=O.LS_SHORT,
                lipschitz=c["Lbar_given"], record_s=True)
    assert list(r["s"][0]) == gold["cases"]["armijo_eps50"]["s0"]
    assert r["alpha"][0] == pytest.approx(c["alpha0_given"]["value"], rel=1e-15)
    np.testing.assert_allclose(r["U"], np.array(c["U1_given"]), rtol=0, atol=1e-15)
    assert r["objective"] == pytest.approx(c["E1_given"]["value"], abs=1e-14)
    # a Lbar small enough that g_0 / (Lbar ||D_0||^2) > 1 takes the full step
    r = O.solve(L, 2, [0, 3], [0, 1], eps=eps, omega0=1000.0, max_iter=1, tol=1e-6, ls=O.LS_SHORT, lipschitz=0.5)
    assert r["alpha"][0] == 1.0
    # the default Lbar
    r = O.solve(L, 2, [0, 3], [0, 1], eps=eps, omega0=1000.0, max_iter=1, tol=1e-6, ls=O.LS_SHORT)
    assert r["alpha"][0] == pytest.approx(c["alpha0_default"]["value"], rel=1e-14)
    assert O.default_lipschitz(L, eps, 1000.0) == pytest.approx(c["Lbar_default"]["value"], rel=1e-15)
    assert O.default_lipschitz(L, eps, 0.0) - 2.0 / eps == pytest.approx(c["rho_max"]["value"], rel=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_default_lipschitz_bounds_the_hessian(seed):
    """Prop. 2: the default Lbar (Gershgorin bound rho_max of L_s, plus 2/eps + omega0) is an
    upper bound of lambda_max(L_s) + 2/eps + omega0, the constant of the proposition; rho_max
    itself equals the largest absolute row sum computed independently with SciPy."""
    g = graphs.sbm_by_degree(300, 3, 8.0, 3.0, 50 + seed)
    L = O.operator_for(g)
    Ld = csgraph.laplacian(_csr(g).astype(np.float64), normed=True)
    lam = np.linalg.eigvalsh(Ld.toarray()).max()
    rho = np.abs(Ld).sum(axis=1).max()
    eps, om = 50.0, 1000.0
    Lbar = O.default_lipschitz(L, eps, om)
    assert Lbar == pytest.approx(rho + 2.0 / eps + om, rel=1e-14)
    assert Lbar >= lam + 2.0 / eps + om - 1e-12


def test_worked_example_osfw_takes_the_vertex():
    """One-shot FW (Alg. 4) at eps = 50, where Armijo would take alpha_0 = 1/2: U_1 = S_0 (rows
    (1,0), (1,0), (0,1), (0,1)), E_1 = 2 - sqrt(2), one update and no further iteration."""
    gold, L = _path4()
    c = gold["cases"]["osfw_eps50"]
    r = O.solve(L, 2, [0, 3], [0, 1], eps=c["eps"], omega0=1000.0, max_iter=10, tol=1e-6, osfw=True)
    assert r["alpha"][0] == c["alpha0"]
    np.testing.assert_array_equal(r["U"], np.array(c["U1"]))
    assert r["objective"] == pytest.approx(c["E1"]["value"], abs=1e-14)
    assert r["iters"] == c["iters"] and np.isnan(r["E"][1])
    assert list(r["labels"]) == [0, 0, 1, 1]


def test_worked_example_one_shot_small_eps():
    gold, L = _path4()
    c = gold["cases"]["armijo_eps0.1_one_shot"]
    r = O.solve(L, 2, [0, 3], [0, 1], eps=c["eps"], omega0=1000.0, max_iter=5, tol=1e-6)
    assert r["q"][0] == pytest.approx(c["q0"]["value"], abs=1e-13)
    assert r["alpha"][0] == 1.0
    assert list(r["labels"]) == c["U1_labels"]
    assert r["objective"] == pytest.approx(c["E1"]["value"], abs=1e-14)
    assert r["iters"] == c["iters"] and r["stop_reason"] == O.STOP_TOL
    assert set(np.unique(r["U"])) <= {0.0, 1.0}


def test_exact_tie_uses_lowest_index_and_stops():
    gold, _ = _path4()
    t = gold["tie_path3"]
    L = O.operator_for(graphs.path_graph(3, 2))
    r = O.solve(L, 2, [0, 2], [0, 1], eps=50.0, omega0=1000.0, max_iter=10, tol=1e-6)
    assert r["iters"] == t["iters"] and r["g"][0] == t["g0"]
    assert list(r["labels"]) == t["labels"]


# ---------------------------------------------------------------------------
# Graph operator (Section 1)
# ---------------------------------------------------------------------------

def _random_weighted_graph(n, p, seed, self_loops=False):
    rg = np.random.default_rng(seed)
    A = np.triu(rg.random((n, n)) < p, 1).astype(float) * rg.uniform(0.1, 2.0, (n, n))
    A = A + A.T
    if self_loops:
        A[np.arange(n), np.arange(n)] = rg.uniform(0, 1, n) * (rg.random(n) < 0.5)
    M = sp.csr_matrix(A)
    M.sort_indices()
    return M


def test_sym_laplacian_matches_scipy_normed_laplacian():
    M = _random_weighted_graph(40, 0.2, 1)
    L = O.sym_laplacian(M.indptr, M.indices, M.data)
    ref = csgraph.laplacian(M.toarray(), normed=True)
    np.testing.assert_allclose(L.dense(), ref, atol=1e-14)


def test_sym_laplacian_self_loops_and_isolated_nodes():
    M = _random_weighted_graph(30, 0.15, 2, self_loops=True).toarray()
    M[7, :] = 0.0
    M[:, 7] = 0.0  # isolated node: the reading gives row e_7
    S = sp.csr_matrix(M)
    S.sort_indices()
    L = O.sym_laplacian(S.indptr, S.indices, S.data).dense()
    d = M.sum(1)
    dm = np.where(d > 0, 1.0 / np.sqrt(np.where(d > 0, d, 1.0)), 0.0)
    ref = np.eye(30) - dm[:, None] * M * dm[None, :]
    np.testing.assert_allclose(L, ref, atol=1e-14)
    assert L[7, 7] == 1.0 and np.count_nonzero(L[7]) == 1


def test_laplacian_null_vector_and_spectrum():
    g = graphs.sbm([30, 30], 0.3, 0.05, 5)
    L = O.operator_for(g)
    d = np.asarray(_csr(g).sum(1)).ravel()
    v = np.sqrt(d)[:, None]
    np.testing.assert_allclose(O.spmm(L, v), 0.0, atol=1e-13)  # L_s D^{1/2} 1 = 0
    ev = np.linalg.eigvalsh(L.dense())
    assert ev.min() > -1e-12 and ev.max() < 2.0 + 1e-12
    # combinatorial L = D - W given as an operator annihilates constants
    Wm = _csr(g)
    Lc = (sp.diags(d) - Wm).tocsr()
    Lc.sort_indices()
    Lop = O.Operator(Lc.indptr, Lc.indices, Lc.data)
    np.testing.assert_allclose(O.spmm(Lop, np.ones((g.n, 3))), 0.0, atol=1e-12)


def test_spmm_matches_scipy():
    g = graphs.sbm([50, 50, 50], 0.2, 0.02, 6)
    L = O.operator_for(g)
    U = np.random.default_rng(0).random((g.n, 3))
    ref = sp.csr_matrix((L.data, L.indices, L.indptr), shape=(g.n, g.n)) @ U
    np.testing.assert_allclose(O.spmm(L, U), ref, atol=1e-13)


# ---------------------------------------------------------------------------
# Objective and gradient (eqs. gl_vv2, gradgl_vv2g; Prop. 2)
# ---------------------------------------------------------------------------

def _small_problem(seed=0, K=3):
    g = graphs.sbm([12, 12, 12][:K] if K <= 3 else [10] * K, 0.4, 0.05, seed)
    idx, lab = graphs.stratified_labels(g.truth, K, 0.2, seed)
    L = O.operator_for(g)
    Uhat, omega = O.fidelity(g.n, K, idx, lab, 1000.0)
    return g, L, idx, lab, Uhat, omega


def _random_sigma(n, K, rg, binary_frac=0.3, partial_frac=0.3):
    U = rg.random((n, K))
    for i in range(n):
        r = rg.random()
        if r < binary_frac:
            U[i] = 0.0
            U[i, rg.integers(K)] = 1.0
        elif r < binary_frac + partial_frac:
            U[i, rg.integers(K)] = 0.0
    return U / U.sum(1, keepdims=True)


def test_gradient_matches_central_differences():
    g, L, idx, lab, Uhat, omega = _small_problem()
    rg = np.random.default_rng(3)
    U = rg.random((g.n, 3))  # E is defined on all of R^{n x K}
    G = O.gradient(L, U, Uhat, omega, 0.7)
    h = 1e-3
    for i, c in [(0, 0), (5, 2), (17, 1), (int(idx[0]), int(lab[0]))]:
        Up = U.copy()
        Up[i, c] += h
        Um = U.copy()
        Um[i, c] -= h
        fd = (O.objective(L, Up, Uhat, omega, 0.7) - O.objective(L, Um, Uhat, omega, 0.7)) / (2 * h)
        # E is quadratic: central differences are exact up to rounding
        assert fd == pytest.approx(G[i, c], abs=1e-8)


def test_gradient_lipschitz_bound_prop2():
    g, L, idx, lab, Uhat, omega = _small_problem(1)
    eps = 0.5
    lam = np.linalg.eigvalsh(L.dense()).max()
    Lbar = lam + 2.0 / eps + 1000.0
    rg = np.random.default_rng(4)
    for _ in range(20):
        A = _random_sigma(g.n, 3, rg)
        B = _random_sigma(g.n, 3, rg)
        lhs = np.linalg.norm(O.gradient(L, A, Uhat, omega, eps) - O.gradient(L, B, Uhat, omega, eps))
        assert lhs <= Lbar * np.linalg.norm(A - B) * (1 + 1e-12)


def test_penalty_vanishes_exactly_on_binary_points():
    g, L, idx, lab, Uhat, omega = _small_problem(2)
    rg = np.random.default_rng(5)
    U = np.zeros((g.n, 3))
    U[np.arange(g.n), rg.integers(0, 3, g.n)] = 1.0
    e_pen = O.objective(L, U, Uhat, omega, 1e-3)
    e_nopen = O.objective(L, U, Uhat, omega, math.inf)
    assert e_pen == e_nopen


def test_diameter_prop1():
    # max ||A - B||_F^2 over vertex pairs of Sigma is 2n (attained by disjoint supports)
    n, K = 3, 3
    verts = [np.eye(K)[list(c)] for c in itertools.product(range(K), repeat=n)]
    best = max(np.sum((A - B) ** 2) for A in verts for B in verts)
    assert best == 2 * n


# ---------------------------------------------------------------------------
# Linear minimisation oracles (Section 4): brute force over all vertices
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mode", [O.LMO_GREEDY, O.LMO_FULL])
@pytest.mark.parametrize("seed", range(6))
def test_lmo_is_brute_force_optimal(mode, seed):
    rg = np.random.default_rng(100 + seed)
    n, K = 5, 3
    U = _random_sigma(n, K, rg, 0.3, 0.4)
    G = rg.standard_normal((n, K))
    if seed % 2:
        G = np.round(G)  # force ties
    s, nb = O.lmo(U, G, mode)
    assert nb == sum(1 for i in range(n) if not set(U[i]) <= {0.0, 1.0})
    best = math.inf
    for combo in itertools.product(range(K), repeat=n):
        ok = True
        for i, c in enumerate(combo):
            binary = set(U[i]) <= {0.0, 1.0}
            if mode == O.LMO_GREEDY and binary and U[i, c] != 1.0:
                ok = False
            if mode == O.LMO_GREEDY and not binary and U[i, c] == 0.0:
                ok = False
        if ok:
            best = min(best, sum(G[i, c] for i, c in enumerate(combo)))
    got = sum(G[i, s[i]] for i in range(n))
    assert got == pytest.approx(best, abs=1e-12)
    for i in range(n):  # lowest index among the minimisers of each row
        binary = set(U[i]) <= {0.0, 1.0}
        if mode == O.LMO_GREEDY and binary:
            assert U[i, s[i]] == 1.0
            continue
        allowed = [c for c in range(K) if mode == O.LMO_FULL or U[i, c] != 0.0]
        m = min(G[i, c] for c in allowed)
        assert s[i] == min(c for c in allowed if G[i, c] == m)


# ---------------------------------------------------------------------------
# Trajectory invariants (Alg. 3, eqs. Armijo, Lemma 1, Thm. 2, Prop. 1)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def sbm_run():
    prob = configs.sbm_small(seed=0, n_per=100)
    L = O.operator_for(prob.graph)
    r = O.solve(L, prob.K, prob.labelled_idx, prob.labels, eps=50.0, omega0=1000.0, max_iter=60,
                tol=-1.0, record_s=True)
    return prob, L, r


def test_rows_stay_on_simplex_and_labelled_rows_frozen(sbm_run):
    prob, L, r = sbm_run
    U = r["U"]
    assert U.min() >= 0.0
    np.testing.assert_allclose(U.sum(1), 1.0, atol=1e-12)
    Uhat, _ = O.fidelity(prob.n, prob.K, prob.labelled_idx, prob.labels, 1000.0)
    np.testing.assert_array_equal(U[prob.labelled_idx], Uhat[prob.labelled_idx])


def test_armijo_sufficient_decrease_and_monotone_objective(sbm_run):
    prob, L, r = sbm_run
    E, g, q, a = r["E"], r["g"], r["q"], r["alpha"]
    k = r["iters"]
    assert np.all(g[:k] >= -1e-12)
    for t in range(k - 1):
        # E_{t+1} is evaluated from its definition at U_{t+1}
        assert E[t] - E[t + 1] >= 1e-6 * a[t] * g[t] - 1e-10
        # E is quadratic, so the change equals a g - a^2 q / 2 (pins the curvature q)
        assert E[t] - E[t + 1] == pytest.approx(a[t] * g[t] - 0.5 * a[t] ** 2 * q[t], abs=1e-9)
        j = -math.log2(a[t])
        assert j == int(j) and j >= 0


def test_armijo_is_the_largest_admissible_power(sbm_run):
    prob, L, r = sbm_run
    for t in range(r["iters"]):
        a, g, q = r["alpha"][t], r["g"][t], r["q"][t]
        assert a * g - 0.5 * a * a * q >= 1e-6 * a * g
        if a < 1.0:
            b = 2 * a
            assert b * g - 0.5 * b * b * q < 1e-6 * b * g


def test_armijo_direct_evaluation_gives_same_steps():
    prob = configs.sbm_small(seed=1, n_per=60)
    L = O.operator_for(prob.graph)
    a = O.solve(L, prob.K, prob.labelled_idx, prob.labels, max_iter=25, tol=-1.0)
    b = O.solve(L, prob.K, prob.labelled_idx, prob.labels, max_iter=25, tol=-1.0, armijo_direct=True)
    np.testing.assert_array_equal(a["alpha"], b["alpha"])
    np.testing.assert_allclose(a["U"], b["U"], atol=1e-13)


def test_lemma1_step_lower_bound(sbm_run):
    prob, L, r = sbm_run
    lam = np.linalg.eigvalsh(L.dense()).max()
    Lc = lam + 2.0 / 50.0 + 1000.0  # Prop. 2 constant
    s_hist = r["s"]
    U = O.fidelity(prob.n, prob.K, prob.labelled_idx, prob.labels, 1000.0)[0]
    for t in range(r["iters"]):
        S = np.eye(prob.K)[s_hist[t]]
        D2 = np.sum((S - U) ** 2)
        lower = min(1.0, 2 * 0.5 * (1 - 1e-6) * r["g"][t] / (Lc * D2))
        assert r["alpha"][t] >= lower * (1 - 1e-12)
        U = (1 - r["alpha"][t]) * U + r["alpha"][t] * S


def test_theorem2_gap_bound(sbm_run):
    prob, L, r = sbm_run
    lam = np.linalg.eigvalsh(L.dense()).max()
    Lc = lam + 2.0 / 50.0 + 1000.0
    rho = 1e-6 * min(1.0, 2 * 0.5 * (1 - 1e-6))
    E0 = r["E"][0]  # E* >= 0 on Sigma (L_s is PSD, the penalty and fidelity are >= 0)
    for T in range(1, r["iters"] + 1):
        gstar = np.min(r["g"][:T])
        bound = max(math.sqrt(Lc * 2 * prob.n * E0 / (rho * T)), 2 * E0 / T)
        assert gstar <= bound


def test_trajectory_independent_of_omega0():
    """From U_0 = Uhat the fidelity rows are binary, GLMO keeps them, and the fidelity
    term and its gradient stay exactly zero (the omega0-invariance of Fig. 2)."""
    prob = configs.sbm_small(seed=2, n_per=80)
    L = O.operator_for(prob.graph)
    runs = [O.solve(L, prob.K, prob.labelled_idx, prob.labels, omega0=w, max_iter=40, tol=-1.0)
            for w in (10.0, 1000.0, 1e4)]
    for r in runs[1:]:
        np.testing.assert_array_equal(r["U"], runs[0]["U"])
        np.testing.assert_array_equal(r["alpha"], runs[0]["alpha"])


# ---------------------------------------------------------------------------
# Closed forms: iteration 0 (weighted vote), one-shot regime (Cor. 1), harmonic limit
# ---------------------------------------------------------------------------

def _weighted_vote(g, idx, lab, K):
    """argmax_c sum_{l labelled, y_l = c} w_il d_l^{-1/2}, lowest index on ties, with the
    margin between the best two classes."""
    W = _csr(g)
    d = np.asarray(W.sum(1)).ravel()
    Y = np.zeros((g.n, K))
    Y[idx, lab] = d[idx] ** -0.5
    V = W @ Y
    srt = np.sort(V, axis=1)
    return np.argmax(V, axis=1), srt[:, -1] - srt[:, -2]


def test_iteration0_is_the_weighted_vote():
    prob = configs.sbm_small(seed=3, n_per=150)
    L = O.operator_for(prob.graph)
    r = O.solve(L, prob.K, prob.labelled_idx, prob.labels, max_iter=1, tol=-1.0, record_s=True)
    vote, margin = _weighted_vote(prob.graph, prob.labelled_idx, prob.labels, prob.K)
    s0 = r["s"][0]
    unl = np.setdiff1d(np.arange(prob.n), prob.labelled_idx)
    clear = unl[margin[unl] > 1e-9]
    np.testing.assert_array_equal(s0[clear], vote[clear])
    W = _csr(prob.graph)
    has_lab_nbr = np.asarray(W[:, prob.labelled_idx].sum(1)).ravel() > 0
    tied = unl[~has_lab_nbr[unl]]  # no labelled neighbour: every column ties exactly
    assert tied.size > 0
    np.testing.assert_array_equal(s0[tied], 0)


def test_one_shot_regime_cor1_equals_osfw_and_vote():
    prob = configs.sbm_small(seed=4, n_per=40)
    L = O.operator_for(prob.graph)
    Ld = L.dense()
    rho_max = np.abs(Ld).sum(1).max()
    eps_tilde = 1.0 / (prob.K * (rho_max + 1000.0))
    Dw = np.zeros(prob.n)
    Dw[prob.labelled_idx] = 1000.0
    eps_bar = 2.0 / np.linalg.eigvalsh(Ld + np.diag(Dw)).max()
    eps = 0.5 * min(eps_tilde, eps_bar)
    gfw = O.solve(L, prob.K, prob.labelled_idx, prob.labels, eps=eps, max_iter=30, tol=1e-6)
    osfw = O.solve(L, prob.K, prob.labelled_idx, prob.labels, eps=eps, max_iter=30, tol=1e-6, osfw=True)
    assert gfw["iters"] == 1 and gfw["alpha"][0] == 1.0 and gfw["stop_reason"] == O.STOP_TOL
    np.testing.assert_array_equal(gfw["U"], osfw["U"])
    vote, margin = _weighted_vote(prob.graph, prob.labelled_idx, prob.labels, prob.K)
    unl = np.setdiff1d(np.arange(prob.n), prob.labelled_idx)
    clear = unl[margin[unl] > 1e-9]
    np.testing.assert_array_equal(gfw["labels"][clear], vote[clear])
    # Thm. 2 proof: below eps_tilde the GLMO and the classic LMO agree, so FW = GFW
    fw = O.solve(L, prob.K, prob.labelled_idx, prob.labels, eps=eps, max_iter=30, tol=1e-6,
                 lmo_mode=O.LMO_FULL)
    np.testing.assert_array_equal(fw["U"], gfw["U"])


def test_harmonic_limit_without_penalty():
    """eps = +inf and the combinatorial L = D - W: E is convex, the constrained minimiser
    is the harmonic extension U_u = -L_uu^{-1} L_ul Y_l, and the FW gap bounds E - E*."""
    g = graphs.sbm([15, 15, 15], 0.35, 0.08, 7)
    K = 3
    idx, lab = graphs.stratified_labels(g.truth, K, 0.2, 7)
    W = _csr(g)
    d = np.asarray(W.sum(1)).ravel()
    Lc = (sp.diags(d) - W).tocsr()
    Lc.sort_indices()
    Lop = O.Operator(Lc.indptr, Lc.indices, Lc.data)
    r = O.solve(Lop, K, idx, lab, eps=math.inf, max_iter=3000, tol=1e-12, ls=O.LS_EXACT)
    unl = np.setdiff1d(np.arange(g.n), idx)
    Y = np.zeros((g.n, K))
    Y[idx, lab] = 1.0
    Uu = spla.spsolve(Lc[unl][:, unl].tocsc(), -(Lc[unl][:, idx] @ Y[idx]))
    Ustar = Y.copy()
    Ustar[unl] = Uu
    Estar = 0.5 * np.sum(Ustar * (Lc @ Ustar))
    assert r["objective"] >= Estar - 1e-10
    gmin = np.nanmin(r["g"])
    assert r["objective"] - Estar <= gmin + 1e-10
    # textbook FW rate for a convex objective: E_T - E* <= 2 L diam^2 / (T + 2), diam^2 = 2n
    lam = np.linalg.eigvalsh(Lc.toarray()).max()
    assert r["objective"] - Estar <= 2 * lam * 2 * g.n / (r["iters"] + 2)
    assert (r["objective"] - Estar) / Estar < 1e-3


# ---------------------------------------------------------------------------
# Thm. 1: for eps <= eps_bar every local minimiser is binary (brute force)
# ---------------------------------------------------------------------------

def test_theorem1_binary_minimisers_small_eps():
    g = graphs.sbm([4, 4], 0.7, 0.15, 11)
    K = 2
    idx, lab = np.array([0, 5], np.int32), g.truth[[0, 5]].astype(np.int32)
    L = O.operator_for(g)
    Uhat, omega = O.fidelity(g.n, K, idx, lab, 10.0)
    eps_bar = 2.0 / np.linalg.eigvalsh(L.dense() + np.diag(omega)).max()
    eps = 0.9 * eps_bar
    r = O.solve(L, K, idx, lab, eps=eps, omega0=10.0, max_iter=200, tol=1e-12)
    U = r["U"]
    assert set(np.unique(U)) <= {0.0, 1.0}
    # global minimum over the vertices (= over Sigma, since E is concave here)
    best = math.inf
    for combo in itertools.product(range(K), repeat=g.n):
        V = np.eye(K)[list(combo)]
        best = min(best, O.objective(L, V, Uhat, omega, eps))
    assert r["objective"] >= best - 1e-12
    rg = np.random.default_rng(0)
    for _ in range(200):
        V = _random_sigma(g.n, K, rg, 0.0, 0.0)
        assert O.objective(L, V, Uhat, omega, eps) >= best - 1e-12


# ---------------------------------------------------------------------------
# Recovery on a cleanly separated SBM (the small SBM workload)
# ---------------------------------------------------------------------------

@pytest.mark.slow
def test_sbm_small_recovery():
    prob = configs.sbm_small(seed=0)
    L = O.operator_for(prob.graph)
    r = O.solve(L, prob.K, prob.labelled_idx, prob.labels, max_iter=prob.max_iter, tol=prob.tol)
    acc = np.mean(r["labels"] == prob.graph.truth)
    assert acc >= 0.98


def test_first_iteration_vertices_override():
    """s_first replaces the (G)LMO's vertices of the first iteration and nothing else: with
    the oracle's own vertices the run is unchanged; with other vertices the update still
    moves every non-kept row to (1 - a) u_i + a e_{s_i} and records the given vertices."""
    prob = configs.sbm_small(4, n_per=60)
    L = O.operator_for(prob.graph)
    base = O.solve(L, prob.K, prob.labelled_idx, prob.labels, max_iter=3, tol=-1, record_s=True)
    same = O.solve(L, prob.K, prob.labelled_idx, prob.labels, max_iter=3, tol=-1, record_s=True,
                   s_first=base["s"][0])
    np.testing.assert_array_equal(base["U"], same["U"])
    Uhat, _ = O.fidelity(prob.n, prob.K, prob.labelled_idx, prob.labels, prob.omega0)
    other = (base["s"][0] + 1) % prob.K
    lab = np.asarray(prob.labelled_idx)
    other[lab] = np.asarray(prob.labels)  # labelled rows are binary: the GLMO keeps them
    r = O.solve(L, prob.K, prob.labelled_idx, prob.labels, max_iter=1, tol=-1, record_s=True, s_first=other)
    np.testing.assert_array_equal(r["s"][0], other)
    a = r["alpha"][0]
    expect = (1 - a) * Uhat
    expect[np.arange(prob.n), other] += a
    expect[lab] = Uhat[lab]
    np.testing.assert_allclose(r["U"], expect, rtol=0, atol=1e-15)


def test_warm_start_moves_only_new_rows():
    """Section 4, closing remarks: warm-started from a point whose old rows are the binary
    solution of the old network, GFW keeps those rows (the GLMO returns a binary row's own
    vertex, so its direction is zero) and only the new rows change."""
    old, full = configs.grown_sbm(n_old=600, n_new=40)
    r_old = O.solve_problem(old, max_iter=200)
    n_old, K = old.n, old.K
    U0 = np.full((full.n, K), 1.0 / K)
    U0[:n_old] = 0.0
    U0[np.arange(n_old), r_old["labels"]] = 1.0
    L = O.operator_for(full.graph)
    r = O.solve(L, K, full.labelled_idx, full.labels, max_iter=60, tol=-1, U0=U0, record_s=True)
    np.testing.assert_array_equal(r["U"][:n_old], U0[:n_old])
    np.testing.assert_array_equal(r["s"][:r["iters"], :n_old],
                                  np.broadcast_to(r_old["labels"], (r["iters"], n_old)))
    assert np.all(r["U"][n_old:] != U0[n_old:])  # every new row moved


# ---------------------------------------------------------------------------
# Fully connected Gaussian graphs (Section 1's similarity on every pair; Section 5.1)
# ---------------------------------------------------------------------------

def test_gaussian_weights_closed_form():
    # points 0, 1, 3 on a line: squared distances 1, 9, 4
    ip, ix, w = O.gaussian_weights(np.array([[0.0], [1.0], [3.0]]), 1.0)
    W = sp.csr_matrix((w, ix, ip), shape=(3, 3)).toarray()
    e_half, e_2, e_9half = 0.6065306597126334, 0.1353352832366127, 0.011108996538242306  # e^-0.5, e^-2, e^-4.5
    np.testing.assert_allclose(W, [[0, e_half, e_9half], [e_half, 0, e_2], [e_9half, e_2, 0]], rtol=1e-15)
    # sigma = 2 divides every exponent by 4 (sigma enters squared)
    ip, ix, w = O.gaussian_weights(np.array([[0.0], [1.0], [3.0]]), 2.0)
    W = sp.csr_matrix((w, ix, ip), shape=(3, 3)).toarray()
    np.testing.assert_allclose(W[0, 1], 0.8824969025845955, rtol=1e-15)  # e^-(1/8)
    np.testing.assert_allclose(W[0, 2], 0.32465246735834974, rtol=1e-15)  # e^-(9/8)
    # in the plane the squared distance sums the coordinates: (0,0)-(3,4) is at distance 5
    ip, ix, w = O.gaussian_weights(np.array([[0.0, 0.0], [3.0, 4.0]]), 5.0)
    np.testing.assert_allclose(w, [0.6065306597126334] * 2, rtol=1e-15)  # e^-(25/50)


def test_gaussian_graph_invariants():
    rg = np.random.default_rng(3)
    x = rg.standard_normal((50, 3))
    ip, ix, w = O.gaussian_weights(x, 0.8)
    W = sp.csr_matrix((w, ix, ip), shape=(50, 50)).toarray()
    assert np.all(np.diag(W) == 0.0) and np.all(W[~np.eye(50, dtype=bool)] > 0.0)
    np.testing.assert_array_equal(W, W.T)
    # a translation of every point leaves W unchanged; a permutation of the points permutes it
    ip2, ix2, w2 = O.gaussian_weights(x + np.array([5.0, -2.0, 0.25]), 0.8)
    np.testing.assert_allclose(sp.csr_matrix((w2, ix2, ip2), shape=(50, 50)).toarray(), W, atol=1e-13)
    perm = rg.permutation(50)
    ip3, ix3, w3 = O.gaussian_weights(x[perm], 0.8)
    np.testing.assert_array_equal(sp.csr_matrix((w3, ix3, ip3), shape=(50, 50)).toarray(), W[np.ix_(perm, perm)])
    # L_s of the graph: D^{1/2} 1 spans its null space, spectrum in [0, 2]
    L = O.sym_laplacian(ip, ix, w)
    v = np.sqrt(W.sum(1))[:, None]
    np.testing.assert_allclose(O.spmm(L, v), 0.0, atol=1e-13)
    ev = np.linalg.eigvalsh(L.dense())
    assert ev.min() > -1e-12 and ev.max() < 2.0 + 1e-12


def test_gaussian_constant_features_give_the_complete_graph():
    # w_ij = 1 for every pair: W = J - I, d = n - 1, L_s = I - (J - I) / (n - 1)
    n = 7
    ip, ix, w = O.gaussian_weights(np.full((n, 2), 0.3), 0.1)
    np.testing.assert_array_equal(w, np.ones(n * (n - 1)))
    L = O.sym_laplacian(ip, ix, w).dense()
    ref = np.eye(n) - (np.ones((n, n)) - np.eye(n)) / (n - 1)
    np.testing.assert_allclose(L, ref, atol=1e-15)


def test_gaussian_rows_match_the_dense_operator():
    # the blocked row evaluation against the C oracle's L_s of the dense CSR, on every row
    rg = np.random.default_rng(4)
    x = rg.random((300, 3))
    U = rg.random((300, 4))
    ip, ix, w = O.gaussian_weights(x, 0.15)
    ref = O.spmm(O.sym_laplacian(ip, ix, w), U)
    for parallel in (False, True):
        got = O.gaussian_laplacian_rows(x, 0.15, U, np.arange(300), parallel=parallel)
        np.testing.assert_allclose(got, ref, atol=1e-13)
    np.testing.assert_array_equal(O.gaussian_degrees(x, 0.15, parallel=False), O.gaussian_degrees(x, 0.15))
    # far clusters: their weights underflow to 0 and L_s splits into the two blocks
    x2 = np.concatenate([rg.random((20, 2)), 1e3 + rg.random((20, 2))])
    ip, ix, w = O.gaussian_weights(x2, 0.5)
    Ld = O.sym_laplacian(ip, ix, w).dense()
    assert np.all(Ld[:20, 20:] == 0.0) and np.all(Ld[20:, :20] == 0.0)
    La = O.sym_laplacian(*O.gaussian_weights(x2[:20], 0.5)).dense()
    np.testing.assert_allclose(Ld[:20, :20], La, atol=1e-15)
