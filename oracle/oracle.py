"""Python front end of the plain FP64 CPU oracle (oracle/gfw_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU leg of
the benchmark.  The product path never imports this module.  It shares no code with
the HIP library; both receive the same inputs from the `synth` generators.

Every function here is argument marshalling around the C oracle, except for the
set-up of U_0, Uhat and omega, which follows the paper's initialisation (Section 5.1:
U_0 = Uhat, unknown rows 1/K in every class; omega_i = omega0 on fidelity nodes and 0
elsewhere, Section 2).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gfw_oracle.c")
_LIB = os.path.join(_HERE, "libgfw_oracle.so")
# timing build of the same source: the row loops split over OpenMP threads, every sum
# across rows serial, so it returns bit for bit what the serial build returns
_LIB_OMP = os.path.join(_HERE, "libgfw_oracle_omp.so")

LMO_GREEDY, LMO_FULL = 0, 1
LS_ARMIJO, LS_EXACT, LS_SHORT = 0, 1, 2
STOP_MAXITER, STOP_TOL, STOP_NUMERIC = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no FP contraction, no fast-math): the serial
    build the tests use, and the OpenMP timing build of the same source."""
    base = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC"]
    for out, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp", "-DORC_OPENMP"])):
        if force or not os.path.exists(out):
            subprocess.run(base + extra + ["-o", out + ".tmp", _SRC, "-lm"], check=True, cwd=_HERE)
            os.replace(out + ".tmp", out)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("eps", C.c_double), ("omega0", C.c_double), ("max_iter", C.c_int32),
                ("tol", C.c_double), ("ls", C.c_int32), ("delta", C.c_double), ("gamma", C.c_double),
                ("lmo", C.c_int32), ("osfw", C.c_int32), ("lipschitz", C.c_double),
                ("armijo_direct", C.c_int32), ("store_f32", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("stop_reason", C.c_int32), ("gap", C.c_double),
                ("objective", C.c_double), ("alpha_last", C.c_double)]


_libs = {}


def lib(parallel: bool = False):
    """The serial build (parallel=False, the parity reference) or the OpenMP timing build."""
    path = _LIB_OMP if parallel else _LIB
    if path not in _libs:
        if not os.path.exists(path):
            build(force=True)
        L = C.CDLL(path)
        p = C.c_void_p
        L.orc_build_sym_laplacian.restype = C.c_int64
        L.orc_build_sym_laplacian.argtypes = [C.c_int64, p, p, p, p, p, p]
        L.orc_spmm.argtypes = [C.c_int64, C.c_int32, p, p, p, p, p]
        L.orc_objective.restype = C.c_double
        L.orc_objective.argtypes = [C.c_int64, C.c_int32, p, p, p, p, p, p, C.c_double]
        L.orc_gradient_from_P.argtypes = [C.c_int64, C.c_int32, p, p, p, p, C.c_double, p]
        L.orc_lmo.restype = C.c_int64
        L.orc_lmo.argtypes = [C.c_int64, C.c_int32, p, p, C.c_int, p]
        L.orc_solve.argtypes = [C.c_int64, C.c_int32, p, p, p, p, p, C.POINTER(_Params), p, p,
                                C.POINTER(_Stats), p, p, p]
        L.orc_gaussian_degrees.argtypes = [C.c_int64, C.c_int64, p, C.c_double, p]
        L.orc_gaussian_rows.argtypes = [C.c_int64, C.c_int64, p, C.c_double, p, C.c_int32, p, C.c_int64, p, p]
        L.orc_threads.restype = C.c_int
        L.orc_threads.argtypes = []
        _libs[path] = L
    return _libs[path]


def threads(parallel: bool = False) -> int:
    """Threads the row loops of a build use (1 for the serial build)."""
    return int(lib(parallel).orc_threads())


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class Operator:
    """CSR n x n operator (L_s built from W, or a user-supplied L), FP64."""

    def __init__(self, indptr, indices, data):
        self.indptr = _i64(indptr)
        self.indices = _i32(indices)
        self.data = _f64(data)
        self.n = self.indptr.shape[0] - 1

    def dense(self) -> np.ndarray:
        M = np.zeros((self.n, self.n))
        for i in range(self.n):
            for p in range(self.indptr[i], self.indptr[i + 1]):
                M[i, self.indices[p]] += self.data[p]
        return M


def sym_laplacian(indptr, indices, data) -> Operator:
    """L_s = I - D^{-1/2} W D^{-1/2} (Section 1), diagonal made explicit."""
    indptr, indices, data = _i64(indptr), _i32(indices), _f64(data)
    n = indptr.shape[0] - 1
    cap = indices.shape[0] + n
    lrp = np.zeros(n + 1, np.int64)
    lci = np.zeros(max(cap, 1), np.int32)
    lv = np.zeros(max(cap, 1), np.float64)
    nnz = lib().orc_build_sym_laplacian(n, _p(indptr), _p(indices), _p(data), _p(lrp), _p(lci), _p(lv))
    if nnz < 0:
        raise RuntimeError("orc_build_sym_laplacian failed")
    return Operator(lrp, lci[:nnz].copy(), lv[:nnz].copy())


def operator_for(graph, kind: str = "W") -> Operator:
    """kind 'W': graph holds weights, the operator is L_s; kind 'L': graph holds L itself."""
    if kind == "W":
        return sym_laplacian(graph.indptr, graph.indices, graph.data)
    return Operator(graph.indptr, graph.indices, graph.data)


def gaussian_weights(features, sigma: float):
    """The fully connected Gaussian graph of the image setting (Section 5.1) with the
    Gaussian similarity of Section 1 on every pair: w_ij = exp(-||x_i - x_j||^2 / (2 sigma^2))
    for i != j, no self-loop.  Returns the CSR (indptr, indices, data) of W holding every
    off-diagonal entry (entries that underflow are kept as zeros).  Dense: small n only."""
    x = _f64(features)
    if x.ndim == 1:
        x = x[:, None]
    n = x.shape[0]
    diff = x[:, None, :] - x[None, :, :]
    r2 = np.sum(diff * diff, axis=2)
    W = np.exp(-r2 / (2.0 * sigma * sigma))
    off = ~np.eye(n, dtype=bool)
    indptr = np.arange(n + 1, dtype=np.int64) * (n - 1)
    indices = np.nonzero(off)[1].astype(np.int32)
    return indptr, indices, W[off]


def gaussian_degrees(features, sigma: float, parallel: bool = True) -> np.ndarray:
    """Degrees d_i = sum_{j != i} w_ij of the fully connected Gaussian graph (the C oracle's
    loop over every pair; the OpenMP build splits the rows only, so it returns the serial
    build's degrees bit for bit)."""
    x = _f64(features)
    if x.ndim == 1:
        x = x[:, None]
    x = np.ascontiguousarray(x)
    n, d = x.shape
    deg = np.zeros(n)
    lib(parallel).orc_gaussian_degrees(n, d, _p(x), float(sigma), _p(deg))
    return deg


def gaussian_laplacian_rows(features, sigma: float, U, rows, deg=None, parallel: bool = True) -> np.ndarray:
    """Rows `rows` of L_s U for the fully connected Gaussian graph at any n, from the
    definitions of Section 1 (L_s = I - D^{-1/2} W D^{-1/2}, a node of degree 0 has
    d^{-1/2} = 0), every weight formed where it is used.  deg: the degrees, if known."""
    x = _f64(features)
    if x.ndim == 1:
        x = x[:, None]
    x = np.ascontiguousarray(x)
    U = np.ascontiguousarray(_f64(U))
    n, d = x.shape
    K = U.shape[1]
    if deg is None:
        deg = gaussian_degrees(x, sigma, parallel)
    deg = np.ascontiguousarray(_f64(deg))
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros((rows.shape[0], K))
    lib(parallel).orc_gaussian_rows(n, d, _p(x), float(sigma), _p(deg), K, _p(U), rows.shape[0], _p(rows), _p(out))
    return out


def spmm(L: Operator, U: np.ndarray) -> np.ndarray:
    U = _f64(U)
    n, K = U.shape
    P = np.zeros_like(U)
    lib().orc_spmm(n, K, _p(L.indptr), _p(L.indices), _p(L.data), _p(U), _p(P))
    return P


def fidelity(n: int, K: int, labelled_idx, labels, omega0: float):
    """Uhat (one-hot on fidelity nodes, 1/K elsewhere) and omega (omega0 on fidelity nodes)."""
    labelled_idx = _i32(labelled_idx)
    labels = _i32(labels)
    Uhat = np.full((n, K), 1.0 / K)
    Uhat[labelled_idx] = 0.0
    Uhat[labelled_idx, labels] = 1.0
    omega = np.zeros(n)
    omega[labelled_idx] = omega0
    return Uhat, omega


def inv_eps(eps: float) -> float:
    return 0.0 if math.isinf(eps) else 1.0 / eps


def objective(L: Operator, U, Uhat, omega, eps: float, parallel: bool = False) -> float:
    U, Uhat, omega = _f64(U), _f64(Uhat), _f64(omega)
    n, K = U.shape
    return lib(parallel).orc_objective(n, K, _p(L.indptr), _p(L.indices), _p(L.data), _p(U), _p(Uhat), _p(omega),
                               inv_eps(eps))


def gradient(L: Operator, U, Uhat, omega, eps: float) -> np.ndarray:
    U, Uhat, omega = _f64(U), _f64(Uhat), _f64(omega)
    n, K = U.shape
    P = spmm(L, U)
    G = np.zeros_like(U)
    lib().orc_gradient_from_P(n, K, _p(P), _p(U), _p(Uhat), _p(omega), inv_eps(eps), _p(G))
    return G


def lmo(U, G, mode: int = LMO_GREEDY):
    """Vertex index per row of the (G)LMO output and the number of non-binary rows."""
    U, G = _f64(U), _f64(G)
    n, K = U.shape
    s = np.zeros(n, np.int32)
    nb = lib().orc_lmo(n, K, _p(U), _p(G), mode, _p(s))
    return s, int(nb)


def default_lipschitz(L: Operator, eps: float, omega0: float) -> float:
    """Prop. 2: Lbar = lambda_max(L) + 2/eps + omega0, with lambda_max bounded above by the
    largest absolute row sum of L (Gershgorin), which keeps Lbar a Lipschitz constant of the
    gradient (the short step of eq. alphabound needs an upper bound, not the exact value)."""
    rs = np.zeros(L.n)
    np.add.at(rs, np.repeat(np.arange(L.n), np.diff(L.indptr)), np.abs(L.data))
    return float(rs.max(initial=0.0)) + 2.0 * inv_eps(eps) + omega0


def solve(L: Operator, K: int, labelled_idx, labels, eps: float = 50.0, omega0: float = 1000.0,
          max_iter: int = 30, tol: float = 1e-6, ls: int = LS_ARMIJO, delta: float = 0.5,
          gamma: float = 1e-6, lmo_mode: int = LMO_GREEDY, osfw: bool = False,
          lipschitz: float | None = None, armijo_direct: bool = False, U0=None,
          record_s: bool = False, s_first=None, store_f32: bool = False, parallel: bool = False) -> dict:
    """Greedy Frank-Wolfe (Alg. 3) with Armijo / exact / short steps; FW (Alg. 2) with
    lmo_mode=LMO_FULL; OSFW (Alg. 4) with osfw=True.  Returns U, labels, stats, history.
    store_f32 rounds U to FP32 after every update (FP64 arithmetic, FP32 storage of the
    iterate); parallel runs the OpenMP timing build (same results, bit for bit)."""
    n = L.n
    Uhat, omega = fidelity(n, K, labelled_idx, labels, omega0)
    U = Uhat.copy() if U0 is None else np.array(U0, dtype=np.float64, copy=True)
    if lipschitz is None:
        lipschitz = default_lipschitz(L, eps, omega0)
    prm = _Params(eps, omega0, max_iter, tol, ls, delta, gamma, lmo_mode, int(osfw), lipschitz,
                  int(armijo_direct), int(store_f32))
    st = _Stats()
    hist = np.full((5, max_iter + 1), np.nan)
    s_hist = np.zeros((max_iter + 1, n), np.int32) if record_s else None
    lab = np.zeros(n, np.int32)
    sf = None if s_first is None else _i32(s_first)
    if sf is not None and sf.shape != (n,):
        raise ValueError("s_first needs one vertex per node")
    rc = lib(parallel).orc_solve(n, K, _p(L.indptr), _p(L.indices), _p(L.data), _p(Uhat), _p(omega), C.byref(prm),
                         _p(U), _p(lab), C.byref(st), _p(hist), _p(s_hist), _p(sf))
    if rc != 0:
        raise RuntimeError(f"orc_solve failed ({rc})")
    out = dict(U=U, labels=lab, iters=st.iters, stop_reason=st.stop_reason, gap=st.gap,
               objective=st.objective, alpha_last=st.alpha_last,
               E=hist[0], g=hist[1], q=hist[2], alpha=hist[3], nonbinary=hist[4])
    if record_s:
        out["s"] = s_hist
    return out


def solve_problem(prob, kind: str = "W", **kw) -> dict:
    """Convenience: build the operator for a `synth.configs.Problem` and solve it."""
    L = operator_for(prob.graph, kind)
    args = dict(eps=prob.eps, omega0=prob.omega0, max_iter=prob.max_iter, tol=prob.tol)
    args.update(kw)
    return solve(L, prob.K, prob.labelled_idx, prob.labels, **args)
