"""Python binding of libgfw (include/gfw.h): argument marshalling only.

Every computation runs in the HIP library; PyTorch supplies device memory and streams.
There is no CPU fallback: if libgfw.so is missing or no gfx950 device is present, the
calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgfw.so")

GFW_OK = 0
STATUS = {0: "GFW_OK", -1: "GFW_E_INVALID_ARG", -2: "GFW_E_GRAPH", -3: "GFW_E_LABELS", -4: "GFW_E_NOMEM",
          -5: "GFW_E_HIP", -6: "GFW_E_UNSUPPORTED", -7: "GFW_E_BUDGET", -8: "GFW_E_NOT_READY",
          -9: "GFW_E_NUMERIC"}
GRAPH_W, GRAPH_L = 0, 1
F32, F64 = 0, 1
HOST, DEVICE = 0, 1
LS_ARMIJO, LS_EXACT, LS_SHORT = 0, 1, 2
LMO_GREEDY, LMO_FULL = 0, 1
STOP_MAXITER, STOP_TOL, STOP_NUMERIC = 0, 1, 2

EXPORTED = [
    "gfw_status_string", "gfw_last_error", "gfw_params_default", "gfw_check_problem", "gfw_check_params",
    "gfw_context_create", "gfw_context_destroy", "gfw_graph_create", "gfw_graph_destroy", "gfw_graph_footprint",
    "gfw_solve", "gfw_solve_batched", "gfw_objective", "gfw_spmm", "gfw_server_create", "gfw_server_submit",
    "gfw_server_poll", "gfw_server_destroy", "gfw_trace_enable", "gfw_trace_reset", "gfw_trace_get",
    "gfw_graph_tune", "gfw_graph_query", "gfw_objective_noalloc", "gfw_copy_bandwidth", "gfw_graph_create_gaussian",
]
GAUSS_AUTO, GAUSS_EXACT, GAUSS_GRID = 0, 1, 2
TUNE_LABEL_PATH, TUNE_LABEL_PLAIN_NS, TUNE_LABEL_SORTED_NS, TUNE_SORTED_WIDE_CHUNKS, TUNE_GAUSS_METHOD = 0, 1, 2, 3, 4
LABEL_PATH_AUTO, LABEL_PATH_PLAIN, LABEL_PATH_SORTED, LABEL_PATH_MEASURED = 0, 1, 2, 3
KERNEL_ROW, KERNEL_LABEL, KERNEL_FINISH, KERNEL_SPMM = 0, 1, 2, 3


class GfwError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("K", C.c_int32), ("kind", C.c_int), ("dtype", C.c_int),
                ("location", C.c_int), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("vals", C.c_void_p),
                ("n_labelled", C.c_int64), ("labelled_idx", C.c_void_p), ("labels", C.c_void_p)]


class GaussianProblem(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("K", C.c_int32), ("dtype", C.c_int), ("location", C.c_int),
                ("features", C.c_void_p), ("sigma", C.c_double), ("method", C.c_int), ("n_labelled", C.c_int64),
                ("labelled_idx", C.c_void_p), ("labels", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("eps", C.c_double), ("omega0", C.c_double), ("max_iter", C.c_int32), ("tol", C.c_double),
                ("ls", C.c_int), ("delta", C.c_double), ("gamma", C.c_double), ("lmo", C.c_int),
                ("one_shot", C.c_int32), ("lipschitz", C.c_double), ("U0", C.c_void_p), ("p_refresh", C.c_int32),
                ("incremental", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("stop_reason", C.c_int32), ("gap", C.c_double), ("objective", C.c_double),
                ("alpha_last", C.c_double)]


_lib = None


def lib():
    """Load libgfw.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2508_09738_amd/build.py")
        # torch ships its own HIP runtime under the same SONAME (libamdhip64.so.7); loading
        # torch first makes libgfw bind to that one, so the process has a single runtime.
        import torch  # noqa: F401

        L = C.CDLL(LIB_PATH)
        p = C.c_void_p
        L.gfw_status_string.restype = C.c_char_p
        L.gfw_status_string.argtypes = [C.c_int]
        L.gfw_last_error.restype = C.c_char_p
        L.gfw_last_error.argtypes = []
        L.gfw_params_default.restype = None
        L.gfw_params_default.argtypes = [C.POINTER(Params)]
        L.gfw_check_problem.argtypes = [C.POINTER(Problem)]
        L.gfw_check_params.argtypes = [C.POINTER(Params), C.c_int32]
        L.gfw_context_create.argtypes = [C.POINTER(p), C.c_int]
        L.gfw_context_destroy.argtypes = [p]
        L.gfw_graph_create.argtypes = [p, C.POINTER(Problem), C.POINTER(p), p]
        L.gfw_graph_create_gaussian.argtypes = [p, C.POINTER(GaussianProblem), C.POINTER(p), p]
        L.gfw_graph_destroy.argtypes = [p]
        L.gfw_graph_footprint.argtypes = [p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
        L.gfw_solve.argtypes = [p, p, C.POINTER(Params), p, p, p, C.POINTER(Stats), p, p]
        L.gfw_solve_batched.argtypes = [p, C.c_int32, p, p, C.c_int32, p, p, p, p]
        L.gfw_objective.argtypes = [p, p, C.POINTER(Params), p, C.POINTER(C.c_double), p]
        L.gfw_spmm.argtypes = [p, p, p, p, p]
        L.gfw_objective_noalloc.argtypes = [p, p, C.POINTER(Params), p, p, p]
        L.gfw_copy_bandwidth.argtypes = [p, C.c_size_t, C.c_int32, C.POINTER(C.c_double)]
        L.gfw_server_create.argtypes = [p, C.c_size_t, C.c_int32, C.POINTER(p)]
        L.gfw_server_submit.argtypes = [p, C.POINTER(Problem), C.POINTER(Params), C.POINTER(C.c_uint64)]
        L.gfw_server_poll.argtypes = [p, C.c_uint64, C.c_int, p, p, C.POINTER(Stats)]
        L.gfw_server_destroy.argtypes = [p]
        L.gfw_graph_tune.argtypes = [p, C.c_int, C.c_int64]
        L.gfw_graph_query.argtypes = [p, C.c_int, C.POINTER(C.c_int64)]
        L.gfw_trace_enable.argtypes = [p, C.c_int]
        L.gfw_trace_reset.argtypes = [p]
        L.gfw_trace_get.argtypes = [p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        for name in EXPORTED:
            f = getattr(L, name)
            if f.restype is None and name != "gfw_params_default":
                f.restype = C.c_int
        L.gfw_params_default.restype = None
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != GFW_OK:
        raise GfwError(status, lib().gfw_last_error().decode())


def params(eps: float = 50.0, omega0: float = 1000.0, max_iter: int = 30, tol: float = 1e-6, ls: int = LS_ARMIJO,
           delta: float = 0.5, gamma: float = 1e-6, lmo: int = LMO_GREEDY, one_shot: bool = False,
           lipschitz: float = 0.0, U0=None, p_refresh: int = 0, incremental: bool = False) -> Params:
    pr = Params()
    lib().gfw_params_default(C.byref(pr))
    pr.eps, pr.omega0, pr.max_iter, pr.tol, pr.ls = eps, omega0, max_iter, tol, ls
    pr.delta, pr.gamma, pr.lmo, pr.one_shot, pr.lipschitz = delta, gamma, lmo, int(one_shot), lipschitz
    pr.U0 = None if U0 is None else U0.data_ptr()
    pr.p_refresh = p_refresh
    pr.incremental = int(incremental)
    return pr


def _stream(stream) -> C.c_void_p:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Context:
    """A HIP device bound for the library (device must be gfx950)."""

    def __init__(self, device: int = 0):
        self.handle = C.c_void_p()
        check(lib().gfw_context_create(C.byref(self.handle), device))
        self.device = device

    def close(self):
        if self.handle:
            lib().gfw_context_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def host_problem(n, K, indptr, indices, data, labelled_idx, labels, dtype: int = F32, kind: int = GRAPH_W):
    """Builds a host-located gfw_problem_t; returns (struct, keep-alive list)."""
    indptr = np.ascontiguousarray(indptr, np.int64)
    indices = np.ascontiguousarray(indices, np.int32)
    vals = None if data is None else np.ascontiguousarray(data, np.float32 if dtype == F32 else np.float64)
    li = np.ascontiguousarray(labelled_idx, np.int32)
    lb = np.ascontiguousarray(labels, np.int32)
    pb = Problem(n, int(indices.shape[0]), K, kind, dtype, HOST, indptr.ctypes.data, indices.ctypes.data,
                 None if vals is None else vals.ctypes.data, int(li.shape[0]), li.ctypes.data, lb.ctypes.data)
    return pb, [indptr, indices, vals, li, lb]


def device_problem(n, K, indptr, indices, data, labelled_idx, labels, dtype: int = F32, kind: int = GRAPH_W):
    """Builds a device-located gfw_problem_t from torch tensors on the GPU."""
    pb = Problem(n, int(indices.shape[0]), K, kind, dtype, DEVICE, indptr.data_ptr(), indices.data_ptr(),
                 None if data is None else data.data_ptr(), int(labelled_idx.shape[0]), labelled_idx.data_ptr(),
                 labels.data_ptr())
    return pb, [indptr, indices, data, labelled_idx, labels]


class Graph:
    """A validated problem resident on the device (gfw_graph_create)."""

    def __init__(self, ctx: Context, problem: Problem, keep=None, stream=None):
        self.ctx = ctx
        self.handle = C.c_void_p()
        self.n, self.K, self.dtype = int(problem.n), int(problem.K), int(problem.dtype)
        self.nnz = int(problem.nnz)
        check(lib().gfw_graph_create(ctx.handle, C.byref(problem), C.byref(self.handle), _stream(stream)))

    @classmethod
    def from_host(cls, ctx, n, K, indptr, indices, data, labelled_idx, labels, dtype=F32, kind=GRAPH_W, stream=None):
        pb, keep = host_problem(n, K, indptr, indices, data, labelled_idx, labels, dtype, kind)
        return cls(ctx, pb, keep, stream)

    @classmethod
    def gaussian(cls, ctx, features, K, sigma, labelled_idx, labels, dtype=F32, method=GAUSS_AUTO, stream=None):
        """Fully connected Gaussian graph (gfw_graph_create_gaussian) on features (n x d): a
        host array, or a torch tensor on the device of the graph's dtype."""
        self = cls.__new__(cls)
        self.ctx = ctx
        self.handle = C.c_void_p()
        if hasattr(features, "data_ptr") and getattr(features, "is_cuda", False):
            n, d = int(features.shape[0]), int(features.shape[1])
            pb = GaussianProblem(n, d, K, dtype, DEVICE, features.data_ptr(), float(sigma), method,
                                 int(labelled_idx.shape[0]), labelled_idx.data_ptr(), labels.data_ptr())
            keep = [features, labelled_idx, labels]
        else:
            x = np.ascontiguousarray(features, np.float32 if dtype == F32 else np.float64)
            if x.ndim != 2:
                raise ValueError("features must be n x d")
            n, d = x.shape
            li = np.ascontiguousarray(labelled_idx, np.int32)
            lb = np.ascontiguousarray(labels, np.int32)
            pb = GaussianProblem(n, d, K, dtype, HOST, x.ctypes.data, float(sigma), method, int(li.shape[0]),
                                 li.ctypes.data, lb.ctypes.data)
            keep = [x, li, lb]
        self.n, self.K, self.dtype, self.nnz = int(n), int(K), int(dtype), 0
        check(lib().gfw_graph_create_gaussian(ctx.handle, C.byref(pb), C.byref(self.handle), _stream(stream)))
        del keep
        return self

    def tune(self, key: int, value: int) -> None:
        check(lib().gfw_graph_tune(self.handle, key, value))

    def query(self, key: int) -> int:
        v = C.c_int64()
        check(lib().gfw_graph_query(self.handle, key, C.byref(v)))
        return v.value

    def footprint(self):
        a, b = C.c_size_t(), C.c_size_t()
        check(lib().gfw_graph_footprint(self.handle, C.byref(a), C.byref(b)))
        return a.value, b.value

    def close(self):
        if self.handle:
            lib().gfw_graph_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def torch_dtype(self):
        import torch

        return torch.float32 if self.dtype == F32 else torch.float64


def solve(ctx: Context, g: Graph, prm: Params, want_U: bool = True, want_labels: bool = True, want_s: bool = False,
          want_stats: bool = True, want_history: bool = False, stream=None) -> dict:
    """gfw_solve; returns device tensors (U, labels, s) and host stats / history."""
    import torch

    dev = torch.device("cuda", ctx.device)
    U = torch.empty((g.n, g.K), dtype=g.torch_dtype(), device=dev) if want_U else None
    lab = torch.empty(g.n, dtype=torch.int32, device=dev) if want_labels else None
    s = torch.empty(g.n, dtype=torch.int32, device=dev) if want_s else None
    st = Stats() if want_stats else None
    hist = np.full(5 * (prm.max_iter + 1), np.nan) if want_history else None
    check(lib().gfw_solve(ctx.handle, g.handle, C.byref(prm), None if U is None else U.data_ptr(),
                          None if lab is None else lab.data_ptr(), None if s is None else s.data_ptr(),
                          None if st is None else C.byref(st),
                          None if hist is None else hist.ctypes.data, _stream(stream)))
    out = dict(U=U, labels=lab, s=s)
    if st is not None:
        out.update(iters=st.iters, stop_reason=st.stop_reason, gap=st.gap, objective=st.objective,
                   alpha_last=st.alpha_last)
    if hist is not None:
        h = hist.reshape(5, prm.max_iter + 1)
        out.update(E=h[0], g=h[1], q=h[2], alpha=h[3], nonbinary=h[4])
    return out


TRACE_OFF, TRACE_ALL, TRACE_LABEL, TRACE_ROW = 0, 1, 2, 3


def trace_enable(ctx: Context, on=True) -> None:
    """on: False/True or a trace mode (TRACE_OFF, TRACE_ALL, TRACE_LABEL: label passes only,
    TRACE_ROW: row kernels only)."""
    check(lib().gfw_trace_enable(ctx.handle, int(on)))


def trace_reset(ctx: Context) -> None:
    check(lib().gfw_trace_reset(ctx.handle))


def trace_get(ctx: Context, kernel: int):
    """(total milliseconds, launches) of a kernel class since the last reset."""
    ms, n = C.c_double(), C.c_int64()
    check(lib().gfw_trace_get(ctx.handle, kernel, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def solve_batched(ctx: Context, graphs: list, prms, want_U: bool = True, want_labels: bool = True,
                  want_stats: bool = True, stream=None) -> list:
    """gfw_solve_batched over `graphs` (one Params, or one per graph); a list of per-graph dicts."""
    import torch

    n = len(graphs)
    dev = torch.device("cuda", ctx.device)
    shared = isinstance(prms, Params)
    if shared:
        parr = prms
    else:
        parr = (Params * n)(*prms)
    gh = (C.c_void_p * n)(*[g.handle.value for g in graphs])
    Us = [torch.empty((g.n, g.K), dtype=g.torch_dtype(), device=dev) if want_U else None for g in graphs]
    labs = [torch.empty(g.n, dtype=torch.int32, device=dev) if want_labels else None for g in graphs]
    uarr = (C.c_void_p * n)(*[u.data_ptr() for u in Us]) if want_U else None
    larr = (C.c_void_p * n)(*[t.data_ptr() for t in labs]) if want_labels else None
    st = (Stats * n)() if want_stats else None
    check(lib().gfw_solve_batched(ctx.handle, n, gh, C.byref(parr) if shared else parr, int(shared), uarr, larr,
                                  st, _stream(stream)))
    out = []
    for i in range(n):
        d = dict(U=Us[i], labels=labs[i])
        if st is not None:
            d.update(iters=st[i].iters, stop_reason=st[i].stop_reason, gap=st[i].gap, objective=st[i].objective,
                     alpha_last=st[i].alpha_last)
        out.append(d)
    return out


class Server:
    """gfw_server_*: continuous-batching request server on one context."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int):
        self.ctx = ctx
        self.handle = C.c_void_p()
        check(lib().gfw_server_create(ctx.handle, int(hbm_budget_bytes), int(max_slots), C.byref(self.handle)))
        self._meta = {}

    def submit(self, n, K, indptr, indices, data, labelled_idx, labels, prm: Params, dtype: int = F32,
               kind: int = GRAPH_W, U0=None) -> int:
        """U0: optional host n x K array (warm start); it is copied at submit."""
        pb, keep = host_problem(n, K, indptr, indices, data, labelled_idx, labels, dtype, kind)
        p2 = Params.from_buffer_copy(prm)
        u0 = None
        if U0 is not None:
            u0 = np.ascontiguousarray(U0, dtype=np.float32 if dtype == F32 else np.float64)
            if u0.shape != (n, K):
                raise ValueError("U0 must be n x K")
            p2.U0 = u0.ctypes.data
        t = C.c_uint64()
        check(lib().gfw_server_submit(self.handle, C.byref(pb), C.byref(p2), C.byref(t)))
        self._meta[t.value] = (n, K, dtype)
        return t.value

    def poll(self, ticket: int, blocking: bool = True):
        """The result dict, or None when not ready (non-blocking)."""
        n, K, dtype = self._meta[ticket]
        U = np.empty((n, K), np.float32 if dtype == F32 else np.float64)
        lab = np.empty(n, np.int32)
        st = Stats()
        rc = lib().gfw_server_poll(self.handle, ticket, int(blocking), U.ctypes.data, lab.ctypes.data, C.byref(st))
        if rc == -8:
            return None
        del self._meta[ticket]
        check(rc)
        return dict(U=U, labels=lab, iters=st.iters, stop_reason=st.stop_reason, gap=st.gap, objective=st.objective,
                    alpha_last=st.alpha_last)

    def close(self):
        if self.handle:
            lib().gfw_server_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def objective(ctx: Context, g: Graph, prm: Params, U, stream=None) -> float:
    E = C.c_double()
    check(lib().gfw_objective(ctx.handle, g.handle, C.byref(prm), U.data_ptr(), C.byref(E), _stream(stream)))
    return E.value


def objective_noalloc(ctx: Context, g: Graph, prm: Params, U, E_dev, stream=None) -> None:
    """gfw_objective_noalloc: E(U) into the one-element FP64 device tensor E_dev, ordered on
    the stream, with no allocation and no synchronisation."""
    check(lib().gfw_objective_noalloc(ctx.handle, g.handle, C.byref(prm), U.data_ptr(), E_dev.data_ptr(),
                                      _stream(stream)))


def copy_bandwidth(ctx: Context, nbytes: int = 1 << 30, reps: int = 10) -> float:
    """gfw_copy_bandwidth: GB/s (read + write) of the library's streaming copy kernel."""
    v = C.c_double()
    check(lib().gfw_copy_bandwidth(ctx.handle, int(nbytes), int(reps), C.byref(v)))
    return v.value


def spmm(ctx: Context, g: Graph, U, stream=None):
    import torch

    P = torch.empty_like(U)
    check(lib().gfw_spmm(ctx.handle, g.handle, U.data_ptr(), P.data_ptr(), _stream(stream)))
    return P


def check_problem_host(n, K, indptr, indices, data, labelled_idx, labels, dtype=F32, kind=GRAPH_W) -> int:
    """gfw_check_problem on host arrays (no GPU needed); returns the status code."""
    pb, keep = host_problem(n, K, indptr, indices, data, labelled_idx, labels, dtype, kind)
    return lib().gfw_check_problem(C.byref(pb))


def check_params(prm: Params, K: int) -> int:
    return lib().gfw_check_params(C.byref(prm), K)


def last_error() -> str:
    return lib().gfw_last_error().decode()
