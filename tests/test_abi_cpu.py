"""Host-only checks of the C ABI: the library loads, exports every declared symbol, and
every argument error is reported from the host with the documented status code."""
import math
import os
import re

import numpy as np
import pytest

from paper_2508_09738_amd import gfw
from synth import graphs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    return gfw.lib()


def test_every_declared_symbol_is_exported(L):
    decl = open(os.path.join(ROOT, "include", "gfw.h")).read()
    names = sorted(set(re.findall(r"^GFW_API [^;]*?\b(gfw_\w+)\(", decl, flags=re.M)))
    assert len(names) >= 18
    assert sorted(gfw.EXPORTED) == names
    for nm in names:
        assert hasattr(L, nm), nm


def test_status_strings(L):
    for code, name in gfw.STATUS.items():
        assert L.gfw_status_string(code)
    assert L.gfw_status_string(12345) == b"unknown status"


def _path_graph():
    g = graphs.path_graph(4, 2)
    return g.n, 2, g.indptr, g.indices, g.data, [0, 3], [0, 1]


def _check(**over):
    n, K, ip, ix, w, li, lb = _path_graph()
    args = dict(n=n, K=K, indptr=np.array(ip), indices=np.array(ix), data=None if w is None else np.array(w),
                labelled_idx=li, labels=lb, dtype=gfw.F64, kind=gfw.GRAPH_W)
    args.update(over)
    return gfw.check_problem_host(**args)


def test_valid_problem_passes():
    assert _check() == gfw.GFW_OK
    assert _check(data=None) == gfw.GFW_OK  # unit weights
    assert _check(dtype=gfw.F32) == gfw.GFW_OK


@pytest.mark.parametrize("case,code", [
    ("K1", -1), ("n0", -1), ("Kbig", -6), ("unsorted", -2), ("duplicate", -2), ("col_range", -2),
    ("negative", -2), ("nan", -2), ("inf", -2), ("asym_pattern", -2), ("asym_value", -2),
    ("rp0", -2), ("rpn", -2), ("rp_decreasing", -2), ("label_range", -3), ("label_class", -3),
    ("label_repeat", -3), ("kindL_novals", -1), ("n_lab_too_many", -3),
])
def test_problem_errors(case, code):
    n, K, ip, ix, w, li, lb = _path_graph()
    ip, ix, w = np.array(ip), np.array(ix), np.array(w, dtype=float)
    kw = {}
    if case == "K1":
        kw = dict(K=1)
    elif case == "n0":
        kw = dict(n=0, indptr=np.array([0]), indices=np.array([], np.int32), data=np.array([]), labelled_idx=[],
                  labels=[])
    elif case == "Kbig":
        kw = dict(K=5000)
    elif case == "unsorted":
        ix2 = ix.copy()
        ix2[ip[1]:ip[2]] = ix2[ip[1]:ip[2]][::-1]
        kw = dict(indices=ix2)
    elif case == "duplicate":
        ix2 = ix.copy()
        ix2[ip[1] + 1] = ix2[ip[1]]
        kw = dict(indices=ix2)
    elif case == "col_range":
        ix2 = ix.copy()
        ix2[-1] = 7
        kw = dict(indices=ix2)
    elif case == "negative":
        w2 = w.copy()
        w2[0] = w2[1] = -1.0
        kw = dict(data=w2)
    elif case == "nan":
        w2 = w.copy()
        w2[0] = math.nan
        kw = dict(data=w2)
    elif case == "inf":
        w2 = w.copy()
        w2[0] = math.inf
        kw = dict(data=w2)
    elif case == "asym_pattern":
        # drop the edge (3,2) but keep (2,3)
        ip2 = ip.copy()
        ip2[4] -= 1
        kw = dict(indptr=ip2, indices=ix[:-1], data=w[:-1])
    elif case == "asym_value":
        w2 = w.copy()
        w2[0] = 2.0
        kw = dict(data=w2)
    elif case == "rp0":
        ip2 = ip.copy()
        ip2[0] = 1
        kw = dict(indptr=ip2)
    elif case == "rpn":
        ip2 = ip.copy()
        ip2[-1] = ip2[-1] - 1
        kw = dict(indptr=ip2)
    elif case == "rp_decreasing":
        ip2 = ip.copy()
        ip2[2] = ip2[1] - 1
        kw = dict(indptr=ip2)
    elif case == "label_range":
        kw = dict(labelled_idx=[0, 9])
    elif case == "label_class":
        kw = dict(labels=[0, 2])
    elif case == "label_repeat":
        kw = dict(labelled_idx=[3, 3])
    elif case == "kindL_novals":
        kw = dict(kind=gfw.GRAPH_L, data=None)
    elif case == "n_lab_too_many":
        kw = dict(labelled_idx=[0, 1, 2, 3, 0], labels=[0, 0, 0, 0, 0])
    assert _check(**kw) == code, gfw.last_error()


def test_nnz_limit():
    pb = gfw.Problem(4, 1 << 31, 2, 0, 0, 0, 1, 1, None, 0, None, None)
    import ctypes as C
    assert gfw.lib().gfw_check_problem(C.byref(pb)) == -2


def test_null_problem():
    import ctypes as C
    assert gfw.lib().gfw_check_problem(None) == -1
    assert gfw.lib().gfw_check_params(None, 3) == -1


@pytest.mark.parametrize("field,value", [
    ("eps", 0.0), ("eps", -1.0), ("eps", math.nan), ("omega0", -1.0), ("omega0", math.inf), ("max_iter", -1),
    ("tol", math.nan), ("ls", 7), ("delta", 0.0), ("delta", 1.0), ("gamma", 0.0), ("gamma", 0.5), ("lmo", 3),
    ("one_shot", 2), ("lipschitz", math.nan), ("p_refresh", -1),
])
def test_param_errors(field, value):
    p = gfw.params()
    assert gfw.check_params(p, 3) == gfw.GFW_OK
    setattr(p, field, value)
    assert gfw.check_params(p, 3) == -1


def test_param_defaults_are_the_papers():
    import ctypes as C
    p = gfw.Params()
    gfw.lib().gfw_params_default(C.byref(p))
    assert (p.eps, p.omega0, p.max_iter, p.tol, p.ls, p.delta, p.gamma, p.lmo, p.one_shot) == \
        (50.0, 1000.0, 30, 1e-6, gfw.LS_ARMIJO, 0.5, 1e-6, gfw.LMO_GREEDY, 0)
    p.eps = math.inf  # eps = +inf (no penalty) is allowed
    assert gfw.check_params(p, 3) == gfw.GFW_OK


def test_context_without_gpu_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import ctypes as C
    h = C.c_void_p()
    rc = gfw.lib().gfw_context_create(C.byref(h), 0)
    assert rc == -5 and not h.value


def test_k_bounds_of_the_many_classes_path():
    # 16 < K <= 1024 runs on the wavefront-per-row kernels; beyond that the problem is rejected
    assert _check(K=17) == gfw.GFW_OK
    assert _check(K=1024) == gfw.GFW_OK
    assert _check(K=1025) == -6


def test_lfr_like_generator_shape():
    """The many-classes input: a symmetric, sorted, duplicate-free CSR without self-loops,
    mean degree near 5, community sizes within the truncation, about 1 - mu of the edges
    inside communities, every community present."""
    n, K, mu = 20000, 300, 0.2
    g = graphs.lfr_like(n, K, 5.0, mu, 3)
    ip, ix = g.indptr, g.indices
    rows = np.repeat(np.arange(n), np.diff(ip))
    assert np.all(rows != ix)
    assert all(np.all(np.diff(ix[ip[i]:ip[i + 1]]) > 0) for i in range(0, n, 97))
    import scipy.sparse as sp
    W = sp.csr_matrix((g.data, ix, ip), shape=(n, n))
    assert (W != W.T).nnz == 0
    deg = np.diff(ip)
    assert 4.2 <= deg.mean() <= 5.2 and deg.max() <= 50
    sizes = np.bincount(g.truth, minlength=K)
    assert sizes.min() >= 3 and sizes.max() <= 8 * n / K + 1 and sizes.sum() == n
    inside = np.mean(g.truth[rows] == g.truth[ix])
    assert 1 - mu - 0.1 <= inside <= 1 - mu + 0.1
