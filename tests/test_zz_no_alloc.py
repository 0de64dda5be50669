"""gfw_objective_noalloc, the entry point that allocates nothing: through the C ABI its
result equals gfw_objective's bit for bit, on two calls in a row (the second on a smaller
graph, so that the shared scratch holds the first call's partials), for FP32 and FP64 and
for both kernel families (K <= 16, K > 16); graphs beyond its fixed scratch are rejected
on the host before any launch."""
import numpy as np
import pytest

from paper_2508_09738_amd import gfw
from synth import configs, graphs

from gpu_helpers import ctx, gpu_graph, say, torch_u

pytestmark = pytest.mark.gpu


def _rows(n, K, seed):
    U = np.random.default_rng(seed).random((n, K))
    return U / U.sum(axis=1, keepdims=True)


@pytest.mark.parametrize("dtype", [gfw.F32, gfw.F64])
def test_noalloc_objective_equals_objective(dtype):
    import torch

    cases = [configs.sbm_small(3, n_per=4000), configs.sbm_small(4, n_per=300),
             configs.lfr_many_classes(seed=8, n=6000, K=70, frac=0.05),
             configs.lfr_many_classes(seed=9, n=1500, K=40, frac=0.05)]
    E_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    for rep, prob in enumerate(cases):
        say(f"[gpu] noalloc objective dtype={dtype} n={prob.n} K={prob.K}")
        G = gpu_graph(prob.graph, prob.K, prob.labelled_idx, prob.labels, dtype)
        U = torch_u(_rows(prob.n, prob.K, rep), dtype)
        prm = gfw.params(eps=prob.eps, omega0=prob.omega0)
        gfw.objective_noalloc(ctx(), G, prm, U, E_dev)
        torch.cuda.synchronize()
        E_ref = gfw.objective(ctx(), G, prm, U)
        assert E_dev.item() == E_ref
        G.close()


def test_noalloc_objective_rejects_graphs_beyond_its_scratch():
    import torch

    K = 17  # a wavefront per row: 65,536 blocks hold 262,144 rows
    g = graphs.path_graph(262_145, K)
    say("[gpu] noalloc objective size limit")
    G = gpu_graph(g, K, [0], [0], gfw.F32)
    U = torch.full((g.n, K), 1.0 / K, dtype=torch.float32, device="cuda")
    E_dev = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    with pytest.raises(gfw.GfwError) as e:
        gfw.objective_noalloc(ctx(), G, gfw.params(), U, E_dev)
    assert e.value.status == -6 and "scratch" in str(e.value)
    assert E_dev.item() == -1.0  # nothing was launched
