"""Tracing of gfw_solve: mode 1 times every hot-path launch, mode 2 only the label passes,
mode 3 only the row kernels;
the iterates are those of the untraced solve (captured iterations replayed) either way."""
import numpy as np
import pytest

from paper_2508_09738_amd import gfw
from synth import configs

from gpu_helpers import ctx, gpu_graph, np_of, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_trace_modes_time_their_kernels_and_keep_the_iterates(mode):
    say(f"[gpu] trace mode {mode}")
    prob = configs.sbm_small(11, n_per=3000)
    G = gpu_graph(prob.graph, prob.K, prob.labelled_idx, prob.labels, gfw.F32)
    prm = gfw.params(max_iter=64, tol=-1.0)
    ref = gfw.solve(ctx(), G, prm, want_history=True)
    gfw.trace_reset(ctx())
    gfw.trace_enable(ctx(), mode)
    try:
        r = gfw.solve(ctx(), G, prm, want_history=True)
    finally:
        gfw.trace_enable(ctx(), gfw.TRACE_OFF)
    np.testing.assert_array_equal(np_of(r["U"]), np_of(ref["U"]))
    np.testing.assert_array_equal(r["alpha"], ref["alpha"])
    ms, labels = gfw.trace_get(ctx(), gfw.KERNEL_LABEL)
    rms, rows = gfw.trace_get(ctx(), gfw.KERNEL_ROW)
    assert labels == (0 if mode == 3 else 64) and rows == (0 if mode == 2 else 64)
    assert (ms > 0.0) == (labels > 0) and (rms > 0.0) == (rows > 0)


def test_trace_mode_out_of_range():
    with pytest.raises(gfw.GfwError):
        gfw.trace_enable(ctx(), 4)
    with pytest.raises(gfw.GfwError):
        gfw.trace_enable(ctx(), -1)
