"""The debugging histogram of retarded-time iterations (lw_set_iteration_histogram and
lw_iteration_histogram, include/lw.h): counting leaves the outputs unchanged, every
(point, time, charge) pair of a call lands in exactly one bin, the closed-form families
(stationary, uniform velocity) take no iterations, the mixed path's correction solve takes
at least one FP32 step and its FP64 step, calls add up, and reset and off work.  Each
test runs on a context of its own, so no other test's calls are counted."""
import numpy as np
import pytest

from paper_2107_12437_amd import inputs as I
from tests.helpers import gpu_ready

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_counting_keeps_outputs_and_counts_every_pair(precision):
    import torch
    from paper_2107_12437_amd import lw
    ctx = lw.Context(0)
    try:
        w = I.workload_grid_mixed(grid_n=37, n_times=5, n_charges=9)
        pts = torch.tensor(w["points"], dtype=torch.float64, device="cuda")
        n_pairs = pts.shape[1] * len(w["times"]) * len(w["charges"]["kind"])
        ref, ref_fl = lw.fields(w["charges"], pts, w["times"], precision=precision, ctx=ctx)
        ref, ref_fl = ref.clone(), ref_fl.clone()
        lw.set_iteration_histogram(True, ctx=ctx)
        out, fl = lw.fields(w["charges"], pts, w["times"], precision=precision, ctx=ctx)
        h = lw.iteration_histogram(ctx=ctx)
        assert torch.equal(out, ref) and torch.equal(fl, ref_fl)
        assert int(h[:lw.ITER_BIN_NOCONV].sum()) == n_pairs
        assert int(h[lw.ITER_BIN_NOCONV]) == 0
        assert int(h[31]) == 0
        if precision == "mixed":
            # linear, circular and accelerated charges: one FP32 step at least, then FP64
            assert int(h[0]) == 0 and int(h[1]) == 0
            assert int(h[lw.ITER_BIN_FALLBACK]) <= n_pairs // 100
        else:
            assert int(h[lw.ITER_BIN_FALLBACK]) == 0
        lw.fields(w["charges"], pts, w["times"], precision=precision, ctx=ctx)
        h2 = lw.iteration_histogram(reset=True, ctx=ctx)
        assert np.array_equal(h2, 2 * h)
        assert not lw.iteration_histogram(ctx=ctx).any()
        lw.set_iteration_histogram(False, ctx=ctx)
        lw.fields(w["charges"], pts, w["times"], precision=precision, ctx=ctx)
        assert not lw.iteration_histogram(ctx=ctx).any()
    finally:
        ctx.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_closed_form_families_take_no_iterations(precision):
    import torch
    from paper_2107_12437_amd import lw
    ctx = lw.Context(0)
    try:
        w = I.workload_uniform_velocity(grid_n=29, n_times=3, n_charges=5)
        ch = I.concat_charges([w["charges"], I.subset_charges(w["charges"], [0])])
        ch["kind"][-1] = I.STATIONARY
        pts = torch.tensor(w["points"], dtype=torch.float64, device="cuda")
        lw.set_iteration_histogram(True, ctx=ctx)
        lw.fields(ch, pts, w["times"], precision=precision, ctx=ctx)
        h = lw.iteration_histogram(ctx=ctx)
        assert int(h[0]) == pts.shape[1] * len(w["times"]) * len(ch["kind"])
        assert int(h[1:].sum()) == 0
    finally:
        ctx.close()


def test_reading_needs_counting_turned_on():
    from paper_2107_12437_amd import lw
    ctx = lw.Context(0)
    try:
        with pytest.raises(lw.LWError) as ei:
            lw.iteration_histogram(ctx=ctx)
        assert ei.value.code == 1
    finally:
        ctx.close()
