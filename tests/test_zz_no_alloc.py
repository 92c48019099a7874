"""lw_fields_noalloc against lw_fields, through the C ABI.

The no-alloc entry point runs the same kernels on a fixed per-GPU scratch, so with the
same launch shape its output must equal lw_fields' bitwise.  Two calls in a row, the
second smaller (fewer charges, times and points, other precision), check that nothing
of the first call's scratch leaks into the second.  A call beyond the scratch's size is
refused on the host.
"""
import ctypes as ct

import numpy as np
import pytest

import oracle as O
from paper_2107_12437_amd import inputs as I
from tests.helpers import assert_fields_close, gpu_ready

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]


def _pair_of_calls(ctx, w, precision):
    import torch
    from paper_2107_12437_amd import lw
    pts = torch.tensor(w["points"], dtype=torch.float64, device="cuda")
    ref = lw.FieldsCall(w["charges"], pts, w["times"], precision=precision, ctx=ctx)
    got = lw.FieldsCall(w["charges"], pts, w["times"], precision=precision, ctx=ctx)
    got.out.fill_(float("nan"))
    got.flags.fill_(-1)
    ref.launch()
    got.launch(noalloc=True)
    torch.cuda.synchronize()
    return (got.out.double().cpu().numpy(), got.flags.cpu().numpy(), ref.out.double().cpu().numpy(),
            ref.flags.cpu().numpy())


def test_noalloc_equals_lw_fields_on_two_calls():
    from paper_2107_12437_amd import lw
    ctx = lw.Context(0)
    ctx.set_autotune(False)          # both entry points then take the context's default launch shape
    big = I.workload_grid_mixed(grid_n=96, n_times=9)
    small = I.workload_grid_mixed(grid_n=41, n_times=3, n_charges=5)
    for w, prec, tol in ((big, "mixed", 1e-5), (small, "fp64", 1e-12)):
        got, gflags, ref, rflags = _pair_of_calls(ctx, w, prec)
        assert np.array_equal(got, ref, equal_nan=True), (prec, np.nanmax(np.abs(got - ref)))
        assert np.array_equal(gflags, rflags)
        # and to the oracle at the parity bar, on a slice of the points
        sel = np.arange(0, w["points"].shape[1], 7)
        oref, _ = O.fields(w["charges"], np.ascontiguousarray(w["points"][:, sel]), w["times"])
        assert_fields_close(got[:, :, sel], oref, tol, f"no-alloc {prec}")
    ctx.close()


def test_noalloc_refuses_more_than_its_scratch():
    import torch
    from paper_2107_12437_amd import lw
    L = lw.load_library()
    w = I.workload_grid_mixed(grid_n=8, n_times=2)
    ch = I.concat_charges([w["charges"]] * 20)            # 320 charges
    times = np.linspace(1e-16, 1e-15, 64)                 # 64 x 320 records: 4.6 MB > 4 MiB
    pts = torch.tensor(w["points"], dtype=torch.float64, device="cuda")
    out = torch.empty((64, 10, pts.shape[1]), dtype=torch.float32, device="cuda")
    arr, n = lw.pack_charges(ch)
    tms = np.ascontiguousarray(times)
    opts = lw.Opts(lw.MIXED, 0, 0, 0, 1e-10)
    ctx = lw.default_context(0)
    code = L.lw_fields_noalloc(ctx.handle, arr, n, ct.c_void_p(pts.data_ptr()), pts.shape[1],
                               tms.ctypes.data_as(ct.POINTER(ct.c_double)), len(tms), ct.byref(opts),
                               ct.c_void_p(out.data_ptr()), None, None)
    assert code == 1 and b"scratch" in L.lw_last_error()
