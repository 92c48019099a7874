"""The launch-shape autotuner: every shape gives the same bits, a tuned shape is cached
in the file LW_TUNE_CACHE names and read back by a later context, and a shape preset in
that file is used without tuning."""
import os

import numpy as np
import pytest

from paper_2107_12437_amd import inputs as I
from tests.helpers import gpu_ready

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]


def _workload():
    # ragged: the points are not a multiple of any block size, the times not of 2 or 4
    w = I.workload_grid_mixed(grid_n=61, n_times=7, n_charges=5)
    return w


def _key(precision_code, n_charges, n_times, n_pts, kinds):
    p2 = 1
    while p2 < n_pts:
        p2 <<= 1
    fam = 0
    for k in kinds:
        fam |= 1 << int(k)
    return f"fields p{precision_code} k0 c{n_charges} t{n_times} n{p2} f{fam}"


@pytest.mark.parametrize("precision,code", [("mixed", 1), ("fp64", 0)])
def test_every_shape_gives_the_same_bits(tmp_path, monkeypatch, precision, code):
    import torch
    from paper_2107_12437_amd import lw
    w = _workload()
    pts = torch.tensor(w["points"], dtype=torch.float64, device="cuda")
    n_pts, n_ch, n_t = pts.shape[1], len(w["charges"]["kind"]), len(w["times"])
    ref = None
    for block in (64, 128, 256):
        for tch in (1, 2, 4):
            f = tmp_path / f"tune_{precision}_{block}_{tch}.txt"
            f.write_text(f"{_key(code, n_ch, n_t, n_pts, w['charges']['kind'])} | {block} {tch}\n")
            monkeypatch.setenv("LW_TUNE_CACHE", str(f))
            ctx = lw.Context(0)
            out, flags = lw.fields(w["charges"], pts, w["times"], precision=precision, ctx=ctx)
            torch.cuda.synchronize()
            ctx.close()
            # a preset shape is used as it is: nothing is appended
            assert f.read_text().count("\n") == 1
            if ref is None:
                ref = (out.clone(), flags.clone())
            else:
                assert torch.equal(out, ref[0]) and torch.equal(flags, ref[1]), (block, tch)


def test_tuned_shape_is_cached_and_reused(tmp_path, monkeypatch):
    import torch
    from paper_2107_12437_amd import lw
    w = _workload()
    pts = torch.tensor(w["points"], dtype=torch.float64, device="cuda")
    f = tmp_path / "tune.txt"
    monkeypatch.setenv("LW_TUNE_CACHE", str(f))
    monkeypatch.delenv("LW_AUTOTUNE", raising=False)
    ctx = lw.Context(0)
    out1, _ = lw.fields(w["charges"], pts, w["times"], precision="mixed", ctx=ctx)
    out2, _ = lw.fields(w["charges"], pts, w["times"], precision="mixed", ctx=ctx)
    torch.cuda.synchronize()
    ctx.close()
    lines = [ln for ln in f.read_text().splitlines() if ln.strip()]
    assert len(lines) == 1, lines                     # tuned once, kept in the context
    key, shape = lines[0].split("|")
    assert key.strip() == _key(1, len(w["charges"]["kind"]), len(w["times"]), pts.shape[1], w["charges"]["kind"])
    block, tch = (int(v) for v in shape.split())
    assert block in (64, 128, 256) and tch in (1, 2, 4)
    assert torch.equal(out1, out2)
    # a new context reads the file and does not tune again
    ctx = lw.Context(0)
    out3, _ = lw.fields(w["charges"], pts, w["times"], precision="mixed", ctx=ctx)
    torch.cuda.synchronize()
    ctx.close()
    assert len([ln for ln in f.read_text().splitlines() if ln.strip()]) == 1
    assert torch.equal(out1, out3)
    # with tuning off and no cache entry the default shape runs, with the same bits
    monkeypatch.delenv("LW_TUNE_CACHE")
    ctx = lw.Context(0)
    ctx.set_autotune(False)
    out4, _ = lw.fields(w["charges"], pts, w["times"], precision="mixed", ctx=ctx)
    torch.cuda.synchronize()
    ctx.close()
    assert torch.equal(out1, out4)
    assert not np.isnan(out1.cpu().numpy()).all()


def test_family_set_is_part_of_the_shape_class(tmp_path, monkeypatch):
    import torch
    from paper_2107_12437_amd import lw
    w = _workload()
    pts = torch.tensor(w["points"], dtype=torch.float64, device="cuda")
    f = tmp_path / "tune.txt"
    monkeypatch.setenv("LW_TUNE_CACHE", str(f))
    monkeypatch.delenv("LW_AUTOTUNE", raising=False)
    still = dict(w["charges"])
    still["kind"] = np.full_like(w["charges"]["kind"], I.STATIONARY)
    ctx = lw.Context(0)
    lw.fields(w["charges"], pts, w["times"], precision="mixed", ctx=ctx)
    lw.fields(still, pts, w["times"], precision="mixed", ctx=ctx)
    torch.cuda.synchronize()
    ctx.close()
    keys = [ln.split("|")[0].strip() for ln in f.read_text().splitlines() if ln.strip()]
    n_ch, n_t, n_pts = len(w["charges"]["kind"]), len(w["times"]), pts.shape[1]
    assert keys == [_key(1, n_ch, n_t, n_pts, w["charges"]["kind"]), _key(1, n_ch, n_t, n_pts, still["kind"])]
