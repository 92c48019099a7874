"""The oscillator-run tuner (stepped_min_n = LW_STEPPED_TUNE): the threshold between the
persistent one-workgroup path and the stepped path is timed once per shape class.

Checks:
- the choice is written once to the file LW_TUNE_CACHE names;
- the run equals, bitwise, a run forced to the chosen threshold;
- a new context reads the choice back instead of tuning again.
"""
import math

import numpy as np
import pytest

from paper_2107_12437_amd import inputs as I
from tests.helpers import gpu_ready

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]


def uneven():
    rng = I.rng_for(85)
    sizes = [3, 5, 9, 17, 40]
    parts = [I.cluster_dipoles(rng, n, 40e-9, 10e-9, 2 * math.pi * 200e12, 0.01, True) for n in sizes]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    return {"dipoles": I.concat_dipoles(parts), "inst_off": off, "dt": 1 / 200e12 / 200}


def dip_lines(path):
    return [ln for ln in path.read_text().splitlines() if ln.startswith("dipoles")] if path.exists() else []


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tuned_threshold_is_cached_and_used(tmp_path, monkeypatch, precision):
    from paper_2107_12437_amd import lw
    f = tmp_path / "tune.txt"
    monkeypatch.setenv("LW_TUNE_CACHE", str(f))
    w = uneven()

    def run(ctx, smn):
        r = lw.dipole_run(w["dipoles"], w["inst_off"], w["dt"], 120, out_stride=4, stepped_min_n=smn, ctx=ctx,
                          precision=precision)
        return {k: v.cpu().numpy() for k, v in r.items()}

    ctx = lw.Context(0)
    a = run(ctx, "tune")
    lines = dip_lines(f)
    assert len(lines) == 1, lines
    T = int(lines[0].split("|")[1])
    assert T in (2, 4, 8, 16, 32, 64, 128)
    b = run(ctx, T)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    ctx.close()
    ctx = lw.Context(0)
    c = run(ctx, "tune")
    ctx.close()
    assert len(dip_lines(f)) == 1
    for k in a:
        assert np.array_equal(a[k], c[k]), k


def test_tuner_trials_do_not_leak_errors(tmp_path, monkeypatch):
    """The tuner's trial runs (256 and 512 steps) may cross the speed limit where the call
    itself does not: a 20-step tuned call whose charges reach 0.59 of their peak speed
    (peak at step 50) under a limit of 0.8 of it must report no error, and an error
    latched by an earlier call and not yet read must survive the tuning."""
    from paper_2107_12437_amd import lw
    monkeypatch.setenv("LW_TUNE_CACHE", str(tmp_path / "tune.txt"))
    w0 = 2 * math.pi * 200e12
    dip = I.cluster_dipoles(I.rng_for(86), 3, 20e-9, 10e-9, w0, 0.0, False)
    dip["d0"][:] = I.E_CHARGE * 1e-12
    dt = 1 / 200e12 / 200
    peak = 0.5 * w0 * 1e-12                   # charge speed: half the moment's rate over q
    ctx = lw.Context(0)
    r = lw.dipole_run(dip, [0, 3], dt, 20, max_vel=0.8 * peak, stepped_min_n="tune", ctx=ctx)
    assert np.isfinite(r["d"].cpu().numpy()).all()
    # a pending error survives a tuned call of a new shape class
    lw.dipole_run(dip, [0, 3], dt, 120, max_vel=0.8 * peak, ctx=ctx, check=False)
    dip5 = I.cluster_dipoles(I.rng_for(87), 5, 25e-9, 10e-9, w0, 0.0, False)
    lw.dipole_run(dip5, [0, 5], dt, 20, stepped_min_n="tune", ctx=ctx, check=False)
    with pytest.raises(lw.LWError) as ei:
        lw.sync_status(ctx)
    assert ei.value.code == 4
    ctx.close()
