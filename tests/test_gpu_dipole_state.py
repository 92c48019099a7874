"""Run state of oscillator runs (lw_dipole_run_state): a run split into calls gives the
outputs of one call.

The state holds everything the next step reads:
- the history rings;
- E_d at the last step;
- the energy sums.

A resumed call repeats the same arithmetic as the undivided run, so the outputs are
compared bitwise on both run paths.
"""
import math

import numpy as np
import pytest

from paper_2107_12437_amd import inputs as I
from tests.helpers import gpu_ready
from tests.test_gpu_dipole import moving_workload

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]

KEYS = ("d", "d_dot", "energy", "Ed", "W_abs", "W_rad")


def small_batch():
    """A 6-dipole and a 3-dipole cluster and one pair (strict dt), seeded."""
    rng = I.rng_for(81)
    a = I.cluster_dipoles(rng, 6, 25e-9, 10e-9, 2 * math.pi * 200e12, 0.01, True)
    b = I.cluster_dipoles(rng, 3, 25e-9, 10e-9, 2 * math.pi * 200e12, 0.01, True)
    p = I.empty_dipoles(2)
    p["origin"][1] = [14e-9, 3e-9, 0.0]
    p["axis"][:] = [[0.0, 1.0, 0.0], [0.0, 0.6, 0.8]]
    p["omega0"][:] = 2 * math.pi * 200e12
    p["d0"][0] = I.E_CHARGE * 1e-12
    return {"dipoles": I.concat_dipoles([a, b, p]), "inst_off": np.array([0, 6, 9, 11], np.int32),
            "dt": 1 / 200e12 / 200}


def run(w, steps, stride, **kw):
    from paper_2107_12437_amd import lw
    r = lw.dipole_run(w["dipoles"], w["inst_off"], w["dt"], steps, out_stride=stride, energy_balance=True, **kw)
    return {k: v.cpu().numpy() for k, v in r.items()}


def split_run(w, parts, stride, **kw):
    """The run in consecutive calls sharing one state; rows joined as one run's."""
    from paper_2107_12437_amd import lw
    state = lw.dipole_state(w["dipoles"], w["inst_off"], w["dt"], policy=kw.get("policy", "strict"))
    rows = None
    for k, steps in enumerate(parts):
        r = run(w, steps, stride, state=state, resume=k > 0, **kw)
        rows = r if rows is None else {key: np.concatenate([rows[key], r[key][1:]]) for key in KEYS}
    return rows


@pytest.mark.parametrize("stepped_min_n", [0, 2])
def test_split_run_equals_one_run(stepped_min_n):
    """600 steps in one call and as 250 + 350 (stride 5; the stepped path replays a
    256-step graph in the second part), on the persistent path and forced onto the
    stepped path."""
    w = small_batch()
    one = run(w, 600, 5, stepped_min_n=stepped_min_n)
    two = split_run(w, [250, 350], 5, stepped_min_n=stepped_min_n)
    for k in KEYS:
        assert one[k].shape == two[k].shape
        assert np.array_equal(one[k], two[k]), (k, np.abs(one[k] - two[k]).max())


def test_split_mixed_moving_run():
    """Moving origins in the mixed form, 3 calls of 150 steps against one of 450."""
    w = moving_workload(5, 450, 83)
    one = run(w, 450, 3, precision="mixed")
    three = split_run(w, [150, 150, 150], 3, precision="mixed")
    for k in KEYS:
        assert np.array_equal(one[k], three[k]), k


def test_state_errors():
    import torch
    from paper_2107_12437_amd import lw
    w = small_batch()
    state = lw.dipole_state(w["dipoles"], w["inst_off"], w["dt"])
    with pytest.raises(lw.LWError) as ei:                      # too small for these dipoles
        run(w, 10, 1, state=state[:-1].contiguous())
    assert ei.value.code == 1
    with pytest.raises(ValueError):
        run(w, 10, 1, resume=True)
    run(w, 10, 1, state=state)
    # a state written for one history depth, resumed with a deeper one
    big = torch.zeros(state.numel() * 4, dtype=torch.float64, device="cuda")
    run(w, 10, 1, state=big, ring_depth=64)
    with pytest.raises(lw.LWError) as ei:
        run(w, 10, 1, state=big, resume=True, ring_depth=128)
    assert ei.value.code == 10
