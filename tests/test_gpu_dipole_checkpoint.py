"""Checkpointed oscillator adjoint (lw_dipole_run_vjp with ckpt_every = K) against the
whole-history adjoint of the same run.

The checkpointed sweep recomputes each segment of K steps from the run state kept at
its start. A resumed run continues the stored run exactly, so the recomputed
history equals the stored one. J and the gradient then differ only by the order of
the sums: J's per-snapshot partials and the gradient's device atomics. Both must
agree to 1e-12 relative. The whole-history path is itself checked against central
differences of the FP64 oracle elsewhere.

Cases:
- K dividing the run and not;
- K = 1;
- snapshots on segment boundaries, at t = 0 and at the run's end;
- the extrapolating dt policy (sources read past their newest step);
- the stepped path (one launch per step);
- the 32-dipole detector workload at K = 250.
"""
import math

import numpy as np
import pytest

from paper_2107_12437_amd import inputs as I
from tests.helpers import gpu_ready

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]


def both(dip, off, dt, steps, pts, times, K, **kw):
    import torch
    from paper_2107_12437_amd import lw
    dpts = pts if isinstance(pts, torch.Tensor) else torch.tensor(pts, dtype=torch.float64, device="cuda")
    J0, g0 = lw.dipole_run_vjp(dip, off, dt, steps, dpts, times, **kw)
    J1, g1 = lw.dipole_run_vjp(dip, off, dt, steps, dpts, times, ckpt_every=K, **kw)
    g0, g1 = g0.cpu().numpy(), g1.cpu().numpy()
    assert abs(J1 / J0 - 1) <= 1e-12, (K, J0, J1)
    err = np.abs(g1 - g0).max() / np.abs(g0).max()
    assert err <= 1e-12, (K, err)
    return g0


def cluster(seed=91, n=5):
    rng = I.rng_for(seed)
    return I.cluster_dipoles(rng, n, 15e-9, 10e-9, 2 * math.pi * 200e12, 0.01, True)


DT = 1 / 200e12 / 200


@pytest.mark.parametrize("K", [50, 64, 299])
def test_cluster_segments(K):
    """Five coupled dipoles, 300 steps: K = 50 divides the run, 64 and 299 leave a short
    last segment. Four snapshots, one 60 nm detector plane."""
    steps = 300
    times = (np.arange(4) + 1) * steps * DT / 4
    both(cluster(), np.array([0, 5], np.int32), DT, steps, I.plane_grid(40e-9, 6, z=60e-9), times, K)


def test_one_step_segments_and_boundary_snapshots():
    """K = 1 (a run state per step); snapshots at t = 0, on segment boundaries of a
    K = 8 run, between steps and at the run's end."""
    steps = 40
    pts = I.plane_grid(40e-9, 4, z=50e-9)
    off = np.array([0, 5], np.int32)
    times = np.array([0.0, 8 * DT, 16 * DT, 23.5 * DT, steps * DT])
    both(cluster(93), off, DT, steps, pts, times, 1)
    both(cluster(93), off, DT, steps, pts, times, 8)


def test_extrapolating_pair_and_far_detector():
    """A 3-dipole cluster and a pair 2 nm apart (below c dt) under the extrapolating
    policy, with a detector 3 um away: its look-back (about 2 steps) exceeds the pairs'
    and sets the run states' depth."""
    rng = I.rng_for(92)
    a = I.cluster_dipoles(rng, 3, 12e-9, 10e-9, 2 * math.pi * 200e12, 0.01, True)
    b = I.empty_dipoles(2)
    b["origin"][:] = [[30e-9, 0, 0], [32e-9, 0, 0]]
    b["axis"][:] = [[0.6, 0.8, 0], [0.6, 0.8, 0]]
    b["omega0"][:] = 2 * math.pi * 200e12
    b["d0"][:] = [I.E_CHARGE * 1e-12, -0.5 * I.E_CHARGE * 1e-12]
    dip = I.concat_dipoles([a, b])
    steps = 200
    times = np.array([60 * DT, 130.25 * DT, steps * DT])
    off = np.array([0, 3, 5], np.int32)
    both(dip, off, DT, steps, I.plane_grid(40e-9, 5, z=50e-9), times, 32, policy="extrapolate")
    both(dip, off, DT, steps, I.plane_grid(200e-9, 3, z=3e-6), times, 17, policy="extrapolate")


def test_stepped_path():
    """Instances of at least 2 dipoles on the stepped path (one launch per step): its
    run state resumes the same way."""
    steps = 120
    times = np.array([40 * DT, 120 * DT])
    both(cluster(94, 8), np.array([0, 8], np.int32), DT, steps, I.plane_grid(40e-9, 4, z=60e-9), times, 25,
         stepped_min_n=2)


def test_detector_workload_checkpointed():
    """The 32-dipole detector workload (5,000 steps, 256x256 detector, 32 snapshots) with
    a run state every 250 steps."""
    import torch
    w = I.workload_dipole_detector()
    dpts = torch.tensor(w["points"], dtype=torch.float64, device="cuda")
    both(w["dipoles"], w["inst_off"], w["dt"], w["steps"], dpts, w["times"], 250)


def test_bad_interval_is_rejected():
    import torch
    from paper_2107_12437_amd import lw
    dpts = torch.zeros((3, 4), dtype=torch.float64, device="cuda")
    dpts[2] = 1e-7
    with pytest.raises(lw.LWError):
        lw.dipole_run_vjp(cluster(), np.array([0, 5], np.int32), DT, 10, dpts, [5 * DT], ckpt_every=-3)
