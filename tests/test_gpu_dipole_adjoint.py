"""Oscillator adjoint (lw_dipole_run_vjp) against central finite differences of the FP64
oracle's detector objective J = (1/n_snap) sum |E|^2.

Finite differences of J in the positions are limited by J's own FP64 rounding (the
detector field is a near-cancelling sum over opposite charges): at h = 1e-12 m the
noise is about 2e-7 relative and the truncation 1e-8.  Richardson extrapolation of the
h and 2h central differences removes the h^2 term; the adjoint must agree to 1e-6
(relative L2 over the gradient).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2107_12437_amd import inputs as I
from tests.helpers import gpu_ready

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]


def oracle_J(dip, off, dt, steps, pts, times, policy):
    r = O.dipole_run(dip, off, dt, steps, policy=policy, want_hist=True)
    E = O.dipole_fields(dip, dt, steps, r["hist"], pts, times)
    return float((E ** 2).sum() / len(times))


def fd_positions(dip, off, dt, steps, pts, times, policy, h=1e-12):
    n = len(dip["omega0"])
    g = np.zeros((n, 3))
    for i in range(n):
        for c in range(3):
            vals = []
            for step in (h, 2 * h):
                dp = {k: np.array(v, copy=True) for k, v in dip.items()}
                dm = {k: np.array(v, copy=True) for k, v in dip.items()}
                dp["origin"][i, c] += step
                dm["origin"][i, c] -= step
                vals.append((oracle_J(dp, off, dt, steps, pts, times, policy) -
                             oracle_J(dm, off, dt, steps, pts, times, policy)) / (2 * step))
            g[i, c] = (4 * vals[0] - vals[1]) / 3
    return g


ORACLE_POLICY = {"strict": O.DT_STRICT, "extrapolate": O.DT_EXTRAPOLATE}


def run_case(dip, off, dt, steps, pts, times, policy):
    import torch
    from paper_2107_12437_amd import lw
    dpts = torch.tensor(pts, dtype=torch.float64, device="cuda")
    J, grad = lw.dipole_run_vjp(dip, off, dt, steps, dpts, times, policy=policy)
    policy = ORACLE_POLICY[policy]
    Jo = oracle_J(dip, off, dt, steps, pts, times, policy)
    assert abs(J / Jo - 1) <= 1e-10, (J, Jo)
    g_fd = fd_positions(dip, off, dt, steps, pts, times, policy)
    g = grad.cpu().numpy()
    err = np.linalg.norm(g - g_fd) / np.linalg.norm(g_fd)
    assert err <= 1e-6, (err, g, g_fd)
    return g


def test_cluster_strict():
    """Five coupled dipoles (random axes, omega_0 spread, random signs), 300 steps at
    T0/200, 6x6 detector 60 nm above, 4 snapshots."""
    rng = I.rng_for(91)
    dip = I.cluster_dipoles(rng, 5, 15e-9, 10e-9, 2 * math.pi * 200e12, 0.01, True)
    dt = 1 / 200e12 / 200
    steps = 300
    times = (np.arange(4) + 1) * steps * dt / 4
    run_case(dip, np.array([0, 5], np.int32), dt, steps, I.plane_grid(40e-9, 6, z=60e-9), times, "strict")


def test_two_instances_with_extrapolation():
    """A 3-dipole cluster and a close pair (2 nm, below c dt: sources read past their
    newest step), one detector seeing both."""
    rng = I.rng_for(92)
    a = I.cluster_dipoles(rng, 3, 12e-9, 10e-9, 2 * math.pi * 200e12, 0.01, True)
    b = I.empty_dipoles(2)
    b["origin"][:] = [[30e-9, 0, 0], [32e-9, 0, 0]]
    b["axis"][:] = [[0.6, 0.8, 0], [0.6, 0.8, 0]]
    b["omega0"][:] = 2 * math.pi * 200e12
    b["d0"][:] = [I.E_CHARGE * 1e-12, -0.5 * I.E_CHARGE * 1e-12]
    dip = I.concat_dipoles([a, b])
    dt = 1 / 200e12 / 200
    steps = 200
    times = (np.arange(3) + 1) * steps * dt / 3
    run_case(dip, np.array([0, 3, 5], np.int32), dt, steps, I.plane_grid(40e-9, 5, z=50e-9), times,
             "extrapolate")


def test_autograd_and_full_detector_workload():
    """The 32-dipole detector workload (5,000 steps, 256x256 detector, 32 snapshots) through
    the autograd Function: the gradient matches central differences of the GPU's own J on
    three coordinates."""
    import torch
    from paper_2107_12437_amd import lw
    w = I.workload_dipole_detector()
    dpts = torch.tensor(w["points"], dtype=torch.float64, device="cuda")
    origins = torch.tensor(w["dipoles"]["origin"], dtype=torch.float64, requires_grad=True)
    J = lw.DipoleDetectorFn.apply(origins, w["dipoles"], w["inst_off"], w["dt"], w["steps"], dpts, w["times"],
                                  "strict")
    J.backward()
    g = origins.grad.numpy()
    for i, c in ((0, 0), (13, 1), (27, 2)):
        vals = []
        for h in (1e-12, 2e-12):
            dp = {k: np.array(v, copy=True) for k, v in w["dipoles"].items()}
            dm = {k: np.array(v, copy=True) for k, v in w["dipoles"].items()}
            dp["origin"][i, c] += h
            dm["origin"][i, c] -= h
            Jp, _ = lw.dipole_run_vjp(dp, w["inst_off"], w["dt"], w["steps"], dpts, w["times"])
            Jm, _ = lw.dipole_run_vjp(dm, w["inst_off"], w["dt"], w["steps"], dpts, w["times"])
            vals.append((Jp - Jm) / (2 * h))
        fd = (4 * vals[0] - vals[1]) / 3
        assert abs(g[i, c] - fd) <= 1e-5 * np.abs(g).max(), (i, c, g[i, c], fd)


def test_large_instance_directional_derivative():
    """A 72-dipole cluster (288 drive pairs per source and step: each lane of the backward
    step takes more than one pair) next to a pair, 200 steps. The gradient's projection on
    a seeded direction of all 222 origin coordinates matches the Richardson-extrapolated
    central difference of the GPU's own J (whose values match the oracle's in the tests
    above), to 1e-5 of |g| |v|."""
    import torch
    from paper_2107_12437_amd import lw
    rng = I.rng_for(95)
    a = I.cluster_dipoles(rng, 72, 60e-9, 10e-9, 2 * math.pi * 200e12, 0.01, True)
    b = I.cluster_dipoles(rng, 2, 20e-9, 10e-9, 2 * math.pi * 200e12, 0.01, True)
    b["origin"] += np.array([200e-9, 0.0, 0.0])
    dip = I.concat_dipoles([a, b])
    off = np.array([0, 72, 74], np.int32)
    dt = 1 / 200e12 / 200
    steps = 200
    times = np.array([100 * dt, 150 * dt, 200 * dt])
    dpts = torch.tensor(I.plane_grid(150e-9, 8, z=120e-9), dtype=torch.float64, device="cuda")
    J, grad = lw.dipole_run_vjp(dip, off, dt, steps, dpts, times)
    g = grad.cpu().numpy()
    v = rng.normal(size=g.shape)
    v /= np.linalg.norm(v)

    def J_at(h):
        d = {k: np.array(x, copy=True) for k, x in dip.items()}
        d["origin"] = d["origin"] + h * v
        return lw.dipole_run_vjp(d, off, dt, steps, dpts, times)[0]

    vals = [(J_at(h) - J_at(-h)) / (2 * h) for h in (1e-12, 2e-12)]
    fd = (4 * vals[0] - vals[1]) / 3
    assert abs((g * v).sum() - fd) <= 1e-5 * np.linalg.norm(g), ((g * v).sum(), fd, np.linalg.norm(g))


def test_full_length_checkpointed_gradient_against_oracle_differences():
    """The 32-dipole adjoint workload for its full 5,000 steps, checkpointed every 250
    steps (the workload's setting), observed on a 64x64 detector over the same plane at
    its 32 snapshots: dJ/dR of 8 seeded origin coordinates against the central
    differences of the oracle's extended-precision build at h = 1e-6 max(|R|, 1 nm)
    (tests/golden/c4b_dipole_detector_fd.json, written by make_goldens.py from the oracle
    alone), to 1e-6 of each entry plus 1e-8 of the largest."""
    import torch
    from paper_2107_12437_amd import lw
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c4b_dipole_detector_fd.json")))
    w = I.workload_dipole_detector()
    assert g["workload"] == w["name"]
    dpts = torch.tensor(I.plane_grid(100e-9, 64, z=200e-9), dtype=torch.float64, device="cuda")
    J, grad = lw.dipole_run_vjp(w["dipoles"], w["inst_off"], w["dt"], w["steps"], dpts, w["times"],
                                ckpt_every=w["ckpt_every"])
    grad = grad.cpu().numpy()
    big = max(abs(e["dJ"]) for e in g["entries"])
    rel = []
    for e in g["entries"]:
        got = grad[e["dipole"], e["axis"]]
        rel.append(abs(got - e["dJ"]) / abs(e["dJ"]))
        assert abs(got - e["dJ"]) <= 1e-6 * abs(e["dJ"]) + 1e-8 * big, (e, got)
    print(f"checkpointed oscillator gradient vs oracle differences: max relative error {max(rel):.2e}")


def test_repeatability_of_the_atomic_sums():
    """The adjoint accumulates history and position cotangents with FP64 device atomics, so
    two calls agree to rounding, not bitwise: the 32-dipole workload (500 steps, 32x32
    detector) twice, gradients within 1e-12 of the largest entry and J bitwise (J's sums
    run in a fixed order)."""
    import torch
    from paper_2107_12437_amd import lw
    w = I.workload_dipole_detector(steps=500, grid_n=32)
    dpts = torch.tensor(w["points"], dtype=torch.float64, device="cuda")
    J1, g1 = lw.dipole_run_vjp(w["dipoles"], w["inst_off"], w["dt"], w["steps"], dpts, w["times"])
    J2, g2 = lw.dipole_run_vjp(w["dipoles"], w["inst_off"], w["dt"], w["steps"], dpts, w["times"])
    g1, g2 = g1.cpu().numpy(), g2.cpu().numpy()
    spread = np.abs(g1 - g2).max() / np.abs(g1).max()
    print(f"oscillator adjoint run-to-run spread: {spread:.2e} of the largest entry")
    assert J1 == J2
    assert spread <= 1e-12
