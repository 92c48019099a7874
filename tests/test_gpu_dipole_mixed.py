"""Mixed-precision oscillator runs against the FP64 oracle.

In the mixed form, each source dipole's static monopole difference (the dominant
near-field term) is formed in FP64 from the exact charge offset. Its velocity and
radiation terms are evaluated in FP32. The retarded times, the state and the sums stay
in FP64.

The FP32 rounding is about 1e-6 of the velocity and radiation terms. In the near field
these are of relative size omega L / c and its square against the static term. Moments,
velocities and energies are compared relative to their largest magnitude per dipole at
1e-5, the stated field tolerance.

The drive allows 1e-5 of its largest magnitude plus the oracle's own rounding, 1e-13 of
the sum of single-charge field magnitudes (the bound of the FP64 parity tests). The
oracle forms each charge's separation R = Delta - rho p in FP64, so the difference of a
pair's two separations is good only to ulp(|Delta|). For the tiny induced moments of
distant dipoles (offsets near 1e-19 m at 700 nm) that leaves about 3 significant digits
in the oracle's pair field. The mixed form takes the offset difference exactly and is
the more accurate of the two there.

The collective rates and the shift are compared at 1e-4 of max(|value|, gamma_0), ten
times inside the stated 1e-3. Over an 8,000-step window the energy decays by only about
4e-6, so this needs the moments to about 1e-9. That requirement is why the static
near-field term stays in FP64.
"""
import math

import numpy as np
import pytest

from oracle import extract as X
from paper_2107_12437_amd import inputs as I
from tests.helpers import gpu_ready
from tests.test_gpu_dipole import gpu_run, moving_workload, oracle_run

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]

TOL_MIXED = 1e-5
TOL_REF_DRIVE = 1e-13


def single_charge_scale(w):
    """Per target dipole, the sum over the other dipoles' charges of k q / L^2 (the scale of
    an FP64 per-charge drive's rounding)."""
    dip, off = w["dipoles"], w["inst_off"]
    k = 1 / (4 * math.pi * 8.8541878128e-12)
    sc = np.zeros(len(dip["omega0"]))
    for a0, a1 in zip(off[:-1], off[1:]):
        o = dip["origin"][a0:a1]
        L2 = ((o[:, None, :] - o[None, :, :]) ** 2).sum(axis=2)
        np.fill_diagonal(L2, np.inf)
        sc[a0:a1] = (2 * k * dip["q"][a0:a1][None, :] / L2).sum(axis=1)
    return sc


def assert_mixed_close(got, ref, w, what, keys=("d", "d_dot", "energy", "Ed"), tol=TOL_MIXED):
    for k in keys:
        scale = np.abs(ref[k]).max(axis=0, keepdims=True)
        scale = np.where(scale > 0, scale, 1.0)
        bound = tol * scale
        if k == "Ed":
            bound = bound + TOL_REF_DRIVE * single_charge_scale(w)[None, :]
        err = np.abs(got[k] - ref[k]) / bound
        assert err.max() <= 1.0, f"{what} {k}: error {err.max():.3e} of the bound"


def test_mixed_pairs_parity():
    """24 two-dipole instances of the pair recipe (1 nm - 1 um, a third closer than c dt),
    1,500 steps with the extrapolation past the newest sample, against the oracle's
    extended-precision build."""
    w = I.workload_dipole_pairs(n_inst=24, steps=1500)
    got = gpu_run(w, "extrapolate", precision="mixed")
    ref = oracle_run(w, "extrapolate", extended=True)
    assert_mixed_close(got, ref, w, "mixed pairs")


@pytest.mark.parametrize("stepped_min_n", [0, 2])
def test_mixed_clusters_parity(stepped_min_n):
    """A 6-dipole and a 3-dipole cluster (random axes, omega_0 spread, strict dt) on the
    persistent path and forced onto the stepped path, 800 steps."""
    rng = I.rng_for(71)
    a = I.cluster_dipoles(rng, 6, 25e-9, 10e-9, 2 * math.pi * 200e12, 0.01, True)
    b = I.cluster_dipoles(rng, 3, 25e-9, 10e-9, 2 * math.pi * 200e12, 0.01, True)
    w = {"dipoles": I.concat_dipoles([a, b]), "inst_off": np.array([0, 6, 9], np.int32),
         "dt": 1 / 200e12 / 200, "steps": 800}
    got = gpu_run(w, "strict", precision="mixed", stepped_min_n=stepped_min_n)
    ref = oracle_run(w, "strict")
    assert_mixed_close(got, ref, w, f"mixed clusters (stepped_min_n={stepped_min_n})")


def test_mixed_moving_parity():
    """Moving origins (Sec. 4.3) in the mixed form, 400 steps."""
    w = moving_workload(6, 400, 97)
    got = gpu_run(w, "strict", precision="mixed")
    ref = oracle_run(w, "strict")
    assert_mixed_close(got, ref, w, "mixed moving")


def test_mixed_gamma_domega_parity():
    """Collective rates and shift of 8 pairs (8,000 steps) from the mixed run's moments
    against those of the oracle's moments: within 1e-4 (the first-order velocity terms are
    FP64, so the mixed rates follow the FP64 ones)."""
    from paper_2107_12437_amd import lw
    w = I.workload_dipole_pairs(n_inst=8, steps=8000)
    got = gpu_run(w, "extrapolate", stride=2, precision="mixed")
    ref = oracle_run(w, "extrapolate", stride=2)
    w0 = w["dipoles"]["omega0"][0]
    skips = [X.default_skip(w["dt"], s) for s in w["separations"]]
    modes = lw.pair_modes(got["d"], w["inst_off"], w["dt"], 2, w0, skips)
    g0 = lw.gamma0(I.E_CHARGE, I.M_E / 2, w0)
    for k in range(8):
        r = X.pair_modes(ref["d"][:, 2 * k], ref["d"][:, 2 * k + 1], w["dt"], 2, w0, skips[k])
        for jj, key in ((0, "gamma_plus"), (1, "gamma_minus"), (4, "delta_omega")):
            scale = max(abs(r[key]), g0)
            assert abs(modes[k, jj] - r[key]) <= 1e-4 * scale, (k, key, modes[k, jj], r[key])


def test_mixed_matches_fp64_on_the_cluster_benchmark():
    """The 64-cluster workload at its full size (12,530 dipoles, clusters of 2 to 955),
    60 steps in both precisions on the GPU: the mixed form agrees with the FP64 form to
    the field tolerance (the oracle cannot run this size)."""
    w = I.workload_clusters(steps=60)
    a = gpu_run(w, "strict", stride=6, precision="mixed")
    b = gpu_run(w, "strict", stride=6)
    assert_mixed_close(a, b, w, "mixed vs FP64, 64 clusters")


def test_mixed_adjoint_is_rejected():
    import torch
    from paper_2107_12437_amd import lw
    w = I.workload_dipole_pairs(n_inst=2, steps=10)
    pts = torch.zeros((3, 4), dtype=torch.float64, device="cuda")
    pts[2] = 1e-7
    opts = lw.RunOpts(lw.MIXED, 0, 1, 0.0, 0, 0)
    arr, n = lw.pack_dipoles(w["dipoles"])
    off = np.ascontiguousarray(w["inst_off"], dtype=np.int32)
    grad = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    J = lw.ct.c_double(0.0)
    times = (lw.ct.c_double * 1)(5 * w["dt"])
    ctx = lw.default_context(0)
    code = lw.load_library().lw_dipole_run_vjp(
        ctx.handle, arr, n, off.ctypes.data_as(lw.ct.POINTER(lw.ct.c_int32)), len(off) - 1, float(w["dt"]), 10,
        lw.ct.byref(opts), lw.ct.c_void_p(pts.data_ptr()), 4, times, 1, 0, lw.ct.c_void_p(grad.data_ptr()),
        lw.ct.byref(J), None)
    assert code == 1
