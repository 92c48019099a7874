"""The C ABI library without a GPU: it loads, exports every declared entry point, its
struct layouts match the header, and its host-only calls agree with the oracle."""
import ctypes as ct
import math
import os
import re

import numpy as np
import pytest

from paper_2107_12437_amd import lw, inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lw_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = lw.load_library()
    names = declared_functions()
    assert set(names) == set(lw.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_struct_layouts_match_header():
    assert ct.sizeof(lw.Traj) == 144
    assert ct.sizeof(lw.Dipole) == 128
    assert ct.sizeof(lw.Opts) == 24
    assert ct.sizeof(lw.RunOpts) == 32


def test_gamma0_host_helper():
    # Fig. 9 caption: 19.791 MHz for q = e, m = m_e/2 at omega_0 = 2 pi 200 THz
    g = lw.gamma0(I.E_CHARGE, I.M_E / 2, 2 * math.pi * 200e12)
    assert round(g / 1e6, 3) == 19.791


def test_null_context_is_rejected_without_gpu():
    L = lw.load_library()
    opts = lw.Opts(0, 0, 0, 0, -1.0)
    arr, n = lw.pack_charges(I.workload_tiny_orbit()["charges"])
    t = (ct.c_double * 1)(0.0)
    assert L.lw_fields(None, arr, n, None, 10, t, 1, ct.byref(opts), None, None, None) == 1
    assert b"null" in L.lw_last_error()


def test_pair_modes_matches_oracle_extraction():
    """Host Prony fit of the library against the oracle's numpy fit on the same signal."""
    import oracle as O
    from oracle import extract as X
    w = I.workload_dipole_pairs(n_inst=3, steps=6000, seps=[5e-9, 40e-9, 300e-9])
    r = O.dipole_run(w["dipoles"], w["inst_off"], w["dt"], w["steps"], policy=O.DT_EXTRAPOLATE, out_stride=2)
    w0 = w["dipoles"]["omega0"][0]
    skips = [X.default_skip(w["dt"], s) for s in w["separations"]]
    got = lw.pair_modes(r["d"], w["inst_off"], w["dt"], 2, w0, skips)
    for k in range(3):
        ref = X.pair_modes(r["d"][:, 2 * k], r["d"][:, 2 * k + 1], w["dt"], 2, w0, skips[k])
        for j, key in enumerate(("gamma_plus", "gamma_minus", "omega_plus", "omega_minus", "delta_omega")):
            assert abs(got[k, j] - ref[key]) <= 1e-6 * abs(ref[key]) + 1e-9 * w0, (k, key, got[k, j], ref[key])


def test_pair_modes_rejects_bad_arguments():
    with pytest.raises(lw.LWError) as ei:
        lw.pair_modes(np.zeros((10, 2)), [0, 2], -1.0, 1, 1e15, 0)
    assert ei.value.code == 1


def test_dipole_packing_matches_the_struct_fields():
    """pack_dipoles writes each field where the C struct (lw_dipole) has it."""
    from paper_2107_12437_amd import lw
    rng = np.random.default_rng(5)
    n = 7
    dip = I.empty_dipoles(n)
    dip["origin"][:] = rng.normal(size=(n, 3))
    dip["axis"][:] = I.unit_sphere(rng, n)
    for k in ("omega0", "q", "m1", "m2", "d0", "motion_omega", "motion_phase"):
        dip[k][:] = rng.uniform(1, 2, size=n)
    dip["motion_amp"][:] = rng.normal(size=(n, 3))
    arr, m = lw.pack_dipoles(dip)
    assert m == n
    for i in range(n):
        d = arr[i]
        assert list(d.origin) == list(dip["origin"][i]) and list(d.axis) == list(dip["axis"][i])
        for k in ("omega0", "q", "m1", "m2", "d0", "motion_omega", "motion_phase"):
            assert getattr(d, k) == dip[k][i], k
        assert list(d.motion_amp) == list(dip["motion_amp"][i])


def test_dipole_state_size():
    """The run state holds a header of 4, a ring of `ring` steps x 3 per dipole, E_d and two
    energy sums per dipole; the ring is the power of two (at least 4) covering
    2 max-separation / (c dt) + 3 steps."""
    n = 5
    dip = I.empty_dipoles(n)
    dip["origin"][:, 0] = np.arange(n) * 20e-9
    dip["omega0"][:] = 2 * math.pi * 200e12
    dt = 1 / 200e12 / 200
    arr, m = lw.pack_dipoles(dip)
    off = np.array([0, 2, 5], np.int32)
    opts = lw.RunOpts(lw.FP64, 0, 1, 0.0, 0, 0)
    size = ct.c_int64(0)
    code = lw.load_library().lw_dipole_state_size(arr, m, off.ctypes.data_as(ct.POINTER(ct.c_int32)), 2, dt,
                                                  ct.byref(opts), ct.byref(size))
    assert code == 0
    need = math.ceil(2 * 40e-9 / 299792458.0 / dt) + 3
    ring = 4
    while ring < need:
        ring *= 2
    assert size.value == 4 + n * ring * 3 + 3 * n
    opts.ring_depth = 256
    lw.load_library().lw_dipole_state_size(arr, m, off.ctypes.data_as(ct.POINTER(ct.c_int32)), 2, dt,
                                           ct.byref(opts), ct.byref(size))
    assert size.value == 4 + n * 256 * 3 + 3 * n
