"""The oracle and the library's host code under AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer (CPU only).

tests/sanitize/build.py builds three standalone executables:
- the oracle's C source, FP64 and extended precision, with gcc's sanitizers;
- the library's sources, with the sanitizers on hipcc's host pass.

Each test feeds a driver inputs through raw files, which the driver reads into
allocations of exactly the file's size. The test fails on any sanitizer report, on a
leak or on a nonzero exit. It then checks the driver's outputs:
- the oracle's against the regular oracle build, bit for bit;
- the host helpers' against the regular library build, bit for bit;
- the argument checks against the status each case must return.
A sanitized build that computed something else would show up there.
"""
from __future__ import annotations

import ctypes as ct
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as O
from paper_2107_12437_amd import inputs as I
from tests.sanitize import build as SB

C = 299792458.0
E = 1.602176634e-19
ME = 9.1093837015e-31
W0 = 2 * math.pi * 200e12
DIP_FIELDS = ("origin", "axis", "omega0", "q", "m1", "m2", "d0", "motion_amp", "motion_omega", "motion_phase")

ENV = dict(os.environ,
           ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


@pytest.fixture(scope="module")
def drivers():
    return {"fp64": SB.oracle_driver(False), "ld": SB.oracle_driver(True), "host": SB.host_driver()}


def run(exe, *args, stdin=None):
    p = subprocess.run([exe, *map(str, args)], input=stdin, capture_output=True, text=True, env=ENV, timeout=300)
    report = [m for m in ("AddressSanitizer", "LeakSanitizer", "runtime error:") if m in p.stderr]
    assert p.returncode == 0 and not report, f"{os.path.basename(exe)} {args[:1]}: rc {p.returncode}\n{p.stderr[-4000:]}"
    return p.stdout


def save(path, a, dtype=np.float64):
    np.ascontiguousarray(a, dtype=dtype).tofile(path)
    return path


def dip_records(dip: dict) -> np.ndarray:
    """[n][16] doubles in the lw_dipole / driver record order."""
    n = len(dip["omega0"])
    cols = [np.reshape(np.asarray(dip[k], dtype=np.float64), (n, -1)) for k in DIP_FIELDS]
    return np.ascontiguousarray(np.concatenate(cols, axis=1))


def one(kind, **kw):
    ch = I.empty_charges(1)
    ch["kind"][0] = kind
    ch["q"][0] = kw.pop("q", E)
    for k, v in kw.items():
        ch[k][0] = v
    return ch


def field_charges():
    """The three oscillating families of the grid workload, plus a stationary and a
    uniformly moving charge."""
    w = I.workload_grid_mixed(grid_n=2, n_times=2)
    return I.concat_charges([w["charges"], one(I.STATIONARY, c0=[3e-9, -2e-9, 1e-9], q=-E),
                             one(I.UNIFORM_VELOCITY, c0=[-4e-9, 1e-9, 0.0], v=[0.3 * C, -0.1 * C, 0.05 * C])])


# ----------------------------------------------------------------------------
# oracle
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp64", "ld"])
def test_oracle_fields(drivers, prec):
    ch = field_charges()
    pts = np.concatenate([I.plane_grid(40e-9, 7, z=5e-9), np.array([[3e-9], [-2e-9], [1e-9]])], axis=1)
    times = np.array([0.0, 1.3e-16, 2.9e-16, 1e-15])
    arr, _ = O.pack(ch)
    with tempfile.TemporaryDirectory() as d:
        fc, fp, ft = (os.path.join(d, n) for n in ("ch.bin", "pts.bin", "t.bin"))
        open(fc, "wb").write(bytes(arr))
        save(fp, pts)
        save(ft, times)
        for kind in (O.TOTAL, O.COULOMB, O.RADIATION):
            fo, ff = os.path.join(d, "out.bin"), os.path.join(d, "flags.bin")
            out = run(drivers[prec], "fields", fc, fp, ft, kind, 1e-10, fo, ff)
            assert out.split() == ["status", "0"]
            got = np.fromfile(fo).reshape(len(times), 10, pts.shape[1])
            flags = np.fromfile(ff, dtype=np.uint32)
            ref, ref_flags = O.fields(ch, pts, times, kind=kind, extended=prec == "ld")
            np.testing.assert_array_equal(got, ref)
            np.testing.assert_array_equal(flags, ref_flags)
            assert flags[-1] & O.FLAG_MASKED


def test_oracle_single_pair_entry_points(drivers):
    ch = field_charges()
    arr, n = O.pack(ch)
    x, t = np.array([7e-9, -3e-9, 11e-9]), 2.1e-16
    with tempfile.TemporaryDirectory() as d:
        fc = os.path.join(d, "ch.bin")
        open(fc, "wb").write(bytes(arr))
        for i in range(n):
            lines = run(drivers["fp64"], "pair", fc, i, *x, t, O.TOTAL, 1e-10).splitlines()
            kin, tau, pair = (np.array([float(v) for v in ln.split()[1:]]) for ln in lines)
            assert kin[0] == 0 and tau[0] == 0
            np.testing.assert_array_equal(kin[1:], np.concatenate(O.kinematics(ch, i, t)))
            assert tau[1] == O.retarded_tau(ch, i, x, t)
            np.testing.assert_array_equal(pair[1:], O.lw_pair(ch, i, x, t))


def _dipole_cases():
    """(name, dipoles, offsets, dt, steps, policy, stride): a collinear pair under the
    strict rule, a 3 nm pair that extrapolates, and a batch of a moving pair and a
    three-dipole cluster."""
    dt = 2 * math.pi / W0 / 200
    strict = I.empty_dipoles(2)
    strict["origin"][1] = [20e-9, 0, 0]
    strict["omega0"][:] = W0
    strict["d0"][0] = E * 1e-12
    close = {k: np.array(v, copy=True) for k, v in strict.items()}
    close["origin"][1] = [3e-9, 0, 0]
    moving = I.empty_dipoles(5)
    moving["omega0"][:] = W0 * np.array([1.0, 1.01, 0.99, 1.0, 1.02])
    moving["origin"][:] = [[0, 0, 0], [30e-9, 5e-9, 0], [0, 0, 0], [15e-9, 0, 4e-9], [-9e-9, 12e-9, 0]]
    moving["axis"][:] = [[0, 0, 1], [0, 0, 1], [1, 0, 0], [0, 1, 0], [0.6, 0.8, 0]]
    moving["d0"][:] = E * 1e-12 * np.array([1, 0, 1, -0.5, 0])
    moving["motion_amp"][1] = [2e-9, 0, 1e-9]
    moving["motion_omega"][1] = 3e13
    moving["motion_phase"][1] = 0.7
    return [("strict", strict, [0, 2], dt, 300, O.DT_STRICT, 7),
            ("extrapolate", close, [0, 2], dt, 200, O.DT_EXTRAPOLATE, 1),
            ("moving_batch", moving, [0, 2, 5], dt, 250, O.DT_STRICT, 10)]


@pytest.mark.parametrize("prec", ["fp64", "ld"])
@pytest.mark.parametrize("case", [c[0] for c in _dipole_cases()])
def test_oracle_dipole_runs_and_detector_fields(drivers, prec, case):
    name, dip, off, dt, steps, policy, stride = next(c for c in _dipole_cases() if c[0] == case)
    pts = np.array([[40e-9, -25e-9, 5e-9], [10e-9, 35e-9, -30e-9], [20e-9, 0.0, 60e-9]])
    times = np.array([0.5 * steps * dt, steps * dt])
    ext = prec == "ld"
    with tempfile.TemporaryDirectory() as d:
        fd, fo = save(os.path.join(d, "dip.bin"), dip_records(dip)), save(os.path.join(d, "off.bin"), off, np.int32)
        fp, ft = save(os.path.join(d, "pts.bin"), pts), save(os.path.join(d, "t.bin"), times)
        pre = os.path.join(d, "run")
        out = run(drivers[prec], "dipole", fd, fo, dt, steps, policy, C / 100, stride, pre, fp, ft)
        assert out.split() == ["run", "0", "fields", "0"]
        ref = O.dipole_run(dip, off, dt, steps, policy=policy, out_stride=stride, want_hist=True, extended=ext)
        n, n_out = len(dip["omega0"]), steps // stride + 1
        for ext_name, key in (("d", "d"), ("v", "d_dot"), ("E", "energy"), ("Ed", "Ed"), ("Wabs", "W_abs"),
                              ("Wrad", "W_rad")):
            np.testing.assert_array_equal(np.fromfile(f"{pre}.{ext_name}").reshape(n_out, n), ref[key])
        np.testing.assert_array_equal(np.fromfile(f"{pre}.hist").reshape(steps + 1, n, 3), ref["hist"])
        field = O.dipole_fields(dip, dt, steps, ref["hist"], pts, times, extended=ext)
        np.testing.assert_array_equal(np.fromfile(f"{pre}.field").reshape(len(times), 3, pts.shape[1]), field)


@pytest.mark.parametrize("prec", ["fp64", "ld"])
def test_oracle_error_returns(drivers, prec):
    """The dt rule and the speed limit end a run with their status and free what it
    allocated (the leak check covers the early returns)."""
    dip = I.empty_dipoles(2)
    dip["origin"][1, 0] = 5e-9
    dip["omega0"][:] = W0
    dip["d0"][0] = E * 1e-12
    with tempfile.TemporaryDirectory() as d:
        fo = save(os.path.join(d, "off.bin"), [0, 2], np.int32)
        fd = save(os.path.join(d, "dip.bin"), dip_records(dip))
        out = run(drivers[prec], "dipole", fd, fo, 2.5e-17, 10, O.DT_STRICT, C / 100, 1, os.path.join(d, "r"))
        assert out.split() == ["run", "3"]
        dip["origin"][1, 0] = 20e-9
        dip["d0"][0] = E * 1e-8
        fd = save(os.path.join(d, "dip.bin"), dip_records(dip))
        out = run(drivers[prec], "dipole", fd, fo, 2.5e-17, 200, O.DT_STRICT, C / 100, 1, os.path.join(d, "r"))
        assert out.split() == ["run", "4"]


@pytest.mark.parametrize("prec", ["fp64", "ld"])
def test_oracle_history_reading(drivers, prec):
    rng = np.random.default_rng(17)
    n, n_dip, dt = 40, 3, 1e-17
    hist = rng.standard_normal((n + 1, n_dip, 3))
    d0 = rng.standard_normal(n_dip)
    with tempfile.TemporaryDirectory() as d:
        fh, f0 = save(os.path.join(d, "h.bin"), hist), save(os.path.join(d, "d0.bin"), d0)
        for jd in range(n_dip):
            for tp in (-3.2 * dt, 0.0, 17.25 * dt, n * dt, (n + 0.6) * dt):
                out = run(drivers[prec], "hist", fh, n_dip, jd, n, dt, f0, tp).split()
                assert out[:2] == ["hist", "0"]
                np.testing.assert_array_equal(np.array([float(v) for v in out[2:]]),
                                              O.hist_at(hist, jd, n, dt, d0, tp, extended=prec == "ld"))


# ----------------------------------------------------------------------------
# library host code
# ----------------------------------------------------------------------------

def _lib():
    from paper_2107_12437_amd import lw
    return lw, lw.load_library()


def test_host_theory_helpers(drivers):
    lw, _ = _lib()
    rng = np.random.default_rng(23)
    lines, expect = [], []
    for q, m in ((E, ME / 2), (20 * E, ME)):
        lines.append(f"gamma0 {q!r} {m!r} {W0!r}")
        expect.append(("gamma0", [lw.gamma0(q, m, W0)]))
    for R in (2e-9, 40e-9, 700e-9):
        for p1, p2 in (([0, 1, 0], [0, 1, 0]), ([1, 0, 0], [1, 0, 0]), tuple(I.unit_sphere(rng, 2))):
            Rv = R * I.unit_sphere(rng, 1)[0]
            lines.append("gf " + " ".join(repr(float(v)) for v in (*Rv, *p1, *p2, W0)))
            expect.append(("gf", [0, *lw.gf_pair(Rv, p1, p2, W0)]))
        Rv, p = np.array([R, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
        lines.append("modes " + " ".join(repr(float(v)) for v in (*Rv, *p, E, ME / 2, W0)))
        expect.append(("modes", [0, *lw.exact_modes(Rv, p, E, ME / 2, W0).values()]))
    lines.append("gf 0 0 0 0 1 0 0 1 0 " + repr(W0))           # coincident dipoles
    expect.append(("gf", None))
    lines.append("modes 1e-8 0 0 0 2 0 " + f"{E!r} {ME!r} {W0!r}")   # axis not a unit vector
    expect.append(("modes", None))
    out = run(drivers["host"], "theory", stdin="\n".join(lines) + "\n").splitlines()
    assert len(out) == len(expect)
    for ln, (op, vals) in zip(out, expect):
        f = ln.split()
        assert f[0] == op
        if vals is None:
            assert int(f[1]) == 1
        else:
            np.testing.assert_array_equal(np.array([float(v) for v in f[1:]]), np.array(vals, dtype=float))


def test_host_pair_modes(drivers):
    lw, _ = _lib()
    dt, stride, rows = 2 * math.pi / W0 / 200, 3, 1500
    t = np.arange(rows) * stride * dt
    g1, g2, w1, w2 = 2e12, 5e11, W0 * 1.002, W0 * 0.997
    plus, minus = np.exp(-g1 * t / 2) * np.cos(w1 * t), 0.4 * np.exp(-g2 * t / 2) * np.cos(w2 * t + 0.3)
    m = np.zeros((rows, 7))
    m[:, 0], m[:, 1] = plus + minus, plus - minus        # both modes
    m[:, 2], m[:, 3] = plus, plus                        # in-phase only
    m[:, 4:7] = np.stack([plus, minus, plus], axis=1)    # three dipoles: not a pair
    off = np.array([0, 2, 4, 7], dtype=np.int32)
    w_ref = np.full(3, W0)
    skip = np.array([30, 0, 0], dtype=np.int64)
    with tempfile.TemporaryDirectory() as d:
        fm, fo = save(os.path.join(d, "m.bin"), m), save(os.path.join(d, "off.bin"), off, np.int32)
        fw, fs = save(os.path.join(d, "w.bin"), w_ref), save(os.path.join(d, "s.bin"), skip, np.int64)
        fout = os.path.join(d, "out.bin")
        out = run(drivers["host"], "pair_modes", fm, 7, fo, dt, stride, fw, fs, fout)
        assert out.split()[:2] == ["pair_modes", "0"]
        got = np.fromfile(fout).reshape(3, 5)
    ref = lw.pair_modes(m, off, dt, stride, w_ref, skip)
    np.testing.assert_array_equal(got, ref)
    assert np.all(np.isnan(got[2])) and np.isnan(got[1, 1])
    assert abs(got[0, 0] - g1) < 1e-3 * g1 and abs(got[0, 1] - g2) < 1e-3 * g2


def _state_cases():
    """(name, dipoles, offsets, dt, precision, policy, stride, max_vel, ring_depth, status)."""
    dt = 2 * math.pi / W0 / 200
    base = I.empty_dipoles(3)
    base["origin"][:] = [[0, 0, 0], [30e-9, 0, 0], [0, 45e-9, 0]]
    base["axis"][:] = [[1, 0, 0], [0, 1, 0], [0, 0, 1]]
    base["omega0"][:] = W0

    def mod(**kw):
        d = {k: np.array(v, copy=True) for k, v in base.items()}
        for key, (idx, val) in kw.items():
            d[key][idx] = val
        return d

    off = [0, 1, 3]
    ok = (0, 0, 1, 0.0, 0)
    cases = [("valid", base, off, dt, *ok, 0),
             ("valid_mixed_ring", base, off, dt, 1, 0, 5, 0.0, 1024, 0),
             ("moving", mod(motion_amp=(1, [1e-9, 0, 0]), motion_omega=(1, 1e13)), off, dt, *ok, 0),
             ("ring_not_power_of_two", base, off, dt, 0, 0, 1, 0.0, 24, 1),
             ("ring_too_short", base, off, dt, 0, 0, 1, 0.0, 4, 1),
             ("dt_rule", mod(origin=(2, [32e-9, 0, 0])), off, dt, *ok, 3),
             ("dt_rule_extrapolate", mod(origin=(2, [32e-9, 0, 0])), off, dt, 0, 1, 1, 0.0, 0, 0),
             ("shared_origin", mod(origin=(2, [30e-9, 0, 0])), off, dt, *ok, 1),
             ("axis_not_unit", mod(axis=(0, [1, 1, 0])), off, dt, *ok, 1),
             ("omega0_zero", mod(omega0=(2, 0.0)), off, dt, *ok, 1),
             ("origin_nan", mod(origin=(0, [np.nan, 0, 0])), off, dt, *ok, 1),
             ("motion_too_fast", mod(motion_amp=(1, [1e-6, 0, 0]), motion_omega=(1, 1e14)), off, dt, *ok, 1),
             ("motion_without_frequency", mod(motion_amp=(1, [1e-9, 0, 0])), off, dt, *ok, 1),
             ("offsets_not_from_zero", base, [1, 1, 3], dt, *ok, 1),
             ("offsets_decreasing", base, [0, 3, 2, 3], dt, *ok, 1),
             ("offsets_short", base, [0, 2], dt, *ok, 1),
             ("unknown_precision", base, off, dt, 7, 0, 1, 0.0, 0, 1),
             ("unknown_policy", base, off, dt, 0, 5, 1, 0.0, 0, 1),
             ("stride_zero", base, off, dt, 0, 0, 0, 0.0, 0, 1),
             ("max_vel_nan", base, off, dt, 0, 0, 1, float("nan"), 0, 1),
             ("dt_zero", base, off, 0.0, *ok, 1),
             ("dt_too_fine", mod(origin=(1, [1e-3, 0, 0])), off, 1e-20, *ok, 1)]
    return cases


@pytest.mark.parametrize("case", [c[0] for c in _state_cases()])
def test_host_run_argument_checks(drivers, case):
    lw, L = _lib()
    _, dip, off, dt, prec, policy, stride, max_vel, ring, status = next(c for c in _state_cases() if c[0] == case)
    with tempfile.TemporaryDirectory() as d:
        fd = save(os.path.join(d, "dip.bin"), dip_records(dip))
        fo = save(os.path.join(d, "off.bin"), off, np.int32)
        f = run(drivers["host"], "state_size", fd, fo, dt, prec, policy, stride, max_vel, ring).split()
    assert f[0] == "state_size" and int(f[1]) == status, " ".join(f)
    arr, n = lw.pack_dipoles(dip)
    o = np.ascontiguousarray(off, dtype=np.int32)
    opts = lw.RunOpts(prec, policy, stride, max_vel, ring, 0)
    size = ct.c_int64(-1)
    st = L.lw_dipole_state_size(arr, n, o.ctypes.data_as(ct.POINTER(ct.c_int32)), len(o) - 1, float(dt),
                                ct.byref(opts), ct.byref(size))
    assert st == status
    if status == 0:
        assert int(f[2]) == size.value > 0


def test_host_entry_points_without_a_context(drivers):
    out = dict((ln.split()[0], ln.split()[1:]) for ln in run(drivers["host"], "null_ctx").splitlines())
    for name in ("sync_status", "set_autotune", "fields", "fields_noalloc", "fields_vjp", "dipole_run",
                 "dipole_state_size_null_out", "dipole_run_state", "dipole_run_vjp", "set_iteration_histogram",
                 "iteration_histogram"):
        assert out[name][0] == "1" and len(out[name]) > 1, (name, out[name])
    assert out["dipole_state_size"] == ["0"] and out["destroy"] == ["0"]


def test_host_create_without_a_device(drivers):
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible: the no-device error path cannot be reached")
    f = run(drivers["host"], "create").split()
    assert f[0] == "create" and int(f[1]) == 6 and len(f) > 2
