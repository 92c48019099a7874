"""FP64 CPU oracle of the Lienard-Wiechert hot path -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU baseline may import this
package.  It shares no code with the HIP library (the seeded input generators
aside) and never calls it.  The arithmetic lives in ``lw_oracle.c`` (plain C,
serial FP64); this module marshals numpy arrays through ctypes and holds the
host-side mode extraction in numpy (``extract``).
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

from . import build as _build

TOTAL, COULOMB, RADIATION = 0, 1, 2
DT_STRICT, DT_EXTRAPOLATE = 0, 1
FLAG_MASKED, FLAG_NOCONV = 1, 2
STATUS = {0: "ok", 1: "invalid", 2: "superluminal", 3: "dt too large", 4: "velocity", 5: "noconv",
          7: "nomem", 8: "non-finite state"}


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what}: status {code} ({STATUS.get(code, '?')})")
        self.code = code


class Traj(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("pad_", ct.c_int32), ("q", ct.c_double),
                ("c0", ct.c_double * 3), ("e1", ct.c_double * 3), ("e2", ct.c_double * 3),
                ("amp", ct.c_double), ("omega", ct.c_double), ("phase", ct.c_double),
                ("accel", ct.c_double), ("v", ct.c_double * 3)]


_libs: dict = {}


def lib(extended: bool = False):
    """The FP64 oracle library, or the same source built in x87 extended precision (a
    64-bit significand, about 3 more decimal digits) when `extended`."""
    if extended not in _libs:
        path = _build.build(force=False, extended=extended)
        L = ct.CDLL(path)
        dp = ct.POINTER(ct.c_double)
        L.or_traj_kin.argtypes = [ct.POINTER(Traj), ct.c_double, dp, dp, dp, dp]
        L.or_retarded_tau.argtypes = [ct.POINTER(Traj), dp, ct.c_double, dp, ct.POINTER(ct.c_int)]
        L.or_lw_pair.argtypes = [ct.POINTER(Traj), dp, ct.c_double, ct.c_int, ct.c_double, dp]
        L.or_lw_pair.restype = ct.c_uint
        L.or_fields.argtypes = [ct.POINTER(Traj), ct.c_int, dp, ct.c_int64, dp, ct.c_int, ct.c_int,
                                ct.c_double, dp, ct.POINTER(ct.c_uint32)]
        L.or_dipole_run.argtypes = [ct.c_int, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, ct.c_int,
                                    ct.POINTER(ct.c_int32), ct.c_double, ct.c_int64, ct.c_int,
                                    ct.c_double, ct.c_int64, dp, dp, dp, dp, dp, dp, dp]
        L.or_dipole_fields.argtypes = [ct.c_int, dp, dp, dp, dp, dp, dp, dp, dp, dp, ct.c_double, ct.c_int64, dp,
                                       dp, ct.c_int64, dp, ct.c_int, dp]
        L.or_hist_at.argtypes = [dp, ct.c_int, ct.c_int, ct.c_int64, ct.c_double, dp, ct.c_double, dp]
        L.or_real_digits.argtypes = []
        _libs[extended] = L
    return _libs[extended]


def real_digits(extended: bool = False) -> int:
    """Significand bits of the oracle's working precision (53, or 64 when extended)."""
    return lib(extended).or_real_digits()


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _motion(dip: dict, n: int):
    """Origin motion arrays (amplitude [n][3], omega, phase) or Nones for fixed origins."""
    if "motion_amp" not in dip or not np.any(dip["motion_amp"]):
        return None, None, None
    return (_f64(np.reshape(dip["motion_amp"], (n, 3))), _f64(dip["motion_omega"]), _f64(dip["motion_phase"]))


def pack(charges: dict):
    """ctypes array of Traj records from an inputs.py charge dict."""
    n = len(charges["kind"])
    arr = (Traj * max(n, 1))()
    for i in range(n):
        t = arr[i]
        t.kind = int(charges["kind"][i])
        t.q = float(charges["q"][i])
        for k in range(3):
            t.c0[k] = float(charges["c0"][i][k])
            t.e1[k] = float(charges["e1"][i][k])
            t.e2[k] = float(charges["e2"][i][k])
            t.v[k] = float(charges["v"][i][k])
        t.amp = float(charges["amp"][i])
        t.omega = float(charges["omega"][i])
        t.phase = float(charges["phase"][i])
        t.accel = float(charges["accel"][i])
    return arr, n


def kinematics(charges: dict, i: int, t: float):
    arr, _ = pack(charges)
    r, v, a, j = (np.zeros(3) for _ in range(4))
    st = lib().or_traj_kin(ct.byref(arr[i]), float(t), _dp(r), _dp(v), _dp(a), _dp(j))
    if st:
        raise OracleError(st, "kinematics")
    return r, v, a, j


def retarded_tau(charges: dict, i: int, x, t: float) -> float:
    arr, _ = pack(charges)
    xx = _f64(x)
    tau = ct.c_double()
    it = ct.c_int()
    st = lib().or_retarded_tau(ct.byref(arr[i]), _dp(xx), float(t), ct.byref(tau), ct.byref(it))
    if st:
        raise OracleError(st, "retarded time")
    return tau.value


def lw_pair(charges: dict, i: int, x, t: float, kind: int = TOTAL, mask_r: float = 0.0):
    """Ten outputs (Phi, A, E, B) of charge i alone; None when masked."""
    arr, _ = pack(charges)
    xx = _f64(x)
    out = np.zeros(10)
    f = lib().or_lw_pair(ct.byref(arr[i]), _dp(xx), float(t), int(kind), float(mask_r), _dp(out))
    return None if f else out


def fields(charges: dict, points, times, kind: int = TOTAL, mask_radius: float = 1e-10, extended: bool = False):
    """[n_times][10][n_pts] outputs (FP64, or computed in extended precision and rounded
    to FP64 when `extended`) and per-point flags."""
    arr, n = pack(charges)
    pts = _f64(points)
    assert pts.ndim == 2 and pts.shape[0] == 3
    tms = _f64(np.atleast_1d(times))
    npts = pts.shape[1]
    out = np.empty((len(tms), 10, npts))
    flags = np.zeros(npts, dtype=np.uint32)
    st = lib(extended).or_fields(arr, n, _dp(pts), npts, _dp(tms), len(tms), int(kind), float(mask_radius),
                         _dp(out), flags.ctypes.data_as(ct.POINTER(ct.c_uint32)))
    if st:
        raise OracleError(st, "fields")
    return out, flags


def dipole_run(dipoles: dict, inst_off, dt: float, steps: int, policy: int = DT_STRICT,
               max_vel: float = 299792458.0 / 100, out_stride: int = 1, want_hist: bool = False,
               extended: bool = False):
    """Runs Algorithm 1 on independent instances.  Returns dict of [n_out][n_dip] arrays
    d, d_dot, energy, Ed, W_abs, W_rad (and hist [(steps+1)][n_dip][3] when asked).  Optional keys
    motion_amp [n][3], motion_omega, motion_phase move the origins as
    origin + motion_amp cos(motion_omega t + motion_phase) (Sec. 4.3).  `extended` runs the
    extended-precision build (state and arithmetic in long double, outputs rounded to FP64)."""
    dip = {k: _f64(v) for k, v in dipoles.items()}
    n = len(dip["omega0"])
    off = np.ascontiguousarray(inst_off, dtype=np.int32)
    n_out = steps // out_stride + 1
    res = {k: np.empty((n_out, n)) for k in ("d", "d_dot", "energy", "Ed", "W_abs", "W_rad")}
    hist = np.empty((steps + 1, n, 3)) if want_hist else None
    mamp, mom, mph = _motion(dip, n)
    st = lib(extended).or_dipole_run(n, _dp(dip["origin"]), _dp(dip["axis"]), _dp(dip["omega0"]), _dp(dip["q"]),
                             _dp(dip["m1"]), _dp(dip["m2"]), _dp(dip["d0"]),
                             _dp(mamp) if mamp is not None else None, _dp(mom) if mom is not None else None,
                             _dp(mph) if mph is not None else None, len(off) - 1,
                             off.ctypes.data_as(ct.POINTER(ct.c_int32)), float(dt), int(steps),
                             int(policy), float(max_vel), int(out_stride), _dp(res["d"]),
                             _dp(res["d_dot"]), _dp(res["energy"]), _dp(res["Ed"]), _dp(res["W_abs"]),
                             _dp(res["W_rad"]), _dp(hist) if hist is not None else None)
    if st:
        raise OracleError(st, "dipole run")
    if hist is not None:
        res["hist"] = hist
    return res


def hist_at(hist, jd: int, n: int, dt: float, d0, tp: float, extended: bool = False):
    """(d, d_dot, d_ddot) of dipole jd at time tp read from samples 0..n of a history
    [(n+1)][n_dip][3], as the oscillator run and the detector field read it."""
    h = _f64(hist)
    d0a = _f64(d0)
    out = np.zeros(3)
    st = lib(extended).or_hist_at(_dp(h), h.shape[1], int(jd), int(n), float(dt), _dp(d0a), float(tp), _dp(out))
    if st:
        raise OracleError(st, "history reading")
    return out


def dipole_fields(dipoles: dict, dt: float, steps: int, hist, points, times, extended: bool = False):
    """E ([n_times][3][n_pts]) of all dipole charges from a finished run's history."""
    dip = {k: _f64(v) for k, v in dipoles.items()}
    n = len(dip["omega0"])
    h = _f64(hist)
    pts = _f64(points)
    tms = _f64(np.atleast_1d(times))
    out = np.empty((len(tms), 3, pts.shape[1]))
    mamp, mom, mph = _motion(dip, n)
    st = lib(extended).or_dipole_fields(n, _dp(dip["origin"]), _dp(dip["axis"]), _dp(dip["q"]), _dp(dip["m1"]),
                                _dp(dip["m2"]), _dp(dip["d0"]),
                                _dp(mamp) if mamp is not None else None, _dp(mom) if mom is not None else None,
                                _dp(mph) if mph is not None else None, float(dt), int(steps), _dp(h), _dp(pts),
                                pts.shape[1], _dp(tms), len(tms), _dp(out))
    if st:
        raise OracleError(st, "dipole fields")
    return out
