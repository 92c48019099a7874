"""Mode extraction from two-dipole runs -- oracle side, TEST INFRASTRUCTURE ONLY.

The paper reads the collective decay rate gamma^+- and the frequency shift
delta_12 of two coupled oscillators off the oscillation of their energy after a
transient (Sec. 2.4, Eq. (KE)).  For identical dipoles the sum s = d1 + d2 and
the difference a = d1 - d2 are the normal coordinates (in-phase and
anti-phase, the classical super- and subradiant states).  Each is a single
damped oscillation after the transient, so an order-2 linear-prediction
(Prony) least-squares fit recovers its complex frequency exactly:

    x[k + 2L] = c1 x[k + L] + c0 x[k],   z^2 - c1 z - c0 = 0,
    z = exp((-gamma/2 + i omega) L Delta),

with Delta the sample spacing and L a lag of about a quarter period (energy
decays at gamma, so the amplitude decays at gamma/2).  delta_omega is
(omega+ - omega-)/2, which cancels the shifts common to both modes.
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 299792458.0


def prony2(x: np.ndarray, lag: int, delta: float):
    """(gamma, omega) of a damped oscillation sampled every ``delta`` seconds."""
    x = np.asarray(x, dtype=np.float64)
    L = int(lag)
    if len(x) < 2 * L + 2:
        raise ValueError("signal too short for the lag")
    X = np.stack([x[L:-L], x[:-2 * L]], axis=1)
    y = x[2 * L:]
    (c1, c0), *_ = np.linalg.lstsq(X, y, rcond=None)
    disc = c1 * c1 + 4.0 * c0
    if disc >= 0:
        return float("nan"), float("nan")
    r = math.sqrt(-c0)
    theta = math.atan2(math.sqrt(-disc) / 2.0, c1 / 2.0)
    gamma = -2.0 * math.log(r) / (L * delta)
    omega = theta / (L * delta)
    return gamma, omega


def default_skip(dt: float, separation: float) -> int:
    """Transient skipped before fitting, in steps: the larger of 2,000 steps and three
    light-crossing times of the pair."""
    return max(2000, int(math.ceil(3.0 * separation / (C_LIGHT * dt))))


def pair_modes(d1, d2, dt: float, stride: int, omega0: float, skip_steps: int,
               min_ratio: float = 1e-6):
    """gamma+, gamma-, omega+, omega-, delta_omega of one two-dipole run.

    A mode whose RMS is below ``min_ratio`` times the other's is reported as NaN,
    and delta_omega then falls back to omega+ - omega0 (or omega0 - omega-)."""
    delta = dt * stride
    k0 = int(math.ceil(skip_steps / stride))
    s = (np.asarray(d1) + np.asarray(d2))[k0:]
    a = (np.asarray(d1) - np.asarray(d2))[k0:]
    lag = max(1, int(round(math.pi / (2.0 * omega0 * delta))))
    rs, ra = float(np.sqrt(np.mean(s * s))), float(np.sqrt(np.mean(a * a)))
    gp = wp = gm = wm = float("nan")
    if rs > min_ratio * ra:
        gp, wp = prony2(s, lag, delta)
    if ra > min_ratio * rs:
        gm, wm = prony2(a, lag, delta)
    if np.isfinite(wp) and np.isfinite(wm):
        dw = 0.5 * (wp - wm)
    elif np.isfinite(wp):
        dw = wp - omega0
    else:
        dw = omega0 - wm
    return {"gamma_plus": gp, "gamma_minus": gm, "omega_plus": wp, "omega_minus": wm,
            "delta_omega": dw}
