"""Seeded synthetic workloads for the Lienard-Wiechert hot path.

This module is the only code shared by the FP64 oracle (``oracle/``) and the
HIP path: it draws sources, observation points and snapshot times, and holds
none of the method's arithmetic (no retarded times, no fields, no dynamics).
Every draw uses ``numpy.random.default_rng(12437 + k)`` for workload k, so the
same inputs reach both sides.

Trajectory records are plain dicts of numpy arrays with the fields

    kind   int32[n]   STATIONARY, UNIFORM_VELOCITY, LINEAR_OSC, CIRCULAR, ACCEL
    q      f64[n]     charge (C)
    c0     f64[n,3]   centre / rest position (m)
    e1,e2  f64[n,3]   unit axes (oscillation axis, orbit plane)
    amp    f64[n]     amplitude or orbit radius (m)
    omega  f64[n]     angular frequency (rad/s)
    phase  f64[n]     phase at t = 0 (rad)
    accel  f64[n]     acceleration magnitude along e1 (m/s^2)
    v      f64[n,3]   constant velocity (m/s)

matching the parametric point-charge trajectories of the paper (Sec. 3.1: a
charge is its value q plus x(t), y(t), z(t)).  Dipole records describe the
Lorentz oscillators of Sec. 2.3 (origin, polarisation axis, omega_0, q, the two
masses, initial moment d0 along the axis) grouped into independent instances
by a CSR offset array.

Physical constants here are CODATA 2018 (the values scipy.constants carried
when the paper was written); the oracle and the HIP library each define their
own copy.
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 299792458.0
E_CHARGE = 1.602176634e-19
M_E = 9.1093837015e-31

STATIONARY, UNIFORM_VELOCITY, LINEAR_OSC, CIRCULAR, ACCEL = 0, 1, 2, 3, 4

SEED_BASE = 12437


def rng_for(k: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + k)


# ----------------------------------------------------------------------------
# record builders
# ----------------------------------------------------------------------------

def empty_charges(n: int) -> dict:
    return {
        "kind": np.zeros(n, np.int32),
        "q": np.zeros(n),
        "c0": np.zeros((n, 3)),
        "e1": np.tile([1.0, 0.0, 0.0], (n, 1)),
        "e2": np.tile([0.0, 1.0, 0.0], (n, 1)),
        "amp": np.zeros(n),
        "omega": np.zeros(n),
        "phase": np.zeros(n),
        "accel": np.zeros(n),
        "v": np.zeros((n, 3)),
    }


def concat_charges(parts: list[dict]) -> dict:
    return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}


def subset_charges(ch: dict, idx) -> dict:
    return {k: np.ascontiguousarray(v[idx]) for k, v in ch.items()}


def unit_sphere(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def orbit_basis(normal: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Two unit vectors spanning the plane orthogonal to ``normal``."""
    n = normal / np.linalg.norm(normal)
    helper = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(n, helper)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(n, e1)
    return e1, e2


def plane_grid(half: float, n: int, z: float = 0.0) -> np.ndarray:
    """SoA [3, n*n] points of ``meshgrid(linspace(-half, half, n), ..., indexing='ij')``
    at height z (the grid layout of the paper's Listing 1)."""
    coord = np.linspace(-half, half, n)
    x, y = np.meshgrid(coord, coord, indexing="ij")
    pts = np.empty((3, n * n))
    pts[0] = x.ravel()
    pts[1] = y.ravel()
    pts[2] = z
    return pts


# ----------------------------------------------------------------------------
# grid workloads
# ----------------------------------------------------------------------------

def circular_charge(q, centre, radius, omega, phase=0.0, e1=(1, 0, 0), e2=(0, 1, 0)) -> dict:
    ch = empty_charges(1)
    ch["kind"][0] = CIRCULAR
    ch["q"][0] = q
    ch["c0"][0] = centre
    ch["e1"][0] = e1
    ch["e2"][0] = e2
    ch["amp"][0] = radius
    ch["omega"][0] = omega
    ch["phase"][0] = phase
    return ch


def workload_tiny_orbit(grid_n: int = 64) -> dict:
    """One +e charge on a 1 nm circular orbit at 0.3c in the z = 0 plane, observed on a
    grid_n x grid_n grid over +-50 nm at t = 10 orbital periods (FP64 method)."""
    radius = 1e-9
    omega = 0.3 * C_LIGHT / radius
    charges = circular_charge(E_CHARGE, (0, 0, 0), radius, omega)
    return {
        "name": "orbit-1q-64x64",
        "charges": charges,
        "points": plane_grid(50e-9, grid_n),
        "times": np.array([10 * 2 * math.pi / omega]),
    }


def random_grid_charges(rng: np.random.Generator, n: int, families=(LINEAR_OSC, CIRCULAR, ACCEL),
                        t_end: float = 1e-15, cube_half: float = 10e-9) -> dict:
    """Seeded sources for the mixed-precision grid workload: half +e, half -e, each drawn
    from linear oscillation, circular orbit or uniform acceleration from rest."""
    signs = np.array([1.0] * (n // 2) + [-1.0] * (n - n // 2))
    signs = rng.permutation(signs)
    ch = empty_charges(n)
    fam = rng.integers(0, len(families), size=n)
    for i in range(n):
        kind = families[fam[i]]
        ch["kind"][i] = kind
        ch["q"][i] = signs[i] * E_CHARGE
        ch["c0"][i] = rng.uniform(-cube_half, cube_half, size=3)
        if kind == LINEAR_OSC:
            u = unit_sphere(rng, 1)[0]
            a = rng.uniform(0.1e-9, 2e-9)
            vmax = rng.uniform(0.1, 0.5) * C_LIGHT
            ch["e1"][i] = u
            ch["e2"][i] = orbit_basis(u)[0]
            ch["amp"][i] = a
            ch["omega"][i] = vmax / a
            ch["phase"][i] = rng.uniform(0, 2 * math.pi)
        elif kind == CIRCULAR:
            normal = unit_sphere(rng, 1)[0]
            e1, e2 = orbit_basis(normal)
            r = rng.uniform(0.5e-9, 2e-9)
            speed = rng.uniform(0.1, 0.5) * C_LIGHT
            ch["e1"][i] = e1
            ch["e2"][i] = e2
            ch["amp"][i] = r
            ch["omega"][i] = speed / r
            ch["phase"][i] = rng.uniform(0, 2 * math.pi)
        elif kind == ACCEL:
            u = unit_sphere(rng, 1)[0]
            alpha = rng.uniform(0.1, 1.0)
            ch["e1"][i] = u
            ch["e2"][i] = orbit_basis(u)[0]
            ch["accel"][i] = alpha * 0.6 * C_LIGHT / t_end
        else:
            raise ValueError(kind)
    return ch


def workload_grid_mixed(grid_n: int = 512, n_times: int = 64, n_charges: int = 16) -> dict:
    """16 charges of three families in a 20 nm cube, 512x512 plane over +-100 nm, 64
    snapshots over the first femtosecond (mixed-precision grid workload)."""
    rng = rng_for(2)
    t_end = 1e-15
    charges = random_grid_charges(rng, n_charges, t_end=t_end)
    times = (np.arange(n_times) + 1) * t_end / n_times
    return {
        "name": f"grid-{n_charges}q-{grid_n}x{grid_n}-{n_times}t",
        "charges": charges,
        "points": plane_grid(100e-9, grid_n),
        "times": times,
    }


def workload_uniform_velocity(grid_n: int = 512, n_times: int = 64, n_charges: int = 16) -> dict:
    """Same geometry as the mixed grid workload with every charge in uniform motion
    (speeds U[0.1, 0.5]c): the retarded time has a closed form, so the run isolates
    the cost of the field expressions."""
    rng = rng_for(12)
    ch = empty_charges(n_charges)
    signs = rng.permutation([1.0] * (n_charges // 2) + [-1.0] * (n_charges - n_charges // 2))
    for i in range(n_charges):
        ch["kind"][i] = UNIFORM_VELOCITY
        ch["q"][i] = signs[i] * E_CHARGE
        ch["c0"][i] = rng.uniform(-10e-9, 10e-9, size=3)
        ch["v"][i] = unit_sphere(rng, 1)[0] * rng.uniform(0.1, 0.5) * C_LIGHT
    times = (np.arange(n_times) + 1) * 1e-15 / n_times
    return {
        "name": f"grid-uv-{n_charges}q-{grid_n}x{grid_n}-{n_times}t",
        "charges": ch,
        "points": plane_grid(100e-9, grid_n),
        "times": times,
    }


def workload_detector(grid_n: int = 256, n_times: int = 32, n_charges: int = 64) -> dict:
    """64 circular-orbit charges (signs 32/32) seen by a detector plane at z = 200 nm,
    32 snapshots over 1 fs (grid adjoint workload)."""
    rng = rng_for(4)
    ch = random_grid_charges(rng, n_charges, families=(CIRCULAR,))
    times = (np.arange(n_times) + 1) * 1e-15 / n_times
    return {
        "name": f"detector-{n_charges}q-{grid_n}x{grid_n}-{n_times}t",
        "charges": ch,
        "points": plane_grid(100e-9, grid_n, z=200e-9),
        "times": times,
    }


def current_loop(n_charges: int, radius: float, speed: float, q: float = E_CHARGE,
                 normal=(0.0, 0.0, 1.0), center=(0.0, 0.0, 0.0)) -> dict:
    """n equal charges sharing one circular orbit at phases 2 pi k / n: a ring charge
    n q with the steady current n q omega / (2 pi) once n is large (a continuous
    source approximated by point charges, Sec. 2.2)."""
    e1, e2 = orbit_basis(np.asarray(normal, float))
    ch = empty_charges(n_charges)
    ch["kind"][:] = CIRCULAR
    ch["q"][:] = q
    ch["c0"][:] = center
    ch["e1"][:] = e1
    ch["e2"][:] = e2
    ch["amp"][:] = radius
    ch["omega"][:] = speed / radius
    ch["phase"][:] = 2 * math.pi * np.arange(n_charges) / n_charges
    return ch


def workload_many_charges(n_charges: int = 1024, grid_n: int = 256, n_times: int = 8) -> dict:
    """Many-charge source: four current loops of n/4 charges each (radii 5-20 nm, speeds
    0.01-0.1 c, seeded orientations, alternating signs, centres below z = 0, so every
    charge stays 10 nm below the plane), seen on a 256x256 plane over +-100 nm at
    z = 30 nm, 8 snapshots over 1 fs."""
    rng = rng_for(6)
    loops = []
    per = n_charges // 4
    for k in range(4):
        normal = unit_sphere(rng, 1)[0]
        loops.append(current_loop(per if k < 3 else n_charges - 3 * per, rng.uniform(5e-9, 20e-9),
                                  rng.uniform(0.01, 0.1) * C_LIGHT, q=E_CHARGE * (1 if k % 2 == 0 else -1),
                                  normal=normal,
                                  center=[rng.uniform(-20e-9, 20e-9), rng.uniform(-20e-9, 20e-9),
                                          rng.uniform(-20e-9, 0.0)]))
    return {
        "name": f"loops-{n_charges}q-{grid_n}x{grid_n}-{n_times}t",
        "charges": concat_charges(loops),
        "points": plane_grid(100e-9, grid_n, z=30e-9),
        "times": (np.arange(n_times) + 1) * 1e-15 / n_times,
    }


# ----------------------------------------------------------------------------
# Lorentz-oscillator workloads
# ----------------------------------------------------------------------------

def empty_dipoles(n: int) -> dict:
    return {
        "origin": np.zeros((n, 3)),
        "axis": np.tile([1.0, 0.0, 0.0], (n, 1)),
        "omega0": np.zeros(n),
        "q": np.full(n, E_CHARGE),
        "m1": np.full(n, M_E),
        "m2": np.full(n, M_E),
        "d0": np.zeros(n),
        # origin motion: origin + motion_amp cos(motion_omega t + motion_phase) (Sec. 4.3)
        "motion_amp": np.zeros((n, 3)),
        "motion_omega": np.zeros(n),
        "motion_phase": np.zeros(n),
    }


def concat_dipoles(parts: list[dict]) -> dict:
    return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}


def workload_dipole_pairs(n_inst: int = 256, steps: int = 20000, orientation: str = "p",
                          seps=None, d0_both: bool = False, omega0: float = 2 * math.pi * 200e12,
                          steps_per_period: int = 200) -> dict:
    """Independent two-dipole instances: dipole 1 at the origin, dipole 2 at (s, 0, 0),
    separations log-uniform in [1 nm, 1 um].  orientation 'p' polarises both along x
    (collinear), 's' along y (side by side).  Dipole 1 starts displaced by 1e-12 m (both
    dipoles when d0_both, the in-phase start of the paper's Listing 2)."""
    rng = rng_for(3)
    if seps is None:
        seps = np.exp(rng.uniform(math.log(1e-9), math.log(1e-6), size=n_inst))
    seps = np.asarray(seps, dtype=float)
    n_inst = len(seps)
    dip = empty_dipoles(2 * n_inst)
    axis = [1.0, 0.0, 0.0] if orientation == "p" else [0.0, 1.0, 0.0]
    dip["axis"][:] = axis
    dip["origin"][1::2, 0] = seps
    dip["omega0"][:] = omega0
    dip["d0"][0::2] = E_CHARGE * 1e-12
    if d0_both:
        dip["d0"][1::2] = E_CHARGE * 1e-12
    t0 = 2 * math.pi / omega0
    return {
        "name": f"pairs-{orientation}-{n_inst}x2-{steps}steps",
        "dipoles": dip,
        "inst_off": np.arange(0, 2 * n_inst + 1, 2, dtype=np.int32),
        "dt": t0 / steps_per_period,
        "steps": steps,
        "separations": seps,
    }


def place_min_spacing(rng: np.random.Generator, n: int, half: float, min_sep: float) -> np.ndarray:
    """Rejection-sample n points uniform in a cube of half-width ``half`` with pairwise
    distance >= min_sep."""
    pts = np.empty((n, 3))
    k = 0
    tries = 0
    while k < n:
        p = rng.uniform(-half, half, size=3)
        tries += 1
        if tries > 10000 * n:
            raise RuntimeError("cannot place points with the requested spacing")
        if k and np.min(np.linalg.norm(pts[:k] - p, axis=1)) < min_sep:
            continue
        pts[k] = p
        k += 1
    return pts


def cluster_dipoles(rng: np.random.Generator, n: int, half: float, min_sep: float,
                    omega_mean: float, omega_rel_sigma: float, random_sign: bool) -> dict:
    dip = empty_dipoles(n)
    dip["origin"][:] = place_min_spacing(rng, n, half, min_sep)
    dip["axis"][:] = unit_sphere(rng, n)
    dip["omega0"][:] = omega_mean * (1.0 + omega_rel_sigma * rng.normal(size=n)) \
        if omega_rel_sigma else omega_mean
    sign = rng.choice([-1.0, 1.0], size=n) if random_sign else np.ones(n)
    dip["d0"][:] = sign * E_CHARGE * 1e-12
    return dip


def workload_clusters(n_clusters: int = 64, steps: int = 50000, n_min: int = 2, n_max: int = 1024,
                      sizes=None) -> dict:
    """Uneven batch: cluster sizes log-uniform in [2, 1024], positions uniform in a 500 nm
    cube with >= 10 nm spacing, axes uniform on the sphere, omega_0 ~ N(2 pi 200 THz, 1%),
    every dipole displaced by 1e-12 m along its axis with a random sign."""
    rng = rng_for(5)
    if sizes is None:
        sizes = np.round(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_clusters)))
    sizes = np.asarray(sizes, dtype=np.int64)
    parts = [cluster_dipoles(rng, int(n), 250e-9, 10e-9, 2 * math.pi * 200e12, 0.01, True)
             for n in sizes]
    off = np.zeros(len(sizes) + 1, dtype=np.int32)
    off[1:] = np.cumsum(sizes)
    t0 = 2 * math.pi / (2 * math.pi * 200e12)
    return {
        "name": f"clusters-{len(sizes)}-{int(sizes.sum())}dip-{steps}steps",
        "dipoles": concat_dipoles(parts),
        "inst_off": off,
        "dt": t0 / 200,
        "steps": steps,
        "sizes": sizes,
    }


def workload_dipole_detector(n_dip: int = 32, steps: int = 5000, grid_n: int = 256, n_snap: int = 32) -> dict:
    """32 dipoles in a 100 nm cube (>= 10 nm spacing) run for 5,000 steps at T0/200 and
    observed on a detector plane at z = 200 nm at 32 snapshots (LO adjoint workload), with
    the adjoint checkpointed every 250 steps."""
    rng = rng_for(44)
    dip = cluster_dipoles(rng, n_dip, 50e-9, 10e-9, 2 * math.pi * 200e12, 0.0, False)
    t0 = 1.0 / 200e12
    dt = t0 / 200
    return {
        "name": f"dipdet-{n_dip}-{steps}steps-{grid_n}x{grid_n}-{n_snap}t",
        "dipoles": dip,
        "inst_off": np.array([0, n_dip], dtype=np.int32),
        "dt": dt,
        "steps": steps,
        "points": plane_grid(100e-9, grid_n, z=200e-9),
        "times": (np.arange(n_snap) + 1) * steps * dt / n_snap,
        "ckpt_every": 250,
    }
