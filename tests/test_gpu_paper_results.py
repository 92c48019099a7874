"""The paper's coupled-dipole results reproduced on the GPU (Sec. 4.2, Figs. 9-11).

Each instance is a pair of identical s or p dipoles, with one dipole excited at t = 0.
The pairs run together in one batch on the GPU. The library's host extraction
(lw_pair_modes) takes the collective rates gamma+- and the shift delta_omega from the
moments. The results are compared two ways.

Against the Green's-function rates of App. A (lw_gf_pair), for separations of at least
7.5 nm: within the paper's 0.2 %, the bound it states for its own simulations against
theory. Below that separation the Markov rates, which are first order in the coupling,
drift from the classical result. There the comparison is against the exact classical
normal modes (lw_exact_modes): gamma+- to 1e-3 gamma_0 and delta_omega to 1e-3.

At 3 nm the exact-mode comparison is replaced by one against the FP64 oracle's run,
extracted the same way (1e-3 gamma_0). There the model's rates differ from the exact
normal modes by about 4e-3 gamma_0 for s dipoles. That difference is the same on the
oracle, does not change with dt (T0/2000 to T0/8000), and scales as R^-6, i.e. second
order in the coupling. At 5 nm it is below 2e-4.
"""
import math

import numpy as np
import pytest

from oracle import extract as X
from paper_2107_12437_amd import inputs as I
from tests.helpers import gpu_ready

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]

W0 = 2 * math.pi * 200e12
SEPS = np.array([3e-9, 5e-9, 8e-9, 15e-9, 30e-9, 80e-9, 200e-9, 600e-9])
STEPS, SPP, STRIDE = 40000, 2000, 4


@pytest.mark.parametrize("orientation", ["s", "p"])
def test_collective_rates_against_theory(orientation):
    import oracle as O
    from paper_2107_12437_amd import lw
    w = I.workload_dipole_pairs(seps=SEPS, orientation=orientation, steps=STEPS, steps_per_period=SPP)
    r = lw.dipole_run(w["dipoles"], w["inst_off"], w["dt"], w["steps"], policy="extrapolate", out_stride=STRIDE)
    skips = [X.default_skip(w["dt"], s) for s in SEPS]
    modes = lw.pair_modes(r["d"], w["inst_off"], w["dt"], STRIDE, W0, skips)
    g0 = lw.gamma0(I.E_CHARGE, I.M_E / 2, W0)
    p = np.array([1.0, 0.0, 0.0]) if orientation == "p" else np.array([0.0, 1.0, 0.0])
    sep_dir = np.array([1.0, 0.0, 0.0])
    for k, R in enumerate(SEPS):
        gp, gm, _, _, dw = modes[k]
        if R < 5e-9:
            one = {key: np.array(v)[2 * k:2 * k + 2] for key, v in w["dipoles"].items()}
            ro = O.dipole_run(one, [0, 2], w["dt"], STEPS, policy=O.DT_EXTRAPOLATE, out_stride=STRIDE)
            ref = X.pair_modes(ro["d"][:, 0], ro["d"][:, 1], w["dt"], STRIDE, W0, skips[k])
        else:
            ref = lw.exact_modes(R * sep_dir, p, I.E_CHARGE, I.M_E / 2, W0)
        assert abs(gp - ref["gamma_plus"]) <= 1e-3 * g0, (orientation, R, "gamma+", gp / g0, ref["gamma_plus"] / g0)
        assert abs(gm - ref["gamma_minus"]) <= 1e-3 * g0, (orientation, R, "gamma-", gm / g0, ref["gamma_minus"] / g0)
        assert abs(dw - ref["delta_omega"]) <= 1e-3 * max(abs(ref["delta_omega"]), g0), (orientation, R, dw / g0)
        if R >= 7.5e-9:
            d12, g12 = lw.gf_pair(R * sep_dir, p, p, W0)
            assert abs(gp / g0 - (1 + g12)) <= 2e-3 * (1 + abs(g12)), (orientation, R, gp / g0, 1 + g12)
            assert abs(dw / g0 - d12) <= 2e-3 * max(abs(d12), 1.0), (orientation, R, dw / g0, d12)


# the paper's own regime (Sec. 4.2, Fig. 9): superradiant (in-phase) s and p pairs at
# 1e4 steps per period, 40,000 steps as in Listing 2
SEPS16 = np.geomspace(7.5e-9, 1e-6, 16)
PAPER_MEAN_REL = {"p": (0.0015, 0.0004), "s": (0.0019, 0.0013)}     # delta_12, gamma+ (Fig. 9 caption)


def paper_regime_errors():
    """Mean relative errors of delta_12 and gamma+ against the Green's-function rates for
    16 separations in [7.5 nm, 1 um] of in-phase s and p pairs, all 32 pairs in one
    lw_dipole_run call at dt = T0/1e4 for 40,000 steps, with the call's own gamma and
    delta_omega outputs.  delta_12 errors are relative to max(|delta_12|, gamma_0), since
    the s pairs' shift crosses zero near 0.3 um."""
    from paper_2107_12437_amd import lw
    ws = [I.workload_dipole_pairs(seps=SEPS16, orientation=o, steps=40000, steps_per_period=10000, d0_both=True)
          for o in ("p", "s")]
    dip = I.concat_dipoles([w["dipoles"] for w in ws])
    off = np.arange(0, 4 * len(SEPS16) + 1, 2, dtype=np.int32)
    dt = ws[0]["dt"]
    r = lw.dipole_run(dip, off, dt, 40000, policy="strict", out_stride=5, modes=True)
    g0 = lw.gamma0(I.E_CHARGE, I.M_E / 2, W0)
    out = {}
    for oi, o in enumerate(("p", "s")):
        axis = np.array([1.0, 0.0, 0.0]) if o == "p" else np.array([0.0, 1.0, 0.0])
        ed, eg = [], []
        for k, R in enumerate(SEPS16):
            inst = oi * len(SEPS16) + k
            d12, g12 = lw.gf_pair(np.array([R, 0.0, 0.0]), axis, axis, W0)
            ed.append(abs(r["delta_omega"][inst] / g0 - d12) / max(abs(d12), 1.0))
            eg.append(abs(r["gamma"][inst, 0] / g0 - (1 + g12)) / (1 + g12))
        out[o] = {"delta12_mean_rel": float(np.mean(ed)), "gamma_plus_mean_rel": float(np.mean(eg)),
                  "delta12_max_rel": float(np.max(ed)), "gamma_plus_max_rel": float(np.max(eg))}
    return out


def test_paper_regime_superradiant_pairs():
    """Sec. 4.2 at the paper's own step (1e4 per period): the mean relative errors of
    delta_12 and gamma+ of superradiant s and p pairs over 16 separations from 7.5 nm to
    1 um stay within the paper's 0.2 % bound (its Fig. 9 reports 0.15 % / 0.04 % for p and
    0.19 % / 0.13 % for s dipoles)."""
    res = paper_regime_errors()
    for o, r in res.items():
        print(f"{o} pairs: delta_12 mean {100 * r['delta12_mean_rel']:.4f} % (paper "
              f"{100 * PAPER_MEAN_REL[o][0]:.2f} %), gamma+ mean {100 * r['gamma_plus_mean_rel']:.4f} % (paper "
              f"{100 * PAPER_MEAN_REL[o][1]:.2f} %); max {100 * r['delta12_max_rel']:.4f} %, "
              f"{100 * r['gamma_plus_max_rel']:.4f} %")
        assert r["delta12_mean_rel"] <= 2e-3 and r["gamma_plus_mean_rel"] <= 2e-3, (o, r)
        assert r["delta12_max_rel"] <= 2e-3 and r["gamma_plus_max_rel"] <= 2e-3, (o, r)
