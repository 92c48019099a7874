#!/usr/bin/env python3
"""Benchmark of the Lienard-Wiechert hot path on one MI355X.

A step is one lw_fields call on the mixed-precision grid workload: 16 charges
(linear oscillation, circular orbit, uniform acceleration; seeded), a 512x512
plane over +-100 nm, 64 snapshots over the first femtosecond -- FP64 retarded
times, FP32 field expressions summed over charges in FP64, FP32 outputs (671 MB
per step).
Inputs are resident in HBM before the timed region.

The JSON line also carries the FP64 form of the same step, the oscillator
throughput (256 two-dipole instances, 20,000 RK4 steps), the errors against the
FP64 oracle on a sample, the roofline of the dominant kernel and the oracle's
CPU throughput on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "charge·point LW evals/s (mixed vs FP64) + dipole-steps/s at stated error"

# Algorithmic work per LW eval (one point, one charge, one time), counted from
# the formulas: 86 FP32 flops for Phi, A, E, B of one charge (FMA = 2 flops)
# and 150 FP64 flops for the retarded-time solve (3 Newton iterations of 50, a
# fixed count that does not follow the solver's actual iterations).
FLOP_LW_FP32 = 86
FLOP_SOLVE_FP64 = 150
# Vector ALU peak of MI355X for FP64 and for unpacked FP32: 256 CUs x 4 SIMDs
# x 16 lanes x 2 flops (FMA) x 2.4 GHz.
PEAK_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# HBM bytes per launch of fields_kernel<float, 2> on this workload from the profiler's
# FETCH_SIZE (x2.0) and WRITE_SIZE (x1.0) counters, calibrated on a plain 1 GiB copy
# (profiles/fields_kernel_mixed_grid512x512x64t.md).  Valid only for the kernel
# sources and code-generation flags they were taken on; reported as null once
# either changes.
TRAFFIC_BYTES = 682.1e6
TRAFFIC_SOURCES_SHA = "a857de27d0f7cbc7"
# Algorithmic FP64 work per charge-pair drive of the oscillator step (one source
# charge seen by one target dipole at one stage time), counted from the method's
# definition: the retarded time on the interpolated history (30 flops, one
# iteration), the charge's position, beta and beta_dot from the moment (15), the
# total field of Eq. (E) (58) and its projection on the target's axis with the sum
# over sources (6).  One square root and two divisions are not counted.
FLOP_DRIVE_FP64 = 109


def kernel_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("lw_fields.hip", "lw_device.hpp"):
        with open(os.path.join(ROOT, "paper_2107_12437_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    from paper_2107_12437_amd.build import CODEGEN_FLAGS
    h.update(" ".join(CODEGEN_FLAGS).encode())
    return h.hexdigest()[:16]


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def timed_calls(call, steps: int, warmup: int):
    import torch
    for _ in range(warmup):
        call.launch()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        call.launch()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = [a.elapsed_time(b) for a, b in evs]
    return wall, sum(kern) / len(kern)


def errors(got, ref):
    """relL2 and relmax of each output group (relative to the group's largest magnitude),
    and the 99.9th percentile of the pointwise relative error |got - ref| / |ref| of the
    group's vector at each unmasked (point, time)."""
    import numpy as np
    res = {}
    ok = np.isfinite(ref).all(axis=1)
    for name, comps in (("phi", [0]), ("A", [1, 2, 3]), ("E", [4, 5, 6]), ("B", [7, 8, 9])):
        g = got[:, comps, :].transpose(0, 2, 1)[ok]
        r = ref[:, comps, :].transpose(0, 2, 1)[ok]
        d = g - r
        den = np.linalg.norm(r, axis=1)
        nz = den > 0
        res[name] = {"relL2": float(np.sqrt((d * d).sum() / (r * r).sum())),
                     "relmax": float(np.abs(d).max() / np.abs(r).max()),
                     "p999_pointwise": float(np.percentile(np.linalg.norm(d, axis=1)[nz] / den[nz], 99.9))}
    return res


def host_cpu() -> dict:
    """The host's CPU model, its physical cores and the threads this process may use."""
    import subprocess
    info = {"model": None, "physical_cores": None, "usable_threads": len(os.sched_getaffinity(0))}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        kv = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        info["model"] = kv.get("Model name")
        if kv.get("Core(s) per socket") and kv.get("Socket(s)"):
            info["physical_cores"] = int(kv["Core(s) per socket"]) * int(kv["Socket(s)"])
    except (OSError, subprocess.SubprocessError, ValueError):
        pass
    return info


def run_part(part: str, cluster_steps: int, precision: str, ckpt_every: int, adjoint_steps: int, I, lw, torch):
    """One workload alone: a warm-up call, then one timed call (for profiler runs)."""
    if part == "pairs":
        pw = I.workload_dipole_pairs()

        def call(steps):
            lw.dipole_run(pw["dipoles"], pw["inst_off"], pw["dt"], steps, policy="extrapolate", check=False)
        call(200)
        steps = pw["steps"]
    elif part == "clusters":
        cw = I.workload_clusters(steps=cluster_steps)

        def call(steps):
            lw.dipole_run(cw["dipoles"], cw["inst_off"], cw["dt"], steps, out_stride=10, check=False,
                          precision=precision)
        call(10)
        steps = cw["steps"]
    elif part == "grid-vjp":
        dw = I.workload_detector()
        dpts = torch.tensor(dw["points"], dtype=torch.float64, device="cuda")
        dout, _ = lw.fields(dw["charges"], dpts, dw["times"], precision="fp64", outputs=("E",))
        cot = 2.0 * dout / len(dw["times"])

        def call(steps):
            lw.fields_vjp(dw["charges"], dpts, dw["times"], cot, outputs=("E",))
        call(0)
        steps = 0
    else:
        ow = I.workload_dipole_detector(steps=adjoint_steps) if adjoint_steps > 0 else I.workload_dipole_detector()
        opts = torch.tensor(ow["points"], dtype=torch.float64, device="cuda")

        def call(steps):
            lw.dipole_run_vjp(ow["dipoles"], ow["inst_off"], ow["dt"], ow["steps"], opts, ow["times"],
                              ckpt_every=ckpt_every)
        call(0)
        steps = ow["steps"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    call(steps)
    torch.cuda.synchronize()
    lw.sync_status()
    log(f"[bench] {part}: {(time.perf_counter() - t0) * 1e3:.2f} ms")


def dipole_cpu_baseline(pw: dict, I) -> dict:
    """The FP64 oracle on a slice of the pair workload: every 4th instance for all its
    steps, instances spread over threads (the C oracle runs with the GIL released), and
    two instances on one core."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    import oracle as O
    hcpu = host_cpu()
    workers = max(1, min(16, hcpu["usable_threads"]))
    inst = list(range(0, len(pw["inst_off"]) - 1, 4))
    dip = pw["dipoles"]

    def one(k, steps):
        sel = slice(int(pw["inst_off"][k]), int(pw["inst_off"][k + 1]))
        sub = {key: np.ascontiguousarray(v[sel]) for key, v in dip.items()}
        O.dipole_run(sub, [0, sel.stop - sel.start], pw["dt"], steps, policy=O.DT_EXTRAPOLATE, out_stride=100)
        return sel.stop - sel.start

    t0 = time.perf_counter()
    with ThreadPoolExecutor(workers) as ex:
        n_dips = list(ex.map(lambda k: one(k, pw["steps"]), inst))
    sec = time.perf_counter() - t0
    t0 = time.perf_counter()
    n1 = one(inst[0], pw["steps"]) + one(inst[1], pw["steps"])
    s1 = time.perf_counter() - t0
    return {"value": sum(n_dips) * pw["steps"] / sec, "unit": "dipole-steps/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(inst)} of the {len(pw['inst_off']) - 1} pair instances (every 4th) x {pw['steps']} "
                      f"steps, {sec:.1f} s wall on {workers} threads, FP64 C oracle",
            "serial_value": n1 * pw["steps"] / s1,
            "serial_sample": f"2 instances x {pw['steps']} steps on one core ({s1:.2f} s)",
            "cpu_model": hcpu["model"], "physical_cores": hcpu["physical_cores"]}


def paper_regime(I, lw, np) -> dict:
    """Sec. 4.2 in the paper's own regime: in-phase s and p pairs at 16 separations from
    7.5 nm to 1 um, dt = T0/1e4, 40,000 steps, all 32 pairs in one lw_dipole_run call with
    its gamma / delta_omega outputs; mean and max relative errors of delta_12 (relative to
    max(|delta_12|, gamma_0)) and gamma+ against the Green's-function rates, beside the
    means the paper reports (Fig. 9 caption)."""
    w0 = 2 * math.pi * 200e12
    seps = np.geomspace(7.5e-9, 1e-6, 16)
    ws = [I.workload_dipole_pairs(seps=seps, orientation=o, steps=40000, steps_per_period=10000, d0_both=True)
          for o in ("p", "s")]
    dip = I.concat_dipoles([w["dipoles"] for w in ws])
    off = np.arange(0, 4 * len(seps) + 1, 2, dtype=np.int32)
    t0 = time.perf_counter()
    r = lw.dipole_run(dip, off, ws[0]["dt"], 40000, out_stride=5, modes=True)
    sec = time.perf_counter() - t0
    g0 = lw.gamma0(I.E_CHARGE, I.M_E / 2, w0)
    out = {"workload": "32 in-phase pairs (16 separations 7.5 nm - 1 um, s and p), T0/1e4, 40,000 steps",
           "ms": round(sec * 1e3, 2), "paper_mean_rel": {"p": [0.0015, 0.0004], "s": [0.0019, 0.0013]}}
    for oi, o in enumerate(("p", "s")):
        axis = np.array([1.0, 0.0, 0.0]) if o == "p" else np.array([0.0, 1.0, 0.0])
        ed, eg = [], []
        for k, R in enumerate(seps):
            d12, g12 = lw.gf_pair(np.array([R, 0.0, 0.0]), axis, axis, w0)
            inst = oi * len(seps) + k
            ed.append(abs(r["delta_omega"][inst] / g0 - d12) / max(abs(d12), 1.0))
            eg.append(abs(r["gamma"][inst, 0] / g0 - (1 + g12)) / (1 + g12))
        out[o] = {"delta12_mean_rel": float(np.mean(ed)), "gamma_plus_mean_rel": float(np.mean(eg)),
                  "delta12_max_rel": float(np.max(ed)), "gamma_plus_max_rel": float(np.max(eg))}
    return out


def tuned_threshold(precision: str):
    """The stepped-path threshold the library tuned for the last oscillator shape class of
    this precision, from the tuning file (LW_TUNE_CACHE); None if there is none."""
    path = os.environ.get("LW_TUNE_CACHE", "")
    if not path or not os.path.exists(path):
        return None
    code = {"fp64": 0, "mixed": 1}[precision]
    found = None
    for line in open(path):
        if line.startswith(f"dipoles p{code} ") and "|" in line:
            found = int(line.split("|")[1])
    return found


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample-points", type=int, default=16384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dipole", action="store_true")
    ap.add_argument("--cluster-steps", type=int, default=50000,
                    help="steps of the uneven-cluster workload to time (its full run: 50,000)")
    ap.add_argument("--grid-only", action="store_true",
                    help="time only the mixed grid step (for profiler runs)")
    ap.add_argument("--grid-family", choices=("mix", "circular", "linear", "accel", "uniform"), default="mix",
                    help="with --grid-only: the benchmark's charges (mix), or 16 charges of one trajectory family "
                         "on the same grid and times, in both precisions (per-family cost)")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64",
                    help="precision of the cluster run in --part clusters")
    ap.add_argument("--part", choices=("pairs", "clusters", "grid-vjp", "adjoint"), default=None,
                    help="run only this workload once after one warm-up, print its time and exit "
                         "(for profiler runs; --cluster-steps sets the cluster run's length)")
    ap.add_argument("--adjoint-steps", type=int, default=0,
                    help="length of the oscillator run in --part adjoint (0: the workload's 5,000 steps; "
                         "shorter runs are for counter passes)")
    ap.add_argument("--ckpt-every", type=int, default=250,
                    help="checkpoint interval of the oscillator adjoint in --part adjoint (0: whole history)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="run one plain device-to-device copy of BYTES and exit (calibrates the "
                         "profiler's byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (each instance or "
              "grid tile is independent, so N GPUs would shard the workload without exchange)",
              file=sys.stderr)
        sys.exit(2)

    # a fresh tuning file, unless one is given: the library writes its tuned launch
    # choices there, and the bench reports the oscillator threshold it picked
    if not os.environ.get("LW_TUNE_CACHE"):
        import tempfile
        fd, tune_path = tempfile.mkstemp(prefix="lw_tune_", suffix=".txt")
        os.close(fd)
        os.environ["LW_TUNE_CACHE"] = tune_path

    import numpy as np
    import torch

    from paper_2107_12437_amd import inputs as I
    from paper_2107_12437_amd import lw

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {4 * n} bytes")
        return
    if args.part:
        run_part(args.part, args.cluster_steps, args.precision, args.ckpt_every, args.adjoint_steps, I, lw, torch)
        return
    w = I.workload_grid_mixed()
    pts = torch.tensor(w["points"], dtype=torch.float64, device="cuda")
    n_pts, n_ch, n_t = pts.shape[1], len(w["charges"]["kind"]), len(w["times"])
    evals = n_pts * n_ch * n_t
    if args.grid_only and args.grid_family != "mix":
        fam = {"circular": I.CIRCULAR, "linear": I.LINEAR_OSC, "accel": I.ACCEL}
        ch = (I.workload_uniform_velocity()["charges"] if args.grid_family == "uniform" else
              I.random_grid_charges(I.rng_for(2), n_ch, families=(fam[args.grid_family],)))
        for prec in ("mixed", "fp64"):
            _, kms = timed_calls(lw.FieldsCall(ch, pts, w["times"], precision=prec), args.steps, args.warmup)
            log(f"[bench] {args.grid_family} {prec}: kernel {kms:.3f} ms, "
                f"{kms * 1e-3 * PEAK_VALU_TFLOPS * 1e12 / 2 / evals:.0f} time-equivalent lane-instructions per eval")
        return

    log(f"[bench] mixed grid: {n_pts} points x {n_ch} charges x {n_t} times")
    mixed = lw.FieldsCall(w["charges"], pts, w["times"], precision="mixed")
    wall, kern_ms = timed_calls(mixed, args.steps, args.warmup)
    ms_per_step = wall / args.steps * 1e3
    value = evals / (wall / args.steps)
    log(f"[bench] mixed: {ms_per_step:.3f} ms/step, kernel {kern_ms:.3f} ms, {value:.4e} evals/s")
    if args.grid_only:
        return

    fp64 = lw.FieldsCall(w["charges"], pts, w["times"], precision="fp64")
    fsteps = max(3, args.steps // 4)
    fwall, fkern_ms = timed_calls(fp64, fsteps, 1)
    fp64_value = evals / (fwall / fsteps)
    log(f"[bench] fp64: {fwall / fsteps * 1e3:.3f} ms/step, {fp64_value:.4e} evals/s")

    achieved = evals * (FLOP_LW_FP32 + FLOP_SOLVE_FP64) / (kern_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_VALU_TFLOPS, 1),
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_VALU_TFLOPS, 4),
                "traffic": TRAFFIC_BYTES if kernel_sources_sha() == TRAFFIC_SOURCES_SHA else None,
                "kernel": "fields_kernel<float, TCH> (TCH: the tuned times per lane)",
                "flop_per_eval": FLOP_LW_FP32 + FLOP_SOLVE_FP64,
                "kernel_ms": round(kern_ms, 4)}

    # errors of both forms against the oracle on a sample of the same launch
    out_m = mixed.out
    out_f = fp64.out
    rng = np.random.default_rng(5)
    n_s = args.cpu_sample_points
    pidx = np.sort(rng.choice(n_pts, size=min(n_s, n_pts), replace=False))
    cpu = None
    err = None
    if not args.no_cpu_baseline:
        import oracle as O
        from concurrent.futures import ThreadPoolExecutor
        # the C oracle runs with the GIL released, so threads over disjoint point
        # slices use that many host cores (capped at the 16 of one GPU's share)
        hcpu = host_cpu()
        workers = max(1, min(16, hcpu["usable_threads"]))
        chunks = [np.ascontiguousarray(w["points"][:, c]) for c in np.array_split(pidx, workers)]
        log(f"[bench] oracle on {len(pidx)} points x {n_ch} charges x {n_t} times ({workers} threads)")
        t0 = time.perf_counter()
        with ThreadPoolExecutor(workers) as ex:
            parts = list(ex.map(lambda c: O.fields(w["charges"], c, w["times"])[0], chunks))
        cpu_s = time.perf_counter() - t0
        ref = np.concatenate(parts, axis=2)
        cpu_evals = len(pidx) * n_ch * n_t
        # one core on a slice of the same sample
        n1 = min(1024, len(pidx))
        t0 = time.perf_counter()
        O.fields(w["charges"], np.ascontiguousarray(w["points"][:, pidx[:n1]]), w["times"])
        s1 = time.perf_counter() - t0
        cpu = {"value": cpu_evals / cpu_s, "unit": "LW evals/s", "cores": workers, "kind": "oracle",
               "sample": f"{len(pidx)} seeded grid points x {n_ch} charges x {n_t} times of the same "
                         f"workload ({cpu_evals} evals, {cpu_s:.1f} s wall on {workers} threads, FP64 C "
                         f"oracle, disjoint point slices)",
               "serial_value": n1 * n_ch * n_t / s1,
               "serial_sample": f"{n1} of those points on one core ({s1:.1f} s)",
               "cpu_model": hcpu["model"], "physical_cores": hcpu["physical_cores"]}
        gm = out_m[:, :, torch.tensor(pidx, device="cuda")].double().cpu().numpy()
        gf = out_f[:, :, torch.tensor(pidx, device="cuda")].cpu().numpy()
        err = {"mixed": errors(gm, ref), "fp64": errors(gf, ref)}
        log(f"[bench] oracle {cpu['value']:.3e} evals/s ({workers} threads), {cpu['serial_value']:.3e} on one "
            f"core; mixed E relmax {err['mixed']['E']['relmax']:.2e}")

    # field stage alone: uniform-velocity charges have a closed-form retarded time
    uw = I.workload_uniform_velocity()
    upts = torch.tensor(uw["points"], dtype=torch.float64, device="cuda")
    u_evals = upts.shape[1] * len(uw["charges"]["kind"]) * len(uw["times"])
    uwall, ukern = timed_calls(lw.FieldsCall(uw["charges"], upts, uw["times"], precision="mixed"),
                               max(3, args.steps // 4), 1)
    u_tf = u_evals * FLOP_LW_FP32 / (ukern * 1e-3) / 1e12
    field_stage = {"workload": uw["name"], "kernel_ms": round(ukern, 4), "evals_per_s": u_evals / (ukern * 1e-3),
                   "fp32_tflops_algorithmic": round(u_tf, 3),
                   "frac_unpacked_fp32_peak": round(u_tf / PEAK_VALU_TFLOPS, 4),
                   "frac_packed_fp32_peak": round(u_tf / 157.3, 4),
                   "note": "86 FP32 flops per eval; the closed-form FP64 retarded time is not counted"}
    log(f"[bench] field stage (uniform velocity): {ukern:.3f} ms, {u_tf:.1f} FP32 TFLOP/s algorithmic")
    del upts
    # many-charge source: 1024 charges on four current loops
    mw = I.workload_many_charges()
    mpts = torch.tensor(mw["points"], dtype=torch.float64, device="cuda")
    m_evals = mpts.shape[1] * len(mw["charges"]["kind"]) * len(mw["times"])
    _, mkern = timed_calls(lw.FieldsCall(mw["charges"], mpts, mw["times"], precision="mixed"),
                           max(3, args.steps // 4), 1)
    many = {"workload": mw["name"], "kernel_ms": round(mkern, 4), "evals_per_s": m_evals / (mkern * 1e-3),
            "precision": "mixed"}
    log(f"[bench] many charges: {mkern:.3f} ms, {many['evals_per_s']:.4e} evals/s")
    del mpts

    dip = None
    if not args.no_dipole:
        pw = I.workload_dipole_pairs()
        n_dip = len(pw["dipoles"]["omega0"])
        lw.dipole_run(pw["dipoles"], pw["inst_off"], pw["dt"], 200, policy="extrapolate")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = lw.dipole_run(pw["dipoles"], pw["inst_off"], pw["dt"], pw["steps"], policy="extrapolate",
                          out_stride=1, check=False)
        torch.cuda.synchronize()
        dsec = time.perf_counter() - t0
        lw.sync_status()
        dip = {"workload": pw["name"], "dipole_steps_per_s": n_dip * pw["steps"] / dsec,
               "ms": round(dsec * 1e3, 3), "dtype": "f64"}
        # the algorithmic FP64 rate against the vector peak: the pair ensemble is a
        # latency chain (one wave per instance), so the fraction is small by construction
        psizes = np.diff(np.asarray(pw["inst_off"]))
        pdrives = int((psizes * (psizes - 1) * 4).sum())    # source charges x targets x 2 new stage times
        pach = pdrives * pw["steps"] * FLOP_DRIVE_FP64 / dsec / 1e12
        dip["roofline"] = {"bound": "latency", "achieved": round(pach, 4), "peak": round(PEAK_VALU_TFLOPS, 1),
                           "unit": "TFLOP/s", "frac": round(pach / PEAK_VALU_TFLOPS, 5), "traffic": None,
                           "kernel": "lo_small_kernel<false> (one wave per two-dipole instance)",
                           "flop_per_drive": FLOP_DRIVE_FP64, "drives_per_step": pdrives,
                           "note": "256 waves on 1,024 SIMDs, each step a dependent chain of about 2,300 cycles "
                                   "(drive, stage sums, RK4 update); wall clock of the whole call"}
        log(f"[bench] dipoles: {dsec * 1e3:.2f} ms, {dip['dipole_steps_per_s']:.3e} dipole-steps/s, "
            f"{pach:.3f} TFLOP/s algorithmic (latency-bound)")
        # the timed run's collective rates (host extraction) against the Green's-function
        # rates of App. A, for the pairs at least 7.5 nm apart (c dt at T0/200)
        w0 = float(pw["dipoles"]["omega0"][0])
        seps = np.asarray(pw["separations"])
        skips = [max(2000, int(math.ceil(3.0 * R / (I.C_LIGHT * pw["dt"])))) for R in seps]
        modes = lw.pair_modes(r["d"], pw["inst_off"], pw["dt"], 1, w0, skips)
        g0 = lw.gamma0(I.E_CHARGE, I.M_E / 2, w0)
        eg, ed = [], []
        for k, R in enumerate(seps):
            if R < 7.5e-9:
                continue
            d12, g12 = lw.gf_pair(np.array([R, 0.0, 0.0]), np.array([1.0, 0.0, 0.0]), np.array([1.0, 0.0, 0.0]), w0)
            eg.append(abs(modes[k, 0] / g0 - (1 + g12)) / (1 + abs(g12)))
            ed.append(abs(modes[k, 4] / g0 - d12) / max(abs(d12), 1.0))
        dip["vs_green_function"] = {
            "pairs": len(eg), "gamma_plus_relmax": float(max(eg)), "gamma_plus_relmedian": float(np.median(eg)),
            "delta_omega_max": float(max(ed)), "delta_omega_median": float(np.median(ed)),
            "note": "gamma+ relative to gamma0 (1 + gamma12); delta_omega in units of gamma0 relative to "
                    "max(|delta12|, 1); pairs at least 7.5 nm apart. At dt = T0/200 RK4's own damping, "
                    "(omega0 dt)^6 / (72 dt) = 0.027 gamma0 on the energy, sets the gamma error; at T0/2000 "
                    "the rates are within 0.2 % of the theory (GPU tests)"}
        log(f"[bench] dipoles vs Green's function ({len(eg)} pairs): gamma+ rel max {max(eg):.2e} "
            f"(median {np.median(eg):.2e}), delta_omega max {max(ed):.2e} (median {np.median(ed):.2e})")
        dip["paper_regime"] = paper_regime(I, lw, np)
        log(f"[bench] paper regime (T0/1e4, 16 separations): p delta12 "
            f"{100 * dip['paper_regime']['p']['delta12_mean_rel']:.3f} % gamma+ "
            f"{100 * dip['paper_regime']['p']['gamma_plus_mean_rel']:.3f} %, s delta12 "
            f"{100 * dip['paper_regime']['s']['delta12_mean_rel']:.3f} % gamma+ "
            f"{100 * dip['paper_regime']['s']['gamma_plus_mean_rel']:.3f} %")
        if not args.no_cpu_baseline:
            dip["cpu_baseline"] = dipole_cpu_baseline(pw, I)
            log(f"[bench] oracle pairs: {dip['cpu_baseline']['value']:.3e} dipole-steps/s on "
                f"{dip['cpu_baseline']['cores']} threads")

    clusters = None
    vjp = None
    dip_vjp = None
    if not args.no_dipole:
        cw = I.workload_clusters(steps=args.cluster_steps)
        n_c = len(cw["dipoles"]["omega0"])
        sizes = np.diff(cw["inst_off"]).astype(np.int64)
        drives = int((sizes * (sizes - 1) * 4).sum())       # source charges x targets x 2 new stage times
        clusters = {"workload": cw["name"], "dipoles": n_c, "steps": cw["steps"],
                    "note": ("the whole 50,000-step run, " if cw["steps"] >= 50000 else
                             "the uneven-cluster workload runs 50,000 steps; this line times a prefix of it, ") +
                            "moments every 10th step. mixed: FP32 velocity and radiation terms of each source "
                            "dipole, FP64 static near-field term, retarded times, state and sums"}
        for prec in ("fp64", "mixed"):
            # the warm-up call tunes the stepped-path threshold for this shape class
            lw.dipole_run(cw["dipoles"], cw["inst_off"], cw["dt"], 10, out_stride=10, precision=prec,
                          stepped_min_n="tune")
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            ev0.record()
            lw.dipole_run(cw["dipoles"], cw["inst_off"], cw["dt"], cw["steps"], out_stride=10, check=False,
                          precision=prec, stepped_min_n="tune")
            ev1.record()
            torch.cuda.synchronize()
            csec = time.perf_counter() - t0
            lw.sync_status()
            step_ms = ev0.elapsed_time(ev1) / cw["steps"]
            ach = drives * FLOP_DRIVE_FP64 / (step_ms * 1e-3) / 1e12
            clusters[prec] = {"dipole_steps_per_s": n_c * cw["steps"] / csec, "ms": round(csec * 1e3, 3),
                              "stepped_min_n": tuned_threshold(prec), "step_us": round(step_ms * 1e3, 2),
                              "roofline": {"bound": "alu", "achieved": round(ach, 3),
                                           "peak": round(PEAK_VALU_TFLOPS, 1), "unit": "TFLOP/s",
                                           "frac": round(ach / PEAK_VALU_TFLOPS, 4), "traffic": None,
                                           "kernel": "lo_step_kernel (one launch per step, graph-replayed)",
                                           "flop_per_drive": FLOP_DRIVE_FP64, "drives_per_step": drives,
                                           "note": "per-step time from events on the launch stream over the "
                                                   "whole run; algorithmic FP64 flops per charge-pair drive"}}
            log(f"[bench] clusters ({prec}, stepped path from {clusters[prec]['stepped_min_n']} dipoles): "
                f"{csec * 1e3:.1f} ms for {cw['steps']} steps, "
                f"{clusters[prec]['dipole_steps_per_s']:.3e} dipole-steps/s")
        clusters["mixed_over_fp64"] = round(clusters["fp64"]["ms"] / clusters["mixed"]["ms"], 3)
        # J = mean over snapshots of sum |E|^2 needs E alone: the forward and the VJP
        # take the three E rows
        dw = I.workload_detector()
        dpts = torch.tensor(dw["points"], dtype=torch.float64, device="cuda")
        dout, _ = lw.fields(dw["charges"], dpts, dw["times"], precision="fp64", outputs=("E",))
        cot = 2.0 * dout / len(dw["times"])
        lw.fields_vjp(dw["charges"], dpts, dw["times"], cot, outputs=("E",))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            lw.fields_vjp(dw["charges"], dpts, dw["times"], cot, outputs=("E",))
        torch.cuda.synchronize()
        vsec = (time.perf_counter() - t0) / 3
        pairs = dpts.shape[1] * len(dw["charges"]["kind"]) * len(dw["times"])
        vjp = {"workload": dw["name"], "ms": round(vsec * 1e3, 3), "pair_vjps_per_s": pairs / vsec, "dtype": "f64",
               "outputs": "E"}
        log(f"[bench] grid VJP: {vsec * 1e3:.2f} ms, {vjp['pair_vjps_per_s']:.3e} pair VJPs/s")
        # oscillator adjoint: forward run, detector VJP, backward sweep; checkpointed every
        # 250 steps (segments recomputed) and with the whole history kept
        ow = I.workload_dipole_detector()
        opts_pts = torch.tensor(ow["points"], dtype=torch.float64, device="cuda")
        n_o = len(ow["dipoles"]["omega0"])
        osec = {}
        for K in (ow["ckpt_every"], 0):
            lw.dipole_run_vjp(ow["dipoles"], ow["inst_off"], ow["dt"], ow["steps"], opts_pts, ow["times"],
                              ckpt_every=K)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lw.dipole_run_vjp(ow["dipoles"], ow["inst_off"], ow["dt"], ow["steps"], opts_pts, ow["times"],
                              ckpt_every=K)
            torch.cuda.synchronize()
            osec[K] = time.perf_counter() - t0
        ck = osec[ow["ckpt_every"]]
        dip_vjp = {"workload": ow["name"], "ckpt_every": ow["ckpt_every"], "ms": round(ck * 1e3, 3),
                   "dipole_steps_per_s": n_o * ow["steps"] / ck, "ms_whole_history": round(osec[0] * 1e3, 3),
                   "gradients": 3 * n_o, "dtype": "f64",
                   "note": "forward run, detector objective and its VJP, backward sweep; one call"}
        log(f"[bench] oscillator adjoint: {ck * 1e3:.2f} ms checkpointed every {ow['ckpt_every']} steps, "
            f"{osec[0] * 1e3:.2f} ms with the whole history, for {n_o} dipoles x {ow['steps']} steps")

    line = {
        "metric": METRIC, "value": value, "unit": "LW evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": w["name"], "precision": "mixed", "points": n_pts, "charges": n_ch,
                   "times": n_t, "evals_per_step": evals},
        "fp64_value": fp64_value, "mixed_over_fp64": value / fp64_value,
        "roofline": roofline, "cpu_baseline": cpu, "errors_vs_oracle": err, "dipoles": dip,
        "clusters": clusters, "grid_vjp": vjp, "oscillator_adjoint": dip_vjp, "field_stage": field_stage,
        "many_charges": many,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
