"""Python binding of liblw.so (argument marshalling only).

Every computation happens in the HIP library; this module converts the seeded
input records (``inputs.py`` dicts) to the C structs of ``include/lw.h``,
allocates outputs as torch tensors on the GPU and passes raw pointers and the
current HIP stream through the C ABI.  There is no fallback: if the library
is missing or no GPU is present the calls raise.

torch is imported before the library is loaded so that both share the HIP
runtime that torch ships (same SONAME).
"""
from __future__ import annotations

import ctypes as ct
import math
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblw.so")

FP64, MIXED = 0, 1
FIELD_KINDS = {"total": 0, "coulomb": 1, "radiation": 2}
PRECISIONS = {"fp64": FP64, "mixed": MIXED}
# output components (LW_OUT_*): bit and rows, in the order of the output rows
OUTPUTS = {"phi": (1, 1), "A": (2, 3), "E": (4, 3), "B": (8, 3), "S": (16, 3)}
DEFAULT_OUTPUTS = ("phi", "A", "E", "B")


def output_mask(outputs) -> tuple[int, int]:
    """(LW_OUT_* mask, rows) of a sequence of component names (None: phi, A, E, B)."""
    names = DEFAULT_OUTPUTS if outputs is None else tuple(outputs)
    bad = [n for n in names if n not in OUTPUTS]
    if bad or not names:
        raise ValueError(f"outputs must name some of {tuple(OUTPUTS)}: {names}")
    mask = 0
    for n in names:
        mask |= OUTPUTS[n][0]
    return mask, sum(r for b, r in OUTPUTS.values() if mask & b)
DT_POLICIES = {"strict": 0, "extrapolate": 1}
FLAG_MASKED, FLAG_NOCONV = 1, 2
STATUS_NAMES = {0: "LW_OK", 1: "LW_E_INVALID", 2: "LW_E_SUPERLUMINAL", 3: "LW_E_DT_TOO_LARGE",
                4: "LW_E_VELOCITY", 5: "LW_E_NOCONV", 6: "LW_E_HIP", 7: "LW_E_NOMEM",
                8: "LW_E_NONFINITE", 9: "LW_E_HISTORY", 10: "LW_E_STATE"}
EXPORTS = ("lw_last_error", "lw_create", "lw_destroy", "lw_sync_status", "lw_set_autotune", "lw_fields",
           "lw_fields_noalloc", "lw_fields_vjp", "lw_dipole_run", "lw_dipole_run_vjp", "lw_pair_modes", "lw_gamma0", "lw_gf_pair",
           "lw_exact_modes", "lw_dipole_state_size", "lw_dipole_run_state", "lw_set_iteration_histogram",
           "lw_iteration_histogram")
ITER_BINS, ITER_BIN_FALLBACK, ITER_BIN_NOCONV = 34, 32, 33
PARAM_NAMES = ("q", "c0x", "c0y", "c0z", "amp", "omega", "phase", "accel", "vx", "vy", "vz")
OUTPUT_NAMES = ("phi", "Ax", "Ay", "Az", "Ex", "Ey", "Ez", "Bx", "By", "Bz")


class LWError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Traj(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("pad_", ct.c_int32), ("q", ct.c_double),
                ("c0", ct.c_double * 3), ("e1", ct.c_double * 3), ("e2", ct.c_double * 3),
                ("amp", ct.c_double), ("omega", ct.c_double), ("phase", ct.c_double),
                ("accel", ct.c_double), ("v", ct.c_double * 3)]


class Opts(ct.Structure):
    _fields_ = [("precision", ct.c_int32), ("field_kind", ct.c_int32), ("max_iter", ct.c_int32),
                ("outputs", ct.c_int32), ("mask_radius", ct.c_double)]


class Dipole(ct.Structure):
    _fields_ = [("origin", ct.c_double * 3), ("axis", ct.c_double * 3), ("omega0", ct.c_double),
                ("q", ct.c_double), ("m1", ct.c_double), ("m2", ct.c_double), ("d0", ct.c_double),
                ("motion_amp", ct.c_double * 3), ("motion_omega", ct.c_double), ("motion_phase", ct.c_double)]


class RunOpts(ct.Structure):
    _fields_ = [("precision", ct.c_int32), ("dt_policy", ct.c_int32), ("out_stride", ct.c_int64),
                ("max_vel", ct.c_double), ("ring_depth", ct.c_int32), ("stepped_min_n", ct.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads liblw.so and declares the C signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_2107_12437_amd.build`")
    L = ct.CDLL(path)
    vp, i32, i64, dbl = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_double
    L.lw_last_error.restype = ct.c_char_p
    L.lw_last_error.argtypes = []
    L.lw_create.argtypes = [ct.POINTER(vp), i32]
    L.lw_destroy.argtypes = [vp]
    L.lw_sync_status.argtypes = [vp, vp]
    L.lw_set_autotune.argtypes = [vp, i32]
    L.lw_fields.argtypes = [vp, ct.POINTER(Traj), i32, vp, i64, ct.POINTER(dbl), i32, ct.POINTER(Opts), vp, vp, vp]
    L.lw_fields_noalloc.argtypes = [vp, ct.POINTER(Traj), i32, vp, i64, ct.POINTER(dbl), i32, ct.POINTER(Opts), vp,
                                    vp, vp]
    L.lw_fields_vjp.argtypes = [vp, ct.POINTER(Traj), i32, vp, i64, ct.POINTER(dbl), i32, ct.POINTER(Opts), vp, vp, vp]
    L.lw_dipole_run.argtypes = [vp, ct.POINTER(Dipole), i32, ct.POINTER(i32), i32, dbl, i64,
                                ct.POINTER(RunOpts), vp, vp, vp, vp, vp, vp, ct.POINTER(dbl), ct.POINTER(dbl), vp]
    L.lw_dipole_run_state.argtypes = [vp, ct.POINTER(Dipole), i32, ct.POINTER(i32), i32, dbl, i64,
                                      ct.POINTER(RunOpts), vp, vp, vp, vp, vp, vp, vp, i64, i32, vp]
    L.lw_dipole_state_size.argtypes = [ct.POINTER(Dipole), i32, ct.POINTER(i32), i32, dbl, ct.POINTER(RunOpts),
                                       ct.POINTER(i64)]
    L.lw_dipole_run_vjp.argtypes = [vp, ct.POINTER(Dipole), i32, ct.POINTER(i32), i32, dbl, i64,
                                    ct.POINTER(RunOpts), vp, i64, ct.POINTER(dbl), i32, i32, vp, ct.POINTER(dbl), vp]
    L.lw_pair_modes.argtypes = [ct.POINTER(dbl), i64, i32, ct.POINTER(i32), i32, dbl, i64,
                                ct.POINTER(dbl), ct.POINTER(i64), ct.POINTER(dbl)]
    L.lw_set_iteration_histogram.argtypes = [vp, i32]
    L.lw_iteration_histogram.argtypes = [vp, ct.POINTER(ct.c_uint64), i32, i32, vp]
    L.lw_gamma0.restype = dbl
    L.lw_gamma0.argtypes = [dbl, dbl, dbl]
    L.lw_gf_pair.argtypes = [ct.POINTER(dbl), ct.POINTER(dbl), ct.POINTER(dbl), dbl, ct.POINTER(dbl)]
    L.lw_exact_modes.argtypes = [ct.POINTER(dbl), ct.POINTER(dbl), dbl, dbl, dbl, ct.POINTER(dbl)]
    for name in ("lw_create", "lw_destroy", "lw_sync_status", "lw_set_autotune", "lw_fields", "lw_fields_noalloc",
                 "lw_fields_vjp",
                 "lw_dipole_run", "lw_dipole_run_vjp", "lw_pair_modes", "lw_gf_pair", "lw_exact_modes",
                 "lw_dipole_state_size", "lw_dipole_run_state", "lw_set_iteration_histogram",
                 "lw_iteration_histogram"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def _check(code: int):
    if code != 0:
        raise LWError(code, load_library().lw_last_error().decode())


class Context:
    """Owns one lw_ctx (workspace, staging, error word) on a device."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the Lienard-Wiechert library needs an MI355X")
        L = load_library()
        self.device = int(device)
        h = ct.c_void_p()
        _check(L.lw_create(ct.byref(h), self.device))
        self.handle = h

    def set_autotune(self, enable: bool):
        _check(load_library().lw_set_autotune(self.handle, int(bool(enable))))

    def close(self):
        if self.handle:
            load_library().lw_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx: dict[int, Context] = {}


def default_context(device: int | None = None) -> Context:
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _default_ctx:
        _default_ctx[dev] = Context(dev)
    return _default_ctx[dev]


def _as_device(device) -> torch.device:
    if isinstance(device, torch.device):
        return device
    return torch.device("cuda", torch.cuda.current_device() if device is None else int(device))


def _stream_ptr(device) -> ct.c_void_p:
    return ct.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def pack_charges(charges: dict):
    n = len(charges["kind"])
    arr = (Traj * max(n, 1))()
    for i in range(n):
        t = arr[i]
        t.kind = int(charges["kind"][i])
        t.q = float(charges["q"][i])
        t.c0[:] = [float(v) for v in charges["c0"][i]]
        t.e1[:] = [float(v) for v in charges["e1"][i]]
        t.e2[:] = [float(v) for v in charges["e2"][i]]
        t.v[:] = [float(v) for v in charges["v"][i]]
        t.amp = float(charges["amp"][i])
        t.omega = float(charges["omega"][i])
        t.phase = float(charges["phase"][i])
        t.accel = float(charges["accel"][i])
    return arr, n


def pack_dipoles(dipoles: dict):
    """lw_dipole records (16 doubles each, in the field order of the C struct) for the
    dipoles, as a ctypes array over one numpy buffer."""
    n = len(dipoles["omega0"])
    a = np.zeros((max(n, 1), 16), dtype=np.float64)
    a[:n, 0:3] = np.asarray(dipoles["origin"], dtype=np.float64).reshape(n, 3)
    a[:n, 3:6] = np.asarray(dipoles["axis"], dtype=np.float64).reshape(n, 3)
    for col, key in ((6, "omega0"), (7, "q"), (8, "m1"), (9, "m2"), (10, "d0")):
        a[:n, col] = np.asarray(dipoles[key], dtype=np.float64).reshape(n)
    if "motion_amp" in dipoles:
        a[:n, 11:14] = np.asarray(dipoles["motion_amp"], dtype=np.float64).reshape(n, 3)
        a[:n, 14] = np.asarray(dipoles["motion_omega"], dtype=np.float64).reshape(n)
        a[:n, 15] = np.asarray(dipoles["motion_phase"], dtype=np.float64).reshape(n)
    return (Dipole * max(n, 1)).from_buffer(a), n


class FieldsCall:
    """A prepared lw_fields call: packed charges, times and options plus output
    buffers, so repeated launches (benchmarks) pay no Python packing cost."""

    def __init__(self, charges: dict, points: torch.Tensor, times, precision: str = "mixed",
                 field_kind: str = "total", mask_radius: float = 1e-10, max_iter: int = 0,
                 with_flags: bool = True, ctx: Context | None = None, outputs=None):
        if not (isinstance(points, torch.Tensor) and points.is_cuda and points.dtype == torch.float64
                and points.dim() == 2 and points.shape[0] == 3):
            raise ValueError("points must be a [3, n] float64 tensor on the GPU")
        self.points = points.contiguous()
        self.ctx = ctx or default_context(points.device.index)
        self.charges, self.n_charges = pack_charges(charges)
        self.times = np.ascontiguousarray(np.atleast_1d(times), dtype=np.float64)
        mask, rows = output_mask(outputs)
        self.opts = Opts(PRECISIONS[precision], FIELD_KINDS[field_kind], int(max_iter), mask, float(mask_radius))
        n_pts = self.points.shape[1]
        dtype = torch.float32 if precision == "mixed" else torch.float64
        self.out = torch.empty((len(self.times), rows, n_pts), dtype=dtype, device=points.device)
        self.flags = torch.empty(n_pts, dtype=torch.int32, device=points.device) if with_flags else None
        self.n_pts = n_pts

    def launch(self, noalloc: bool = False):
        """Enqueues the call; noalloc takes lw_fields_noalloc (no allocation, fixed scratch)."""
        L = load_library()
        fn = L.lw_fields_noalloc if noalloc else L.lw_fields
        _check(fn(self.ctx.handle, self.charges, self.n_charges, ct.c_void_p(self.points.data_ptr()),
                           self.n_pts, self.times.ctypes.data_as(ct.POINTER(ct.c_double)), len(self.times),
                           ct.byref(self.opts), ct.c_void_p(self.out.data_ptr()),
                           ct.c_void_p(self.flags.data_ptr()) if self.flags is not None else None,
                           _stream_ptr(self.points.device)))
        return self.out, self.flags


def fields(charges: dict, points: torch.Tensor, times, precision: str = "mixed", field_kind: str = "total",
           mask_radius: float = 1e-10, max_iter: int = 0, ctx: Context | None = None, outputs=None):
    """Phi, A, E, B (or the components named in `outputs`, from phi, A, E, B and the
    Poynting vector S) of the charges at points ([3, n] float64 on the GPU) and times.
    Returns (out [n_times][rows][n_pts], flags [n_pts] int32); rows follow the order
    phi, A, E, B, S."""
    return FieldsCall(charges, points, times, precision, field_kind, mask_radius, max_iter, True, ctx,
                      outputs).launch()


def fields_noalloc(charges: dict, points: torch.Tensor, times, precision: str = "mixed", field_kind: str = "total",
                   mask_radius: float = 1e-10, max_iter: int = 0, ctx: Context | None = None, outputs=None):
    """fields() through lw_fields_noalloc: the library allocates nothing during the call (its
    inputs go to a fixed per-GPU scratch of LW_NOALLOC_SCRATCH_BYTES).  The output tensors are
    allocated here, by torch, before the call."""
    return FieldsCall(charges, points, times, precision, field_kind, mask_radius, max_iter, True, ctx,
                      outputs).launch(noalloc=True)


def fields_vjp(charges: dict, points: torch.Tensor, times, cotangent: torch.Tensor, field_kind: str = "total",
               mask_radius: float = 1e-10, max_iter: int = 0, ctx: Context | None = None,
               outputs=None) -> torch.Tensor:
    """Gradient [n_charges][11] (PARAM_NAMES order) of sum(cotangent * fields(...)) with respect
    to each charge's trajectory parameters.  cotangent has the layout of fields' output for the
    same `outputs` (phi, A, E, B; not S); its dtype (float32 / float64) selects the matching
    precision."""
    if not (isinstance(points, torch.Tensor) and points.is_cuda and points.dtype == torch.float64):
        raise ValueError("points must be a [3, n] float64 tensor on the GPU")
    pts = points.contiguous()
    ctx = ctx or default_context(pts.device.index)
    arr, n = pack_charges(charges)
    tms = np.ascontiguousarray(np.atleast_1d(times), dtype=np.float64)
    cot = cotangent.contiguous()
    mask, rows = output_mask(outputs)
    if cot.shape != (len(tms), rows, pts.shape[1]) or cot.device != pts.device:
        raise ValueError(f"cotangent must be [n_times][{rows}][n_pts] on the points' device")
    prec = {torch.float32: MIXED, torch.float64: FP64}[cot.dtype]
    opts = Opts(prec, FIELD_KINDS[field_kind], int(max_iter), mask, float(mask_radius))
    grad = torch.empty((n, len(PARAM_NAMES)), dtype=torch.float64, device=pts.device)
    L = load_library()
    _check(L.lw_fields_vjp(ctx.handle, arr, n, ct.c_void_p(pts.data_ptr()), pts.shape[1],
                           tms.ctypes.data_as(ct.POINTER(ct.c_double)), len(tms), ct.byref(opts),
                           ct.c_void_p(cot.data_ptr()), ct.c_void_p(grad.data_ptr()), _stream_ptr(pts.device)))
    return grad


def charges_to_params(charges: dict) -> torch.Tensor:
    """[n, 11] float64 tensor of the differentiable trajectory parameters."""
    c = charges
    cols = [c["q"][:, None], c["c0"], c["amp"][:, None], c["omega"][:, None], c["phase"][:, None],
            c["accel"][:, None], c["v"]]
    return torch.tensor(np.concatenate(cols, axis=1), dtype=torch.float64)


def params_to_charges(params: torch.Tensor, template: dict) -> dict:
    """Charge dict with the parameters of `params` and the kinds and axes of `template`."""
    p = params.detach().cpu().numpy()
    c = {k: np.array(v, copy=True) for k, v in template.items()}
    c["q"], c["c0"], c["amp"], c["omega"] = p[:, 0], p[:, 1:4], p[:, 4], p[:, 5]
    c["phase"], c["accel"], c["v"] = p[:, 6], p[:, 7], p[:, 8:11]
    return c


class LWFieldsFn(torch.autograd.Function):
    """Phi, A, E, B on the GPU as a differentiable function of the [n, 11] trajectory
    parameters (CPU float64 tensor): the backward pass calls lw_fields_vjp."""

    @staticmethod
    def forward(fctx, params, points, template, times, precision, field_kind, mask_radius):
        charges = params_to_charges(params, template)
        out, _ = fields(charges, points, times, precision=precision, field_kind=field_kind,
                        mask_radius=mask_radius)
        fctx.save_for_backward(params)
        fctx.meta = (points, template, times, field_kind, mask_radius)
        return out

    @staticmethod
    def backward(fctx, grad_out):
        (params,) = fctx.saved_tensors
        points, template, times, field_kind, mask_radius = fctx.meta
        charges = params_to_charges(params, template)
        g = fields_vjp(charges, points, times, grad_out, field_kind=field_kind, mask_radius=mask_radius)
        return g.cpu(), None, None, None, None, None, None


STEPPED_TUNE = -2     # stepped_min_n: threshold timed per shape class (also "tune")


def _run_opts(policy, out_stride, max_vel, ring_depth, stepped_min_n, precision) -> RunOpts:
    smn = STEPPED_TUNE if stepped_min_n == "tune" else int(stepped_min_n)
    return RunOpts(PRECISIONS[precision], DT_POLICIES[policy], int(out_stride), float(max_vel), int(ring_depth), smn)


def dipole_state(dipoles: dict, inst_off, dt: float, policy: str = "strict", ring_depth: int = 0,
                 device=None) -> torch.Tensor:
    """A zeroed run-state buffer (float64 on the GPU) for dipole_run(..., state=...)."""
    arr, n = pack_dipoles(dipoles)
    off = np.ascontiguousarray(inst_off, dtype=np.int32)
    opts = _run_opts(policy, 1, 0.0, ring_depth, 0, "fp64")
    size = ct.c_int64(0)
    _check(load_library().lw_dipole_state_size(arr, n, off.ctypes.data_as(ct.POINTER(ct.c_int32)), len(off) - 1,
                                               float(dt), ct.byref(opts), ct.byref(size)))
    return torch.zeros(size.value, dtype=torch.float64, device=_as_device(device))


def dipole_run(dipoles: dict, inst_off, dt: float, steps: int, policy: str = "strict", out_stride: int = 1,
               max_vel: float = 0.0, ring_depth: int = 0, stepped_min_n: int | str = 0, device=None,
               check: bool = True, ctx: Context | None = None, energy_balance: bool = False,
               precision: str = "fp64", state: torch.Tensor | None = None, resume: bool = False,
               modes: bool = False):
    """Self-consistent oscillator run (Algorithm 1).  Returns a dict of [n_out][n_dip]
    float64 GPU tensors: d, d_dot, energy, Ed, and with energy_balance the work absorbed
    from the drive field W_abs and the Larmor energy radiated W_rad since t = 0 (Sec. 2.5:
    the sum over an instance of energy - W_abs + W_rad is conserved).  precision "mixed"
    evaluates each source dipole's pair field in FP32 (retarded times, state and sums stay
    FP64).  With a run state (dipole_state) the run's state after its last step is kept
    there, and resume=True continues the run that state holds: row 0 is then the state's
    step and `steps` more are taken.  stepped_min_n="tune" lets the library time the
    instance-size threshold of the stepped path for this shape class (cached).  modes=True
    also returns, from the library, numpy arrays gamma [n_inst][2] (gamma+, gamma-) and
    delta_omega [n_inst] of the two-dipole instances (the call then synchronises)."""
    dev = _as_device(device)
    ctx = ctx or default_context(dev.index)
    arr, n = pack_dipoles(dipoles)
    off = np.ascontiguousarray(inst_off, dtype=np.int32)
    n_out = int(steps) // int(out_stride) + 1
    keys = ("d", "d_dot", "energy", "Ed") + (("W_abs", "W_rad") if energy_balance else ())
    res = {k: torch.empty((n_out, n), dtype=torch.float64, device=dev) for k in keys}
    opts = _run_opts(policy, out_stride, max_vel, ring_depth, stepped_min_n, precision)
    L = load_library()
    args = (ctx.handle, arr, n, off.ctypes.data_as(ct.POINTER(ct.c_int32)), len(off) - 1, float(dt), int(steps),
            ct.byref(opts), ct.c_void_p(res["d"].data_ptr()), ct.c_void_p(res["d_dot"].data_ptr()),
            ct.c_void_p(res["energy"].data_ptr()), ct.c_void_p(res["Ed"].data_ptr()),
            ct.c_void_p(res["W_abs"].data_ptr()) if energy_balance else None,
            ct.c_void_p(res["W_rad"].data_ptr()) if energy_balance else None)
    if state is None:
        if resume:
            raise ValueError("resume needs a run state")
        n_inst = len(off) - 1
        gam = np.full((n_inst, 2), np.nan) if modes else None
        dom = np.full(n_inst, np.nan) if modes else None
        dp = ct.POINTER(ct.c_double)
        _check(L.lw_dipole_run(*args, gam.ctypes.data_as(dp) if modes else None,
                               dom.ctypes.data_as(dp) if modes else None, _stream_ptr(dev)))
        if modes:
            res["gamma"], res["delta_omega"] = gam, dom
    else:
        if modes:
            raise ValueError("modes are fitted by dipole_run without a run state")
        if not (state.is_cuda and state.dtype == torch.float64 and state.is_contiguous()):
            raise ValueError("state must be a contiguous float64 GPU tensor (dipole_state)")
        _check(L.lw_dipole_run_state(*args, ct.c_void_p(state.data_ptr()), state.numel(), int(bool(resume)),
                                     _stream_ptr(dev)))
    if check:
        sync_status(ctx, dev)
    return res


def dipole_run_vjp(dipoles: dict, inst_off, dt: float, steps: int, det_points: torch.Tensor, snap_times,
                   policy: str = "strict", max_vel: float = 0.0, ring_depth: int = 0, stepped_min_n: int = 0,
                   ckpt_every: int = 0, ctx: Context | None = None):
    """(J, dJ/d origin [n_dip, 3] GPU tensor) of J = (1/n_snap) sum |E|^2 of all oscillator
    charges over the detector points ([3, n] float64 on the GPU) at snap_times.
    ckpt_every = K > 0 recomputes the backward sweep's history in segments of K steps from
    run states kept every K steps; 0 keeps the whole forward history."""
    if not (isinstance(det_points, torch.Tensor) and det_points.is_cuda and det_points.dtype == torch.float64):
        raise ValueError("det_points must be a [3, n] float64 tensor on the GPU")
    pts = det_points.contiguous()
    dev = pts.device
    ctx = ctx or default_context(dev.index)
    arr, n = pack_dipoles(dipoles)
    off = np.ascontiguousarray(inst_off, dtype=np.int32)
    tms = np.ascontiguousarray(np.atleast_1d(snap_times), dtype=np.float64)
    grad = torch.empty((n, 3), dtype=torch.float64, device=dev)
    J = ct.c_double()
    opts = RunOpts(FP64, DT_POLICIES[policy], 1, float(max_vel), int(ring_depth), int(stepped_min_n))
    _check(load_library().lw_dipole_run_vjp(ctx.handle, arr, n, off.ctypes.data_as(ct.POINTER(ct.c_int32)),
                                            len(off) - 1, float(dt), int(steps), ct.byref(opts),
                                            ct.c_void_p(pts.data_ptr()), pts.shape[1],
                                            tms.ctypes.data_as(ct.POINTER(ct.c_double)), len(tms), int(ckpt_every),
                                            ct.c_void_p(grad.data_ptr()), ct.byref(J), _stream_ptr(dev)))
    return J.value, grad


class DipoleDetectorFn(torch.autograd.Function):
    """J = (1/n_snap) sum |E|^2 of the oscillators' charges on a detector as a differentiable
    function of the origins ([n_dip, 3] CPU float64 tensor); backward uses the stored gradient
    of lw_dipole_run_vjp."""

    @staticmethod
    def forward(fctx, origins, template, inst_off, dt, steps, det_points, snap_times, policy, ckpt_every=0):
        dip = {k: np.array(v, copy=True) for k, v in template.items()}
        dip["origin"] = origins.detach().cpu().numpy()
        J, grad = dipole_run_vjp(dip, inst_off, dt, steps, det_points, snap_times, policy=policy,
                                 ckpt_every=ckpt_every)
        fctx.save_for_backward(grad.cpu())
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(fctx, gJ):
        (grad,) = fctx.saved_tensors
        return gJ * grad, None, None, None, None, None, None, None, None


def sync_status(ctx: Context | None = None, device=None):
    dev = _as_device(device)
    ctx = ctx or default_context(dev.index)
    _check(load_library().lw_sync_status(ctx.handle, _stream_ptr(dev)))


def set_iteration_histogram(enable: bool, ctx: Context | None = None, device=None):
    """Debugging: count the retarded-time solves of later fields() calls on the context by
    their iterations (include/lw.h, lw_set_iteration_histogram)."""
    dev = _as_device(device)
    ctx = ctx or default_context(dev.index)
    _check(load_library().lw_set_iteration_histogram(ctx.handle, int(bool(enable))))


def iteration_histogram(reset: bool = False, ctx: Context | None = None, device=None) -> np.ndarray:
    """The context's iteration histogram, uint64 [ITER_BINS] (bins 0..31: iterations;
    ITER_BIN_FALLBACK, ITER_BIN_NOCONV), optionally cleared after reading."""
    dev = _as_device(device)
    ctx = ctx or default_context(dev.index)
    out = np.zeros(ITER_BINS, dtype=np.uint64)
    _check(load_library().lw_iteration_histogram(ctx.handle, out.ctypes.data_as(ct.POINTER(ct.c_uint64)), ITER_BINS,
                                                  int(bool(reset)), _stream_ptr(dev)))
    return out


def pair_modes(moment, inst_off, dt: float, out_stride: int, omega_ref, skip_steps):
    """gamma+, gamma-, omega+, omega-, delta_omega per two-dipole instance ([n_inst, 5])
    from moments [n_rows][n_dip] (host copy of dipole_run's d)."""
    m = np.ascontiguousarray(moment.cpu().numpy() if isinstance(moment, torch.Tensor) else moment,
                             dtype=np.float64)
    off = np.ascontiguousarray(inst_off, dtype=np.int32)
    n_inst = len(off) - 1
    w = np.ascontiguousarray(np.broadcast_to(np.asarray(omega_ref, dtype=np.float64), (n_inst,)))
    sk = np.ascontiguousarray(np.broadcast_to(np.asarray(skip_steps, dtype=np.int64), (n_inst,)))
    out = np.empty((n_inst, 5))
    dp = ct.POINTER(ct.c_double)
    _check(load_library().lw_pair_modes(m.ctypes.data_as(dp), m.shape[0], m.shape[1],
                                        off.ctypes.data_as(ct.POINTER(ct.c_int32)), n_inst, float(dt),
                                        int(out_stride), w.ctypes.data_as(dp),
                                        sk.ctypes.data_as(ct.POINTER(ct.c_int64)), out.ctypes.data_as(dp)))
    return out


def gamma0(q: float, m: float, omega0: float) -> float:
    return float(load_library().lw_gamma0(q, m, omega0))


def _vec3(v):
    a = (ct.c_double * 3)(*[float(x) for x in np.asarray(v, dtype=np.float64).reshape(3)])
    return a


def gf_pair(R, p1, p2, omega0: float) -> tuple[float, float]:
    """(delta_12 / gamma_0, gamma_12 / gamma_0) of two identical dipoles with axes p1, p2
    at separation vector R from the free-space dyadic Green's function (App. A)."""
    out = (ct.c_double * 2)()
    _check(load_library().lw_gf_pair(_vec3(R), _vec3(p1), _vec3(p2), float(omega0), out))
    return out[0], out[1]


def exact_modes(R, p, q: float, m: float, omega0: float) -> dict:
    """Exact classical normal modes of two identical oscillators with common axis p at
    separation vector R: gamma_plus, gamma_minus, omega_plus, omega_minus, delta_omega."""
    out = (ct.c_double * 5)()
    _check(load_library().lw_exact_modes(_vec3(R), _vec3(p), float(q), float(m), float(omega0), out))
    return dict(zip(("gamma_plus", "gamma_minus", "omega_plus", "omega_minus", "delta_omega"), list(out)))
