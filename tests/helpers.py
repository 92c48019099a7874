"""Shared test utilities: error norms and GPU availability."""
import numpy as np

GROUPS = {"phi": [0], "A": [1, 2, 3], "E": [4, 5, 6], "B": [7, 8, 9]}


def gpu_ready() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def field_errors(got: np.ndarray, ref: np.ndarray) -> dict:
    """relL2 and relmax per output group over the (time, point) entries that are finite in
    the reference; got and ref are [n_times][10][n_pts]."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    ok = np.isfinite(ref).all(axis=1)                     # [n_times][n_pts]
    res = {}
    for name, comps in GROUPS.items():
        g = got[:, comps, :].transpose(0, 2, 1)[ok]       # [n_ok][len(comps)]
        r = ref[:, comps, :].transpose(0, 2, 1)[ok]
        den2 = np.sqrt((r * r).sum())
        denm = np.abs(r).max() if r.size else 0.0
        d = g - r
        res[name] = (np.sqrt((d * d).sum()) / den2 if den2 > 0 else float(np.abs(d).max(initial=0.0)),
                     np.abs(d).max(initial=0.0) / denm if denm > 0 else float(np.abs(d).max(initial=0.0)))
    return res


def pointwise_rel_p999(got: np.ndarray, ref: np.ndarray) -> dict:
    """99.9th percentile over unmasked (point, time) entries of the pointwise relative error
    |got - ref| / |ref| of each output group's vector (Phi as a scalar), so that the weak
    field far from the charges is judged on its own scale, not the group's maximum."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    ok = np.isfinite(ref).all(axis=1)
    res = {}
    for name, comps in GROUPS.items():
        g = got[:, comps, :].transpose(0, 2, 1)[ok]
        r = ref[:, comps, :].transpose(0, 2, 1)[ok]
        num = np.linalg.norm(g - r, axis=1)
        den = np.linalg.norm(r, axis=1)
        nz = den > 0
        res[name] = float(np.percentile(num[nz] / den[nz], 99.9)) if nz.any() else 0.0
    return res


def assert_fields_close(got, ref, tol: float, what: str = ""):
    errs = field_errors(got, ref)
    bad = {k: v for k, v in errs.items() if not (v[0] <= tol and v[1] <= tol)}
    assert not bad, f"{what}: relL2/relmax above {tol}: {bad} (all: {errs})"
    return errs
