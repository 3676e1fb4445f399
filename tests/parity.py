"""Comparison helpers for the GPU-vs-oracle parity tests."""
from __future__ import annotations

import numpy as np

# FP64 path: per-stage results must agree to 1e-12 relative.  The scale of a
# compared quantity is its largest magnitude over the DOF array; the momentum
# vector counts as one quantity (its components share the scale of the larger
# one), so a momentum component that is zero up to rounding (a flow along x
# only) is not compared against its own rounding noise.
REL_TOL_FP64 = 1e-12


def _scales(grid, B: dict, name: str):
    nc = grid.ncomp
    s = [max(float(np.nanmax(np.abs(B[name][k]))) if np.isfinite(B[name][k]).any() else 0.0,
             1e-300) for k in range(nc)]
    mom = list(range(1, nc - 1))
    m = max(s[k] for k in mom)
    for k in mom:
        s[k] = m
    return s


def rel_errors(grid, a: np.ndarray, b: np.ndarray) -> dict:
    """max |a-b| / scale per (DOF array, component); NaN at the same place on
    both sides counts as equal"""
    A, B = grid.split(a), grid.split(b)
    out = {}
    for name in A:
        sc = _scales(grid, B, name)
        for k in range(grid.ncomp):
            x, y = A[name][k], B[name][k]
            nx, ny = ~np.isfinite(x), ~np.isfinite(y)
            if np.any(nx != ny):
                out[(name, k)] = np.inf
                continue
            ok = ~nx
            d = np.abs(x[ok] - y[ok]).max() if ok.any() else 0.0
            out[(name, k)] = float(d / sc[k])
    return out


def assert_close(grid, gpu: np.ndarray, ref: np.ndarray, tol: float = REL_TOL_FP64, what: str = ""):
    assert gpu.shape == ref.shape
    errs = rel_errors(grid, gpu, ref)
    worst = max(errs.items(), key=lambda kv: kv[1])
    assert worst[1] <= tol, f"{what}: worst relative error {worst[1]:.3e} at {worst[0]} (tol {tol:g})"
    return worst[1]


# A pointwise view of the same bar: each value against its own magnitude,
# floored at 1e-3 of its array's scale (a value near zero is measured against
# the floor, not against its own rounding).  On the shock tube, whose density
# spans two decades, this holds the light side to the bar itself, where the
# normwise metric above would allow it a hundred times more.
POINT_FLOOR = 1e-3


def pointwise_rel_error(grid, a: np.ndarray, b: np.ndarray) -> float:
    A, B = grid.split(a), grid.split(b)
    worst = 0.0
    for name in A:
        sc = _scales(grid, B, name)
        for k in range(grid.ncomp):
            x, y = A[name][k], B[name][k]
            ok = np.isfinite(x) & np.isfinite(y)
            if np.any(np.isfinite(x) != np.isfinite(y)):
                return np.inf
            if not ok.any():
                continue
            den = np.maximum(np.abs(y[ok]), POINT_FLOOR * sc[k])
            worst = max(worst, float((np.abs(x[ok] - y[ok]) / den).max()))
    return worst


def assert_close_pointwise(grid, gpu: np.ndarray, ref: np.ndarray, tol: float, what: str = ""):
    e = pointwise_rel_error(grid, gpu, ref)
    print(f"{what}: pointwise relative error {e:.3e}", flush=True)
    assert e <= tol, f"{what}: pointwise relative error {e:.3e} (tol {tol:g})"
    return e

