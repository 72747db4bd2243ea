"""Comparison protocol between the device results and the CPU oracle.

Fitness (float32 on the device, float64 in the oracle). For every valid tree
the oracle gives the float64 value m64 and the envelope [lo, hi] of every
float32 evaluation its arithmetic model allows (oracle/envelope.py), with a
flag where a NaN is possible. The device value must lie inside the envelope
(NaN only where a NaN is possible): every tree, no exceptions. Where the
envelope lies within tol = max(1e-5 |m64|, 1e-6) of m64 (a "tight" tree), the
containment is the relative 1e-5 / absolute 1e-6 bar itself. Elsewhere no
float32 evaluation is determined to that bar, and the envelope is the bar.
Invalid trees must give NaN.

Gradients: the same with the gradient envelopes and tol = 1e-3 |g64|
(relative 1e-3) per component: constants' gradients and X gradients.

The reports give the count of each class and the largest relative error of
the device value against m64 over the tight trees.
"""

import numpy as np

import oracle as O
from oracle import envelope as E

REL = 1e-5
ABS = 1e-6
GRAD_REL = 1e-3


class FitnessRef:
    """float64 fitness and float32 envelopes of a set of rows."""

    def __init__(self, pop_type, pop_value, pop_size, X, Y, n_out=1, rows=None):
        self.m64 = O.mse(pop_type, pop_value, pop_size, X, Y, n_out, rows=rows)
        self.lo, self.hi, self.nan = E.fitness(pop_type, pop_value, pop_size, X, Y, n_out, rows=rows)


def inside(v, lo, hi, nan):
    v = np.asarray(v, np.float64)
    with np.errstate(invalid="ignore"):
        return np.where(np.isnan(v), nan, (lo <= v) & (v <= hi))


def compare_fitness(got, ref, label=""):
    """Assert the protocol on device fitness values `got` (same rows as ref); return a report."""
    got = np.asarray(got, np.float64)
    m64 = ref.m64
    valid = ~np.isnan(ref.lo) | ~np.isnan(ref.hi)
    invalid = ~valid
    bad_invalid = invalid & ~np.isnan(got)
    assert not bad_invalid.any(), f"{label}: invalid trees without NaN fitness: {np.nonzero(bad_invalid)[0][:5]}"
    ok = inside(got, ref.lo, ref.hi, ref.nan) | invalid
    if not ok.all():
        i = np.nonzero(~ok)[0][:5]
        raise AssertionError(f"{label}: {int((~ok).sum())}/{len(got)} device fitness values outside the float32 "
                             f"envelope; e.g. rows {i.tolist()} gpu {got[i].tolist()} envelope "
                             f"{list(zip(ref.lo[i].tolist(), ref.hi[i].tolist()))} float64 {m64[i].tolist()}")
    tol = np.maximum(REL * np.abs(m64), ABS)
    with np.errstate(invalid="ignore"):
        tight = valid & np.isfinite(m64) & ~ref.nan & (ref.lo >= m64 - tol) & (ref.hi <= m64 + tol)
        err = np.abs(got - m64)
        rel = err[tight] / np.maximum(np.abs(m64[tight]), ABS / REL)
        width = (ref.hi - ref.lo) / np.abs(m64)
    wide = valid & ~tight
    return {"n": len(got), "tight": int(tight.sum()), "wide": int(wide.sum()), "invalid": int(invalid.sum()),
            "nan_possible": int((valid & ref.nan).sum()),
            "max_rel_err_tight": float(rel.max()) if rel.size else 0.0,
            "median_rel_width_wide": float(np.median(width[wide])) if wide.any() else 0.0}


class GradRef:
    """float64 gradients and float32 envelopes of sum_t g_t fitness_t over a set of rows.
    lanes_k: the points-per-lane values the device may use; the envelope bounds the sums over
    points for each of them."""

    def __init__(self, pop_type, pop_value, pop_size, X, Y, n_out=1, rows=None, g=None, lanes_k=(2, 3, 4)):
        self.m64, self.gv64, self.gx64 = O.grad(pop_type, pop_value, pop_size, X, Y, n_out, rows=rows, g=g)
        (self.gv_lo, self.gv_hi, self.gv_nan,
         self.gx_lo, self.gx_hi, self.gx_nan) = E.grad(pop_type, pop_value, pop_size, X, Y, n_out, rows=rows, g=g,
                                                       lanes_k=lanes_k)
        rows = list(range(pop_type.shape[0]) if rows is None else rows)
        self.const = np.asarray(pop_type)[rows] == O.T_CONST


def _grad_check(got, g64, lo, hi, nan, mask, label):
    got = np.asarray(got, np.float64)
    ok = inside(got, lo, hi, nan) | ~mask
    if not ok.all():
        idx = np.argwhere(~ok)[:5]
        raise AssertionError(f"{label}: {int((~ok).sum())}/{int(mask.sum())} components outside the float32 "
                             f"envelope; e.g. {[(tuple(int(x) for x in i), float(got[tuple(i)]), float(lo[tuple(i)]), float(hi[tuple(i)]), float(g64[tuple(i)])) for i in idx]}")
    tol = GRAD_REL * np.abs(g64)
    with np.errstate(invalid="ignore"):
        tight = mask & np.isfinite(g64) & ~nan & (lo >= g64 - tol) & (hi <= g64 + tol)
        rel = np.abs(got - g64)[tight] / np.maximum(np.abs(g64[tight]), 1e-300)
        width = (hi - lo) / np.abs(g64)
    wide = mask & ~tight
    return {"n": int(mask.sum()), "tight": int(tight.sum()), "wide": int(wide.sum()),
            "nan_possible": int((mask & nan).sum()),
            "max_rel_err_tight": float(rel.max()) if rel.size else 0.0,
            "median_rel_width_wide": float(np.nanmedian(width[wide])) if wide.any() else 0.0}


def compare_grad_value(got, ref, label=""):
    """Constant gradients [R][Lmax] against the envelopes; zero off the constants."""
    got = np.asarray(got, np.float64)
    assert (got[~ref.const] == 0).all(), f"{label}: non-zero gradient at a non-constant position"
    return _grad_check(got, ref.gv64, ref.gv_lo, ref.gv_hi, ref.gv_nan, ref.const, label + " grad_value")


def compare_grad_x(got, ref, label=""):
    """X gradients [V][D] against the envelopes."""
    got = np.asarray(got, np.float64)
    return _grad_check(got, ref.gx64, ref.gx_lo, ref.gx_hi, ref.gx_nan, np.ones(got.shape, bool), label + " grad_X")
