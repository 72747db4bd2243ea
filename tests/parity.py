"""Comparison protocol between the device results and the CPU oracle.

Fitness values (float32 on the device, float64 in the oracle):
  a tree is well-conditioned when the float64 oracle value m64 and the
  float32 shadow value m32s are both finite and |m32s - m64| <= 0.1 * tol,
  tol = max(1e-5 |m64|, 1e-6). Well-conditioned trees must satisfy
  |m_gpu - m64| <= tol (the relative 1e-5 / absolute 1e-6 bar).
  The rest are reported; for them the device value must agree with the
  shadow (same non-finite class, or within 1e-3 relative) for all but a
  small fraction, since float32 evaluation of an ill-conditioned tree has
  no unique answer (branch flips of protected operators, cancellation).

  The device's transcendental functions are a float32 library within a few
  ulp of the correctly rounded results the shadow uses. So `shadows()` also
  returns two shadows whose transcendental results move by random steps of
  up to 2 ulp, and a tree is well-conditioned only if every shadow passes.
"""

import numpy as np

import oracle as O

REL = 1e-5
ABS = 1e-6
LIB_ULP = 2
SEEDS = (1, 2)


def shadows(pop_type, pop_value, pop_size, X, Y, n_out=1, rows=None):
    """[3][R]: the float32 shadow, then two with transcendental results perturbed by up to LIB_ULP ulp."""
    out = [O.mse_shadow32(pop_type, pop_value, pop_size, X, Y, n_out, rows=rows)]
    for seed in SEEDS:
        out.append(O.mse_shadow32(pop_type, pop_value, pop_size, X, Y, n_out, rows=rows, ulp=LIB_ULP, seed=seed))
    return np.stack(out)


def classify(m64, m32s):
    """m32s: one shadow [R] or shadows [S][R] (the first unperturbed)."""
    m64 = np.asarray(m64, np.float64)
    m32s = np.atleast_2d(np.asarray(m32s, np.float64))
    tol = np.maximum(REL * np.abs(m64), ABS)
    with np.errstate(invalid="ignore"):
        well = np.isfinite(m64) & np.all(np.isfinite(m32s) & (np.abs(m32s - m64) <= 0.1 * tol), axis=0)
    return well, tol


def compare_fitness(got, m64, m32s, max_ill_mismatch=0.05, label=""):
    """Assert the protocol; return a small report dict."""
    got = np.asarray(got, np.float64)
    m64 = np.asarray(m64, np.float64)
    well, tol = classify(m64, m32s)
    m32s = np.atleast_2d(np.asarray(m32s, np.float64))[0]
    with np.errstate(invalid="ignore"):
        err = np.abs(got - m64)
        bad = well & ~(err <= tol)
    if bad.any():
        i = np.nonzero(bad)[0][:5]
        raise AssertionError(f"{label}: {int(bad.sum())}/{int(well.sum())} well-conditioned trees out of "
                             f"tolerance; e.g. idx {i.tolist()} gpu {got[i].tolist()} oracle {m64[i].tolist()}")
    ill = ~well
    with np.errstate(invalid="ignore"):
        fin = np.isfinite(m32s)
        ok = np.where(fin, np.abs(got - m32s) <= 1e-3 * np.abs(m32s) + 1e-6,
                      ~np.isfinite(got) & (np.isnan(got) == np.isnan(m32s)))
    ill_bad = ill & ~ok
    frac = float(ill_bad.sum()) / max(1, len(got))
    assert frac <= max_ill_mismatch, f"{label}: {int(ill_bad.sum())} ill-conditioned mismatches ({frac:.3%})"
    rel = err[well] / np.maximum(np.abs(m64[well]), 1e-30)
    return {"n": len(got), "well": int(well.sum()), "ill": int(ill.sum()), "ill_mismatch": int(ill_bad.sum()),
            "max_rel_err_well": float(rel.max()) if rel.size else 0.0}


def grad_shadows(pop_type, pop_value, pop_size, X, Y, rows=None):
    """Float32 shadows of the gradient sweep: [(grad_value, grad_X)] unperturbed, then perturbed as in shadows()."""
    out = []
    for ulp, seed in [(0, 0)] + [(LIB_ULP, sd) for sd in SEEDS]:
        _, gv, gx = O.grad(pop_type, pop_value, pop_size, X, Y, rows=rows, shadow=True, ulp=ulp, seed=seed)
        out.append((gv, gx))
    return out


def grad_close(g, ref, rel):
    """|g - ref| <= rel * max(|ref|, 1e-3 * max|ref| of the row) + 1e-7, elementwise, per row."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref), axis=-1, keepdims=True))
    with np.errstate(invalid="ignore"):
        return np.abs(g - ref) <= rel * scale + 1e-7


def well_grad(shadow_list, gv64, gx64, rel_v=1e-4, rel_x=2e-4):
    """Components whose every float32 shadow agrees with float64 to a tenth of the tolerance."""
    wv = np.ones(np.shape(gv64), bool)
    wx = np.ones(np.shape(gx64), bool)
    for gv, gx in shadow_list:
        wv &= grad_close(gv, gv64, rel_v)
        wx &= grad_close(gx, gx64, rel_x)
    return wv, wx
