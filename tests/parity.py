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
"""

import numpy as np

REL = 1e-5
ABS = 1e-6


def classify(m64, m32s):
    m64 = np.asarray(m64, np.float64)
    m32s = np.asarray(m32s, np.float64)
    tol = np.maximum(REL * np.abs(m64), ABS)
    with np.errstate(invalid="ignore"):
        well = np.isfinite(m64) & np.isfinite(m32s) & (np.abs(m32s - m64) <= 0.1 * tol)
    return well, tol


def compare_fitness(got, m64, m32s, max_ill_mismatch=0.05, label=""):
    """Assert the protocol; return a small report dict."""
    got = np.asarray(got, np.float64)
    m64 = np.asarray(m64, np.float64)
    m32s = np.asarray(m32s, np.float64)
    well, tol = classify(m64, m32s)
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
