"""The oracle's references for the full-size parity tests: read from
tests/golden/fullsize_refs.npz (written by tests/golden/make_fullsize_refs.py
from oracle/ and synth/ only) when the stored input hash matches the
workload, computed with the oracle otherwise."""

import os
import sys

import numpy as np

from parity import FitnessRef, GradRef

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)
import make_fullsize_refs as M  # noqa: E402

_npz = None


def _stored():
    global _npz
    if _npz is None:
        path = os.path.join(GOLDEN, "fullsize_refs.npz")
        _npz = dict(np.load(path, allow_pickle=False)) if os.path.exists(path) else {}
    return _npz


def current(name, w, Y, key="hash", extra=b""):
    """Whether the stored entry was computed from exactly these inputs."""
    st = _stored()
    k = f"{name}/{key}"
    return k in st and str(st[k]) == M.input_hash(w, Y, np.asarray(w.sample), extra)


def fullsize_fitness_ref(name, w, Y):
    if current(name, w, Y):
        st = _stored()
        ref = FitnessRef.__new__(FitnessRef)
        ref.m64, ref.lo, ref.hi, ref.nan = (st[f"{name}/{k}"] for k in ("m64", "lo", "hi", "nan"))
        return ref
    print(f"[{name}] stored references are stale or missing: computing them", flush=True)
    return FitnessRef(w.type, w.value, w.size, w.X, Y, w.n_out, rows=list(w.sample))


def fullsize_grad_ref(w, Y):
    """(GradRef of the sample trees with grad_X restricted to the reference points, points)."""
    pts = M.grad_points(w.D)
    rows = list(w.sample)
    st = _stored()
    ref = GradRef.__new__(GradRef)
    if current("grad", w, Y, "ghash", pts.tobytes()):
        ref.m64 = st["grad/m64"]
        ref.gv64, ref.gv_lo, ref.gv_hi, ref.gv_nan = (st[f"grad/{k}"] for k in ("gv64", "gv_lo", "gv_hi", "gv_nan"))
        ref.gx64, ref.gx_lo, ref.gx_hi, ref.gx_nan = (st[f"grad/{k}"] for k in ("gx64", "gx_lo", "gx_hi", "gx_nan"))
    else:
        print("[grad] stored gradient references are stale or missing: computing them", flush=True)
        full = GradRef(w.type, w.value, w.size, w.X, Y, rows=rows, lanes_k=M.GRAD_LANES_K)
        ref.m64, ref.gv64, ref.gv_lo, ref.gv_hi, ref.gv_nan = full.m64, full.gv64, full.gv_lo, full.gv_hi, full.gv_nan
        ref.gx64, ref.gx_lo, ref.gx_hi, ref.gx_nan = (a[:, pts] for a in (full.gx64, full.gx_lo, full.gx_hi, full.gx_nan))
    ref.const = w.type[rows] == 1
    return ref, pts
