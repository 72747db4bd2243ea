#!/usr/bin/env python3
"""Write tests/golden/fullsize_refs.npz: the oracle's references for the full-size parity tests.

For every workload recipe at its full size, on the workload's oracle sample of trees: the
float64 fitness and its float32 envelope (oracle/envelope.py). For the differentiation
workload also the float64 constant gradients of the sample trees with their envelopes, and the
X gradient of the sample trees (all weights 1) at 4,096 seeded points with its envelopes.

Only oracle/ and synth/ are called. Each entry stores a hash of the exact inputs it was
computed from (the sample rows, X, Y, the points), so a test can tell a stale file from a
current one. Run from the repository root:  python tests/golden/make_fullsize_refs.py
"""

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from oracle import envelope as E  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "fullsize_refs.npz")
WORKLOADS = ("plain", "hybrid", "dataparallel", "batched", "grad")
GRAD_POINTS = 4096
GRAD_LANES_K = (2, 3, 4)


def targets(w):
    Y = w.Y if w.Y is not None else w.targets_from(O.predict(*w.hidden, w.X, 1)[:, 0, :])
    return np.ascontiguousarray(np.asarray(Y, np.float32).reshape(w.n_out, w.D))


def input_hash(w, Y, rows, extra=b""):
    h = hashlib.sha256()
    for a in (w.type[rows], w.value[rows], w.size[rows], w.X, Y):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(extra)
    return h.hexdigest()[:32]


def grad_points(D):
    return np.sort(np.random.default_rng(1234).choice(D, size=min(GRAD_POINTS, D), replace=False))


def main():
    out = {}
    for name in WORKLOADS:
        t0 = time.time()
        w = synth.workload(name)
        Y = targets(w)
        rows = np.asarray(w.sample)
        m64 = O.mse(w.type, w.value, w.size, w.X, Y, w.n_out, rows=list(rows))
        lo, hi, nan = E.fitness(w.type, w.value, w.size, w.X, Y, w.n_out, rows=list(rows))
        out[f"{name}/hash"] = np.array(input_hash(w, Y, rows))
        out[f"{name}/rows"] = rows
        out[f"{name}/m64"] = m64
        out[f"{name}/lo"] = lo
        out[f"{name}/hi"] = hi
        out[f"{name}/nan"] = nan
        if name == "grad":
            pts = grad_points(w.D)
            m, gv64, gx64 = O.grad(w.type, w.value, w.size, w.X, Y, rows=list(rows))
            glo, ghi, gnan, xlo, xhi, xnan = E.grad(w.type, w.value, w.size, w.X, Y, rows=list(rows),
                                                    lanes_k=GRAD_LANES_K)
            out["grad/ghash"] = np.array(input_hash(w, Y, rows, pts.tobytes()))
            out["grad/points"] = pts
            for k, v in (("gv64", gv64), ("gv_lo", glo), ("gv_hi", ghi), ("gv_nan", gnan)):
                out[f"grad/{k}"] = v
            for k, v in (("gx64", gx64), ("gx_lo", xlo), ("gx_hi", xhi), ("gx_nan", xnan)):
                out[f"grad/{k}"] = v[:, pts]
        print(f"{name}: {len(rows)} rows, {time.time() - t0:.1f} s", flush=True)
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT} ({os.path.getsize(OUT) / 1e6:.2f} MB)")


if __name__ == "__main__":
    main()
