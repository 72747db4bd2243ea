"""Readers for the text fixtures under tests/golden/."""

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_tree(name, Lmax=16):
    """Returns (type, value, size) float32 rows padded with NaN to Lmax, plan figures, and the
    remaining tagged rows {tag: [list of float lists]}."""
    rows = {}
    nodes = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tag, *vals = line.split()
            vals = [float(v) for v in vals]
            if tag == "node":
                nodes.append(vals)
            else:
                rows.setdefault(tag, []).append(vals)
    n = len(nodes)
    t = np.full(Lmax, np.nan, np.float32)
    v = np.full(Lmax, np.nan, np.float32)
    s = np.full(Lmax, np.nan, np.float32)
    arr = np.array(nodes, np.float32)
    t[:n], v[:n], s[:n] = arr[:, 0], arr[:, 1], arr[:, 2]
    return (t, v, s), rows
