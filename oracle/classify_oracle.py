"""Plain CPU oracle for classification fitness -- TEST INFRASTRUCTURE.

Only the test suite, the package smoke check and the benchmark's
CPU-baseline leg may import or run this module. It shares no code with the
device library.

Classification (the classification domain of §V-D) evaluates a
multi-output tree (§IV-C) with one output per class. The predicted class of
a point is the index of the largest output, and the fitness is the fraction
of points whose predicted class equals the label (accuracy, higher is
better).

Readings where the paper is silent: ties go to the first (lowest) index; a
NaN output counts below every number (so a row of NaN outputs predicts
class 0); labels are class ids stored as float32, and a label outside
[0, C) never matches. The device takes the argmax on float32 outputs; the
oracle evaluates in float64 and, to tell robust decisions from near-ties,
also in the float32 shadows (plain and with perturbed transcendentals).
"""

import numpy as np

from .tgp_oracle import OK, Ulps, decode, eval_shadow32, eval_stack


def classes(out):
    """Predicted class per point from outputs [C][D]: the first index of the largest value,
    NaN below every number."""
    out = np.asarray(out, np.float64)
    C, D = out.shape
    cls = np.zeros(D, np.int64)
    best = out[0].copy()
    for o in range(1, C):
        v = out[o]
        take = (v > best) | (np.isnan(best) & ~np.isnan(v))
        cls[take] = o
        best[take] = v[take]
    return cls


def accuracy(pop_type, pop_value, pop_size, X, labels, n_classes, rows=None):
    """Accuracy float64 [len(rows)] from the float64 evaluator; NaN for invalid trees."""
    X = np.asarray(X)
    V = X.shape[0]
    lab = np.asarray(labels, np.float64).reshape(-1)
    rows = list(range(pop_type.shape[0]) if rows is None else rows)
    res = np.full(len(rows), np.nan)
    for k, p in enumerate(rows):
        d = decode(pop_type[p], pop_value[p], pop_size[p], V, n_classes)
        if d.status == OK:
            res[k] = np.mean(classes(eval_stack(d, X, n_classes)) == lab)
    return res


def accuracy_bounds(pop_type, pop_value, pop_size, X, labels, n_classes, rows=None, ulp=2, seeds=(1, 2)):
    """Per tree, the range a float32 evaluation may land in: (lo, hi) where lo counts the points
    whose class is the same under the float64 evaluator and every float32 shadow and matches
    the label, and hi adds the points where those evaluations disagree. NaN for invalid trees."""
    X = np.asarray(X)
    V = X.shape[0]
    lab = np.asarray(labels, np.float64).reshape(-1)
    D = lab.size
    rows = list(range(pop_type.shape[0]) if rows is None else rows)
    lo = np.full(len(rows), np.nan)
    hi = np.full(len(rows), np.nan)
    for k, p in enumerate(rows):
        d = decode(pop_type[p], pop_value[p], pop_size[p], V, n_classes)
        if d.status != OK:
            continue
        with np.errstate(all="ignore"):
            variants = [classes(eval_stack(d, X, n_classes)), classes(eval_shadow32(d, X, n_classes))]
            variants += [classes(eval_shadow32(d, X, n_classes, Ulps(ulp, s))) for s in seeds]
        agree = np.all([v == variants[0] for v in variants[1:]], axis=0)
        hits = (variants[0] == lab) & agree
        lo[k] = hits.sum() / D
        hi[k] = (hits.sum() + (~agree).sum()) / D
    return lo, hi
