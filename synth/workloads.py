"""The five seeded workloads of the fitness-evaluation path, plus scaled-down variants.

Each workload draws, from one numpy PCG64 stream seeded per workload and in
this order: the population, the input matrix X, the hidden target tree(s),
the noise, and the oracle sample. Sizes follow the paper's symbolic
regression setting (populations of 100..1e6 trees, up to 512 nodes, 60 to
1e5 data points, several input variables; §V-A, §V-C) and extend it.

Target values: the 'plain' workload uses the closed form x^3 + x^2 + x plus
noise, 'pagie' the Pagie polynomial 1/(1+x^-4) + 1/(1+y^-4) (the
threshold study of §V-B), and 'classify' class labels (one row) from the
argmax of random linear projections of X (the classification domain of
§V-D); all are computed here. The other workloads use hidden expression
trees; their targets are hidden(X) + noise, assembled by the caller from
`hidden` and `noise` with the evaluator the caller owns (see
`Workload.targets_from`).
"""

from dataclasses import dataclass, field

import numpy as np

from . import trees as tr

WORKLOADS = {
    # name: recipe
    "plain": dict(
        desc="64 trees, Lmax 64, grow depth<=5, {+,-,*,pdiv}, 1 var U(-1,1), 256 points, "
             "y = x^3+x^2+x + N(0,0.01)",
        P=64, Lmax=64, V=1, D=256, funcs="F4", shape=("grow", 5, 5), x=("uniform", -1.0, 1.0),
        target="poly3", sigma=0.01, n_out=1, seed=0, n_sample=None),
    "hybrid": dict(
        desc="10,000 trees, Lmax 256, ramped half-and-half depth 2..8, 11 ops, 2 vars U(-4,4), "
             "2,000 points, hidden full(4) tree + N(0,0.01)",
        P=10_000, Lmax=256, V=2, D=2_000, funcs="F11", shape=("ramped", 2, 8), x=("uniform", -4.0, 4.0),
        target=("full", 4), sigma=0.01, n_out=1, seed=1, n_sample=None),
    "dataparallel": dict(
        desc="1,000 trees, Lmax 512, ramped half-and-half depth 2..10, 11 ops, 5 vars U(-3,3), "
             "1,000,000 points, hidden full(5) tree + N(0,0.05)",
        P=1_000, Lmax=512, V=5, D=1_000_000, funcs="F11", shape=("ramped", 2, 10), x=("uniform", -3.0, 3.0),
        target=("full", 5), sigma=0.05, n_out=1, seed=2, n_sample=20),
    "batched": dict(
        desc="200,000 trees, Lmax 1024, exact lengths log-uniform in [3,1024], 11 ops, 4 vars U(-2,2), "
             "4,096 points, 3 outputs (three hidden full(4) trees + N(0,0.01)), 10% Modi trees",
        P=200_000, Lmax=1024, V=4, D=4_096, funcs="F11", shape=("loguniform", 3, 1024), x=("uniform", -2.0, 2.0),
        target=("full", 4), sigma=0.01, n_out=3, seed=3, n_sample=2_000, modi_frac=0.1),
    "grad": dict(
        desc="50,000 trees, Lmax 256, ramped half-and-half depth 2..8, <=32 constants per tree, 11 ops, "
             "8 vars N(0,1), 65,536 points, hidden full(4) tree + N(0,0.01)",
        P=50_000, Lmax=256, V=8, D=65_536, funcs="F11", shape=("ramped", 2, 8), x=("normal", 0.0, 1.0),
        target=("full", 4), sigma=0.01, n_out=1, seed=4, n_sample=100, const_cap=32),
    # the same shapes with only the cheap arithmetic operators: the interpreter's dispatch cost is
    # then most of the work per node
    "hybrid-arith": dict(
        desc="10,000 trees, Lmax 256, ramped half-and-half depth 2..8, {+,-,*,pdiv}, 2 vars U(-4,4), "
             "2,000 points, hidden full(4) tree + N(0,0.01)",
        P=10_000, Lmax=256, V=2, D=2_000, funcs="F4", shape=("ramped", 2, 8), x=("uniform", -4.0, 4.0),
        target=("full", 4), sigma=0.01, n_out=1, seed=11, n_sample=None),
    "batched-arith": dict(
        desc="200,000 trees, Lmax 1024, exact lengths log-uniform in [3,1024] (even ones less one), {+,-,*,pdiv}, 4 vars "
             "U(-2,2), 4,096 points, 3 outputs (three hidden full(4) trees + N(0,0.01)), 10% Modi trees",
        P=200_000, Lmax=1024, V=4, D=4_096, funcs="F4", shape=("loguniform", 3, 1024), x=("uniform", -2.0, 2.0),
        target=("full", 4), sigma=0.01, n_out=3, seed=13, n_sample=2_000, modi_frac=0.1),
    "classify": dict(
        desc="classification, Wine-shaped: 5,000 multi-output trees (Modi outputs for 3 classes), ramped "
             "half-and-half depth 2..6, 11 ops, 13 vars N(0,1), 178 points, labels = argmax of 3 random "
             "linear projections",
        P=5_000, Lmax=256, V=13, D=178, funcs="F11", shape=("ramped", 2, 6), x=("normal", 0.0, 1.0),
        target="linear_argmax", sigma=0.0, n_out=3, seed=6, n_sample=None, modi_frac=1.0),
    "yeast": dict(
        desc="classification, Yeast-shaped: 5,000 multi-output trees (Modi outputs for 10 classes), ramped "
             "half-and-half depth 2..6, 11 ops, 8 vars N(0,1), 1,484 points, labels = argmax of 10 random "
             "linear projections",
        P=5_000, Lmax=256, V=8, D=1_484, funcs="F11", shape=("ramped", 2, 6), x=("normal", 0.0, 1.0),
        target="linear_argmax", sigma=0.0, n_out=10, seed=8, n_sample=None, modi_frac=1.0),
    "pagie": dict(
        desc="Pagie polynomial 1/(1+x^-4) + 1/(1+y^-4): trees ramped half-and-half depth 2..8, Lmax 512, "
             "{+,-,*,pdiv,sin,cos,tan}, 2 vars U(-5,5), no noise",
        P=10_000, Lmax=512, V=2, D=16_384, funcs="F7", shape=("ramped", 2, 8), x=("uniform", -5.0, 5.0),
        target="pagie", sigma=0.0, n_out=1, seed=5, n_sample=None),
}


@dataclass
class Workload:
    name: str
    desc: str
    P: int
    Lmax: int
    V: int
    D: int
    n_out: int
    type: np.ndarray            # float32 [P][Lmax]
    value: np.ndarray           # float32 [P][Lmax]
    size: np.ndarray            # float32 [P][Lmax]
    X: np.ndarray               # float32 [V][D]  (variable-major)
    noise: np.ndarray           # float32 [n_out][D]
    Y: np.ndarray = None        # float32 [n_out][D] when the target has a closed form
    hidden: tuple = None        # (type, value, size) float32 [n_out][Lh] when the target is a hidden tree
    sample: np.ndarray = None   # int64 tree indices for oracle-sized checks
    meta: dict = field(default_factory=dict)

    def lengths(self):
        return self.size[:, 0].astype(np.int64)

    def targets_from(self, hidden_pred):
        """Targets = hidden-tree prediction (any precision, [n_out][D]) + noise, as float32."""
        hp = np.asarray(hidden_pred, np.float64).reshape(self.n_out, self.D)
        return (hp + self.noise.astype(np.float64)).astype(np.float32)


def _draw_x(rng, spec, V, D):
    kind, a, b = spec
    if kind == "uniform":
        X = rng.uniform(a, b, size=(V, D))
    else:
        X = rng.normal(a, b, size=(V, D))
    return X.astype(np.float32)


def _population(rng, r, P):
    funcs = getattr(tr, r["funcs"])
    kind = r["shape"][0]
    if kind == "grow":
        d = r["shape"][2]
        T, Vv, S = tr.depth_limited(rng, P, d, False, funcs, r["V"], r["Lmax"], r.get("const_cap"))
        return T, Vv, S, None
    if kind == "ramped":
        lo, hi = r["shape"][1], r["shape"][2]
        depth = rng.integers(lo, hi + 1, P)
        full = (np.arange(P) % 2) == 0
        T, Vv, S = tr.depth_limited(rng, P, depth, full, funcs, r["V"], r["Lmax"], r.get("const_cap"))
        modi = tr.assign_modi(rng, T, r["n_out"], r["modi_frac"]) if r.get("modi_frac") else None
        return T, Vv, S, modi
    if kind == "loguniform":
        lo, hi = r["shape"][1], r["shape"][2]
        L = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), P))).astype(np.int64)
        L = np.clip(L, lo, min(hi, r["Lmax"]))
        if not (tr.ARITY[np.asarray(funcs)] == 1).any():
            L = L - (L % 2 == 0)          # binary ops only: a tree has an odd number of nodes
        T, Vv, S = tr.exact_length(rng, L, funcs, r["V"], r["Lmax"])
        modi = None
        if r.get("modi_frac"):
            modi = tr.assign_modi(rng, T, r["n_out"], r["modi_frac"])
        return T, Vv, S, modi
    raise ValueError(kind)


def workload(name, P=None, D=None, seed=None):
    """Build a workload by name; P and D may be overridden for scaled-down parity cases."""
    r = dict(WORKLOADS[name])
    P = r["P"] if P is None else int(P)
    D = r["D"] if D is None else int(D)
    seed = r["seed"] if seed is None else int(seed)
    rng = np.random.default_rng(seed)
    T, Vv, S, modi = _population(rng, r, P)
    X = _draw_x(rng, r["x"], r["V"], D)
    hidden = None
    Y = None
    if r["target"] not in ("poly3", "pagie", "linear_argmax"):
        depth = r["target"][1]
        Lh = 2 ** (depth + 1)
        hidden = tr.depth_limited(rng, r["n_out"], depth, True, getattr(tr, r["funcs"]), r["V"], Lh)
    noise = (rng.normal(0.0, r["sigma"], size=(r["n_out"], D))).astype(np.float32)
    if r["target"] == "poly3":
        x = X[0].astype(np.float64)
        Y = ((x ** 3 + x ** 2 + x)[None, :] + noise.astype(np.float64)).astype(np.float32)
    if r["target"] == "linear_argmax":
        W = rng.normal(0.0, 1.0, size=(r["n_out"], r["V"]))
        Y = np.argmax(W @ X.astype(np.float64), axis=0).astype(np.float32)[None, :]
    if r["target"] == "pagie":
        x, y = X[0].astype(np.float64), X[1].astype(np.float64)
        with np.errstate(divide="ignore"):
            f = 1.0 / (1.0 + x ** -4) + 1.0 / (1.0 + y ** -4)
        Y = (f[None, :] + noise.astype(np.float64)).astype(np.float32)
    n_sample = r.get("n_sample")
    lengths = S[:, 0].astype(np.int64)
    if n_sample is None or n_sample >= P:
        sample = np.arange(P)
    else:
        longest = np.argsort(-lengths, kind="stable")[:5]
        must = set(longest.tolist())
        if modi is not None and len(modi):
            must |= set(modi[:50].tolist())
        rest = np.setdiff1d(np.arange(P), np.fromiter(must, np.int64))
        extra = rng.choice(rest, size=max(n_sample - len(must), 0), replace=False)
        sample = np.sort(np.concatenate([np.fromiter(must, np.int64), extra]))
    meta = {"seed": seed, "modi_trees": modi, "sigma": r["sigma"], "recipe": name}
    return Workload(name=name, desc=r["desc"], P=P, Lmax=r["Lmax"], V=r["V"], D=D, n_out=r["n_out"],
                    type=T, value=Vv, size=S, X=X, noise=noise, Y=Y, hidden=hidden, sample=sample, meta=meta)
