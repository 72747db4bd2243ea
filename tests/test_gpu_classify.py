"""Classification fitness (argmax accuracy over multi-output trees) on the GPU
against the oracle. The device takes the argmax on float32 outputs, so each
tree's hit count must lie between the oracle's robust hits and robust hits
plus near-ties (points where float64 and float32 evaluations disagree), and
equal it exactly where there are none. Needs an MI355X."""

import numpy as np
import pytest
import torch

import oracle as O
import paper_2501_17168_amd as tgp
import synth
from synth import trees as ST

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

MODES = {
    "tree-major-k4": dict(mode=1, points_per_lane=4, block_waves=1),
    "point-major-k8": dict(mode=2, points_per_lane=8, block_waves=4, trees_per_unit=4),
    "persist-k4": dict(mode=3, points_per_lane=4, block_waves=4, trees_per_unit=1),
    "persist-static-k8": dict(mode=3, points_per_lane=8, block_waves=1, trees_per_unit=2, flags=2),
}


def check(w, labels, n_classes, cfg, label, min_exact=0.9):
    pop = tgp.Population(*(torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (w.type, w.value, w.size)))
    X = torch.from_numpy(w.X).to(DEV)
    lab = torch.from_numpy(np.ascontiguousarray(labels, np.float32)).to(DEV)
    acc = tgp.eval_accuracy(pop, X, lab, n_classes, config=tgp.cfg(cfg) if cfg else None).cpu().numpy()
    lo, hi = O.accuracy_bounds(w.type, w.value, w.size, w.X, labels, n_classes)
    D = w.X.shape[1]
    valid = ~np.isnan(lo)
    np.testing.assert_array_equal(np.isnan(acc), ~valid)
    hits = np.rint(acc[valid].astype(np.float64) * D)
    lo_h, hi_h = np.rint(lo[valid] * D), np.rint(hi[valid] * D)
    assert np.all((hits >= lo_h) & (hits <= hi_h)), f"{label}: counts outside the oracle's bounds"
    exact = lo_h == hi_h
    assert exact.mean() > min_exact
    print(f"[{label}] {valid.sum()} trees, {exact.sum()} without near-ties, mean accuracy "
          f"{acc[valid].mean():.3f}", flush=True)


@pytest.mark.parametrize("mode", list(MODES))
def test_wine_shaped_all_schedules(mode):
    w = synth.workload("classify", P=600)
    check(w, w.Y[0], 3, MODES[mode], f"classify {mode}")


@pytest.mark.parametrize("n_classes,D", [(2, 1000), (4, 1484)])
def test_other_class_counts_with_invalid_and_plain_trees(n_classes, D):
    """2 and 4 classes (the breast-cancer and a Yeast-length shape, features capped at 13),
    labels with out-of-range values, single-output trees mixed in, and an invalid tree."""
    rng = np.random.default_rng(n_classes)
    w = synth.workload("classify", P=400, D=D)
    T, V, S = (a.copy() for a in (w.type, w.value, w.size))
    T = np.where(T >= 3, np.where(T - 3 < n_classes, T, 2), T).astype(np.float32)   # Modi outputs < C
    plain = rng.random(400) < 0.2
    T[plain] = np.where(T[plain] >= 3, 2.0, T[plain])                                # no Modi nodes
    S[7, 0] = 999.0                                                                   # invalid length
    w.type, w.value, w.size = T, V, S
    labels = rng.integers(-1, n_classes + 1, D).astype(np.float32)
    check(w, labels, n_classes, None, f"{n_classes} classes")


def test_fullsize_wine_shaped_autotuned():
    w = synth.workload("classify")
    pop = tgp.Population(*(torch.from_numpy(a).to(DEV) for a in (w.type, w.value, w.size)))
    cfg = tgp.autotune(pop, torch.from_numpy(w.X).to(DEV), torch.from_numpy(np.zeros((3, w.D), np.float32)).to(DEV),
                       n_out=3)
    check(w, w.Y[0], 3, cfg, "classify full size")


def test_status_output_and_host_checks():
    """tree_status matches the plan's status codes; a single class is refused on the host."""
    w = synth.workload("classify", P=64)
    S = w.size.copy()
    S[3, 0] = np.nan
    pop = tgp.Population(*(torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (w.type, w.value, S)))
    X = torch.from_numpy(w.X).to(DEV)
    lab = torch.from_numpy(np.ascontiguousarray(w.Y[0])).to(DEV)
    st = torch.empty(64, dtype=torch.int32, device=DEV)
    acc = tgp.eval_accuracy(pop, X, lab, 3, tree_status=st).cpu().numpy()
    info = O.plan(w.type, w.value, S, w.V, 3)
    np.testing.assert_array_equal(st.cpu().numpy(), info[:, 0])
    assert np.isnan(acc[3]) and np.isfinite(np.delete(acc, 3)).all()
    with pytest.raises(tgp.TgpError):
        tgp.eval_accuracy(pop, X, lab, 1)


@pytest.mark.parametrize("mode", ["tree-major-k4", "persist-k4"])
def test_ten_classes_yeast_shaped(mode):
    """10 classes (the Yeast shape of §V-D: 8 features, 1,484 points): every tree has Modi outputs
    for up to 10 classes, so the kernel runs with its wide output accumulators."""
    w = synth.workload("yeast", P=300)
    assert w.n_out == 10 and len(np.unique(w.type[w.type >= 3])) == 10
    # ten outputs give more near-ties between the top two classes: 86% of these trees have none
    check(w, w.Y[0], 10, MODES[mode], f"yeast {mode}", min_exact=0.8)


def test_ten_class_predictions():
    """Per-output predictions of 10-output trees against the oracle's float64 outputs (the wide
    accumulators and the output index carried by the accumulate word)."""
    w = synth.workload("yeast", P=120, D=500)
    pop = tgp.Population(*(torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (w.type, w.value, w.size)))
    _, pred = tgp.eval_multi_output(pop, torch.from_numpy(w.X).to(DEV), None, n_out=10, want_pred=True)
    pred = pred.cpu().numpy().astype(np.float64)
    ref = O.predict(w.type, w.value, w.size, w.X, 10)
    fin = np.isfinite(ref) & (np.abs(ref) < 1e6)
    err = np.abs(pred - ref)[fin] / np.maximum(np.abs(ref[fin]), 1.0)
    assert (err < 1e-3).mean() > 0.99, np.sort(err)[-5:]
    # outputs that a tree has no Modi node for are exactly 0
    for t in range(w.P):
        used = set((w.type[t][w.type[t] >= 3] - 3).astype(int).tolist())
        for o in range(10):
            if o not in used:
                assert (pred[t, o] == 0).all()
