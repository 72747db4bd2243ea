"""The seeded input generators: determinism, validity of every tree, recipe properties."""

import numpy as np
import pytest

import oracle as O
import synth


@pytest.mark.parametrize("name,P,D", [("plain", None, None), ("hybrid", 300, 500), ("dataparallel", 40, 3000),
                                      ("batched", 300, 700), ("grad", 300, 600)])
def test_deterministic_and_valid(name, P, D):
    a = synth.workload(name, P=P, D=D)
    b = synth.workload(name, P=P, D=D)
    for f in ("type", "value", "size", "X", "noise"):
        assert getattr(a, f).tobytes() == getattr(b, f).tobytes(), f
    assert a.type.dtype == np.float32 and a.type.shape == (a.P, a.Lmax)
    assert a.X.shape == (a.V, a.D)
    pl = O.plan(a.type, a.value, a.size, a.V, a.n_out)
    assert (pl[:, 0] == 0).all(), np.bincount(pl[:, 0])
    if a.hidden is not None:
        hp = O.plan(*a.hidden, a.V, 1)
        assert (hp[:, 0] == 0).all()


def test_different_seeds_differ():
    a = synth.workload("hybrid", P=50, D=50, seed=1)
    b = synth.workload("hybrid", P=50, D=50, seed=2)
    assert a.type.tobytes() != b.type.tobytes()


def test_exact_lengths_loguniform():
    w = synth.workload("batched", P=4000, D=64)
    L = w.lengths()
    assert L.min() >= 3 and L.max() <= 1024
    # mean of round(exp(U(ln 3, ln 1024))) is about (1024 - 3) / ln(1024 / 3) = 175
    assert 150 < L.mean() < 200
    modi = w.meta["modi_trees"]
    assert 0.07 < len(modi) / w.P < 0.13
    pl = O.plan(w.type, w.value, w.size, w.V, 3)
    assert (pl[modi, 4] > 0).mean() > 0.95
    assert pl[:, 4].max() == 3


def test_const_cap_and_ranges():
    w = synth.workload("grad", P=2000, D=16)
    assert (w.type == 1).sum(1).max() <= 32
    c = w.value[w.type == 1]
    assert c.min() >= -5 and c.max() <= 5
    w = synth.workload("hybrid", P=2000, D=4000)
    assert w.X.min() >= -4 and w.X.max() <= 4
    ops = w.value[w.type == 2].astype(int)
    assert set(np.unique(ops)) == set(range(11))


def test_plain_target_closed_form():
    w = synth.workload("plain")
    x = w.X[0].astype(np.float64)
    np.testing.assert_allclose(w.Y[0], (x ** 3 + x ** 2 + x + w.noise[0]).astype(np.float32))
    assert w.Y.dtype == np.float32 and w.hidden is None


def test_hidden_targets_are_finite_and_vary():
    for name in ("hybrid", "dataparallel", "batched", "grad"):
        w = synth.workload(name, P=20, D=5000)
        hp = O.predict(*w.hidden, w.X, 1)[:, 0, :]
        assert np.isfinite(hp).all(), name
        assert (hp.var(axis=1) > 1e-6).all(), name
