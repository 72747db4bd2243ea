"""Pins for the classification-fitness oracle: the argmax rule on special
values, and accuracies of trees whose predicted class has a closed form
(§IV-C output rules, §V-D accuracy)."""

import numpy as np

import oracle as O

NAN = np.nan


def rows(nodes, sizes, L=8):
    out = [np.full((1, L), np.nan, np.float32) for _ in range(3)]
    for r, src in zip(out, ([n[0] for n in nodes], [n[1] for n in nodes], sizes)):
        r[0, :len(src)] = src
    return out


def test_argmax_rule():
    out = np.array([[1.0, 2.0, NAN, NAN, -np.inf, 3.0],
                    [1.0, 5.0, 0.0, NAN, NAN, 3.0],
                    [0.5, 5.0, -1.0, NAN, -5.0, 4.0]])
    np.testing.assert_array_equal(O.classes(out), [0, 1, 1, 0, 2, 2])


def data(seed=0, D=500, V=3):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, (V, D)).astype(np.float32)
    labels = rng.integers(0, 3, D).astype(np.float32)
    return X, labels


def test_two_variable_outputs():
    """M0(ADD)(x0, M1(ADD)(x1, 0)): outputs (x0, x1), class 1 exactly where x1 > x0."""
    X, lab = data()
    t, v, s = rows([(3, 0), (0, 0), (4, 0), (0, 1), (1, 0.0)], [5, 1, 3, 1, 1])
    acc = O.accuracy(t, v, s, X, lab, 2)
    want = np.mean((X[1] > X[0]).astype(np.float32) == lab)
    assert acc[0] == want


def test_single_output_tree_against_zeros():
    """A tree without Modi nodes predicts (root, 0, 0): class 0 where x0 >= 0 (ties to the first
    index), else class 1 (the first of the two zeros)."""
    X, lab = data(1)
    t, v, s = rows([(0, 0)], [1])
    acc = O.accuracy(t, v, s, X, lab, 3)
    want = np.mean(np.where(X[0] >= 0, 0.0, 1.0) == lab)
    assert acc[0] == want


def test_constant_class_and_out_of_range_labels():
    """Outputs (0, 0, 1) predict class 2 everywhere: accuracy is the share of label 2; a label
    of 3 or -1 never matches."""
    X, lab = data(2)
    lab[:50] = 3.0
    lab[50:60] = -1.0
    # M2(ADD)(1.0, 0.0): out2 = 1; no other Modi output, so out0 = out1 = 0
    t, v, s = rows([(5, 0), (1, 1.0), (1, 0.0)], [3, 1, 1])
    acc = O.accuracy(t, v, s, X, lab, 3)
    assert acc[0] == np.mean(lab == 2.0)


def test_invalid_tree_and_bounds():
    X, lab = data(3)
    t, v, s = rows([(2, 0), (0, 0)], [2, 1])      # ADD with one child: invalid
    assert np.isnan(O.accuracy(t, v, s, X, lab, 2)[0])
    t, v, s = rows([(3, 0), (0, 0), (4, 0), (0, 1), (1, 0.0)], [5, 1, 3, 1, 1])
    lo, hi = O.accuracy_bounds(t, v, s, X, lab, 2)
    acc = O.accuracy(t, v, s, X, lab, 2)
    assert lo[0] == hi[0] == acc[0]              # no transcendental, no near-tie: exact
