"""Pins of the CPU oracle against things other than itself: the paper's worked
examples (closed forms), textbook identities, an arbitrary-precision SymPy
evaluation, finite differences of the value function and a second evaluator.
"""

import math

import numpy as np
import pytest
import sympy as sp

import oracle as O
import synth
from golden_io import load_tree

rng0 = np.random.default_rng(12345)


# ------------------------------------------------------------------ worked examples
def test_sigmoid_tree_closed_form():
    (t, v, s), rows = load_tree("sigmoid_tree.txt")
    d = O.decode(t, v, s, 1, 1)
    assert d.status == O.OK
    want_plan = [int(x) for x in rows["plan"][0]]
    assert [d.length, d.max_stack, d.n_const, d.n_modi, d.bucket] == want_plan
    xs = np.array([r[0] for r in rows["value"]])
    vals = np.array([r[1] for r in rows["value"]])
    for ev in (O.eval_stack, O.eval_recursive):
        got = ev(d, xs[None, :], 1)[0]
        np.testing.assert_allclose(got, vals, rtol=1e-15, atol=0)
    # and against the sigmoid written out directly, at many points
    x = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(O.eval_stack(d, x[None, :], 1)[0], 1.0 / (1.0 + np.exp(-x)), rtol=1e-15)


def test_modi_tree_closed_forms():
    (t, v, s), rows = load_tree("modi_tree.txt")
    d = O.decode(t, v, s, 5, 3)
    assert d.status == O.OK
    assert [d.length, d.max_stack, d.n_const, d.n_modi, d.bucket] == [int(x) for x in rows["plan"][0]]
    pts = np.array(rows["point"])
    X = pts[:, :5].T
    want = pts[:, 5:].T
    for ev in (O.eval_stack, O.eval_recursive):
        np.testing.assert_allclose(ev(d, X, 3), want, rtol=1e-15, atol=1e-15)
    # a Modi(o) output index beyond n_out is an encoding error
    assert O.decode(t, v, s, 5, 2).status == O.E_TYPE


def test_modi_outputs_random_points():
    (t, v, s), _ = load_tree("modi_tree.txt")
    d = O.decode(t, v, s, 5, 3)
    X = rng0.uniform(-3, 3, size=(5, 200))
    X[2][np.abs(X[2]) < 1e-3] = 0.5
    a, b, c, dd, e = X
    out = O.eval_stack(d, X, 3)
    np.testing.assert_allclose(out[0], a / c * 0.5, rtol=1e-14)
    np.testing.assert_allclose(out[1], np.maximum(b, c) + (dd - 0.5), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(out[2], e + 0.5, rtol=1e-14, atol=1e-15)


# ------------------------------------------------------------------ operators
def test_operator_special_points():
    x = np.array([-3.0, -0.5, 0.0, 0.25, 7.0])
    np.testing.assert_array_equal(O.apply_op(3, x, x - x), np.ones_like(x))          # protected div
    np.testing.assert_array_equal(O.apply_op(3, x, np.full_like(x, 5e-7)), np.ones_like(x))
    np.testing.assert_allclose(O.apply_op(3, x, np.full_like(x, 2.0)), x / 2.0)
    assert O.apply_op(7, np.array([25.0]))[0] == math.exp(20.0)                       # exp clamp
    assert O.apply_op(7, np.array([-25.0]))[0] == math.exp(-20.0)
    assert O.apply_op(7, np.array([3.0]))[0] == math.exp(3.0)
    assert O.apply_op(8, np.array([0.0]))[0] == math.log(float(np.float32(1e-6)))      # protected log
    assert O.apply_op(8, np.array([-2.0]))[0] == math.log(2.0 + float(np.float32(1e-6)))
    assert np.isnan(O.apply_op(7, np.array([np.nan]))[0])
    assert O.apply_op(9, np.array([np.nan]), np.array([2.0]))[0] == 2.0                # fmax ignores NaN
    assert O.apply_op(10, np.array([1.0]), np.array([np.nan]))[0] == 1.0
    assert O.apply_op(9, np.array([1.5]), np.array([1.5]))[0] == 1.5
    np.testing.assert_allclose(O.apply_op(11, np.array([0.3])), [math.tan(0.3)])
    assert O.TAU == float(np.float32(1e-6)) and O.LOG_EPS == float(np.float32(1e-6))


@pytest.mark.parametrize("op", range(12))
def test_partials_match_finite_differences(op):
    """d f/d operand from the oracle's table vs a central difference of the value function,
    away from kinks (protected-div threshold, exp clamp, log at 0, max/min ties)."""
    r = np.random.default_rng(op)
    a = r.uniform(-3, 3, 400)
    b = r.uniform(-3, 3, 400)
    keep = (np.abs(b) > 0.05) & (np.abs(a) > 0.05) & (np.abs(a - b) > 0.05)
    if op == 11:
        keep &= np.abs(np.cos(a)) > 0.2
    a, b = a[keep], b[keep]
    h = 1e-6
    arity = O.OPS[op][1]
    if arity == 2:
        da, db = O.op_partials(op, a, b)
        fa = (O.apply_op(op, a + h, b) - O.apply_op(op, a - h, b)) / (2 * h)
        fb = (O.apply_op(op, a, b + h) - O.apply_op(op, a, b - h)) / (2 * h)
        np.testing.assert_allclose(da, fa, rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(db, fb, rtol=1e-6, atol=1e-7)
    else:
        da, _ = O.op_partials(op, a)
        fa = (O.apply_op(op, a + h) - O.apply_op(op, a - h)) / (2 * h)
        np.testing.assert_allclose(da, fa, rtol=1e-6, atol=1e-7)


# The conventions at the operators' kinks (the operator table's readings): the value of
# protected division switches to 1 only strictly below tau, the clamped exp keeps its slope
# at exactly +-20, protected log has slope 0 at a = 0 (either sign), and max / min give the
# whole slope to the first operand at a tie (and to the operand returned when the other is NaN).
# Expected values are written out by hand from those readings.
_TAU32 = float(np.float32(1e-6))
_BELOW_TAU = float(np.nextafter(np.float32(1e-6), np.float32(0)))
_ABOVE_20 = float(np.nextafter(np.float32(20.0), np.float32(np.inf)))
KINK_PARTIALS = [
    # op, a, b, d/da, d/db
    (9, 1.5, 1.5, 1.0, 0.0), (9, -2.0, -2.0, 1.0, 0.0), (9, 0.0, -0.0, 1.0, 0.0),
    (9, 1.0, 2.0, 0.0, 1.0), (9, 2.0, 1.0, 1.0, 0.0),
    (9, np.nan, 2.0, 0.0, 1.0), (9, 2.0, np.nan, 1.0, 0.0),
    (10, 1.5, 1.5, 1.0, 0.0), (10, -2.0, -2.0, 1.0, 0.0), (10, -0.0, 0.0, 1.0, 0.0),
    (10, 1.0, 2.0, 1.0, 0.0), (10, 2.0, 1.0, 0.0, 1.0),
    (10, np.nan, 2.0, 0.0, 1.0), (10, 2.0, np.nan, 1.0, 0.0),
    (3, 3.0, _TAU32, 1.0 / _TAU32, -3.0 / (_TAU32 * _TAU32)),
    (3, 3.0, -_TAU32, -1.0 / _TAU32, -3.0 / (_TAU32 * _TAU32)),
    (3, 3.0, _BELOW_TAU, 0.0, 0.0), (3, 3.0, -_BELOW_TAU, 0.0, 0.0),
    (3, 3.0, 0.0, 0.0, 0.0), (3, 3.0, -0.0, 0.0, 0.0),
    (8, 0.0, None, 0.0, None), (8, -0.0, None, 0.0, None),
    (8, 2.0, None, 1.0 / (2.0 + _TAU32), None), (8, -2.0, None, -1.0 / (2.0 + _TAU32), None),
    (7, 20.0, None, math.exp(20.0), None), (7, -20.0, None, math.exp(-20.0), None),
    (7, _ABOVE_20, None, 0.0, None), (7, -_ABOVE_20, None, 0.0, None),
    (7, 25.0, None, 0.0, None), (7, -25.0, None, 0.0, None),
]
KINK_VALUES = [
    # op, a, b, f(a, b)
    (3, 3.0, _TAU32, 3.0 / _TAU32), (3, 3.0, -_TAU32, -3.0 / _TAU32),
    (3, 3.0, _BELOW_TAU, 1.0), (3, 3.0, -_BELOW_TAU, 1.0), (3, -7.0, 0.0, 1.0),
    (7, 20.0, None, math.exp(20.0)), (7, _ABOVE_20, None, math.exp(20.0)), (7, -25.0, None, math.exp(-20.0)),
    (8, 0.0, None, math.log(_TAU32)), (8, -0.0, None, math.log(_TAU32)),
    (9, np.nan, 2.0, 2.0), (10, 2.0, np.nan, 2.0), (9, np.nan, np.nan, np.nan),
]


@pytest.mark.parametrize("op,a,b,da,db", KINK_PARTIALS)
def test_partials_at_kinks(op, a, b, da, db):
    A = np.array([a])
    if b is None:
        got, _ = O.op_partials(op, A)
        assert got[0] == da
    else:
        ga, gb = O.op_partials(op, A, np.array([b]))
        assert ga[0] == da and gb[0] == db


@pytest.mark.parametrize("op,a,b,f", KINK_VALUES)
def test_values_at_kinks(op, a, b, f):
    got = O.apply_op(op, np.array([a])) if b is None else O.apply_op(op, np.array([a]), np.array([b]))
    if np.isnan(f):
        assert np.isnan(got[0])
    else:
        assert got[0] == f


def test_tree_gradient_at_ties_goes_to_first_operand():
    """MAX(c, x0) and MIN(x0, c) with x0 equal to c at some points: at those points the whole
    slope goes to the first operand, written out here as the gradient of the mean square."""
    c = 1.5
    X = np.array([[1.5, 0.5, 1.5, 3.0, 1.5]])
    Y = np.array([[0.25, -1.0, 2.0, 0.0, 1.0]])
    D = X.shape[1]
    for op, first_is_const in ((9, True), (10, False)):
        nodes = [(2, op, 3), (1, c, 1), (0, 0, 1)] if first_is_const else [(2, op, 3), (0, 0, 1), (1, c, 1)]
        t, v, s = _rows(nodes, 8)
        m, gv, gX = O.grad(t[None], v[None], s[None], X, Y)
        x = X[0]
        out = np.maximum(c, x) if op == 9 else np.minimum(x, c)
        r = 2.0 / D * (out - Y[0])
        if op == 9:
            to_c = x <= c          # c is first: ties go to c
        else:
            to_c = x > c           # x0 is first: ties go to x0
        ci = 1 if first_is_const else 2
        assert gv[0, ci] == pytest.approx(float(np.sum(np.where(to_c, r, 0.0))), rel=1e-15, abs=1e-300)
        np.testing.assert_allclose(gX[0], np.where(to_c, 0.0, r), rtol=1e-15, atol=0)


def test_shadow32_matches_float32_arithmetic():
    r = np.random.default_rng(7)
    a = r.uniform(-10, 10, 1000).astype(np.float32)
    b = r.uniform(-10, 10, 1000).astype(np.float32)
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    for op, f in ((0, np.add), (1, np.subtract), (2, np.multiply), (3, np.divide)):
        got = O.apply_op_shadow32(op, a64, b64)
        np.testing.assert_array_equal(got, f(a, b).astype(np.float64))


# ------------------------------------------------------------------ evaluators
def _random_tiny_population(n, seed, modi=True, Lmax=24):
    r = np.random.default_rng(seed)
    T, Vv, S = synth.depth_limited(r, n, r.integers(1, 5, n), r.random(n) < 0.5, synth.F11, 3, Lmax)
    # add tan nodes and Modi tags so every op and every node kind appears
    tan_sites = (T == 2) & (np.isin(Vv, [4, 5])) & (r.random(T.shape) < 0.3)
    Vv[tan_sites] = 11
    if modi:
        synth.trees.assign_modi(r, T, 3, 0.4)
    return T, Vv, S


def test_stack_and_recursive_evaluators_agree_bitwise():
    T, Vv, S = _random_tiny_population(3000, 1)
    X = np.random.default_rng(2).uniform(-4, 4, size=(3, 16)).astype(np.float32)
    n_modi_trees = 0
    for p in range(T.shape[0]):
        d = O.decode(T[p], Vv[p], S[p], 3, 3)
        assert d.status == O.OK
        n_modi_trees += d.n_modi > 0
        a = O.eval_stack(d, X, 3)
        b = O.eval_recursive(d, X, 3)
        assert np.array_equal(a, b, equal_nan=True), p
    assert n_modi_trees > 500


def _to_sympy(d, xs):
    """Independent conversion of a decoded single-output tree to a SymPy expression."""
    tau = sp.Float(O.TAU, 30)
    eps = sp.Float(O.LOG_EPS, 30)

    def rec(i):
        if d.kind[i] == O.T_CONST:
            return sp.Float(d.arg[i], 30), i + 1
        if d.kind[i] == O.T_VAR:
            return xs[d.arg[i]], i + 1
        op = d.arg[i]
        a, j = rec(i + 1)
        if O.OPS[op][1] == 2:
            b, j = rec(j)
        return {
            0: lambda: a + b, 1: lambda: a - b, 2: lambda: a * b,
            3: lambda: sp.Piecewise((sp.Integer(1), sp.Abs(b) < tau), (a / b, True)),
            4: lambda: sp.sin(a), 5: lambda: sp.cos(a), 6: lambda: sp.tanh(a),
            7: lambda: sp.exp(sp.Min(sp.Max(a, -20), 20)), 8: lambda: sp.log(sp.Abs(a) + eps),
            9: lambda: sp.Max(a, b), 10: lambda: sp.Min(a, b), 11: lambda: sp.tan(a),
        }[op](), j

    e, j = rec(0)
    assert j == d.length
    return e


def test_oracle_against_sympy_high_precision():
    T, Vv, S = _random_tiny_population(150, 3, modi=False, Lmax=15)
    xs = sp.symbols("x0:3")
    r = np.random.default_rng(4)
    checked = 0
    for p in range(T.shape[0]):
        d = O.decode(T[p], Vv[p], S[p], 3, 1)
        expr = _to_sympy(d, xs)
        pts = r.uniform(-2, 2, size=(3, 3))
        got = O.eval_stack(d, pts, 1)[0]
        for k in range(3):
            ref = expr.evalf(40, subs={xs[i]: sp.Float(float(pts[i, k]), 40) for i in range(3)})
            if not ref.is_real or not ref.is_finite:
                continue
            ref = float(ref)
            if abs(ref) > 1e8:
                continue
            assert abs(got[k] - ref) <= 1e-9 * max(1.0, abs(ref)), (p, k, got[k], ref)
            checked += 1
    assert checked > 300


# ------------------------------------------------------------------ plan figures and validation
def _rows(nodes, Lmax=12):
    t = np.full(Lmax, np.nan, np.float32)
    v = np.full(Lmax, np.nan, np.float32)
    s = np.full(Lmax, np.nan, np.float32)
    for i, (a, b, c) in enumerate(nodes):
        t[i], v[i], s[i] = a, b, c
    return t, v, s


LEFT_COMB = [(2, 0, 7), (2, 0, 5), (2, 0, 3), (0, 0, 1), (0, 1, 1), (0, 0, 1), (0, 1, 1)]   # ((x+y)+x)+y
RIGHT_COMB = [(2, 0, 7), (0, 0, 1), (2, 0, 5), (0, 1, 1), (2, 0, 3), (0, 0, 1), (0, 1, 1)]  # x+(y+(x+y))


def test_max_stack_extremes():
    d = O.decode(*_rows(LEFT_COMB), 2, 1)
    assert (d.status, d.length, d.max_stack, d.bucket) == (0, 7, 4, 3)   # (len+1)/2 for a left comb
    d = O.decode(*_rows(RIGHT_COMB), 2, 1)
    assert (d.status, d.length, d.max_stack) == (0, 7, 2)
    assert [O.length_bucket(n) for n in (1, 2, 3, 4, 5, 8, 9, 512, 513, 1024)] == [0, 1, 2, 2, 3, 3, 4, 9, 10, 10]


def test_max_stack_leaf_formula():
    """Max stack depth equals the largest, over leaves l, of 1 + sum over ancestors a of
    (arity(a) - j_a), with l inside child j_a (1-based) of a."""
    T, Vv, S = _random_tiny_population(400, 9, modi=False, Lmax=40)
    for p in range(T.shape[0]):
        d = O.decode(T[p], Vv[p], S[p], 3, 1)
        best = 0
        stack = [(0, 0)]  # (node, accumulated)
        while stack:
            i, acc = stack.pop()
            if d.kind[i] != O.T_FUNC:
                best = max(best, 1 + acc)
                continue
            ar = O.OPS[d.arg[i]][1]
            c = i + 1
            for j in range(1, ar + 1):
                stack.append((c, acc + ar - j))
                c += d.size[c]
        assert best == d.max_stack


def test_validator_fault_list():
    t, v, s = _rows(RIGHT_COMB)
    ok = O.decode(t, v, s, 2, 1)
    assert ok.status == O.OK

    def code(mut, V=2, n_out=1):
        tt, vv, ss = t.copy(), v.copy(), s.copy()
        mut(tt, vv, ss)
        return O.decode(tt, vv, ss, V, n_out).status

    assert code(lambda a, b, c: c.__setitem__(0, 13.0)) == O.E_LEN        # size[0] > Lmax
    assert code(lambda a, b, c: c.__setitem__(0, 6.5)) == O.E_LEN         # non-integer len
    assert code(lambda a, b, c: c.__setitem__(0, np.nan)) == O.E_LEN
    assert code(lambda a, b, c: b.__setitem__(3, np.nan)) == O.E_NAN       # NaN inside len
    assert code(lambda a, b, c: a.__setitem__(9, 0.0)) == O.E_TAIL        # non-NaN after len
    assert code(lambda a, b, c: a.__setitem__(2, 2.5)) == O.E_TYPE        # non-integer type
    assert code(lambda a, b, c: a.__setitem__(2, 4.0)) == O.E_TYPE        # Modi(1) with n_out = 1
    assert code(lambda a, b, c: a.__setitem__(2, 4.0), n_out=2) == O.OK
    assert code(lambda a, b, c: b.__setitem__(2, 12.0)) == O.E_OP         # unknown op id
    assert code(lambda a, b, c: b.__setitem__(3, 2.0)) == O.E_VAR         # var index >= V
    assert code(lambda a, b, c: b.__setitem__(3, 0.5)) == O.E_VAR
    assert code(lambda a, b, c: c.__setitem__(4, 2.0)) == O.E_SIZE        # size invariant broken
    assert code(lambda a, b, c: c.__setitem__(1, 1.5)) == O.E_SIZE
    assert code(lambda a, b, c: b.__setitem__(2, 4.0)) == O.E_SIZE        # binary -> unary: structure breaks
    # smallest code wins when several faults are present
    assert code(lambda a, b, c: (b.__setitem__(3, np.nan), a.__setitem__(10, 1.0))) == O.E_NAN
    assert code(lambda a, b, c: (b.__setitem__(3, 7.0), b.__setitem__(2, 20.0))) == O.E_OP


def test_plan_figures_vs_generator_counts():
    w = synth.workload("hybrid", P=300, D=10)
    pl = O.plan(w.type, w.value, w.size, w.V, 1)
    assert (pl[:, 0] == 0).all()
    np.testing.assert_array_equal(pl[:, 1], w.lengths())
    np.testing.assert_array_equal(pl[:, 3], (w.type == 1).sum(1))
    assert (pl[:, 4] == 0).all()


# ------------------------------------------------------------------ fitness closed forms
def _poly_tree():
    # ADD(MUL(x, MUL(x, x)), ADD(MUL(x, x), x)) = x^3 + x^2 + x
    nodes = [(2, 0, 11), (2, 2, 5), (0, 0, 1), (2, 2, 3), (0, 0, 1), (0, 0, 1),
             (2, 0, 5), (2, 2, 3), (0, 0, 1), (0, 0, 1), (0, 0, 1)]
    return _rows(nodes, 16)


def test_mse_closed_forms_on_plain_workload():
    w = synth.workload("plain")
    x = w.X[0].astype(np.float64)
    y = w.Y[0].astype(np.float64)
    t, v, s = _poly_tree()
    m = O.mse(t[None], v[None], s[None], w.X, w.Y)[0]
    assert m == pytest.approx(np.mean((y - (x ** 3 + x ** 2 + x)) ** 2), rel=1e-12)
    assert m == pytest.approx(np.mean(w.noise.astype(np.float64) ** 2), rel=1e-3)
    c = np.float32(1.25)
    m = O.mse(*(a[None] for a in _rows([(1, c, 1)], 16)), w.X, w.Y)[0]
    assert m == pytest.approx(np.mean((float(c) - y) ** 2), rel=1e-12)
    m = O.mse(*(a[None] for a in _rows([(0, 0, 1)], 16)), w.X, w.Y)[0]
    assert m == pytest.approx(np.mean((x - y) ** 2), rel=1e-12)


def test_multi_output_mse_sums_outputs():
    (t, v, s), _ = load_tree("modi_tree.txt")
    X = rng0.uniform(-2, 2, size=(5, 50))
    X[2] = np.where(np.abs(X[2]) < 0.1, 0.7, X[2])
    Y = rng0.normal(size=(3, 50))
    a, b, c, d, e = X
    outs = np.stack([a / c * 0.5, np.maximum(b, c) + (d - 0.5), e + 0.5])
    m = O.mse(t[None], v[None], s[None], X, Y, n_out=3)[0]
    assert m == pytest.approx(np.sum(np.mean((outs - Y) ** 2, axis=1)), rel=1e-12)
    # a plain tree in a 3-output problem predicts (root, 0, 0)
    tt, vv, ss = _rows([(0, 4, 1)], 16)
    m = O.mse(tt[None], vv[None], ss[None], X, Y, n_out=3)[0]
    want = np.mean((e - Y[0]) ** 2) + np.mean(Y[1] ** 2) + np.mean(Y[2] ** 2)
    assert m == pytest.approx(want, rel=1e-12)


# ------------------------------------------------------------------ gradients
def test_gradient_closed_form_mul_const_var():
    t, v, s = _rows([(2, 2, 3), (1, 1.75, 1), (0, 0, 1)], 8)    # MUL(c, x0)
    X = rng0.normal(size=(1, 64))
    Y = rng0.normal(size=(1, 64))
    m, gv, gX = O.grad(t[None], v[None], s[None], X, Y)
    c = 1.75
    x, y = X[0], Y[0]
    D = 64
    assert gv[0, 1] == pytest.approx(2.0 / D * np.sum((c * x - y) * x), rel=1e-13)
    np.testing.assert_allclose(gX[0], 2.0 / D * (c * x - y) * c, rtol=1e-13)
    assert gv[0, 0] == 0 and gv[0, 2] == 0


def test_gradient_vs_central_differences():
    w = synth.workload("grad", P=60, D=40)
    hp = O.predict(*w.hidden, w.X, 1)[:, 0, :]
    Y = w.targets_from(hp)
    m, gv, gX = O.grad(w.type, w.value, w.size, w.X, Y)
    checked = 0
    for p in range(w.P):
        if not (np.isfinite(m[p]) and m[p] < 1e4):
            continue                                           # FD in float64 cancels badly on huge fitness values
        d = O.decode(w.type[p], w.value[p], w.size[p], w.V, 1)
        for i in range(d.length):
            if d.kind[i] != O.T_CONST:
                continue
            f1 = O.fd_grad_const(w.type, w.value, w.size, w.X, Y, p, i, h=1e-5)
            f2 = O.fd_grad_const(w.type, w.value, w.size, w.X, Y, p, i, h=5e-6)
            if abs(f1 - f2) > 1e-3 * max(1.0, abs(f1)):      # kink-adjacent: skip
                continue
            fr = (4.0 * f2 - f1) / 3.0                        # Richardson: O(h^4) truncation
            assert gv[p, i] == pytest.approx(fr, rel=1e-6, abs=1e-6), (p, i)
            checked += 1
    assert checked > 30
    rows = [p for p in range(w.P) if np.isfinite(m[p]) and m[p] < 1e4]
    m2, gv2, gX = O.grad(w.type, w.value, w.size, w.X, Y, rows=rows)
    for v_, j in [(0, 3), (2, 17), (5, 30), (7, 1)]:
        f = O.fd_grad_x(w.type, w.value, w.size, w.X, Y, rows, v_, j, h=1e-5)
        assert gX[v_, j] == pytest.approx(f, rel=1e-4, abs=1e-6)


def test_modi_gradient_vs_central_differences():
    (t, v, s), _ = load_tree("modi_tree.txt")
    r = np.random.default_rng(3)
    X = r.uniform(-2, 2, size=(5, 30))
    X[2] = np.where(np.abs(X[2]) < 0.2, 0.9, X[2])
    Y = r.normal(size=(3, 30))
    m, gv, gX = O.grad(t[None], v[None], s[None], X, Y, n_out=3)
    f = O.fd_grad_const(t[None], v[None], s[None], X, Y, 0, 12, h=1e-6, n_out=3)
    assert gv[0, 12] == pytest.approx(f, rel=1e-6)
    for vv_, j in [(0, 0), (1, 5), (2, 9), (3, 11), (4, 29)]:
        f = O.fd_grad_x(t[None], v[None], s[None], X, Y, [0], vv_, j, h=1e-6, n_out=3)
        assert gX[vv_, j] == pytest.approx(f, rel=1e-5, abs=1e-9)


def test_gradient_shadow_exact_on_representable_values():
    # MUL(ADD(x0, 0.5), x1) on small integers: every value, partial and product
    # is exact in float32, so the float32 shadow equals the float64 sweep.
    t, v, s = _rows([(2, 2, 5), (2, 0, 3), (0, 0, 1), (1, 0.5, 1), (0, 1, 1)], 8)
    X = np.array([[1.0, -2.0, 3.0, 0.0], [2.0, 1.0, -1.0, 4.0]])
    Y = np.array([[1.0, 2.0, -3.0, 0.5]])
    g64 = O.grad(t[None], v[None], s[None], X, Y)
    g32 = O.grad(t[None], v[None], s[None], X, Y, shadow=True)
    for a, b in zip(g64, g32):
        np.testing.assert_array_equal(a, b)
    # closed form: d/dc mean((x0 + c) x1 - y)^2 = 2/D sum(((x0 + c) x1 - y) x1)
    r = (X[0] + 0.5) * X[1] - Y[0]
    assert g32[1][0, 3] == 2.0 / 4 * np.sum(r * X[1])


def test_gradient_shadow_singular_quotient():
    # COS(DIV(c, x0)) at x0 just above the protection threshold: the quotient is
    # about 6e5, where one float32 ulp (1/16) moves cos noticeably. The shadow
    # gradient follows float32 arithmetic written out here; the float64 one
    # differs, which is what marks such components as ill-conditioned.
    c, x, y = 1.7, 2.9e-6, 0.25
    t, v, s = _rows([(2, 5, 4), (2, 3, 3), (1, c, 1), (0, 0, 1)], 8)
    X = np.array([[x]], dtype=np.float32)
    Y = np.array([[y]], dtype=np.float32)
    _, gv32, _ = O.grad(t[None], v[None], s[None], X, Y, shadow=True)
    _, gv64, _ = O.grad(t[None], v[None], s[None], X, Y)
    f = np.float32
    c32, x32 = f(c), f(x)
    q = f(c32 / x32)
    e = f(f(np.cos(np.float64(q))) - f(y))
    gout = f(f(f(2.0) * e) * f(1.0))
    d_cos = f(-np.sin(np.float64(q)))
    d_div = f(1.0 / np.float64(x32))
    want = f(f(gout * d_cos) * d_div)
    assert gv32[0, 2] == pytest.approx(float(want), rel=1e-6)
    qe = c32 / np.float64(x32)
    want64 = 2.0 * (np.cos(qe) - y) * -np.sin(qe) / np.float64(x32)
    assert gv64[0, 2] == pytest.approx(want64, rel=1e-12)
    assert abs(gv32[0, 2] - gv64[0, 2]) > 1e-3 * abs(gv64[0, 2])


def test_gradient_shadow_close_on_random_trees():
    # no dropped or misplaced term in the shadow sweep: on a random population
    # most constant components agree with float64 to 1e-4
    w = synth.workload("grad", P=200, D=64)
    Y = w.targets_from(O.predict(*w.hidden, w.X, 1)[:, 0, :])
    m, gv, _ = O.grad(w.type, w.value, w.size, w.X, Y)
    _, gs, _ = O.grad(w.type, w.value, w.size, w.X, Y, shadow=True)
    const = (w.type == O.T_CONST) & np.isfinite(m)[:, None] & np.isfinite(gv) & (np.abs(gv) > 1e-6)
    close = np.abs(gs - gv) <= 1e-4 * np.abs(gv)
    assert const.sum() > 100
    assert close[const].mean() > 0.9


def test_shadow_ulp_perturbation():
    # SIN(x0): the perturbed shadow moves each point by an integer number of
    # float32 ulps in [-2, 2], each step count occurring; without
    # transcendental nodes nothing moves
    t, v, s = _rows([(2, 4, 2), (0, 0, 1)], 8)
    d = O.decode(t, v, s, 1, 1)
    X = rng0.uniform(-3, 3, size=(1, 4000))
    base = O.eval_shadow32(d, X, 1)[0].astype(np.float32)
    pert = O.eval_shadow32(d, X, 1, ulps=O.Ulps(2, 7))[0].astype(np.float32)
    steps = np.zeros(base.shape, np.int64)
    for k in (1, 2):
        up, dn = base.copy(), base.copy()
        for _ in range(k):
            up = np.nextafter(up, np.float32(np.inf))
            dn = np.nextafter(dn, np.float32(-np.inf))
        steps[pert == up] = k
        steps[pert == dn] = -k
    moved = pert != base
    assert np.all(moved == (steps != 0))
    assert set(np.unique(steps).tolist()) == {-2, -1, 0, 1, 2}
    assert 0.7 < moved.mean() < 0.9
    # + - * / only: identical
    t, v, s = _rows([(2, 3, 5), (2, 0, 3), (0, 0, 1), (1, 0.5, 1), (0, 0, 1)], 8)
    d = O.decode(t, v, s, 1, 1)
    np.testing.assert_array_equal(O.eval_shadow32(d, X, 1), O.eval_shadow32(d, X, 1, ulps=O.Ulps(2, 3)))
    # fitness: ulp=0 is the plain shadow
    w = synth.workload("hybrid", P=30, D=64)
    Y = w.targets_from(O.predict(*w.hidden, w.X, 1)[:, 0, :])
    np.testing.assert_array_equal(O.mse_shadow32(w.type, w.value, w.size, w.X, Y),
                                  O.mse_shadow32(w.type, w.value, w.size, w.X, Y, ulp=0, seed=5))


def test_adam_reference_matches_torch():
    torch = pytest.importorskip("torch")
    A = np.diag([1.0, 3.0, 0.5])
    b = np.array([1.0, -2.0, 0.3])
    theta0 = np.array([0.5, 0.5, -1.0])
    ours = O.adam_reference(theta0, lambda th: A @ th - b, 10, lr=1e-2)
    p = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-2)
    At, bt = torch.tensor(A), torch.tensor(b)
    for _ in range(10):
        opt.zero_grad()
        p.grad = At @ p.detach() - bt
        opt.step()
    np.testing.assert_allclose(ours, p.detach().numpy(), rtol=1e-12, atol=1e-14)
