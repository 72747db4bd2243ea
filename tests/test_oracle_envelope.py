"""Pins of the float32 envelopes (oracle/envelope.py) against things other than
themselves:

* the float32 shadow (every operation correctly rounded) and shadows whose
  transcendental results move by up to 3 float32 ulp (still inside the
  model's 4 ulp of the exact value);
* a third evaluator written here in numpy float32 arithmetic, with numpy's own
  float32 math library (measured below within 4 ulp of the exact functions)
  and float32 sums grouped as a wavefront reduction groups them;
* closed cases: library-free trees are points equal to the shadow, and the
  envelope takes both branches of a protected division whose denominator may
  cross the threshold, and the whole line near a pole of tan.
"""

import numpy as np
import pytest

import oracle as O
from oracle import envelope as E
import synth

f32 = np.float32


def _work(name, **kw):
    w = synth.workload(name, **kw)
    Y = w.Y if w.Y is not None else w.targets_from(O.predict(*w.hidden, w.X, 1)[:, 0, :])
    return w, np.asarray(Y, np.float64).reshape(w.n_out, w.D)


def _inside(v, lo, hi, nan):
    v = np.asarray(v, np.float64)
    with np.errstate(invalid="ignore"):
        return np.where(np.isnan(v), nan, (lo <= v) & (v <= hi))


# ------------------------------------------------------------------ a float32 evaluator of its own
def _np32_op(op, a, b=None):
    """The operator table in numpy float32 arithmetic with numpy's float32 math library."""
    with np.errstate(all="ignore"):
        if op == 0:
            return a + b
        if op == 1:
            return a - b
        if op == 2:
            return a * b
        if op == 3:
            return np.where(np.abs(b) < f32(1e-6), f32(1.0), a / b).astype(f32)
        if op == 4:
            return np.sin(a)
        if op == 5:
            return np.cos(a)
        if op == 6:
            return np.tanh(a)
        if op == 7:
            return np.exp(np.minimum(np.maximum(a, f32(-20.0)), f32(20.0)))
        if op == 8:
            return np.log(np.abs(a) + f32(1e-6))
        if op == 9:
            return np.fmax(a, b)
        if op == 10:
            return np.fmin(a, b)
        return np.tan(a)


def _np32_outputs(d, X, n_out):
    """Outputs in float32 by recursion over subtree sizes (not a stack): Modi contributions
    added in decreasing node index (the reverse of the shadow's order)."""
    X = np.asarray(X, f32)
    D = X.shape[1]
    contrib = []

    def val(i):
        if d.kind[i] == O.T_CONST:
            return np.full(D, f32(d.arg[i]), f32)
        if d.kind[i] == O.T_VAR:
            return X[d.arg[i]]
        op = d.arg[i]
        a = val(i + 1)
        if O.OPS[op][1] == 2:
            b = val(i + 1 + d.size[i + 1])
            r, right = _np32_op(op, a, b), b
        else:
            r, right = _np32_op(op, a), a
        if d.out[i] >= 0:
            contrib.append((i, d.out[i], r))
            return right
        return r

    root = val(0)
    out = np.zeros((n_out, D), f32)
    if d.n_modi == 0:
        out[0] = root
    else:
        for _, o, r in sorted(contrib, reverse=True):
            out[o] = out[o] + r
    return out


def _wave_sum32(terms, k):
    """Float32 sum grouped as a wavefront reduction: k terms per lane in order, a pairwise tree
    over 64 lanes, then the tiles in order (the grouping the envelope's sum bound describes)."""
    t = np.asarray(terms, f32)
    tile = 64 * k
    n = -(-t.size // tile) * tile
    t = np.concatenate([t, np.zeros(n - t.size, f32)]).reshape(-1, k, 64)   # [tile][j][lane]
    lane = t[:, 0, :]
    for j in range(1, k):
        lane = lane + t[:, j, :]
    while lane.shape[1] > 1:
        lane = lane[:, 0::2] + lane[:, 1::2]
    acc = f32(0.0)
    for v in lane[:, 0]:
        acc = f32(acc + v)
    return float(acc)


def _np32_fitness(d, X, Y, n_out, k=8):
    out = _np32_outputs(d, X, n_out)
    e = out - np.asarray(Y, f32)
    with np.errstate(all="ignore"):
        sq = (e * e).astype(f32)
    s = sum(_wave_sum32(sq[o], k) for o in range(n_out))
    return float(f32(s / X.shape[1]))


def test_numpy_float32_library_within_model():
    """numpy's float32 transcendentals are a library of the kind the model assumes (within
    LIB_ULP ulp of the exact function), so the evaluator above is a valid float32 evaluation."""
    r = np.random.default_rng(0)
    x = np.concatenate([r.uniform(-30, 30, 200_000), np.exp(r.uniform(-15, 15, 100_000)) * r.choice([-1, 1], 100_000)])
    x = x.astype(f32)
    for f, dom in ((np.sin, None), (np.cos, None), (np.tanh, None), (np.exp, (-20, 20)), (np.log, "pos"), (np.tan, None)):
        xx = np.abs(x) + f32(1e-6) if dom == "pos" else (np.clip(x, *dom).astype(f32) if dom else x)
        with np.errstate(all="ignore"):
            got = f(xx).astype(np.float64)
            ref = f(xx.astype(np.float64))
        ok = np.isfinite(ref)
        a = np.abs(ref[ok]).astype(f32)
        ulp = np.nextafter(a, f32(np.inf)).astype(np.float64) - a.astype(np.float64)
        assert np.max(np.abs(got[ok] - ref[ok]) / ulp) <= E.LIB_ULP


# ------------------------------------------------------------------ fitness envelopes
CASES = [("plain", {}), ("hybrid", dict(P=300, D=2000)), ("grad", dict(P=150, D=3100)),
         ("batched", dict(P=200, D=1000)), ("pagie", dict(P=200, D=2000)), ("dataparallel", dict(P=30, D=20000))]


@pytest.mark.parametrize("name,kw", CASES)
def test_fitness_envelope_holds_float32_evaluations(name, kw):
    w, Y = _work(name, **kw)
    lo, hi, nan = E.fitness(w.type, w.value, w.size, w.X, Y, w.n_out)
    m64 = O.mse(w.type, w.value, w.size, w.X, Y, w.n_out)
    fin = np.isfinite(m64)
    for ulp, seed in ((0, 0), (3, 1), (3, 2)):
        s = O.mse_shadow32(w.type, w.value, w.size, w.X, Y, w.n_out, ulp=ulp, seed=seed)
        assert _inside(s, lo, hi, nan).all(), ("shadow outside", ulp, seed)
    V = w.V
    n32 = np.array([_np32_fitness(O.decode(w.type[p], w.value[p], w.size[p], V, w.n_out), w.X, Y, w.n_out)
                    for p in range(w.P)])
    bad = ~_inside(n32, lo, hi, nan)
    assert not bad.any(), ("numpy float32 evaluation outside", np.nonzero(bad)[0][:5])
    # the envelope is narrow for most trees: within the fitness tolerance of the float64 value
    tol = np.maximum(1e-5 * np.abs(m64), 1e-6)
    with np.errstate(invalid="ignore"):
        tight = fin & ~nan & (lo >= m64 - tol) & (hi <= m64 + tol)
    assert tight.mean() >= 0.5, tight.mean()


def test_library_free_trees_are_points():
    """+ - * / max min over float32 leaves: every correctly rounded evaluation gives the
    shadow's bits, so the outputs are points equal to the shadow's."""
    w, Y = _work("plain")        # the plain workload uses + - * / only
    for p in range(w.P):
        d = O.decode(w.type[p], w.value[p], w.size[p], 1, 1)
        outs, _ = E.forward(d, w.X, 1)
        sh = O.eval_shadow32(d, w.X, 1)[0]
        assert outs[0].pt.all()
        np.testing.assert_array_equal(outs[0].lo, sh)


def _tree(nodes, Lmax=8):
    t, v, s = (np.full((1, Lmax), np.nan, f32) for _ in range(3))
    for i, (a, b, c) in enumerate(nodes):
        t[0, i], v[0, i], s[0, i] = a, b, c
    return t, v, s


def test_division_branch_may_flip():
    """DIV(1, SUB(EXP(x0), c)) with exp(x0) - c within a few ulp of tau: the library's exp may
    land on either side, so the envelope holds both 1 and the quotient."""
    x = f32(0.5)
    c = f32(np.exp(np.float64(x)) - 1e-6)          # exp(x) - c is about tau
    t, v, s = _tree([(2, 3, 6), (1, 1.0, 1), (2, 1, 4), (2, 7, 2), (0, 0, 1), (1, float(c), 1)])
    d = O.decode(t[0], v[0], s[0], 1, 1)
    outs, _ = E.forward(d, np.array([[x]]), 1)
    lo, hi = outs[0].lo[0], outs[0].hi[0]
    assert lo <= 1.0 <= hi
    assert hi > 1e5                                 # the quotient 1 / (about tau) is also possible


def test_tan_near_pole_is_unbounded():
    """TAN(LOG(x0)) where log(|x0| + eps) is within the library's error of pi/2."""
    t, v, s = _tree([(2, 11, 3), (2, 8, 2), (0, 0, 1)])
    d = O.decode(t[0], v[0], s[0], 1, 1)
    x = f32(np.exp(np.pi / 2) - 1e-6)
    outs, _ = E.forward(d, np.array([[x]]), 1)
    assert outs[0].lo[0] == -np.inf and outs[0].hi[0] == np.inf
    assert not outs[0].pt[0]
    # away from the pole the envelope is narrow
    outs, _ = E.forward(d, np.array([[f32(2.0)]]), 1)
    assert outs[0].hi[0] - outs[0].lo[0] < 1e-5 * abs(np.tan(np.log(2.0)))


# ------------------------------------------------------------------ gradient envelopes
@pytest.mark.parametrize("name,kw", [("plain", {}), ("hybrid", dict(P=120, D=2000)), ("grad", dict(P=120, D=3100)),
                                     ("pagie", dict(P=120, D=2000)), ("batched", dict(P=60, D=700))])
def test_gradient_envelope_holds_float32_evaluations(name, kw):
    w, Y = _work(name, **kw)
    ks = (2, 3, 4)
    glo, ghi, gnan, xlo, xhi, xnan = E.grad(w.type, w.value, w.size, w.X, Y, w.n_out, lanes_k=ks)
    const = w.type == O.T_CONST
    for ulp, seed in ((0, 0), (3, 1), (3, 2)):
        _, gvs, gxs = O.grad(w.type, w.value, w.size, w.X, Y, w.n_out, shadow=True, ulp=ulp, seed=seed)
        assert _inside(gvs, glo, ghi, gnan)[const].all(), ("shadow constant gradient outside", ulp)
        assert _inside(gxs, xlo, xhi, xnan).all(), ("shadow X gradient outside", ulp)
    # the shadow's per-point adjoints summed in float32 as a wavefront reduction groups them
    # (the envelope's sum bound) stay inside too
    checked = 0
    for p in range(min(w.P, 40)):
        d = O.decode(w.type[p], w.value[p], w.size[p], w.V, w.n_out)
        for j in np.nonzero(const[p])[0][:2]:
            lam = _const_adjoint_shadow(w, Y, p, j)
            for k in ks:
                g32 = _wave_sum32(lam, k)
                assert _inside(g32, glo[p, j], ghi[p, j], gnan[p, j]), (p, j, k, g32, glo[p, j], ghi[p, j])
            checked += 1
        del d
    assert checked > 10


def test_gradient_envelope_over_several_lane_widths_is_the_widest():
    """With several points-per-lane values the sum bound is the longest of their addition chains:
    at 256 points four per lane make the longest chain (3 + 6 + 1 against 1 + 6 + 2 at two), at
    4,096 two per lane do."""
    for D, widest in ((256, 4), (4096, 2)):
        w, Y = _work("grad", P=8, D=D)
        one = {k: E.grad(w.type, w.value, w.size, w.X, Y, w.n_out, lanes_k=k) for k in (2, 3, 4)}
        many = E.grad(w.type, w.value, w.size, w.X, Y, w.n_out, lanes_k=(2, 3, 4))
        const = w.type == O.T_CONST
        for k in (2, 3, 4):
            assert (many[0][const] <= one[k][0][const]).all() and (many[1][const] >= one[k][1][const]).all()
        assert np.array_equal(many[0][const], one[widest][0][const])
        assert np.array_equal(many[1][const], one[widest][1][const])


def _const_adjoint_shadow(w, Y, p, j):
    """Per-point shadow adjoint of constant j of tree p: the tree with node j read from an extra
    variable holding the constant; that variable's shadow X gradient is the adjoint."""
    t, v = w.type[p:p + 1].copy(), w.value[p:p + 1].copy()
    c = v[0, j]
    t[0, j], v[0, j] = 0, w.V
    X2 = np.concatenate([w.X, np.full((1, w.D), c, f32)])
    _, _, gx = O.grad(t, v, w.size[p:p + 1], X2, Y, w.n_out, shadow=True)
    return gx[w.V]


def test_gradient_kinks_widen_to_both_sides():
    """MAX(x0, EXP(LOG(x0))): the second operand is x0 + eps (about 4 ulp above x0 at 2 and 3)
    up to the library's errors, so a float32 evaluation may pick either operand; the slope's
    envelope spans both assignments and holds the float64 gradient."""
    t, v, s = _tree([(2, 9, 5), (0, 0, 1), (2, 7, 3), (2, 8, 2), (0, 0, 1)])
    X = np.array([[f32(2.0), f32(3.0)]])
    Y = np.zeros((1, 2))
    d = O.decode(t[0], v[0], s[0], 1, 1)
    assert d.status == O.OK
    _, _, _, xlo, xhi, _ = E.grad(t, v, s, X, Y)
    _, _, gx = O.grad(t, v, s, X, Y)
    assert (xlo <= gx).all() and (gx <= xhi).all()
    pa, pb = E.iv_partials(9, *E.forward(d, X, 1, keep=True)[1][1:3])
    assert (pa.lo == 0).all() and (pa.hi == 1).all() and (pb.lo == 0).all() and (pb.hi == 1).all()


# ------------------------------------------------------------------ one operator at a time
def _f32_op_values(op, a, b):
    """Float32 results of op on float32 operands in two ways: correctly rounded (the exact value
    rounded once) and numpy's float32 arithmetic and library."""
    a32 = a.astype(f32)
    b32 = b.astype(f32) if b is not None else None
    exact = O.apply_op(op, a32.astype(np.float64), None if b is None else b32.astype(np.float64))
    return [exact.astype(f32).astype(np.float64), _np32_op(op, a32, b32).astype(np.float64)]


def _random_boxes(r, n, center_scale):
    c = r.normal(size=n) * center_scale
    w = np.abs(c) * 10.0 ** r.uniform(-7, -1, n) + 10.0 ** r.uniform(-9, -3, n)
    return (c - w).astype(f32).astype(np.float64), (c + w).astype(f32).astype(np.float64)


@pytest.mark.parametrize("op", range(12))
def test_operator_intervals_sound_and_tight(op):
    """For random operand intervals (and intervals around each kink), every float32 result of
    the operator at sampled operands lies inside the computed interval, and the interval is no
    wider than the sampled exact range plus the rounding widening (and 1% of its width)."""
    r = np.random.default_rng(100 + op)
    n = 300
    scale = 3.0 if op != 7 else 15.0
    alo, ahi = _random_boxes(r, n, scale)
    blo, bhi = _random_boxes(r, n, scale)
    if op == 3:                       # denominators around the threshold
        blo[:60], bhi[:60] = (0.9e-6, 1.1e-6) if True else (0, 0)
    if op in (9, 10):                 # overlapping operands (ties)
        blo[:60], bhi[:60] = alo[:60], ahi[:60]
    binary = O.OPS[op][1] == 2
    A = E.Iv(alo, ahi, np.zeros(n, bool), alo == ahi)
    B = E.Iv(blo, bhi, np.zeros(n, bool), blo == bhi) if binary else None
    iv = E.iv_op(op, A, B) if binary else E.iv_op(op, A)
    t = np.linspace(0.0, 1.0, 41)
    ex_min = np.full(n, np.inf)
    ex_max = np.full(n, -np.inf)
    for ta in t:
        a = alo + ta * (ahi - alo)
        for tb in (t if binary else [0.0]):
            b = blo + tb * (bhi - blo) if binary else None
            for v in _f32_op_values(op, a, b):
                assert E._contains(iv.lo, iv.hi, v)[np.isfinite(v)].all(), (op, ta, tb)
            ex = O.apply_op(op, a.astype(f32).astype(np.float64),
                            None if b is None else b.astype(f32).astype(np.float64))
            ex_min = np.fmin(ex_min, ex)
            ex_max = np.fmax(ex_max, ex)
    fin = np.isfinite(iv.lo) & np.isfinite(iv.hi) & np.isfinite(ex_min) & np.isfinite(ex_max)
    width = iv.hi - iv.lo
    slack = 2.0 * (2 * E.LIB_ULP * E.U) * np.maximum(np.abs(ex_min), np.abs(ex_max)) + 1e-300 + 0.01 * width
    if op == 8:
        slack += 4.0 * E.U          # the rounding of |a| + eps moves log by about u absolute
    assert (iv.lo[fin] >= ex_min[fin] - slack[fin]).all(), op
    assert (iv.hi[fin] <= ex_max[fin] + slack[fin]).all(), op


def _np32_partials(op, a, b):
    """Float32 partial derivatives as a float32 implementation of the oracle's table forms them."""
    one, zero = f32(1.0), f32(0.0)
    with np.errstate(all="ignore"):
        if op in (0, 1):
            return np.full_like(a, one), np.full_like(a, one if op == 0 else f32(-1.0))
        if op == 2:
            return b, a
        if op == 3:
            small = np.abs(b) < f32(1e-6)
            rr = (one / b).astype(f32)
            return np.where(small, zero, rr).astype(f32), np.where(small, zero, (-a * rr * rr).astype(f32)).astype(f32)
        if op == 9:
            pa = (a >= b) | np.isnan(b)
            return np.where(pa, one, zero), np.where(pa, zero, one)
        if op == 10:
            pa = (a <= b) | np.isnan(b)
            return np.where(pa, one, zero), np.where(pa, zero, one)
        if op == 4:
            return np.cos(a), None
        if op == 5:
            return -np.sin(a), None
        if op == 6:
            th = np.tanh(a)
            return (one - th * th).astype(f32), None
        if op == 7:
            return np.where((a >= f32(-20)) & (a <= f32(20)), np.exp(a), zero).astype(f32), None
        if op == 8:
            return np.where(a == zero, zero, (np.copysign(one, a) / (np.abs(a) + f32(1e-6))).astype(f32)), None
        tn = np.tan(a)
        return (one + tn * tn).astype(f32), None


@pytest.mark.parametrize("op", range(12))
def test_partial_intervals_hold_float32_partials(op):
    """Float32 partials at sampled operands (numpy's float32 arithmetic and library) lie inside
    the partial-derivative intervals, for exact operands and for operand intervals."""
    r = np.random.default_rng(200 + op)
    n = 400
    scale = 2.0 if op != 7 else 12.0
    alo, ahi = _random_boxes(r, n, scale)
    blo, bhi = _random_boxes(r, n, scale)
    # points (half of them) and tiny values, where roundings of 1 - x dominate
    alo[:200] = ahi[:200]
    blo[:200] = bhi[:200]
    alo[:40] = ahi[:40] = (r.normal(size=40) * 1e-4).astype(f32)
    binary = O.OPS[op][1] == 2
    A = E.Iv(alo, ahi, np.zeros(n, bool), alo == ahi)
    B = E.Iv(blo, bhi, np.zeros(n, bool), blo == bhi)
    pa, pb = E.iv_partials(op, A, B) if binary else E.iv_partials(op, A)
    for ta in np.linspace(0, 1, 9):
        a = (alo + ta * (ahi - alo)).astype(f32)
        for tb in (np.linspace(0, 1, 9) if binary else [0.0]):
            b = (blo + tb * (bhi - blo)).astype(f32)
            da, db = _np32_partials(op, a, b)
            ok = E._contains(pa.lo, pa.hi, da.astype(np.float64)) | ~np.isfinite(da)
            assert ok.all(), (op, np.nonzero(~ok)[0][:3], a[~ok][:3], da[~ok][:3], pa.lo[~ok][:3], pa.hi[~ok][:3])
            if binary:
                ok = E._contains(pb.lo, pb.hi, db.astype(np.float64)) | ~np.isfinite(db)
                assert ok.all(), (op, np.nonzero(~ok)[0][:3])


@pytest.mark.parametrize("name,kw", [("batched", dict(P=120, D=600)), ("pagie", dict(P=150, D=800)),
                                     ("hybrid", dict(P=150, D=800))])
def test_output_envelopes_hold_float32_outputs(name, kw):
    """Per point and output (multi-output trees included): the shadow's outputs and the numpy
    float32 evaluator's (Modi contributions summed in the reverse order) lie inside."""
    w, Y = _work(name, **kw)
    for p in range(w.P):
        d = O.decode(w.type[p], w.value[p], w.size[p], w.V, w.n_out)
        outs, _ = E.forward(d, w.X, w.n_out)
        sh = O.eval_shadow32(d, w.X, w.n_out)
        n32 = _np32_outputs(d, w.X, w.n_out).astype(np.float64)
        for o in range(w.n_out):
            for v in (sh[o], n32[o]):
                ok = _inside(v, outs[o].lo, outs[o].hi, outs[o].nan)
                assert ok.all(), (name, p, o, np.nonzero(~ok)[0][:3])


def test_output_envelopes_several_contributions_per_output():
    """Random small trees with Modi tags on 40% of function nodes: several contributions per
    output, summed by the shadow in increasing node index and by the numpy float32 evaluator in
    the reverse order; both lie inside every point's output envelope."""
    r = np.random.default_rng(31)
    T, Vv, S = synth.depth_limited(r, 400, r.integers(2, 6, 400), r.random(400) < 0.5, synth.F11, 3, 40)
    func = T == O.T_FUNC
    tag = func & (r.random(T.shape) < 0.5)
    T[tag] = O.T_MODI0 + r.integers(0, 3, T.shape)[tag]
    X = r.uniform(-3, 3, size=(3, 96)).astype(f32)
    several = 0
    for p in range(T.shape[0]):
        d = O.decode(T[p], Vv[p], S[p], 3, 3)
        assert d.status == O.OK
        several += max([d.out.count(o) for o in range(3)]) > 1
        outs, _ = E.forward(d, X, 3)
        sh = O.eval_shadow32(d, X, 3)
        n32 = _np32_outputs(d, X, 3).astype(np.float64)
        for o in range(3):
            for v in (sh[o], n32[o]):
                assert _inside(v, outs[o].lo, outs[o].hi, outs[o].nan).all(), (p, o)
    assert several > 100
