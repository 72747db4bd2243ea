"""Envelopes of float32 evaluation: interval bounds derived from the oracle's definitions.

TEST INFRASTRUCTURE. Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import or run this module. It shares no
code with the device library.

Why it exists. A tree evaluated in float32 has no unique answer: every node
result is rounded, a float32 math library is only within a few ulp of the
exact function, and long sums depend on their order. So, next to the
float64 value of a fitness or a gradient component, the comparison protocol
needs the set of values that *some* float32 evaluation following the
arithmetic model below can return. This module computes an interval
containing that set (its envelope), per tree and per gradient component, by
interval arithmetic over the same definitions the oracle evaluates (node
semantics, the reversed-prefix order, Modi outputs, the mean square, the
reverse sweep): every node carries, per data point, an interval [lo, hi]
holding every value the node can take, and a flag for a possible NaN.

Arithmetic model of a float32 evaluation:
  * inputs X, Y and the constants are float32 values, read exactly;
  * + - * / are IEEE float32 operations (correctly rounded, overflow to
    inf); max, min (NaN operands ignored), |a|, negation and the exp clamp
    are exact;
  * sin, cos, tanh, exp, log and tan are a float32 library within LIB_ULP
    ulp of the exact function of the rounded argument; one ulp of r is at
    most 2u|r| (u = 2^-24), or 2^-149 below the normal range;
  * protected log rounds |a| + eps once before the logarithm;
  * each partial derivative is formed from the node's operands by the
    formula of the oracle's table with at most PARTIAL_ROUNDINGS roundings;
    a product of an adjoint and a partial is rounded once, and a Modi
    node's pass-through sum once (possibly fused with the product);
  * a sum of squared errors is formed in float32 partial sums no deeper
    than log2(K_MAX) + n_out + 5 levels (lane, then wavefront), the partial
    sums are added in float64, and the mean is rounded to float32;
  * a gradient sum (a constant's adjoints over the points, a point's X
    adjoints over every variable leaf of the trees) is a float32 sum in any
    order and grouping, in which no term passes through more than h
    additions: within h u sum|terms| of the exact sum.

Intervals. A node whose operands are exact float32 values (points) and
whose operation is correctly rounded is a point: the float32 shadow's value
(tgp_oracle.apply_op_shadow32), since every correctly rounded evaluation
returns those bits. Otherwise the node's interval is the exact range of the
operation over its operands' intervals (monotone pieces, critical points,
the union of a protected operator's branches), widened outward by the
operation's rounding. Rounding to float32 is monotone, so the widened
range holds every float32 result. The float64 arithmetic used to form the
endpoints rounds by at most 2^-53 relative, far inside the float32 widening.

What the envelope is for: the device value must lie inside it (NaN only
where a NaN is possible), and where the envelope lies within the stated
tolerance of the float64 value, that tolerance is met. Pins:
tests/test_oracle_envelope.py.
"""

import numpy as np

from .tgp_oracle import (EXP_CLAMP, LOG_EPS, OK, OPS, T_CONST, T_FUNC, TAU, _r32, apply_op_shadow32, decode,
                         op_partials)

U = 2.0 ** -24                 # unit roundoff of float32 (round to nearest)
TINY = 2.0 ** -149             # one ulp below the normal range
LIB_ULP = 4                    # assumed accuracy of the float32 math library, in ulp
PARTIAL_ROUNDINGS = 4          # roundings a float32 implementation spends on one partial derivative
K_MAX = 16                     # points per lane of the widest evaluation kernel
FLT_MAX = float(np.finfo(np.float32).max)
INF = np.inf
CHUNK = 65536                  # points per pass of the gradient tape
TRANSCENDENTAL = frozenset((4, 5, 6, 7, 8, 11))
TWO_PI = 2.0 * np.pi
TANH2 = 4.0 / (3.0 * 3.0 ** 0.5)


class Iv:
    """Per-point intervals: lo <= every possible value <= hi, nan = a NaN is possible,
    pt = the value is exactly lo (== hi) in every evaluation of the model."""

    __slots__ = ("lo", "hi", "nan", "pt")

    def __init__(self, lo, hi, nan, pt):
        self.lo, self.hi, self.nan, self.pt = lo, hi, nan, pt

    @staticmethod
    def point(v):
        v = np.asarray(v, np.float64)
        nan = np.isnan(v)
        return Iv(np.where(nan, -INF, v), np.where(nan, INF, v), nan, ~nan)

    def mag(self):
        """Largest magnitude in the interval."""
        return np.maximum(np.abs(self.lo), np.abs(self.hi))


def _clean(lo, hi):
    """Endpoints formed from infinities may be NaN: widen them to the whole line."""
    if np.isnan(lo).any():
        lo = np.where(np.isnan(lo), -INF, lo)
    if np.isnan(hi).any():
        hi = np.where(np.isnan(hi), INF, hi)
    return lo, hi


def _round_out(lo, hi, rel, k_tiny=1.0):
    """Widen [lo, hi] outward by a rounding of relative size rel (and k_tiny subnormal ulps),
    then map what rounds past the float32 range to +-inf (and keep finite values that round
    to the largest float32 inside)."""
    with np.errstate(all="ignore"):
        lo2 = lo - (rel * np.abs(lo) + k_tiny * TINY)
        hi2 = hi + (rel * np.abs(hi) + k_tiny * TINY)
        big = np.abs(lo2) > FLT_MAX
        if big.any():
            lo2 = np.where(lo2 < -FLT_MAX, -INF, np.where(lo2 > FLT_MAX, FLT_MAX, lo2))
        big = np.abs(hi2) > FLT_MAX
        if big.any():
            hi2 = np.where(hi2 > FLT_MAX, INF, np.where(hi2 < -FLT_MAX, -FLT_MAX, hi2))
    return _clean(lo2, hi2)


def _hull(*parts):
    """Hull of (lo, hi, valid) pieces; pieces with valid False are ignored."""
    lo = hi = None
    for plo, phi, ok in parts:
        plo = np.where(ok, plo, INF)
        phi = np.where(ok, phi, -INF)
        lo = plo if lo is None else np.minimum(lo, plo)
        hi = phi if hi is None else np.maximum(hi, phi)
    return lo, hi


def _products(alo, ahi, blo, bhi):
    """Range of x*y over the box, ignoring 0*inf (handled as a NaN by the caller)."""
    with np.errstate(all="ignore"):
        p1, p2, p3, p4 = alo * blo, alo * bhi, ahi * blo, ahi * bhi
    # fmin / fmax skip a NaN product (0 * inf); an all-NaN corner set is cleaned by the caller
    lo = np.fmin(np.fmin(p1, p2), np.fmin(p3, p4))
    hi = np.fmax(np.fmax(p1, p2), np.fmax(p3, p4))
    return _clean(lo, hi)


def _contains(lo, hi, v):
    return (lo <= v) & (v <= hi)


def _has_inf(a):
    return np.isinf(a.lo) | np.isinf(a.hi)


def _zero_inf_nan(a, b):
    """A product may be NaN: one factor may be 0 and the other infinite."""
    return (_contains(a.lo, a.hi, 0.0) & _has_inf(b)) | (_contains(b.lo, b.hi, 0.0) & _has_inf(a))


def _finish(lo, hi, nan, pt_mask, pt_val):
    lo = np.where(pt_mask, pt_val, lo)
    hi = np.where(pt_mask, pt_val, hi)
    return Iv(lo, hi, nan & ~pt_mask, pt_mask)


# ------------------------------------------------------------------ operators on intervals
def _sin_range(lo, hi, phase):
    """Range of sin(x + phase) over [lo, hi] (finite endpoints)."""
    with np.errstate(all="ignore"):
        flo, fhi = np.sin(lo + phase), np.sin(hi + phase)
        r_lo, r_hi = np.minimum(flo, fhi), np.maximum(flo, fhi)
        wide = (hi - lo) >= TWO_PI
        # a maximum at x + phase = pi/2 + 2 k pi, a minimum at -pi/2 + 2 k pi
        kmax = np.ceil((lo + phase - np.pi / 2) / TWO_PI)
        kmin = np.ceil((lo + phase + np.pi / 2) / TWO_PI)
        has_max = np.pi / 2 + kmax * TWO_PI <= hi + phase
        has_min = -np.pi / 2 + kmin * TWO_PI <= hi + phase
    r_hi = np.where(wide | has_max, 1.0, r_hi)
    r_lo = np.where(wide | has_min, -1.0, r_lo)
    return r_lo, r_hi


def _abs_range(a):
    zero_in = _contains(a.lo, a.hi, 0.0)
    lo = np.where(zero_in, 0.0, np.minimum(np.abs(a.lo), np.abs(a.hi)))
    return lo, a.mag()


def iv_op(op, a, b=None):
    """Interval of op applied to interval operands (the value rule of the operator table)."""
    binary = OPS[op][1] == 2
    lib = 2.0 * LIB_ULP * U
    if binary:
        pt = a.pt & b.pt
        pv = apply_op_shadow32(op, np.where(a.pt, a.lo, 0.0), np.where(b.pt, b.lo, 0.0))
        if pt.all():
            return Iv(pv, pv.copy(), np.zeros(pt.shape, bool), pt)
    else:
        pt = a.pt & (op not in TRANSCENDENTAL)
        pv = np.zeros(np.shape(a.lo))
        if a.pt.all() and op in (4, 5, 6, 11):
            # a library function of exact operands: the exact value, widened by the library error
            f = {4: np.sin, 5: np.cos, 6: np.tanh, 11: np.tan}[op]
            with np.errstate(all="ignore"):
                r = f(a.lo)
            lo, hi = _round_out(r, r, lib, LIB_ULP)
            fin = np.isfinite(a.lo)
            nan = ~fin & (op != 6)
            return Iv(np.where(fin | (op == 6), lo, -INF), np.where(fin | (op == 6), hi, INF), nan,
                      np.zeros(pt.shape, bool))
    with np.errstate(all="ignore"):
        if op == 0:
            lo, hi = _clean(a.lo + b.lo, a.hi + b.hi)
            nan = a.nan | b.nan | ((a.hi == INF) & (b.lo == -INF)) | ((a.lo == -INF) & (b.hi == INF))
            lo, hi = _round_out(lo, hi, U)
        elif op == 1:
            lo, hi = _clean(a.lo - b.hi, a.hi - b.lo)
            nan = a.nan | b.nan | ((a.hi == INF) & (b.hi == INF)) | ((a.lo == -INF) & (b.lo == -INF))
            lo, hi = _round_out(lo, hi, U)
        elif op == 2:
            lo, hi = _products(a.lo, a.hi, b.lo, b.hi)
            nan = a.nan | b.nan | _zero_inf_nan(a, b)
            lo, hi = _round_out(lo, hi, U)
        elif op == 3:
            # protected: |b| < tau gives 1; otherwise a / b over the parts of b beyond tau
            small_part = (b.lo < TAU) & (b.hi > -TAU)
            pos_lo, pos_hi = np.maximum(b.lo, TAU), b.hi
            neg_lo, neg_hi = b.lo, np.minimum(b.hi, -TAU)
            pos = pos_lo <= pos_hi
            neg = neg_lo <= neg_hi
            qlo_p, qhi_p = _quotients(a, pos_lo, pos_hi)
            qlo_n, qhi_n = _quotients(a, neg_lo, neg_hi)
            qlo_p, qhi_p = _round_out(qlo_p, qhi_p, U)
            qlo_n, qhi_n = _round_out(qlo_n, qhi_n, U)
            one = np.ones(np.shape(a.lo))
            lo, hi = _hull((qlo_p, qhi_p, pos), (qlo_n, qhi_n, neg), (one, one, small_part))
            beyond = pos | neg
            nan = b.nan | ((a.nan | (_has_inf(a) & _has_inf(b))) & beyond)
            lo, hi = _fill_empty(lo, hi)
        elif op == 9 or op == 10:
            f = np.fmax if op == 9 else np.fmin
            lo, hi = f(a.lo, b.lo), f(a.hi, b.hi)
            # a NaN operand is ignored: the other operand's value is returned
            lo = np.where(a.nan, np.minimum(lo, b.lo), lo)
            hi = np.where(a.nan, np.maximum(hi, b.hi), hi)
            lo = np.where(b.nan, np.minimum(lo, a.lo), lo)
            hi = np.where(b.nan, np.maximum(hi, a.hi), hi)
            nan = a.nan & b.nan
        elif op in (4, 5):
            fin = np.isfinite(a.lo) & np.isfinite(a.hi)
            lo, hi = _sin_range(np.where(fin, a.lo, 0.0), np.where(fin, a.hi, 0.0), 0.0 if op == 4 else np.pi / 2)
            lo, hi = np.where(fin, lo, -1.0), np.where(fin, hi, 1.0)
            lo, hi = _round_out(lo, hi, lib, LIB_ULP)
            nan = a.nan | ~fin
        elif op == 6:
            lo, hi = _round_out(np.tanh(a.lo), np.tanh(a.hi), lib, LIB_ULP)
            nan = a.nan
        elif op == 7:
            lo = np.exp(np.clip(a.lo, -EXP_CLAMP, EXP_CLAMP))
            hi = np.exp(np.clip(a.hi, -EXP_CLAMP, EXP_CLAMP))
            lo, hi = _round_out(lo, hi, lib, LIB_ULP)
            nan = a.nan
        elif op == 8:
            alo, ahi = _abs_range(a)
            tlo, thi = alo + LOG_EPS, ahi + LOG_EPS
            # the rounded argument: the shadow's bits where a is a point
            tpt = _r32(np.where(a.pt, np.abs(a.lo), 0.0) + LOG_EPS)
            tlo, thi = _round_out(tlo, thi, U)
            tlo, thi = np.where(a.pt, tpt, tlo), np.where(a.pt, tpt, thi)
            lo, hi = _round_out(np.log(tlo), np.log(thi), lib, LIB_ULP)
            nan = a.nan
        elif op == 11:
            fin = np.isfinite(a.lo) & np.isfinite(a.hi)
            alo, ahi = np.where(fin, a.lo, 0.0), np.where(fin, a.hi, 0.0)
            # a pole pi/2 + k pi inside the interval: any value
            k = np.ceil((alo - np.pi / 2) / np.pi)
            pole = (np.pi / 2 + k * np.pi <= ahi) | ((ahi - alo) >= np.pi)
            lo, hi = _round_out(np.tan(alo), np.tan(ahi), lib, LIB_ULP)
            lo = np.where(pole | ~fin, -INF, lo)
            hi = np.where(pole | ~fin, INF, hi)
            nan = a.nan | ~fin
        else:
            raise ValueError(op)
    return _finish(lo, hi, nan, pt, pv)


def _quotients(a, blo, bhi):
    """Range of a / b for b in [blo, bhi] of one sign (beyond tau); inf / inf ignored."""
    with np.errstate(all="ignore"):
        qs = np.stack([a.lo / blo, a.lo / bhi, a.hi / blo, a.hi / bhi])
    lo = np.min(np.where(np.isnan(qs), INF, qs), axis=0)
    hi = np.max(np.where(np.isnan(qs), -INF, qs), axis=0)
    return lo, hi


def _fill_empty(lo, hi):
    """An empty hull (only NaN outcomes) becomes the whole line, with the NaN flag set by the caller."""
    empty = lo > hi
    return np.where(empty, -INF, lo), np.where(empty, INF, hi)


# ------------------------------------------------------------------ partial derivatives on intervals
def iv_partials(op, a, b=None):
    """Intervals of the partial derivatives (d/da, d/db) a float32 evaluation can form at operands
    in the intervals a, b: the oracle's table (its conventions at kinks) over every operand pair,
    rounded PARTIAL_ROUNDINGS times, and the library's error where a library function is used.
    A partial that is exactly an operand or a constant keeps that operand's interval."""
    binary = OPS[op][1] == 2
    shape = np.shape(a.lo)
    one = Iv.point(np.ones(shape))
    zero = Iv.point(np.zeros(shape))
    R = PARTIAL_ROUNDINGS * U
    lib = 2.0 * LIB_ULP * U
    with np.errstate(all="ignore"):
        if op == 0:
            return one, one
        if op == 1:
            return one, Iv.point(-np.ones(shape))
        if op == 2:
            return b, a
        if op == 9 or op == 10:
            # the slope goes to a where a >= b (max) or a <= b (min), or where b is NaN; to b
            # where the opposite comparison holds or a is NaN (and b is not)
            if op == 9:
                may_a = (a.hi >= b.lo) | b.nan
                may_b = (a.lo < b.hi) | (a.nan & ~b.nan)
            else:
                may_a = (a.lo <= b.hi) | b.nan
                may_b = (a.hi > b.lo) | (a.nan & ~b.nan)
            # points: the comparison is decided exactly as the table does
            both_pt = a.pt & b.pt
            pick_a = ((a.lo >= b.lo) if op == 9 else (a.lo <= b.lo))
            may_a = np.where(both_pt, pick_a, may_a)
            may_b = np.where(both_pt, ~pick_a, may_b)
            da = _sel(may_a, may_b)
            db = _sel(may_b, may_a)
            return da, db
        if op == 3:
            small_part = (b.lo < TAU) & (b.hi > -TAU)
            parts_a, parts_b = [], []
            for blo, bhi in ((np.maximum(b.lo, TAU), b.hi), (b.lo, np.minimum(b.hi, -TAU))):
                ok = blo <= bhi
                r_lo, r_hi = _recip(blo, bhi)
                parts_a.append(_round_out(r_lo, r_hi, U) + (ok,))
                # -a / b^2 over the box
                s_lo, s_hi = _recip_sq(blo, bhi)
                p_lo, p_hi = _products(-a.hi, -a.lo, s_lo, s_hi)
                parts_b.append(_round_out(p_lo, p_hi, R) + (ok,))
            zero_part = (np.zeros(shape), np.zeros(shape), small_part)
            lo_a, hi_a = _fill_empty(*_hull(parts_a[0], parts_a[1], zero_part))
            lo_b, hi_b = _fill_empty(*_hull(parts_b[0], parts_b[1], zero_part))
            nan = a.nan | b.nan
            # points: 1/b is rounded once on both sides (the same bits); -a/b^2 is not
            pb = a.pt & b.pt
            rb = np.where(pb, b.lo, 1.0)
            pa_val = np.where(np.abs(rb) < TAU, 0.0, _r32(1.0 / rb))
            da = _finish(lo_a, hi_a, b.nan, pb, pa_val)
            db = Iv(lo_b, hi_b, nan | (_has_inf(a) & _has_inf(b)), np.zeros(shape, bool))
            return da, db
        # unary
        if op == 4 or op == 5:
            fin = np.isfinite(a.lo) & np.isfinite(a.hi)
            lo, hi = _sin_range(np.where(fin, a.lo, 0.0), np.where(fin, a.hi, 0.0),
                                np.pi / 2 if op == 4 else np.pi)     # cos a, or -sin a = sin(a + pi)
            lo, hi = np.where(fin, lo, -1.0), np.where(fin, hi, 1.0)
            lo, hi = _round_out(lo, hi, lib, LIB_ULP)
            return Iv(lo, hi, a.nan | ~fin, np.zeros(shape, bool)), None
        if op == 6:
            th_lo, th_hi = _round_out(np.tanh(a.lo), np.tanh(a.hi), lib, LIB_ULP)
            sq_lo = np.where(_contains(th_lo, th_hi, 0.0), 0.0, np.minimum(th_lo ** 2, th_hi ** 2))
            sq_hi = np.maximum(th_lo ** 2, th_hi ** 2)
            lo, hi = 1.0 - sq_hi, 1.0 - sq_lo
            lo = lo - R * (sq_hi + np.abs(lo)) - TINY
            hi = hi + R * (sq_hi + np.abs(hi)) + TINY
            return Iv(lo, hi, a.nan, np.zeros(shape, bool)), None
        if op == 7:
            inside_all = (a.lo >= -EXP_CLAMP) & (a.hi <= EXP_CLAMP)
            outside_any = (a.lo < -EXP_CLAMP) | (a.hi > EXP_CLAMP) | a.nan
            inside_any = (a.hi >= -EXP_CLAMP) & (a.lo <= EXP_CLAMP)
            e_lo = np.exp(np.clip(a.lo, -EXP_CLAMP, EXP_CLAMP))
            e_hi = np.exp(np.clip(a.hi, -EXP_CLAMP, EXP_CLAMP))
            e_lo, e_hi = _round_out(e_lo, e_hi, lib, LIB_ULP)
            z = np.zeros(shape)
            lo, hi = _fill_empty(*_hull((e_lo, e_hi, inside_any), (z, z, outside_any & ~inside_all)))
            return Iv(lo, hi, np.zeros(shape, bool), np.zeros(shape, bool)), None
        if op == 8:
            # sign(a) / (|a| + eps), 0 at a == 0 (either sign of zero)
            pos_lo, pos_hi = np.maximum(a.lo, 0.0), a.hi
            neg_lo, neg_hi = a.lo, np.minimum(a.hi, 0.0)
            pos = (pos_hi > 0) & (pos_lo <= pos_hi)
            neg = (neg_lo < 0) & (neg_lo <= neg_hi)
            zero_in = _contains(a.lo, a.hi, 0.0)
            # device: |a| + eps rounded, then the quotient rounded; the shadow: exact, rounded once
            p_lo, p_hi = 1.0 / (pos_hi + LOG_EPS), 1.0 / (np.maximum(pos_lo, 0.0) + LOG_EPS)
            # on the negative side -1/(|a| + eps) is lowest at the smallest |a| (the upper end)
            n_lo, n_hi = -1.0 / (np.maximum(-neg_hi, 0.0) + LOG_EPS), -1.0 / (np.maximum(-neg_lo, 0.0) + LOG_EPS)
            p_lo, p_hi = _round_out(p_lo, p_hi, R)
            n_lo, n_hi = _round_out(n_lo, n_hi, R)
            z = np.zeros(shape)
            lo, hi = _fill_empty(*_hull((p_lo, p_hi, pos), (n_lo, n_hi, neg), (z, z, zero_in)))
            return Iv(lo, hi, a.nan, np.zeros(shape, bool)), None
        if op == 11:
            t = iv_op(11, a)
            sq_lo = np.where(_contains(t.lo, t.hi, 0.0), 0.0, np.minimum(t.lo ** 2, t.hi ** 2))
            sq_hi = np.maximum(t.lo ** 2, t.hi ** 2)
            lo, hi = _round_out(1.0 + sq_lo, 1.0 + sq_hi, R)
            return Iv(lo, hi, t.nan, np.zeros(shape, bool)), None
    raise ValueError(op)


def _sel(may_first, may_second):
    """The 0/1 slope an operand receives: 1 where only it can be picked, 0 where only the
    other can, [0, 1] where either can."""
    lo = np.where(may_first & ~may_second, 1.0, 0.0)
    hi = np.where(may_first, 1.0, 0.0)
    pt = lo == hi
    return Iv(lo, hi, np.zeros(np.shape(lo), bool), pt)


def _recip(blo, bhi):
    """Range of 1/b over [blo, bhi] of one sign."""
    with np.errstate(all="ignore"):
        r1, r2 = 1.0 / blo, 1.0 / bhi
    return np.minimum(r1, r2), np.maximum(r1, r2)


def _recip_sq(blo, bhi):
    """Range of 1/b^2 over [blo, bhi] of one sign."""
    with np.errstate(all="ignore"):
        r1, r2 = 1.0 / (blo * blo), 1.0 / (bhi * bhi)
    return np.minimum(r1, r2), np.maximum(r1, r2)


def iv_mul_round(x, y):
    """Interval of fl(x * y): the shadow's bits for two points."""
    pt = x.pt & y.pt
    with np.errstate(all="ignore"):
        pv = _r32(np.where(pt, x.lo, 0.0) * np.where(pt, y.lo, 0.0))
    if pt.all():
        return Iv(pv, pv.copy(), np.zeros(pt.shape, bool), pt)
    lo, hi = _products(x.lo, x.hi, y.lo, y.hi)
    lo, hi = _round_out(lo, hi, U)
    return _finish(lo, hi, x.nan | y.nan | _zero_inf_nan(x, y), pt, pv)


def iv_add_round(x, y, fused=False):
    """Interval of fl(x + y), or of a sum the device may fuse with the product that formed x
    (x's interval already holds the unrounded product, so one outward rounding covers both)."""
    pt = x.pt & y.pt & (not fused)
    with np.errstate(all="ignore"):
        pv = _r32(np.where(pt, x.lo, 0.0) + np.where(pt, y.lo, 0.0))
        lo, hi = _clean(x.lo + y.lo, x.hi + y.hi)
    lo, hi = _round_out(lo, hi, U)
    nan = x.nan | y.nan | ((x.hi == INF) & (y.lo == -INF)) | ((x.lo == -INF) & (y.hi == INF))
    return _finish(lo, hi, nan, pt, pv)


# ------------------------------------------------------------------ trees
def _leaf(d, i, X):
    if d.kind[i] == T_CONST:
        return Iv.point(_r32(np.full(X.shape[1], float(d.arg[i]))))
    return Iv.point(_r32(X[d.arg[i]]))


def _modi_sum(parts, D):
    """Interval of a float32 sum of Modi contributions in any order: the exact range of the sum,
    widened by (n - 1) u times the largest possible sum of magnitudes; one term is exact."""
    if not parts:
        return Iv.point(np.zeros(D))
    if len(parts) == 1:
        return parts[0]
    lo = sum(p.lo for p in parts)
    hi = sum(p.hi for p in parts)
    mag = sum(p.mag() for p in parts)
    lo, hi = _clean(lo, hi)
    n = len(parts)
    with np.errstate(all="ignore"):
        w = (n - 1) * U * mag + n * TINY
        lo, hi = _round_out(lo - w, hi + w, 0.0, 0.0)
    any_pinf = np.any([p.hi == INF for p in parts], axis=0)
    any_ninf = np.any([p.lo == -INF for p in parts], axis=0)
    nan = np.any([p.nan for p in parts], axis=0) | (any_pinf & any_ninf)
    return Iv(lo, hi, nan, np.zeros(D, bool))


def forward(d, X, n_out, keep=False):
    """Output intervals [n_out] of a valid tree over the points of X (and, with keep, every
    node's interval: the value it hands to its parent, and a Modi node's own result)."""
    X = np.asarray(X, np.float64)
    D = X.shape[1]
    stack = []
    contrib = {}
    nodes = [None] * d.length if keep else None
    for i in range(d.length - 1, -1, -1):
        if d.kind[i] != T_FUNC:
            v = _leaf(d, i, X)
            stack.append(v)
            if keep:
                nodes[i] = v
            continue
        op = d.arg[i]
        if OPS[op][1] == 2:
            a, b = stack.pop(), stack.pop()
            r = iv_op(op, a, b)
            right = b
        else:
            a = stack.pop()
            r = iv_op(op, a)
            right = a
        if d.out[i] >= 0:
            contrib.setdefault(d.out[i], []).append(r)
            stack.append(right)
        else:
            stack.append(r)
        if keep:
            nodes[i] = stack[-1]
    if d.n_modi == 0:
        outs = [stack[0]] + [Iv.point(np.zeros(D)) for _ in range(n_out - 1)]
    else:
        outs = [_modi_sum(contrib.get(o, []), D) for o in range(n_out)]
    return outs, nodes


def fitness_tree(d, X, Y, n_out):
    """(lo, hi, nan): an interval holding every float32 evaluation's fitness of one decoded
    tree, and whether a NaN is possible. Invalid trees give (nan, nan, True)."""
    if d.status != OK:
        return float("nan"), float("nan"), True
    X = np.asarray(X, np.float64)
    D = X.shape[1]
    Yd = _r32(np.asarray(Y, np.float64).reshape(n_out, D))
    outs, _ = forward(d, X, n_out)
    s_lo = s_hi = 0.0
    nan = False
    with np.errstate(all="ignore"):
        for o in range(n_out):
            y = Iv.point(Yd[o])
            r = iv_op(1, outs[o], y)
            sq_lo = np.where(_contains(r.lo, r.hi, 0.0), 0.0, np.minimum(r.lo * r.lo, r.hi * r.hi))
            sq_hi = np.maximum(r.lo * r.lo, r.hi * r.hi)
            sq_lo, sq_hi = _round_out(sq_lo, sq_hi, U)
            pv = _r32(np.where(r.pt, r.lo, 0.0) ** 2)
            sq_lo, sq_hi = np.where(r.pt, pv, sq_lo), np.where(r.pt, pv, sq_hi)
            s_lo += float(np.sum(np.maximum(sq_lo, 0.0)))
            s_hi += float(np.sum(sq_hi))
            nan = nan or bool(np.any(r.nan))
        depth = np.log2(K_MAX) + n_out + 5
        g = depth * U + (D * n_out + D) * 2.0 ** -53
        m_lo = s_lo * (1.0 - g) / D
        m_hi = s_hi * (1.0 + g) / D
        m_lo, m_hi = _round_out(np.array(m_lo), np.array(m_hi), U + 2.0 ** -52)
    return float(m_lo), float(m_hi), nan


def fitness(pop_type, pop_value, pop_size, X, Y, n_out=1, rows=None):
    """Fitness envelopes (lo [R], hi [R], nan [R]) of the given rows."""
    X = np.asarray(X)
    V = X.shape[0]
    rows = list(range(pop_type.shape[0]) if rows is None else rows)
    res = [fitness_tree(decode(pop_type[p], pop_value[p], pop_size[p], V, n_out), X, Y, n_out) for p in rows]
    if not res:
        return np.zeros(0), np.zeros(0), np.zeros(0, bool)
    lo, hi, nan = zip(*res)
    return np.array(lo), np.array(hi), np.array(nan, bool)


# ------------------------------------------------------------------ gradients
def grad_tree(d, X, Y, n_out, g=1.0, D_total=None):
    """Per-point adjoint intervals of one tree's constants and variable leaves, for the points
    of X (a slice of D_total points; default all). The output adjoint is
    fl(fl(fl(2 g) * residual) * fl(1 / D)). Returns ({node: Iv}, [(v, Iv)])."""
    X = np.asarray(X, np.float64)
    D = X.shape[1]
    n = d.length
    outs, nodes = forward(d, X, n_out, keep=True)
    Yd = _r32(np.asarray(Y, np.float64).reshape(n_out, D))
    q2g = Iv.point(np.full(D, float(_r32(2.0 * g))))
    inv = Iv.point(np.full(D, float(_r32(1.0 / (D if D_total is None else D_total)))))
    gout = [iv_mul_round(iv_mul_round(q2g, iv_op(1, outs[o], Iv.point(Yd[o]))), inv) for o in range(n_out)]
    zero = Iv.point(np.zeros(D))
    adj = [None] * n
    adj[0] = gout[0] if d.n_modi == 0 else zero
    const, var = {}, []
    for i in range(n):
        lam = adj[i]
        if d.kind[i] == T_CONST:
            const[i] = lam
            continue
        if d.kind[i] != T_FUNC:
            var.append((d.arg[i], lam))
            continue
        op = d.arg[i]
        c1 = i + 1
        kids = [c1] if OPS[op][1] == 1 else [c1, c1 + d.size[c1]]
        if len(kids) == 2:
            pa, pb = iv_partials(op, nodes[kids[0]], nodes[kids[1]])
            parts = [pa, pb]
        else:
            pa, _ = iv_partials(op, nodes[kids[0]])
            parts = [pa]
        modi = d.out[i] >= 0
        base = gout[d.out[i]] if modi else lam
        for c, p in zip(kids, parts):
            adj[c] = iv_mul_round(base, p)
        if modi:
            adj[kids[-1]] = iv_add_round(adj[kids[-1]], lam, fused=True)
    return const, var


def _sum_iv(terms_lo, terms_hi, terms_mag, h):
    """Interval of a float32 sum of terms in which no term passes more than h additions."""
    lo, hi = _clean(terms_lo, terms_hi)
    w = h * U * terms_mag
    return lo - w, hi + w


def grad(pop_type, pop_value, pop_size, X, Y, n_out=1, rows=None, g=None, lanes_k=4, chunk=CHUNK):
    """Gradient envelopes of sum_t g_t fitness_t over the listed rows.

    Returns (gv_lo, gv_hi, gv_nan [R][Lmax], gX_lo, gX_hi, gX_nan [V][D]). A constant's gradient
    is a float32 sum of its per-point adjoints: k - 1 additions in a lane of k points, 6 in a
    wavefront, then one per point tile of 64 k points. lanes_k is one k or several; the bound
    takes the longest of their addition chains, so it holds for each of them. A point's X
    gradient is a float32 sum over every variable leaf of the listed trees. Positions that are
    not constants are 0."""
    X = np.asarray(X, np.float64)
    V, D = X.shape
    Yd = np.asarray(Y, np.float64).reshape(n_out, D)
    rows = list(range(pop_type.shape[0]) if rows is None else rows)
    Lmax = pop_type.shape[1]
    R = len(rows)
    gv = np.zeros((3, R, Lmax))          # lo, hi, magnitude sums
    gv_nan = np.zeros((R, Lmax), bool)
    gX = np.zeros((3, V, D))
    gX_nan = np.zeros((V, D), bool)
    nX = np.zeros(V)
    for k, p in enumerate(rows):
        d = decode(pop_type[p], pop_value[p], pop_size[p], V, n_out)
        if d.status != OK:
            continue
        gt = 1.0 if g is None else float(g[p])
        for p0 in range(0, D, chunk):
            sl = slice(p0, min(D, p0 + chunk))
            const, var = grad_tree(d, X[:, sl], Yd[:, sl], n_out, gt, D_total=D)
            with np.errstate(all="ignore"):
                for j, lam in const.items():
                    gv[0, k, j] += float(np.sum(lam.lo))
                    gv[1, k, j] += float(np.sum(lam.hi))
                    gv[2, k, j] += float(np.sum(lam.mag()))
                    gv_nan[k, j] |= bool(lam.nan.any())
                for v, lam in var:
                    gX[0, v, sl] += lam.lo
                    gX[1, v, sl] += lam.hi
                    gX[2, v, sl] += lam.mag()
                    gX_nan[v, sl] |= lam.nan
        for i in range(d.length):
            if d.kind[i] == 0:
                nX[d.arg[i]] += 1
    ks = (int(lanes_k),) if np.ndim(lanes_k) == 0 else tuple(int(k) for k in lanes_k)
    h = max(k - 1 + 6 + -(-D // (64 * k)) for k in ks)
    with np.errstate(all="ignore"):
        gv_lo, gv_hi = _sum_iv(gv[0], gv[1], gv[2], h + D * 2.0 ** -29)
        hX = np.maximum(nX - 1, 0)[:, None] + nX[:, None] * 2.0 ** -29
        gX_lo, gX_hi = _sum_iv(gX[0], gX[1], gX[2], hX)
    return gv_lo, gv_hi, gv_nan, gX_lo, gX_hi, gX_nan
