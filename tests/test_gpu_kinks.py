"""The forward and adjoint kernels at the operators' kinks, compared with the
CPU oracle point by point. Inputs sit exactly on the protected-division
threshold (|b| = tau and the float32 neighbours of tau), on max/min ties, on
the exp clamp edges (+-20 and their neighbours) and at log(0), in variable
leaves and in function-node operands (whose values the adjoint recomputes).
Needs an MI355X."""

import numpy as np
import pytest
import torch

import oracle as O
import paper_2501_17168_amd as tgp

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

TAU = np.float32(1e-6)
BELOW = np.nextafter(TAU, np.float32(0))
ABOVE = np.nextafter(TAU, np.float32(1))
E20 = np.nextafter(np.float32(20), np.float32(np.inf))
BASE = np.array([TAU, -TAU, BELOW, -BELOW, ABOVE, 0.0, -0.0, 1.5, -2.0, 20.0, -20.0, E20, -E20, 25.0, -25.0,
                 2.0, 0.5, 3.0], np.float32)
# every pair of base values: ties on the diagonal, 324 points (a ragged last tile)
X = np.ascontiguousarray(np.stack(np.meshgrid(BASE, BASE, indexing="ij")).reshape(2, -1))
D = X.shape[1]
Y = np.full((1, D), 0.3, np.float32)

A0 = [(2, 0, 3), (0, 0, 1), (1, 0.0, 1)]     # ADD(x0, 0): a function node whose value is x0
A1 = [(2, 0, 3), (0, 1, 1), (1, 0.0, 1)]     # ADD(x1, 0)


def fn(op, *kids):
    """Prefix rows of op applied to the given child row lists."""
    size = 1 + sum(len(k) for k in kids)
    rows = [(2, op, size)]
    for k in kids:
        rows += k
    return rows


X0, X1 = [(0, 0, 1)], [(0, 1, 1)]
TREES = {
    "div(x0,x1)": fn(3, X0, X1), "div(f,f)": fn(3, A0, A1), "div(3,x1)": fn(3, [(1, 3.0, 1)], X1),
    "max(x0,x1)": fn(9, X0, X1), "min(x0,x1)": fn(10, X0, X1),
    "max(f,f)": fn(9, A0, A1), "min(f,f)": fn(10, A0, A1),
    "max(1.5,x0)": fn(9, [(1, 1.5, 1)], X0), "min(x0,-2)": fn(10, X0, [(1, -2.0, 1)]),
    "max(x0,f)": fn(9, X0, A1), "min(f,x1)": fn(10, A0, X1),
    "exp(x0)": fn(7, X0), "exp(f)": fn(7, A0), "log(x0)": fn(8, X0), "log(f)": fn(8, A0),
    "tan(x1)": fn(11, X1),
}
TRANSC = {"exp(x0)", "exp(f)", "log(x0)", "log(f)", "tan(x1)"}
LMAX = 8


def encode(rows):
    t, v, s = (np.full((1, LMAX), np.nan, np.float32) for _ in range(3))
    for i, (a, b, c) in enumerate(rows):
        t[0, i], v[0, i], s[0, i] = a, b, c
    return t, v, s


def ulp32(x):
    x = np.abs(np.asarray(x, np.float32))
    return np.nextafter(x, np.float32(np.inf)).astype(np.float64) - x.astype(np.float64)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("name", list(TREES))
@pytest.mark.parametrize("mode", [1, 2, 3])
def test_forward_at_kinks(name, mode):
    t, v, s = encode(TREES[name])
    pop = tgp.Population(dev(t), dev(v), dev(s))
    _, pred = tgp.eval_multi_output(pop, dev(X), None, n_out=1, want_pred=True,
                                    config=tgp.cfg(mode=mode, points_per_lane=4))
    m = tgp.eval_mse(pop, dev(X), dev(Y), config=tgp.cfg(mode=mode, points_per_lane=4))
    torch.cuda.synchronize()
    got = pred.cpu().numpy()[0, 0].astype(np.float64)
    ref = O.predict(t, v, s, X, 1)[0, 0]
    np.testing.assert_array_equal(np.isnan(got), np.isnan(ref), err_msg=name)
    fin = np.isfinite(ref)
    if name in TRANSC:
        # a float32 library function: within a few ulp of the float64 value
        bad = np.abs(got[fin] - ref[fin]) > 4 * ulp32(ref[fin])
    else:
        # correctly rounded division, exact max/min/add: the float64 value rounded once
        bad = got[fin] != ref[fin].astype(np.float32).astype(np.float64)
    assert not bad.any(), (name, X[:, fin][:, bad][:, :4].T.tolist(), got[fin][bad][:4], ref[fin][bad][:4])
    m64 = O.mse(t, v, s, X, Y)[0]
    assert abs(float(m.cpu()[0]) - m64) <= 1e-5 * abs(m64), (name, float(m.cpu()[0]), m64)


@pytest.mark.parametrize("name", list(TREES))
@pytest.mark.parametrize("k", [2, 4])
def test_adjoint_at_kinks(name, k):
    t, v, s = encode(TREES[name])
    pop = tgp.Population(dev(t), dev(v), dev(s))
    mse, gv, gx = tgp.eval_mse_grad(pop, dev(X), dev(Y), config=tgp.cfg(mode=2, points_per_lane=k, block_waves=1))
    torch.cuda.synchronize()
    m64, gv64, gx64 = O.grad(t, v, s, X, Y)
    assert abs(float(mse.cpu()[0]) - m64[0]) <= 1e-5 * abs(m64[0])
    gx = gx.cpu().numpy().astype(np.float64)
    # per point: a product of a few float32 roundings of the same factors
    np.testing.assert_allclose(gx, gx64, rtol=2e-6 if name not in TRANSC else 1e-5, atol=0, err_msg=name)
    gvd = gv.cpu().numpy().astype(np.float64)[0]
    const = t[0] == 1
    assert (gvd[~const] == 0).all()
    for j in np.nonzero(const)[0]:
        # a constant's gradient is a float32 sum over the points: recursive summation of n terms
        # is within n u sum|terms| of the exact sum (u = 2^-24)
        lam = const_adjoint(t, v, s, j)
        assert lam.sum() == pytest.approx(gv64[0, j], rel=1e-12, abs=1e-300)
        bound = D * 2.0 ** -24 * np.abs(lam).sum() + 2e-6 * abs(gv64[0, j])
        assert abs(gvd[j] - gv64[0, j]) <= bound, (name, j, gvd[j], gv64[0, j], bound)


def const_adjoint(t, v, s, j):
    """Per-point adjoint of constant node j: the same tree with node j read from a third
    variable that holds the constant at every point; its X gradient is that adjoint."""
    t2, v2 = t.copy(), v.copy()
    c = v[0, j]
    t2[0, j], v2[0, j] = 0, 2
    X3 = np.concatenate([X, np.full((1, D), c, np.float32)])
    _, _, gx = O.grad(t2, v2, s, X3, Y)
    return gx[2]
