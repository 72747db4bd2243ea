"""Device gradients (adjoint kernel through tgp_eval_mse_grad) against the CPU
oracle's tape gradient, its float32 envelopes and central finite
differences; autograd and Adam with a gradient check at every step."""

import numpy as np
import pytest
import torch

import oracle as O
import paper_2501_17168_amd as tgp
import synth
from parity import FitnessRef, GradRef, compare_fitness, compare_grad_value, compare_grad_x

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
_cache = {}


def work(name="grad", **kw):
    key = (name, tuple(sorted(kw.items())))
    if key not in _cache:
        w = synth.workload(name, **kw)
        Y = w.Y if w.Y is not None else w.targets_from(O.predict(*w.hidden, w.X, 1)[:, 0, :])
        _cache[key] = (w, np.ascontiguousarray(Y, dtype=np.float32))
    return _cache[key]


def dev_pop(w, value=None):
    v = w.value if value is None else value
    return tgp.Population(*(torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (w.type, v, w.size)))


_grefs = {}


def grad_ref(name, w, Y, g=None):
    key = (name, w.P, w.D, None if g is None else g.tobytes())
    if key not in _grefs:
        _grefs[key] = GradRef(w.type, w.value, w.size, w.X, Y, g=g)
    return _grefs[key]


# every workload shape that has single-output trees: the 11-op set (hybrid, grad), the paper's
# set with tan (pagie), the 4-op set (plain) and a data-parallel shape (5 variables, D far above
# one point tile, a ragged last tile)
GRAD_CASES = [("grad", dict(P=300, D=3100)), ("hybrid", dict(P=250, D=2000)), ("plain", {}),
              ("pagie", dict(P=250, D=2000)), ("dataparallel", dict(P=24, D=131_077))]


@pytest.mark.parametrize("name,kw", GRAD_CASES)
@pytest.mark.parametrize("k", [2, 3, 4])
def test_grad_matches_oracle(name, kw, k):
    w, Y = work(name, **kw)
    pop = dev_pop(w)
    X = torch.from_numpy(w.X).to(DEV)
    Yd = torch.from_numpy(Y).to(DEV)
    mse, gv, gx = tgp.eval_mse_grad(pop, X, Yd, config=tgp.cfg(mode=2, points_per_lane=k))
    torch.cuda.synchronize()
    ref = grad_ref(name, w, Y)
    fref = FitnessRef(w.type, w.value, w.size, w.X, Y)
    rep_f = compare_fitness(mse.cpu().numpy(), fref, label=f"{name} fitness")
    rep_v = compare_grad_value(gv.cpu().numpy(), ref, label=name)
    rep_x = compare_grad_x(gx.cpu().numpy(), ref, label=name)
    print(f"{name} K={k}: fitness {rep_f}\n  grad_value {rep_v}\n  grad_X {rep_x}", flush=True)
    # the envelopes are narrow enough to mean something on most constant gradients
    assert rep_v["tight"] >= 0.25 * rep_v["n"], rep_v
    # grad_X sums over every tree, so one tree with a wide envelope (tan near its poles, a
    # near-singular quotient) widens the sum at every point. The same call on the sub-population
    # of trees whose fitness envelope is within 1e-5 checks the X gradient of the well-determined
    # trees at the 1e-3 bar.
    tol = np.maximum(1e-5 * np.abs(fref.m64), 1e-6)
    with np.errstate(invalid="ignore"):
        good = np.isfinite(fref.m64) & ~fref.nan & (fref.lo >= fref.m64 - tol) & (fref.hi <= fref.m64 + tol)
    sub = [np.ascontiguousarray(a[good]) for a in (w.type, w.value, w.size)]
    pop_sub = tgp.Population(*(torch.from_numpy(a).to(DEV) for a in sub))
    _, _, gxs = tgp.eval_mse_grad(pop_sub, X, Yd, config=tgp.cfg(mode=2, points_per_lane=k))
    torch.cuda.synchronize()
    rep_xs = compare_grad_x(gxs.cpu().numpy(), GradRef(*sub, w.X, Y), label=name + " well-determined")
    print(f"  grad_X over the {int(good.sum())} well-determined trees {rep_xs}", flush=True)
    assert rep_xs["tight"] >= 0.25 * rep_xs["n"], rep_xs


def test_grad_vs_finite_differences():
    """Device constant gradients against central differences of the float64 fitness (h = 1e-4)
    on sampled constants whose float32 envelope is within 1e-3 of the float64 gradient; the
    difference quotient's own error is estimated from h and h/4 and allowed for."""
    w, Y = work("grad", P=300, D=3100)
    pop = dev_pop(w)
    X = torch.from_numpy(w.X).to(DEV)
    Yd = torch.from_numpy(Y).to(DEV)
    _, gv, _ = tgp.eval_mse_grad(pop, X, Yd)
    gv = gv.cpu().numpy()
    ref = grad_ref("grad", w, Y)
    tol = 1e-3 * np.abs(ref.gv64)
    with np.errstate(invalid="ignore"):
        tight = ref.const & ~ref.gv_nan & (ref.gv_lo >= ref.gv64 - tol) & (ref.gv_hi <= ref.gv64 + tol)
    rng = np.random.default_rng(0)
    cand = np.argwhere(tight & (np.abs(ref.gv64) > 1e-6))
    checked = 0
    for p, i in cand[rng.choice(len(cand), size=min(100, len(cand)), replace=False)]:
        if not (ref.m64[p] < 1e4):
            continue                    # the difference quotient cancels badly on huge fitness values
        f1 = O.fd_grad_const(w.type, w.value, w.size, w.X, Y, p, i, h=1e-4)
        f2 = O.fd_grad_const(w.type, w.value, w.size, w.X, Y, p, i, h=2.5e-5)
        fd_err = abs(f1 - f2)           # the quotient at h/4 is within about this of the derivative
        assert abs(gv[p, i] - f2) <= 1e-3 * abs(f2) + 2.0 * fd_err + 1e-9, (p, i, gv[p, i], f1, f2)
        checked += 1
    assert checked >= 50


def test_autograd_matches_direct_call():
    """TreeMSE backward with upstream weights equals the direct call's gradients up to the order
    of the float32 sums: both inside the envelopes of the weighted gradients."""
    w, Y = work("grad", P=200, D=2000)
    value = torch.from_numpy(w.value.copy()).to(DEV).requires_grad_(True)
    type_ = torch.from_numpy(w.type).to(DEV)
    size = torch.from_numpy(w.size).to(DEV)
    X = torch.from_numpy(w.X).to(DEV).requires_grad_(True)
    Yd = torch.from_numpy(Y).to(DEV)
    mse = tgp.TreeMSE.apply(value, type_, size, X, Yd)
    wt = np.linspace(0.5, 1.5, w.P).astype(np.float32)
    (mse * torch.from_numpy(wt).to(DEV)).sum().backward()
    pop = tgp.Population(type_, value.detach(), size)
    _, gv, gx = tgp.eval_mse_grad(pop, X.detach(), Yd, grad_mse=torch.from_numpy(wt).to(DEV))
    ref = grad_ref("grad-weighted", w, Y, g=wt)
    for label, a, b in (("autograd", value.grad, X.grad), ("direct", gv, gx)):
        compare_grad_value(a.cpu().numpy(), ref, label)
        compare_grad_x(b.cpu().numpy(), ref, label)


def _adam_with_checks(w, Y, rows_per_step, steps=10, lr=1e-2, value_rows=None):
    """Adam (torch.optim.Adam, lr 1e-2) on the constants through TreeMSE. Before every step the
    device gradient of the checked rows is compared with the oracle's envelopes at the device's
    current constants. Returns the first and last fitness."""
    value = torch.from_numpy(w.value.copy()).to(DEV).requires_grad_(True)
    type_ = torch.from_numpy(w.type).to(DEV)
    size = torch.from_numpy(w.size).to(DEV)
    X = torch.from_numpy(w.X).to(DEV)
    Yd = torch.from_numpy(Y).to(DEV)
    opt = torch.optim.Adam([value], lr=lr)
    m_first = None
    for step in range(steps):
        opt.zero_grad()
        mse = tgp.TreeMSE.apply(value, type_, size, X, Yd)
        mse.sum().backward()
        torch.cuda.synchronize()
        if m_first is None:
            m_first = mse.detach().cpu().numpy()
        rows = rows_per_step(step)
        cur = value.detach().cpu().numpy()
        ref = GradRef(w.type, cur, w.size, w.X, Y, rows=rows)
        compare_fitness(mse.detach().cpu().numpy()[rows], FitnessRef(w.type, cur, w.size, w.X, Y, rows=rows),
                        label=f"Adam step {step} fitness")
        rep = compare_grad_value(value.grad.cpu().numpy()[rows], ref, label=f"Adam step {step}")
        print(f"step {step}: {len(rows)} trees, grad_value {rep}", flush=True)
        opt.step()
    m_last = tgp.TreeMSE.apply(value.detach(), type_, size, X, Yd).cpu().numpy()
    return value.detach().cpu().numpy(), m_first, m_last


def test_adam_steps_with_gradient_checks():
    w, Y = work("grad", P=200, D=2000)
    vv, m0, m1 = _adam_with_checks(w, Y, lambda step: list(range(w.P)))
    # padding and non-constant fields never move; NaN stays NaN
    fixed = w.type != 1
    np.testing.assert_array_equal(np.isnan(vv), np.isnan(w.value))
    keep = fixed & ~np.isnan(w.value)
    assert np.array_equal(vv[keep], w.value[keep])
    fin = np.isfinite(m0) & np.isfinite(m1) & ((w.type == 1).sum(1) > 0)
    assert (m1[fin] <= m0[fin] * (1 + 1e-6)).mean() > 0.8


def test_graph_replay_matches_eager():
    w, Y = work("hybrid", P=600, D=2000)
    pop = dev_pop(w)
    X = torch.from_numpy(w.X).to(DEV)
    Yd = torch.from_numpy(Y).to(DEV)
    ws = tgp.Workspace(DEV)
    out = torch.empty(w.P, device=DEV)
    c = tgp.cfg(mode=3, points_per_lane=4, trees_per_unit=4)
    eager = tgp.eval_mse(pop, X, Yd, config=c, ws=ws).cpu().numpy()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tgp.eval_mse(pop, X, Yd, config=c, ws=ws, out=out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        tgp.eval_mse(pop, X, Yd, config=c, ws=ws, out=out)
    for _ in range(4):
        out.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        np.testing.assert_allclose(got, eager, rtol=1e-6, atol=0, equal_nan=True)
        _ = tgp.eval_mse(pop, X, Yd, config=tgp.cfg(mode=1), ws=tgp.Workspace(DEV))   # eager work between replays


@pytest.mark.parametrize("cfg", [dict(block_waves=1, trees_per_unit=1), dict(block_waves=2, trees_per_unit=4),
                                 dict(block_waves=4, trees_per_unit=64),
                                 dict(points_per_lane=2, block_waves=1, trees_per_unit=4),
                                 dict(points_per_lane=2, block_waves=4, trees_per_unit=16),
                                 dict(points_per_lane=4, block_waves=1, trees_per_unit=16), "tuned"])
def test_grad_launch_shapes_agree(cfg):
    """Every workgroup shape and trees-per-unit choice of the gradient call, and the autotuned one
    (tgp_autotune with want_grad, then a call without a configuration): fitness and gradients
    inside the oracle's envelopes."""
    w, Y = work("grad", P=300, D=3100)
    pop = dev_pop(w)
    X = torch.from_numpy(w.X).to(DEV)
    Yd = torch.from_numpy(Y).to(DEV)
    if cfg == "tuned":
        tuned = tgp.autotune(pop, X, Yd, want_grad=True)
        print(f"tuned gradient launch: {tuned}", flush=True)
        assert tuned["mode"] == 2 and tuned["points_per_lane"] in (2, 3, 4)
        got = tgp.eval_mse_grad(pop, X, Yd)
    else:
        got = tgp.eval_mse_grad(pop, X, Yd, config=tgp.cfg(mode=2, **cfg))
    torch.cuda.synchronize()
    mse, gv, gx = (t.cpu().numpy() for t in got)
    ref = grad_ref("grad", w, Y)
    compare_fitness(mse, FitnessRef(w.type, w.value, w.size, w.X, Y), label=f"{cfg} fitness")
    compare_grad_value(gv, ref, label=str(cfg))
    compare_grad_x(gx, ref, label=str(cfg))


@pytest.mark.parametrize("k", [2, 3, 4])
def test_path_and_recompute_sweeps_agree(k):
    """The heavy-path sweep and the recompute sweep (TGP_FLAG_ADJ_RECOMPUTE) on the same trees:
    the fitness comes from the same forward run and is bitwise equal; the gradients differ only
    in the order of float32 sums, and both lie inside the oracle's envelopes."""
    w, Y = work("hybrid", P=250, D=2000)
    pop = dev_pop(w)
    X = torch.from_numpy(w.X).to(DEV)
    Yd = torch.from_numpy(Y).to(DEV)
    ref = grad_ref("hybrid", w, Y)
    res = {}
    for name, flags in (("path", 0), ("recompute", 4)):
        got = tgp.eval_mse_grad(pop, X, Yd, config=tgp.cfg(mode=2, points_per_lane=k, flags=flags))
        torch.cuda.synchronize()
        res[name] = [t.cpu().numpy() for t in got]
        compare_grad_value(res[name][1], ref, label=name)
        compare_grad_x(res[name][2], ref, label=name)
    np.testing.assert_array_equal(res["path"][0].view(np.uint32), res["recompute"][0].view(np.uint32))


def test_deep_trees_mix_both_sweeps():
    """Single-output trees of the batched recipe (exact lengths up to 1024, Lmax 1024): the deep
    ones need more than the heavy-path sweep's LDS budget and go to the recompute sweep, the rest
    to the heavy-path sweep, in one call. Fitness and gradients inside the envelopes."""
    wb = synth.workload("batched", P=160, D=700)
    plain = np.setdiff1d(np.arange(wb.P), wb.meta["modi_trees"])
    sub = [np.ascontiguousarray(a[plain]) for a in (wb.type, wb.value, wb.size)]
    # target: the first hidden tree plus its noise row
    hp = O.predict(*(np.ascontiguousarray(h[:1]) for h in wb.hidden), wb.X, 1)[0, 0]
    Y = (hp + wb.noise[0].astype(np.float64)).astype(np.float32)[None, :]
    # heavy-path values the sweep holds per tree (the plan's budget is 16)
    lengths = sub[2][:, 0]
    assert lengths.max() > 600
    pop = tgp.Population(*(torch.from_numpy(a).to(DEV) for a in sub))
    X = torch.from_numpy(wb.X).to(DEV)
    Yd = torch.from_numpy(Y).to(DEV)
    mse, gv, gx = (t.cpu().numpy() for t in tgp.eval_mse_grad(pop, X, Yd, config=tgp.cfg(mode=2, points_per_lane=2)))
    compare_fitness(mse, FitnessRef(*sub, wb.X, Y), label="deep fitness")
    ref = GradRef(*sub, wb.X, Y)
    rep_v = compare_grad_value(gv, ref, label="deep")
    rep_x = compare_grad_x(gx, ref, label="deep")
    print(f"deep trees: grad_value {rep_v}\n  grad_X {rep_x}", flush=True)


def _multi_output_case(w, Y, k, label):
    pop = dev_pop(w)
    X = torch.from_numpy(w.X).to(DEV)
    Yd = torch.from_numpy(Y).to(DEV)
    mse, gv, gx = (t.cpu().numpy() for t in tgp.eval_mse_grad(pop, X, Yd, config=tgp.cfg(mode=2, points_per_lane=k)))
    compare_fitness(mse, FitnessRef(w.type, w.value, w.size, w.X, Y, w.n_out), label=f"{label} fitness")
    ref = GradRef(w.type, w.value, w.size, w.X, Y, w.n_out)
    rep_v = compare_grad_value(gv, ref, label=label)
    rep_x = compare_grad_x(gx, ref, label=label)
    print(f"{label} K={k}: grad_value {rep_v}\n  grad_X {rep_x}", flush=True)
    return gv, ref, rep_v


@pytest.mark.parametrize("k", [2, 3, 4])
def test_multi_output_gradients(k):
    """Gradients of multi-output trees (§IV-C): the classification recipe's trees (every one with
    Modi nodes for 3 outputs, depth <= 6, 13 variables) against 3 rows of regression targets.
    Fitness sums the outputs' mean squared errors; a Modi node passes the adjoint of its own output
    to its children. Fitness and gradients inside the oracle's envelopes."""
    w = synth.workload("classify", P=400, D=600)
    Y = np.random.default_rng(9).normal(size=(w.n_out, w.D)).astype(np.float32)
    gv, ref, rep_v = _multi_output_case(w, Y, k, "multi-output")
    assert np.any(gv[ref.const] != 0)
    assert rep_v["tight"] >= 0.25 * rep_v["n"], rep_v


def test_multi_output_gradients_long_trees():
    """The batched recipe's population (lengths up to 1024, 10% Modi trees with 3 outputs, the rest
    plain trees predicting (root, 0, 0)): most trees exceed the heavy-path budget, so both sweeps
    run with four output adjoints. Every value inside its envelope; long trees leave few envelopes
    within the 1e-3 bar (about 15% of the constant gradients here)."""
    w, Y = work("batched", P=120, D=600)
    assert w.n_out == 3 and len(w.meta["modi_trees"]) > 5
    gv, ref, rep_v = _multi_output_case(w, Y, 2, "multi-output long")
    modi = np.asarray(w.meta["modi_trees"])
    assert np.any(gv[modi][ref.const[modi]] != 0)
    assert rep_v["tight"] >= 0.1 * rep_v["n"], rep_v


def _complete_tree_var_const(depth, rng, Lmax):
    """Complete binary tree of the given depth over + - * (mostly + and -, so values stay finite);
    every bottom node combines a variable (first child) and a constant (second child)."""
    nodes = []

    def rec(d, first):
        if d == depth:
            nodes.append((0, int(rng.integers(0, 2)), 1) if first else (1, float(rng.uniform(-1, 1)), 1))
            return 1
        i = len(nodes)
        nodes.append(None)
        n = 1 + rec(d + 1, True) + rec(d + 1, False)
        nodes[i] = (2, int(rng.choice([0, 1, 2], p=[0.45, 0.45, 0.1])), n)
        return n

    rec(0, True)
    t = np.full(Lmax, np.nan, np.float32)
    v, s = t.copy(), t.copy()
    for i, (a, b, c) in enumerate(nodes):
        t[i], v[i], s[i] = a, b, c
    return t, v, s


def test_deep_complete_trees_gradients():
    """Complete trees of depth 8 and 9 (up to 1,023 nodes) whose bottom nodes combine a variable
    and a constant: each bottom node is one word (the variable pre-loaded, the constant in the
    payload) and carries the capture level of its parent, up to 9. Runs of the sweeps then start on
    words whose level sets bit 31, with a constant payload that must survive the interpreter's
    widening of its first word. Both sweeps, 2 to 4 points per lane; fitness and gradients inside
    the oracle's envelopes."""
    r = np.random.default_rng(21)
    Lmax = 1024
    rows = [_complete_tree_var_const(9, r, Lmax) for _ in range(3)] + [_complete_tree_var_const(8, r, Lmax)]
    T, V, S = (np.stack([x[i] for x in rows]) for i in range(3))
    D = 300
    X = r.uniform(-1, 1, (2, D)).astype(np.float32)
    Y = r.normal(size=(1, D)).astype(np.float32)
    pop = tgp.Population(*(torch.from_numpy(a).to(DEV) for a in (T, V, S)))
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    fref = FitnessRef(T, V, S, X, Y)
    ref = GradRef(T, V, S, X, Y)
    for k in (2, 3, 4):
        for flags in (0, 4):
            label = f"complete K={k} flags={flags}"
            mse, gv, gx = (t.cpu().numpy() for t in
                           tgp.eval_mse_grad(pop, Xd, Yd, config=tgp.cfg(mode=2, points_per_lane=k, flags=flags)))
            assert np.isfinite(mse).all(), label
            compare_fitness(mse, fref, label=label)
            compare_grad_value(gv, ref, label=label)
            compare_grad_x(gx, ref, label=label)
