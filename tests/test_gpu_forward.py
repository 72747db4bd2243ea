"""Device parity of the plan and forward kernels against the CPU oracle, called
through the C-ABI (Python binding). Needs an MI355X."""

import numpy as np
import pytest
import torch

import oracle as O
import paper_2501_17168_amd as tgp
import synth
from golden_io import load_tree
from parity import FitnessRef, compare_fitness, inside
from oracle import envelope as E

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

# scaled-down instances of every workload recipe: several tiles and a ragged tail
SMALL = {"plain": dict(), "hybrid": dict(P=600, D=2000), "dataparallel": dict(P=40, D=9000),
         "batched": dict(P=500, D=1000), "grad": dict(P=500, D=3100), "pagie": dict(P=400, D=2000)}
_cache = {}


def work(name, **kw):
    key = (name, tuple(sorted(kw.items())))
    if key not in _cache:
        w = synth.workload(name, **kw)
        Y = w.Y if w.Y is not None else w.targets_from(O.predict(*w.hidden, w.X, 1)[:, 0, :])
        _cache[key] = (w, Y)
    return _cache[key]


def to_dev(w, Y):
    pop = tgp.Population(*(torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (w.type, w.value, w.size)))
    return pop, torch.from_numpy(w.X).to(DEV), torch.from_numpy(np.ascontiguousarray(Y)).to(DEV)


_refs = {}


def oracle_fit(name, w, Y):
    """float64 fitness and float32 envelopes of a workload's trees (cached per workload)."""
    key = (name, w.P, w.D)
    if key not in _refs:
        _refs[key] = FitnessRef(w.type, w.value, w.size, w.X, Y, w.n_out)
    return _refs[key]


def device_fit(pop, X, Y, n_out, config=None):
    if n_out == 1:
        m = tgp.eval_mse(pop, X, Y, config=config)
    else:
        m, _ = tgp.eval_multi_output(pop, X, Y, config=config)
    torch.cuda.synchronize()
    return m.cpu().numpy()


@pytest.mark.parametrize("name", list(SMALL))
def test_plan_bitexact(name):
    w, _ = work(name, **SMALL[name])
    pop, X, Y = to_dev(w, w.noise)
    info, st = tgp.plan(pop, w.V, w.n_out)
    torch.cuda.synchronize()
    ref = O.plan(w.type, w.value, w.size, w.V, w.n_out)
    np.testing.assert_array_equal(info.cpu().numpy(), ref)
    np.testing.assert_array_equal(st.cpu().numpy(), ref[:, 0])


def _faulty_population():
    """The validator fault list (one tree per fault), plus valid trees, Lmax 12."""
    base = [(2, 0, 7), (0, 0, 1), (2, 0, 5), (0, 1, 1), (2, 0, 3), (0, 0, 1), (0, 1, 1)]
    Lmax = 12
    rows = []

    def mk(mut=None):
        t = np.full(Lmax, np.nan, np.float32)
        v = np.full(Lmax, np.nan, np.float32)
        s = np.full(Lmax, np.nan, np.float32)
        for i, (a, b, c) in enumerate(base):
            t[i], v[i], s[i] = a, b, c
        if mut:
            mut(t, v, s)
        rows.append((t, v, s))

    mk()
    mk(lambda t, v, s: s.__setitem__(0, 13.0))
    mk(lambda t, v, s: s.__setitem__(0, 6.5))
    mk(lambda t, v, s: s.__setitem__(0, np.nan))
    mk(lambda t, v, s: v.__setitem__(3, np.nan))
    mk(lambda t, v, s: t.__setitem__(9, 0.0))
    mk(lambda t, v, s: t.__setitem__(2, 2.5))
    mk(lambda t, v, s: t.__setitem__(2, 5.0))
    mk(lambda t, v, s: v.__setitem__(2, 12.0))
    mk(lambda t, v, s: v.__setitem__(3, 2.0))
    mk(lambda t, v, s: v.__setitem__(3, 0.5))
    mk(lambda t, v, s: s.__setitem__(4, 2.0))
    mk(lambda t, v, s: s.__setitem__(1, 1.5))
    mk(lambda t, v, s: v.__setitem__(2, 4.0))
    mk(lambda t, v, s: (v.__setitem__(3, np.nan), t.__setitem__(10, 1.0)))
    mk(lambda t, v, s: (v.__setitem__(3, 7.0), v.__setitem__(2, 20.0)))
    mk(lambda t, v, s: t.__setitem__(2, 3.0))                     # Modi(0): valid with n_out >= 1
    T = np.stack([r[0] for r in rows])
    Vv = np.stack([r[1] for r in rows])
    S = np.stack([r[2] for r in rows])
    return T, Vv, S


def test_invalid_trees_status_and_nan():
    T, Vv, S = _faulty_population()
    ref = O.plan(T, Vv, S, 2, 1)
    assert len(set(ref[:, 0].tolist())) >= 8
    pop = tgp.Population(*(torch.from_numpy(a).to(DEV) for a in (T, Vv, S)))
    info, st = tgp.plan(pop, 2, 1)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(info.cpu().numpy(), ref)
    X = np.random.default_rng(0).normal(size=(2, 300)).astype(np.float32)
    Y = np.random.default_rng(1).normal(size=(1, 300)).astype(np.float32)
    stt = torch.empty(len(T), dtype=torch.int32, device=DEV)
    m = tgp.eval_mse(pop, torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV), tree_status=stt).cpu().numpy()
    np.testing.assert_array_equal(stt.cpu().numpy(), ref[:, 0])
    valid = ref[:, 0] == 0
    assert np.isnan(m[~valid]).all()
    compare_fitness(m, FitnessRef(T, Vv, S, X, Y), label="the fault list")


MODES = [("tree", dict(mode=1)), ("tree-bw1", dict(mode=1, block_waves=1)), ("point", dict(mode=2)),
         ("point-tpu7", dict(mode=2, trees_per_unit=7)), ("persist", dict(mode=3)),
         ("persist-tpu1", dict(mode=3, trees_per_unit=1)),
         ("persist-tpu3-bw2", dict(mode=3, trees_per_unit=3, block_waves=2)),
         ("persist-static-tpu2", dict(mode=3, trees_per_unit=2, flags=2))]


@pytest.mark.parametrize("K", [16, 8, 4])
@pytest.mark.parametrize("mode", [m[0] for m in MODES])
@pytest.mark.parametrize("name", list(SMALL))
def test_forward_parity(name, mode, K):
    w, Y = work(name, **SMALL[name])
    pop, X, Yd = to_dev(w, Y)
    c = dict(dict(MODES)[mode])
    c["points_per_lane"] = K
    got = device_fit(pop, X, Yd, w.n_out, tgp.cfg(**c))
    rep = compare_fitness(got, oracle_fit(name, w, Y), label=f"{name}/{mode}/K{K}")
    print(f"{name}/{mode}/K{K}: {rep}")
    assert rep["tight"] >= 0.5 * rep["n"], rep


def test_multi_output_predictions():
    w, Y = work("batched", P=300, D=700)
    pop, X, Yd = to_dev(w, Y)
    m, pred = tgp.eval_multi_output(pop, X, Yd, want_pred=True)
    torch.cuda.synchronize()
    pred = pred.cpu().numpy().astype(np.float64)
    # every prediction inside its float32 envelope (per tree, output and point)
    tight = total = 0
    ref = O.predict(w.type, w.value, w.size, w.X, 3)
    for p in range(w.P):
        outs, _ = E.forward(O.decode(w.type[p], w.value[p], w.size[p], w.V, 3), w.X, 3)
        for o in range(3):
            ok = inside(pred[p, o], outs[o].lo, outs[o].hi, outs[o].nan)
            assert ok.all(), (p, o, np.nonzero(~ok)[0][:5], pred[p, o][~ok][:5], outs[o].lo[~ok][:5],
                              outs[o].hi[~ok][:5])
            scale = np.maximum(np.abs(ref[p, o]), 1.0)
            with np.errstate(invalid="ignore"):
                tight += int(((outs[o].lo >= ref[p, o] - 1e-5 * scale) & (outs[o].hi <= ref[p, o] + 1e-5 * scale)).sum())
            total += w.D
    print(f"predictions: {tight}/{total} with an envelope within 1e-5 of float64")
    assert tight >= 0.8 * total
    m_ref = FitnessRef(w.type, w.value, w.size, w.X, Y, 3)
    compare_fitness(m.cpu().numpy(), m_ref, label="multi-output fitness")
    modi = w.meta["modi_trees"]
    assert len(modi) > 10
    # plain trees predict zeros for outputs 1 and 2
    plain = np.setdiff1d(np.arange(w.P), modi)
    assert (pred[plain][:, 1:] == 0).all()
    # prediction-only call (no targets)
    _, pred2 = tgp.eval_multi_output(pop, X, None, n_out=3, want_pred=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(pred2.cpu().numpy(), pred.astype(np.float32))


def test_worked_examples_on_device():
    (t, v, s), rows = load_tree("modi_tree.txt")
    pts = np.array(rows["point"])
    X = np.ascontiguousarray(pts[:, :5].T.astype(np.float32))
    pop = tgp.Population(*(torch.from_numpy(a[None].copy()).to(DEV) for a in (t, v, s)))
    _, pred = tgp.eval_multi_output(pop, torch.from_numpy(X).to(DEV), None, n_out=3, want_pred=True)
    np.testing.assert_allclose(pred.cpu().numpy()[0], pts[:, 5:].T, rtol=1e-6, atol=1e-6)
    (t, v, s), rows = load_tree("sigmoid_tree.txt")
    vals = np.array(rows["value"])
    pop = tgp.Population(*(torch.from_numpy(a[None].copy()).to(DEV) for a in (t, v, s)))
    X = torch.from_numpy(vals[:, :1].T.astype(np.float32).copy()).to(DEV)
    _, pred = tgp.eval_multi_output(pop, X, None, n_out=1, want_pred=True)
    np.testing.assert_allclose(pred.cpu().numpy()[0, 0], vals[:, 1], rtol=1e-6)


def _complete_tree(depth, rng, Lmax):
    """Complete binary tree of the given depth (leaves at depth `depth`), + - * only:
    needs depth-1 spill slots, so depth 9 (1023 nodes) exercises all 8."""
    nodes = []

    def rec(d):
        if d == depth:
            nodes.append((0, int(rng.integers(0, 2)), 1))
            return 1
        i = len(nodes)
        nodes.append(None)
        n = 1 + rec(d + 1) + rec(d + 1)
        nodes[i] = (2, int(rng.choice([0, 1, 2])), n)
        return n

    rec(0)
    t = np.full(Lmax, np.nan, np.float32)
    v = np.full(Lmax, np.nan, np.float32)
    s = np.full(Lmax, np.nan, np.float32)
    for i, (a, b, c) in enumerate(nodes):
        t[i], v[i], s[i] = a, b, c
    return t, v, s


@pytest.mark.parametrize("K", [16, 8, 4])
def test_edge_shapes(K):
    r = np.random.default_rng(5)
    Lmax = 1024
    rows = [_complete_tree(d, r, Lmax) for d in (9, 8, 6, 5, 1)]
    for kind, val in ((0, 1), (1, 2.5)):                             # single-node trees
        t = np.full(Lmax, np.nan, np.float32); v = t.copy(); s = t.copy()
        t[0], v[0], s[0] = kind, val, 1
        rows.append((t, v, s))
    T = np.stack([x[0] for x in rows]); Vv = np.stack([x[1] for x in rows]); S = np.stack([x[2] for x in rows])
    for D in (1, 63, 64 * K + 1, 3 * 64 * K - 5):
        X = r.uniform(-1, 1, size=(2, D)).astype(np.float32)
        Y = r.normal(size=(1, D)).astype(np.float32)
        pop = tgp.Population(*(torch.from_numpy(a).to(DEV) for a in (T, Vv, S)))
        ref = FitnessRef(T, Vv, S, X, Y)
        for mode in (1, 2, 3):
            got = device_fit(pop, torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV), 1,
                             tgp.cfg(mode=mode, points_per_lane=K))
            compare_fitness(got, ref, label=f"D={D} mode={mode}")


# every schedule, the dynamic persistent queue included: per-(tree, tile) partials summed in a fixed
# order make the fitness independent of which wave finished first
REPEAT_SCHEDULES = [None, dict(mode=1, points_per_lane=4, block_waves=4),
                    dict(mode=2, points_per_lane=8, block_waves=4, trees_per_unit=16),
                    dict(mode=3, points_per_lane=8, block_waves=1, trees_per_unit=1),
                    dict(mode=3, points_per_lane=4, block_waves=4, trees_per_unit=2, flags=2)]


@pytest.mark.parametrize("sched", REPEAT_SCHEDULES, ids=["default", "tree", "point", "persistent", "static"])
def test_repeat_runs_identical(sched):
    w, Y = work("hybrid", **SMALL["hybrid"])
    pop, X, Yd = to_dev(w, Y)
    c = tgp.cfg(sched) if sched else None
    runs = [device_fit(pop, X, Yd, 1, config=c) for _ in range(4)]
    for r in runs[1:]:
        np.testing.assert_array_equal(r.view(np.uint32), runs[0].view(np.uint32))


def test_repeat_runs_identical_multi_output():
    w, Y = work("batched", **SMALL["batched"])
    pop, X, Yd = to_dev(w, Y)
    c = tgp.cfg(mode=3, points_per_lane=8, block_waves=1, trees_per_unit=1)
    runs = [device_fit(pop, X, Yd, w.n_out, config=c) for _ in range(3)]
    for r in runs[1:]:
        np.testing.assert_array_equal(r.view(np.uint32), runs[0].view(np.uint32))


def test_strided_rows_and_views():
    w, Y = work("plain")
    Lpad = w.Lmax + 7
    big = [np.full((w.P, Lpad), np.nan, np.float32) for _ in range(3)]
    for b, a in zip(big, (w.type, w.value, w.size)):
        b[:, :w.Lmax] = a
    tens = [torch.from_numpy(b).to(DEV)[:, :w.Lmax] for b in big]
    pop = tgp.Population(*tens)
    Xw = torch.zeros((w.V, w.D + 33), device=DEV)
    Xw[:, :w.D] = torch.from_numpy(w.X).to(DEV)
    got = device_fit(pop, Xw[:, :w.D], torch.from_numpy(Y).to(DEV), 1)
    compare_fitness(got, oracle_fit("plain", w, Y), label="strided")


def _encode(node, rows):
    """Prefix-encode a nested tuple tree into (type, value, size) rows: ("x", i), ("c", v) or
    ("f", op, modi_output_or_None, *children)."""
    t, v, s = rows
    k = len(t)
    t.append(0.0); v.append(0.0); s.append(0.0)
    if node[0] == "x":
        t[k], v[k] = 0.0, float(node[1])
    elif node[0] == "c":
        t[k], v[k] = 1.0, float(node[1])
    else:
        t[k] = 2.0 if node[2] is None else 3.0 + node[2]
        v[k] = float(node[1])
        for ch in node[3:]:
            _encode(ch, rows)
    s[k] = float(len(t) - k)


def _folding_trees():
    """Trees for every way a unary node is folded into the forward program: into its binary
    child's last word (a fused op word, a pre-loaded one, a Modi child's ACC), as the second action
    of a load (of a constant or a variable) or of a binary node's last word, Modi or not, at the
    program's first word or after a spill, chains of 2 to 5 unary nodes, a folded root (whose
    child's word then ends the program) and leaf roots."""
    SIN, COS, TANH, EXP, LOG, TAN = 4, 5, 6, 7, 8, 11
    ADD, SUB, MUL, DIV, MAX = 0, 1, 2, 3, 9
    x = lambda i: ("x", i)
    c = lambda v: ("c", v)
    f = lambda op, *ch, m=None: ("f", op, m, *ch)
    big = f(MUL, f(MUL, x(0), x(1)), f(ADD, x(2), x(0)))
    return [
        f(EXP, f(ADD, f(SIN, f(SIN, c(-4.537)), m=2), f(TANH, f(TANH, x(2), m=1))), m=0),
        f(EXP, f(SIN, f(LOG, f(LOG, x(1))))),
        f(SIN, f(COS, f(ADD, c(0.3), c(0.9)))),
        f(SIN, f(COS, f(MUL, x(0), c(0.5)))),
        f(ADD, f(TANH, f(EXP, f(DIV, x(0), x(1))), m=1), x(2)),
        f(TAN, f(SUB, x(0), x(1))),
        f(COS, f(SIN, f(ADD, x(0), x(1)), m=1), m=2),
        f(SIN, f(ADD, x(0), x(1), m=0)),
        f(LOG, c(2.5)),
        f(EXP, f(LOG, c(-3.0), m=1), m=0),
        f(SIN, f(COS, f(TANH, f(EXP, f(LOG, f(MUL, x(0), x(1))))))),
        c(1.25),
        x(2),
        f(ADD, big, f(SIN, f(COS, c(0.7)))),
        f(ADD, big, f(SIN, f(COS, c(-1.1)), m=2)),
        f(MAX, big, f(TANH, f(COS, f(SUB, x(1), c(0.25))), m=1), m=0),
        f(SIN, f(COS, f(TANH, c(0.4)))),
        f(EXP, f(TANH, f(ADD, x(0), x(1), m=2), m=1)),
    ]


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_unary_folding_patterns(mode):
    """Every prediction of the folding trees inside its float32 envelope (and close to float64),
    under each schedule; the first-word constant loads carry a second Modi action, whose word has
    bit 31 set."""
    trees = _folding_trees()
    L = 32
    T = np.full((len(trees), L), np.nan, np.float32)
    V, S = T.copy(), T.copy()
    for p, tr in enumerate(trees):
        rows = ([], [], [])
        _encode(tr, rows)
        n = len(rows[0])
        T[p, :n], V[p, :n], S[p, :n] = rows
    rng = np.random.default_rng(11)
    D = 700
    X = rng.uniform(-2.0, 2.0, (3, D)).astype(np.float32)
    pop = tgp.Population(*(torch.from_numpy(a).to(DEV) for a in (T, V, S)))
    _, pred = tgp.eval_multi_output(pop, torch.from_numpy(X).to(DEV), None, n_out=3, want_pred=True,
                                    config=tgp.cfg(mode=mode))
    torch.cuda.synchronize()
    pred = pred.cpu().numpy().astype(np.float64)
    ref = O.predict(T, V, S, X, 3)
    for p in range(len(trees)):
        outs, _ = E.forward(O.decode(T[p], V[p], S[p], 3, 3), X, 3)
        for o in range(3):
            ok = inside(pred[p, o], outs[o].lo, outs[o].hi, outs[o].nan)
            assert ok.all(), (p, o, np.nonzero(~ok)[0][:5], pred[p, o][~ok][:5], ref[p, o][~ok][:5])
            scale = np.maximum(np.abs(ref[p, o]), 1.0)
            assert np.all(np.abs(pred[p, o] - ref[p, o]) <= 1e-4 * scale), (p, o)
