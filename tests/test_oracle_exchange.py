"""Pins for the subtree-exchange oracle (§III-B), checked against things
other than the oracle's own splice: hand-derived trees, an independent
tree-structured construction (parse to nested nodes, substitute, print back
with recomputed sizes), the validity rules of the encoding (§III-A), the
length limit, and the operators the paper builds on the primitive."""

import numpy as np
import pytest

import oracle as O
from synth import trees as ST

NAN = np.nan
ARITY = {0: 2, 1: 2, 2: 2, 3: 2, 4: 1, 5: 1, 6: 1, 7: 1, 8: 1, 9: 2, 10: 2, 11: 1}


def rows(nodes, L):
    """(type, value) pairs in prefix order -> padded rows with sizes from a recursive count."""
    t = [a for a, _ in nodes]
    v = [b for _, b in nodes]
    size = [0] * len(nodes)

    def walk(i):
        n = 1
        j = i + 1
        for _ in range(0 if t[i] in (0, 1) else ARITY[int(v[i])]):
            c = walk(j)
            n += c
            j += c
        size[i] = n
        return n

    walk(0)
    out = [np.full(L, np.nan, np.float32) for _ in range(3)]
    for r, src in zip(out, (t, v, size)):
        r[:len(nodes)] = src
    return out


# (x0 + 2.5) * sin(x1): mul add x0 2.5 sin x1
OLD = [(2, 2), (2, 0), (0, 0), (1, 2.5), (2, 4), (0, 1)]
# x0 - x1: sub x0 x1
NEW = [(2, 1), (0, 0), (0, 1)]


def test_hand_example_replace_unary_subtree():
    """Node 4 (the sin subtree, 2 nodes) replaced by a 3-node tree: dn = +1 is added to
    the root only (the sole ancestor), the add subtree keeps its size."""
    L = 8
    old = rows(OLD, L)
    new = rows(NEW, L)
    (t, v, s), st = O.subtree_exchange([r[None] for r in old], [r[None] for r in new], [4])
    assert st[0] == O.X_OK
    exp_t = [2, 2, 0, 1, 2, 0, 0, NAN]
    exp_v = [2, 0, 0, 2.5, 1, 0, 1, NAN]
    exp_s = [7, 3, 1, 1, 3, 1, 1, NAN]
    np.testing.assert_array_equal(t[0], np.float32(exp_t))
    np.testing.assert_array_equal(v[0], np.float32(exp_v))
    np.testing.assert_array_equal(s[0], np.float32(exp_s))


def test_hand_example_shrink_inner_leaf():
    """Node 2 (x0, inside the add subtree) replaced by the constant 7: both ancestors (the
    add node and the root) change by dn = 0; then the add subtree (node 1, 3 nodes) replaced
    by x1 shrinks the root by 2."""
    L = 6
    old = rows(OLD, L)
    const = rows([(1, 7.0)], L)
    (t, v, s), st = O.subtree_exchange([r[None] for r in old], [r[None] for r in const], [2])
    assert st[0] == O.X_OK
    np.testing.assert_array_equal(v[0], np.float32([2, 0, 7.0, 2.5, 4, 1]))
    np.testing.assert_array_equal(t[0], np.float32([2, 2, 1, 1, 2, 0]))
    np.testing.assert_array_equal(s[0], old[2])
    x1 = rows([(0, 1)], L)
    (t, v, s), st = O.subtree_exchange([r[None] for r in old], [r[None] for r in x1], [1])
    assert st[0] == O.X_OK
    np.testing.assert_array_equal(t[0], np.float32([2, 0, 2, 0, NAN, NAN]))
    np.testing.assert_array_equal(v[0], np.float32([2, 1, 4, 1, NAN, NAN]))
    np.testing.assert_array_equal(s[0], np.float32([4, 1, 2, 1, NAN, NAN]))


def test_length_limit_boundary():
    """The result of OLD with node 4 replaced has 7 nodes: accepted at max_len 7, refused
    at 6 with the old tree returned unchanged (§III-B)."""
    L = 8
    old = [r[None] for r in rows(OLD, L)]
    new = [r[None] for r in rows(NEW, L)]
    _, st = O.subtree_exchange(old, new, [4], max_len=7)
    assert st[0] == O.X_OK
    out, st = O.subtree_exchange(old, new, [4], max_len=6)
    assert st[0] == O.X_TOO_LONG
    for a, b in zip(out, old):
        np.testing.assert_array_equal(a[0], b[0])


# ---------------------------------------------------------- independent construction

def parse(t, v, n):
    """Prefix rows -> nested (type, value, children) by recursive descent on arities."""
    pos = [0]

    def node():
        i = pos[0]
        pos[0] += 1
        ti, vi = int(t[i]), float(v[i])
        kids = [] if ti in (0, 1) else [node() for _ in range(ARITY[int(vi)])]
        return (ti, vi, kids)

    root = node()
    assert pos[0] == n
    return root


def preorder(tree):
    out = [tree]
    for c in tree[2]:
        out += preorder(c)
    return out


def substitute(tree, k, new):
    """Replace the k-th node in pre-order (0-based) by the nested tree `new`."""
    counter = [0]

    def go(node):
        i = counter[0]
        counter[0] += 1
        if i == k:
            counter[0] += len(preorder(node)) - 1
            return new
        return (node[0], node[1], [go(c) for c in node[2]])

    return go(tree)


def serialize(tree, L):
    nodes = [(n[0], n[1]) for n in preorder(tree)]
    return rows(nodes, L)


def population(seed, n, L, depth=6, V=3):
    rng = np.random.default_rng(seed)
    return ST.depth_limited(rng, n, depth, rng.random(n) < 0.5, ST.F11, V, L)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_tree_structured_construction(seed):
    """Random valid trees, random target node and random donor subtree: the oracle's row
    splice equals substitution in a nested tree printed back with recomputed sizes."""
    L = 64
    old = population(seed, 60, L)
    don = population(seed + 100, 60, L, depth=4)
    rng = np.random.default_rng(seed + 7)
    lo = old[2][:, 0].astype(int)
    ld = don[2][:, 0].astype(int)
    k = (rng.random(60) * lo).astype(int)
    j = (rng.random(60) * ld).astype(int)
    out, st = O.subtree_exchange(old, don, k, j, max_len=L)
    n_ok = 0
    for b in range(60):
        t_old = parse(old[0][b], old[1][b], lo[b])
        sub = parse(don[0][b][j[b]:], don[1][b][j[b]:], int(don[2][b][j[b]]))
        want_tree = substitute(t_old, k[b], sub)
        n_new = len(preorder(want_tree))
        if n_new > L:
            assert st[b] == O.X_TOO_LONG
            want = [r[b] for r in old]
        else:
            assert st[b] == O.X_OK
            want = serialize(want_tree, L)
            n_ok += 1
        for a, w in zip(out, want):
            np.testing.assert_array_equal(a[b], w)
    assert n_ok > 40


def test_outputs_are_valid_trees():
    """Every result passes the encoding's validity rules (§III-A) and its length is
    len_old - size_old[k] + size_new[j]."""
    L = 128
    old = population(5, 200, L, depth=7)
    don = population(6, 200, L, depth=5)
    rng = np.random.default_rng(3)
    u = rng.random(200).astype(np.float32)
    w = rng.random(200).astype(np.float32)
    out, st = O.subtree_exchange(old, don, u, w, max_len=L, flags=O.OLD_UNIFORM | O.NEW_UNIFORM)
    info = O.plan(*out, 3, 1)
    assert (info[:, 0] == 0).all()
    lo = old[2][:, 0].astype(int)
    ld = don[2][:, 0].astype(int)
    for b in range(200):
        k = O.pick_node(u[b], lo[b])
        jj = O.pick_node(w[b], ld[b])
        n = lo[b] - int(old[2][b, k]) + int(don[2][b, jj])
        assert info[b, 1] == (n if st[b] == O.X_OK else lo[b])


def test_operators_built_on_exchange():
    """Hoist mutation exchange(T, 0, T's subtree at k) gives that subtree alone; exchanging
    node 0 for the whole of the same tree gives the tree back; exchanging node k for the
    subtree already at k changes nothing."""
    L = 64
    pop = population(9, 40, L)
    n = pop[2][:, 0].astype(int)
    rng = np.random.default_rng(4)
    k = (rng.random(40) * n).astype(int)
    hoist, st = O.subtree_exchange(pop, pop, np.zeros(40, int), k)
    assert (st == O.X_OK).all()
    for b in range(40):
        e = k[b] + int(pop[2][b, k[b]])
        for r in range(3):
            np.testing.assert_array_equal(hoist[r][b, :e - k[b]], pop[r][b, k[b]:e])
            assert np.isnan(hoist[r][b, e - k[b]:]).all()
    same, st = O.subtree_exchange(pop, pop, np.zeros(40, int), np.zeros(40, int))
    assert (st == O.X_OK).all()
    for r in range(3):
        np.testing.assert_array_equal(same[r], pop[r])
    same, st = O.subtree_exchange(pop, pop, k, k)
    for r in range(3):
        np.testing.assert_array_equal(same[r], pop[r])


def test_crossover_rows_and_semantics():
    """One-point crossover between a tree and another row of the population: evaluating the
    child equals evaluating the first parent with the chosen subtree's value replaced by the
    donor subtree's value (recursive evaluation of the nested form)."""
    L = 64
    pop = population(11, 30, L, V=2)
    rng = np.random.default_rng(12)
    mate = rng.permutation(30)
    n = pop[2][:, 0].astype(int)
    k = (rng.random(30) * n).astype(int)
    j = (rng.random(30) * n[mate]).astype(int)
    child, st = O.subtree_exchange(pop, pop, k, j, old_row=np.arange(30), new_row=mate)
    X = rng.uniform(-2, 2, (2, 16)).astype(np.float32)
    ok = st == O.X_OK
    pred_child = O.predict(*(c[ok] for c in child), X)[:, 0, :]
    for i, b in enumerate(np.nonzero(ok)[0]):
        t_old = parse(pop[0][b], pop[1][b], n[b])
        sub = parse(pop[0][mate[b]][j[b]:], pop[1][mate[b]][j[b]:], int(pop[2][mate[b]][j[b]]))
        want = serialize(substitute(t_old, k[b], sub), L)
        pw = O.predict(*(r[None] for r in want), X)[0, 0, :]
        np.testing.assert_array_equal(pred_child[i], pw)


def test_pick_node():
    """floor(u * n) in float32, clamped: u = 0 gives the root, the largest float32 below 1
    gives the last node (the product rounds up to n for large n), and every node is
    reachable on a grid of u values."""
    assert O.pick_node(0.0, 5) == 0
    below1 = np.nextafter(np.float32(1), np.float32(0))
    assert O.pick_node(below1, 5) == 4
    assert O.pick_node(below1, 1 << 20) == (1 << 20) - 1
    assert O.pick_node(1.0, 5) is None
    assert O.pick_node(-0.1, 5) is None
    assert O.pick_node(np.nan, 5) is None
    hits = {O.pick_node(u, 7) for u in np.arange(0, 1, 1 / 70, dtype=np.float32)}
    assert hits == set(range(7))


def test_status_codes_and_fallback_rows():
    """The checks in their order: bad old row -> NaN row; bad old length -> verbatim copy;
    bad node -> old tree; bad donor -> old tree."""
    L = 8
    old = [np.stack([r, r]) for r in rows(OLD, L)]
    don = [r[None] for r in rows(NEW, L)]
    out, st = O.subtree_exchange(old, don, [0], old_row=[2])
    assert st[0] == O.X_BAD_OLD and all(np.isnan(r[0]).all() for r in out)
    bad = [r.copy() for r in old]
    bad[2][1, 0] = 9.0          # len beyond Lmax
    out, st = O.subtree_exchange(bad, don, [0], old_row=[1])
    assert st[0] == O.X_BAD_OLD
    for a, b in zip(out, bad):
        np.testing.assert_array_equal(a[0], b[1])
    for k in (-1, 6, 100):
        out, st = O.subtree_exchange(old, don, [k])
        assert st[0] == O.X_BAD_OLD
        np.testing.assert_array_equal(out[0][0], old[0][0])
    out, st = O.subtree_exchange(old, don, [1], [3])       # donor node in the NaN tail
    assert st[0] == O.X_BAD_DONOR
    out, st = O.subtree_exchange(old, don, [1], [0], new_row=[1])
    assert st[0] == O.X_BAD_DONOR
    out, st = O.subtree_exchange(old, don, [np.float32(1.5)], flags=O.OLD_UNIFORM)
    assert st[0] == O.X_BAD_OLD
