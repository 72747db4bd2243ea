"""Pins for the tree-generation oracle: the random generator against its
published known-answer vectors, the generated trees against the encoding's
validity rules (§III-A), the depth rules of the grow and full methods, and
the node distributions against the stated probabilities."""

import os

import numpy as np
import pytest

import oracle as O
from oracle import generate_oracle as G

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
F7 = [0, 1, 2, 3, 4, 5, 11]
ARITY = {0: 2, 1: 2, 2: 2, 3: 2, 4: 1, 5: 1, 6: 1, 7: 1, 8: 1, 9: 2, 10: 2, 11: 1}


def kat_rows():
    out = []
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("kat"):
            w = [int(x, 16) for x in line.split()[1:]]
            out.append((tuple(w[:4]), tuple(w[4:6]), tuple(w[6:10])))
    return out


def test_philox_known_answers():
    rows = kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert G.philox4x32_10(ctr, key) == want


def test_unit_mapping():
    assert G.to_unit(0) == 0.0
    assert G.to_unit(0xFFFFFFFF) == np.float32(1 - 2.0 ** -24)
    assert G.to_unit(0x80000000) == np.float32(0.5)
    assert G.to_unit(0x000000FF) == 0.0      # the low 8 bits are dropped


def depths(t, v, n):
    """Depth of every node by a prefix walk on arities (independent of the size row)."""
    d = [0] * n
    open_slots = []
    for i in range(n):
        d[i] = open_slots.pop() if open_slots else 0
        a = 0 if t[i] in (0, 1) else ARITY[int(v[i])]
        open_slots.extend([d[i] + 1] * a)
    return d


@pytest.mark.parametrize("method", [G.GROW, G.FULL, G.RAMPED])
def test_trees_are_valid_and_obey_depth_rules(method):
    P, L, V = 300, 256, 3
    (t, v, s), att = G.generate(P, L, V, F7, method=method, d_min=2, d_max=6, seed=11)
    info = O.plan(t, v, s, V, 1)
    assert (info[:, 0] == 0).all()                     # validator: encoding, sizes, op ids, variables
    for i in range(P):
        n = int(s[i, 0])
        dl, full = G.tree_depth_limit(i, method, 2, 6)
        assert att[i] >= 1
        if att[i] > 8:
            continue                                   # depth limit was lowered after failed attempts
        d = depths(t[i], v[i], n)
        leaves = [d[j] for j in range(n) if t[i, j] in (0, 1)]
        assert max(d) <= dl
        assert t[i, 0] == 2                            # the root is a function (depth limit > 0)
        if full:
            assert set(leaves) == {dl}                 # every leaf at the depth limit
        funcs_inside = [d[j] for j in range(n) if t[i, j] == 2]
        assert all(x < dl for x in funcs_inside)


def test_ramped_assignment():
    for t in range(20):
        d, full = G.tree_depth_limit(t, G.RAMPED, 2, 6)
        assert d == 2 + (t // 2) % 5 and full == (t % 2 == 0)
    assert G.tree_depth_limit(7, G.GROW, 2, 6) == (6, False)
    assert G.tree_depth_limit(7, G.FULL, 2, 6) == (6, True)


def test_node_distributions():
    """Grow nodes below the root and above the limit are functions with probability p_func;
    terminals are constants with probability p_const, constants uniform in [lo, hi), variables
    and op ids uniform. Binomial/uniform checks at 5 sigma on 2,000 trees."""
    P, L, V = 2000, 512, 4
    (t, v, s), att = G.generate(P, L, V, F7, method=G.GROW, d_max=7, seed=5)
    pf, pc = G.default_p_func(len(F7), V), G.default_p_const(V)
    inner, inner_f, consts, vars_, ops = 0, 0, [], [], []
    n_term = 0
    for i in range(P):
        if att[i] > 8:
            continue
        n = int(s[i, 0])
        d = depths(t[i], v[i], n)
        for j in range(n):
            if 0 < d[j] < 7:
                inner += 1
                inner_f += t[i, j] == 2
            if t[i, j] == 2:
                ops.append(int(v[i, j]))
            else:
                n_term += 1
                (consts if t[i, j] == 1 else vars_).append(v[i, j])
    assert abs(inner_f / inner - pf) < 5 * np.sqrt(pf * (1 - pf) / inner)
    assert abs(len(consts) / n_term - pc) < 5 * np.sqrt(pc * (1 - pc) / n_term)
    c = np.array(consts)
    assert c.min() >= -5.0 and c.max() < 5.0 and abs(c.mean()) < 5 * 10 / np.sqrt(12 * len(c))
    for vals, k in ((np.array(vars_, int), V), (np.array(ops), None)):
        cats = np.arange(V) if k else np.array(F7)
        counts = np.array([(vals == x).sum() for x in cats])
        e = len(vals) / len(cats)
        assert np.all(np.abs(counts - e) < 5 * np.sqrt(e))


def test_length_limit_falls_back_to_smaller_depths():
    """Full trees of depth 6 over binary ops do not fit in 16 nodes: each attempt fails until
    the limit has dropped to depth 3 (15 nodes), after 8 failed attempts per level."""
    (t, v, s), att = G.generate(10, 16, 2, [0, 2], method=G.FULL, d_max=6, seed=3)
    assert (O.plan(t, v, s, 2, 1)[:, 0] == 0).all()
    assert (s[:, 0] == 15).all()
    assert (att == 3 * 8 + 1).all()


def test_determinism_and_slices():
    a, _ = G.generate(30, 64, 2, F7, seed=99)
    b, _ = G.generate(30, 64, 2, F7, seed=99)
    c, _ = G.generate(30, 64, 2, F7, seed=100)
    tail, _ = G.generate(10, 64, 2, F7, seed=99, first_tree=20)
    for x, y, z, w in zip(a, b, c, tail):
        np.testing.assert_array_equal(x, y)
        np.testing.assert_array_equal(x[20:], w)
    assert not np.array_equal(a[1], c[1])
