"""Plain CPU oracle for random tree generation -- TEST INFRASTRUCTURE.

Only the test suite, the package smoke check and the benchmark's
CPU-baseline leg may import or run this module. It shares no code with the
device library.

Tree initialisation (the paper lists it among the operations that run one
individual per GPU thread, §III and the parallelism figure) with the
classic grow / full / ramped half-and-half methods, written out in prefix
order for the padded encoding of §III-A.

Random numbers come from Philox4x32-10, the counter-based generator of
Salmon, Moraes, Dror and Shaw ("Parallel random numbers: as easy as 1, 2,
3", SC 2011), restated here from its published definition. Every draw is
addressed by a counter, so the device library, which implements the same
generator, produces the same trees bit for bit:
    counter = (tree, attempt, position, 0), key = (seed low, seed high);
the four output words of one call serve one node.

One tree, depth limit d, method full or grow (readings where the paper is
silent, fixed here):
* Slots are filled in prefix order from a stack of open child slots, each
  carrying its depth; the root slot has depth 0.
* At a slot of depth h the node is a function when
    full:  h < d;
    grow:  h < d and (h == 0 or u0 < p_func),
  else a terminal. u0..u3 are the four words of the node's Philox call
  mapped to [0, 1) as (w >> 8) * 2^-24 (exact in float32).
* A function takes op = funcs[floor(u1 * nF)] (float32 product, clamped);
  its children's slots (depth h + 1) are pushed so that the first child is
  filled next.
* A terminal is a constant when u1 < p_const, with value
  lo + (hi - lo) * u2 (float32, each operation rounded), else variable
  floor(u2 * V) (float32 product, clamped).
* p_func and p_const are float32; their defaults are nF / (nF + V + 1) and
  1 / (V + 1).
* A tree longer than Lmax is abandoned and drawn again with the next
  attempt number; after `attempts_per_depth` failed attempts the depth limit
  drops by one (the attempt numbers keep counting). A depth limit of 0
  gives a single terminal, which always fits.
* Ramped half-and-half: tree t gets the depth limit
  d_min + (t // 2) mod (d_max - d_min + 1) and the full method when t is
  even, grow when odd. The grow and full methods use d_max for every tree.
* Subtree sizes: a reverse pass over the prefix sequence (a node's size is
  one plus its children's sizes).
"""

import numpy as np

from .tgp_oracle import OPS, T_CONST, T_FUNC, T_VAR

GROW, FULL, RAMPED = 0, 1, 2

_M0, _M1 = 0xD2511F53, 0xCD9E8D57          # Philox4x32 multipliers
_W0, _W1 = 0x9E3779B9, 0xBB67AE85          # Weyl key increments
_MASK = 0xFFFFFFFF


def philox4x32_10(counter, key):
    """Philox4x32 with 10 rounds on one 128-bit counter and 64-bit key (Python ints)."""
    c0, c1, c2, c3 = (int(x) & _MASK for x in counter)
    k0, k1 = (int(x) & _MASK for x in key)
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> 32, p0 & _MASK
        hi1, lo1 = p1 >> 32, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def to_unit(w):
    """32-bit word -> float32 in [0, 1): the top 24 bits times 2^-24 (exact)."""
    return np.float32((int(w) >> 8) * (1.0 / 16777216.0))


def default_p_func(n_funcs, V):
    return np.float32(n_funcs) / np.float32(n_funcs + V + 1)


def default_p_const(V):
    return np.float32(1) / np.float32(V + 1)


def _draw_once(t, attempt, depth, full, funcs, V, Lmax, p_func, p_const, lo, hi, key):
    """One attempt at tree t; returns (types, values) or None if it outgrew Lmax."""
    nF = len(funcs)
    types, values = [], []
    slots = [0]  # depths of open child slots, top = next to fill
    n = 0
    while slots:
        h = slots.pop()
        if n == Lmax:
            return None
        w = philox4x32_10((t, attempt, n, 0), key)
        u0, u1, u2 = to_unit(w[0]), to_unit(w[1]), to_unit(w[2])
        if full:
            is_func = h < depth
        else:
            is_func = h < depth and (h == 0 or u0 < p_func)
        if is_func:
            op = int(funcs[min(int(np.floor(np.float32(u1 * np.float32(nF)))), nF - 1)])
            types.append(T_FUNC)
            values.append(np.float32(op))
            slots.extend([h + 1] * OPS[op][1])
        elif u1 < p_const:
            span = np.float32(np.float32(hi) - np.float32(lo))
            types.append(T_CONST)
            values.append(np.float32(np.float32(lo) + np.float32(span * u2)))
        else:
            types.append(T_VAR)
            values.append(np.float32(min(int(np.floor(np.float32(u2 * np.float32(V)))), V - 1)))
        n += 1
    return types, values


def _sizes(types, values):
    """Subtree sizes by a reverse pass: one plus the sizes of the children."""
    stack = []
    out = [0] * len(types)
    for i in range(len(types) - 1, -1, -1):
        a = 0 if types[i] in (T_VAR, T_CONST) else OPS[int(values[i])][1]
        s = 1 + sum(stack.pop() for _ in range(a))
        out[i] = s
        stack.append(s)
    return out


def tree_depth_limit(t, method, d_min, d_max):
    if method == RAMPED:
        return d_min + (t // 2) % (d_max - d_min + 1), t % 2 == 0
    return d_max, method == FULL


def generate(P, Lmax, V, funcs, method=RAMPED, d_min=2, d_max=6, seed=0, lo=-5.0, hi=5.0,
             p_func=None, p_const=None, attempts_per_depth=8, first_tree=0):
    """P trees as padded (type, value, size) float32 rows [P][Lmax], and the attempt count per tree.

    first_tree offsets the tree index used in the counters (for drawing a slice of a population)."""
    funcs = [int(f) for f in funcs]
    p_func = default_p_func(len(funcs), V) if p_func is None else np.float32(p_func)
    p_const = default_p_const(V) if p_const is None else np.float32(p_const)
    key = (seed & _MASK, (seed >> 32) & _MASK)
    rows = [np.full((P, Lmax), np.nan, np.float32) for _ in range(3)]
    attempts = np.zeros(P, np.int32)
    for i in range(P):
        t = first_tree + i
        depth, full = tree_depth_limit(t, method, d_min, d_max)
        attempt = 0
        while True:
            res = _draw_once(t, attempt, depth, full, funcs, V, Lmax, p_func, p_const, lo, hi, key)
            attempt += 1
            if res is not None:
                break
            if attempt % attempts_per_depth == 0 and depth > 0:
                depth -= 1
        types, values = res
        n = len(types)
        rows[0][i, :n] = types
        rows[1][i, :n] = values
        rows[2][i, :n] = _sizes(types, values)
        attempts[i] = attempt
    return tuple(rows), attempts
