"""Random expression trees in the padded prefix encoding.

Encoding (paper §III-A): a tree is three float32 rows of length Lmax --
node type, node value and subtree size -- holding the prefix (pre-order)
node sequence in the first len entries and NaN after them.

Type codes: 0 = variable (value = input index), 1 = constant (value = the
constant), 2 = function (value = op id), 3 + o = multi-output ("Modi")
function node that contributes to output o (value = op id).

Op ids and arities used by the generators (names only; no arithmetic):
0 add/2, 1 sub/2, 2 mul/2, 3 protected div/2, 4 sin/1, 5 cos/1, 6 tanh/1,
7 clamped exp/1, 8 protected log/1, 9 max/2, 10 min/2, 11 tan/1.

All generators are vectorised across trees: position by position, every
tree still under construction draws its next node, so the random stream is
consumed in a fixed order for a given seed.
"""

import numpy as np

TYPE_VAR = 0
TYPE_CONST = 1
TYPE_FUNC = 2
TYPE_MODI0 = 3

ARITY = np.array([2, 2, 2, 2, 1, 1, 1, 1, 1, 2, 2, 1], dtype=np.int64)
F4 = np.array([0, 1, 2, 3], dtype=np.int64)             # + - * protected-div
F11 = np.arange(11, dtype=np.int64)                     # F4 + sin cos tanh exp log max min
F7 = np.array([0, 1, 2, 3, 4, 5, 11], dtype=np.int64)   # the paper's SR set: + - * pdiv sin cos tan

CONST_LO, CONST_HI = -5.0, 5.0


def _terminals(rng, m, V, nconst, const_cap):
    """Draw m terminals: constant with probability 1/(V+1), else a uniform variable."""
    is_const = rng.random(m) < 1.0 / (V + 1)
    var = rng.integers(0, V, m)
    cval = rng.uniform(CONST_LO, CONST_HI, m)
    if const_cap is not None:
        is_const &= nconst < const_cap          # a draw beyond the cap becomes a variable
    typ = np.where(is_const, TYPE_CONST, TYPE_VAR)
    val = np.where(is_const, cval.astype(np.float32).astype(np.float64), var.astype(np.float64))
    return typ, val, is_const


def _sizes_sorted(types_cm, values_cm, lengths_desc):
    """Subtree sizes by a reverse scan over positions, vectorised over trees.

    Columns must be ordered by non-increasing length, so the trees still
    live at a position form a leading slice. Reads only node arities.
    """
    Lmax, n = types_cm.shape
    live_count = n - np.searchsorted(np.sort(lengths_desc), np.arange(Lmax), side="right")
    size = np.zeros((Lmax + 2, n), np.int32)
    cols = np.arange(n)
    for pos in range(Lmax - 1, -1, -1):
        m = int(live_count[pos])
        if m == 0:
            continue
        t = types_cm[pos, :m]
        isf = t >= TYPE_FUNC
        a = np.zeros(m, np.int64)
        a[isf] = ARITY[values_cm[pos, :m][isf].astype(np.int64)]
        s1 = np.where(a >= 1, size[pos + 1, :m], 0)
        c2 = np.minimum(pos + 1 + s1, Lmax)
        s2 = np.where(a == 2, size[c2, cols[:m]], 0)
        size[pos, :m] = 1 + s1 + s2
    return size[:Lmax]


def _emit_sorted(tc, vc, Lc, ids, T, Vv, S):
    """Write a length-sorted column-major chunk into row-major outputs at rows `ids`."""
    Lmax = tc.shape[0]
    sizes = _sizes_sorted(tc, vc, Lc).astype(np.float32)
    sizes[np.arange(Lmax)[:, None] >= Lc[None, :]] = np.nan
    T[ids] = tc.T
    Vv[ids] = vc.T
    S[ids] = sizes.T


def pad_rows(types_cm, values_cm, lengths, Lmax):
    """Pack column-major prefix sequences (NaN beyond each length) into row-major
    float32 (type, value, size) rows [n][Lmax]."""
    lengths = np.asarray(lengths, np.int64)
    n = lengths.size
    order = np.argsort(-lengths, kind="stable")
    T = np.empty((n, Lmax), np.float32)
    Vv = np.empty((n, Lmax), np.float32)
    S = np.empty((n, Lmax), np.float32)
    B = 8192
    for c in range(0, n, B):
        ids = order[c:c + B]
        _emit_sorted(types_cm[:, ids], values_cm[:, ids], lengths[ids], ids, T, Vv, S)
    return T, Vv, S


def _depth_limited_once(rng, max_depth, full, funcs, V, Lmax, const_cap):
    n = max_depth.shape[0]
    nF = len(funcs)
    p_func = nF / (nF + V + 1.0)
    cap = Lmax + 2
    stack = np.zeros((n, cap), np.int16)           # pending slot depths
    sp = np.ones(n, np.int64)                      # each tree starts with one slot at depth 0
    types = np.full((Lmax, n), np.nan, np.float32)
    values = np.full((Lmax, n), np.nan, np.float32)
    nconst = np.zeros(n, np.int64)
    length = np.zeros(n, np.int64)
    alive = np.ones(n, bool)
    idx = np.arange(n)
    for pos in range(Lmax):
        if idx.size == 0:
            break
        m = idx.size
        sp[idx] -= 1
        d = stack[idx, sp[idx]].astype(np.int64)
        dm = max_depth[idx]
        u = rng.random(m)
        op = funcs[rng.integers(0, nF, m)]
        want_f = np.where(d >= dm, False, np.where(full[idx] | (d == 0), True, u < p_func))
        ttyp, tval, tconst = _terminals(rng, m, V, nconst[idx], const_cap)
        types[pos, idx] = np.where(want_f, TYPE_FUNC, ttyp)
        values[pos, idx] = np.where(want_f, op.astype(np.float64), tval)
        nconst[idx] += (~want_f) & tconst
        length[idx] += 1
        ar = np.where(want_f, ARITY[op], 0)
        for k in (1, 2):
            push = ar >= k
            j = idx[push]
            stack[j, sp[j]] = d[push] + 1
            sp[j] += 1
        done = sp[idx] == 0
        alive[idx[done]] = False
        idx = idx[~done]
    ok = ~alive
    return types, values, length, ok


def depth_limited(rng, n, max_depth, full, funcs, V, Lmax, const_cap=None, max_redraw=100):
    """Koza-style grow/full trees, vectorised.

    grow(d): the root is a function; a slot at depth < d becomes a function
    with probability |F|/(|F|+V+1), else a terminal; at depth d it is a
    terminal. full(d): functions down to depth d, then terminals. A terminal
    is a constant (U(-5,5), stored as float32) with probability 1/(V+1), else
    a uniform variable. Draws longer than Lmax are redrawn; after max_redraw
    failures a tree falls back to grow(d-1), then grow(d-2), ...

    Returns float32 (type, value, size) rows [n][Lmax].
    """
    max_depth = np.broadcast_to(np.asarray(max_depth, np.int64), (n,)).copy()
    full = np.broadcast_to(np.asarray(full, bool), (n,)).copy()
    funcs = np.asarray(funcs, np.int64)
    types = np.full((Lmax, n), np.nan, np.float32)
    values = np.full((Lmax, n), np.nan, np.float32)
    length = np.zeros(n, np.int64)
    todo = np.arange(n)
    attempts = 0
    while todo.size:
        t, v, L, ok = _depth_limited_once(rng, max_depth[todo], full[todo], funcs, V, Lmax, const_cap)
        good = todo[ok]
        types[:, good], values[:, good], length[good] = t[:, ok], v[:, ok], L[ok]
        todo = todo[~ok]
        attempts += 1
        if todo.size and attempts >= max_redraw:
            max_depth[todo] = np.maximum(max_depth[todo] - 1, 1)
            full[todo] = False
            attempts = 0
    return pad_rows(types, values, length, Lmax)


def exact_length(rng, lengths, funcs, V, Lmax, chunk=8192):
    """Trees with exactly the requested node counts (open-slot prefix builder).

    With s open child slots and r nodes still to place (this one included),
    a node of arity a keeps the sequence completable iff s-1+a <= r-1, and it
    must not close the tree early: s-1+a >= 1 unless r == 1. The arity is
    drawn uniformly among the feasible ones, then a uniform op of that arity
    (or a terminal as in depth_limited). Trees are built longest first, in
    chunks of `chunk` trees.
    """
    lengths = np.asarray(lengths, np.int64)
    n = lengths.size
    funcs = np.asarray(funcs, np.int64)
    un = funcs[ARITY[funcs] == 1]
    bi = funcs[ARITY[funcs] == 2]
    if un.size == 0 and (lengths % 2 == 0).any():
        raise ValueError("with binary ops only, a tree has an odd number of nodes")
    order = np.argsort(-lengths, kind="stable")
    Ls = lengths[order]
    T = np.empty((n, Lmax), np.float32)
    Vv = np.empty((n, Lmax), np.float32)
    S = np.empty((n, Lmax), np.float32)
    tc = np.empty((Lmax, min(chunk, n)), np.float32)
    vc = np.empty_like(tc)
    for c0 in range(0, n, chunk):
        ids = order[c0:c0 + chunk]
        L = Ls[c0:c0 + chunk]
        w = ids.size
        t_, v_ = tc[:, :w], vc[:, :w]
        t_.fill(np.nan)
        v_.fill(np.nan)
        open_ = np.ones(w, np.int64)
        live_count = w - np.searchsorted(np.sort(L), np.arange(Lmax), side="right")
        for pos in range(int(L[0])):
            m = int(live_count[pos])
            r = L[:m] - pos
            s = open_[:m]
            feas = np.stack([(s - 1 + a <= r - 1) & ((s - 1 + a >= 1) | (r == 1)) & (a != 1 or un.size > 0)
                             for a in (0, 1, 2)], 1)
            cnt = feas.sum(1)
            k = np.minimum((rng.random(m) * cnt).astype(np.int64), cnt - 1)
            cum = np.cumsum(feas, 1)
            a = np.argmax((cum > k[:, None]) & feas, axis=1)
            uop = un[rng.integers(0, un.size, m)] if un.size else np.zeros(m, np.int64)
            bop = bi[rng.integers(0, bi.size, m)]
            ttyp, tval, _ = _terminals(rng, m, V, np.zeros(m, np.int64), None)
            t_[pos, :m] = np.where(a == 0, ttyp, TYPE_FUNC)
            v_[pos, :m] = np.where(a == 0, tval, np.where(a == 1, uop, bop).astype(np.float64))
            open_[:m] = s - 1 + a
        _emit_sorted(t_, v_, L, ids, T, Vv, S)
    return T, Vv, S


def assign_modi(rng, T, n_out, frac):
    """Turn a random fraction of trees into multi-output trees (in place).

    A chosen tree gets its root tagged Modi(0) and n_out-1 further distinct
    random function nodes tagged Modi(1), ..., Modi(n_out-1) (as many as the
    tree has function nodes). Returns the indices of the chosen trees.
    """
    n, Lmax = T.shape
    chosen = np.nonzero(rng.random(n) < frac)[0]
    for t in chosen:
        fpos = np.nonzero(T[t] == TYPE_FUNC)[0]
        if fpos.size == 0 or fpos[0] != 0:
            continue
        T[t, 0] = TYPE_MODI0
        rest = fpos[1:]
        k = min(n_out - 1, rest.size)
        if k:
            pick = rng.choice(rest, size=k, replace=False)
            for o, p in enumerate(pick, start=1):
                T[t, p] = TYPE_MODI0 + o
    return chosen
