"""Plain CPU oracle for the subtree-exchange primitive -- TEST INFRASTRUCTURE.

Only the test suite, the package smoke check and the benchmark's
CPU-baseline leg may import or run this module. It shares no code with the
device library.

Subtree exchange (§III-B): exchange(T_old, k, T_new) -> T* replaces the
subtree rooted at node k of T_old with the tree T_new. With s the position
of k and e = s + size_old[k] the end of its subtree, each of the three
rows of T* is the old row before s, then the new subtree's row, then the
old row from e on; in the size row, every ancestor of k first has
dn = size_new[0] - size_old[k] added. When size_old[0] + dn exceeds the
maximum tree length the exchange is refused and T_old is returned.
One-point crossover takes T_new as a subtree of a second parent, subtree
mutation a freshly generated tree, hoist mutation a subtree of T_old
itself (§III-B, the genetic-operations figure).

This module follows those steps literally, one output tree at a time:
ancestors are found by walking parent links of a prefix parse driven by
node arities (not by any subtree-size test), and the three rows are built
by concatenation. Positions are 0-based.

Readings (where the paper is silent):
* Batch form. Output b takes old tree old_row[b], node old_node[b], and
  the subtree of donor tree new_row[b] at node new_node[b] (node 0 is the
  whole donor tree). Output rows have the old population's row length.
* Random node choice. With the uniform flag for a side, its node argument
  is a float32 u in [0, 1) and the node is floor(u * len) with the product
  rounded to float32, clamped to len - 1 (len = size[0] of that tree).
* Checks and outcomes (status codes, first failing check wins):
    BAD_OLD   old_row outside [0, P_old): the output row is all NaN;
    BAD_OLD   size_old[0] not an integer in [1, Lmax_old]: the output row
              is a verbatim copy of the old row;
    BAD_OLD   k outside [0, len_old), or size_old[k] not an integer in
              [1, len_old - k]: T_old is returned;
    BAD_DONOR new_row outside [0, P_new), in uniform mode size_new[0] not
              an integer in [1, Lmax_new], j outside [0, Lmax_new), or
              size_new[j] not an integer in [1, Lmax_new - j]: T_old;
    TOO_LONG  len_old - size_old[k] + size_new[j] > max_len: T_old;
    OK        the exchange result.
  "T_old is returned" means the old row's first len_old entries followed
  by NaN, which for a valid tree is the row itself.
* The result is defined for valid old and donor trees (plan status 0).
  For other trees only the checks above are made.
* Writing into output rows that already hold padded trees (the device
  library's padded-output option) only skips rewriting NaN that is already
  there; the rows are the same, so the oracle has no such option.
"""

import math

import numpy as np

from .tgp_oracle import OPS, T_CONST, T_VAR

X_OK, X_TOO_LONG, X_BAD_OLD, X_BAD_DONOR = range(4)
OLD_UNIFORM, NEW_UNIFORM = 1, 2


def _int_in(x, lo, hi):
    """x (a float) is an integer in [lo, hi]."""
    x = float(x)
    return math.isfinite(x) and x == math.floor(x) and lo <= x <= hi


def pick_node(u, n):
    """Uniform random node of a tree of n nodes from u in [0, 1):
    floor(u * n) with the product rounded to float32, clamped to n - 1.
    Returns None when u is not in [0, 1)."""
    u = np.float32(u)
    if not (0.0 <= u < 1.0):
        return None
    k = int(np.floor(np.float32(u * np.float32(n))))
    return min(k, n - 1)


def _arity(t, v):
    t = int(t)
    if t in (T_VAR, T_CONST):
        return 0
    return OPS[int(v)][1]


def ancestors(type_row, value_row, n, k):
    """Ancestors of node k in the prefix sequence of n nodes, nearest first.

    A prefix parse assigns each node to the nearest open function node
    that still needs a child; a node with children opens itself. The
    parent links then give the ancestor chain.
    """
    parent = [-1] * n
    open_nodes = []  # [node, children still to assign]
    for i in range(n):
        if open_nodes:
            parent[i] = open_nodes[-1][0]
            open_nodes[-1][1] -= 1
            if open_nodes[-1][1] == 0:
                open_nodes.pop()
        a = _arity(type_row[i], value_row[i])
        if a:
            open_nodes.append([i, a])
    chain = []
    p = parent[k]
    while p >= 0:
        chain.append(p)
        p = parent[p]
    return chain


def exchange_tree(old, k, new_sub, max_len, Lout):
    """exchange(T_old, k, T_new) for one valid tree (§III-B).

    old, new_sub: (type, value, size) rows; new_sub holds exactly the
    inserted subtree (its first entry is the subtree's root). Returns the
    three output rows of length Lout and the status (OK or TOO_LONG).
    """
    ot, ov, osz = (np.asarray(r, np.float64) for r in old)
    nt, nv, nsz = (np.asarray(r, np.float64) for r in new_sub)
    n_old = int(osz[0])
    s = k
    e = s + int(osz[k])
    dn = int(nsz[0]) - int(osz[k])
    if n_old + dn > max_len:
        return _old_tree(old, Lout), X_TOO_LONG
    updated = osz[:n_old].copy()
    for a in ancestors(ot, ov, n_old, k):
        updated[a] += dn
    rows = (np.concatenate([ot[:s], nt, ot[e:n_old]]),
            np.concatenate([ov[:s], nv, ov[e:n_old]]),
            np.concatenate([updated[:s], nsz, osz[e:n_old]]))
    return tuple(_pad(r, Lout) for r in rows), X_OK


def _pad(r, L):
    out = np.full(L, np.nan, np.float32)
    out[:len(r)] = np.asarray(r, np.float32)
    return out


def _old_tree(old, Lout):
    n = int(float(old[2][0]))
    return tuple(_pad(np.asarray(r, np.float32)[:n], Lout) for r in old)


def subtree_exchange(old_pop, new_pop, old_node, new_node=None, old_row=None, new_row=None,
                     max_len=None, flags=0):
    """Batched subtree exchange: one output tree per entry of old_node.

    old_pop, new_pop: (type, value, size) float32 arrays [P][Lmax].
    old_node / new_node: int node indices, or float32 uniforms for the
    sides whose flag (OLD_UNIFORM, NEW_UNIFORM) is set; new_node None
    means node 0. old_row / new_row: int rows (None: b). max_len defaults
    to the old rows' length.
    Returns ((type, value, size) float32 [B][Lmax_old], status int32 [B]).
    """
    ot, ov, osz = (np.asarray(a, np.float32) for a in old_pop)
    nt, nv, nsz = (np.asarray(a, np.float32) for a in new_pop)
    P_old, L_old = ot.shape
    P_new, L_new = nt.shape
    B = len(old_node)
    max_len = L_old if max_len is None else int(max_len)
    out = [np.full((B, L_old), np.nan, np.float32) for _ in range(3)]
    status = np.zeros(B, np.int32)
    for b in range(B):
        orow = b if old_row is None else int(old_row[b])
        nrow = b if new_row is None else int(new_row[b])
        res, st = _one(ot, ov, osz, nt, nv, nsz, P_old, L_old, P_new, L_new, orow, nrow,
                       old_node[b], 0 if new_node is None else new_node[b], max_len, flags)
        status[b] = st
        if res is not None:
            for r in range(3):
                out[r][b] = res[r]
    return tuple(out), status


def _one(ot, ov, osz, nt, nv, nsz, P_old, L_old, P_new, L_new, orow, nrow, kn, jn, max_len, flags):
    if not (0 <= orow < P_old):
        return None, X_BAD_OLD
    old = (ot[orow], ov[orow], osz[orow])
    if not _int_in(osz[orow, 0], 1, L_old):
        return tuple(r.copy() for r in old), X_BAD_OLD
    n_old = int(osz[orow, 0])
    if flags & OLD_UNIFORM:
        k = pick_node(kn, n_old)
    else:
        k = int(kn)
    if k is None or not (0 <= k < n_old) or not _int_in(osz[orow, k], 1, n_old - k):
        return _old_tree(old, L_old), X_BAD_OLD
    if not (0 <= nrow < P_new):
        return _old_tree(old, L_old), X_BAD_DONOR
    if flags & NEW_UNIFORM:
        if not _int_in(nsz[nrow, 0], 1, L_new):
            return _old_tree(old, L_old), X_BAD_DONOR
        j = pick_node(jn, int(nsz[nrow, 0]))
    else:
        j = int(jn)
    if j is None or not (0 <= j < L_new) or not _int_in(nsz[nrow, j], 1, L_new - j):
        return _old_tree(old, L_old), X_BAD_DONOR
    e = j + int(nsz[nrow, j])
    sub = (nt[nrow, j:e], nv[nrow, j:e], nsz[nrow, j:e])
    return exchange_tree(old, k, sub, max_len, L_old)
