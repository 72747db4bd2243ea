"""Plain CPU oracle for tree-GP symbolic-regression fitness evaluation.

TEST INFRASTRUCTURE. Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import or run this module. It shares no
code, tables or constants with the device library.

What it computes, and where the paper defines it:

* Node semantics (§II-A): a constant node yields its value, a variable node
  yields x[val], a function node applies its function to its children.
* Encoding (§III-A): prefix node sequence stored as three rows (type,
  value, subtree size), NaN after the tree's len entries; len is size[0].
* Evaluation order (§III-C, closing paragraph): nodes are visited from the
  last to the first; leaves push their value, a function pops as many
  values as its arity and pushes its result.
* Multi-output trees (§IV-C and the multi-output tree figure): a Modi node
  adds its function value to its output slot (contributions are summed) and
  hands its rightmost child's value to its parent.
* Fitness (§III-C first paragraph, Alg. 1): squared error between the
  prediction and the targets over all data points, reduced to a mean per
  tree (lower is better; Alg. 1 maximises its negation).

Everything runs in float64 on the float32 inputs, vectorised over data
points only; trees and nodes are plain Python loops. The float32 "shadow"
evaluator rounds every node result to float32 and exists only to classify
trees as well- or ill-conditioned for comparisons.

Readings where the paper is silent (type codes, op ids, operand order,
protection rules, Modi output rules) are fixed in the module constants and
the functions below.
"""

import math

import numpy as np

# ---------------------------------------------------------------- encoding
T_VAR, T_CONST, T_FUNC, T_MODI0 = 0, 1, 2, 3

# op id -> (name, arity)
OPS = (
    ("add", 2), ("sub", 2), ("mul", 2), ("div", 2),
    ("sin", 1), ("cos", 1), ("tanh", 1), ("exp", 1), ("log", 1),
    ("max", 2), ("min", 2), ("tan", 1),
)
N_OPS = len(OPS)

TAU = float(np.float32(1e-6))      # protected division: |b| < TAU gives 1
LOG_EPS = float(np.float32(1e-6))  # protected log: log(|a| + LOG_EPS)
EXP_CLAMP = 20.0                   # exp argument clamped to [-20, 20]

# per-tree status codes; a tree's status is the smallest code that applies
OK, E_LEN, E_NAN, E_TAIL, E_TYPE, E_OP, E_VAR, E_SIZE = range(8)


class Decoded:
    """A validated tree: node list plus the integer plan figures."""

    __slots__ = ("status", "length", "max_stack", "n_const", "n_modi", "bucket",
                 "kind", "arg", "out", "size")

    def __init__(self):
        self.status = OK
        self.length = 0
        self.max_stack = 0
        self.n_const = 0
        self.n_modi = 0
        self.bucket = 0
        self.kind = []   # T_VAR / T_CONST / T_FUNC per node
        self.arg = []    # var index (int), constant (float) or op id (int)
        self.out = []    # Modi output index, or -1
        self.size = []


def _is_int(x):
    return math.isfinite(x) and float(x) == math.floor(x)


def length_bucket(n):
    """Power-of-two length class: 0 for len 1, else ceil(log2(len))."""
    return 0 if n <= 1 else (int(n) - 1).bit_length()


def decode(type_row, value_row, size_row, V, n_out):
    """Validate one NaN-padded tree row and return its Decoded form.

    Checks, each giving a status code (the smallest applicable code wins):
    E_LEN  size[0] is not an integer in [1, Lmax];
    E_NAN  a NaN in any of the three rows inside the first len entries;
    E_TAIL a non-NaN entry at or after len (the padding rule of §III-A);
    E_TYPE a type that is not 0, 1, 2 or 3+o with o < n_out;
    E_OP   a function/Modi value that is not an integer op id;
    E_VAR  a variable value that is not an integer in [0, V);
    E_SIZE (only when none of the above) the subtree sizes do not describe
           the prefix sequence: with c1 = i+1 and c2 = c1+size[c1],
           size[i] must be 1, 1+size[c1] or 1+size[c1]+size[c2] for arity
           0, 1, 2, with every child inside the tree (§III-A size array).
    Invalid trees report zero for every other figure.
    """
    t = [float(x) for x in type_row]
    v = [float(x) for x in value_row]
    s = [float(x) for x in size_row]
    Lmax = len(t)
    d = Decoded()
    s0 = s[0] if Lmax else float("nan")
    if not (_is_int(s0) and 1 <= s0 <= Lmax):
        d.status = E_LEN
        return d
    n = int(s0)
    codes = set()
    for i in range(n):
        if math.isnan(t[i]) or math.isnan(v[i]) or math.isnan(s[i]):
            codes.add(E_NAN)
    for i in range(n, Lmax):
        if not (math.isnan(t[i]) and math.isnan(v[i]) and math.isnan(s[i])):
            codes.add(E_TAIL)
    kinds, args, outs = [], [], []
    for i in range(n):
        ti, vi = t[i], v[i]
        if math.isnan(ti) or math.isnan(vi):
            kinds.append(None); args.append(None); outs.append(-1)
            continue
        if not _is_int(ti) or ti < 0 or ti >= T_MODI0 + n_out:
            codes.add(E_TYPE)
            kinds.append(None); args.append(None); outs.append(-1)
            continue
        ti = int(ti)
        if ti == T_CONST:
            kinds.append(T_CONST); args.append(vi); outs.append(-1)
        elif ti == T_VAR:
            if not (_is_int(vi) and 0 <= vi < V):
                codes.add(E_VAR)
            kinds.append(T_VAR); args.append(int(vi) if _is_int(vi) else None); outs.append(-1)
        else:
            if not (_is_int(vi) and 0 <= vi < N_OPS):
                codes.add(E_OP)
            kinds.append(T_FUNC); args.append(int(vi) if _is_int(vi) else None)
            outs.append(ti - T_MODI0 if ti >= T_MODI0 else -1)
    if codes:
        d.status = min(codes)
        return d
    sizes = []
    for i in range(n):
        if not _is_int(s[i]):
            d.status = E_SIZE
            return d
        sizes.append(int(s[i]))
    for i in range(n):
        a = OPS[args[i]][1] if kinds[i] == T_FUNC else 0
        want = 1
        c = i + 1
        for _ in range(a):
            if c >= n:
                d.status = E_SIZE
                return d
            if sizes[c] < 1:
                d.status = E_SIZE
                return d
            want += sizes[c]
            c += sizes[c]
        if sizes[i] != want or i + sizes[i] > n:
            d.status = E_SIZE
            return d
    # plan figures: stack depth of the reversed-prefix evaluation (§III-C)
    depth = 0
    best = 0
    for i in range(n - 1, -1, -1):
        a = OPS[args[i]][1] if kinds[i] == T_FUNC else 0
        depth = depth - a + 1
        best = max(best, depth)
    d.length = n
    d.max_stack = best
    d.n_const = sum(1 for k in kinds if k == T_CONST)
    d.n_modi = sum(1 for o in outs if o >= 0)
    d.bucket = length_bucket(n)
    d.kind, d.arg, d.out, d.size = kinds, args, outs, sizes
    return d


def plan(pop_type, pop_value, pop_size, V, n_out):
    """Integer plan figures for a population: int64 [P][6] =
    (status, len, max_stack, n_const, n_modi, bucket)."""
    P = pop_type.shape[0]
    r = np.zeros((P, 6), np.int64)
    for p in range(P):
        d = decode(pop_type[p], pop_value[p], pop_size[p], V, n_out)
        r[p] = (d.status, d.length, d.max_stack, d.n_const, d.n_modi, d.bucket)
    return r


# ---------------------------------------------------------------- operators (float64)
def apply_op(op, a, b=None):
    """Value of op on float64 arrays (b is None for unary ops)."""
    with np.errstate(all="ignore"):
        if op == 0:
            return a + b
        if op == 1:
            return a - b
        if op == 2:
            return a * b
        if op == 3:
            return np.where(np.abs(b) < TAU, 1.0, a / np.where(np.abs(b) < TAU, 1.0, b))
        if op == 4:
            return np.sin(a)
        if op == 5:
            return np.cos(a)
        if op == 6:
            return np.tanh(a)
        if op == 7:
            return np.exp(np.where(a > EXP_CLAMP, EXP_CLAMP, np.where(a < -EXP_CLAMP, -EXP_CLAMP, a)))
        if op == 8:
            return np.log(np.abs(a) + LOG_EPS)
        if op == 9:
            return np.fmax(a, b)
        if op == 10:
            return np.fmin(a, b)
        if op == 11:
            return np.tan(a)
    raise ValueError(op)


def op_partials(op, a, b=None):
    """(d f/d a, d f/d b) on float64 arrays, with the conventions at kinks:
    protected div and the clamped exp have zero slope where they are flat;
    protected log has slope sign(a)/(|a|+eps) and 0 at a == 0; max/min send
    the whole slope to the operand they return (the first one at a tie or when
    the other is NaN)."""
    one = np.ones_like(a)
    zero = np.zeros_like(a)
    with np.errstate(all="ignore"):
        if op == 0:
            return one, one
        if op == 1:
            return one, -one
        if op == 2:
            return b, a
        if op == 3:
            small = np.abs(b) < TAU
            bb = np.where(small, 1.0, b)
            return np.where(small, 0.0, 1.0 / bb), np.where(small, 0.0, -a / (bb * bb))
        if op == 4:
            return np.cos(a), None
        if op == 5:
            return -np.sin(a), None
        if op == 6:
            th = np.tanh(a)
            return 1.0 - th * th, None
        if op == 7:
            inside = (a >= -EXP_CLAMP) & (a <= EXP_CLAMP)
            return np.where(inside, np.exp(np.where(inside, a, 0.0)), 0.0), None
        if op == 8:
            return np.sign(a) / (np.abs(a) + LOG_EPS), None
        if op == 9:
            pick_a = (a >= b) | np.isnan(b)
            return np.where(pick_a, 1.0, 0.0), np.where(pick_a, 0.0, 1.0)
        if op == 10:
            pick_a = (a <= b) | np.isnan(b)
            return np.where(pick_a, 1.0, 0.0), np.where(pick_a, 0.0, 1.0)
        if op == 11:
            tn = np.tan(a)
            return 1.0 + tn * tn, None
    raise ValueError(op)


# ---------------------------------------------------------------- evaluation
def _leaf(d, i, X, D):
    if d.kind[i] == T_CONST:
        return np.full(D, float(np.float64(d.arg[i])))
    return np.asarray(X[d.arg[i]], np.float64)


def _outputs(d, root, contrib, n_out, D):
    """Outputs of a tree. A tree with no Modi node has out[0] = root value and
    zeros elsewhere. A tree with Modi nodes has out[o] = sum of the
    contributions tagged o, added in increasing node index; its root value
    is not an output by itself."""
    out = np.zeros((n_out, D))
    if d.n_modi == 0:
        out[0] = root
        return out
    for i in sorted(contrib):
        o, r = contrib[i]
        out[o] = out[o] + r
    return out


def eval_stack(d, X, n_out):
    """Outputs [n_out][D] of a valid tree by the reversed-prefix stack machine (§III-C).

    The first child (index i+1) is on top of the stack when node i runs, so
    a binary node computes f(first, second) = f(pop(), pop())."""
    X = np.asarray(X, np.float64)
    D = X.shape[1]
    stack = []
    contrib = {}
    for i in range(d.length - 1, -1, -1):
        if d.kind[i] != T_FUNC:
            stack.append(_leaf(d, i, X, D))
            continue
        op = d.arg[i]
        if OPS[op][1] == 2:
            a = stack.pop()
            b = stack.pop()
            r = apply_op(op, a, b)
            right = b
        else:
            a = stack.pop()
            r = apply_op(op, a)
            right = a
        if d.out[i] >= 0:
            contrib[i] = (d.out[i], r)
            stack.append(right)
        else:
            stack.append(r)
    assert len(stack) == 1
    return _outputs(d, stack[0], contrib, n_out, D)


def eval_recursive(d, X, n_out):
    """Outputs [n_out][D] by recursive descent over subtree sizes: an
    evaluator independent of the stack machine, used to cross-check it."""
    X = np.asarray(X, np.float64)
    D = X.shape[1]
    contrib = {}

    def val(i):
        if d.kind[i] != T_FUNC:
            return _leaf(d, i, X, D)
        op = d.arg[i]
        c1 = i + 1
        a = val(c1)
        if OPS[op][1] == 2:
            b = val(c1 + d.size[c1])
            r = apply_op(op, a, b)
            right = b
        else:
            r = apply_op(op, a)
            right = a
        if d.out[i] >= 0:
            contrib[i] = (d.out[i], r)
            return right
        return r

    root = val(0)
    return _outputs(d, root, contrib, n_out, D)


def _r32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def apply_op_shadow32(op, a, b=None):
    """Float32 shadow of apply_op: operands are float32 values, the result is
    rounded to float32. For + - * / the float64 result rounded once equals the
    correctly rounded float32 result; branch tests use the float32 operands."""
    with np.errstate(all="ignore"):
        if op == 8:
            return _r32(np.log(_r32(np.abs(a) + LOG_EPS)))
        return _r32(apply_op(op, a, b))


# Unary transcendental ops: sin, cos, tanh, exp, log, tan. A float32 library
# implementation of these may differ from the correctly rounded result by a
# few ulp, so classification shadows may move their results by a random
# number of ulps (see Ulps).
TRANSCENDENTAL = frozenset((4, 5, 6, 7, 8, 11))


class Ulps:
    """Random perturbation of transcendental results in the float32 shadow:
    each result (per node and point) moves by an integer number of float32
    ulps drawn uniformly from [-k, k], from a generator seeded by `seed`."""

    def __init__(self, k, seed):
        self.k = int(k)
        self.rng = np.random.default_rng(seed)

    def __call__(self, op, r):
        if self.k <= 0 or op not in TRANSCENDENTAL:
            return r
        r32 = np.asarray(r, np.float64).astype(np.float32)
        steps = self.rng.integers(-self.k, self.k + 1, size=r32.shape)
        out = r32.copy()
        for direction, sel in ((np.float32(np.inf), steps > 0), (np.float32(-np.inf), steps < 0)):
            cur = r32.copy()
            for n in range(1, self.k + 1):
                cur = np.nextafter(cur, direction)
                out = np.where(sel & (np.abs(steps) == n), cur, out)
        return out.astype(np.float64)


def eval_shadow32(d, X, n_out, ulps=None):
    """Float32 shadow evaluation (same order as eval_stack). With `ulps` (an
    Ulps), transcendental results are perturbed as a library might round."""
    X = _r32(X)
    D = X.shape[1]
    stack = []
    contrib = {}
    for i in range(d.length - 1, -1, -1):
        if d.kind[i] != T_FUNC:
            stack.append(_r32(_leaf(d, i, X, D)))
            continue
        op = d.arg[i]
        if OPS[op][1] == 2:
            a = stack.pop(); b = stack.pop()
            r = apply_op_shadow32(op, a, b); right = b
        else:
            a = stack.pop()
            r = apply_op_shadow32(op, a); right = a
        if ulps is not None:
            r = ulps(op, r)
        if d.out[i] >= 0:
            contrib[i] = (d.out[i], r)
            stack.append(right)
        else:
            stack.append(r)
    out = np.zeros((n_out, D))
    if d.n_modi == 0:
        out[0] = stack[0]
    else:
        for i in sorted(contrib):
            o, r = contrib[i]
            out[o] = _r32(out[o] + r)
    return out


# ---------------------------------------------------------------- fitness
def _Y(Y, n_out, D):
    return np.asarray(Y, np.float64).reshape(n_out, D)


def mse_tree(d, X, Y, n_out, evaluator=eval_stack):
    """Fitness of one decoded tree: sum over outputs of mean squared error.
    NaN for an invalid tree."""
    if d.status != OK:
        return float("nan")
    X = np.asarray(X, np.float64)
    D = X.shape[1]
    out = evaluator(d, X, n_out)
    with np.errstate(all="ignore"):
        e = out - _Y(Y, n_out, D)
        return float(np.sum(e * e) / D)


def mse_tree_shadow32(d, X, Y, n_out, ulps=None):
    """Shadow fitness: float32 residuals and squares, float64 sum, float32 result."""
    if d.status != OK:
        return float("nan")
    D = np.asarray(X).shape[1]
    out = eval_shadow32(d, X, n_out, ulps)
    with np.errstate(all="ignore"):
        e = _r32(out - _r32(_Y(Y, n_out, D)))
        e2 = _r32(e * e)
        return float(np.float32(np.sum(e2) / D))


def mse(pop_type, pop_value, pop_size, X, Y, n_out=1, rows=None, evaluator=eval_stack):
    """float64 fitness per tree (all rows, or the given row indices)."""
    X = np.asarray(X)
    V = X.shape[0]
    rows = range(pop_type.shape[0]) if rows is None else rows
    return np.array([mse_tree(decode(pop_type[p], pop_value[p], pop_size[p], V, n_out), X, Y, n_out,
                              evaluator) for p in rows])


def mse_shadow32(pop_type, pop_value, pop_size, X, Y, n_out=1, rows=None, ulp=0, seed=0):
    """Float32 shadow fitness per tree; ulp > 0 perturbs transcendental results
    by up to `ulp` float32 ulps (one generator seeded by `seed` for the call)."""
    X = np.asarray(X)
    V = X.shape[0]
    rows = range(pop_type.shape[0]) if rows is None else rows
    ulps = Ulps(ulp, seed) if ulp else None
    return np.array([mse_tree_shadow32(decode(pop_type[p], pop_value[p], pop_size[p], V, n_out), X, Y, n_out,
                                       ulps) for p in rows])


def predict(pop_type, pop_value, pop_size, X, n_out=1, rows=None):
    """Outputs float64 [len(rows)][n_out][D]; NaN rows for invalid trees."""
    X = np.asarray(X)
    V, D = X.shape
    rows = list(range(pop_type.shape[0]) if rows is None else rows)
    res = np.full((len(rows), n_out, D), np.nan)
    for k, p in enumerate(rows):
        d = decode(pop_type[p], pop_value[p], pop_size[p], V, n_out)
        if d.status == OK:
            res[k] = eval_stack(d, X, n_out)
    return res


# ---------------------------------------------------------------- gradients
def grad_tree(d, X, Y, n_out, g=1.0, shadow=False, ulps=None):
    """Reverse-mode gradient of g * fitness for one tree, with a full tape.

    Returns (mse, grad_value [len], grad_X [V][D]). grad_value is non-zero
    only at constant nodes. Output adjoint: g * 2 (out_o - Y_o) / D. A plain
    function node passes adj * df/dchild to each child; a Modi node for
    output o passes (output adjoint of o) * df/dchild to each child and also
    its own parent adjoint to its rightmost child (the value it hands up).

    shadow=True is the float32 shadow of the same sweep: node values come
    from the float32 shadow operators, and the residual, the output adjoint,
    each partial derivative, each product and each adjoint sum are rounded
    to float32 (the per-constant sums over points stay float64). It only
    classifies gradient components as well- or ill-conditioned.
    """
    q = _r32 if shadow else (lambda v: v)
    if shadow and ulps is not None:
        def op_val(op, a, b=None):
            return ulps(op, apply_op_shadow32(op, a, b))
    else:
        op_val = apply_op_shadow32 if shadow else apply_op
    X = q(np.asarray(X, np.float64))
    V, D = X.shape
    n = d.length
    val = [None] * n
    contrib = {}
    stack = []
    for i in range(n - 1, -1, -1):
        if d.kind[i] != T_FUNC:
            val[i] = q(_leaf(d, i, X, D))
            stack.append(val[i])
            continue
        op = d.arg[i]
        if OPS[op][1] == 2:
            a = stack.pop(); b = stack.pop()
            r = op_val(op, a, b); right = b
        else:
            a = stack.pop()
            r = op_val(op, a); right = a
        if d.out[i] >= 0:
            contrib[i] = (d.out[i], r)
            val[i] = right
        else:
            val[i] = r
        stack.append(val[i])
    out = _outputs(d, stack[0], contrib, n_out, D)
    Yd = q(_Y(Y, n_out, D))
    with np.errstate(all="ignore"):
        resid = q(q(out) - Yd)
        m = float(np.sum(resid * resid) / D)
        gout = q(q(q(g * 2.0) * resid) * q(1.0 / D)) if shadow else g * 2.0 * resid / D
    adj = [np.zeros(D) for _ in range(n)]
    if d.n_modi == 0:
        adj[0] = gout[0].copy()
    gv = np.zeros(n)
    gX = np.zeros((V, D))
    with np.errstate(all="ignore"):
        for i in range(n):
            if d.kind[i] == T_CONST:
                gv[i] = float(np.sum(adj[i]))
                continue
            if d.kind[i] == T_VAR:
                gX[d.arg[i]] += adj[i]
                continue
            op = d.arg[i]
            c1 = i + 1
            kids = [c1] if OPS[op][1] == 1 else [c1, c1 + d.size[c1]]
            if len(kids) == 2:
                da, db = op_partials(op, val[kids[0]], val[kids[1]])
                parts = [q(da), q(db)]
            else:
                da, _ = op_partials(op, val[kids[0]])
                parts = [q(da)]
            if d.out[i] >= 0:
                go = gout[d.out[i]]
                for c, p in zip(kids, parts):
                    adj[c] = q(adj[c] + q(go * p))
                adj[kids[-1]] = q(adj[kids[-1]] + adj[i])
            else:
                for c, p in zip(kids, parts):
                    adj[c] = q(adj[c] + q(adj[i] * p))
    return m, gv, gX


def grad(pop_type, pop_value, pop_size, X, Y, n_out=1, rows=None, g=None, shadow=False, ulp=0, seed=0):
    """Gradients of sum_t g_t * fitness_t.

    Returns (mse [R], grad_value [R][Lmax] (zero off constant nodes, zero for
    invalid trees), grad_X [V][D] summed over the listed trees). shadow=True
    gives the float32 shadow of the same gradients (see grad_tree); ulp > 0
    also perturbs its transcendental node values (see Ulps)."""
    X = np.asarray(X, np.float64)
    V, D = X.shape
    rows = list(range(pop_type.shape[0]) if rows is None else rows)
    Lmax = pop_type.shape[1]
    m = np.full(len(rows), np.nan)
    gv = np.zeros((len(rows), Lmax))
    gX = np.zeros((V, D))
    ulps = Ulps(ulp, seed) if (shadow and ulp) else None
    for k, p in enumerate(rows):
        d = decode(pop_type[p], pop_value[p], pop_size[p], V, n_out)
        if d.status != OK:
            continue
        gt = 1.0 if g is None else float(g[p])
        m[k], gvt, gXt = grad_tree(d, X, Y, n_out, gt, shadow=shadow, ulps=ulps)
        gv[k, :d.length] = gvt
        gX += gXt
    return m, gv, gX


def fd_grad_const(pop_type, pop_value, pop_size, X, Y, p, i, h=1e-4, n_out=1):
    """Central difference of fitness of tree p with respect to the constant at node i."""
    V = np.asarray(X).shape[0]
    base = decode(pop_type[p], pop_value[p], pop_size[p], V, n_out)
    c0 = float(base.arg[i])
    vals = []
    for sgn in (1.0, -1.0):
        base.arg[i] = c0 + sgn * h
        vals.append(mse_tree(base, X, Y, n_out))
    base.arg[i] = c0
    return (vals[0] - vals[1]) / (2 * h)


def fd_grad_x(pop_type, pop_value, pop_size, X, Y, rows, v, j, h=1e-4, n_out=1, g=None):
    """Central difference of sum_t g_t fitness_t with respect to X[v][j]."""
    X = np.asarray(X, np.float64).copy()
    x0 = X[v, j]
    tot = []
    for sgn in (1.0, -1.0):
        X[v, j] = x0 + sgn * h
        m = mse(pop_type, pop_value, pop_size, X, Y, n_out, rows)
        w = np.ones(len(m)) if g is None else np.asarray([g[r] for r in rows])
        tot.append(float(np.sum(w * m)))
    return (tot[0] - tot[1]) / (2 * h)


def adam_reference(theta, grads_fn, steps, lr=1e-2, betas=(0.9, 0.999), eps=1e-8):
    """Adam (Kingma & Ba, 2015) in float64 on a parameter vector; grads_fn(theta) -> gradient."""
    theta = np.asarray(theta, np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    for t in range(1, steps + 1):
        gr = grads_fn(theta)
        m = betas[0] * m + (1 - betas[0]) * gr
        v = betas[1] * v + (1 - betas[1]) * gr * gr
        mh = m / (1 - betas[0] ** t)
        vh = v / (1 - betas[1] ** t)
        theta = theta - lr * mh / (np.sqrt(vh) + eps)
    return theta
