"""Torch-facing wrappers of the C-ABI (same names as the C entry points).

Torch supplies device memory and the current stream; the wrappers only
check tensor properties, build the ABI structs and call the library.
Populations are three float32 CUDA tensors [P][Lmax] (type, value, size) in
the NaN-padded prefix encoding of the paper's §III-A; X is [V][D] float32
(variable-major), Y is [n_out][D] float32.
"""

import ctypes
import os

import torch

from . import _lib
from ._lib import TgpCfg, TgpData, TgpExchange, TgpGenCfg, TgpPop, check

__all__ = ["Population", "Workspace", "cfg", "workspace_bytes", "plan", "eval_mse", "eval_mse_noalloc",
           "eval_multi_output", "eval_accuracy",
           "eval_mse_grad", "autotune", "subtree_exchange", "crossover", "mutation", "generate", "TreeMSE"]


def _dev(t, name, dtype=torch.float32):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if t.dim() >= 1 and t.stride(-1) != 1:
        raise ValueError(f"{name} must have unit stride in its last dimension")
    return t


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Population:
    """Three [P][Lmax] float32 device tensors sharing one row stride."""

    def __init__(self, type, value, size):
        for n, t in (("type", type), ("value", value), ("size", size)):
            _dev(t, n)
            if t.dim() != 2:
                raise ValueError(f"{n} must be 2-D [P][Lmax]")
        if not (type.shape == value.shape == size.shape):
            raise ValueError("type, value and size must have the same shape")
        if not (type.stride(0) == value.stride(0) == size.stride(0)):
            raise ValueError("type, value and size must share one row stride")
        self.type, self.value, self.size = type, value, size

    @property
    def P(self):
        return self.type.shape[0]

    @property
    def Lmax(self):
        return self.type.shape[1]

    def abi(self):
        return TgpPop(self.type.data_ptr(), self.value.data_ptr(), self.size.data_ptr(), self.P, self.Lmax,
                      max(self.type.stride(0), self.Lmax))


def _data(X, Y=None, n_out=None):
    _dev(X, "X")
    if X.dim() != 2:
        raise ValueError("X must be 2-D [V][D]")
    V, D = X.shape
    ldy = 0
    yp = None
    if Y is not None:
        _dev(Y, "Y")
        if Y.dim() == 1:
            Y = Y.unsqueeze(0)
        if Y.shape[1] != D:
            raise ValueError("Y must be [n_out][D] with the same D as X")
        n_out = Y.shape[0] if n_out is None else n_out
        if Y.shape[0] != n_out:
            raise ValueError("Y rows must equal n_out")
        ldy = Y.stride(0) if Y.shape[0] > 1 else D
        yp = Y.data_ptr()
    n_out = 1 if n_out is None else int(n_out)
    ldx = X.stride(0) if V > 1 else D
    return TgpData(X.data_ptr(), V, D, ldx, yp, n_out, ldy), Y


def cfg(mode=0, block_waves=0, points_per_lane=0, trees_per_unit=0, flags=0):
    """Launch configuration (zeros = defaults). mode: 0 auto, 1 tree-major, 2 point-major, 3 persistent."""
    if isinstance(mode, TgpCfg):
        return mode
    if isinstance(mode, dict):
        return TgpCfg(**mode)
    return TgpCfg(int(mode), int(block_waves), int(points_per_lane), int(trees_per_unit), int(flags))


def _cfgp(c):
    return None if c is None else ctypes.byref(cfg(c))


def workspace_bytes(pop, X=None, n_out=1, want_grad=False, V=None, D=None):
    lib = _lib.load()
    p = pop.abi()
    if X is not None:
        d, _ = _data(X, None, n_out)
        dp = ctypes.byref(d)
    else:
        dp = None
    n = lib.tgp_workspace_bytes(ctypes.byref(p), dp, int(n_out), int(bool(want_grad)))
    if n == 0:
        raise _lib.TgpError(_lib.TGP_E_UNSUPPORTED, "tgp_workspace_bytes")
    return n


class Workspace:
    """A caller-owned device workspace that grows on demand (allocation happens
    here, outside the library's evaluation calls)."""

    def __init__(self, device="cuda"):
        self.buf = None
        self.device = device

    def get(self, nbytes):
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self.buf

    def ptr_size(self, nbytes):
        b = self.get(nbytes)
        return ctypes.c_void_p(b.data_ptr()), b.numel()


_default_ws = {}


def _ws(ws, nbytes, device):
    if ws is None:
        key = str(device)
        ws = _default_ws.setdefault(key, Workspace(device))
    return ws.ptr_size(nbytes)


def plan(pop, V, n_out=1, config=None, ws=None, stream=None):
    """Validate and plan every tree. Returns (info int32 [P][6], tree_status int32 [P])."""
    lib = _lib.load()
    p = pop.abi()
    dev = pop.type.device
    info = torch.empty((pop.P, 6), dtype=torch.int32, device=dev)
    st = torch.empty((pop.P,), dtype=torch.int32, device=dev)
    nbytes = lib.tgp_workspace_bytes(ctypes.byref(p), None, int(n_out), 0)
    if nbytes == 0:
        raise _lib.TgpError(_lib.TGP_E_UNSUPPORTED, "tgp_plan")
    wp, wn = _ws(ws, nbytes, dev)
    check(lib.tgp_plan(ctypes.byref(p), int(V), int(n_out), _cfgp(config), ctypes.c_void_p(info.data_ptr()),
                       ctypes.c_void_p(st.data_ptr()), wp, wn, _stream(stream)), "tgp_plan")
    return info, st


def eval_mse(pop, X, y, config=None, ws=None, out=None, tree_status=None, stream=None):
    """Fitness (mean squared error) of every tree against y [D] or [1][D]. Returns float32 [P]."""
    lib = _lib.load()
    d, _ = _data(X, y, 1)
    p = pop.abi()
    mse = torch.empty((pop.P,), dtype=torch.float32, device=X.device) if out is None else out
    nbytes = lib.tgp_workspace_bytes(ctypes.byref(p), ctypes.byref(d), 1, 0)
    if nbytes == 0:
        raise _lib.TgpError(_lib.TGP_E_UNSUPPORTED, "tgp_eval_mse")
    wp, wn = _ws(ws, nbytes, X.device)
    stp = ctypes.c_void_p(tree_status.data_ptr()) if tree_status is not None else None
    check(lib.tgp_eval_mse(ctypes.byref(p), ctypes.byref(d), _cfgp(config), ctypes.c_void_p(mse.data_ptr()), stp,
                           wp, wn, _stream(stream)), "tgp_eval_mse")
    return mse


def eval_mse_noalloc(pop, X, y, config=None, out=None, tree_status=None, stream=None):
    """eval_mse through tgp_eval_mse_noalloc: the library's static scratch buffer replaces the
    workspace, so the call allocates nothing on the device (pass `out`, and `tree_status` if
    wanted, to allocate nothing here either). Calls on one device must not overlap in time.
    Returns float32 [P]."""
    lib = _lib.load()
    d, _ = _data(X, y, 1)
    p = pop.abi()
    mse = torch.empty((pop.P,), dtype=torch.float32, device=X.device) if out is None else out
    stp = ctypes.c_void_p(tree_status.data_ptr()) if tree_status is not None else None
    check(lib.tgp_eval_mse_noalloc(ctypes.byref(p), ctypes.byref(d), _cfgp(config), ctypes.c_void_p(mse.data_ptr()),
                                   stp, _stream(stream)), "tgp_eval_mse_noalloc")
    return mse


def eval_accuracy(pop, X, labels, n_classes, config=None, ws=None, out=None, tree_status=None, stream=None):
    """Classification accuracy of every tree: the argmax of its n_classes outputs against labels
    (float32 [D] or [1][D] holding class ids). Returns float32 [P]."""
    lib = _lib.load()
    _dev(labels, "labels")
    lab = labels.reshape(1, -1)
    d, _ = _data(X, lab, 1)
    d.n_out = int(n_classes)
    p = pop.abi()
    acc = torch.empty((pop.P,), dtype=torch.float32, device=X.device) if out is None else out
    nbytes = lib.tgp_workspace_bytes(ctypes.byref(p), ctypes.byref(d), int(n_classes), 0)
    if nbytes == 0:
        raise _lib.TgpError(_lib.TGP_E_UNSUPPORTED, "tgp_eval_accuracy")
    wp, wn = _ws(ws, nbytes, X.device)
    stp = ctypes.c_void_p(tree_status.data_ptr()) if tree_status is not None else None
    check(lib.tgp_eval_accuracy(ctypes.byref(p), ctypes.byref(d), _cfgp(config), ctypes.c_void_p(acc.data_ptr()),
                                stp, wp, wn, _stream(stream)), "tgp_eval_accuracy")
    return acc


def eval_multi_output(pop, X, Y=None, n_out=None, want_mse=True, want_pred=False, config=None, ws=None,
                      tree_status=None, stream=None, out=None):
    """Multi-output evaluation. Returns (mse [P] or None, pred [P][n_out][D] or None)."""
    lib = _lib.load()
    if Y is None:
        want_mse = False
    d, Y = _data(X, Y, n_out)
    n_out = d.n_out
    p = pop.abi()
    D = X.shape[1]
    mse = (torch.empty((pop.P,), dtype=torch.float32, device=X.device) if out is None else out) if want_mse else None
    pred = torch.empty((pop.P, n_out, D), dtype=torch.float32, device=X.device) if want_pred else None
    nbytes = lib.tgp_workspace_bytes(ctypes.byref(p), ctypes.byref(d), n_out, 0)
    if nbytes == 0:
        raise _lib.TgpError(_lib.TGP_E_UNSUPPORTED, "tgp_eval_multi_output")
    wp, wn = _ws(ws, nbytes, X.device)
    stp = ctypes.c_void_p(tree_status.data_ptr()) if tree_status is not None else None
    check(lib.tgp_eval_multi_output(
        ctypes.byref(p), ctypes.byref(d), _cfgp(config),
        ctypes.c_void_p(mse.data_ptr()) if mse is not None else None,
        ctypes.c_void_p(pred.data_ptr()) if pred is not None else None, D, stp, wp, wn, _stream(stream)),
        "tgp_eval_multi_output")
    return mse, pred


def eval_mse_grad(pop, X, y, grad_mse=None, want_grad_value=True, want_grad_x=True, config=None, ws=None,
                  tree_status=None, stream=None):
    """Fitness and gradients against y [D] or Y [n_out][D] (n_out 1..4: multi-output trees, fitness
    summed over outputs). Returns (mse [P], grad_value [P][Lmax] or None, grad_X [V][D] or None)."""
    lib = _lib.load()
    d, _ = _data(X, y)
    p = pop.abi()
    mse = torch.empty((pop.P,), dtype=torch.float32, device=X.device)
    gv = torch.empty((pop.P, pop.type.stride(0)), dtype=torch.float32, device=X.device) if want_grad_value else None
    gx = torch.empty((X.shape[0], d.ldx), dtype=torch.float32, device=X.device) if want_grad_x else None
    nbytes = lib.tgp_workspace_bytes(ctypes.byref(p), ctypes.byref(d), d.n_out, 1)
    if nbytes == 0:
        raise _lib.TgpError(_lib.TGP_E_UNSUPPORTED, "tgp_eval_mse_grad")
    wp, wn = _ws(ws, nbytes, X.device)
    gm = None
    if grad_mse is not None:
        _dev(grad_mse, "grad_mse")
        gm = ctypes.c_void_p(grad_mse.data_ptr())
    stp = ctypes.c_void_p(tree_status.data_ptr()) if tree_status is not None else None
    check(lib.tgp_eval_mse_grad(
        ctypes.byref(p), ctypes.byref(d), _cfgp(config), gm, ctypes.c_void_p(mse.data_ptr()),
        ctypes.c_void_p(gv.data_ptr()) if gv is not None else None,
        ctypes.c_void_p(gx.data_ptr()) if gx is not None else None, stp, wp, wn, _stream(stream)),
        "tgp_eval_mse_grad")
    if gv is not None:
        gv = gv[:, :pop.Lmax]
    if gx is not None:
        gx = gx[:, :X.shape[1]]
    return mse, gv, gx


def autotune(pop, X, Y, n_out=None, want_grad=False, ws=None, stream=None):
    """Time the candidate schedules on this workload and cache the fastest. Returns the chosen cfg dict."""
    lib = _lib.load()
    d, _ = _data(X, Y, n_out)
    p = pop.abi()
    nbytes = lib.tgp_workspace_bytes(ctypes.byref(p), ctypes.byref(d), d.n_out, int(bool(want_grad)))
    if nbytes == 0:
        raise _lib.TgpError(_lib.TGP_E_UNSUPPORTED, "tgp_autotune")
    wp, wn = _ws(ws, nbytes, X.device)
    out = TgpCfg()
    check(lib.tgp_autotune(ctypes.byref(p), ctypes.byref(d), d.n_out, int(bool(want_grad)), ctypes.byref(out),
                           wp, wn, _stream(stream)), "tgp_autotune")
    return out.as_dict()


def op_apply(op, x, out=None, stream=None):
    """The evaluation kernels' unary operator `op` (sin 4, cos 5, tanh 6, exp 7, log 8, tan 11, with
    the protection of exp and log) applied elementwise to a contiguous float32 device tensor."""
    _dev(x, "x")
    if not x.is_contiguous():
        raise ValueError("x must be contiguous")
    y = torch.empty_like(x) if out is None else out
    check(_lib.load().tgp_op_apply(int(op), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                   x.numel(), _stream(stream)), "tgp_op_apply")
    return y


def autotune_cached(pop, X, Y, n_out=None, want_grad=False):
    """The configuration a call without one would take from the autotune cache for this workload
    on the current device (a cfg dict), or None."""
    lib = _lib.load()
    d, _ = _data(X, Y, n_out)
    p = pop.abi()
    out, found = TgpCfg(), ctypes.c_int32(0)
    check(lib.tgp_autotune_cached(ctypes.byref(p), ctypes.byref(d), d.n_out, int(bool(want_grad)),
                                  ctypes.byref(out), ctypes.byref(found)), "tgp_autotune_cached")
    return out.as_dict() if found.value else None


def autotune_cache_load(path):
    """Read an autotune cache file (one JSON line per shape) into the process's cache.
    Returns (entries loaded, lines rejected)."""
    lib = _lib.load()
    n_ok, n_bad = ctypes.c_int32(0), ctypes.c_int32(0)
    check(lib.tgp_autotune_cache_load(os.fsencode(path), ctypes.byref(n_ok), ctypes.byref(n_bad)),
          "tgp_autotune_cache_load")
    return n_ok.value, n_bad.value


def autotune_cache_save(path):
    """Write every cached launch configuration to an autotune cache file."""
    check(_lib.load().tgp_autotune_cache_save(os.fsencode(path)), "tgp_autotune_cache_save")


def _node_arg(t, name, B, uniform):
    if t is None:
        return None
    _dev(t, name, torch.float32 if uniform else torch.int32)
    if t.dim() != 1 or t.shape[0] != B or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 1-D tensor of {B} entries")
    return ctypes.c_void_p(t.data_ptr())


def subtree_exchange(old, donor, old_node, new_node=None, old_row=None, new_row=None, max_len=None,
                     old_uniform=False, new_uniform=False, out=None, out_padded=False, status=None, stream=None):
    """Batched subtree exchange (§III-B): output tree b replaces the subtree at node old_node[b] of
    old tree old_row[b] (default b) by the subtree at node new_node[b] (default 0) of donor tree
    new_row[b] (default b). Node tensors are int32 indices, or float32 uniforms in [0, 1) on a side
    whose *_uniform flag is set. out_padded: `out` already holds valid padded trees, so only the
    columns that change are written. Returns (Population [B][old.Lmax], status int32 [B])."""
    lib = _lib.load()
    B = old_node.shape[0] if isinstance(old_node, torch.Tensor) else 0
    if out_padded and out is None:
        raise ValueError("out_padded needs an output population to write into")
    flags = ((_lib.XCHG_OLD_UNIFORM if old_uniform else 0) | (_lib.XCHG_NEW_UNIFORM if new_uniform else 0)
             | (_lib.XCHG_OUT_PADDED if out_padded else 0))
    x = TgpExchange(None, _node_arg(old_node, "old_node", B, old_uniform), None,
                    _node_arg(new_node, "new_node", B, new_uniform), B,
                    old.Lmax if max_len is None else int(max_len), flags)
    for name, r in (("old_row", old_row), ("new_row", new_row)):
        if r is not None:
            _dev(r, name, torch.int32)
            if r.dim() != 1 or r.shape[0] != B or not r.is_contiguous():
                raise ValueError(f"{name} must be a contiguous 1-D int32 tensor of {B} entries")
            setattr(x, name, r.data_ptr())
    dev = old.type.device
    if out is None:
        out = Population(*(torch.empty((B, old.Lmax), dtype=torch.float32, device=dev) for _ in range(3)))
    elif out.P != B or out.Lmax < old.Lmax:
        raise ValueError(f"out must hold {B} rows of at least {old.Lmax} columns")
    if status is None:
        status = torch.empty((B,), dtype=torch.int32, device=dev)
    op, dp, ob = old.abi(), donor.abi(), out.abi()
    check(lib.tgp_subtree_exchange(ctypes.byref(op), ctypes.byref(dp), ctypes.byref(x),
                                   ctypes.c_void_p(out.type.data_ptr()), ctypes.c_void_p(out.value.data_ptr()),
                                   ctypes.c_void_p(out.size.data_ptr()), ob.row_stride,
                                   ctypes.c_void_p(status.data_ptr()), _stream(stream)), "tgp_subtree_exchange")
    return out, status


def crossover(pop, mate, u_old, u_new, max_len=None, out=None, out_padded=False, status=None, stream=None):
    """One-point crossover (§III-B): child b takes tree b of pop and replaces a random node's subtree
    by a random subtree of tree mate[b]; nodes are drawn on the device from the uniforms u_old,
    u_new (float32 [P] in [0, 1))."""
    return subtree_exchange(pop, pop, u_old, u_new, new_row=mate, max_len=max_len, old_uniform=True,
                            new_uniform=True, out=out, out_padded=out_padded, status=status, stream=stream)


def mutation(pop, new_trees, u_old, max_len=None, out=None, out_padded=False, status=None, stream=None):
    """Subtree mutation (§III-B): child b replaces a random node's subtree of tree b of pop by the
    whole of new_trees' tree b; the node is drawn on the device from u_old (float32 [P])."""
    return subtree_exchange(pop, new_trees, u_old, None, max_len=max_len, old_uniform=True, out=out,
                            out_padded=out_padded, status=status, stream=stream)


_METHODS = {"grow": _lib.GEN_GROW, "full": _lib.GEN_FULL, "ramped": _lib.GEN_RAMPED}


def generate(P, Lmax, V, funcs, method="ramped", depth_min=2, depth_max=6, seed=0, const_range=(-5.0, 5.0),
             p_func=None, p_const=None, attempts_per_depth=8, first_tree=0, out=None, attempts=None,
             device="cuda", stream=None):
    """Random trees (grow / full / ramped half-and-half) drawn on the device from Philox4x32-10
    counters. funcs: op ids. p_func / p_const None: the library's defaults. Returns
    (Population [P][Lmax], attempts int32 [P])."""
    lib = _lib.load()
    fl = (ctypes.c_int32 * len(funcs))(*[int(f) for f in funcs])
    g = TgpGenCfg(_METHODS[method], int(depth_min), int(depth_max), int(V), fl, len(funcs),
                  float(const_range[0]), float(const_range[1]), -1.0 if p_func is None else float(p_func),
                  -1.0 if p_const is None else float(p_const), int(attempts_per_depth), int(seed) & (2**64 - 1),
                  int(first_tree))
    if out is None:
        out = Population(*(torch.empty((P, Lmax), dtype=torch.float32, device=device) for _ in range(3)))
    elif out.P != P or out.Lmax < Lmax:
        raise ValueError(f"out must hold {P} rows of at least {Lmax} columns")
    if attempts is None:
        attempts = torch.empty((P,), dtype=torch.int32, device=out.type.device)
    check(lib.tgp_generate(ctypes.byref(g), int(P), int(Lmax), ctypes.c_void_p(out.type.data_ptr()),
                           ctypes.c_void_p(out.value.data_ptr()), ctypes.c_void_p(out.size.data_ptr()),
                           out.abi().row_stride, ctypes.c_void_p(attempts.data_ptr()), _stream(stream)),
          "tgp_generate")
    return out, attempts


class TreeMSE(torch.autograd.Function):
    """Fitness of every tree as a differentiable function of the node values and X.

    ``TreeMSE.apply(value, type, size, X, y)`` returns float32 [P] (y [D], or Y [n_out][D] for
    multi-output trees, whose fitness sums the outputs' mean squared errors). Backward calls
    tgp_eval_mse_grad with the incoming gradient as the per-tree weights and
    returns (grad_value, None, None, grad_X, None). grad_value is zero at
    every non-constant and padding position, so an optimizer step on ``value``
    moves only the constants (a zero gradient gives Adam a zero step, and NaN
    padding stays NaN)."""

    @staticmethod
    def forward(ctx, value, type, size, X, y):
        pop = Population(type, value, size)
        if y.dim() == 2 and y.shape[0] > 1:
            mse, _ = eval_multi_output(pop, X, y)
        else:
            mse = eval_mse(pop, X, y)
        ctx.save_for_backward(value, type, size, X, y)
        return mse

    @staticmethod
    def backward(ctx, grad_mse):
        value, type, size, X, y = ctx.saved_tensors
        pop = Population(type, value, size)
        want_v = ctx.needs_input_grad[0]
        want_x = ctx.needs_input_grad[3]
        _, gv, gx = eval_mse_grad(pop, X, y, grad_mse=grad_mse.contiguous().float(), want_grad_value=want_v,
                                  want_grad_x=want_x)
        return gv, None, None, gx, None


class GraphedCall:
    """A fixed sequence of library calls captured once in a HIP graph and replayed.

    fn() enqueues the calls on the current stream, with every buffer passed in (ws= and out= for
    the evaluation calls, so that a replay touches the same memory). It runs once on a side stream
    first (capture needs warmed-up calls) and is then captured. If the capture fails (a call that
    synchronises, allocates or is otherwise not capturable, or fn raising), the graph is dropped,
    the reason kept in .reason, and every later call runs fn() eagerly instead: the results are
    the same, only the launch overhead differs. .mode says which ("graph" or "eager")."""

    def __init__(self, fn, warmup=1):
        self.fn = fn
        self.graph = None
        self.reason = None
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                fn()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        try:
            with torch.cuda.graph(g):
                fn()
        except Exception as e:  # noqa: BLE001 - any capture failure falls back to eager calls
            self.reason = f"{type(e).__name__}: {e}"
            torch.cuda.synchronize()
            return
        self.graph = g

    @property
    def mode(self):
        return "eager" if self.graph is None else "graph"

    def __call__(self):
        if self.graph is None:
            self.fn()
        else:
            self.graph.replay()
