#!/usr/bin/env python3
"""Throughput of symbolic-regression fitness evaluation on one MI355X.

A step is one pass of the whole evaluation path over the resident workload:
validate + compile every tree (plan kernel), evaluate every tree on every
data point and reduce the squared errors (evaluation kernel), write one
fitness per tree (finalize). The metric is GPops/s = sum of tree lengths x
data points / time (Langdon's measure as used in the paper's §V-C, with one
generation per step). Inputs are seeded synthetic data of the workload's
shape, already in device memory when the timed region starts. The default
workload is the largest: 200,000 trees of lengths 3..1024 (10% with three
Modi outputs) on 4,096 points, one persistent launch.

Prints one JSON line. Extra objects:
  roofline      the evaluation kernel against the vector-ALU issue peak, with
                algorithmic operations from a fixed operator cost table;
  cpu_baseline  the CPU oracle timed on the host (a baseline, not a target);
  forms         the same workload through the plain forward kernel (one tree
                per workgroup, fixed shape) and the batched persistent queue
                replayed as a captured hipGraph, each in GPops/s and as a
                ratio to the plain forward kernel;
  differentiation  the differentiation workload (50,000 trees, 65,536
                points): forward + adjoint (fitness, d/d constants, d/dX)
                against the plain forward kernel, and the adjoint kernel's
                roofline;
  data_parallel the data-parallel workload (1,000 trees, 10^6 points): step
                throughput and the evaluation kernel's HBM bytes per second;
  exchange      the subtree-exchange kernel (§III-B) producing the next
                population by one-point crossover, in children per second,
                against the HBM bandwidth peak;
  generation    random ramped half-and-half trees drawn on the device, in
                trees per second, against the HBM bandwidth peak;
  classification  argmax accuracy of multi-output trees on a Wine-shaped
                data set (§V-D), in GPops/s.
"""

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GPops/s (tree nodes × points / s), fwd MSE and fwd+adjoint vs plain fwd"
# MI355X: 256 CUs x 4 SIMD x 16 lanes, one fp32 lane-op per lane per clock (non-packed), 2.4 GHz
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
OP_NAMES = ("add", "sub", "mul", "div", "sin", "cos", "tanh", "exp", "log", "max", "min", "tan")
# Fixed operator cost table, in vector-ALU issue slots per application and lane: the cost of
# each operator in compiled (not interpreted) gfx950 code, measured once on MI355X with the
# per-operator loop of tgp_op_cost (spread random inputs, so lanes take the library's
# data-dependent branches) and frozen here, so that the algorithmic operation count of a
# workload does not depend on the build being measured. max and min are one instruction each.
OP_COST = (1.0, 1.0, 1.0, 14.1, 16.9, 15.2, 20.3, 11.6, 9.4, 1.0, 1.0, 22.5)
# Cost of an operator's partial derivatives in the adjoint, same units, given the forward values
# (a compiled reverse sweep keeps them): div 1/b (a division) and -a/b^2 (two products) and the
# protection select; sin -> cos; cos -> sin; tanh 1 - t^2 from its value t; exp its own value
# behind the clamp test; log sign(a) / (|a| + eps) (a division, an add, the a = 0 select);
# max / min one compare; tan 1 + t^2 from its value t; add, sub, mul need no arithmetic.
# exp and log in OP_COST are the library's own implementations (ops.h), measured the same way.
PARTIAL_COST = (0.0, 0.0, 0.0, 17.1, 15.2, 16.9, 2.0, 1.0, 16.1, 1.0, 1.0, 2.0)
EVAL_SOURCES = ("eval_impl.h", "interp.h", "ops.h", "tgp_isa.h", "tgp_kernels.h")
ADJ_SOURCES = ("adjoint_impl.h", "interp.h", "ops.h", "tgp_isa.h", "tgp_kernels.h")
XCHG_SOURCES = ("exchange.hip", "tgp_exchange.h")
GEN_SOURCES = ("generate.hip", "tgp_generate.h")
PEAK_HBM_GBS = 8000.0
XCHG_MIN_CHILDREN = 200_000


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batched",
                    choices=["plain", "hybrid", "dataparallel", "batched", "grad", "hybrid-arith", "batched-arith"])
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--save-cfg", default=None, help="write the chosen launch configuration (JSON) here")
    ap.add_argument("--load-cfg", default=None, help="use this launch configuration (JSON file) instead of tuning")
    ap.add_argument("--cfg", default=None, help="use this launch configuration (JSON text) instead of tuning")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the plain-forward / batched-persistent graph / forward+adjoint comparison")
    ap.add_argument("--form-steps", type=int, default=10, help="timed steps of each compared form")
    ap.add_argument("--adj-cfg", default=None,
                    help="launch configuration (JSON text) of the gradient call instead of tuning it")
    ap.add_argument("--no-differentiation", action="store_true",
                    help="skip the forward+adjoint measurement on the differentiation workload")
    ap.add_argument("--no-data-parallel", action="store_true",
                    help="skip the measurement on the data-parallel workload")
    ap.add_argument("--op-cost-live", action="store_true",
                    help="also measure the operator costs on this GPU (reported beside the fixed table)")
    ap.add_argument("--no-exchange", action="store_true", help="skip the subtree-exchange measurement")
    ap.add_argument("--exchange-steps", type=int, default=20)
    ap.add_argument("--no-generation", action="store_true", help="skip the tree-generation measurement")
    ap.add_argument("--no-classification", action="store_true", help="skip the classification measurement")
    ap.add_argument("--pagie-sweep", action="store_true",
                    help="instead of the benchmark: the threshold study of §V-B (Pagie polynomial, populations "
                         "100..10,000, D swept), every schedule timed, printed as one JSON line")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after the timed steps, copy this many MiB device to device once: a kernel of known "
                         "traffic for calibrating memory counters")
    return ap.parse_args()


def eval_source_hash(files=EVAL_SOURCES):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2501_17168_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(workload, src_hash, kernel="eval"):
    """HBM bytes per launch of a kernel from the committed rocprofv3 --pmc summary, if it was
    taken on the kernel's current source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"source hash:\s*([0-9a-f]+)", txt)
    m_bytes = re.search(r"bytes per launch:\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_bytes or m_hash.group(1) != src_hash:
        return None
    return float(m_bytes.group(1))


def op_costs_live():
    """Cost of each operator in vector-ALU issue slots, measured on this GPU (reported only)."""
    from paper_2501_17168_amd import _lib
    return [max(1.0, _lib.op_cost(o)) for o in range(len(OP_NAMES))]


def op_counts(w):
    """Function nodes of the workload's trees, per op id."""
    import numpy as np
    fn = w.type >= 2
    return np.bincount(w.value[fn].astype(np.int64), minlength=len(OP_NAMES))


def fwd_ops_per_point(w):
    """Algorithmic forward operations per data point: every function node at its cost, plus the
    residual and the squared accumulate of every output of every tree. Leaves cost nothing."""
    import numpy as np
    return float(np.dot(op_counts(w), OP_COST)) + 2.0 * w.P * w.n_out


def adj_ops_per_point(w):
    """Algorithmic forward + adjoint operations per data point: the forward operations; every
    function node's partial derivatives; one product per child edge (the child's adjoint) and one
    add per leaf (the gradient accumulation); two products per tree for the output adjoint.
    Recomputation is not counted."""
    import numpy as np
    lengths = w.lengths()
    edges = float(lengths.sum() - w.P)
    leaves = float(np.count_nonzero((w.type == 0) | (w.type == 1)))
    return fwd_ops_per_point(w) + float(np.dot(op_counts(w), PARTIAL_COST)) + edges + leaves + 2.0 * w.P


def alu_roofline(ops_per_launch, kernel_ms, node_evals, kernel, src_hash, traffic):
    achieved = ops_per_launch / (kernel_ms * 1e-3)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12, "unit": "Top/s",
            "frac": achieved / PEAK_LANE_OPS, "traffic": traffic, "kernel": kernel, "kernel_ms": kernel_ms,
            "algo_ops_per_launch": ops_per_launch,
            "node_evals_per_s": node_evals / (kernel_ms * 1e-3),
            "node_evals_frac": node_evals / (kernel_ms * 1e-3) / PEAK_LANE_OPS,
            "op_cost": dict(zip(OP_NAMES, OP_COST)), "source_hash": src_hash}


def timed_ms(torch, fn, steps, warmup=2):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def exchange_bench(tgp, torch, w, workload, steps, warmup=3):
    """One-point crossover (§III-B) producing the next population: parents are the workload's
    trees repeated to at least XCHG_MIN_CHILDREN rows, child b = parent b with a random node's
    subtree replaced by a random subtree of a random mate; nodes drawn on the device from
    seeded uniforms. Two output modes: a fresh buffer (every column written) and a buffer that
    already holds padded trees (only the changed columns written), the steady state when two
    population buffers take turns. Timed with HIP events on the launch stream (the exchange
    kernel is the only launch inside each timed region)."""
    import numpy as np
    reps = -(-XCHG_MIN_CHILDREN // w.P)
    dev = torch.device("cuda:0")
    par = tgp.Population(*(torch.from_numpy(a).to(dev).repeat(reps, 1).contiguous()
                           for a in (w.type, w.value, w.size)))
    B, L = par.P, par.Lmax
    rng = np.random.default_rng(2025)
    mate = torch.from_numpy(rng.integers(0, B, B).astype(np.int32)).to(dev)
    u = torch.from_numpy(rng.random(B).astype(np.float32)).to(dev)
    v = torch.from_numpy(rng.random(B).astype(np.float32)).to(dev)
    out = tgp.Population(*(torch.empty((B, L), dtype=torch.float32, device=dev) for _ in range(3)))
    status = torch.empty(B, dtype=torch.int32, device=dev)
    full_ms = timed_ms(torch, lambda: tgp.crossover(par, mate, u, v, out=out, status=status), steps, warmup)
    st = status.cpu().numpy()
    child_len = out.size[:, 0].cpu().numpy().astype(np.int64)
    # the same call into rows that hold the children already (steady state of two buffers)
    pad_ms = timed_ms(torch, lambda: tgp.crossover(par, mate, u, v, out=out, out_padded=True, status=status),
                      steps, warmup)
    read = 12.0 * float(child_len.sum()) + 16.0 * B     # each child's nodes, mate row, two uniforms, status
    full_bytes = 12.0 * B * L + read                      # every output column written
    pad_bytes = 12.0 * float(child_len.sum()) + 4.0 * B + read   # the child's columns, plus its current length
    src_hash = eval_source_hash(XCHG_SOURCES)

    def roof(nbytes, ms, mode):
        gbs = nbytes / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                "traffic": stored_traffic(f"{workload}_{mode}", src_hash, kernel="exchange"),
                "kernel": "exchange_kernel", "kernel_ms": ms, "algo_bytes_per_launch": nbytes,
                "exchange_source_hash": src_hash}

    return {"workload": f"one-point crossover, {B:,} children from the {workload} trees repeated {reps}x "
                        f"(Lmax {L}), nodes from seeded uniforms",
            "value": B / (pad_ms * 1e-3), "unit": "trees/s", "mode": "padded output rows (two buffers in turn)",
            "children": B, "exchanged": float(np.mean(st == 0)), "mean_child_len": float(child_len.mean()),
            "padded": {"ms": pad_ms, "trees/s": B / (pad_ms * 1e-3), "roofline": roof(pad_bytes, pad_ms, "padded")},
            "full_write": {"ms": full_ms, "trees/s": B / (full_ms * 1e-3),
                           "roofline": roof(full_bytes, full_ms, "full")}}

def device_workload(tgp, torch, w):
    """The workload's population, X and Y in device memory. Targets of hidden trees are the
    library's own predictions of those trees plus the workload's noise."""
    import numpy as np
    dev = torch.device("cuda:0")
    pop = tgp.Population(*(torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (w.type, w.value, w.size)))
    X = torch.from_numpy(w.X).to(dev)
    if w.Y is not None:
        Y = torch.from_numpy(w.Y).to(dev)
    else:
        hidden = tgp.Population(*(torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in w.hidden))
        # each hidden tree is a plain (single-output) tree: its root value is target row o
        _, hp = tgp.eval_multi_output(hidden, X, None, n_out=1, want_pred=True)
        Y = (hp[:, 0, :] + torch.from_numpy(w.noise).to(dev)).contiguous()
    torch.cuda.synchronize()
    return pop, X, Y


def profiled_ms(torch, fn, steps, warmup=2):
    """Mean step time (HIP events on the current stream) and mean evaluation- or adjoint-kernel
    time per launch (HIP events the library records around that launch, on the same stream)."""
    from paper_2501_17168_amd import _lib
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    _lib.profile(True)
    _lib.profile_read()
    ms = timed_ms(torch, fn, steps, warmup=0)
    k_total, launches = _lib.profile_read()
    _lib.profile(False)
    return ms, k_total / max(launches, 1)


def compare_forms(tgp, torch, pop, X, Y, w, gpops_per_step, steps, tuned=None):
    """Plain forward vs batched persistent (hipGraph replay) on one workload."""
    res = {}
    plain = tgp.cfg(mode=1, points_per_lane=4, block_waves=4)
    ws = tgp.Workspace(X.device)
    out = torch.empty(w.P, dtype=torch.float32, device=X.device)

    def fwd(c):
        if w.n_out == 1:
            tgp.eval_mse(pop, X, Y, config=c, ws=ws, out=out)
        else:
            tgp.eval_multi_output(pop, X, Y, config=c, ws=ws, out=out)

    ms_plain = timed_ms(torch, lambda: fwd(plain), steps)
    res["plain_fwd"] = {"cfg": "tree-major, 4 points/lane, 4 waves/workgroup", "ms": ms_plain,
                        "GPops/s": gpops_per_step / (ms_plain * 1e-3)}

    if not tuned:
        tuned = tgp.autotune(pop, X, Y, n_out=w.n_out)
    pers_d = {"mode": 3, "points_per_lane": tuned.get("points_per_lane", 4),
              "trees_per_unit": tuned.get("trees_per_unit", 4) if tuned.get("mode") == 3 else 4,
              "block_waves": tuned.get("block_waves", 4), "flags": 0}
    pers = tgp.cfg(pers_d)
    fwd(pers)
    g = tgp.GraphedCall(lambda: fwd(pers))
    ms_graph = timed_ms(torch, g, steps)
    res["batched_persistent_graph"] = {"cfg": pers_d, "ms": ms_graph, "GPops/s": gpops_per_step / (ms_graph * 1e-3),
                                       "vs_plain_fwd": ms_plain / ms_graph, "launch": g.mode}
    del g

    if w.n_out == 1:
        adj_cfg = tgp.autotune(pop, X, Y, want_grad=True, ws=ws)
        ms_adj = timed_ms(torch, lambda: tgp.eval_mse_grad(pop, X, Y, ws=ws), steps)
        res["fwd_adjoint"] = {"outputs": "fitness, d/d constants, d/dX", "cfg": adj_cfg, "ms": ms_adj,
                              "GPops/s": gpops_per_step / (ms_adj * 1e-3), "vs_plain_fwd": ms_plain / ms_adj}
    return res


def differentiation_bench(tgp, torch, steps, adj_cfg=None):
    """Forward + adjoint on the differentiation workload (50,000 trees, <= 32 constants each,
    8 variables, 65,536 points): fitness, d(sum of fitness)/d constants and d/dX in one call at
    the gradient autotuner's launch shape, against the plain forward kernel (tree-major, 4 points
    per lane, 4 waves per workgroup) and the autotuned forward on the same trees. The adjoint
    kernel's roofline counts forward operations, partial derivatives and the sweep's products
    and accumulations per point (no recomputation)."""
    import synth
    w = synth.workload("grad")
    pop, X, Y = device_workload(tgp, torch, w)
    ws = tgp.Workspace(X.device)
    node_evals = float(w.lengths().sum()) * w.D
    plain = tgp.cfg(mode=1, points_per_lane=4, block_waves=4)
    ms_plain = timed_ms(torch, lambda: tgp.eval_mse(pop, X, Y, config=plain, ws=ws), steps)
    fwd_cfg = tgp.autotune(pop, X, Y, ws=ws)
    ms_fwd, fwd_kernel_ms = profiled_ms(torch, lambda: tgp.eval_mse(pop, X, Y, ws=ws), steps)
    if adj_cfg is None:
        adj_cfg = tgp.autotune(pop, X, Y, want_grad=True, ws=ws)
    ac = tgp.cfg(adj_cfg)
    ms_adj, adj_kernel_ms = profiled_ms(torch, lambda: tgp.eval_mse_grad(pop, X, Y, config=ac, ws=ws), steps)
    roof = alu_roofline(adj_ops_per_point(w) * w.D, adj_kernel_ms, node_evals, "adjoint_kernel",
                        eval_source_hash(ADJ_SOURCES), stored_traffic("grad", eval_source_hash(ADJ_SOURCES),
                                                                      kernel="adjoint"))
    roof["partial_cost"] = dict(zip(OP_NAMES, PARTIAL_COST))
    return {"workload": f"grad: {w.desc}", "P": w.P, "D": w.D, "sum_len": int(w.lengths().sum()),
            "plain_fwd": {"cfg": "tree-major, 4 points/lane, 4 waves/workgroup", "ms": ms_plain,
                          "GPops/s": node_evals / (ms_plain * 1e-3)},
            "tuned_fwd": {"cfg": fwd_cfg, "ms": ms_fwd, "GPops/s": node_evals / (ms_fwd * 1e-3),
                          "eval_kernel_ms": fwd_kernel_ms},
            "fwd_adjoint": {"outputs": "fitness, d/d constants, d/dX", "cfg": adj_cfg, "ms": ms_adj,
                            "GPops/s": node_evals / (ms_adj * 1e-3), "vs_plain_fwd": ms_plain / ms_adj,
                            "vs_tuned_fwd": ms_fwd / ms_adj, "adjoint_kernel_ms": adj_kernel_ms},
            "roofline": roof}


def data_parallel_bench(tgp, torch, steps):
    """The data-parallel workload (1,000 trees, 5 variables, 10^6 points): autotuned step
    throughput, the evaluation kernel against the vector-ALU peak, and its HBM bytes per second:
    algorithmic (X and Y read once, the encoding, one fitness per tree) and, when the committed
    counter summary matches the kernel source, measured."""
    import synth
    w = synth.workload("dataparallel")
    pop, X, Y = device_workload(tgp, torch, w)
    ws = tgp.Workspace(X.device)
    sum_len = int(w.lengths().sum())
    node_evals = float(sum_len) * w.D
    cfg = tgp.autotune(pop, X, Y, ws=ws)
    ms, kernel_ms = profiled_ms(torch, lambda: tgp.eval_mse(pop, X, Y, ws=ws), steps)
    src = eval_source_hash()
    traffic = stored_traffic("dataparallel", src)
    algo_bytes = 4.0 * w.D * (w.V + w.n_out) + 12.0 * sum_len + 4.0 * w.P
    hbm = {"bound": "hbm", "achieved": algo_bytes / (kernel_ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": algo_bytes / (kernel_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, "traffic": traffic,
           "traffic_GBs": None if traffic is None else traffic / (kernel_ms * 1e-3) / 1e9,
           "algo_bytes_per_launch": algo_bytes, "kernel": "eval_kernel", "kernel_ms": kernel_ms}
    return {"workload": f"dataparallel: {w.desc}", "P": w.P, "D": w.D, "sum_len": sum_len, "schedule": cfg,
            "ms": ms, "GPops/s": node_evals / (ms * 1e-3),
            "roofline": alu_roofline(fwd_ops_per_point(w) * w.D, kernel_ms, node_evals, "eval_kernel", src, traffic),
            "hbm": hbm}


_CPU = {}  # workload and targets for the oracle pool (inherited by forked workers)


def _oracle_chunk(rows):
    import oracle as O
    w, Y = _CPU["w"], _CPU["Y"]
    O.mse(w.type, w.value, w.size, w.X, Y, w.n_out, rows=list(rows))
    return len(rows)


def cpu_baseline(w, seconds, max_workers=16):
    """The CPU oracle (float64 numpy, unchanged) on a bounded sample of the workload: first one
    core, then a pool of worker processes over the host cores. Runs before the GPU is touched, so
    the pool can fork."""
    import multiprocessing as mp
    import numpy as np
    import oracle as O

    Y = w.Y if w.Y is not None else w.targets_from(O.predict(*w.hidden, w.X, 1)[:, 0, :])
    _CPU["w"], _CPU["Y"] = w, Y
    lengths = w.lengths()
    order = np.random.default_rng(0).permutation(w.P)
    # one core, about a fifth of the budget
    t0 = time.perf_counter()
    k1 = len1 = 0
    while k1 < w.P and time.perf_counter() - t0 < seconds / 5:
        _oracle_chunk([int(order[k1])])
        len1 += int(lengths[order[k1]])
        k1 += 1
    el1 = time.perf_counter() - t0
    rate1 = len1 * w.D / el1
    # all cores: the random order from its start, up to about `seconds` of one-core work (the
    # whole workload when it is smaller)
    workers = max(1, min(max_workers, len(os.sched_getaffinity(0))))
    budget = seconds * rate1 / w.D            # lengths' worth of trees one core does in `seconds`
    cum = np.cumsum(lengths[order])
    n = min(w.P, int(np.searchsorted(cum, budget)) + 1)
    sample = order[:n]
    res = {"value": rate1, "unit": "GPops/s", "cores": 1, "kind": "oracle",
           "sample": f"{k1} of {w.P} trees (random order) x all {w.D} points, float64 numpy, {el1:.1f} s on one core"}
    if workers > 1 and len(sample) >= workers:
        chunks = [sample[i::workers * 4] for i in range(workers * 4)]
        ctx = mp.get_context("fork")
        with ctx.Pool(workers) as pool:
            pool.map(_oracle_chunk, [[int(order[0])]] * workers)   # start every worker
            t0 = time.perf_counter()
            pool.map(_oracle_chunk, [[int(x) for x in c] for c in chunks], chunksize=1)
            elN = time.perf_counter() - t0
        lenN = int(lengths[sample].sum())
        res = {"value": lenN * w.D / elN, "unit": "GPops/s", "cores": workers, "kind": "oracle",
               "sample": f"{len(sample)} of {w.P} trees (random order) x all {w.D} points, float64 numpy, "
                         f"{elN:.1f} s wall on {workers} worker processes",
               "single_core": {"value": rate1, "sample": res["sample"]}}
    return res


def generation_bench(tgp, torch, steps=20, warmup=3):
    """Ramped half-and-half initialisation on the device: 200,000 trees, depth 2..8, the 11-op set,
    2 variables, Lmax 256 (the hybrid workload's shape), Philox4x32-10 draws. Timed with HIP
    events on the launch stream."""
    import numpy as np
    P, L, V = XCHG_MIN_CHILDREN, 256, 2
    funcs = list(range(11))
    dev = torch.device("cuda:0")
    out = tgp.Population(*(torch.empty((P, L), dtype=torch.float32, device=dev) for _ in range(3)))
    att = torch.empty(P, dtype=torch.int32, device=dev)
    kw = dict(method="ramped", depth_min=2, depth_max=8, seed=7, out=out, attempts=att)
    ms = timed_ms(torch, lambda: tgp.generate(P, L, V, funcs, **kw), steps, warmup)
    lens = out.size[:, 0].cpu().numpy().astype(np.int64)
    algo_bytes = 12.0 * P * L + 4.0 * P       # every column of every row, and the attempt counts
    gbs = algo_bytes / (ms * 1e-3) / 1e9
    return {"workload": f"ramped half-and-half, {P:,} trees, depth 2..8, 11 ops, {V} variables, Lmax {L}",
            "value": P / (ms * 1e-3), "unit": "trees/s", "ms": ms, "mean_len": float(lens.mean()),
            "nodes/s": float(lens.sum()) / (ms * 1e-3), "mean_attempts": float(att.float().mean().item()),
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": gbs / PEAK_HBM_GBS,
                         "traffic": stored_traffic("hybrid", eval_source_hash(GEN_SOURCES), kernel="generate"),
                         "kernel": "generate_kernel", "kernel_ms": ms, "algo_bytes_per_launch": algo_bytes,
                         "generate_source_hash": eval_source_hash(GEN_SOURCES)}}


def classification_bench(tgp, torch, steps=20, warmup=3):
    """Classification fitness (§V-D) on two shapes: Wine (5,000 multi-output trees, 13 features,
    3 classes, 178 points) and Yeast (5,000 trees, 8 features, 10 classes, 1,484 points: the wide
    output accumulators). Autotuned launch, timed with HIP events per call."""
    import numpy as np
    import synth
    dev = torch.device("cuda:0")
    res = {}
    for name in ("classify", "yeast"):
        w = synth.workload(name)
        pop = tgp.Population(*(torch.from_numpy(a).to(dev) for a in (w.type, w.value, w.size)))
        X = torch.from_numpy(w.X).to(dev)
        lab = torch.from_numpy(np.ascontiguousarray(w.Y[0])).to(dev)
        cfg = tgp.autotune(pop, X, torch.zeros((w.n_out, w.D), device=dev), n_out=w.n_out)
        c = tgp.cfg(cfg)
        out = torch.empty(w.P, device=dev)
        ms = timed_ms(torch, lambda: tgp.eval_accuracy(pop, X, lab, w.n_out, config=c, out=out), steps, warmup)
        gpops = float(w.lengths().sum()) * w.D
        acc = out.cpu().numpy()
        res["wine" if name == "classify" else "yeast"] = {
            "workload": f"{name}: {w.desc}", "value": gpops / (ms * 1e-3), "unit": "GPops/s", "ms": ms,
            "schedule": cfg, "mean_accuracy": float(np.nanmean(acc)), "best_accuracy": float(np.nanmax(acc))}
    out = dict(res["wine"])
    out["yeast"] = res["yeast"]
    return out


SWEEP_P = (100, 1_000, 5_000, 10_000)
SWEEP_D = (256, 1_024, 4_096, 8_192, 16_384, 32_768, 65_536, 262_144)
LANES = 256 * 64  # MI355X: 256 CUs x 64 lanes, the counterpart of the paper's CUDA-core count


def _mode_grid(mode, V):
    """Launch configurations tried per schedule in the threshold study."""
    ks = [4, 8] + ([16] if V <= 2 else [])
    if mode == 1:
        return [dict(mode=1, points_per_lane=k, block_waves=b) for k in ks for b in (1, 2, 4)]
    if mode == 2:
        return [dict(mode=2, points_per_lane=k, block_waves=b, trees_per_unit=t)
                for k in ks for b in (1, 4) for t in (1, 4, 16, 64)]
    return [dict(mode=3, points_per_lane=k, block_waves=b, trees_per_unit=t, flags=f)
            for k in ks for b in (1, 4) for t in (1, 2, 4) for f in (0, 2)]


def pagie_sweep(steps=5):
    """The threshold study of §V-B on this GPU: Pagie-polynomial populations of 100..10,000 trees,
    D swept from 256 to 262,144. At each point every schedule is timed at its best launch
    configuration from a small grid (HIP events): tree-major and persistent (the work unit is
    a tree: parallelism from the population) and point-major (the work unit is a point tile
    swept across a run of trees: parallelism from the data). The autotuner's choice is timed
    too, and set beside the paper's rule, which moves to data parallelism once D reaches the
    core count (here the lane count, 16,384)."""
    import numpy as np
    import torch

    import synth
    import paper_2501_17168_amd as tgp

    dev = torch.device("cuda:0")
    names = {1: "tree-major", 2: "point-major", 3: "persistent"}
    rows = []
    for P in SWEEP_P:
        w = synth.workload("pagie", P=P, D=max(SWEEP_D))
        pop = tgp.Population(*(torch.from_numpy(a).to(dev) for a in (w.type, w.value, w.size)))
        sum_len = int(w.lengths().sum())
        for D in SWEEP_D:
            X = torch.from_numpy(np.ascontiguousarray(w.X[:, :D])).to(dev)
            Y = torch.from_numpy(np.ascontiguousarray(w.Y[:, :D])).to(dev)
            ms, best_cfg = {}, {}
            for mode, name in names.items():
                for cand in _mode_grid(mode, w.V):
                    c = tgp.cfg(cand)
                    t = timed_ms(torch, lambda: tgp.eval_mse(pop, X, Y, config=c), steps, warmup=1)
                    if name not in ms or t < ms[name]:
                        ms[name], best_cfg[name] = t, cand
            tuned = tgp.autotune(pop, X, Y)
            ct = tgp.cfg(tuned)
            ms["autotuned"] = timed_ms(torch, lambda: tgp.eval_mse(pop, X, Y, config=ct), steps)
            # the same call replayed from a hipGraph: device time without the host's per-call cost
            ws, out = tgp.Workspace(dev), torch.empty(P, device=dev)
            graph = tgp.GraphedCall(lambda: tgp.eval_mse(pop, X, Y, config=ct, ws=ws, out=out))
            ms["autotuned_graph"] = timed_ms(torch, graph, steps)
            del graph
            best = min(names.values(), key=ms.get)
            pop_best = min(ms["tree-major"], ms["persistent"])
            row = {"P": P, "D": D, "ms": {k: round(v, 5) for k, v in ms.items()},
                   "GPops/s": {k: sum_len * D / (v * 1e-3) for k, v in ms.items()},
                   "best": best, "data_over_population": pop_best / ms["point-major"],
                   "rule": "point-major" if D >= LANES else "population", "tuned": tuned,
                   "best_cfg": best_cfg}
            rows.append(row)
            print(f"P={P:6d} D={D:7d} " + " ".join(f"{k}={v * 1e3:8.1f}us" for k, v in ms.items())
                  + f" best={best} tuned-mode={tuned['mode']}", file=sys.stderr, flush=True)
    # crossovers per population: the first D from which the data-parallel schedule stays ahead
    # of the tree-per-workgroup one (the paper's comparison), and of every population schedule
    def first_ahead(P, key):
        rs = [r for r in rows if r["P"] == P]
        ahead = [key(r) > 1.0 for r in rs]
        return next((rs[i]["D"] for i in range(len(rs)) if all(ahead[i:])), None)

    cross_tree = {P: first_ahead(P, lambda r: r["ms"]["tree-major"] / r["ms"]["point-major"]) for P in SWEEP_P}
    cross_all = {P: first_ahead(P, lambda r: r["data_over_population"]) for P in SWEEP_P}
    print(json.dumps({"sweep": "pagie threshold (§V-B)", "lanes": LANES, "P": SWEEP_P, "D": SWEEP_D,
                      "crossover_D_vs_tree_major": cross_tree, "crossover_D_vs_all_population": cross_all,
                      "rows": rows}), flush=True)
    return 0

def main():
    args = parse()
    if args.pagie_sweep:
        return pagie_sweep()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    import paper_2501_17168_amd as tgp
    from paper_2501_17168_amd import _lib

    w = synth.workload(args.workload)
    cpu = None if args.no_cpu_baseline else cpu_baseline(w, args.cpu_seconds)
    dev = torch.device("cuda:0")
    pop, X, Y = device_workload(tgp, torch, w)

    lengths = w.lengths()
    sum_len = int(lengths.sum())
    gpops_per_step = float(sum_len) * w.D

    cfg = None
    if args.cfg:
        cfg = json.loads(args.cfg)
    elif args.load_cfg:
        with open(args.load_cfg) as f:
            cfg = json.load(f)
    elif not args.no_autotune:
        cfg = tgp.autotune(pop, X, Y, n_out=w.n_out)
    if args.save_cfg and cfg:
        with open(args.save_cfg, "w") as f:
            json.dump(cfg, f)
    step_cfg = tgp.cfg(cfg) if cfg else None
    step_ws = tgp.Workspace(dev)
    step_out = torch.empty(w.P, dtype=torch.float32, device=dev)

    def step():
        if w.n_out == 1:
            tgp.eval_mse(pop, X, Y, config=step_cfg, ws=step_ws, out=step_out)
        else:
            tgp.eval_multi_output(pop, X, Y, config=step_cfg, ws=step_ws, out=step_out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the timed steps, without the library's kernel events
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = e0.elapsed_time(e1)
    # the same steps again with an event pair around each evaluation launch: its kernel time
    _lib.profile(True)
    _lib.profile_read()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    eval_ms_total, launches = _lib.profile_read()
    _lib.profile(False)
    ms_step = ms / args.steps
    value = gpops_per_step * args.steps / (ms * 1e-3)
    print(f"{args.workload}: {ms_step:.3f} ms per step, {value:.3e} GPops/s", file=sys.stderr, flush=True)

    if args.copy_mb > 0:
        src = torch.empty(args.copy_mb << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- roofline of the evaluation kernel (fixed operator cost table) ----
    eval_ms = eval_ms_total / max(launches, 1)
    src_hash = eval_source_hash()
    roofline = alu_roofline(fwd_ops_per_point(w) * w.D, eval_ms, gpops_per_step, "eval_kernel", src_hash,
                            stored_traffic(args.workload, src_hash))
    if args.op_cost_live:
        roofline["op_cost_live"] = dict(zip(OP_NAMES, (round(c, 2) for c in op_costs_live())))

    forms = None if args.no_forms else compare_forms(tgp, torch, pop, X, Y, w, gpops_per_step, args.form_steps, cfg)
    if forms:
        print(f"forms: {json.dumps(forms)}", file=sys.stderr, flush=True)
    diff = None if args.no_differentiation else differentiation_bench(
        tgp, torch, args.form_steps, json.loads(args.adj_cfg) if args.adj_cfg else None)
    if diff:
        print(f"differentiation: {json.dumps(diff)}", file=sys.stderr, flush=True)
    dpar = None if args.no_data_parallel else data_parallel_bench(tgp, torch, args.form_steps)
    if dpar:
        print(f"data_parallel: {json.dumps(dpar)}", file=sys.stderr, flush=True)
    exchange = None if args.no_exchange else exchange_bench(tgp, torch, w, args.workload, args.exchange_steps)
    generation = None if args.no_generation else generation_bench(tgp, torch)
    classification = None if args.no_classification else classification_bench(tgp, torch)

    out = {"metric": METRIC, "value": value, "unit": "GPops/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{args.workload}: {w.desc}", "P": w.P, "Lmax": w.Lmax, "V": w.V, "D": w.D,
                      "n_out": w.n_out, "sum_len": sum_len, "schedule": cfg, "wall_s": t_wall},
           "roofline": roofline, "cpu_baseline": cpu, "forms": forms, "differentiation": diff,
           "data_parallel": dpar, "exchange": exchange, "generation": generation,
           "classification": classification}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
