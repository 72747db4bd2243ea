"""Parity at the full workload sizes, in the launch configuration the
benchmark uses (the autotuner's choice), checked on each workload's oracle
sample of trees (the sample includes the longest trees and every Modi kind).
The oracle's references for the samples are read from
tests/golden/fullsize_refs.npz (written by tests/golden/make_fullsize_refs.py
from oracle/ and synth/ only) when its input hashes match the workload, and
are computed here otherwise. Needs an MI355X."""

import numpy as np
import pytest
import torch

import oracle as O
import paper_2501_17168_amd as tgp
import synth
from golden_refs import fullsize_fitness_ref, fullsize_grad_ref
from parity import FitnessRef, GradRef, compare_fitness, compare_grad_value, compare_grad_x, inside

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

_cache = {}


def full(name):
    if name not in _cache:
        w = synth.workload(name)
        Y = w.Y if w.Y is not None else w.targets_from(O.predict(*w.hidden, w.X, 1)[:, 0, :])
        Y = np.ascontiguousarray(np.asarray(Y, np.float32).reshape(w.n_out, w.D))
        pop = tgp.Population(*(torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (w.type, w.value, w.size)))
        _cache[name] = (w, Y, pop, torch.from_numpy(w.X).to(DEV), torch.from_numpy(Y).to(DEV))
    return _cache[name]


def fitness(pop, X, Yd, n_out, cfg, ws=None, out=None):
    if n_out == 1:
        return tgp.eval_mse(pop, X, Yd, config=cfg, ws=ws, out=out)
    m, _ = tgp.eval_multi_output(pop, X, Yd, config=cfg, ws=ws, out=out)
    return m


@pytest.mark.parametrize("name", ["plain", "hybrid", "dataparallel", "batched", "grad"])
def test_fullsize_sampled_parity(name):
    w, Y, pop, X, Yd = full(name)
    rows = w.sample
    print(f"[{name}] P={w.P} D={w.D} sample={len(rows)}", flush=True)
    cfg = tgp.autotune(pop, X, Yd, n_out=w.n_out)
    print(f"[{name}] autotuned {cfg}", flush=True)
    m = fitness(pop, X, Yd, w.n_out, tgp.cfg(cfg)).cpu().numpy()
    info, st = tgp.plan(pop, w.V, w.n_out)
    info = info.cpu().numpy()
    ref = O.plan(w.type[rows], w.value[rows], w.size[rows], w.V, w.n_out)
    np.testing.assert_array_equal(info[rows], ref)
    # every tree: NaN fitness exactly for the invalid ones
    np.testing.assert_array_equal(np.isnan(m) & (info[:, 0] != 0), info[:, 0] != 0)
    rep = compare_fitness(m[rows], fullsize_fitness_ref(name, w, Y), label=f"{name} full size")
    print(f"[{name}] {rep}", flush=True)


def test_fullsize_batched_persistent_graph():
    """The batched workload as one persistent, length-bucketed launch replayed from a hipGraph."""
    w, Y, pop, X, Yd = full("batched")
    tuned = tgp.autotune(pop, X, Yd, n_out=w.n_out)
    cfg = tgp.cfg(mode=3, points_per_lane=tuned["points_per_lane"], block_waves=tuned["block_waves"],
                  trees_per_unit=tuned["trees_per_unit"] if tuned["mode"] == 3 else 4)
    ws = tgp.Workspace(DEV)
    out = torch.empty(w.P, device=DEV)
    eager = fitness(pop, X, Yd, w.n_out, cfg, ws=ws, out=out).cpu().numpy()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fitness(pop, X, Yd, w.n_out, cfg, ws=ws, out=out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fitness(pop, X, Yd, w.n_out, cfg, ws=ws, out=out)
    for _ in range(3):
        out.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        np.testing.assert_allclose(got, eager, rtol=1e-6, atol=0, equal_nan=True)
    compare_fitness(got[w.sample], fullsize_fitness_ref("batched", w, Y), label="batched persistent graph")


def test_fullsize_gradients():
    """Fitness gradients at the full differentiation workload in the tuned gradient launch.
    Constant gradients: the full population's call (each tree's gradient is its own), on the
    sample rows. X gradients: the same launch on a population of the sample trees only (the X
    gradient sums over the trees of a call), at the reference's sampled points."""
    w, Y, pop, X, Yd = full("grad")
    rows = np.asarray(w.sample)
    tuned = tgp.autotune(pop, X, Yd, want_grad=True)
    print(f"[grad] tuned gradient launch {tuned}", flush=True)
    mse, gv, _ = tgp.eval_mse_grad(pop, X, Yd, want_grad_x=False)
    torch.cuda.synchronize()
    compare_fitness(mse.cpu().numpy()[rows], fullsize_fitness_ref("grad", w, Y), label="grad workload fitness")
    ref, pts = fullsize_grad_ref(w, Y)
    rep_v = compare_grad_value(gv.cpu().numpy()[rows], ref, label="grad full size")
    sub = tgp.Population(*(torch.from_numpy(np.ascontiguousarray(a[rows])).to(DEV) for a in (w.type, w.value, w.size)))
    _, _, gx = tgp.eval_mse_grad(sub, X, Yd, config=tgp.cfg(tuned), want_grad_value=False)
    torch.cuda.synchronize()
    rep_x = compare_grad_x(gx.cpu().numpy()[:, pts], ref, label="grad full size")
    print(f"[grad] grad_value {rep_v}\n[grad] grad_X {rep_x}", flush=True)


def test_fullsize_adam_steps_with_gradient_checks():
    """10 Adam steps (lr 1e-2) on the constants of the full differentiation workload through
    TreeMSE. Before every step, the device's fitness and constant gradients of 10 sample trees
    (a different ten each step, all 100 over the run) are checked against the oracle's float64
    values and envelopes at the device's current constants."""
    w, Y, pop, X, Yd = full("grad")
    rows_all = np.asarray(w.sample)
    value = pop.value.clone().requires_grad_(True)
    opt = torch.optim.Adam([value], lr=1e-2)
    m0 = None
    for step in range(10):
        opt.zero_grad()
        mse = tgp.TreeMSE.apply(value, pop.type, pop.size, X, Yd)
        mse.sum().backward()
        torch.cuda.synchronize()
        if m0 is None:
            m0 = mse.detach().cpu().numpy()
        rows = list(rows_all[step::10])
        cur = value.detach()[rows].cpu().numpy()
        t, s = w.type[rows], w.size[rows]
        ref = GradRef(t, cur, s, w.X, Y)
        compare_fitness(mse.detach().cpu().numpy()[rows], FitnessRef(t, cur, s, w.X, Y), label=f"step {step} fitness")
        rep = compare_grad_value(value.grad[rows].cpu().numpy(), ref, label=f"step {step}")
        print(f"[adam] step {step}: {len(rows)} trees, grad_value {rep}", flush=True)
        opt.step()
    vv = value.detach().cpu().numpy()
    fixed = w.type != 1
    np.testing.assert_array_equal(np.isnan(vv), np.isnan(w.value))
    keep = fixed & ~np.isnan(w.value)
    assert np.array_equal(vv[keep], w.value[keep])
    m1 = tgp.TreeMSE.apply(value.detach(), pop.type, pop.size, X, Yd).cpu().numpy()
    fin = np.isfinite(m0) & np.isfinite(m1) & ((w.type == 1).sum(1) > 0)
    frac = float((m1[fin] <= m0[fin] * (1 + 1e-6)).mean())
    print(f"[adam] fitness not worse after 10 steps on {frac:.3f} of {int(fin.sum())} trees with constants")
    assert frac > 0.8
