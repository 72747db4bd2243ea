"""Parity at the full workload sizes, in the launch configuration the
benchmark uses (the autotuner's choice), checked on each workload's oracle
sample of trees. The sample includes the longest trees and every Modi kind.
Needs an MI355X."""

import numpy as np
import pytest
import torch

import oracle as O
import paper_2501_17168_amd as tgp
import synth
from parity import shadows, classify, compare_fitness, grad_close, grad_shadows, well_grad

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


_cache = {}


def full(name):
    if name not in _cache:
        _cache[name] = _full(name)
    return _cache[name]


def _full(name):
    w = synth.workload(name)
    Y = w.Y if w.Y is not None else w.targets_from(O.predict(*w.hidden, w.X, 1)[:, 0, :])
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    pop = tgp.Population(*(torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (w.type, w.value, w.size)))
    return w, Y, pop, torch.from_numpy(w.X).to(DEV), torch.from_numpy(Y).to(DEV)


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
    m64, m32 = (O.mse(w.type, w.value, w.size, w.X, Y, w.n_out, rows=rows),
                shadows(w.type, w.value, w.size, w.X, Y, w.n_out, rows=rows))
    rep = compare_fitness(m[rows], m64, m32, label=f"{name} full size")
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
    rows = w.sample
    m64 = O.mse(w.type, w.value, w.size, w.X, Y, w.n_out, rows=rows)
    m32 = shadows(w.type, w.value, w.size, w.X, Y, w.n_out, rows=rows)
    compare_fitness(got[rows], m64, m32, label="batched persistent graph")


def test_fullsize_gradients():
    """Fitness gradients at the full differentiation workload, on its sample of trees."""
    w, Y, pop, X, Yd = full("grad")
    rows = w.sample
    m64 = O.mse(w.type, w.value, w.size, w.X, Y, rows=rows)
    m32 = shadows(w.type, w.value, w.size, w.X, Y, rows=rows)
    well, _ = classify(m64, m32)
    wr = rows[well]
    gw = np.zeros(w.P, np.float32)
    gw[wr] = 1.0
    mse, gv, gx = tgp.eval_mse_grad(pop, X, Yd, grad_mse=torch.from_numpy(gw).to(DEV))
    torch.cuda.synchronize()
    compare_fitness(mse.cpu().numpy()[rows], m64, m32, label="grad workload fitness")
    _, gv64, gx64 = O.grad(w.type, w.value, w.size, w.X, Y, rows=wr)
    const = w.type[wr] == 1
    wv, wellx = well_grad(grad_shadows(w.type, w.value, w.size, w.X, Y, rows=wr), gv64, gx64)
    wellg = wv & const
    ok = grad_close(gv.cpu().numpy()[wr], gv64, 1e-3) | ~wellg
    print(f"[grad] {len(wr)} trees, {wellg.sum()} well-conditioned constant gradients, "
          f"{(const & ~wellg).sum()} ill-conditioned", flush=True)
    assert wellg.sum() >= 0.8 * const.sum()
    assert ok[wellg].mean() >= 0.995
    okx = grad_close(gx.cpu().numpy(), gx64, 2e-3) | ~wellx
    assert wellx.mean() >= 0.9
    assert okx.mean() >= 0.995
