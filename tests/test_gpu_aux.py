"""The library's auxiliary paths on the device: the persistent autotune cache (in process and
across processes through TGP_AUTOTUNE_CACHE), the TGP_FORCE_MODE override, and graph capture with
its fallback to eager calls. Needs an MI355X."""

import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import oracle as O
import paper_2501_17168_amd as tgp
import synth
from parity import FitnessRef, compare_fitness

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _case(P=300, D=2000):
    w = synth.workload("hybrid", P=P, D=D)
    Y = w.targets_from(O.predict(*w.hidden, w.X, 1)[:, 0, :]).astype(np.float32)
    pop = tgp.Population(*(torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (w.type, w.value, w.size)))
    return w, Y, pop, torch.from_numpy(w.X).to(DEV), torch.from_numpy(Y).to(DEV)


def _device_id():
    p = torch.cuda.get_device_properties(0)
    return p.gcnArchName.split(":")[0], p.multi_processor_count


def _line(arch, cus, w, grad, cfg):
    e = dict(arch=arch, cus=cus, P=w.P, Lmax=w.type.shape[1], V=w.V, D=w.D, n_out=1, grad=grad, **cfg)
    return "{" + ",".join(f'"{k}":"{v}"' if k == "arch" else f'"{k}":{v}' for k, v in e.items()) + "}"


def test_cache_file_entry_is_used(tmp_path):
    """A cache line for this device and shape makes a call without a configuration use it
    (tgp_autotune_cached reports it), and the result equals the explicit call's bitwise; a line
    for another device is loaded but never matches."""
    w, Y, pop, X, Yd = _case(P=211, D=1500)
    arch, cus = _device_id()
    want = dict(mode=2, block_waves=2, points_per_lane=4, trees_per_unit=4, flags=0)
    path = tmp_path / "cache.jsonl"
    path.write_text(_line(arch, cus, w, 0, want) + "\n"
                    + _line(arch, cus + 1, w, 1, dict(mode=2, block_waves=1, points_per_lane=2, trees_per_unit=1,
                                                      flags=0)) + "\n")
    assert tgp.autotune_cache_load(str(path)) == (2, 0)
    assert tgp.autotune_cached(pop, X, Yd) == want
    assert tgp.autotune_cached(pop, X, Yd, want_grad=True) is None      # the other device's entry
    ws = tgp.Workspace(DEV)
    auto = tgp.eval_mse(pop, X, Yd, ws=ws).cpu().numpy()
    expl = tgp.eval_mse(pop, X, Yd, config=tgp.cfg(**want), ws=ws).cpu().numpy()
    np.testing.assert_array_equal(auto.view(np.uint32), expl.view(np.uint32))
    compare_fitness(auto, FitnessRef(w.type, w.value, w.size, w.X, Y), label="cached configuration")


_CHILD = r"""
import json, sys
import numpy as np, torch
sys.path.insert(0, sys.argv[1])
import oracle as O, synth, paper_2501_17168_amd as tgp
w = synth.workload("hybrid", P=173, D=1300)
Y = w.targets_from(O.predict(*w.hidden, w.X, 1)[:, 0, :]).astype(np.float32)
dev = torch.device("cuda:0")
pop = tgp.Population(*(torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (w.type, w.value, w.size)))
X, Yd = torch.from_numpy(w.X).to(dev), torch.from_numpy(Y).to(dev)
before = tgp.autotune_cached(pop, X, Yd, want_grad=True)
tuned = tgp.autotune(pop, X, Yd, want_grad=True) if sys.argv[2] == "tune" else None
print(json.dumps({"before": before, "tuned": tuned}), flush=True)
"""


def _child(path, what):
    env = dict(os.environ, TGP_AUTOTUNE_CACHE=str(path))
    r = subprocess.run([sys.executable, "-c", _CHILD, ROOT, what], env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_cache_persists_across_processes(tmp_path):
    """TGP_AUTOTUNE_CACHE: a process that tunes the gradient call appends its choice to the file
    (one exact line for this device); a later process finds it without tuning."""
    path = tmp_path / "tgp_cache.jsonl"
    first = _child(path, "tune")
    assert first["before"] is None and first["tuned"]["mode"] == 2
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    arch, cus = _device_id()
    e = json.loads(lines[0])
    assert (e["arch"], e["cus"], e["P"], e["D"], e["grad"]) == (arch, cus, 173, 1300, 1)
    second = _child(path, "lookup")
    assert second["before"] == first["tuned"]


def test_force_mode_overrides_the_schedule():
    """TGP_FORCE_MODE replaces the schedule of every forward call: a tree-major configuration
    under TGP_FORCE_MODE=point-major gives the point-major call's fitness bit for bit, and an
    unknown value changes nothing."""
    w, Y, pop, X, Yd = _case()
    ws = tgp.Workspace(DEV)
    c_tree = tgp.cfg(mode=1, points_per_lane=8, block_waves=4)
    c_point = tgp.cfg(mode=2, points_per_lane=8, block_waves=4)
    plain = tgp.eval_mse(pop, X, Yd, config=c_point, ws=ws).cpu().numpy()
    tree = tgp.eval_mse(pop, X, Yd, config=c_tree, ws=ws).cpu().numpy()
    old = os.environ.get("TGP_FORCE_MODE")
    try:
        os.environ["TGP_FORCE_MODE"] = "point-major"
        forced = tgp.eval_mse(pop, X, Yd, config=c_tree, ws=ws).cpu().numpy()
        os.environ["TGP_FORCE_MODE"] = "sideways"
        unknown = tgp.eval_mse(pop, X, Yd, config=c_tree, ws=ws).cpu().numpy()
    finally:
        if old is None:
            os.environ.pop("TGP_FORCE_MODE", None)
        else:
            os.environ["TGP_FORCE_MODE"] = old
    np.testing.assert_array_equal(forced.view(np.uint32), plain.view(np.uint32))
    np.testing.assert_array_equal(unknown.view(np.uint32), tree.view(np.uint32))
    compare_fitness(forced, FitnessRef(w.type, w.value, w.size, w.X, Y), label="forced point-major")


def test_graphed_call_and_capture_fallback():
    """GraphedCall: a captured evaluation replays to the eager result (eager work between
    replays); a capture that fails (here the callable raises while it is being captured) leaves
    the helper in eager mode with the reason kept, and its calls still give the eager result."""
    w, Y, pop, X, Yd = _case()
    ws = tgp.Workspace(DEV)
    c = tgp.cfg(mode=3, points_per_lane=8, block_waves=4, trees_per_unit=2)
    out = torch.empty(w.P, device=DEV)
    eager = tgp.eval_mse(pop, X, Yd, config=c, ws=ws, out=out).cpu().numpy()
    g = tgp.GraphedCall(lambda: tgp.eval_mse(pop, X, Yd, config=c, ws=ws, out=out))
    assert g.mode == "graph" and g.reason is None
    other = tgp.Workspace(DEV)
    for _ in range(3):
        out.fill_(-1.0)
        torch.cuda.synchronize()
        g()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), eager.view(np.uint32))
        tgp.eval_mse(pop, X, Yd, config=tgp.cfg(mode=1), ws=other)     # eager work between replays
    calls = {"n": 0}

    def refuse_capture():
        calls["n"] += 1
        tgp.eval_mse(pop, X, Yd, config=c, ws=ws, out=out)
        if torch.cuda.is_current_stream_capturing():
            raise RuntimeError("this call cannot be captured")

    f = tgp.GraphedCall(refuse_capture)
    assert f.mode == "eager" and "cannot be captured" in f.reason
    for _ in range(2):
        out.fill_(-1.0)
        f()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), eager.view(np.uint32))
    assert calls["n"] == 4          # warm-up, the failed capture, two eager calls
