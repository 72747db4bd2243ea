"""The allocation-free fitness entry point (tgp_eval_mse_noalloc, static scratch buffer) against
tgp_eval_mse with a caller-owned workspace, through the C-ABI. Two calls in a row, the second on a
smaller population and data set, each bitwise equal to the regular call at the same launch
configuration and inside the oracle's float32 envelopes. Needs an MI355X."""

import numpy as np
import pytest
import torch

import oracle as O
import paper_2501_17168_amd as tgp
import synth
from paper_2501_17168_amd import _lib
from parity import FitnessRef, compare_fitness

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _case(name, **kw):
    w = synth.workload(name, **kw)
    Y = w.Y if w.Y is not None else w.targets_from(O.predict(*w.hidden, w.X, 1)[:, 0, :])
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    pop = tgp.Population(*(torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (w.type, w.value, w.size)))
    return w, Y, pop, torch.from_numpy(w.X).to(DEV), torch.from_numpy(Y).to(DEV)


def _check(name, kw, config):
    w, Y, pop, X, Yd = _case(name, **kw)
    c = tgp.cfg(config)
    st_a = torch.full((w.P,), -1, dtype=torch.int32, device=DEV)
    st_b = torch.full((w.P,), -1, dtype=torch.int32, device=DEV)
    out = torch.full((w.P,), -1.0, device=DEV)
    got = tgp.eval_mse_noalloc(pop, X, Yd, config=c, out=out, tree_status=st_a)
    ref = tgp.eval_mse(pop, X, Yd, config=c, ws=tgp.Workspace(DEV), tree_status=st_b)
    torch.cuda.synchronize()
    got, ref = got.cpu().numpy(), ref.cpu().numpy()
    np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))
    np.testing.assert_array_equal(st_a.cpu().numpy(), st_b.cpu().numpy())
    rep = compare_fitness(got, FitnessRef(w.type, w.value, w.size, w.X, Y), label=f"noalloc {name}")
    print(f"noalloc {name} {kw}: {rep}", flush=True)
    assert rep["tight"] >= 0.5 * rep["n"]


@pytest.mark.parametrize("config", [dict(mode=3, points_per_lane=8, block_waves=1, trees_per_unit=1),
                                    dict(mode=1, points_per_lane=4, block_waves=4)], ids=["persistent", "tree"])
def test_noalloc_matches_regular_call_twice(config):
    # first call: 600 trees of Lmax 256 on 2,000 points (3.9 MB of scratch); second call: the
    # 64-tree workload on 256 points, smaller in every dimension, over the first call's contents
    _check("hybrid", dict(P=600, D=2000), config)
    _check("plain", {}, config)


def test_noalloc_rejects_oversize_without_work():
    w, Y, pop, X, Yd = _case("hybrid", P=5299, D=2000)
    assert tgp.workspace_bytes(pop, X) > _lib.NOALLOC_SCRATCH_BYTES
    out = torch.full((w.P,), -1.0, device=DEV)
    with pytest.raises(_lib.TgpError) as e:
        tgp.eval_mse_noalloc(pop, X, Yd, out=out)
    assert e.value.code == _lib.TGP_E_TOO_LARGE
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == -1.0).all()
