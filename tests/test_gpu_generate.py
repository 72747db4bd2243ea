"""Random tree generation on the GPU against the oracle: both draw from the
same Philox4x32-10 counters, so the trees must agree bit for bit. Needs an
MI355X."""

import numpy as np
import pytest
import torch

import oracle as O
from oracle import generate_oracle as G
import paper_2501_17168_amd as tgp

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
F7 = [0, 1, 2, 3, 4, 5, 11]
F11 = list(range(11))


def bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def same(got, want, label):
    for name, g, w in zip(("type", "value", "size"), (got.type, got.value, got.size), want):
        gb, wb = bits(g.cpu().numpy()), bits(w)
        bad = np.nonzero((gb != wb).any(axis=1))[0]
        assert bad.size == 0, f"{label}: {name} differs in {bad.size} rows, first {bad[:5]}"


CASES = [
    # P, Lmax, V, funcs, method, dmin, dmax, seed, range, p_func, p_const, apd, first
    (3000, 256, 3, F11, "ramped", 2, 6, 7, (-5.0, 5.0), None, None, 8, 0),
    (1000, 64, 2, F7, "grow", 0, 9, 2**40 + 3, (-1.0, 1.0), None, None, 4, 0),
    (500, 16, 2, [0, 2], "full", 0, 6, 3, (-5.0, 5.0), None, None, 8, 0),
    (777, 128, 5, [3, 4, 8, 9], "ramped", 1, 7, 5, (0.0, 10.0), 0.6, 0.3, 2, 123_456),
    (130, 1024, 1, [0, 1, 2, 3], "grow", 0, 12, 0, (-5.0, 5.0), 0.7, None, 8, 0),
    # ramped trees run in waves of one (depth limit, method) class: classes barely filled, a
    # single depth limit, and a first tree that does not start a class cycle
    (5, 64, 2, F7, "ramped", 3, 3, 9, (-5.0, 5.0), None, None, 8, 7),
    (65, 32, 2, F11, "ramped", 0, 8, 11, (-5.0, 5.0), None, None, 8, 1_000_001),
    (1, 16, 1, F7, "ramped", 1, 4, 12, (-5.0, 5.0), None, None, 8, 3),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_bit_exact_against_oracle(case):
    P, L, V, funcs, method, dmin, dmax, seed, rng, pf, pc, apd, first = CASES[case]
    print(f"[generate] case {case}: P={P} Lmax={L} {method} depth {dmin}..{dmax}", flush=True)
    m = {"grow": G.GROW, "full": G.FULL, "ramped": G.RAMPED}[method]
    want, watt = G.generate(P, L, V, funcs, method=m, d_min=dmin, d_max=dmax, seed=seed, lo=rng[0], hi=rng[1],
                            p_func=pf, p_const=pc, attempts_per_depth=apd, first_tree=first)
    got, gatt = tgp.generate(P, L, V, funcs, method=method, depth_min=dmin, depth_max=dmax, seed=seed,
                             const_range=rng, p_func=pf, p_const=pc, attempts_per_depth=apd, first_tree=first)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(gatt.cpu().numpy(), watt)
    same(got, want, f"case {case}")
    info, _ = tgp.plan(got, V, 1)
    assert (info[:, 0].cpu().numpy() == 0).all()


def test_fullsize_sample_and_graph_replay():
    """200,000 ramped trees (depth 2..8, Lmax 256, 11 ops, 2 variables): a sample of rows against
    the oracle, every tree valid on the device, and graph replays identical to the eager call."""
    P, L = 200_000, 256
    kw = dict(method="ramped", depth_min=2, depth_max=8, seed=2024)
    got, att = tgp.generate(P, L, 2, F11, **kw)
    torch.cuda.synchronize()
    rows = np.sort(np.random.default_rng(0).choice(P, 400, replace=False))
    for r in rows:
        want, watt = G.generate(1, L, 2, F11, method=G.RAMPED, d_min=2, d_max=8, seed=2024, first_tree=int(r))
        assert att[r].item() == watt[0]
        for g, w in zip((got.type, got.value, got.size), want):
            assert (bits(g[r].cpu().numpy()) == bits(w[0])).all(), f"row {r}"
    info, _ = tgp.plan(got, 2, 1)
    info = info.cpu().numpy()
    assert (info[:, 0] == 0).all()
    print(f"[generate full] mean length {info[:, 1].mean():.1f}, max {info[:, 1].max()}", flush=True)
    ref = [t.clone() for t in (got.type, got.value, got.size)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tgp.generate(P, L, 2, F11, out=got, attempts=att, **kw)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        tgp.generate(P, L, 2, F11, out=got, attempts=att, **kw)
    for _ in range(3):
        for t in (got.type, got.value, got.size):
            t.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((got.type, got.value, got.size), ref):
            assert torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_strided_output_rows():
    """Generation into a row-strided view writes the first Lmax columns of each row only."""
    P, L = 333, 64
    want, watt = G.generate(P, L, 2, F7, method=G.RAMPED, d_min=1, d_max=5, seed=77)
    outs = [torch.full((P, L + 11), 5.0, device=DEV) for _ in range(3)]
    out = tgp.Population(*(t[:, :L] for t in outs))
    got, att = tgp.generate(P, L, 2, F7, method="ramped", depth_min=1, depth_max=5, seed=77, out=out)
    torch.cuda.synchronize()
    same(got, want, "strided")
    np.testing.assert_array_equal(att.cpu().numpy(), watt)
    for t in outs:
        assert (t[:, L:] == 5.0).all()
