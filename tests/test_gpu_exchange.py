"""Subtree exchange (§III-B) on the GPU against the oracle: bit-exact rows and
status codes. Needs an MI355X."""

import numpy as np
import pytest
import torch

import oracle as O
import paper_2501_17168_amd as tgp
from synth import trees as ST

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def population(seed, n, L, depth, V=3):
    rng = np.random.default_rng(seed)
    return ST.depth_limited(rng, n, depth, rng.random(n) < 0.5, ST.F11, V, L)


def dev_pop(rows):
    return tgp.Population(*(torch.from_numpy(np.ascontiguousarray(r)).to(DEV) for r in rows))


def bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def assert_same(got_pop, got_status, want_rows, want_status, label):
    st = got_status.cpu().numpy()
    np.testing.assert_array_equal(st, want_status, err_msg=f"{label}: status")
    for name, g, w in zip(("type", "value", "size"), (got_pop.type, got_pop.value, got_pop.size), want_rows):
        gb, wb = bits(g.cpu().numpy()), bits(w)
        bad = np.nonzero((gb != wb).any(axis=1))[0]
        assert bad.size == 0, f"{label}: {name} differs in {bad.size} rows, first {bad[:5]}"


def t_i32(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.int32)).to(DEV)


def t_f32(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV)


@pytest.mark.parametrize("L,B", [(64, 1), (64, 7), (256, 513), (1024, 130)])
def test_index_mode_with_invalid_cases(L, B):
    """Explicit node indices, rows drawn across both populations, with out-of-range rows and
    nodes, a tree whose length is unreadable and a tight length limit mixed in."""
    print(f"[exchange index] L={L} B={B}", flush=True)
    rng = np.random.default_rng(L + B)
    P = 40
    old = population(L, P, L, depth=7 if L >= 256 else 5)
    don = population(L + 1, P, L, depth=4)
    old[2][3, 0] = np.nan                      # unreadable length: verbatim copy
    for r in range(3):
        old[r][3, 5] = 1.5                     # (garbage after the bad length is copied too)
    lo = np.nan_to_num(old[2][:, 0], nan=4).astype(int)
    ld = don[2][:, 0].astype(int)
    orow = rng.integers(-2, P + 2, B)
    nrow = rng.integers(-2, P + 2, B)
    k = np.array([rng.integers(-1, (lo[r] if 0 <= r < P else 4) + 2) for r in orow])
    j = np.array([rng.integers(-1, (ld[r] if 0 <= r < P else 4) + 2) for r in nrow])
    max_len = int(np.percentile(lo, 60))      # tight enough that some results are too long
    want, wst = O.subtree_exchange(old, don, k, j, old_row=orow, new_row=nrow, max_len=max_len)
    got, gst = tgp.subtree_exchange(dev_pop(old), dev_pop(don), t_i32(k), t_i32(j), old_row=t_i32(orow),
                                    new_row=t_i32(nrow), max_len=max_len)
    torch.cuda.synchronize()
    assert_same(got, gst, want, wst, f"index L={L} B={B}")
    if B > 100:
        assert set(np.unique(wst)) == {O.X_OK, O.X_TOO_LONG, O.X_BAD_OLD, O.X_BAD_DONOR}


@pytest.mark.parametrize("L", [32, 128, 512])
def test_uniform_mode_crossover(L):
    """One-point crossover with nodes drawn on the device from float32 uniforms, including
    uniforms at 0, just below 1, at 1 and NaN."""
    print(f"[exchange crossover] L={L}", flush=True)
    P = 300
    pop = population(7 * L, P, L, depth=8 if L >= 128 else 4)
    rng = np.random.default_rng(L)
    mate = rng.permutation(P)
    u = rng.random(P).astype(np.float32)
    w = rng.random(P).astype(np.float32)
    below1 = np.nextafter(np.float32(1), np.float32(0))
    u[:6] = [0.0, below1, 1.0, np.nan, -0.0, 0.5]
    w[6:12] = [0.0, below1, 1.0, np.nan, 2.0, 0.25]
    want, wst = O.subtree_exchange(pop, pop, u, w, new_row=mate, flags=O.OLD_UNIFORM | O.NEW_UNIFORM)
    dp = dev_pop(pop)
    got, gst = tgp.crossover(dp, t_i32(mate), t_f32(u), t_f32(w))
    torch.cuda.synchronize()
    assert_same(got, gst, want, wst, f"crossover L={L}")
    ok = wst == O.X_OK
    info, _ = tgp.plan(got, 3, 1)
    assert (info[:, 0].cpu().numpy()[ok] == 0).all()


def test_mutation_with_shorter_donor_rows():
    """Subtree mutation: donors are whole trees of a population with a shorter row length;
    the length limit is below the row length."""
    P, L, Ld = 1000, 256, 32
    pop = population(21, P, L, depth=8)
    new = population(22, P, Ld, depth=3)
    u = np.random.default_rng(5).random(P).astype(np.float32)
    want, wst = O.subtree_exchange(pop, new, u, None, max_len=200, flags=O.OLD_UNIFORM)
    got, gst = tgp.mutation(dev_pop(pop), dev_pop(new), t_f32(u), max_len=200)
    torch.cuda.synchronize()
    assert_same(got, gst, want, wst, "mutation")
    assert (wst == O.X_OK).mean() > 0.5


def test_hoist_and_identity():
    """Hoist mutation (old node 0, donor = the same tree at node k) and self-exchange at the
    same node, which must return the population unchanged."""
    P, L = 200, 128
    pop = population(31, P, L, depth=7)
    n = pop[2][:, 0].astype(int)
    k = (np.random.default_rng(2).random(P) * n).astype(np.int32)
    dp = dev_pop(pop)
    want, wst = O.subtree_exchange(pop, pop, np.zeros(P, int), k)
    got, gst = tgp.subtree_exchange(dp, dp, t_i32(np.zeros(P)), t_i32(k))
    torch.cuda.synchronize()
    assert_same(got, gst, want, wst, "hoist")
    got, gst = tgp.subtree_exchange(dp, dp, t_i32(k), t_i32(k))
    torch.cuda.synchronize()
    assert_same(got, gst, pop, np.zeros(P, np.int32), "identity")


def test_empty_batch():
    pop = dev_pop(population(1, 4, 16, depth=2))
    got, gst = tgp.subtree_exchange(pop, pop, torch.empty(0, dtype=torch.int32, device=DEV))
    torch.cuda.synchronize()
    assert got.P == 0 and gst.numel() == 0


def test_fullsize_crossover_and_graph_replay():
    """Crossover over the hybrid-size population (10,000 trees, Lmax 256) replicated to
    200,000 outputs, in the launch the benchmark times: checked against the oracle on a
    sample of outputs, every output's validity checked on the device, and replayed from a
    hipGraph."""
    from synth import workloads as W
    w = W.workload("hybrid")
    pop = (w.type, w.value, w.size)
    P, B = w.P, 200_000
    rng = np.random.default_rng(17)
    orow = rng.integers(0, P, B).astype(np.int32)
    nrow = rng.integers(0, P, B).astype(np.int32)
    u = rng.random(B).astype(np.float32)
    v = rng.random(B).astype(np.float32)
    dp = dev_pop(pop)
    args = (t_f32(u), t_f32(v))
    kw = dict(old_row=t_i32(orow), new_row=t_i32(nrow), old_uniform=True, new_uniform=True)
    got, gst = tgp.subtree_exchange(dp, dp, *args, **kw)
    torch.cuda.synchronize()
    sample = np.sort(rng.choice(B, 3000, replace=False))
    want, wst = O.subtree_exchange(pop, pop, u[sample], v[sample], old_row=orow[sample], new_row=nrow[sample],
                                   flags=O.OLD_UNIFORM | O.NEW_UNIFORM)
    st = gst.cpu().numpy()
    np.testing.assert_array_equal(st[sample], wst)
    for g, r in zip((got.type, got.value, got.size), want):
        np.testing.assert_array_equal(bits(g.cpu().numpy()[sample]), bits(r))
    info, _ = tgp.plan(got, w.V, 1)
    info = info.cpu().numpy()
    assert (info[st == 0, 0] == 0).all()
    print(f"[exchange full] {B} outputs, {np.mean(st == 0):.3f} exchanged", flush=True)

    ref = [t.clone() for t in (got.type, got.value, got.size)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tgp.subtree_exchange(dp, dp, *args, out=got, status=gst, **kw)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        tgp.subtree_exchange(dp, dp, *args, out=got, status=gst, **kw)
    for _ in range(3):
        for t in (got.type, got.value, got.size):
            t.fill_(-1.0)
        gst.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((got.type, got.value, got.size), ref):
            assert torch.equal(a.view(torch.int32), b.view(torch.int32))
        np.testing.assert_array_equal(gst.cpu().numpy(), st)


@pytest.mark.parametrize("L", [64, 256, 1024])
def test_padded_output_rows(L):
    """With the output rows already holding padded trees, only the changed columns are written
    and the rows equal those of a full write; rows whose current length is unreadable are
    written whole."""
    print(f"[exchange padded] L={L}", flush=True)
    P = 500
    pop = population(41 + L, P, L, depth=8 if L >= 256 else 5)
    prev = population(42 + L, P, L, depth=9 if L >= 256 else 5)     # what the buffer held before
    prev[2][:10, 0] = np.nan                                          # unreadable: written whole
    for r in range(3):
        prev[r][:10, L // 2:] = 7.0                                   # (its garbage must be overwritten)
    rng = np.random.default_rng(L)
    mate = rng.permutation(P)
    u = rng.random(P).astype(np.float32)
    w = rng.random(P).astype(np.float32)
    want, wst = O.subtree_exchange(pop, pop, u, w, new_row=mate, flags=O.OLD_UNIFORM | O.NEW_UNIFORM)
    dp = dev_pop(pop)
    out = dev_pop(prev)
    got, gst = tgp.crossover(dp, t_i32(mate), t_f32(u), t_f32(w), out=out, out_padded=True)
    torch.cuda.synchronize()
    assert got is out
    assert_same(got, gst, want, wst, f"padded L={L}")
    # again into the same rows (now holding the children): still the same result
    got, gst = tgp.crossover(dp, t_i32(mate), t_f32(u), t_f32(w), out=out, out_padded=True)
    torch.cuda.synchronize()
    assert_same(got, gst, want, wst, f"padded again L={L}")


def test_strided_rows_and_wider_donor():
    """Old rows as a view of a wider tensor (row stride > Lmax), donors with 512-column rows
    into 256-column outputs (long donor subtrees are refused by the length limit), and an
    output population whose rows are a strided view too."""
    P, L, Ld = 700, 256, 512
    old = population(51, P, L, depth=8)
    don = population(52, P, Ld, depth=9)
    rng = np.random.default_rng(8)
    u = rng.random(P).astype(np.float32)
    w = rng.random(P).astype(np.float32)
    mate = rng.permutation(P)
    want, wst = O.subtree_exchange(old, don, u, w, new_row=mate, flags=O.OLD_UNIFORM | O.NEW_UNIFORM)

    def wide(rows, L, extra):
        out = []
        for r in rows:
            t = torch.full((r.shape[0], L + extra), 7.0, device=DEV)
            t[:, :L] = torch.from_numpy(r).to(DEV)
            out.append(t[:, :L])
        return tgp.Population(*out)

    dold, ddon = wide(old, L, 9), wide(don, Ld, 3)
    assert dold.abi().row_stride == L + 9
    outs = [torch.full((P, L + 5), -3.0, device=DEV) for _ in range(3)]
    out = tgp.Population(*(t[:, :L] for t in outs))
    got, gst = tgp.subtree_exchange(dold, ddon, t_f32(u), t_f32(w), new_row=t_i32(mate), old_uniform=True,
                                    new_uniform=True, out=out)
    torch.cuda.synchronize()
    assert_same(got, gst, want, wst, "strided")
    assert (wst == O.X_TOO_LONG).sum() > 0
    for t in outs:                                   # the columns past Lmax are untouched
        assert (t[:, L:] == -3.0).all()
