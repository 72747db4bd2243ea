"""The C-ABI library on the host: it loads, exports every declared symbol, and
rejects bad arguments synchronously before any device work (no GPU needed)."""

import ctypes
import os
import re

import pytest

import paper_2501_17168_amd as tgp
from paper_2501_17168_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x10000  # never dereferenced: every call below fails a host check first


def _declared():
    txt = open(os.path.join(ROOT, "include", "tgp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tgp_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    lib = tgp.load()
    names = _declared()
    assert set(names) == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def pop(P=10, Lmax=64, stride=None):
    return _lib.TgpPop(FAKE, FAKE, FAKE, P, Lmax, Lmax if stride is None else stride)


def data(V=2, D=100, ldx=None, Y=FAKE, n_out=1, ldy=None):
    return _lib.TgpData(FAKE, V, D, D if ldx is None else ldx, Y, n_out, D if ldy is None else ldy)


def ws_bytes(p, d, n_out=1, grad=0):
    return tgp.load().tgp_workspace_bytes(ctypes.byref(p), ctypes.byref(d) if d else None, n_out, grad)


def test_workspace_bytes():
    small = ws_bytes(pop(10, 64), data())
    big = ws_bytes(pop(1000, 64), data())
    assert small > 0 and big > small
    assert ws_bytes(pop(10, 1025), data()) == 0          # Lmax beyond 1024
    assert ws_bytes(pop(10, 64), data(V=17)) == 0
    assert ws_bytes(pop(10, 64), data(), n_out=13) == 0           # more than 12 outputs
    assert ws_bytes(pop(10, 64, stride=32), data()) == 0
    # program store: (3 Lmax + 2) instructions of 8 bytes per tree dominates
    assert ws_bytes(pop(1000, 1024), data()) >= 1000 * (3 * 1024 + 2) * 8


def call_mse(p, d, ws=FAKE * 16, nbytes=1 << 40, mse=FAKE):
    lib = tgp.load()
    return lib.tgp_eval_mse(ctypes.byref(p) if p else None, ctypes.byref(d) if d else None, None,
                            ctypes.c_void_p(mse) if mse else None, None, ctypes.c_void_p(ws) if ws else None,
                            nbytes, None)


def test_eval_mse_host_checks():
    assert call_mse(None, data()) == _lib.TGP_E_ARG
    assert call_mse(pop(), None) == _lib.TGP_E_ARG
    assert call_mse(pop(), data(), mse=0) == _lib.TGP_E_ARG
    assert call_mse(pop(), data(Y=0)) == _lib.TGP_E_ARG
    assert call_mse(pop(Lmax=0), data()) == _lib.TGP_E_SHAPE
    assert call_mse(pop(Lmax=2048), data()) == _lib.TGP_E_UNSUPPORTED
    assert call_mse(pop(stride=10), data()) == _lib.TGP_E_SHAPE
    assert call_mse(pop(P=-1), data()) == _lib.TGP_E_SHAPE
    assert call_mse(pop(), data(V=0)) == _lib.TGP_E_SHAPE
    assert call_mse(pop(), data(V=17)) == _lib.TGP_E_UNSUPPORTED
    assert call_mse(pop(), data(D=0)) == _lib.TGP_E_SHAPE
    assert call_mse(pop(), data(ldx=50)) == _lib.TGP_E_SHAPE
    assert call_mse(pop(), data(ldy=50)) == _lib.TGP_E_SHAPE
    assert call_mse(pop(), data(n_out=2)) == _lib.TGP_E_SHAPE
    assert call_mse(pop(), data(), ws=0) == _lib.TGP_E_WORKSPACE
    assert call_mse(pop(), data(), ws=FAKE * 16 + 8) == _lib.TGP_E_WORKSPACE   # misaligned
    assert call_mse(pop(), data(), nbytes=64) == _lib.TGP_E_WORKSPACE
    # an empty population is a no-op, nothing is launched
    assert call_mse(pop(P=0), data()) == _lib.TGP_OK


def test_multi_output_and_plan_host_checks():
    lib = tgp.load()
    p, d = pop(), data(n_out=3)
    r = lib.tgp_eval_multi_output(ctypes.byref(p), ctypes.byref(d), None, None, None, 0, None,
                                  ctypes.c_void_p(FAKE * 16), 1 << 40, None)
    assert r == _lib.TGP_E_ARG                              # neither mse nor pred
    r = lib.tgp_eval_multi_output(ctypes.byref(p), ctypes.byref(d), None, None, ctypes.c_void_p(FAKE), 10, None,
                                  ctypes.c_void_p(FAKE * 16), 1 << 40, None)
    assert r == _lib.TGP_E_SHAPE                            # ldp < D
    d13 = data(n_out=13)
    r = lib.tgp_eval_multi_output(ctypes.byref(p), ctypes.byref(d13), None, ctypes.c_void_p(FAKE), None, 0, None,
                                  ctypes.c_void_p(FAKE * 16), 1 << 40, None)
    assert r == _lib.TGP_E_UNSUPPORTED                      # more than 12 outputs
    assert lib.tgp_plan(ctypes.byref(p), 0, 1, None, None, None, ctypes.c_void_p(FAKE * 16), 1 << 40,
                        None) == _lib.TGP_E_SHAPE
    assert lib.tgp_plan(ctypes.byref(p), 2, 1, None, None, None, None, 1 << 40, None) == _lib.TGP_E_WORKSPACE
    out = _lib.TgpCfg()
    assert lib.tgp_autotune(ctypes.byref(p), ctypes.byref(d), 1, 0, None, None, 0, None) == _lib.TGP_E_ARG


def call_xchg(old=None, don=None, B=4, max_len=64, flags=0, old_node=FAKE, new_node=None, outs=None,
              out_stride=64, x=True):
    lib = tgp.load()
    old = pop(10, 64) if old is None else old
    don = pop(10, 64) if don is None else don
    outs = (FAKE * 64, FAKE * 128, FAKE * 192) if outs is None else outs
    xx = _lib.TgpExchange(None, old_node, None, new_node, B, max_len, flags)
    return lib.tgp_subtree_exchange(ctypes.byref(old) if old else None, ctypes.byref(don) if don else None,
                                    ctypes.byref(xx) if x else None,
                                    *(ctypes.c_void_p(o) if o else None for o in outs), out_stride, None, None)


def test_subtree_exchange_host_checks():
    assert call_xchg(x=False) == _lib.TGP_E_ARG
    assert call_xchg(old=pop(P=-1)) == _lib.TGP_E_SHAPE
    assert call_xchg(don=pop(Lmax=2048)) == _lib.TGP_E_UNSUPPORTED
    assert call_xchg(old=pop(stride=10)) == _lib.TGP_E_SHAPE
    assert call_xchg(B=-1) == _lib.TGP_E_SHAPE
    assert call_xchg(flags=8) == _lib.TGP_E_ARG
    assert call_xchg(max_len=0) == _lib.TGP_E_SHAPE
    assert call_xchg(max_len=65) == _lib.TGP_E_SHAPE       # above the old rows' Lmax
    assert call_xchg(old_node=None) == _lib.TGP_E_ARG
    assert call_xchg(flags=2) == _lib.TGP_E_ARG            # uniform donor nodes need new_node
    assert call_xchg(outs=(FAKE * 64, 0, FAKE * 192)) == _lib.TGP_E_ARG
    assert call_xchg(out_stride=63) == _lib.TGP_E_SHAPE
    # outputs overlapping an input or each other
    assert call_xchg(outs=(FAKE, FAKE * 128, FAKE * 192)) == _lib.TGP_E_ARG
    assert call_xchg(outs=(FAKE * 64, FAKE * 64 + 512, FAKE * 192)) == _lib.TGP_E_ARG
    # nothing to do: no launch, whatever the pointers
    assert call_xchg(B=0, old_node=None, outs=(0, 0, 0)) == _lib.TGP_OK


def call_gen(P=10, Lmax=64, stride=64, outs=(FAKE * 64, FAKE * 128, FAKE * 192), **kw):
    lib = tgp.load()
    funcs = kw.pop("funcs", [0, 1, 2])
    fl = (ctypes.c_int32 * len(funcs))(*funcs)
    cfg = dict(method=2, depth_min=2, depth_max=6, V=2, funcs=fl, n_funcs=len(funcs), const_lo=-5.0,
               const_hi=5.0, p_func=-1.0, p_const=-1.0, attempts_per_depth=8, seed=1, first_tree=0)
    cfg.update(kw)
    g = _lib.TgpGenCfg(**cfg)
    return lib.tgp_generate(ctypes.byref(g), P, Lmax, *(ctypes.c_void_p(o) if o else None for o in outs),
                            stride, None, None)


def test_generate_host_checks():
    assert tgp.load().tgp_generate(None, 1, 8, None, None, None, 8, None, None) == _lib.TGP_E_ARG
    assert call_gen(P=-1) == _lib.TGP_E_SHAPE
    assert call_gen(Lmax=0) == _lib.TGP_E_SHAPE
    assert call_gen(stride=32) == _lib.TGP_E_SHAPE
    assert call_gen(Lmax=2048, stride=2048) == _lib.TGP_E_UNSUPPORTED
    assert call_gen(method=3) == _lib.TGP_E_ARG
    assert call_gen(depth_min=5, depth_max=4) == _lib.TGP_E_ARG
    assert call_gen(depth_max=31) == _lib.TGP_E_UNSUPPORTED
    assert call_gen(V=0) == _lib.TGP_E_ARG
    assert call_gen(funcs=[0, 12]) == _lib.TGP_E_ARG
    assert call_gen(funcs=[1, 1]) == _lib.TGP_E_ARG
    assert call_gen(const_lo=1.0, const_hi=1.0) == _lib.TGP_E_ARG
    assert call_gen(const_hi=float("inf")) == _lib.TGP_E_ARG
    assert call_gen(attempts_per_depth=0) == _lib.TGP_E_ARG
    assert call_gen(first_tree=(1 << 32) - 5) == _lib.TGP_E_ARG      # counters beyond 32 bits
    assert call_gen(p_func=float("nan")) == _lib.TGP_E_ARG
    assert call_gen(outs=(FAKE, 0, FAKE)) == _lib.TGP_E_ARG
    assert call_gen(P=0, outs=(0, 0, 0)) == _lib.TGP_OK


def test_accuracy_and_gradient_tuning_host_checks():
    lib = tgp.load()
    p = pop()
    acc = ctypes.c_void_p(FAKE)
    ws = ctypes.c_void_p(FAKE * 16)
    d1 = data(n_out=1)
    assert lib.tgp_eval_accuracy(ctypes.byref(p), ctypes.byref(d1), None, acc, None, ws, 1 << 40,
                                 None) == _lib.TGP_E_SHAPE             # one class
    d0 = data(n_out=3, Y=0)
    assert lib.tgp_eval_accuracy(ctypes.byref(p), ctypes.byref(d0), None, acc, None, ws, 1 << 40,
                                 None) == _lib.TGP_E_ARG               # no labels
    d3 = data(n_out=3)
    assert lib.tgp_eval_accuracy(ctypes.byref(p), ctypes.byref(d3), None, None, None, ws, 1 << 40,
                                 None) == _lib.TGP_E_ARG               # no output
    out = _lib.TgpCfg()
    d13 = data(n_out=13)
    assert lib.tgp_autotune(ctypes.byref(p), ctypes.byref(d13), 13, 1, ctypes.byref(out), ws, 1 << 40,
                            None) == _lib.TGP_E_UNSUPPORTED            # more outputs than the library's 12
    d5 = data(n_out=5)
    assert lib.tgp_eval_mse_grad(ctypes.byref(p), ctypes.byref(d5), None, None, acc, None, None, None, ws,
                                 1 << 40, None) == _lib.TGP_E_UNSUPPORTED   # gradients: at most 4 outputs
    assert lib.tgp_autotune(ctypes.byref(p), ctypes.byref(d1), 1, 1, ctypes.byref(out), ws, 64,
                            None) == _lib.TGP_E_WORKSPACE              # gradient workspace too small


def test_status_strings():
    for code in (0, -1, -2, -4, -5, -6, -7, -8, 7):
        s = tgp.status_str(code)
        assert isinstance(s, str) and s


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libtgp.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()


def call_noalloc(p, d, mse=FAKE):
    lib = tgp.load()
    return lib.tgp_eval_mse_noalloc(ctypes.byref(p) if p else None, ctypes.byref(d) if d else None, None,
                                    ctypes.c_void_p(mse) if mse else None, None, None)


def test_eval_mse_noalloc_host_checks():
    """The allocation-free call rejects what tgp_eval_mse rejects, with the same codes, and a
    call whose workspace would not fit its static scratch buffer with TGP_E_TOO_LARGE; all before
    any device work."""
    assert call_noalloc(None, data()) == _lib.TGP_E_ARG
    assert call_noalloc(pop(), None) == _lib.TGP_E_ARG
    assert call_noalloc(pop(), data(), mse=0) == _lib.TGP_E_ARG
    assert call_noalloc(pop(Lmax=2048), data()) == _lib.TGP_E_UNSUPPORTED
    assert call_noalloc(pop(stride=10), data()) == _lib.TGP_E_SHAPE
    assert call_noalloc(pop(), data(V=17)) == _lib.TGP_E_UNSUPPORTED
    assert call_noalloc(pop(), data(n_out=2)) == _lib.TGP_E_SHAPE
    assert call_noalloc(pop(), data(Y=0)) == _lib.TGP_E_ARG
    # the largest population of Lmax 256 on 2,000 points that fits, and one tree more
    fits = max(P for P in range(1, 6000, 1) if ws_bytes(pop(P, 256), data(D=2000)) <= _lib.NOALLOC_SCRATCH_BYTES)
    assert fits > 2000
    assert call_noalloc(pop(fits + 1, 256), data(D=2000)) == _lib.TGP_E_TOO_LARGE
    assert call_noalloc(pop(200_000, 1024), data(V=4, D=4096)) == _lib.TGP_E_TOO_LARGE
    assert "static buffer" in _lib.status_str(_lib.TGP_E_TOO_LARGE)


def _cache_line(**kw):
    e = dict(arch="gfx950", cus=256, P=1000, Lmax=64, V=2, D=5000, n_out=1, grad=0, mode=1, block_waves=4,
             points_per_lane=8, trees_per_unit=1, flags=0)
    e.update(kw)
    return ("{" + ",".join(f'"{k}":"{v}"' if k == "arch" else f'"{k}":{v}' for k, v in e.items()) + "}")


def test_autotune_cache_file_round_trip(tmp_path):
    """The persistent autotune cache, on the host: exact lines load, every malformed or
    out-of-range line is skipped and counted, and a save writes the loaded entries back in the
    same line format (no device needed)."""
    good = [_cache_line(), _cache_line(P=2000, mode=3, points_per_lane=4, trees_per_unit=2, flags=2),
            _cache_line(grad=1, mode=2, points_per_lane=3, block_waves=1, trees_per_unit=64),
            _cache_line(arch="gfx942", cus=304, D=70000, n_out=12, points_per_lane=4) + "  "]
    bad = ["", "not json", _cache_line()[:-1],                       # truncated
           _cache_line() + "x",                                      # trailing garbage
           _cache_line(mode=0), _cache_line(mode=4),                 # unknown schedules
           _cache_line(points_per_lane=3),                           # forward calls: 4, 8 or 16
           _cache_line(grad=1, mode=2, points_per_lane=8),           # gradient calls: 2 to 4
           _cache_line(grad=1, mode=1, points_per_lane=2),           # gradient calls are point-major
           _cache_line(block_waves=3), _cache_line(trees_per_unit=0),
           _cache_line(flags=8), _cache_line(grad=1, mode=2, points_per_lane=2, flags=2),
           _cache_line(V=17), _cache_line(Lmax=2048), _cache_line(n_out=13),
           _cache_line(grad=1, mode=2, points_per_lane=2, n_out=5),
           _cache_line(P=0), _cache_line(D=-5), _cache_line(cus=0), _cache_line(grad=2),
           _cache_line(arch="GFX950"), _cache_line(arch="gfx950:xnack-"),
           _cache_line(arch="x" * 40),                               # longer than any architecture name
           '{"cus":256,' + _cache_line()[1:],                        # keys out of order
           "z" * 3000]                                               # longer than a line buffer
    path = tmp_path / "cache.jsonl"
    path.write_text("\n".join(good[:2] + bad + good[2:]) + "\n")
    n_ok, n_bad = tgp.api.autotune_cache_load(str(path))
    assert n_ok == len(good)
    assert n_bad == len(bad) - 1          # the empty line is skipped without counting
    out = tmp_path / "saved.jsonl"
    tgp.api.autotune_cache_save(str(out))
    saved = set(out.read_text().splitlines())
    assert {g.strip() for g in good} <= saved
    # what was saved loads again, line for line
    n2, b2 = tgp.api.autotune_cache_load(str(out))
    assert (n2, b2) == (len(saved), 0)
    lib = tgp.load()
    assert lib.tgp_autotune_cache_load(None, None, None) == _lib.TGP_E_ARG
    assert lib.tgp_autotune_cache_save(None) == _lib.TGP_E_ARG
    assert lib.tgp_autotune_cache_load(os.fsencode(tmp_path / "missing.jsonl"), None, None) == _lib.TGP_E_IO
    assert lib.tgp_autotune_cache_save(os.fsencode(tmp_path / "no_dir" / "x.jsonl")) == _lib.TGP_E_IO
    assert "cache" in _lib.status_str(_lib.TGP_E_IO)


def test_op_apply_host_checks():
    """tgp_op_apply rejects binary and unknown ops, negative sizes and null arrays before any
    device work; an empty call does nothing."""
    lib = tgp.load()
    f = ctypes.c_void_p(FAKE)
    for op in (0, 3, 9, 10, 12, -1):
        assert lib.tgp_op_apply(op, f, f, 10, None) == _lib.TGP_E_ARG
    assert lib.tgp_op_apply(7, f, f, -1, None) == _lib.TGP_E_ARG
    assert lib.tgp_op_apply(7, None, f, 10, None) == _lib.TGP_E_ARG
    assert lib.tgp_op_apply(7, f, None, 10, None) == _lib.TGP_E_ARG
    assert lib.tgp_op_apply(7, None, None, 0, None) == _lib.TGP_OK
