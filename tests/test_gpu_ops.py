"""Accuracy of the evaluation kernels' unary operators on the device (tgp_op_apply), against
float64 on dense samples of their domains. The float32 envelopes assume every one of them within
4 ulp of the exact function of its float32 argument (oracle/envelope.py); this checks that
assumption. exp and log are the library's own implementations (hardware base-2 instructions with a
compensated change of base): exp must stay within 2 ulp, and log, whose error is that of the
hardware base-2 log, within 2.5 (torch.log on the device, another implementation, is printed beside
it). sin, cos, tanh and tan come from the device math library. Needs an MI355X."""

import numpy as np
import pytest
import torch

import paper_2501_17168_amd as tgp

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
OP_SIN, OP_COS, OP_TANH, OP_EXP, OP_LOG, OP_TAN = 4, 5, 6, 7, 8, 11


def _floats_between(lo, hi, step):
    """Every `step`-th float32 in [lo, hi] (bit patterns of each sign walked in order), plus both ends."""
    out = []
    for a, b in ((lo, min(hi, -0.0)), (max(lo, 0.0), hi)):
        if a > b:
            continue
        ba = np.float32(a).view(np.uint32).astype(np.int64)
        bb = np.float32(b).view(np.uint32).astype(np.int64)
        first, last = min(ba, bb), max(ba, bb)
        out.append(np.arange(first, last + 1, step, dtype=np.int64).astype(np.uint32).view(np.float32))
    out.append(np.array([lo, hi], np.float32))
    return np.concatenate(out)


def _ulp_err(got, ref):
    """|got - ref| in units of the float32 spacing at ref (ref in float64)."""
    ref32 = np.abs(ref).astype(np.float32)
    ulp = np.spacing(np.maximum(ref32, np.float32(np.finfo(np.float32).tiny))).astype(np.float64)
    return np.abs(got.astype(np.float64) - ref) / ulp


def _apply(op, x):
    return tgp.op_apply(op, torch.from_numpy(x).to(DEV)).cpu().numpy()


def test_exp_within_two_ulp():
    """exp on its clamped domain: every 32nd float32 of [-20, 20] (about 6.9e7 values) and the
    clamp's surroundings; NaN stays NaN and arguments beyond the clamp give exp(±20)."""
    x = _floats_between(-20.0, 20.0, 32)
    got = _apply(OP_EXP, x)
    err = _ulp_err(got, np.exp(x.astype(np.float64)))
    print(f"exp: {x.size} values, max {err.max():.3f} ulp, mean {err.mean():.3f}", flush=True)
    assert err.max() <= 2.0
    edge = np.array([np.nan, np.inf, -np.inf, 1e30, -1e30, 20.0, -20.0, np.nextafter(np.float32(20), np.float32(30)),
                     0.0, -0.0], np.float32)
    e = _apply(OP_EXP, edge)
    assert np.isnan(e[0])
    np.testing.assert_array_equal(e[[1, 3, 5, 7]], np.full(4, e[5]))          # everything above 20 is exp(20)
    np.testing.assert_array_equal(e[[2, 4, 6]], np.full(3, e[6]))             # everything below -20 is exp(-20)
    assert e[8] == 1.0 and e[9] == 1.0
    assert _ulp_err(e[5:7], np.exp(np.array([20.0, -20.0]))).max() <= 2.0


def _log_case(x, label):
    arg = (np.abs(x) + np.float32(1e-6)).astype(np.float32)
    ref = np.log(arg.astype(np.float64))
    err = _ulp_err(_apply(OP_LOG, x), ref)
    lib = _ulp_err(torch.log(torch.from_numpy(arg).to(DEV)).cpu().numpy(), ref)
    print(f"log {label}: {x.size} values, max {err.max():.3f} ulp (mean {err.mean():.3f}); device library "
          f"logf max {lib.max():.3f} (mean {lib.mean():.3f})", flush=True)
    assert err.max() <= 2.5        # measured 2.31; the envelopes assume 4


def test_log_within_envelope_and_library():
    """log(|x| + 1e-6), the protected log: the float32 sum is the argument, its log is compared
    with float64; every 1024th float32 of each sign over the whole range (about 4.2e6 values), and
    every 4th float32 of [0.5, 2], where log is small and its relative accuracy hardest."""
    _log_case(_floats_between(-3.4e38, 3.4e38, 1024), "whole range")
    _log_case(_floats_between(0.5, 2.0, 4), "near 1")


def test_log_special_values():
    """NaN stays NaN, infinities of either sign give +inf, and 0 gives log(1e-6)."""
    special = _apply(OP_LOG, np.array([np.nan, np.inf, -np.inf, 0.0], np.float32))
    assert np.isnan(special[0]) and special[1] == np.inf and special[2] == np.inf
    assert abs(special[3] - np.log(np.float64(np.float32(1e-6)))) <= 2 * np.spacing(np.float32(13.8))


@pytest.mark.parametrize("op,lo,hi", [(OP_SIN, -1e4, 1e4), (OP_COS, -1e4, 1e4), (OP_TANH, -30.0, 30.0),
                                      (OP_TAN, -1.5, 1.5)])
def test_library_ops_within_envelope_assumption(op, lo, hi):
    """The device library's sin, cos, tanh and tan stay within the 4 ulp the float32 envelopes
    assume, on every 64th float32 of the range (tan away from its poles)."""
    x = _floats_between(lo, hi, 64)
    got = _apply(op, x)
    f = {OP_SIN: np.sin, OP_COS: np.cos, OP_TANH: np.tanh, OP_TAN: np.tan}[op]
    ref = f(x.astype(np.float64))
    err = _ulp_err(got, ref)
    print(f"op {op}: {x.size} values, max {err.max():.3f} ulp", flush=True)
    assert err.max() <= 4.0
