"""ctypes binding of libtgp.so (the C-ABI declared in include/tgp.h).

Argument marshalling only: every step of the evaluation runs in the
library's HIP kernels. The library is loaded from this package directory;
a missing library is an error, never a fallback.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtgp.so")

TGP_OK = 0
TGP_E_ARG = -1
TGP_E_SHAPE = -2
TGP_E_WORKSPACE = -4
TGP_E_UNSUPPORTED = -5
TGP_E_HIP = -6
TGP_E_TOO_LARGE = -7
TGP_E_IO = -8
NOALLOC_SCRATCH_BYTES = 32 << 20

MODE_AUTO, MODE_TREE_MAJOR, MODE_POINT_MAJOR, MODE_PERSISTENT = 0, 1, 2, 3
FLAG_NO_TAIL_CHECK = 1
FLAG_STATIC_ORDER = 2
FLAG_ADJ_RECOMPUTE = 4

# symbols the header declares; the CPU tests check that each one is exported
EXPORTS = ("tgp_workspace_bytes", "tgp_plan", "tgp_eval_mse", "tgp_eval_mse_noalloc", "tgp_eval_multi_output",
           "tgp_eval_accuracy",
           "tgp_eval_mse_grad", "tgp_autotune", "tgp_subtree_exchange", "tgp_generate", "tgp_status_str", "tgp_op_cost",
           "tgp_profile", "tgp_profile_read", "tgp_autotune_cache_load", "tgp_autotune_cache_save",
           "tgp_autotune_cached", "tgp_op_apply")

XCHG_OK, XCHG_TOO_LONG, XCHG_BAD_OLD, XCHG_BAD_DONOR = 0, 1, 2, 3
XCHG_OLD_UNIFORM, XCHG_NEW_UNIFORM, XCHG_OUT_PADDED = 1, 2, 4
GEN_GROW, GEN_FULL, GEN_RAMPED = 0, 1, 2


class TgpPop(ctypes.Structure):
    _fields_ = [("type", ctypes.c_void_p), ("value", ctypes.c_void_p), ("size", ctypes.c_void_p),
                ("P", ctypes.c_int64), ("Lmax", ctypes.c_int32), ("row_stride", ctypes.c_int64)]


class TgpData(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("V", ctypes.c_int32), ("D", ctypes.c_int64),
                ("ldx", ctypes.c_int64), ("Y", ctypes.c_void_p), ("n_out", ctypes.c_int32),
                ("ldy", ctypes.c_int64)]


class TgpCfg(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("block_waves", ctypes.c_int32),
                ("points_per_lane", ctypes.c_int32), ("trees_per_unit", ctypes.c_int32),
                ("flags", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TgpExchange(ctypes.Structure):
    _fields_ = [("old_row", ctypes.c_void_p), ("old_node", ctypes.c_void_p), ("new_row", ctypes.c_void_p),
                ("new_node", ctypes.c_void_p), ("B", ctypes.c_int64), ("max_len", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class TgpGenCfg(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("depth_min", ctypes.c_int32), ("depth_max", ctypes.c_int32),
                ("V", ctypes.c_int32), ("funcs", ctypes.POINTER(ctypes.c_int32)), ("n_funcs", ctypes.c_int32),
                ("const_lo", ctypes.c_float), ("const_hi", ctypes.c_float), ("p_func", ctypes.c_float),
                ("p_const", ctypes.c_float), ("attempts_per_depth", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("first_tree", ctypes.c_int64)]


class TgpError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: status {code} ({status_str(code)})")


_lib = None


def load():
    """Load libtgp.so once. Raises if it is missing: there is no CPU fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                          f"or `python paper_2501_17168_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    i32 = ctypes.c_int32
    lib.tgp_workspace_bytes.argtypes = [P(TgpPop), P(TgpData), i32, i32]
    lib.tgp_workspace_bytes.restype = ctypes.c_size_t
    lib.tgp_plan.argtypes = [P(TgpPop), i32, i32, P(TgpCfg), vp, vp, vp, ctypes.c_size_t, vp]
    lib.tgp_plan.restype = i32
    lib.tgp_eval_mse.argtypes = [P(TgpPop), P(TgpData), P(TgpCfg), vp, vp, vp, ctypes.c_size_t, vp]
    lib.tgp_eval_mse.restype = i32
    lib.tgp_eval_mse_noalloc.argtypes = [P(TgpPop), P(TgpData), P(TgpCfg), vp, vp, vp]
    lib.tgp_eval_mse_noalloc.restype = i32
    lib.tgp_eval_multi_output.argtypes = [P(TgpPop), P(TgpData), P(TgpCfg), vp, vp, ctypes.c_int64, vp, vp,
                                          ctypes.c_size_t, vp]
    lib.tgp_eval_multi_output.restype = i32
    lib.tgp_eval_accuracy.argtypes = [P(TgpPop), P(TgpData), P(TgpCfg), vp, vp, vp, ctypes.c_size_t, vp]
    lib.tgp_eval_accuracy.restype = i32
    lib.tgp_eval_mse_grad.argtypes = [P(TgpPop), P(TgpData), P(TgpCfg), vp, vp, vp, vp, vp, vp, ctypes.c_size_t,
                                      vp]
    lib.tgp_eval_mse_grad.restype = i32
    lib.tgp_autotune.argtypes = [P(TgpPop), P(TgpData), i32, i32, P(TgpCfg), vp, ctypes.c_size_t, vp]
    lib.tgp_autotune.restype = i32
    lib.tgp_autotune_cache_load.argtypes = [ctypes.c_char_p, P(i32), P(i32)]
    lib.tgp_autotune_cache_load.restype = i32
    lib.tgp_autotune_cache_save.argtypes = [ctypes.c_char_p]
    lib.tgp_autotune_cache_save.restype = i32
    lib.tgp_autotune_cached.argtypes = [P(TgpPop), P(TgpData), i32, i32, P(TgpCfg), P(i32)]
    lib.tgp_autotune_cached.restype = i32
    lib.tgp_subtree_exchange.argtypes = [P(TgpPop), P(TgpPop), P(TgpExchange), vp, vp, vp, ctypes.c_int64, vp,
                                         vp]
    lib.tgp_subtree_exchange.restype = i32
    lib.tgp_generate.argtypes = [P(TgpGenCfg), ctypes.c_int64, i32, vp, vp, vp, ctypes.c_int64, vp, vp]
    lib.tgp_generate.restype = i32
    lib.tgp_op_apply.argtypes = [i32, vp, vp, ctypes.c_int64, vp]
    lib.tgp_op_apply.restype = i32
    lib.tgp_op_cost.argtypes = [i32, P(ctypes.c_double)]
    lib.tgp_op_cost.restype = i32
    lib.tgp_profile.argtypes = [i32]
    lib.tgp_profile.restype = i32
    lib.tgp_profile_read.argtypes = [P(ctypes.c_double), P(ctypes.c_int64)]
    lib.tgp_profile_read.restype = i32
    lib.tgp_status_str.argtypes = [i32]
    lib.tgp_status_str.restype = ctypes.c_char_p
    _lib = lib
    return lib


def status_str(code):
    try:
        return load().tgp_status_str(int(code)).decode()
    except ImportError:
        return "library not loaded"


def check(code, where):
    if code != TGP_OK:
        raise TgpError(code, where)


def op_cost(op):
    """Cost of operator `op` in vector-ALU issue slots, measured on the current device."""
    r = ctypes.c_double()
    check(load().tgp_op_cost(int(op), ctypes.byref(r)), "tgp_op_cost")
    return r.value


def profile(enable):
    check(load().tgp_profile(int(bool(enable))), "tgp_profile")


def profile_read():
    """(summed evaluation-kernel ms, number of launches) since the last read."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    check(load().tgp_profile_read(ctypes.byref(ms), ctypes.byref(n)), "tgp_profile_read")
    return ms.value, n.value
