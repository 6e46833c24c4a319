"""ctypes declarations of the C ABI in include/ttn.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libttn.so")

TTN_OK, TTN_EINVAL, TTN_ENOMEM, TTN_EDEVICE, TTN_ENONFINITE, TTN_EPROB = 0, -1, -2, -3, -4, -5
TTN_C64, TTN_C128 = 0, 1
TTN_AD_KRAUS, TTN_AD_TROTTER = 0, 1
TTN_RUN_DYNAMIC, TTN_RUN_STATIC, TTN_RUN_GRAPH = 0, 1, 2
TTN_DECODE_STATIC_MAX_CHECKS = 16
STATUS_NAMES = {0: "TTN_OK", -1: "TTN_EINVAL", -2: "TTN_ENOMEM", -3: "TTN_EDEVICE",
                -4: "TTN_ENONFINITE", -5: "TTN_EPROB"}

# every symbol the header declares
SYMBOLS = ("ttn_create", "ttn_destroy", "ttn_last_error", "ttn_init_product", "ttn_apply_1q",
           "ttn_apply_2q", "ttn_measure_project", "ttn_kraus_jump", "ttn_oplist_upload",
           "ttn_oplist_free", "ttn_batch_run_circuit", "ttn_set_run_mode", "ttn_log_prob", "ttn_log_prob_grad", "ttn_trace_probs",
           "ttn_decode", "ttn_decode_static",
           "ttn_compress",
           "ttn_to_statevector", "ttn_bond_dims", "ttn_uniforms", "ttn_philox_uniform_host",
           "ttn_version", "ttn_test_leg_apply", "ttn_test_gram", "ttn_test_eigh", "ttn_test_move",
           "ttn_test_sweep_plan",
           "ttn_profile_enable", "ttn_profile_read", "ttn_autotune")
CLASSES = {"contract": 0, "gram": 1, "eigh_small": 2, "eigh_large": 3, "leaf": 4, "extend": 5, "other": 6,
           "move": 7}


class Config(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("leaf_of_qubit", C.POINTER(C.c_int32)),
                ("chi_max", C.c_int32), ("cutoff", C.c_double), ("dtype", C.c_int32),
                ("ad_mode", C.c_int32), ("batch", C.c_int32), ("seed", C.c_uint64), ("stream", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("max_rank", C.c_int32), ("discarded_weight", C.c_double),
                ("degenerate_cuts", C.c_int64), ("flagged_rows", C.c_int32),
                ("hops", C.c_int64), ("launches", C.c_int64),
                ("gemm_flops", C.c_double), ("gram_flops", C.c_double), ("block_hops", C.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib() -> C.CDLL:
    """Load libttn.so; raises if it is not built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    sig = {
        "ttn_create": (i32, [C.POINTER(Config), C.POINTER(vp)]),
        "ttn_destroy": (i32, [vp]),
        "ttn_last_error": (C.c_char_p, [vp]),
        "ttn_init_product": (i32, [vp, vp]),
        "ttn_apply_1q": (i32, [vp, i32, vp, i64]),
        "ttn_apply_2q": (i32, [vp, i32, i32, vp]),
        "ttn_measure_project": (i32, [vp, i32, i32, vp, vp, vp, u64, i32]),
        "ttn_kraus_jump": (i32, [vp, i32, vp, i64, vp, vp, vp, u64, i32]),
        "ttn_oplist_upload": (i32, [vp, vp, i32, i32, i32, i32, C.POINTER(vp)]),
        "ttn_oplist_free": (i32, [vp]),
        "ttn_batch_run_circuit": (i32, [vp, vp, vp, vp, i64, u64, vp, vp, vp, C.POINTER(Stats)]),
        "ttn_log_prob": (i32, [vp, vp, vp, vp, vp, vp, i64, vp, C.POINTER(Stats)]),
        "ttn_set_run_mode": (i32, [vp, i32, C.POINTER(i64), C.POINTER(i64)]),
        "ttn_log_prob_grad": (i32, [vp, vp, vp, vp, vp, vp, i64, vp, vp, vp, C.POINTER(Stats)]),
        "ttn_trace_probs": (i32, [vp, vp, i64]),
        "ttn_decode": (i32, [vp, vp, i32, vp, i32, vp, i32, vp]),
        "ttn_decode_static": (i32, [vp, vp, i32, vp, i32, vp, i32, vp]),
        "ttn_compress": (i32, [vp]),
        "ttn_to_statevector": (i32, [vp, i32, vp]),
        "ttn_bond_dims": (i32, [vp, i32, vp]),
        "ttn_uniforms": (i32, [vp, u64, i32, i32, vp]),
        "ttn_philox_uniform_host": (dbl, [u64, u64, u64]),
        "ttn_version": (C.c_char_p, []),
        "ttn_test_leg_apply": (i32, [vp, i32, vp, i32, vp, i64, vp, i64, i32, vp, i64]),
        "ttn_test_gram": (i32, [vp, i32, vp, i32, vp, i64, vp, i64, i32]),
        "ttn_profile_enable": (i32, [vp, i32]),
        "ttn_profile_read": (i32, [vp, i32, C.POINTER(dbl), C.POINTER(i64), C.POINTER(dbl), C.POINTER(dbl)]),
        "ttn_autotune": (i32, [vp, i32, C.POINTER(i64), C.POINTER(i64)]),
        "ttn_test_eigh": (i32, [vp, i32, i32, i32, i32, dbl, vp, i64, vp, vp, i64, vp, vp, i32]),
        "ttn_test_move": (i32, [vp, i32, i32, i32, i32, dbl, vp, i64, vp, vp, i64, vp, i32]),
        "ttn_test_sweep_plan": (i32, [i32, C.POINTER(C.c_uint32), i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class TTNError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code: int, ctx=None) -> int:
    if code != TTN_OK:
        msg = lib().ttn_last_error(ctx).decode() if ctx else ""
        raise TTNError(code, msg)
    return code
