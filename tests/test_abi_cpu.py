"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every entry point include/ttn.h declares, and its host-side generator is the
oracle's stream."""
import os
import re
import ctypes

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ttn.h")).read()
    return sorted(set(re.findall(r"^(?:ttn_status|double|int32_t|const char\*)\s+(ttn_[a-z0-9_]+)\s*\(", text, re.M)))


def _lib():
    from paper_2511_05719_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libttn.so not built")
    return _abi.lib()


def test_library_exports_every_declared_symbol():
    L = _lib()
    decl = _declared()
    assert len(decl) >= 20
    for name in decl:
        assert hasattr(L, name), name
    from paper_2511_05719_amd import _abi
    assert sorted(_abi.SYMBOLS) == decl


def test_host_generator_is_the_oracle_stream():
    _lib()
    from paper_2511_05719_amd import philox_uniform_host
    from oracle.rng import uniforms
    for seed, tid in [(0, 0), (3, 2 ** 32 + 17), (2 ** 63 + 5, 123456789)]:
        ref = uniforms(seed, [tid], 9)[0]
        got = np.array([philox_uniform_host(seed, tid, k) for k in range(9)])
        assert np.array_equal(got, ref)


def test_create_rejects_bad_config_without_gpu_work():
    L = _lib()
    from paper_2511_05719_amd import _abi
    cfg = _abi.Config()
    leaf = (ctypes.c_int32 * 2)(0, 0)      # not injective
    cfg.n_qubits = 2
    cfg.leaf_of_qubit = ctypes.cast(leaf, ctypes.POINTER(ctypes.c_int32))
    cfg.chi_max = 4
    cfg.cutoff = 1e-10
    cfg.dtype = 0
    cfg.batch = 1
    h = ctypes.c_void_p()
    assert L.ttn_create(ctypes.byref(cfg), ctypes.byref(h)) == _abi.TTN_EINVAL
    cfg.chi_max = 0
    assert L.ttn_create(ctypes.byref(cfg), ctypes.byref(h)) == _abi.TTN_EINVAL
    assert L.ttn_version().decode().startswith("ttn-mi355x")
