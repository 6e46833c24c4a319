"""ttn_decode_static (the decoder entry point that allocates nothing: its
tables live in a fixed device array of the library) against ttn_decode and
the oracle's decoder, through the C ABI: two calls in a row on one context,
the second with a smaller code (fewer checks, data bits and record columns),
then a call on a second context with a smaller batch."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workload import build_color_code  # noqa: E402
from oracle import decoder  # noqa: E402


def _decode(fn, eng, records, data_rec, checks):
    from paper_2511_05719_amd._abi import check
    data_rec = np.ascontiguousarray(np.asarray(data_rec, dtype=np.int32))
    checks = np.ascontiguousarray(np.asarray(checks, dtype=np.uint8))
    fail = torch.full((eng.batch,), 7, dtype=torch.uint8, device="cuda")
    check(fn(eng._ctx, C.c_void_p(records.data_ptr()), int(records.shape[1]), data_rec.ctypes.data,
             int(data_rec.size), checks.ctypes.data, int(checks.shape[0]), C.c_void_p(fail.data_ptr())), eng._ctx)
    torch.cuda.synchronize()
    return fail.cpu().numpy()


def _case(eng, d, n_rec, g):
    code = build_color_code(d)
    data_rec = g.permutation(n_rec)[:code.n]
    rec = g.integers(0, 2, (eng.batch, n_rec), dtype=np.uint8)
    rec_d = torch.as_tensor(rec, device="cuda").contiguous()
    return code, data_rec, rec, rec_d


def test_decode_static_matches_decode_and_oracle():
    from paper_2511_05719_amd import TTNEngine
    from paper_2511_05719_amd._abi import lib
    g = np.random.default_rng(17)
    eng = TTNEngine(13, 3000, np.arange(13), chi_max=8, cutoff=1e-10, dtype="c64", seed=0)
    for d, n_rec in ((5, 109), (3, 13)):          # the second call is smaller
        code, data_rec, rec, rec_d = _case(eng, d, n_rec, g)
        want = decoder.decode_fail(code.checks, rec[:, data_rec])
        got_static = _decode(lib().ttn_decode_static, eng, rec_d, data_rec, code.checks)
        got = _decode(lib().ttn_decode, eng, rec_d, data_rec, code.checks)
        assert np.array_equal(got_static, want), d
        assert np.array_equal(got, want), d
    eng.close()
    small = TTNEngine(13, 37, np.arange(13), chi_max=8, cutoff=1e-10, dtype="c64", seed=0)
    code, data_rec, rec, rec_d = _case(small, 3, 25, g)
    got_static = _decode(lib().ttn_decode_static, small, rec_d, data_rec, code.checks)
    assert np.array_equal(got_static, decoder.decode_fail(code.checks, rec[:, data_rec]))
    assert np.array_equal(got_static, _decode(lib().ttn_decode, small, rec_d, data_rec, code.checks))
    small.close()


def test_decode_static_rejects_too_many_checks():
    from paper_2511_05719_amd import TTNEngine, TTNError
    from paper_2511_05719_amd._abi import lib, TTN_DECODE_STATIC_MAX_CHECKS
    eng = TTNEngine(13, 4, np.arange(13), chi_max=8, cutoff=1e-10, dtype="c64", seed=0)
    n = 20
    checks = np.eye(TTN_DECODE_STATIC_MAX_CHECKS + 1, n, dtype=np.uint8)
    rec_d = torch.zeros(4, n, dtype=torch.uint8, device="cuda")
    with pytest.raises(TTNError):
        _decode(lib().ttn_decode_static, eng, rec_d, np.arange(n), checks)
    eng.close()
