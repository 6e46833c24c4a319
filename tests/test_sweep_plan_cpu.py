"""Host-side sweep plans of the coset-ordered Jacobi solver (no GPU).

A cyclic Jacobi sweep must visit every index pair once; the plan for
N = 2^k is the matchings {(i, i ^ d)}, d = 1 .. N - 1, in groups whose
matchings all act inside the cosets of {0, a, b, a ^ b} (App. B's binary
tree sizes: N = 64, 128 and 256 are the bond Gram sizes of chi_max 32, 64
and 128 after a two-qubit gate doubles a bond)."""
import ctypes as C
import os

import numpy as np
import pytest


def _lib():
    from paper_2511_05719_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libttn.so not built")
    return _abi.lib()


def _plan(k):
    L = _lib()
    buf = (C.c_uint32 * 256)()
    ng = L.ttn_test_sweep_plan(k, buf, 256)
    assert ng > 0
    return [(g & 0xFF, (g >> 8) & 0xFF, g >> 16) for g in buf[:ng]]


@pytest.mark.parametrize("k", range(2, 9))
def test_every_pair_once_per_sweep(k):
    N = 1 << k
    seen = np.zeros((N, N), dtype=int)
    for a, b, m in _plan(k):
        assert m in (1, 2, 3)
        assert 0 < a < N and 0 < b < N and a != b
        for d in (a, b, a ^ b)[:m]:
            for i in range(N):
                if i < i ^ d:
                    seen[i, i ^ d] += 1
    iu = np.triu_indices(N, 1)
    assert np.all(seen[iu] == 1)
    assert np.all(np.tril(seen) == 0)


@pytest.mark.parametrize("k", range(2, 9))
def test_group_matchings_stay_in_cosets(k):
    N = 1 << k
    for a, b, m in _plan(k):
        H = {0, a, b, a ^ b}
        coset_of = {}
        for i in range(N):
            coset_of[i] = min(i ^ h for h in H)
        for d in (a, b, a ^ b)[:m]:
            for i in range(N):
                assert coset_of[i ^ d] == coset_of[i]


def test_group_counts():
    # a partition of F_2^k minus 0 into 2-dimensional subspaces exists for
    # even k (N - 1 = 3 * groups); for odd k at most (N - 5) / 3 triples fit
    for k in range(2, 9):
        N = 1 << k
        g = _plan(k)
        triples = sum(1 for _, _, m in g if m == 3)
        if k % 2 == 0:
            assert triples == (N - 1) // 3 and len(g) == (N - 1) // 3
        else:
            assert triples <= (N - 5) // 3
            assert len(g) <= (N - 1) // 3 + 2


def test_bad_arguments():
    L = _lib()
    buf = (C.c_uint32 * 256)()
    assert L.ttn_test_sweep_plan(1, buf, 256) == -1
    assert L.ttn_test_sweep_plan(9, buf, 256) == -1
    assert L.ttn_test_sweep_plan(7, buf, 3) == -1
