"""Kernel-level parity on the GPU: the counter-based generator, the MFMA
contraction and Gram kernels and the FP64 Jacobi centre-move factors, each
against a direct numpy evaluation of its definition."""
import ctypes as C
import zlib

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _engine(dtype="c128", n_qubits=16, chi=64, batch=8):
    from paper_2511_05719_amd import TTNEngine
    return TTNEngine(n_qubits, batch, np.arange(n_qubits), chi_max=chi, cutoff=1e-13, dtype=dtype, seed=5)


def _dev_complex(a, dtype):
    t = torch.view_as_real(torch.as_tensor(a.astype(np.complex128 if dtype == "c128" else np.complex64)))
    return t.contiguous().cuda()


def _host_complex(t):
    a = t.cpu().numpy()
    return a[..., 0].astype(np.float64) + 1j * a[..., 1].astype(np.float64)


def _dev_gram(G):
    # the Gram matrices as the engine hands them to its solvers: only the
    # upper triangle is guaranteed (the Gram launch skips tiles below the
    # diagonal), so the strictly lower entries are poisoned with NaN here
    Gp = G.copy()
    n = G.shape[-1]
    Gp[..., np.tril_indices(n, -1)[0], np.tril_indices(n, -1)[1]] = np.nan
    return torch.view_as_real(torch.as_tensor(Gp)).contiguous().cuda()


def _kept_band(w, cutoff, dtype):
    # the kept counts a solve may return for normalised eigenvalues w: exact
    # in complex128; complex64 contexts stop the Jacobi sweeps once every
    # off-diagonal ratio is below sqrt(1e-10) / 4, which resolves eigenvalues
    # to ~1e-11 of the trace, so a value within that of the cutoff may fall
    # either side
    if dtype == "c128":
        k = int((w > cutoff).sum())
        return k, k
    return int((w > cutoff + 1e-11).sum()), int((w > cutoff - 1e-11).sum())


def test_device_uniforms_match_oracle_stream():
    from oracle.rng import uniforms
    eng = _engine()
    got = eng.uniforms(traj_offset=11, rows=9, n_draws=37)
    ref = uniforms(5, np.arange(11, 20), 37)
    assert np.array_equal(got, ref)
    eng.close()


SHAPES = [(2, 2, 4), (3, 5, 7), (16, 16, 64), (64, 64, 16), (1, 70, 33), (8, 40, 48), (4, 130, 20)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("leg", [0, 1, 2])
@pytest.mark.parametrize("newd", [1, 5, 40, 100])
def test_leg_contraction(dtype, shape, leg, newd):
    # newd and the shapes cover every output tile shape (32 x 32 with the K
    # chunk split over the waves, 128 x 32, 32 x 128, 64 x 64), ragged edges
    # and K ranges of several chunks
    from paper_2511_05719_amd._abi import lib, check
    g = np.random.default_rng(zlib.crc32(repr((dtype, shape, leg, newd)).encode()))
    rows = 3
    n = shape[leg]
    T = g.normal(size=(rows,) + shape) + 1j * g.normal(size=(rows,) + shape)
    W = g.normal(size=(rows, newd, n)) + 1j * g.normal(size=(rows, newd, n))
    eng = _engine(dtype)
    Td, Wd = _dev_complex(T, dtype), _dev_complex(W, dtype)
    oshape = list(shape)
    oshape[leg] = newd
    out = torch.zeros((rows,) + tuple(oshape) + (2,), dtype=Td.dtype, device="cuda")
    dims = (C.c_int32 * 3)(*shape)
    check(lib().ttn_test_leg_apply(eng._ctx, rows, dims, leg, Td.data_ptr(), T.size, Wd.data_ptr(), W.size,
                                   newd, out.data_ptr(), out.numel() // 2), eng._ctx)
    sub = {0: "tijk,tai->tajk", 1: "tijk,taj->tiak", 2: "tijk,tak->tija"}[leg]
    Tr, Wr = T, W
    if dtype == "c64":
        Tr, Wr = T.astype(np.complex64).astype(np.complex128), W.astype(np.complex64).astype(np.complex128)
    ref = np.einsum(sub, Tr, Wr)
    got = _host_complex(out)
    tol = 1e-12 if dtype == "c128" else 2e-6
    assert np.abs(got - ref).max() <= tol * np.sqrt(n) * np.abs(ref).max()
    eng.close()


# every output-tile shape on every kind of launch, whatever the shape would
# be chosen for: 64x64, 128x32, 32x128, 32x32 and 16x16 with the K chunk
# split over the waves, 16x128 (ragged edges in both directions, several
# tiles, K ranges of one and of several chunks, both operand layouts)
FORCED_SHAPES = [(3, 5, 7), (20, 33, 17), (1, 70, 40), (40, 6, 130)]


@pytest.mark.parametrize("cfg", range(6))
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("shape", FORCED_SHAPES)
def test_every_tile_shape_contracts_and_grams(cfg, dtype, shape):
    from paper_2511_05719_amd._abi import lib, check
    g = np.random.default_rng(zlib.crc32(repr((cfg, dtype, shape)).encode()))
    rows = 3
    eng = _engine(dtype)
    eng.autotune(True, force_cfg=cfg)
    T = g.normal(size=(rows,) + shape) + 1j * g.normal(size=(rows,) + shape)
    if dtype == "c64":
        T = T.astype(np.complex64).astype(np.complex128)
    Td = _dev_complex(T, dtype)
    dims = (C.c_int32 * 3)(*shape)
    tol = 1e-12 if dtype == "c128" else 2e-6
    for leg in range(3):
        n = shape[leg]
        for newd in (3, 37):
            W = g.normal(size=(rows, newd, n)) + 1j * g.normal(size=(rows, newd, n))
            if dtype == "c64":
                W = W.astype(np.complex64).astype(np.complex128)
            oshape = list(shape)
            oshape[leg] = newd
            out = torch.full((rows,) + tuple(oshape) + (2,), float("nan"), dtype=Td.dtype, device="cuda")
            check(lib().ttn_test_leg_apply(eng._ctx, rows, dims, leg, Td.data_ptr(), T.size,
                                           _dev_complex(W, dtype).data_ptr(), W.size, newd, out.data_ptr(),
                                           out.numel() // 2), eng._ctx)
            sub = {0: "tijk,tai->tajk", 1: "tijk,taj->tiak", 2: "tijk,tak->tija"}[leg]
            ref = np.einsum(sub, T, W)
            got = _host_complex(out)
            assert np.abs(got - ref).max() <= tol * np.sqrt(n) * np.abs(ref).max(), (leg, newd)
        G = torch.full((1, rows, n, n, 2), float("nan"), dtype=torch.float64, device="cuda")
        check(lib().ttn_test_gram(eng._ctx, rows, dims, leg, Td.data_ptr(), T.size, G.data_ptr(),
                                  rows * n * n, 1), eng._ctx)
        Tm = np.moveaxis(T, 1 + leg, -1).reshape(rows, -1, n)
        ref = np.einsum("tmi,tmj->tij", Tm.conj(), Tm)
        got = _host_complex(G)[0]
        up = np.triu_indices(n)
        assert np.abs(got[:, up[0], up[1]] - ref[:, up[0], up[1]]).max() <= 1e-13 * np.abs(ref).max(), leg
        # the diagonal of a Hermitian matrix is written real
        assert np.all(got[:, np.arange(n), np.arange(n)].imag == 0.0)
    eng.autotune(None)
    eng.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("leg", [0, 1, 2])
@pytest.mark.parametrize("ksplit", [1, 3])
def test_gram_fp64(dtype, shape, leg, ksplit):
    from paper_2511_05719_amd._abi import lib, check
    g = np.random.default_rng(7 + zlib.crc32(repr((dtype, shape, leg)).encode()))
    rows = 2
    n = shape[leg]
    T = g.normal(size=(rows,) + shape) + 1j * g.normal(size=(rows,) + shape)
    if dtype == "c64":
        T = T.astype(np.complex64).astype(np.complex128)     # the kernel sees these exact values
    eng = _engine(dtype)
    Td = _dev_complex(T, dtype)
    # slices start as NaN: every slice (an empty K part too) must be written
    G = torch.full((ksplit, rows, n, n, 2), float("nan"), dtype=torch.float64, device="cuda")
    dims = (C.c_int32 * 3)(*shape)
    check(lib().ttn_test_gram(eng._ctx, rows, dims, leg, Td.data_ptr(), T.size, G.data_ptr(),
                              ksplit * rows * n * n, ksplit), eng._ctx)
    Tm = np.moveaxis(T, 1 + leg, -1).reshape(rows, -1, n)
    ref = np.einsum("tmi,tmj->tij", Tm.conj(), Tm)
    got = _host_complex(G).sum(axis=0)
    # FP64 accumulation of exact products: rounding only; the upper triangle
    # is written (tiles wholly below the diagonal are skipped)
    up = np.triu_indices(n)
    assert np.abs(got[:, up[0], up[1]] - ref[:, up[0], up[1]]).max() <= 1e-13 * np.abs(ref).max()
    eng.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,rank", [(1, 1), (2, 2), (4, 3), (16, 16), (64, 40), (64, 64), (80, 80), (95, 70),
                                    (100, 100), (113, 90), (120, 120), (121, 100), (128, 128), (128, 77),
                                    (150, 120), (200, 150), (240, 200), (256, 256), (256, 90)])
def test_eigh_centre_move_factors(dtype, n, rank):
    # n > 128: chi_max = 128 contexts, packed Gram matrix in device memory.
    # Above 64, sizes below 15/16 of the next power of two take the circle-
    # ordered solver (here n = 80, 95 and 113 (odd), 100, 150, 200); the
    # others the coset-ordered one, padded to 128 or 256 (n = 120, 121 (odd),
    # 240) or not (128, 256).
    from paper_2511_05719_amd._abi import lib, check
    g = np.random.default_rng(n * 1000 + rank)
    rows, m = 4, max(n, 8) * 3
    M = (g.normal(size=(rows, m, rank)) + 1j * g.normal(size=(rows, m, rank))) @ \
        (g.normal(size=(rows, rank, n)) + 1j * g.normal(size=(rows, rank, n)))
    M *= (10.0 ** (-np.arange(n) / 12.0))[None, None, :]          # graded spectrum
    M /= np.linalg.norm(M.reshape(rows, -1), axis=1)[:, None, None]
    G = np.einsum("tmi,tmj->tij", M.conj(), M)
    eng = _engine(dtype, chi=128 if n > 128 else 64)
    Gd = _dev_gram(G)
    wdt = torch.float64 if dtype == "c128" else torch.float32
    Wi = torch.zeros(rows, n, n, 2, dtype=wdt, device="cuda")
    Wa = torch.zeros(rows, n, n, 2, dtype=wdt, device="cuda")
    rk = torch.zeros(rows, dtype=torch.int32, device="cuda")
    cutoff = 1e-13
    check(lib().ttn_test_eigh(eng._ctx, rows, n, n, n, cutoff, Gd.data_ptr(), rows * n * n, Wi.data_ptr(),
                              Wa.data_ptr(), rows * n * n, rk.data_ptr(), None, 1), eng._ctx)
    Wi, Wa, rk = _host_complex(Wi), _host_complex(Wa), rk.cpu().numpy()
    for t in range(rows):
        s = np.linalg.svd(M[t], compute_uv=False)
        k_lo, k_hi = _kept_band(s ** 2 / (s ** 2).sum(), cutoff, dtype)
        assert k_lo <= rk[t] <= k_hi
        k = rk[t]
        # c128: components of weight near the cutoff mix across it by
        # ~eps * |G| / gap, i.e. up to ~1e-3 sqrt(cutoff) in amplitude
        tol = (1e-11 + 1e-3 * np.sqrt(cutoff)) if dtype == "c128" else 2e-5
        # (M V S^-1)(S V^H) is the renormalised best rank-k approximation of M
        u_, s_, vh_ = np.linalg.svd(M[t], full_matrices=False)
        Mk = (u_[:, :k] * s_[:k]) @ vh_[:k]
        Mk /= np.linalg.norm(Mk)
        U = M[t] @ Wi[t, :k].T
        assert np.abs(U @ Wa[t, :k] - Mk).max() < tol
        # M V = U S has Gram diag(s^2): orthogonal columns weighted by s
        sa = np.linalg.norm(Wa[t, :k], axis=1)
        US = U * sa[None, :]
        assert np.abs(US.conj().T @ US - np.diag(sa ** 2)).max() < tol * s[0] ** 2
        # the kept values are the largest singular values, descending
        assert np.abs(sa - s[:k]).max() < tol * s[0]
        assert np.all(np.diff(sa) <= 1e-12)
        assert np.all(Wi[t, k:] == 0) and np.all(Wa[t, k:] == 0)
    eng.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,blocks", [(24, 1), (64, 1), (100, 1), (128, 1), (200, 1), (64, 2), (128, 2), (256, 2)])
def test_eigh_zero_rows_are_compacted(dtype, n, blocks):
    # a bond padded beyond this row's dimension: columns of M (rows and
    # columns of G) exactly zero, as a prefix or scattered (the unused rows of
    # a block), down to one live row and none; the solver works on the live
    # rows only and must return the factors of the full problem, with exact
    # zeros in the dead columns
    from paper_2511_05719_amd._abi import lib, check
    g = np.random.default_rng(n * 7 + blocks)
    rows, K = 6, 2 * n
    h = n // blocks
    live = np.zeros((rows, n), bool)
    for b in range(blocks):
        sl = slice(b * h, (b + 1) * h)
        live[0, sl] = np.arange(h) < h // 2                     # prefix
        live[1, sl] = g.random(h) < 0.6                          # scattered
        live[2, sl] = np.arange(h) < 1                           # one live row
        live[3, sl] = True                                       # none dead
        live[4, sl] = (np.arange(h) % 3) != 1                    # regular holes
        live[5, sl] = False                                      # all dead
    live[5, 0] = blocks == 2                                     # block 0 of row 5 keeps one row
    M = np.zeros((rows, K, n), complex)
    for t in range(rows):
        for b in range(blocks):
            idx = np.nonzero(live[t, b * h:(b + 1) * h])[0] + b * h
            if len(idx) == 0:
                continue
            r = max(1, (2 * len(idx)) // 3)
            A = (g.normal(size=(K, r)) + 1j * g.normal(size=(K, r))) @ \
                (g.normal(size=(r, len(idx))) + 1j * g.normal(size=(r, len(idx))))
            A *= (10.0 ** (-np.arange(len(idx)) / 12.0))[None, :]
            M[t][:, idx] = A
        nrm = np.linalg.norm(M[t])
        if nrm > 0:
            M[t] /= nrm
    G = np.zeros((rows, n, n), complex)
    for b in range(blocks):
        sl = slice(b * h, (b + 1) * h)
        G[:, sl, sl] = np.einsum("tki,tkj->tij", M[:, :, sl].conj(), M[:, :, sl])
    eng = _engine(dtype, chi=128 if n > 128 else 64)
    Gd = _dev_gram(G)
    wdt = torch.float64 if dtype == "c128" else torch.float32
    Wi = torch.full((rows, n, n, 2), 7.0, dtype=wdt, device="cuda")
    Wa = torch.full((rows, n, n, 2), 7.0, dtype=wdt, device="cuda")
    rk = torch.full((rows,), -1, dtype=torch.int32, device="cuda")
    cutoff = 1e-12
    check(lib().ttn_test_eigh(eng._ctx, rows, n, n, n // blocks, cutoff, Gd.data_ptr(), rows * n * n,
                              Wi.data_ptr(), Wa.data_ptr(), rows * n * n,
                              rk.data_ptr() if blocks == 1 else None, None, blocks), eng._ctx)
    Wi, Wa, rk = _host_complex(Wi), _host_complex(Wa), rk.cpu().numpy()
    tol = 1e-9 if dtype == "c128" else 3e-5
    for t in range(rows):
        assert np.all(Wi[t][:, ~live[t]] == 0) and np.all(Wa[t][:, ~live[t]] == 0)
        for b in range(blocks):
            sl = slice(b * h, (b + 1) * h)
            Mb = M[t][:, sl]
            s = np.linalg.svd(Mb, compute_uv=False)
            tot = np.linalg.norm(M[t]) ** 2
            k_lo, k_hi = _kept_band(s ** 2 / tot, cutoff, dtype) if tot > 0 else (0, 0)
            wi, wa = Wi[t, sl, sl], Wa[t, sl, sl]
            k = int(np.sum(np.linalg.norm(wa, axis=1) > 0))
            assert k_lo <= k <= k_hi, (t, b, k, k_lo, k_hi)
            if blocks == 1:
                assert rk[t] == k
            assert np.all(wi[k:] == 0) and np.all(wa[k:] == 0)
            if blocks == 2:
                other = slice((1 - b) * h, (2 - b) * h)
                assert np.all(Wi[t, sl, other] == 0) and np.all(Wa[t, sl, other] == 0)
            if k == 0:
                continue
            u_, s_, vh_ = np.linalg.svd(Mb, full_matrices=False)
            Mk = (u_[:, :k] * s_[:k]) @ vh_[:k]
            if blocks == 1:
                Mk /= np.linalg.norm(Mk)
            U = Mb @ wi[:k].T
            assert np.abs(U @ wa[:k] - Mk).max() < tol * max(1.0, s[0])
            sa = np.linalg.norm(wa[:k], axis=1)          # descending kept values
            assert np.all(np.diff(sa) <= (1e-12 if dtype == "c128" else 1e-6) * sa[0])
    eng.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,rank,blocks", [(1, 1, 1), (5, 3, 1), (16, 16, 1), (40, 17, 1), (64, 64, 1), (64, 30, 1),
                                           (32, 9, 2), (128, 50, 2), (65, 65, 1), (100, 70, 1), (128, 128, 1),
                                           (128, 20, 1)])
def test_exact_move_factors(dtype, n, rank, blocks):
    # pivoted Cholesky centre move: x W_iso^T must be an isometry and, since
    # nothing above the cutoff is dropped, (x W_iso^T) W_abs must rebuild the
    # node (normalised by the kept weight, or by the whole trace for blocks);
    # the rank is the numerical rank; dead rows (zero Gram diagonal)
    # scattered in
    from paper_2511_05719_amd._abi import lib, check
    g = np.random.default_rng(n * 31 + rank + blocks)
    rows, K = 4, 3 * n + 4
    h = n // blocks
    M = np.zeros((rows, K, n), complex)
    for t in range(rows):
        for b in range(blocks):
            cols = np.arange(b * h, (b + 1) * h)
            dead = g.random(h) < (0.25 if t % 2 else 0.0)
            live = cols[~dead]
            if len(live) == 0:
                continue
            r = min(rank // blocks if blocks > 1 else rank, len(live))
            A = (g.normal(size=(K, r)) + 1j * g.normal(size=(K, r))) @ \
                (g.normal(size=(r, len(live))) + 1j * g.normal(size=(r, len(live))))
            A *= (10.0 ** (-np.arange(len(live)) / 32.0))[None, :]
            M[t][:, live] = A
        if np.linalg.norm(M[t]) > 0:
            M[t] /= np.linalg.norm(M[t])
    G = np.zeros((rows, n, n), complex)
    for b in range(blocks):
        sl = slice(b * h, (b + 1) * h)
        G[:, sl, sl] = np.einsum("tki,tkj->tij", M[:, :, sl].conj(), M[:, :, sl])
    eng = _engine(dtype, chi=64 if n <= 64 or blocks == 2 else 128)
    Gd = _dev_gram(G)
    wdt = torch.float64 if dtype == "c128" else torch.float32
    Wi = torch.full((rows, n, n, 2), 7.0, dtype=wdt, device="cuda")
    Wa = torch.full((rows, n, n, 2), 7.0, dtype=wdt, device="cuda")
    rk = torch.full((rows,), -1, dtype=torch.int32, device="cuda")
    cutoff = 1e-12
    check(lib().ttn_test_move(eng._ctx, rows, n, n, h, cutoff, Gd.data_ptr(), rows * n * n, Wi.data_ptr(),
                              Wa.data_ptr(), rows * n * n, rk.data_ptr() if blocks == 1 else None, blocks), eng._ctx)
    Wi, Wa, rk = _host_complex(Wi), _host_complex(Wa), rk.cpu().numpy()
    tol = 1e-9 if dtype == "c128" else 3e-5
    for t in range(rows):
        for b in range(blocks):
            sl = slice(b * h, (b + 1) * h)
            Mb = M[t][:, sl]
            s = np.linalg.svd(Mb, compute_uv=False) if np.any(Mb) else np.zeros(1)
            r_num = int((s ** 2 > 1e-9 * np.sum(s ** 2)).sum()) if np.any(s) else 0
            wi, wa = Wi[t, sl, sl], Wa[t, sl, sl]
            k = int(np.sum(np.linalg.norm(wa, axis=1) > 0))
            assert k >= r_num and k <= min(h, Mb.shape[0])
            if blocks == 1:
                assert rk[t] == k
            assert np.all(wi[k:] == 0) and np.all(wa[k:] == 0)
            if blocks == 2:
                other = slice((1 - b) * h, (2 - b) * h)
                assert np.all(Wi[t, sl, other] == 0) and np.all(Wa[t, sl, other] == 0)
            if k == 0:
                continue
            Q = Mb @ wi[:k].T
            if blocks == 1:
                target = Mb
            else:
                target = Mb / np.linalg.norm(M[t])
            assert np.abs(Q.conj().T @ Q - np.eye(k)).max() < tol * 10
            assert np.abs(Q @ wa[:k] - target).max() < tol
    eng.close()


@pytest.mark.parametrize("dtype,n,cap", [("c128", 64, 10), ("c64", 64, 10), ("c64", 128, 64), ("c64", 40, 33)])
def test_eigh_truncation_cap(dtype, n, cap):
    # the cap binds (Sec. IV.A: keep the largest Schmidt values): the factors
    # reproduce numpy's best rank-cap approximation, renormalised; complex64
    # factors carry their storage rounding (the eigen-decomposition is FP64)
    from paper_2511_05719_amd._abi import lib, check
    g = np.random.default_rng(3 + n + cap)
    rows, m = 3, 3 * n
    M = g.normal(size=(rows, m, n)) + 1j * g.normal(size=(rows, m, n))
    M *= (10.0 ** (-np.arange(n) / 40.0))[None, None, :]
    M /= np.linalg.norm(M.reshape(rows, -1), axis=1)[:, None, None]
    G = np.einsum("tmi,tmj->tij", M.conj(), M)
    eng = _engine(dtype)
    Gd = _dev_gram(G)
    wdt = torch.float64 if dtype == "c128" else torch.float32
    Wi = torch.zeros(rows, cap, n, 2, dtype=wdt, device="cuda")
    Wa = torch.zeros(rows, cap, n, 2, dtype=wdt, device="cuda")
    rk = torch.zeros(rows, dtype=torch.int32, device="cuda")
    check(lib().ttn_test_eigh(eng._ctx, rows, n, cap, cap, 1e-10, Gd.data_ptr(), rows * n * n, Wi.data_ptr(),
                              Wa.data_ptr(), rows * cap * n, rk.data_ptr(), None, 1), eng._ctx)
    Wi, Wa = _host_complex(Wi), _host_complex(Wa)
    assert (rk.cpu().numpy() == cap).all()
    tol = 1e-10 if dtype == "c128" else 2e-6
    for t in range(rows):
        u, s, vh = np.linalg.svd(M[t])
        best = (u[:, :cap] * s[:cap]) @ vh[:cap]
        best /= np.linalg.norm(best)
        got = (M[t] @ Wi[t].T) @ Wa[t]                        # renormalised rank-cap truncation
        assert np.abs(got - best).max() < tol, (t, np.abs(got - best).max())
    eng.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("m", [20, 40, 100, 128])
def test_eigh_block_diagonal(dtype, m):
    # a controlled gate's bond: G = diag(G0, G1), each half solved apart
    # (m <= 64: vectors in LDS; m > 64: rotation log and replay per block);
    # the cutoff refers to the whole trace, the normalisation is the trace's
    from paper_2511_05719_amd._abi import lib, check
    g = np.random.default_rng(m)
    rows, K, n = 3, 3 * m, 2 * m
    Ms = []
    for b in range(2):
        rank = m if b == 0 else max(1, m // 3)
        Mb = (g.normal(size=(rows, K, rank)) + 1j * g.normal(size=(rows, K, rank))) @ \
             (g.normal(size=(rows, rank, m)) + 1j * g.normal(size=(rows, rank, m)))
        Mb *= (10.0 ** (-np.arange(m) / 15.0))[None, None, :]
        Ms.append(Mb * (0.8 if b == 0 else 0.3))
    tot = sum(np.linalg.norm(x.reshape(rows, -1), axis=1) ** 2 for x in Ms)
    Ms = [x / np.sqrt(tot)[:, None, None] for x in Ms]
    G = np.zeros((rows, n, n), complex)
    G[:, :m, :m] = np.einsum("tki,tkj->tij", Ms[0].conj(), Ms[0])
    G[:, m:, m:] = np.einsum("tki,tkj->tij", Ms[1].conj(), Ms[1])
    eng = _engine(dtype, chi=128 if n > 128 else 64)
    Gd = _dev_gram(G)
    wdt = torch.float64 if dtype == "c128" else torch.float32
    Wi = torch.full((rows, n, n, 2), 7.0, dtype=wdt, device="cuda")
    Wa = torch.full((rows, n, n, 2), 7.0, dtype=wdt, device="cuda")
    cutoff = 1e-12
    check(lib().ttn_test_eigh(eng._ctx, rows, n, n, m, cutoff, Gd.data_ptr(), rows * n * n, Wi.data_ptr(),
                              Wa.data_ptr(), rows * n * n, None, None, 2), eng._ctx)
    Wi, Wa = _host_complex(Wi), _host_complex(Wa)
    tol = 1e-9 if dtype == "c128" else 3e-5
    for t in range(rows):
        for b in range(2):
            Mb = Ms[b][t]
            s = np.linalg.svd(Mb, compute_uv=False)
            k_lo, k_hi = _kept_band(s ** 2, cutoff, dtype)     # the trace is 1
            rws = slice(b * m, (b + 1) * m)
            own = slice(b * m, (b + 1) * m)
            other = slice((1 - b) * m, (2 - b) * m)
            assert np.all(Wi[t, rws, other] == 0) and np.all(Wa[t, rws, other] == 0)
            wi, wa = Wi[t, rws, own], Wa[t, rws, own]
            k = int(np.sum(np.linalg.norm(wa, axis=1) > 0))
            assert k_lo <= k <= k_hi, (b, k, k_lo, k_hi)
            assert np.all(wi[k:] == 0) and np.all(wa[k:] == 0)
            u_, s_, vh_ = np.linalg.svd(Mb, full_matrices=False)
            Mk = (u_[:, :k] * s_[:k]) @ vh_[:k]
            U = Mb @ wi[:k].T
            assert np.abs(U @ wa[:k] - Mk).max() < tol * max(1.0, s[0])
            assert np.abs(np.linalg.norm(wa[:k], axis=1) - s[:k]).max() < tol * s[0]
    eng.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("m", [1, 8, 32])
def test_eigh_degenerate_diagonal_converges(dtype, m):
    # A Gram matrix whose diagonal is exactly degenerate and whose large
    # entries sit beside noise-sized ones (the stabilizer-state Gram matrices
    # of complex64 runs, where the noise is the storage rounding): the
    # noise-driven rotations turn by 45 degrees and move the large entries
    # around within a sweep, so convergence must be judged on the whole
    # matrix after the sweep.  G = A (x) I_m + E with A = [[1,0,1,0],
    # [0,1,0,-1], [1,0,1,0], [0,-1,0,1]] / 4 (eigenvalues 1/2, 1/2, 0, 0), E
    # Hermitian of size ~3e-8; the cap keeps the 2m values near 1/2.
    from paper_2511_05719_amd._abi import lib, check
    g = np.random.default_rng(m)
    A = np.array([[1, 0, 1, 0], [0, 1, 0, -1], [1, 0, 1, 0], [0, -1, 0, 1]], float) / 4
    n, cap, rows = 4 * m, 2 * m, 3
    G = np.zeros((rows, n, n), complex)
    for t in range(rows):
        E = 3e-8 * (g.normal(size=(n, n)) + (1j * g.normal(size=(n, n)) if t == 2 else 0))
        E = (E + E.conj().T) / 2
        np.fill_diagonal(E, 0.0)
        G[t] = np.kron(A, np.eye(m)) + E
    eng = _engine(dtype, chi=128)
    Gd = _dev_gram(G)
    wdt = torch.float64 if dtype == "c128" else torch.float32
    Wi = torch.zeros(rows, cap, n, 2, dtype=wdt, device="cuda")
    Wa = torch.zeros(rows, cap, n, 2, dtype=wdt, device="cuda")
    rk = torch.zeros(rows, dtype=torch.int32, device="cuda")
    check(lib().ttn_test_eigh(eng._ctx, rows, n, cap, cap, 1e-10, Gd.data_ptr(), rows * n * n, Wi.data_ptr(),
                              Wa.data_ptr(), rows * cap * n, rk.data_ptr(), None, 1), eng._ctx)
    Wi, Wa = _host_complex(Wi), _host_complex(Wa)
    assert (rk.cpu().numpy() == cap).all()
    tol = 1e-9 if dtype == "c128" else 1e-5
    for t in range(rows):
        w, v = np.linalg.eigh(G[t])
        P = v[:, -cap:] @ v[:, -cap:].conj().T                # the kept eigenspace
        Gk = P @ G[t] @ P
        iso = Wi[t].conj() @ G[t] @ Wi[t].T
        assert np.abs(iso - np.eye(cap)).max() < tol, t
        rec = Wa[t].conj().T @ Wa[t] * np.trace(Gk).real     # W_abs is renormalised by the kept weight
        assert np.abs(rec - Gk).max() < tol, (t, np.abs(rec - Gk).max())
    eng.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_exact_move_try_leaves_wide_rows_to_the_eigensolver(dtype):
    # 65..128 columns without blocks: the pivoted Cholesky is the batch
    # driver's try before a truncating eigen-decomposition; rows whose rank
    # at the cutoff exceeds the cap report -1 and leave W untouched, the
    # others get exact factors (rank at the cutoff <= cap)
    from paper_2511_05719_amd._abi import lib, check
    g = np.random.default_rng(11)
    rows, n, cap, K = 4, 96, 40, 200
    ranks = [30, 40, 41, 70]
    M = np.zeros((rows, K, n), complex)
    for t, r in enumerate(ranks):
        M[t] = (g.normal(size=(K, r)) + 1j * g.normal(size=(K, r))) @ (g.normal(size=(r, n)) + 1j * g.normal(size=(r, n)))
        M[t] /= np.linalg.norm(M[t])
    G = np.einsum("tki,tkj->tij", M.conj(), M)
    eng = _engine(dtype, chi=128)
    Gd = _dev_gram(G)
    wdt = torch.float64 if dtype == "c128" else torch.float32
    Wi = torch.full((rows, cap, n, 2), 7.0, dtype=wdt, device="cuda")
    Wa = torch.full((rows, cap, n, 2), 7.0, dtype=wdt, device="cuda")
    rk = torch.full((rows,), -2, dtype=torch.int32, device="cuda")
    check(lib().ttn_test_move(eng._ctx, rows, n, cap, cap, 1e-10, Gd.data_ptr(), rows * n * n, Wi.data_ptr(),
                              Wa.data_ptr(), rows * cap * n, rk.data_ptr(), 1), eng._ctx)
    Wi, Wa, rk = _host_complex(Wi), _host_complex(Wa), rk.cpu().numpy()
    tol = 1e-9 if dtype == "c128" else 3e-5
    for t, r in enumerate(ranks):
        if r > cap:
            assert rk[t] == -1 and np.all(Wi[t] == 7 + 7j) and np.all(Wa[t] == 7 + 7j), t
            continue
        assert rk[t] == r, (t, rk[t])
        Q = M[t] @ Wi[t, :r].T
        assert np.abs(Q.conj().T @ Q - np.eye(r)).max() < 10 * tol
        assert np.abs(Q @ Wa[t, :r] - M[t]).max() < tol
        assert np.all(Wi[t, r:] == 0) and np.all(Wa[t, r:] == 0)
    eng.close()
