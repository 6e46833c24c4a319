"""Circuit-level parity of the HIP engine with the FP64 oracle (through the
C ABI).  Untruncated runs must reproduce the oracle's amplitudes, sampled
records, Kraus branches and log P; truncated runs are compared where the
result is unique (see the tolerance notes in each test)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workload import build_circuit, custom_circuit, random_program  # noqa: E402
from oracle import chp, decoder, stabrank  # noqa: E402
from oracle import statevector as sv  # noqa: E402

# The FP64 Gram route resolves squared Schmidt weights down to its rounding
# floor (~1e-16 of the bond's weight for these sizes); "untruncated" runs
# drop only weights below this cutoff, i.e. numerical zeros.
CUT_EXACT = 1e-15


def _engine(circ, rows, dtype="c128", chi=64, cutoff=CUT_EXACT, seed=0):
    from paper_2511_05719_amd import TTNEngine
    return TTNEngine(circ.n_qubits, rows, circ.leaf_of_qubit, chi_max=chi, cutoff=cutoff, dtype=dtype, seed=seed)


def _amp_tol(dtype, disc):
    # truncation error (sqrt of the discarded weight) plus arithmetic rounding
    return np.sqrt(max(disc, 0.0)) + (1e-10 if dtype == "c128" else 1e-5)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_random_circuit_amplitudes(dtype, seed):
    g = np.random.default_rng(seed)
    nq = [6, 9, 11, 13][seed]
    prog = [p for p in random_program(nq, 10, g, noise=("srx",), measure_every=4) if p[0] != "meas" or True]
    prog = prog[:-nq]                      # drop the final measurements: compare the state
    circ = custom_circuit(nq, prog)
    rows = 3
    th = g.uniform(0.05, 0.8, (rows, circ.n_loc))
    eng = _engine(circ, rows, dtype, seed=seed)
    res = eng.run_circuit(eng.upload(circ), theta=th, gamma=0.0)
    torch.cuda.synchronize()
    ref_res, st = sv.run(circ, th, 0.0, seed, np.arange(rows), stop_after_op=circ.n_ops - 1)
    full = st.full_state(nq)
    if circ.n_rec:
        assert np.array_equal(res.records.cpu().numpy(), ref_res.records)
    tol = _amp_tol(dtype, res.stats["discarded_weight"])
    for r in range(rows):
        amp = eng.statevector(r)
        assert np.abs(amp - full[r]).max() < tol, (r, np.abs(amp - full[r]).max())
    assert np.allclose(res.logp.cpu().numpy(), ref_res.logp, atol=1e-9 if dtype == "c128" else 1e-5)
    eng.close()


def test_config1_per_shot_records():
    # d=3 colour code, 13 qubits, 1 round, SRX theta=0.05 at every location,
    # complex128, untruncated, 1000 trajectories, seed 0
    circ = build_circuit(3, 1, "srx")
    rows = 1000
    eng = _engine(circ, rows, "c128", seed=0)
    res = eng.run_circuit(eng.upload(circ), theta=0.05, gamma=0.0)
    ref = sv.run(circ, 0.05, 0.0, 0, np.arange(rows))
    rec = res.records.cpu().numpy()
    assert np.array_equal(rec, ref.records)
    assert np.abs(res.logp.cpu().numpy() - ref.logp).max() < 1e-9
    assert res.stats["flagged_rows"] == 0
    fail = eng.decode(res.records, circ.data_rec, circ.code.checks).cpu().numpy()
    assert np.array_equal(fail, decoder.decode_fail(circ.code.checks, ref.records[:, circ.data_rec]))
    eng.close()


@pytest.mark.parametrize("gamma", [1e-2, 0.2])
def test_config2_ad_records_and_branches(gamma):
    # d=3, 3 rounds, amplitude damping on every location (exact Kraus unravelling)
    circ = build_circuit(3, 3, "ad")
    rows = 128
    eng = _engine(circ, rows, "c128", seed=1)
    res = eng.run_circuit(eng.upload(circ), theta=0.0, gamma=gamma, traj_offset=40)
    ref = sv.run(circ, 0.0, gamma, 1, np.arange(40, 40 + rows))
    assert np.array_equal(res.records.cpu().numpy(), ref.records)
    assert np.array_equal(res.branches.cpu().numpy(), ref.branches)
    assert np.abs(res.logp.cpu().numpy() - ref.logp).max() < 1e-9
    eng.close()


def test_combined_channel_per_row_parameters():
    circ = build_circuit(3, 2, "srx+ad")
    rows = 64
    g = np.random.default_rng(7)
    th = g.uniform(0.02, 0.3, (rows, circ.n_loc))
    ga = g.uniform(1e-3, 5e-2, (rows, circ.n_loc))
    eng = _engine(circ, rows, "c128", seed=3)
    res = eng.run_circuit(eng.upload(circ), theta=th, gamma=ga)
    ref = sv.run(circ, th, ga, 3, np.arange(rows))
    assert np.array_equal(res.records.cpu().numpy(), ref.records)
    assert np.array_equal(res.branches.cpu().numpy(), ref.branches)
    assert np.abs(res.logp.cpu().numpy() - ref.logp).max() < 1e-8
    eng.close()


@pytest.mark.parametrize("channel,theta,gamma", [("pta_srx", 0.3, 0.0), ("pta_ad", 0.0, 0.3), ("none", 0.0, 0.0)])
def test_twirled_limit_matches_stabilizer_simulation(channel, theta, gamma):
    circ = build_circuit(3, 2, channel)
    rows = 128
    eng = _engine(circ, rows, "c128", seed=4)
    res = eng.run_circuit(eng.upload(circ), theta=theta, gamma=gamma)
    recs, _ = chp.run(circ, theta, gamma, 4, np.arange(rows))
    assert np.array_equal(res.records.cpu().numpy(), recs)
    if channel == "none":
        assert np.allclose(res.logp.cpu().numpy(), -2 * circ.code.n_plaq * np.log(2.0), atol=1e-10)
    eng.close()


def test_bond_dims_equal_stabilizer_ranks():
    g = np.random.default_rng(11)
    nq = 12
    prog = random_program(nq, 8, g, noise=("pauli_srx",), measure_every=3)[:-nq]
    circ = custom_circuit(nq, prog)
    th = np.full(circ.n_loc, 0.9)
    rows = 4
    eng = _engine(circ, rows, "c128", seed=2)
    eng.run_circuit(eng.upload(circ), theta=th, gamma=0.0)
    eng.compress()
    recs, tab = chp.run(circ, th, 0.0, 2, np.arange(rows))
    for r in range(rows):
        one = chp.run(circ, th, 0.0, 2, np.arange(r, r + 1))[1]
        want = stabrank.tree_bond_ranks(one.stabilizers(), circ.leaf_of_qubit, circ.n_leaves)
        got = eng.bond_dims(r)
        for node, rank in want.items():
            assert got[node] == rank, (r, node, got[node], rank)
    eng.close()


def test_c64_matches_c128_records_mostly():
    circ = build_circuit(3, 1, "srx")
    rows = 512
    e1 = _engine(circ, rows, "c128", seed=0)
    r1 = e1.run_circuit(e1.upload(circ), theta=0.05, gamma=0.0)
    e2 = _engine(circ, rows, "c64", cutoff=1e-10, seed=0)
    r2 = e2.run_circuit(e2.upload(circ), theta=0.05, gamma=0.0)
    a, b = r1.records.cpu().numpy(), r2.records.cpu().numpy()
    diverged = np.any(a != b, axis=1).mean()
    assert diverged <= 0.01
    same = np.all(a == b, axis=1)
    assert np.abs(r1.logp.cpu().numpy()[same] - r2.logp.cpu().numpy()[same]).max() < 1e-4
    e1.close(); e2.close()


def test_log_prob_of_oracle_records():
    circ = build_circuit(3, 2, "srx+ad")
    rows = 32
    ref = sv.run(circ, 0.1, 5e-3, 9, np.arange(rows))
    eng = _engine(circ, rows, "c128", seed=0)
    lp, st = eng.log_prob(eng.upload(circ), ref.records, ref.branches, theta=0.1, gamma=5e-3)
    assert np.abs(lp.cpu().numpy() - ref.logp).max() < 1e-9
    eng.close()


def test_single_op_entry_points():
    from oracle import channels
    nq, rows = 5, 64
    circ = custom_circuit(nq, [("init", q, 1) for q in range(nq)] +
                          [("cnot", 0, 4), ("srx", 2), ("cnot", 2, 3), ("ad", 4), ("meas", 4, 0), ("meas", 0, 1)])
    eng = _engine(circ, rows, "c128", seed=8)
    eng.init_product([1] * nq)
    cn = np.eye(4)[[0, 1, 3, 2]]
    eng.apply_2q(0, 4, cn)
    eng.apply_1q(2, channels.srx_unitary(0.7))
    eng.apply_2q(2, 3, cn)
    k0, k1 = channels.ad_kraus(0.4)
    br, logp = eng.kraus_jump(4, k0, k1, draw=0)
    b1, logp = eng.measure(4, 0, draw=1, logp=logp)
    b2, logp = eng.measure(0, 1, draw=2, logp=logp)
    th = np.array([0.0, 0.7, 0.0]); ga = np.array([0.0, 0.0, 0.4])
    # the same program through the oracle (locations: srx -> loc 0 ... keep params aligned)
    circ2 = custom_circuit(nq, [("init", q, 1) for q in range(nq)] +
                           [("cnot", 0, 4), ("srx", 2), ("cnot", 2, 3), ("ad", 4), ("meas", 4, 0), ("meas", 0, 1)])
    ref = sv.run(circ2, np.array([0.7, 0.0]), np.array([0.0, 0.4]), 8, np.arange(rows))
    assert np.array_equal(br.cpu().numpy(), ref.branches[:, 0])
    assert np.array_equal(b1.cpu().numpy(), ref.records[:, 0])
    assert np.array_equal(b2.cpu().numpy(), ref.records[:, 1])
    assert np.abs(logp.cpu().numpy() - ref.logp).max() < 1e-10
    eng.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_block_diagonal_zip_moves(dtype):
    # 14 qubits on 16 leaves: the root bond (8 | 6 qubits) reaches 64, so a
    # controlled gate across it rides a 128-wide bond that is solved as two
    # diagonal blocks (block-split Gram, eigensolver and both contractions);
    # chi = 64 bounds every bond of this tree, so the run is untruncated.
    g = np.random.default_rng(21)
    nq = 14
    prog = random_program(nq, 14, g, noise=("srx",), measure_every=5)[:-nq]
    circ = custom_circuit(nq, prog)
    rows = 3
    th = g.uniform(0.1, 1.2, (rows, circ.n_loc))
    eng = _engine(circ, rows, dtype, seed=5)
    res = eng.run_circuit(eng.upload(circ), theta=th, gamma=0.0)
    assert res.stats["block_hops"] > 0
    ref_res, st = sv.run(circ, th, 0.0, 5, np.arange(rows), stop_after_op=circ.n_ops - 1)
    full = st.full_state(nq)
    if circ.n_rec:
        assert np.array_equal(res.records.cpu().numpy(), ref_res.records)
    tol = _amp_tol(dtype, res.stats["discarded_weight"])
    for r in range(rows):
        amp = eng.statevector(r)
        assert np.abs(amp - full[r]).max() < tol, (r, np.abs(amp - full[r]).max())
    eng.close()


def test_profile_ledger_bounded_by_executed_work():
    # the algorithmic flops ledgered from actual dimensions never exceed the
    # flops of the padded launches, and every hot class has a ledger
    circ = build_circuit(3, 1, "srx")
    rows = 64
    eng = _engine(circ, rows, "c64", cutoff=1e-10, seed=0)
    ol = eng.upload(circ)
    eng.profile(True)
    res = eng.run_circuit(ol, theta=0.05, gamma=0.0)
    prof = eng.profile_read()
    eng.profile(False)
    st = res.stats
    assert prof["gram"]["launches"] > 0 and prof["contract"]["launches"] > 0
    assert 0 < prof["gram"]["alg_flops"] <= st["gram_flops"] * (1 + 1e-12)
    assert 0 < prof["contract"]["alg_flops"] <= st["gemm_flops"] * (1 + 1e-12)
    assert prof["eigh_small"]["alg_flops"] + prof["eigh_large"]["alg_flops"] > 0
    assert all(v["ms"] >= 0 for v in prof.values())
    eng.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_chi128_random_circuit_amplitudes(dtype):
    # 15 qubits on 16 leaves with chi_max = 128: the root bond (8 | 7 qubits)
    # reaches 128, so a controlled gate across it rides a 256-wide bond:
    # forward moves solve two 128-wide diagonal blocks (rotation log and
    # replay per block), the truncating sweep back a dense 256-wide problem
    # (packed Gram matrix in device memory).  chi_max bounds no bond of this
    # tree, so the run is untruncated.
    g = np.random.default_rng(31)
    nq = 15
    prog = random_program(nq, 24, g, noise=("srx",), measure_every=8)[:-nq]
    circ = custom_circuit(nq, prog)
    rows = 2
    th = g.uniform(0.2, 1.4, (rows, circ.n_loc))
    eng = _engine(circ, rows, dtype, chi=128, seed=6)
    res = eng.run_circuit(eng.upload(circ), theta=th, gamma=0.0)
    assert res.stats["block_hops"] > 0
    assert res.stats["max_rank"] > 64
    ref_res, st = sv.run(circ, th, 0.0, 6, np.arange(rows), stop_after_op=circ.n_ops - 1)
    full = st.full_state(nq)
    if circ.n_rec:
        assert np.array_equal(res.records.cpu().numpy(), ref_res.records)
    tol = _amp_tol(dtype, res.stats["discarded_weight"])
    for r in range(rows):
        amp = eng.statevector(r)
        assert np.abs(amp - full[r]).max() < tol, (r, np.abs(amp - full[r]).max())
    eng.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_autotuned_tile_shapes_keep_parity(dtype):
    # d=3, 3 rounds, SRX + AD at per-row parameters, untruncated: with the
    # tile-shape tuner measuring every new GEMM shape (run 1), then reusing
    # its choices without measuring (run 2), records and Kraus branches equal
    # the oracle's and log P agrees; forgetting the choices returns to the
    # fixed rule
    circ = build_circuit(3, 3, "srx+ad")
    rows = 256
    g = np.random.default_rng(11)
    th = g.uniform(0.02, 0.3, (rows, circ.n_loc))
    ga = g.uniform(1e-3, 2e-2, (rows, circ.n_loc))
    ref = sv.run(circ, th, ga, 4, np.arange(rows))
    eng = _engine(circ, rows, dtype=dtype, seed=4)
    ol = eng.upload(circ)
    # complex64: log P sums ~300 log terms, each probability within ~1e-5
    tol = 1e-9 if dtype == "c128" else 1e-4
    for on in (True, False):
        eng.autotune(on)
        res = eng.run_circuit(ol, theta=th, gamma=ga)
        got, gbr, glp = res.records.cpu().numpy(), res.branches.cpu().numpy(), res.logp.cpu().numpy()
        same = np.all(got == ref.records, axis=1) & np.all(gbr == ref.branches, axis=1)
        if dtype == "c128":
            assert same.all()
        else:
            # complex64 rows may take another branch only where a draw lands
            # within the complex64 rounding of a probability
            assert same.mean() >= 0.99, same.mean()
        assert np.abs(glp[same] - ref.logp[same]).max() < tol
    shapes, changed = eng.autotune(False)
    assert shapes > 0 and 0 <= changed <= shapes
    assert eng.autotune(None) == (0, 0)
    eng.close()
