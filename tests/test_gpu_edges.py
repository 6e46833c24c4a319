"""Edge cases of the engine through the C ABI, against the FP64 oracle:
the smallest trees, a single trajectory (the plain path), a batch that is not
a multiple of the kernels' 256-row blocks, an empty op list, deterministic
outcomes and an impossible forced record."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workload import build_circuit, custom_circuit  # noqa: E402
from oracle import statevector as sv  # noqa: E402

CUT_EXACT = 1e-15


def _engine(circ, rows, dtype="c128", chi=64, cutoff=CUT_EXACT, seed=0):
    from paper_2511_05719_amd import TTNEngine
    return TTNEngine(circ.n_qubits, rows, circ.leaf_of_qubit, chi_max=chi, cutoff=cutoff, dtype=dtype, seed=seed)


@pytest.mark.parametrize("nq", [1, 2, 3])
def test_smallest_trees(nq):
    # one and two leaves per bottom node, the root itself a bottom node (N <= 2)
    prog = [("init", q, q % 2) for q in range(nq)]
    for q in range(nq):
        prog += [("srxad", q)]
    if nq > 1:
        prog += [("cnot", 0, nq - 1), ("srxad", 0), ("srxad", nq - 1)]
    prog += [("meas", q, q % 2) for q in range(nq)]
    circ = custom_circuit(nq, prog)
    rows = 64
    g = np.random.default_rng(nq)
    th = g.uniform(0.1, 1.5, (rows, circ.n_loc))
    ga = g.uniform(0.05, 0.4, (rows, circ.n_loc))
    eng = _engine(circ, rows, seed=nq)
    res = eng.run_circuit(eng.upload(circ), theta=th, gamma=ga)
    ref = sv.run(circ, th, ga, nq, np.arange(rows))
    assert np.array_equal(res.records.cpu().numpy(), ref.records)
    assert np.array_equal(res.branches.cpu().numpy(), ref.branches)
    assert np.abs(res.logp.cpu().numpy() - ref.logp).max() < 1e-10
    eng.close()


def test_single_trajectory_plain_path():
    # B = 1 in complex128: the plain path the batched runs are compared with
    circ = build_circuit(3, 1, "srx+ad")
    for tid in (0, 5, 17):
        eng = _engine(circ, 1, seed=0)
        res = eng.run_circuit(eng.upload(circ), theta=0.1, gamma=5e-3, traj_offset=tid)
        ref = sv.run(circ, 0.1, 5e-3, 0, np.arange(tid, tid + 1))
        assert np.array_equal(res.records.cpu().numpy(), ref.records)
        assert np.array_equal(res.branches.cpu().numpy(), ref.branches)
        assert abs(float(res.logp[0]) - ref.logp[0]) < 1e-9
        eng.close()


def test_batch_not_a_multiple_of_the_block():
    circ = build_circuit(3, 1, "srx")
    rows = 257
    eng = _engine(circ, rows, seed=0)
    res = eng.run_circuit(eng.upload(circ), theta=0.05, gamma=0.0, traj_offset=1000)
    ref = sv.run(circ, 0.05, 0.0, 0, np.arange(1000, 1000 + rows))
    assert np.array_equal(res.records.cpu().numpy(), ref.records)
    assert np.abs(res.logp.cpu().numpy() - ref.logp).max() < 1e-9
    eng.close()


def test_empty_op_list_keeps_the_product_state():
    circ = custom_circuit(5, [])
    rows = 3
    eng = _engine(circ, rows)
    res = eng.run_circuit(eng.upload(circ), theta=0.0, gamma=0.0)
    assert np.all(res.logp.cpu().numpy() == 0.0)
    for r in range(rows):
        amp = eng.statevector(r)
        want = np.zeros(2 ** 5, complex)
        want[0] = 1.0
        assert np.abs(amp - want).max() < 1e-14
    eng.close()


def test_deterministic_outcomes_cost_nothing():
    # |+> measured in X and |0> in Z: probability 1, log P = 0
    circ = custom_circuit(2, [("init", 0, 1), ("init", 1, 0), ("meas", 0, 1), ("meas", 1, 0)])
    eng = _engine(circ, 8)
    res = eng.run_circuit(eng.upload(circ), theta=0.0, gamma=0.0)
    assert np.all(res.records.cpu().numpy() == 0)
    assert np.abs(res.logp.cpu().numpy()).max() < 1e-14
    eng.close()


def test_impossible_forced_record_is_flagged():
    # noiseless d=3 circuit: the first round's Z syndromes are 0; forcing a 1
    # has probability 0, so log P = -inf and the row is flagged
    circ = build_circuit(3, 1, "none")
    rows = 4
    ref = sv.run(circ, 0.0, 0.0, 0, np.arange(rows))
    rec = ref.records.copy()
    rec[1, circ.zsyn_rec[0][0]] ^= 1
    eng = _engine(circ, rows)
    lp, st = eng.log_prob(eng.upload(circ), rec, None, theta=0.0, gamma=0.0)
    lp = lp.cpu().numpy()
    assert np.isneginf(lp[1])
    assert np.abs(np.delete(lp, 1) - np.delete(ref.logp, 1)).max() < 1e-10
    assert st["flagged_rows"] == 1
    eng.close()
