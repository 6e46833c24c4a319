"""Adjoint gradient of log P (ttn_log_prob_grad) against the oracle's exact
derivatives (shift rules, oracle/gradient.py) on untruncated runs, through
the C ABI."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workload import build_circuit, custom_circuit  # noqa: E402
from oracle import gradient  # noqa: E402
from oracle import statevector as sv  # noqa: E402

# "Untruncated" runs keep Schmidt weights above 1e-15 of a bond's weight, the
# rounding floor of the FP64 Gram route, so amplitudes are resolved to about
# sqrt(1e-15) ~ 3e-8 of the norm.  Probabilities are quadratic in the
# amplitudes, but a later projection onto a rare outcome divides by its
# probability, and the overlaps <lambda|N|psi> that the gradient is built from
# are linear in them; hence the complex128 tolerances: log P 1e-7, gradient
# 1e-6 relative (the oracle's values are exact to ~1e-13).
CUT_EXACT = 1e-15
TOL_C128 = {"logp": 1e-7, "grad": 1e-6}


def _engine(circ, rows, dtype="c128", chi=64, cutoff=CUT_EXACT, seed=0):
    from paper_2511_05719_amd import TTNEngine
    return TTNEngine(circ.n_qubits, rows, circ.leaf_of_qubit, chi_max=chi, cutoff=cutoff, dtype=dtype, seed=seed)


def _program(nq, layers, g, meas_p=0.35):
    prog = [("init", q, int(g.integers(2))) for q in range(nq)]
    for _ in range(layers):
        perm = g.permutation(nq)
        for i in range(0, nq - 1, 2):
            a, b = int(perm[i]), int(perm[i + 1])
            prog += [("cnot", a, b)]
        prog += [("srxad", q) for q in range(nq)]
        if g.random() < meas_p:
            q = int(g.integers(nq))
            prog += [("meas", q, int(g.integers(2))), ("init", q, int(g.integers(2))), ("srxad", q)]
    prog += [("meas", q, 0) for q in range(nq)]
    return prog


def _oracle_grads(circ, th, ga, recs, brs):
    out = [gradient.log_prob_grad(circ, th[r], ga[r], recs[r], brs[r] if circ.n_ad else None)
           for r in range(recs.shape[0])]
    return (np.array([o[0] for o in out]), np.stack([o[1] for o in out]), np.stack([o[2] for o in out]))


def _compare(circ, rows, dtype, seed, tol, th=None, ga=None):
    g = np.random.default_rng(seed)
    if th is None:
        th = g.uniform(0.05, 0.5, (rows, circ.n_loc))
    if ga is None:
        ga = g.uniform(0.005, 0.08, (rows, circ.n_loc))
    ref = sv.run(circ, th, ga, seed, np.arange(rows))
    eng = _engine(circ, rows, dtype, seed=seed)
    lp, dth, dga, st = eng.log_prob_grad(eng.upload(circ), ref.records, ref.branches, theta=th, gamma=ga)
    assert st["flagged_rows"] == 0
    lp0, dth0, dga0 = _oracle_grads(circ, th, ga, ref.records, ref.branches)
    lp, dth, dga = lp.cpu().numpy(), dth.cpu().numpy(), dga.cpu().numpy()
    assert np.abs(lp - lp0).max() < tol["logp"]
    scale_t = np.maximum(1.0, np.abs(dth0))
    scale_g = np.maximum(1.0, np.abs(dga0))
    assert np.max(np.abs(dth - dth0) / scale_t) < tol["grad"], np.max(np.abs(dth - dth0) / scale_t)
    assert np.max(np.abs(dga - dga0) / scale_g) < tol["grad"], np.max(np.abs(dga - dga0) / scale_g)
    eng.close()
    return st


@pytest.mark.parametrize("seed,nq,layers", [(0, 4, 4), (1, 6, 5), (2, 7, 6), (3, 9, 5)])
def test_random_circuit_gradient_c128(seed, nq, layers):
    g = np.random.default_rng(100 + seed)
    circ = custom_circuit(nq, _program(nq, layers, g))
    _compare(circ, 3, "c128", seed, TOL_C128)


def test_block_moves_gradient_c128():
    # 14 qubits: controlled gates across the root bond ride 128-wide bonds
    # solved as two diagonal blocks, in both the state and the adjoint tree
    g = np.random.default_rng(41)
    nq = 14
    circ = custom_circuit(nq, _program(nq, 4, g, meas_p=0.5))
    st = _compare(circ, 2, "c128", 4, TOL_C128)
    assert st["block_hops"] > 0


def test_colour_code_d3_gradient_c128_and_c64():
    # d=3 colour code, one round, SRX theta = 0.1 and AD gamma = 5e-3 at
    # every location (the differentiation workload's parameters at d=3)
    circ = build_circuit(3, 1, "srx+ad")
    rows = 6
    th = np.full((rows, circ.n_loc), 0.1)
    ga = np.full((rows, circ.n_loc), 5e-3)
    _compare(circ, rows, "c128", 9, TOL_C128, th, ga)
    _compare(circ, rows, "c64", 9, {"logp": 1e-4, "grad": 2e-3}, th, ga)


def test_per_row_parameters_and_shared_parameters_agree():
    circ = build_circuit(3, 1, "srx+ad")
    rows = 4
    ref = sv.run(circ, 0.12, 4e-3, 2, np.arange(rows))
    eng = _engine(circ, rows, "c128")
    ol = eng.upload(circ)
    a = eng.log_prob_grad(ol, ref.records, ref.branches, theta=0.12, gamma=4e-3)
    b = eng.log_prob_grad(ol, ref.records, ref.branches, theta=np.full((rows, circ.n_loc), 0.12),
                          gamma=np.full((rows, circ.n_loc), 4e-3))
    for x, y in zip(a[:3], b[:3]):
        assert np.allclose(x.cpu().numpy(), y.cpu().numpy(), rtol=1e-12, atol=1e-12)
    eng.close()


def test_twirled_op_list_is_rejected():
    from paper_2511_05719_amd._abi import TTNError
    circ = build_circuit(3, 1, "pta_srx")
    rows = 2
    eng = _engine(circ, rows)
    rec = np.zeros((rows, circ.n_rec), np.uint8)
    with pytest.raises(TTNError):
        eng.log_prob_grad(eng.upload(circ), rec, None, theta=0.1, gamma=0.0)
    eng.close()


def test_d5_gradient_matches_central_differences():
    # d=5 colour code (37 qubits), one round, amplitude damping gamma = 5e-3
    # at every location, clustered layout: the exact bond dimension (32) is
    # within chi_max = 64, so the run is untruncated and the adjoint must
    # equal central differences (step 1e-4) of the engine's own complex128
    # log P.  (With SRX added the state needs more than 64 Schmidt values at
    # d=5, the log P being differentiated is then a truncated one, and the
    # theta derivatives are checked against the oracle at d=3 instead.)
    circ = build_circuit(5, 1, "ad", leaf_of_qubit="optimized")
    rows = 8
    eng = _engine(circ, rows, "c128", seed=4)
    ol = eng.upload(circ)
    res = eng.run_circuit(ol, theta=0.0, gamma=5e-3)
    assert abs(res.stats["discarded_weight"]) < 1e-12 * rows
    rec, br = res.records.clone(), res.branches.clone()
    lp, dth, dga, st = eng.log_prob_grad(ol, rec, br, theta=0.0, gamma=5e-3)
    assert st["flagged_rows"] == 0
    assert np.abs(lp.cpu().numpy() - res.logp.cpu().numpy()).max() < 1e-9
    dga = dga.cpu().numpy()
    h = 1e-4
    g = np.random.default_rng(17)
    for l in g.choice(circ.n_loc, 6, replace=False):
        ga = np.full((rows, circ.n_loc), 5e-3)
        ga[:, l] += h
        lpp, _ = eng.log_prob(ol, rec, br, theta=0.0, gamma=ga)
        ga[:, l] -= 2 * h
        lpm, _ = eng.log_prob(ol, rec, br, theta=0.0, gamma=ga)
        fd = ((lpp - lpm) / (2 * h)).cpu().numpy()
        # central-difference error (h^2 times the third derivative) plus the
        # rounding of log P divided by h
        err = np.max(np.abs(fd - dga[:, l]) / np.maximum(1.0, np.abs(dga[:, l])))
        assert err < 1e-6, (l, fd, dga[:, l])
    eng.close()
