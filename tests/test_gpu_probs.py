"""Every sampled probability of the HIP engine against the FP64 oracle, draw by
draw (through the C ABI's probability trace): the Born probability of each
measurement outcome, the jump / no-jump probability of each amplitude-damping
location (Sec. III.C, Eq. 2-3) and the probability of each twirled Pauli
(Eq. 9), on the same random streams, compared on the rows whose sampled
events agree with the oracle's (complex64 rows may take another branch where
a draw lands within the complex64 rounding of a probability; their share is
bounded at 1%).  Also the paper-literal Trotterised AD reading (ad_mode
trotter) against the oracle's.

Tolerances (absolute, per probability), from the arithmetic:
* complex128 with no cutoff (every non-zero Gram eigenvalue kept): the FP64
  Gram route resolves a bond's squared Schmidt weights to ~1e-16 of its total,
  so a probability carries ~1e-12..1e-11 after a few hundred centre moves
  (config 1: 1e-12; the 3-round AD circuit: 2e-11).  Wide Schmidt spectra
  (damping up to 0.3) lose more: the Gram route gives a Schmidt value s a
  relative accuracy of ~1e-16 s_max^2 / s^2, so there 99.9% of the
  probabilities agree to 1e-12 and all to 1e-9.  Any cutoff w > 0 drops
  weights whose amplitude sqrt(w) can interfere with kept ones: at the
  rounding-floor cutoff 1e-15 probabilities move by up to ~4e-10, which is
  why these comparisons keep everything.
* complex64: every tensor entry is stored with relative rounding 2^-24 and
  every contraction accumulates in FP32; the rounding is amplified where a
  measurement or jump renormalises onto a small component, and it adds up
  over the trajectory's centre moves (the eigen-decompositions are FP64 and
  their precision does not move these figures).  On the config-2 workload
  99.9% of the probabilities agree to 1e-6 and all to 1e-5; on random
  circuits with large angles and damping (theta up to 0.6, gamma up to 0.3)
  99.9% agree to 1e-5 and all to 1e-4."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workload import build_circuit, custom_circuit, random_program  # noqa: E402
from oracle import statevector as sv  # noqa: E402

CUT_EXACT = 1e-15
GAMMAS = (1e-3, 2e-3, 5e-3, 1e-2)


def _engine(circ, rows, dtype="c128", chi=64, cutoff=None, seed=0, ad_mode="kraus"):
    from paper_2511_05719_amd import TTNEngine
    if cutoff is None:
        cutoff = CUT_EXACT if dtype == "c128" else 1e-10
    return TTNEngine(circ.n_qubits, rows, circ.leaf_of_qubit, chi_max=chi, cutoff=cutoff, dtype=dtype,
                     seed=seed, ad_mode=ad_mode)


def _traced_run(eng, circ, theta, gamma, traj_offset=0):
    probs = torch.full((eng.batch, max(circ.n_draws, 1)), float("nan"), dtype=torch.float64, device=eng.device)
    eng.trace_probs(probs)
    res = eng.run_circuit(eng.upload(circ), theta=theta, gamma=gamma, traj_offset=traj_offset)
    eng.trace_probs(None)
    torch.cuda.synchronize()
    return res, probs.cpu().numpy()[:, :circ.n_draws]


def _compare(res, probs, ref, tol, max_diverged, tol999=None):
    """tol bounds every probability; tol999 (if given) their 99.9th percentile."""
    rec, br = res.records.cpu().numpy(), res.branches.cpu().numpy()
    same = np.all(rec == ref.records, axis=1)
    if ref.branches.shape[1]:
        same &= np.all(br == ref.branches, axis=1)
    assert 1.0 - same.mean() <= max_diverged, 1.0 - same.mean()
    a, b = probs[same], ref.probs[same]
    assert np.array_equal(np.isnan(a), np.isnan(b))
    ok = ~np.isnan(b)
    errs = np.abs(a[ok] - b[ok])
    err = errs.max() if errs.size else 0.0
    print(f"probabilities: {errs.size}, max error {err:.2e}, 99.9th percentile "
          f"{np.quantile(errs, 0.999) if errs.size else 0.0:.2e}, rows diverged {1.0 - same.mean():.4f}")
    assert err < tol, err
    if tol999 is not None:
        assert np.quantile(errs, 0.999) < tol999, np.quantile(errs, 0.999)
    return same, err


def test_config1_every_born_probability():
    # d=3, 1 round, SRX theta = 0.05, complex128, untruncated, 1000 rows, seed 0
    circ = build_circuit(3, 1, "srx")
    rows = 1000
    eng = _engine(circ, rows, "c128", seed=0)
    res, probs = _traced_run(eng, circ, 0.05, 0.0)
    ref = sv.run(circ, 0.05, 0.0, 0, np.arange(rows))
    same, err = _compare(res, probs, ref, 1e-12, 0.0)
    assert np.isfinite(probs).all()               # every op of this list with a draw is a measurement
    eng.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_config2_every_born_and_kraus_probability(dtype):
    # d=3, 3 rounds, AD at every location, the four damping strengths over the
    # rows (one launch), seed 1: 25 Born + 265 jump probabilities per row
    circ = build_circuit(3, 3, "ad")
    rows = 512
    ga = np.repeat(np.asarray(GAMMAS)[np.arange(rows) % 4][:, None], circ.n_loc, axis=1)
    eng = _engine(circ, rows, dtype, seed=1, cutoff=0.0 if dtype == "c128" else 1e-10)
    res, probs = _traced_run(eng, circ, 0.0, ga, traj_offset=7)
    ref = sv.run(circ, 0.0, ga, 1, np.arange(7, 7 + rows))
    if dtype == "c128":
        same, err = _compare(res, probs, ref, 2e-11, 0.0)
    else:
        same, err = _compare(res, probs, ref, 1e-5, 0.01, tol999=1e-6)
    assert np.abs(res.logp.cpu().numpy()[same] - ref.logp[same]).max() < (1e-10 if dtype == "c128" else 1e-4)
    eng.close()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_circuits_every_probability_c64(seed):
    # random 8-12 qubit circuits with SRX + AD after every gate and
    # mid-circuit measurements in both bases, per-row parameters, complex64
    g = np.random.default_rng(40 + seed)
    nq = [8, 10, 12][seed]
    prog = random_program(nq, 12, g, noise=("srxad",), measure_every=4)
    circ = custom_circuit(nq, prog)
    rows = 256
    th = g.uniform(0.05, 0.6, (rows, circ.n_loc))
    ga = g.uniform(0.005, 0.1, (rows, circ.n_loc))
    eng = _engine(circ, rows, "c64", seed=seed)
    res, probs = _traced_run(eng, circ, th, ga)
    ref = sv.run(circ, th, ga, seed, np.arange(rows))
    _compare(res, probs, ref, 1e-4, 0.01, tol999=1e-5)
    eng.close()


def test_twirled_probabilities():
    # the twirled twins (Eq. 9): the probability of the Pauli each draw picks
    circ = build_circuit(3, 2, "pta_srx+ad")
    rows = 256
    eng = _engine(circ, rows, "c128", seed=6)
    res, probs = _traced_run(eng, circ, 0.3, 0.2)
    ref = sv.run(circ, 0.3, 0.2, 6, np.arange(rows))
    _compare(res, probs, ref, 1e-12, 0.0)
    eng.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_trotter_ad_reading_matches_oracle(dtype):
    # ad_mode trotter: the no-jump branch evolves by diag(1, e^{-gamma/2})
    # (Sec. III.C); records, branches, log P and every probability equal the
    # oracle's with the same reading, and differ from the exact-Kraus run
    circ = build_circuit(3, 2, "srx+ad")
    rows = 256
    g = np.random.default_rng(9)
    th = g.uniform(0.05, 0.3, (rows, circ.n_loc))
    ga = g.uniform(0.05, 0.3, (rows, circ.n_loc))
    eng = _engine(circ, rows, dtype, seed=2, ad_mode="trotter", cutoff=0.0 if dtype == "c128" else 1e-10)
    res, probs = _traced_run(eng, circ, th, ga)
    ref = sv.run(circ, th, ga, 2, np.arange(rows), ad_mode="trotter")
    if dtype == "c128":
        same, _ = _compare(res, probs, ref, 1e-9, 0.0, tol999=1e-12)
    else:
        same, _ = _compare(res, probs, ref, 1e-4, 0.01, tol999=1e-5)
    assert np.abs(res.logp.cpu().numpy()[same] - ref.logp[same]).max() < (1e-8 if dtype == "c128" else 1e-3)
    kraus = sv.run(circ, th, ga, 2, np.arange(rows))
    assert np.abs(kraus.logp - ref.logp).max() > 1e-6
    eng.close()


def test_trace_arguments_are_checked():
    from paper_2511_05719_amd import TTNError
    circ = build_circuit(3, 1, "srx")
    eng = _engine(circ, 4, "c128")
    narrow = torch.zeros(4, circ.n_draws - 1, dtype=torch.float64, device="cuda")
    eng.trace_probs(narrow)
    with pytest.raises(TTNError):
        eng.run_circuit(eng.upload(circ), theta=0.05, gamma=0.0)
    eng.trace_probs(None)
    eng.run_circuit(eng.upload(circ), theta=0.05, gamma=0.0)
    with pytest.raises(ValueError):
        eng.trace_probs(torch.zeros(3, circ.n_draws, dtype=torch.float64, device="cuda"))
    eng.close()
