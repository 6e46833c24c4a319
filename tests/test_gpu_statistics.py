"""Logical error rates of batched trajectories against exact values and
between precisions and bond dimensions (through the C ABI).

Config 2 shape: d=3, 3 rounds, amplitude damping (Eq. 2-3) at every location,
gamma in {1e-3, 2e-3, 5e-3, 1e-2}, 10^4 trajectories per gamma in one batched
launch; complex64 (FP32 MFMA contractions, FP64 eigen-decompositions and
probabilities) and complex128.  The exact failure probability of the
final-data decoder comes from the oracle's density matrix
(tests/golden/config2_exact_pfail.json, written by make_config2_pfail.py):
each measured rate must lie inside its 99.9% binomial interval.

Config 3 shape: d=5, 5 rounds, SRX (Eq. 1), chi_max = 64, cutoff 1e-10,
clustered layout (App. B).  chi = 64 truncates some bonds (Sec. IV.A), and no
dense oracle exists at 28 live qubits, so the run is pinned by its own
convergence: complex64 against complex128 on the same random streams, and
chi_max = 64 against chi_max = 128, with failure rates inside each other's
binomial intervals and mean log P within five standard errors."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workload import build_circuit  # noqa: E402
from oracle import decoder  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
GAMMAS = (1e-3, 2e-3, 5e-3, 1e-2)
Z999 = 3.2905267314918945


def _run(circ, rows, dtype, theta, gamma, seed, chi=64, cutoff=1e-10, traj_offset=0):
    from paper_2511_05719_amd import TTNEngine
    eng = TTNEngine(circ.n_qubits, rows, circ.leaf_of_qubit, chi_max=chi, cutoff=cutoff, dtype=dtype, seed=seed)
    res = eng.run_circuit(eng.upload(circ), theta=theta, gamma=gamma, traj_offset=traj_offset)
    fail = eng.decode(res.records, circ.data_rec, circ.code.checks).cpu().numpy().astype(bool)
    out = (res.records.cpu().numpy(), res.branches.cpu().numpy(), res.logp.cpu().numpy(), fail, res.stats)
    eng.close()
    return out


def test_config2_failure_rates_match_density_matrix():
    with open(os.path.join(GOLDEN, "config2_exact_pfail.json")) as f:
        exact = {float(k): v for k, v in json.load(f)["p_fail"].items()}
    circ = build_circuit(3, 3, "ad")
    per = 10 ** 4
    rows = per * len(GAMMAS)
    gam = np.repeat(np.asarray(GAMMAS), per)
    ga = torch.as_tensor(np.repeat(gam[:, None], circ.n_loc, axis=1), device="cuda")
    runs = {dt: _run(circ, rows, dt, 0.0, ga, seed=1) for dt in ("c64", "c128")}
    for dt, (rec, br, lp, fail, st) in runs.items():
        assert st["flagged_rows"] == 0
        for j, g in enumerate(GAMMAS):
            k = int(fail[j * per:(j + 1) * per].sum())
            lo, hi = decoder.wilson_interval(k, per, Z999)
            print(f"{dt} gamma={g}: p_fail {k / per:.4f} in [{lo:.4f}, {hi:.4f}], exact {exact[g]:.4f}")
            assert lo <= exact[g] <= hi, (dt, g, k / per, exact[g])
    # the two precisions draw the same trajectories except where a draw
    # lands within complex64 rounding of a probability
    (r64, b64, l64, _, _), (r128, b128, l128, _, _) = runs["c64"], runs["c128"]
    same = np.all(r64 == r128, axis=1) & np.all(b64 == b128, axis=1)
    print(f"complex64 rows diverging from complex128: {1 - same.mean():.2e}")
    assert same.mean() >= 0.99
    # log P sums ~290 log terms with per-probability errors up to ~1e-5
    assert np.abs(l64[same] - l128[same]).max() < 1e-3


def _theta_rows(circ, thetas, rows):
    th = np.asarray(thetas)[np.arange(rows) % len(thetas)]
    return np.repeat(th[:, None], circ.n_loc, axis=1), th


def _agree(a, b, th, thetas, tag):
    (ra, _, la, fa, sa), (rb, _, lb, fb, sb) = a, b
    for t in thetas:
        m = th == t
        n = int(m.sum())
        ka, kb = int(fa[m].sum()), int(fb[m].sum())
        lo_a, hi_a = decoder.wilson_interval(ka, n)
        lo_b, hi_b = decoder.wilson_interval(kb, n)
        print(f"{tag} theta={t}: p_fail {ka / n:.4f} vs {kb / n:.4f} ({n} shots)")
        assert lo_a <= kb / n <= hi_a and lo_b <= ka / n <= hi_b, (tag, t, ka / n, kb / n)
        se = np.sqrt(la[m].var() / n + lb[m].var() / n)
        assert abs(la[m].mean() - lb[m].mean()) < 5 * se + 1e-9, (tag, t, la[m].mean(), lb[m].mean(), se)
    same = np.all(ra == rb, axis=1)
    print(f"{tag}: identical records in {same.mean():.3f} of rows")
    return same


def test_config3_complex64_matches_complex128():
    circ = build_circuit(5, 5, "srx", leaf_of_qubit="optimized")
    thetas = (0.02, 0.09714)
    rows = 1024
    par, th = _theta_rows(circ, thetas, rows)
    a = _run(circ, rows, "c64", par, 0.0, seed=2)
    b = _run(circ, rows, "c128", par, 0.0, seed=2)
    for r in (a, b):
        st = r[4]
        assert st["flagged_rows"] == 0 and st["max_rank"] <= 64
        assert np.all(np.isfinite(r[2])) and np.all(r[2] <= 1e-9)
    same = _agree(a, b, th, thetas, "c64 vs c128")
    assert same.mean() >= 0.9
    # single rows may hold different (equally valid) truncations: a cut inside
    # a cluster of near-equal Schmidt values keeps a subspace chosen by
    # rounding, so log P is compared row by row only as a share
    close = np.abs(a[2] - b[2]) < 1e-3
    print(f"rows with log P within 1e-3: {close.mean():.3f}")
    assert close.mean() >= 0.9
    da, db = a[4]["discarded_weight"] / rows, b[4]["discarded_weight"] / rows
    print(f"mean discarded weight per shot: c64 {da:.4f}, c128 {db:.4f}")
    assert abs(da - db) <= 0.2 * max(da, db) + 1e-6


def test_config3_chi_convergence():
    # chi_max = 64 against 128 on the same streams (complex64): the larger
    # bond dimension discards less and the failure rates agree
    circ = build_circuit(5, 5, "srx", leaf_of_qubit="optimized")
    thetas = (0.02, 0.09714)
    rows = 256
    par, th = _theta_rows(circ, thetas, rows)
    a = _run(circ, rows, "c64", par, 0.0, seed=2, chi=64)
    b = _run(circ, rows, "c64", par, 0.0, seed=2, chi=128)
    assert a[4]["flagged_rows"] == 0 and b[4]["flagged_rows"] == 0
    assert a[4]["max_rank"] <= 64 and b[4]["max_rank"] <= 128
    _agree(a, b, th, thetas, "chi 64 vs 128")
    da, db = a[4]["discarded_weight"] / rows, b[4]["discarded_weight"] / rows
    print(f"mean discarded weight per shot: chi 64 {da:.4f}, chi 128 {db:.4f}")
    assert db <= da
