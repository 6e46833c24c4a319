"""Host-side parts of the studies: the threshold fit of Eq. 8 recovers the
threshold and exponent of failure rates drawn from the ansatz itself, and the
binomial interval matches the oracle's (an independent implementation)."""
import numpy as np

from oracle import decoder


def test_threshold_fit_recovers_synthetic_parameters():
    from paper_2511_05719_amd.studies import fit_threshold, threshold_ansatz
    g = np.random.default_rng(0)
    tau, nu = 0.015, 1.2
    pts = []
    for d in (3, 5, 7):
        for p in np.linspace(0.005, 0.03, 8):
            y = threshold_ansatz((p, d), 0.1, 2.0, 5.0, tau, nu)
            pts.append({"d": d, "p_err": p, "failures": int(g.binomial(20000, y)), "shots": 20000})
    fit = fit_threshold(pts, 0.02)
    lo, hi = fit["tau_ci99"]
    assert lo <= tau <= hi and hi - lo < 0.003
    assert abs(fit["params"]["nu"] - nu) < 4 * fit["stderr"]["nu"] + 0.05
    assert fit["dof"] == len(pts) - 5


def test_study_interval_matches_oracle_interval():
    from paper_2511_05719_amd.studies import wilson
    for k, n in ((0, 10), (3, 1000), (500, 1000), (999, 1000)):
        assert np.allclose(wilson(k, n), decoder.wilson_interval(k, n), atol=1e-14)


def test_crossing_of_two_failure_curves():
    from paper_2511_05719_amd.studies import crossing
    ps = [0.01, 0.02, 0.03, 0.04]
    pts = [{"d": 3, "p_err": p, "p_fail": 0.1 * p / 0.025} for p in ps] + \
          [{"d": 5, "p_err": p, "p_fail": 0.1 * (p / 0.025) ** 2} for p in ps]
    assert abs(crossing(pts) - 0.025) < 0.0026          # linear interpolation of the two curves
    flat = [{"d": d, "p_err": p, "p_fail": 0.5} for d in (3, 5) for p in ps[:1]]
    assert crossing(flat) != crossing(flat)              # nan without a sign change
