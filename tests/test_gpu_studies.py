"""The study functions (paper_2511_05719_amd.studies) on small samples:
the twirled failure rate equals the stabilizer oracle's on the same streams,
the noiseless circuit at chi = chi_exact never fails, and the untruncated AD
trajectories' largest bond at d=3, C=1 is Table III's 8."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workload import build_circuit  # noqa: E402
from oracle import chp, decoder  # noqa: E402


@pytest.mark.parametrize("channel,theta,gamma", [("pta_srx", 2 * math.pi * 1e-2, 0.0), ("pta_ad", 0.0, 4e-3)])
def test_pta_failure_rate_equals_stabilizer_oracle(channel, theta, gamma):
    from paper_2511_05719_amd.studies import failure_rate
    circ = build_circuit(3, 1, channel, leaf_of_qubit="optimized")
    shots, seed = 3000, 5
    r = failure_rate(circ, shots, theta, gamma, chi=64, seed=seed, batch=1024)
    recs, _ = chp.run(circ, theta, gamma, seed, np.arange(shots))
    want = int(decoder.decode_fail(circ.code.checks, recs[:, circ.data_rec]).sum())
    assert r["failures"] == want and r["shots"] == shots
    assert r["ci99"][0] <= r["p_fail"] <= r["ci99"][1]


def test_truncation_background_vanishes_at_chi_exact():
    from paper_2511_05719_amd.studies import truncation_background
    res = truncation_background(3, (1, 8), shots=2048)
    assert res["chi_exact"] == 8
    pts = {p["chi"]: p for p in res["points"]}
    assert pts[8]["failures"] == 0 and pts[8]["mean_discarded_weight"] < 1e-9
    # (a controlled gate's zip carries its two-valued index exactly before
    # the sweep back truncates to chi, so the running maximum is 2 at chi = 1)
    assert pts[1]["max_rank"] <= 2


def test_exact_bond_dimension_d3_c1():
    from paper_2511_05719_amd.studies import exact_bond_dimension
    for lay in ("default", "snake", "optimized"):
        r = exact_bond_dimension(3, 1, lay, chi=64, rows=16)
        assert r["max_rank"] == 8 and not r["cap_reached"], r


def test_exact_bond_dimension_table3_ad():
    # Table III's AD columns on this schedule: d=3, C=3 reaches 16 in all three
    # orderings (paper 32/16/16); d=5, C=1 with the clustered layout 32
    # (paper 16 for its optimised ordering; the default and snake orderings
    # exceed 128 here, as the paper's 512 / 256)
    from paper_2511_05719_amd.studies import exact_bond_dimension
    for lay in ("default", "snake", "optimized"):
        assert exact_bond_dimension(3, 3, lay, chi=64, rows=16)["max_rank"] == 16
    r = exact_bond_dimension(5, 1, "optimized", chi=128, rows=8)
    assert r["max_rank"] == 32 and not r["cap_reached"]


def test_srx_grid_against_its_twirl_small():
    # the study's structure on a small sample: both channels on the same
    # streams per theta, the twirled circuit never above the stabilizer rank
    # of the clustered layout (16 at d = 5) while the coherent one may reach chi
    from paper_2511_05719_amd.studies import srx_grid_vs_twirl
    res = srx_grid_vs_twirl(thetas=(0.05, 0.2), shots=64, batch=64)
    assert [p["theta"] for p in res["points"]] == [0.05, 0.2]
    for p in res["points"]:
        for tag in ("srx", "twirl"):
            r = p[tag]
            assert r["shots"] == 64 and 0.0 <= r["p_fail"] <= 1.0 and r["ci99"][0] <= r["p_fail"] <= r["ci99"][1]
        assert p["twirl"]["max_rank"] <= 16 and p["twirl"]["mean_discarded_weight"] < 1e-6
        assert p["srx"]["max_rank"] <= 64

