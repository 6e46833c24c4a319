"""Writes config2_exact_pfail.json: the exact logical failure probability of
the d=3 colour code, 3 rounds, amplitude damping (Eq. 2-3) at every location
with gamma in {1e-3, 2e-3, 5e-3, 1e-2}, final-data lookup decoder.

Computed only by the oracle's exact density-matrix evolution (the channel of
Eq. 2 applied exactly, mid-circuit measurements dephased and reset) and its
decoder; run from the repository root:  python tests/golden/make_config2_pfail.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from workload import build_circuit  # noqa: E402
from oracle import densitymatrix as dm, decoder  # noqa: E402

GAMMAS = (1e-3, 2e-3, 5e-3, 1e-2)


def exact_pfail(gamma: float) -> float:
    circ = build_circuit(3, 3, "ad")
    probs = dm.final_data_distribution(circ, np.zeros(circ.n_loc), np.full(circ.n_loc, gamma))
    n = circ.code.n
    bits = (np.arange(2 ** n)[:, None] >> (n - 1 - np.arange(n))) & 1
    return float((probs * decoder.decode_fail(circ.code.checks, bits)).sum())


if __name__ == "__main__":
    out = {"workload": "d=3 colour code, 3 rounds, AD at every location, final-data lookup decoder",
           "source": "oracle.densitymatrix.final_data_distribution + oracle.decoder.decode_fail",
           "p_fail": {repr(g): exact_pfail(g) for g in GAMMAS}}
    with open(os.path.join(HERE, "config2_exact_pfail.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)
