"""Schmidt rank of a stabilizer state across a cut.

For a pure stabilizer state of n qubits with generator matrix G (n x 2n over
GF(2)), the entanglement entropy of a region A is
    E(A) = rank_GF2(G restricted to the 2|A| columns of A) - |A|,
and the Schmidt spectrum across A|rest is flat with 2^E(A) equal values
(Fattal, Cubitt, Yamamoto, Bravyi, Chuang, quant-ph/0406168, 2004).  A tree
tensor network that represents such a state exactly therefore needs bond
dimension 2^E on the bond above the subtree holding A -- the bond dimension the
paper calls chi_exact (Sec. IV.A) is the maximum of these over bonds and time.
"""
from __future__ import annotations

import numpy as np


def gf2_rank(m: np.ndarray) -> int:
    a = (np.array(m, dtype=np.uint8) & 1).copy()
    rows, cols = a.shape
    r = 0
    for c in range(cols):
        piv = next((i for i in range(r, rows) if a[i, c]), None)
        if piv is None:
            continue
        a[[r, piv]] = a[[piv, r]]
        for i in range(rows):
            if i != r and a[i, c]:
                a[i] ^= a[r]
        r += 1
        if r == rows:
            break
    return r


def entanglement(G: np.ndarray, region) -> int:
    n = G.shape[0]
    region = list(region)
    if not region:
        return 0
    cols = region + [n + q for q in region]
    return gf2_rank(G[:, cols]) - len(region)


def schmidt_rank(G: np.ndarray, region) -> int:
    return 2 ** entanglement(G, region)


def tree_bond_ranks(G: np.ndarray, leaf_of_qubit, n_leaves: int) -> dict:
    """Schmidt rank above every node of a complete binary tree over
    `n_leaves` leaves (heap numbering: root 1, children 2i and 2i+1, node
    i >= n_leaves/2 is a bottom node holding leaves 2(i - L/2), +1)."""
    qubit_at = {int(l): q for q, l in enumerate(leaf_of_qubit)}
    out = {}
    L = n_leaves

    def leaves(node):
        # leaf range covered by heap node `node`
        depth = int(np.log2(node))
        span = L >> depth
        start = (node - (1 << depth)) * span
        return range(start, start + span)

    for node in range(2, L):
        region = [qubit_at[l] for l in leaves(node) if l in qubit_at]
        out[node] = schmidt_rank(G, region)
    return out
