"""Final-data lookup decoder and logical readout (oracle side).

The paper's concatenated matching decoder (App. A.2) needs a library that is
not available, so the reading used is a final-data decoder: from the n final
data bits compute the Z-check syndrome, correct with a minimum-weight X
error consistent with it, and read Z-bar = Z^n as the parity of the corrected
bits (Sec. III: the data start in |0-bar>, so a parity of 1 is a logical
failure).  Minimum-weight leaders come from a breadth-first search over
single-qubit flips, trying qubits in ascending index and keeping the first
leader that reaches each syndrome.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def syndrome(checks: np.ndarray, bits: np.ndarray) -> np.ndarray:
    """[..., P] check parities of data bits [..., n]."""
    return (np.asarray(bits, dtype=np.int64) @ checks.T.astype(np.int64)) % 2


def leader_table(checks: np.ndarray) -> np.ndarray:
    """leader[s] = minimum-weight flip pattern (as [n] bits) of syndrome index
    s = sum_p s_p 2^p (first found by BFS)."""
    P, n = checks.shape
    cols = [int(sum(int(checks[p, k]) << p for p in range(P))) for k in range(n)]
    table = -np.ones((1 << P, n), dtype=np.int64)
    table[0] = 0
    seen = np.zeros(1 << P, dtype=bool)
    seen[0] = True
    dq = deque([(0, np.zeros(n, dtype=np.int64))])
    while dq:
        s, pat = dq.popleft()
        for k in range(n):
            if pat[k]:
                continue
            s2 = s ^ cols[k]
            if not seen[s2]:
                seen[s2] = True
                p2 = pat.copy()
                p2[k] = 1
                table[s2] = p2
                dq.append((s2, p2))
    return table


def decode_fail(checks: np.ndarray, data_bits: np.ndarray, table=None) -> np.ndarray:
    """Logical failure bit per shot from final data bits [T, n]."""
    if table is None:
        table = leader_table(checks)
    syn = syndrome(checks, data_bits)
    P = checks.shape[0]
    sidx = (syn * (1 << np.arange(P))).sum(axis=1)
    corr = table[sidx]
    fixed = (np.asarray(data_bits, dtype=np.int64) + corr) % 2
    return (fixed.sum(axis=1) % 2).astype(np.uint8)


def wilson_interval(k: int, n: int, z: float = 2.5758293035489004):
    """Binomial confidence interval (99% by default) of k successes in n."""
    if n == 0:
        return 0.0, 1.0
    p = k / n
    den = 1 + z * z / n
    c = (p + z * z / (2 * n)) / den
    h = z * np.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / den
    return max(0.0, c - h), min(1.0, c + h)
