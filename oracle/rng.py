"""Uniform draws for the oracle.

The paper leaves sampling unspecified.  The reading used here: every random
decision of trajectory `traj_id` (a Born outcome, a Kraus branch, a twirled
Pauli) consumes one uniform u in [0, 1) from the counter-based generator
Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by (seed, traj_id),
in op-list order.  numpy ships that generator; its Generator.random() maps
each 64-bit output word w to (w >> 11) * 2**-53.
"""
from __future__ import annotations

import numpy as np


def uniforms(seed: int, traj_ids, n_draws: int) -> np.ndarray:
    """[len(traj_ids), n_draws] float64 uniforms, row t keyed by (seed, traj_ids[t])."""
    traj_ids = np.asarray(traj_ids, dtype=np.uint64).reshape(-1)
    out = np.empty((traj_ids.size, n_draws), dtype=np.float64)
    for t, tid in enumerate(traj_ids):
        gen = np.random.Generator(np.random.Philox(key=np.array([seed, tid], dtype=np.uint64)))
        out[t] = gen.random(n_draws)
    return out


def raw_words(seed: int, traj_id: int, n_words: int) -> np.ndarray:
    """The raw 64-bit output words of the same stream (for cross-checks)."""
    bg = np.random.Philox(key=np.array([seed, traj_id], dtype=np.uint64))
    return bg.random_raw(n_words).astype(np.uint64)
